// Fourier-space metric solves (Sec. 3.1 of the paper), one thread per mode of the half spectrum.
//
// With the sources of the forward pass X (S_phi, Sigma_ij, S_i) and the
// lattice wave vector kt_d = 2 n sin(pi m_d / n) (so that -kt^2 is the symbol
// of the 7-point Laplacian and every projector is exactly idempotent):
//   phi(k) = S_phi(k) / (-kt^2 - 3 H / dtau' - 6 H^2 - ebar)      Hamiltonian constraint, Eq. 4
//   chi(k) = -3 / (4 kt^4) (kt_i kt_j Sigma_ij - kt^2 Sigma_ii / 3)  scalar part of Eq. 5
//   B_i(k) = 4 / kt^2 (delta_ij - kt_i kt_j / kt^2) S_j(k)         momentum constraint, Eq. 6
//   h:  h'' + 2 H h' + kt^2 h = Lambda^TT Sigma                   tensor part of Eq. 5,
//       advanced by one Crank-Nicolson step on two polarisation amplitudes.
// The k = 0 mode of phi uses the FP64 sum of its source (the homogeneous mode
// evolves, Sec. 3.1); chi, B and h have no k = 0 mode.  Solutions are scaled by
// 1/n^3 so that the unnormalised inverse FFT returns real-space fields.
#include "kernels.h"

namespace gpm {

template <typename T>
__device__ __forceinline__ void polarisation_basis(T kx, T ky, T kz, T k2, T* e1, T* e2) {
  const T r2 = kx * kx + ky * ky;
  if (r2 > (T)0) {
    const T ir = (T)1 / sqrt(r2);
    e1[0] = ky * ir; e1[1] = -kx * ir; e1[2] = 0;
  } else {
    e1[0] = 1; e1[1] = 0; e1[2] = 0;
  }
  const T ik = (T)1 / sqrt(k2);
  const T h0 = kx * ik, h1 = ky * ik, h2 = kz * ik;
  e2[0] = h1 * e1[2] - h2 * e1[1];
  e2[1] = h2 * e1[0] - h0 * e1[2];
  e2[2] = h0 * e1[1] - h1 * e1[0];
}

template <typename T>
__device__ __forceinline__ void cn_step(cplx<T>& h, cplx<T>& p, cplx<T> s, T k2, T d, T hh) {
  const T q = (T)0.25 * d * d * k2;
  const T inv_den = (T)1 / ((T)1 + q + d * hh);
  const T cp = (T)1 - q - d * hh;
  cplx<T> pn = mk((p.x * cp + d * s.x - d * k2 * h.x) * inv_den, (p.y * cp + d * s.y - d * k2 * h.y) * inv_den);
  h = mk(h.x + (T)0.5 * d * (pn.x + p.x), h.y + (T)0.5 * d * (pn.y + p.y));
  p = pn;
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void solve_kernel(SolveArgs<T> a) {
  const int n = a.n, nh = n / 2 + 1;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)n * n * nh;
  if (t >= total) return;
  const int kx = (int)(t % nh);
  const long r = t / nh;
  const int ky = (int)(r % n), kz = (int)(r / n);
  const long idx = ((long)kz * n + ky) * a.nhp + kx;
  const T k[3] = {a.kt[kx], a.kt[ky], a.kt[kz]};
  const T k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  const T s = (T)a.inv_n3;
  cplx<T>* sp = a.spec;
  const long cs = a.comp_stride;
  const bool zero = (kx == 0 && ky == 0 && kz == 0);
  // chi, B and h have no Nyquist-plane modes: their projectors hold factors odd in
  // one component (kt_x kt_y, ...), whose sign is undefined where k_d = -k_d.
  const int nh2 = n / 2;
  const bool nyq = (kx == nh2 || ky == nh2 || kz == nh2);

  if constexpr (MODE == MODE_NEWTONIAN) {
    const cplx<T> src = sp[idx];
    sp[idx] = zero ? mk<T>(0, 0) : scale(src, -s / k2);
    return;
  } else {
    cplx<T> src[10];
    constexpr int NS = mode_nsrc(MODE);
#pragma unroll
    for (int c = 0; c < NS; ++c) src[c] = sp[c * cs + idx];
    // phi
    const T den = -k2 - (T)(3.0 * a.hc * a.inv_dt + 6.0 * a.hc * a.hc + a.ebar);
    cplx<T> phi = scale(src[0], s / den);
    if (zero && a.dc) {
      // FP64 homogeneous mode: unnormalised k = 0 coefficient sum(S_phi) / d0
      const double d0 = -(3.0 * a.hc * a.inv_dt + 6.0 * a.hc * a.hc + a.ebar);
      const double src0 = a.dc[0] + a.kap_a2 * a.dc[2] - a.n3_ebar;
      const double mean = src0 / d0 * a.inv_n3;
      phi = mk<T>((T)mean, 0);
      if (a.phibar_out) a.phibar_out[0] = mean;
    }
    // chi: scalar projection of Sigma
    const cplx<T>* sg = src + 1;
    const int si[6] = {0, 0, 0, 1, 1, 2}, sj[6] = {0, 1, 2, 1, 2, 2};
    cplx<T> contr = mk<T>(0, 0);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const T m = (si[q] == sj[q] ? (T)1 : (T)2) * k[si[q]] * k[sj[q]];
      contr = mk(contr.x + m * sg[q].x, contr.y + m * sg[q].y);
    }
    const cplx<T> tr = sg[0] + sg[3] + sg[5];
    cplx<T> chi = mk<T>(0, 0);
    if (!zero && !nyq) {
      const T f = -(T)0.75 / (k2 * k2) * s;
      chi = mk(f * (contr.x - k2 * tr.x / (T)3), f * (contr.y - k2 * tr.y / (T)3));
    }
    sp[idx] = phi;
    sp[cs + idx] = chi;
    if constexpr (MODE == MODE_FULL || MODE == MODE_FULLP) {
      cplx<T> B[3] = {mk<T>(0, 0), mk<T>(0, 0), mk<T>(0, 0)};
      if constexpr (MODE == MODE_FULL) {
        // B: transverse projection of the momentum source (Eq. 6)
        const cplx<T>* S = src + 7;
        cplx<T> Bu[3] = {mk<T>(0, 0), mk<T>(0, 0), mk<T>(0, 0)};
        if (!zero && !nyq) {
          const T ik2 = (T)1 / k2;
          const cplx<T> kd = mk((k[0] * S[0].x + k[1] * S[1].x + k[2] * S[2].x) * ik2,
                                (k[0] * S[0].y + k[1] * S[1].y + k[2] * S[2].y) * ik2);
          const T f = (T)4 * ik2;
#pragma unroll
          for (int i = 0; i < 3; ++i) Bu[i] = mk(f * (S[i].x - k[i] * kd.x), f * (S[i].y - k[i] * kd.y));
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) B[i] = scale(Bu[i], s);
        if (a.b_op == 1) {
          // start of the parabolic route: a^2 B from the momentum constraint
          const T a2 = (T)a.a2_now;
#pragma unroll
          for (int i = 0; i < 3; ++i) a.a2b[i][idx] = scale(Bu[i], a2);
        }
      } else {
        // B from the vector part of Eq. 5: d_tau (a^2 B_j) = -i a^2 w_j / |kt|,
        // w = P (Sigma khat) the spin-1 part of the trace-free source
        cplx<T> st[3] = {mk<T>(0, 0), mk<T>(0, 0), mk<T>(0, 0)};
        if (!zero && !nyq) {
          const T kn = sqrt(k2), ikn = (T)1 / kn;
          const T kh[3] = {k[0] * ikn, k[1] * ikn, k[2] * ikn};
          const cplx<T> v[3] = {
              mk(sg[0].x * kh[0] + sg[1].x * kh[1] + sg[2].x * kh[2], sg[0].y * kh[0] + sg[1].y * kh[1] + sg[2].y * kh[2]),
              mk(sg[1].x * kh[0] + sg[3].x * kh[1] + sg[4].x * kh[2], sg[1].y * kh[0] + sg[3].y * kh[1] + sg[4].y * kh[2]),
              mk(sg[2].x * kh[0] + sg[4].x * kh[1] + sg[5].x * kh[2], sg[2].y * kh[0] + sg[4].y * kh[1] + sg[5].y * kh[2])};
          const cplx<T> kv = mk(kh[0] * v[0].x + kh[1] * v[1].x + kh[2] * v[2].x,
                                kh[0] * v[0].y + kh[1] * v[1].y + kh[2] * v[2].y);
          const T f = (T)a.dtau * (T)a.a2_mid * ikn;
          const T out_scale = s / (T)a.a2_now;
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            const cplx<T> w = mk(v[j].x - kh[j] * kv.x, v[j].y - kh[j] * kv.y);
            const cplx<T> old = a.a2b[j][idx];
            st[j] = mk(old.x + f * w.y, old.y - f * w.x);  // -i w = (w.y, -w.x)
            B[j] = scale(st[j], out_scale);
          }
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) a.a2b[j][idx] = st[j];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) sp[(2 + i) * cs + idx] = B[i];
      // h: two polarisation amplitudes
      if (a.tensor_op == 1 || (a.tensor_op == 2 && nyq)) {
        a.hp[idx] = mk<T>(0, 0); a.hx[idx] = mk<T>(0, 0);
        a.pp[idx] = mk<T>(0, 0); a.px[idx] = mk<T>(0, 0);
      } else if (a.tensor_op == 2 && !zero) {
        T e1[3], e2[3];
        polarisation_basis(k[0], k[1], k[2], k2, e1, e2);
        // s_plus = (e1 Sigma e1 - e2 Sigma e2) / 2, s_cross = e1 Sigma e2
        cplx<T> spl = mk<T>(0, 0), scr = mk<T>(0, 0);
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const int i = si[q], j = sj[q];
          const T mult = (i == j) ? (T)1 : (T)2;
          const T cpl = (T)0.5 * mult * (e1[i] * e1[j] - e2[i] * e2[j]);
          const T ccr = (i == j) ? e1[i] * e2[j] : (e1[i] * e2[j] + e2[i] * e1[j]);
          spl = mk(spl.x + cpl * sg[q].x, spl.y + cpl * sg[q].y);
          scr = mk(scr.x + ccr * sg[q].x, scr.y + ccr * sg[q].y);
        }
        cplx<T> hp = a.hp[idx], pp = a.pp[idx], hx = a.hx[idx], px = a.px[idx];
        cn_step(hp, pp, spl, k2, (T)a.dtau, (T)a.hc_half);
        cn_step(hx, px, scr, k2, (T)a.dtau, (T)a.hc_half);
        a.hp[idx] = hp; a.pp[idx] = pp; a.hx[idx] = hx; a.px[idx] = px;
      }
    }
  }
}

template <typename T>
void launch_solve(const SolveArgs<T>& a, hipStream_t st) {
  const long total = (long)a.n * a.n * (a.n / 2 + 1);
  dim3 grid((unsigned)((total + 255) / 256));
  if (a.mode == MODE_NEWTONIAN)
    hipLaunchKernelGGL((solve_kernel<T, MODE_NEWTONIAN>), grid, dim3(256), 0, st, a);
  else if (a.mode == MODE_SCALAR)
    hipLaunchKernelGGL((solve_kernel<T, MODE_SCALAR>), grid, dim3(256), 0, st, a);
  else if (a.mode == MODE_FULLP)
    hipLaunchKernelGGL((solve_kernel<T, MODE_FULLP>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((solve_kernel<T, MODE_FULL>), grid, dim3(256), 0, st, a);
}

// h_ij(k) = h_plus e+_ij + h_cross ex_ij with e+ = e1 e1 - e2 e2, ex = e1 e2 + e2 e1
template <typename T>
__global__ __launch_bounds__(256) void tensor_components_kernel(cplx<T>* spec, long cs, int n, int nhp, const T* kt,
                                                               const cplx<T>* hp, const cplx<T>* hx) {
  const int nh = n / 2 + 1;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)n * n * nh) return;
  const int kx = (int)(t % nh);
  const long r = t / nh;
  const int ky = (int)(r % n), kz = (int)(r / n);
  const long idx = ((long)kz * n + ky) * nhp + kx;
  const T k[3] = {kt[kx], kt[ky], kt[kz]};
  const T k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  const int si[6] = {0, 0, 0, 1, 1, 2}, sj[6] = {0, 1, 2, 1, 2, 2};
  if (k2 == (T)0 || kx == n / 2 || ky == n / 2 || kz == n / 2) {
    for (int q = 0; q < 6; ++q) spec[q * cs + idx] = mk<T>(0, 0);
    return;
  }
  T e1[3], e2[3];
  polarisation_basis(k[0], k[1], k[2], k2, e1, e2);
  const cplx<T> a = hp[idx], b = hx[idx];
  for (int q = 0; q < 6; ++q) {
    const int i = si[q], j = sj[q];
    const T ep = e1[i] * e1[j] - e2[i] * e2[j];
    const T ex = e1[i] * e2[j] + e2[i] * e1[j];
    spec[q * cs + idx] = mk(ep * a.x + ex * b.x, ep * a.y + ex * b.y);
  }
}

template <typename T>
void launch_tensor_components(cplx<T>* spec, long comp_stride, int n, int nhp, const T* kt, const cplx<T>* hp,
                              const cplx<T>* hx, double, hipStream_t st) {
  const long total = (long)n * n * (n / 2 + 1);
  hipLaunchKernelGGL((tensor_components_kernel<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, spec,
                     comp_stride, n, nhp, kt, hp, hx);
}

// deterministic FP64 sum (input values widened to FP64): a fixed number of
// workgroups reduce contiguous slices, then one workgroup adds the partials
constexpr int SUM_BLOCKS = 512;

template <typename T>
__global__ __launch_bounds__(256) void sum_partial_kernel(const T* in, long count, double* part) {
  __shared__ double red[256];
  const long per = (count + SUM_BLOCKS - 1) / SUM_BLOCKS;
  const long b = (long)blockIdx.x * per, e = min(count, b + per);
  double acc = 0.0;
  for (long i = b + threadIdx.x; i < e; i += 256) acc += (double)in[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void sum_final_kernel(const double* part, double* out) {
  __shared__ double red[256];
  red[threadIdx.x] = part[threadIdx.x] + part[threadIdx.x + 256];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// out[0] = sum; out[1 .. SUM_BLOCKS] is scratch for the partials
template <typename T>
static void sum_to_f64(const T* in, long count, double* out, hipStream_t st) {
  static_assert(SUM_BLOCKS == 512, "final kernel adds two partials per thread");
  hipLaunchKernelGGL((sum_partial_kernel<T>), dim3(SUM_BLOCKS), dim3(256), 0, st, in, count, out + 8);
  hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(256), 0, st, out + 8, out);
}

void launch_sum_f64(const double* in, long count, double* out, hipStream_t st) { sum_to_f64<double>(in, count, out, st); }
void launch_sum_as_f64(const float* in, long count, double* out, hipStream_t st) { sum_to_f64<float>(in, count, out, st); }

template void launch_solve<float>(const SolveArgs<float>&, hipStream_t);
template void launch_solve<double>(const SolveArgs<double>&, hipStream_t);
template void launch_tensor_components<float>(cplx<float>*, long, int, int, const float*, const cplx<float>*,
                                              const cplx<float>*, double, hipStream_t);
template void launch_tensor_components<double>(cplx<double>*, long, int, int, const double*, const cplx<double>*,
                                               const cplx<double>*, double, hipStream_t);

}  // namespace gpm
