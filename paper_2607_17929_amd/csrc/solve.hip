// Fourier-space metric solves (Sec. 3.1 of the paper), per mode of the half spectrum, inside the
// kernel that also runs the transforms along z.
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
#include <type_traits>

#include "fft_lds.h"
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

// Per-mode state held in registers by the Fourier-space kernel: the tensor record (h+, hx, pi+,
// pix) and the parabolic record a^2 (B_x, B_y, B_z), loaded before the forward transform so that
// their latency hides behind it.
template <typename T>
struct ModeState {
  cplx<T> h[4];
  cplx<T> b[3];
};

template <typename T, int MODE>
__device__ __forceinline__ bool mode_has_state(const SolveArgs<T>& a, int kx) {
  return (MODE == MODE_FULL || MODE == MODE_FULLP) && kx <= a.n / 2;
}

template <typename T, int MODE>
__device__ __forceinline__ void load_state(const SolveArgs<T>& a, int kx, int ky, int kz, ModeState<T>& m) {
  if (!mode_has_state<T, MODE>(a, kx)) return;
  const long sidx = state_index(a.n, a.nhp, kx, ky, kz);
  if (a.tensor_op == 2) {
#pragma unroll
    for (int q = 0; q < 4; ++q) m.h[q] = a.hst[sidx * 4 + q];
  }
  if (MODE == MODE_FULLP) {
#pragma unroll
    for (int q = 0; q < 3; ++q) m.b[q] = a.a2b[sidx * 3 + q];
  }
}

// Solution of one mode (kx, ky, kz) of the half spectrum from its NS source values; writes the
// NOUT unnormalised solution coefficients (phi, chi, B_x, B_y, B_z) to o, advances the mode's
// tensor and parabolic-B state in m and stores it.  kx beyond n/2 (row padding) gives zeros and
// touches no state.
template <typename T, int MODE>
__device__ __forceinline__ void solve_mode(const SolveArgs<T>& a, int kx, int ky, int kz, const cplx<T>* src,
                                           cplx<T>* o, ModeState<T>& ms) {
  const int n = a.n, nh2 = n / 2;
  constexpr int NO = mode_nout(MODE);
  if (kx > nh2) {
#pragma unroll
    for (int c = 0; c < NO; ++c) o[c] = mk<T>(0, 0);
    return;
  }
  const T k[3] = {a.kt[kx], a.kt[ky], a.kt[kz]};
  const T k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  const T s = (T)a.inv_n3;
  const bool zero = (kx == 0 && ky == 0 && kz == 0);
  // chi, B and h have no Nyquist-plane modes: their projectors hold factors odd in
  // one component (kt_x kt_y, ...), whose sign is undefined where k_d = -k_d.
  const bool nyq = (kx == nh2 || ky == nh2 || kz == nh2);
  if constexpr (MODE == MODE_NEWTONIAN) {
    o[0] = zero ? mk<T>(0, 0) : scale(src[0], -s / k2);
    return;
  } else {
    // phi
    const T den = -k2 - (T)(3.0 * a.hc * a.inv_dt + 6.0 * a.hc * a.hc + a.ebar);
    cplx<T> phi = scale(src[0], s / den);
    if (zero && a.dc) {
      // FP64 homogeneous mode: unnormalised k = 0 coefficient sum(S_phi) / d0
      const double d0 = -(3.0 * a.hc * a.inv_dt + 6.0 * a.hc * a.hc + a.ebar);
      const double src0 = a.dc[0] + a.kap_a2 * a.dc[2] - a.n3_ebar;
      const double mean = src0 / d0 * a.inv_n3;
      phi = mk<T>((T)mean, 0);
      if (a.phibar_out) a.phibar_out[0] = a.incr ? a.phibar_out[0] + mean : mean;
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
    o[0] = phi;
    o[1] = chi;
    if constexpr (MODE == MODE_FULL || MODE == MODE_FULLP) {
      const long sidx = state_index(n, a.nhp, kx, ky, kz);
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
          for (int i = 0; i < 3; ++i) a.a2b[sidx * 3 + i] = scale(Bu[i], a2);
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
            const cplx<T> old = ms.b[j];
            st[j] = mk(old.x + f * w.y, old.y - f * w.x);  // -i w = (w.y, -w.x)
            B[j] = scale(st[j], out_scale);
          }
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) a.a2b[sidx * 3 + j] = st[j];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) o[2 + i] = B[i];
      // h: two polarisation amplitudes, state record (h+, hx, pi+, pix)
      cplx<T>* hs = a.hst + sidx * 4;
      if (a.tensor_op == 1 || (a.tensor_op == 2 && nyq)) {
#pragma unroll
        for (int q = 0; q < 4; ++q) hs[q] = mk<T>(0, 0);
      } else if (a.tensor_op == 2 && !zero) {
        cplx<T>* hr = ms.h;
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
        cplx<T> hp = hr[0], hx = hr[1], pp = hr[2], px = hr[3];
        cn_step(hp, pp, spl, k2, (T)a.dtau, (T)a.hc_half);
        cn_step(hx, px, scr, k2, (T)a.dtau, (T)a.hc_half);
        hs[0] = hp; hs[1] = hx; hs[2] = pp; hs[3] = px;
      }
    }
  }
}

// Fourier-space stage of the solve, fused: for one ky and KXT consecutive kx, the NS source
// columns along z (component-interleaved, so a row of the tile is KXT * NS contiguous complex
// values) are transformed along z in LDS, every mode is solved, and the NOUT solution columns
// are transformed back along z and written to the output spectrum.  Each value of the source
// and output spectra crosses HBM once.
// grid: x = kx tile, y = ky.
constexpr bool KS_TWPOW = true;  // twiddle powers by products (the table may live in global memory)

template <typename T, int N, int MODE, int KXT, int NT, bool TW_LDS>
__global__ __launch_bounds__(NT) void kspace_kernel(SolveArgs<T> a) {
  constexpr int NS = mode_nsrc(MODE), NO = mode_nout(MODE);
  constexpr int CI = KXT * NS, CO = KXT * NO;
  static_assert(nstages(N) >= 2, "the first stage's barrier publishes the twiddle table");
  using IX = typename std::conditional<((long)N * N * (N / 2 + 16) * NS < (1L << 31)), uint32_t, uint64_t>::type;
  __shared__ cplx<T> sm[N * CI];
  __shared__ cplx<T> stw_s[TW_LDS ? N : 1];
  const cplx<T>* stw = a.tw;
  if constexpr (TW_LDS) {
    for (int j = threadIdx.x; j < N; j += NT) stw_s[j] = a.tw[j];
    stw = stw_s;
  }
  // neighbouring kx tiles share cache lines (a row of a tile is KXT * NS complex values, not a whole
  // number of lines at n = 1024): the XCD-aware order keeps them in one L2 (1024^3: 42.6 -> 33.8 ms)
  int bxl, byl, bzl;
  xcd_block3(bxl, byl, bzl);
  const int ky = byl, kx0 = bxl * KXT;
  const cplx<T>* gin = a.spec + ((long)ky * a.nhp + kx0) * NS;
  cplx<T>* gout = a.out + ((long)ky * a.nhp + kx0) * NO;
  constexpr int MODES = N * KXT;
  constexpr int PM = (MODES + NT - 1) / NT;
  // this thread's modes: kxl fastest; their state records are requested first
  ModeState<T> ms[PM];
#pragma unroll
  for (int p = 0; p < PM; ++p) {
    const int m = threadIdx.x + p * NT;
    if (MODES % NT == 0 || m < MODES) load_state<T, MODE>(a, kx0 + m % KXT, ky, m / KXT, ms[p]);
  }
  // forward transform along z: global -> LDS
  col_stages<T, N, CI, NT, 0, false, true, false, IX, KS_TWPOW>(sm, gin, (IX)N * a.nhp * NS, nullptr, (IX)0, stw);
  // solves: the sources of this thread's modes to registers, barrier, solutions to LDS as CO columns
  cplx<T> src[PM][NS];
#pragma unroll
  for (int p = 0; p < PM; ++p) {
    const int m = threadIdx.x + p * NT;
    if (MODES % NT == 0 || m < MODES) {
      const int kxl = m % KXT, kz = m / KXT;
#pragma unroll
      for (int c = 0; c < NS; ++c) src[p][c] = sm[kz * CI + kxl * NS + c];
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PM; ++p) {
    const int m = threadIdx.x + p * NT;
    if (MODES % NT == 0 || m < MODES) {
      const int kxl = m % KXT, kz = m / KXT;
      cplx<T> o[NO];
      solve_mode<T, MODE>(a, kx0 + kxl, ky, kz, src[p], o, ms[p]);
#pragma unroll
      for (int c = 0; c < NO; ++c) sm[kz * CO + kxl * NO + c] = o[c];
    }
  }
  __syncthreads();
  // inverse transform along z: LDS -> global
  col_stages<T, N, CO, NT, 0, true, false, true, IX, KS_TWPOW>(sm, nullptr, (IX)0, gout, (IX)N * a.nhp * NO, stw);
}

// Tile shape (measured at 512^3, FP32 full physics: rows of 4 kx x 10 components = 320 B in a
// 160 KB tile, one workgroup per CU, run faster than 160 B rows with two workgroups per CU; 1024
// threads, 16 waves on the CU's one tile, 3.54 ms against 3.63 with 512)
constexpr int KS_ROW_BYTES = 256;   // contiguous bytes wanted per row of a tile
constexpr long KS_LDS = 163840;     // LDS budget of a tile
constexpr int KS_NT = 1024;         // threads of a workgroup when the tile has that many modes
// kx values per workgroup: KXT * NS * sizeof(complex) >= KS_ROW_BYTES contiguous bytes where the
// LDS tile allows
template <typename T, int N, int NS> constexpr int kspace_kxt() {
  constexpr int want = (KS_ROW_BYTES + NS * (int)sizeof(cplx<T>) - 1) / (NS * (int)sizeof(cplx<T>));
  int k = 1;
  while (k < want) k *= 2;
  while (k > 1 && (long)N * k * NS * (long)sizeof(cplx<T>) > KS_LDS) k /= 2;
  return k;
}

template <typename T, int N, int MODE>
static void launch_kspace_n(const SolveArgs<T>& a, hipStream_t st) {
  constexpr int NS = mode_nsrc(MODE);
  constexpr int KXT = kspace_kxt<T, N, NS>();
  constexpr int NT = N * KXT >= KS_NT ? KS_NT : (N * KXT >= 256 ? 256 : 64);
  constexpr bool TW_LDS = (long)N * KXT * NS * (long)sizeof(cplx<T>) + N * (long)sizeof(cplx<T>) <= KS_LDS;
  static_assert((long)N * KXT * NS * (long)sizeof(cplx<T>) + (TW_LDS ? N : 0) * (long)sizeof(cplx<T>) <= 160 * 1024,
                "LDS tile too large");
  const int nh = N / 2 + 1;
  dim3 grid((unsigned)((nh + KXT - 1) / KXT), N);
  hipLaunchKernelGGL((kspace_kernel<T, N, MODE, KXT, NT, TW_LDS>), grid, dim3(NT), 0, st, a);
}

template <typename T, int N>
static void launch_kspace_modes(const SolveArgs<T>& a, hipStream_t st) {
  switch (a.mode) {
    case MODE_NEWTONIAN: launch_kspace_n<T, N, MODE_NEWTONIAN>(a, st); break;
    case MODE_SCALAR: launch_kspace_n<T, N, MODE_SCALAR>(a, st); break;
    case MODE_FULLP: launch_kspace_n<T, N, MODE_FULLP>(a, st); break;
    default: launch_kspace_n<T, N, MODE_FULL>(a, st); break;
  }
}

template <typename T>
void launch_solve(const SolveArgs<T>& a, hipStream_t st) {
  switch (a.n) {
    case 16: launch_kspace_modes<T, 16>(a, st); break;
    case 32: launch_kspace_modes<T, 32>(a, st); break;
    case 64: launch_kspace_modes<T, 64>(a, st); break;
    case 128: launch_kspace_modes<T, 128>(a, st); break;
    case 256: launch_kspace_modes<T, 256>(a, st); break;
    case 512: launch_kspace_modes<T, 512>(a, st); break;
    default: launch_kspace_modes<T, 1024>(a, st); break;
  }
}

// h_ij(k) = h_plus e+_ij + h_cross ex_ij with e+ = e1 e1 - e2 e2, ex = e1 e2 + e2 e1, written as
// six separate half spectra [q][z][y][kx] (stride cs) for the inverse transform
template <typename T>
__global__ __launch_bounds__(256) void tensor_components_kernel(cplx<T>* spec, long cs, int n, int nhp, const T* kt,
                                                               const cplx<T>* hst) {
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
  const long sidx = state_index(n, nhp, kx, ky, kz);
  const cplx<T> a = hst[sidx * 4 + 0], b = hst[sidx * 4 + 1];
  for (int q = 0; q < 6; ++q) {
    const int i = si[q], j = sj[q];
    const T ep = e1[i] * e1[j] - e2[i] * e2[j];
    const T ex = e1[i] * e2[j] + e2[i] * e1[j];
    spec[q * cs + idx] = mk(ep * a.x + ex * b.x, ep * a.y + ex * b.y);
  }
}

template <typename T>
void launch_tensor_components(cplx<T>* spec, long comp_stride, int n, int nhp, const T* kt, const cplx<T>* hst,
                              hipStream_t st) {
  const long total = (long)n * n * (n / 2 + 1);
  hipLaunchKernelGGL((tensor_components_kernel<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, spec,
                     comp_stride, n, nhp, kt, hst);
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
                                              hipStream_t);
template void launch_tensor_components<double>(cplx<double>*, long, int, int, const double*, const cplx<double>*,
                                               hipStream_t);

}  // namespace gpm
