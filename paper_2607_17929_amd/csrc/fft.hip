// 3D real-to-complex FFT passes for an n^3 periodic mesh on gfx950.
//
// Layouts (x fastest, as in the paper's rod decomposition, Sec. 2):
//   real field      [z][y][x]                     n^3 values
//   half spectrum   [z][y][kx][c], kx = 0 .. n/2  rows padded to NHP kx values;
//                   the c components of a mode are adjacent (interleaved)
// A forward 3D transform is three passes, each reading and writing the whole
// half spectrum once:
//   pass X  (rows along x, contiguous): source assembly fused in, R2C by the
//           half-length complex FFT with the usual even/odd post-processing;
//   pass Y  (columns along y) and pass Z (columns along z): batched complex
//           FFTs on LDS tiles of n elements x C contiguous (kx, c) columns, so
//           that every global access is a C*sizeof(complex) = 128-byte segment.
// The inverse runs pass Z, pass Y and the C2R pass X.  In the PM solve, pass Z,
// the Fourier-space solves and the inverse pass Z are one fused kernel
// (solve.hip).  Every 1D FFT, along x too, is the Stockham auto-sort
// radix-8/4/2 transform of fft_lds.h on an LDS tile of interleaved columns
// (the lines of pass X sit in LDS as [element][line]).  The first stage of a
// column pass reads straight from global memory and its last stage writes
// straight to global memory.  Twiddles come from a table of
// exp(-2 pi i j / n) computed in FP64 on the host.
#include "common.h"
#include "fft_lds.h"
#include "kernels.h"

namespace gpm {

// grid: x = column tile, y = outer index, z = component.  Rows are padded to a
// multiple of C columns, so every tile is whole (the padding columns are
// transformed too and never read).  es < 2^32 elements for every supported n.
template <typename T, int N, int C, int NT, bool INV>
__global__ __launch_bounds__(NT) void fft_cols_kernel(cplx<T>* data, uint32_t es, long outer_stride, long comp_stride,
                                                      const cplx<T>* __restrict__ tw) {
  static_assert(nstages(N) >= 2, "the first stage's barrier publishes the twiddle table");
  __shared__ cplx<T> sm[N * C];
  __shared__ cplx<T> stw[N];
  for (int j = threadIdx.x; j < N; j += NT) stw[j] = tw[j];
  cplx<T>* g = data + (long)blockIdx.z * comp_stride + (long)blockIdx.y * outer_stride + (long)blockIdx.x * C;
  col_stages<T, N, C, NT, 0, INV, true, true, uint32_t, false, true>(sm, g, es, g, es, stw);
}

// ---------------------------------------------------------------------------
// Source assembly (the paper's per-site mesh kernel, Sec. 2.2), fused into pass X.
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T expm1_minus_x(T x) {
  // exp(x) - 1 - x; Taylor series for small |x| keeps full relative precision
  if (fabs(x) < (T)1e-2) {
    return x * x * ((T)0.5 + x * ((T)(1.0 / 6) + x * ((T)(1.0 / 24) + x * ((T)(1.0 / 120) + x * (T)(1.0 / 720)))));
  }
  return expm1(x) - x;
}

template <typename T>
struct SrcArgs {
  const T* dep;    // deposit components, stride n^3
  const T* phi1;   // lagged phi_{n-1} (null: zero)
  const T* dphi1;  // increment phi_{n-1} - phi_{n-2} of the lagged solve
  const T* chi1;   // lagged chi
  const T* raw;    // MODE_RAW: the field to transform
  double* rowsum;  // FP64 row sums [z][y] of the phi source without its E - ebar term (may be null)
  T kap;           // 4 pi G m / dx^3 / a^2
  T ebar;          // 4 pi G a^2 rho_bar
  T hc;            // H_conf at the solve time
  T inv_dt;        // 1 / (tau_n - tau_{n-1}), 0 for a quasi-static solve
  T inv_dtl;       // 1 / (tau_{n-1} - tau_{n-2}) for the lagged phi-dot, 0 if unknown
  T half_n;        // n / 2: centred difference factor
  T n2;            // n^2: 7-point Laplacian factor
  int incr;        // source of the increment phi_n - phi_{n-1}
};

// Writes the n_src sources of vertex (x, y, z) to out[c * cstride].
template <typename T, int MODE>
__device__ __forceinline__ T assemble_point(const SrcArgs<T>& a, int n, int x, int y, int z, T* out, int cstride) {
  const long nn = (long)n * n;
  const long idx = (long)z * nn + (long)y * n + x;
  if constexpr (MODE == MODE_RAW) {
    out[0] = a.raw[idx];
    return out[0];
  } else if constexpr (MODE == MODE_NEWTONIAN) {
    const T s = a.kap * a.dep[idx] - a.ebar;
    out[0] = s;
    return s;
  } else {
    const long n3 = nn * n;
    const T E = a.kap * a.dep[idx];
    T p = 0, c = 0, pd = 0, lap = 0, gp[3] = {0, 0, 0}, gc[3] = {0, 0, 0};
    if (a.phi1) {
      const int xm = wrapi(x - 1, n), xp = wrapi(x + 1, n);
      const int ym = wrapi(y - 1, n), yp = wrapi(y + 1, n);
      const int zm = wrapi(z - 1, n), zp = wrapi(z + 1, n);
      const long rz = (long)z * nn, ry = (long)y * n;
      const long ix[3][2] = {{rz + ry + xp, rz + ry + xm},
                             {rz + (long)yp * n + x, rz + (long)ym * n + x},
                             {(long)zp * nn + ry + x, (long)zm * nn + ry + x}};
      p = a.phi1[idx];
      c = a.chi1[idx];
      // lagged time derivative from the increment of the lagged solve (not from the difference of
      // two stored solutions, which in FP32 would carry both solutions' rounding)
      pd = a.dphi1[idx] * a.inv_dtl;
      T nb = 0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T up = a.phi1[ix[d][0]], dn = a.phi1[ix[d][1]];
        gp[d] = (up - dn) * a.half_n;
        gc[d] = (a.chi1[ix[d][0]] - a.chi1[ix[d][1]]) * a.half_n;
        nb += up + dn;
      }
      lap = (nb - (T)6 * p) * a.n2;
    }
    const T hc = a.hc, eb = a.ebar;
    // non-linear remainder of the Hamiltonian constraint (lagged fields)
    const T w = (T)2 * p - c;
    const T g2 = gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2];
    const T hmd = hc - pd;
    const T R = (T)0.5 * g2 + (E - eb) * p + E * expm1_minus_x(p) -
                (T)1.5 * (hmd * hmd * expm1_minus_x((T)-2 * w) + (T)2 * w * ((T)2 * hc * pd - pd * pd) + pd * pd);
    // the mean of E - ebar is taken from an FP64 sum over particles; the rest is summed here.
    // Semi-implicit form (L - 3H/dtau' - 6H^2 - ebar) phi_n = (E - ebar) - (3H/dtau') phi_{n-1}
    // - 3H^2 chi_{n-1} + R with L the 7-point Laplacian; for the increment delta = phi_n - phi_{n-1}
    // the same operator has the source (E - ebar) + R - 3H^2 chi_{n-1} - L phi_{n-1} + (6H^2 + ebar) phi_{n-1}
    const T rest = a.incr ? R - (T)3 * hc * hc * c - lap + ((T)6 * hc * hc + eb) * p
                          : R - (T)3 * hc * a.inv_dt * p - (T)3 * hc * hc * c;
    const T rhs = (E - eb) + rest;
    out[0] = rhs;
    // trace-free space-space source (symmetric, order xx xy xz yy yz zz)
    const T e3 = exp((T)3 * p);
    const int si[6] = {0, 0, 0, 1, 1, 2}, sj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = si[s], j = sj[s];
      const T K = a.kap * a.dep[(4 + s) * n3 + idx];
      out[(1 + s) * cstride] = (T)4 * e3 * K + (T)4 * gp[i] * gp[j] - (T)4 * (gp[i] * gc[j] + gc[i] * gp[j]) +
                               (T)2 * gc[i] * gc[j];
    }
    if constexpr (MODE == MODE_FULL) {
      const T ef = exp((p - c) + (T)3 * p);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T J = a.kap * a.dep[(1 + i) * n3 + idx];
        out[(7 + i) * cstride] = ef * J - pd * (gp[i] - gc[i]);
      }
    }
    return rest;
  }
}

// ---------------------------------------------------------------------------
// Pass X forward: assembly + R2C.  grid: x = y-chunk (RY rows), y = z plane.
// The L = NSRC * RY lines (line = c * RY + r) sit in LDS as [element][line], so that
// the half-length transforms are the column stages of fft_lds.h over L columns
// (consecutive lanes touch consecutive words in every stage) and the post-processing,
// component fastest, reads consecutive words too.
// ---------------------------------------------------------------------------
template <typename T, int N, int MODE, int RY, int NT>
__global__ __launch_bounds__(NT) void fft_x_r2c_kernel(SrcArgs<T> a, cplx<T>* spec, int nhp,
                                                       const cplx<T>* __restrict__ tw) {
  constexpr int M = N / 2;
  constexpr int NSRC = mode_nsrc(MODE);
  constexpr int L = NSRC * RY;
  __shared__ cplx<T> cs[M * L];
  __shared__ cplx<T> stw[M];   // W_N^j (j < M) for the post-processing
  __shared__ cplx<T> stwm[M];  // W_M^j = W_N^(2j) for the half-length transforms
  __shared__ double red[RY][NT / 64];
  const int y0 = blockIdx.x * RY, z = blockIdx.y;
  const int tid = threadIdx.x;
  for (int j = tid; j < M; j += NT) stw[j] = tw[j];
  for (int j = tid; j < M; j += NT) stwm[j] = tw[2 * j];
  // 1. assemble the sources of RY rows: real x of line (c, r) is element x / 2, real (x even) or
  //    imaginary (x odd) part
  T* smr = reinterpret_cast<T*>(cs);
  double acc[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) acc[r] = 0.0;
  for (int p = tid; p < RY * N; p += NT) {
    const int r = p / N, x = p % N;
    const T s0 = assemble_point<T, MODE>(a, N, x, y0 + r, z, smr + ((x >> 1) * L + r) * 2 + (x & 1), 2 * RY);
#pragma unroll
    for (int rr = 0; rr < RY; ++rr)
      if (rr == r) acc[rr] += (double)s0;
  }
  if (a.rowsum) {
    // fixed-order FP64 row sums: within each wave, then the waves in order
#pragma unroll
    for (int r = 0; r < RY; ++r) {
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) acc[r] += __shfl_down(acc[r], d);
      if ((tid & 63) == 0) red[r][tid >> 6] = acc[r];
    }
    __syncthreads();
    if (tid < RY) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) t += red[tid][w];
      a.rowsum[(long)z * N + y0 + tid] = t;
    }
  } else {
    __syncthreads();
  }
  // 2. half-length complex FFT of every line (pairs of reals are complex values)
  col_stages<T, M, L, NT, 0, false, false, false, uint32_t>(cs, nullptr, 0u, nullptr, 0u, stwm);
  // 3. post-process Z_k -> X_k (k = 0..M) and store the rows, component fastest: the
  //    spectrum is component-interleaved, so the stores of a row are contiguous
  for (int job = tid; job < L * (M + 1); job += NT) {
    const int c = job % NSRC, rk = job / NSRC;
    const int k = rk % (M + 1), r = rk / (M + 1);
    const int line = c * RY + r;
    const cplx<T> zk = cs[(k == M ? 0 : k) * L + line];
    const cplx<T> zc = conj(cs[(k == 0 ? 0 : M - k) * L + line]);
    const cplx<T> ev = scale(zk + zc, (T)0.5);
    const cplx<T> od = scale(zk - zc, (T)0.5);  // = i * O_k
    // X_k = E_k + W^k O_k with O_k = -i * od
    const cplx<T> w = stw[k == M ? 0 : k];
    const cplx<T> wk = (k == M) ? mk<T>(-1, 0) : w;
    const cplx<T> o = mk(od.y, -od.x);
    const cplx<T> xk = ev + cmul(wk, o);
    store_nt(spec + ((((long)z * N + (y0 + r)) * nhp + k) * NSRC + c), xk);  // streamed to the column pass
  }
}

// ---------------------------------------------------------------------------
// Pass X inverse: C2R of NOUT components into separate real arrays; the lines sit in
// LDS as [element][line] like the forward pass.
// ---------------------------------------------------------------------------
template <typename T>
struct OutPtrs {
  T* p[8];
  const T* base0;  // non-null: component 0 is an increment added to base0 ...
  T* delta0;       // ... and stored as it is here
};

template <typename T, int N, int NOUT, int RY, int NT>
__global__ __launch_bounds__(NT) void fft_x_c2r_kernel(const cplx<T>* spec, int nhp, OutPtrs<T> out, T out_scale,
                                                       const cplx<T>* __restrict__ tw) {
  constexpr int M = N / 2;
  constexpr int L = NOUT * RY;
  __shared__ cplx<T> cs[M * L];
  __shared__ cplx<T> stw[M];   // W_N^j (j < M) for the pre-processing
  __shared__ cplx<T> stwm[M];  // W_M^j = W_N^(2j), formed from stw (W_N^M = -1)
  const int y0 = blockIdx.x * RY, z = blockIdx.y;
  const int tid = threadIdx.x;
  // 1. pre-process X_k -> Z_k = E_k + i O_k, E_k = X_k + conj X_{M-k}, O_k = (X_k - conj X_{M-k}) W^-k;
  //    the spectrum (component-interleaved) is read component fastest, so that the loads of a row
  //    are contiguous; the reads are issued first, the twiddle table is staged while they are in flight
  //    and the half-length table is formed from it in LDS
  constexpr int PJ = (L * M + NT - 1) / NT;
  cplx<T> xk[PJ], xm[PJ];
#pragma unroll
  for (int q = 0; q < PJ; ++q) {
    const int job = tid + q * NT;
    if ((L * M) % NT == 0 || job < L * M) {
      const int c = job % NOUT, rk = job / NOUT;
      const int k = rk % M, r = rk / M;
      const cplx<T>* row = spec + ((long)z * N + (y0 + r)) * nhp * NOUT;
      xk[q] = row[k * NOUT + c];
      xm[q] = row[(M - k) * NOUT + c];
    }
  }
  for (int j = tid; j < M; j += NT) stw[j] = tw[j];
  __syncthreads();
  for (int j = tid; j < M; j += NT) stwm[j] = 2 * j < M ? stw[2 * j] : mk(-stw[2 * j - M].x, -stw[2 * j - M].y);
#pragma unroll
  for (int q = 0; q < PJ; ++q) {
    const int job = tid + q * NT;
    if ((L * M) % NT == 0 || job < L * M) {
      const int c = job % NOUT, rk = job / NOUT;
      const int k = rk % M, r = rk / M;
      const int line = c * RY + r;
      cplx<T> a = xk[q], b = xm[q];
      if (k == 0) {
        a.y = 0;
        b.y = 0;
      }
      const cplx<T> bc = conj(b);
      const cplx<T> ev = a + bc;
      const cplx<T> od = cmulc(a - bc, stw[k]);
      cs[k * L + line] = mk(ev.x - od.y, ev.y + od.x);
    }
  }
  __syncthreads();
  col_stages<T, M, L, NT, 0, true, false, false, uint32_t>(cs, nullptr, 0u, nullptr, 0u, stwm);
  // 2. z_n = x_{2n} + i x_{2n+1}: real x of line (c, r) is element x / 2
  const T* rs = reinterpret_cast<const T*>(cs);
  for (int job = tid; job < L * N; job += NT) {
    const int line = job / N, x = job % N;
    const int c = line / RY, r = line % RY;
    const long o = ((long)z * N + (y0 + r)) * N + x;
    const T v = rs[((x >> 1) * L + line) * 2 + (x & 1)] * out_scale;
    if (c == 0 && out.base0) {
      out.delta0[o] = v;
      out.p[0][o] = out.base0[o] + v;
    } else {
      out.p[c][o] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
constexpr int X_ROW_BYTES = 2048;  // real row bytes per pass-X workgroup
constexpr int COL_BYTES = 128;     // contiguous bytes of one column-tile row
template <typename T, int N> constexpr int rows_per_block() {
  constexpr int r = X_ROW_BYTES / (N * (int)sizeof(T));
  return r < 1 ? 1 : (r > N ? N : r);
}
template <typename T> constexpr int col_tile() { return COL_BYTES / (int)sizeof(cplx<T>); }

template <typename T, int N>
static void launch_cols(cplx<T>* spec, int ncomp, bool inv, bool along_z, int nhp, const cplx<T>* tw, hipStream_t st) {
  constexpr int C = col_tile<T>();
  // n = 1024: the 128 KB tile leaves one workgroup per CU, so it takes 16 waves (23.6 -> 19.9 ms
  // forward at 1024^3); at n = 512 two 256-thread workgroups share a CU and 512 threads gain nothing
  constexpr int NT = N >= 1024 ? 1024 : ((N * C / 8 < 256) ? (N * C / 8 < 64 ? 64 : N * C / 8) : 256);
  static_assert(16 % C == 0, "tiles divide the 16-column row padding");
  const long comp_stride = (long)N * N * nhp;
  dim3 grid(nhp / C, N, ncomp);
  const uint32_t es = along_z ? (uint32_t)(N * nhp) : (uint32_t)nhp;
  const long os = along_z ? (long)nhp : (long)N * nhp;
  if (inv)
    hipLaunchKernelGGL((fft_cols_kernel<T, N, C, NT, true>), grid, dim3(NT), 0, st, spec, es, os, comp_stride, tw);
  else
    hipLaunchKernelGGL((fft_cols_kernel<T, N, C, NT, false>), grid, dim3(NT), 0, st, spec, es, os, comp_stride, tw);
}

template <typename T, int N>
static void launch_r2c(const SrcArgs<T>& a, int mode, cplx<T>* spec, int nhp, const cplx<T>* tw, hipStream_t st) {
  constexpr int RY = rows_per_block<T, N>();
  constexpr int NT = N >= 1024 ? 512 : 256;  // 1024^3: 25.0 -> 21.2 ms
  dim3 grid(N / RY, N);
  switch (mode) {
    case MODE_RAW:
      hipLaunchKernelGGL((fft_x_r2c_kernel<T, N, MODE_RAW, RY, NT>), grid, dim3(NT), 0, st, a, spec, nhp, tw);
      break;
    case MODE_NEWTONIAN:
      hipLaunchKernelGGL((fft_x_r2c_kernel<T, N, MODE_NEWTONIAN, RY, NT>), grid, dim3(NT), 0, st, a, spec, nhp, tw);
      break;
    case MODE_SCALAR:
      hipLaunchKernelGGL((fft_x_r2c_kernel<T, N, MODE_SCALAR, RY, NT>), grid, dim3(NT), 0, st, a, spec, nhp, tw);
      break;
    default:
      hipLaunchKernelGGL((fft_x_r2c_kernel<T, N, MODE_FULL, RY, NT>), grid, dim3(NT), 0, st, a, spec, nhp, tw);
      break;
  }
}

template <typename T, int N, int NOUT>
static void launch_c2r_n(const cplx<T>* spec, int nhp, const OutPtrs<T>& out, T scale_, const cplx<T>* tw,
                         hipStream_t st) {
  constexpr int RY0 = rows_per_block<T, N>();
  constexpr int RY = (NOUT > 2 && RY0 > 1) ? RY0 / 2 : RY0;
  constexpr int NT = N >= 1024 ? 512 : 256;  // 1024^3: 15.0 -> 11.6 ms
  dim3 grid(N / RY, N);
  hipLaunchKernelGGL((fft_x_c2r_kernel<T, N, NOUT, RY, NT>), grid, dim3(NT), 0, st, spec, nhp, out, scale_, tw);
}

template <typename T, int N>
static void launch_c2r(const cplx<T>* spec, int nhp, int nout, const OutPtrs<T>& out, T scale_, const cplx<T>* tw,
                       hipStream_t st) {
  switch (nout) {
    case 1: launch_c2r_n<T, N, 1>(spec, nhp, out, scale_, tw, st); break;
    case 2: launch_c2r_n<T, N, 2>(spec, nhp, out, scale_, tw, st); break;
    case 3: launch_c2r_n<T, N, 3>(spec, nhp, out, scale_, tw, st); break;
    case 5: launch_c2r_n<T, N, 5>(spec, nhp, out, scale_, tw, st); break;
    default: launch_c2r_n<T, N, 6>(spec, nhp, out, scale_, tw, st); break;
  }
}

#define GPM_FOR_EACH_N(X) X(16) X(32) X(64) X(128) X(256) X(512) X(1024)

template <typename T>
void fft_r2c_x(const SrcArgsH<T>& ah, int mode, int n, int nhp, cplx<T>* spec, const cplx<T>* tw, hipStream_t st) {
  SrcArgs<T> a;
  a.dep = ah.dep; a.phi1 = ah.phi1; a.dphi1 = ah.dphi1; a.chi1 = ah.chi1; a.raw = ah.raw; a.rowsum = ah.rowsum;
  a.kap = (T)ah.kap; a.ebar = (T)ah.ebar; a.hc = (T)ah.hc; a.inv_dt = (T)ah.inv_dt; a.inv_dtl = (T)ah.inv_dtl;
  a.half_n = (T)(0.5 * n);
  a.n2 = (T)((double)n * n);
  a.incr = ah.incr;
  switch (n) {
#define X(NN) case NN: launch_r2c<T, NN>(a, mode, spec, nhp, tw, st); break;
    GPM_FOR_EACH_N(X)
#undef X
  }
}

template <typename T>
void fft_cols(int n, int nhp, cplx<T>* spec, int ncomp, bool inv, bool along_z, const cplx<T>* tw, hipStream_t st) {
  switch (n) {
#define X(NN) case NN: launch_cols<T, NN>(spec, ncomp, inv, along_z, nhp, tw, st); break;
    GPM_FOR_EACH_N(X)
#undef X
  }
}

template <typename T>
void fft_c2r_x(int n, int nhp, const cplx<T>* spec, int nout, T* const* outp, double out_scale, const cplx<T>* tw,
               hipStream_t st, const T* base0, T* delta0) {
  OutPtrs<T> o;
  for (int i = 0; i < 8; ++i) o.p[i] = (i < nout) ? outp[i] : nullptr;
  o.base0 = base0;
  o.delta0 = base0 ? delta0 : nullptr;
  switch (n) {
#define X(NN) case NN: launch_c2r<T, NN>(spec, nhp, nout, o, (T)out_scale, tw, st); break;
    GPM_FOR_EACH_N(X)
#undef X
  }
}

template <typename T>
void fft_forward(const SrcArgsH<T>& ah, int mode, int n, int nhp, cplx<T>* spec, int ncomp, const cplx<T>* tw,
                 hipStream_t st) {
  fft_r2c_x<T>(ah, mode, n, nhp, spec, tw, st);
  fft_cols<T>(n, nhp * ncomp, spec, 1, false, false, tw, st);
  fft_cols<T>(n, nhp * ncomp, spec, 1, false, true, tw, st);
}

template <typename T>
void fft_inverse(int n, int nhp, cplx<T>* spec, int nout, T* const* outp, double out_scale, const cplx<T>* tw,
                 hipStream_t st) {
  fft_cols<T>(n, nhp * nout, spec, 1, true, true, tw, st);
  fft_cols<T>(n, nhp * nout, spec, 1, true, false, tw, st);
  fft_c2r_x<T>(n, nhp, spec, nout, outp, out_scale, tw, st);
}

#define GPM_FFT_INST(T)                                                                                          \
  template void fft_r2c_x<T>(const SrcArgsH<T>&, int, int, int, cplx<T>*, const cplx<T>*, hipStream_t);          \
  template void fft_cols<T>(int, int, cplx<T>*, int, bool, bool, const cplx<T>*, hipStream_t);                   \
  template void fft_c2r_x<T>(int, int, const cplx<T>*, int, T* const*, double, const cplx<T>*, hipStream_t,       \
                             const T*, T*);                                                                      \
  template void fft_forward<T>(const SrcArgsH<T>&, int, int, int, cplx<T>*, int, const cplx<T>*, hipStream_t);    \
  template void fft_inverse<T>(int, int, cplx<T>*, int, T* const*, double, const cplx<T>*, hipStream_t);
GPM_FFT_INST(float)
GPM_FFT_INST(double)

}  // namespace gpm
