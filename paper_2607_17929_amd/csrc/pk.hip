// Shell-averaged matter power spectrum of the particles (evaluation of results;
// the paper computes spectra on the fly, Sec. 4.1, and judges accuracy by their
// ratios, Sec. 4.4).  From the forward transform of the CIC count field:
//   P(k) = |count_k|^2 L^3 / (N_p^2 W(k)^2) - L^3 / N_p,  W = prod_d sinc^2(pi m_d / n),
// averaged over shells of width k_f = 2 pi / L, shell b = round(|m|), b = 1 .. n/2; a
// half-spectrum entry with 0 < m_x < n/2 stands for the two modes k and -k.
#include "kernels.h"

namespace gpm {

constexpr int PK_NT = 256;

__device__ __forceinline__ double sinc_d(double t) { return t == 0.0 ? 1.0 : sin(t) / t; }

// per-block sums [count | P | |m|] over shells, in LDS, then one row of partials per block
template <typename T>
__global__ __launch_bounds__(PK_NT) void pk_bin_kernel(const cplx<T>* __restrict__ spec, int n, int nhp, double amp2,
                                                       double shot, long per_block, double* __restrict__ part) {
  extern __shared__ double sh[];
  const int nb = n / 2 + 1, nh = n / 2 + 1;
  for (int i = threadIdx.x; i < 3 * nb; i += PK_NT) sh[i] = 0.0;
  __syncthreads();
  const long total = (long)n * n * nh;
  const long t0 = (long)blockIdx.x * per_block, t1 = min(total, t0 + per_block);
  const double pin = M_PI / n;
  for (long t = t0 + threadIdx.x; t < t1; t += PK_NT) {
    const int kx = (int)(t % nh);
    const long r = t / nh;
    const int ky = (int)(r % n), kz = (int)(r / n);
    const int my = ky <= n / 2 ? ky : ky - n, mz = kz <= n / 2 ? kz : kz - n;
    const double m2 = (double)kx * kx + (double)my * my + (double)mz * mz;
    const double km = sqrt(m2);
    const int b = (int)rint(km);
    if (b < 1 || b >= nb) continue;
    const double w = sinc_d(pin * kx) * sinc_d(pin * my) * sinc_d(pin * mz);
    const double w2 = w * w;
    const cplx<T> c = spec[((long)kz * n + ky) * nhp + kx];
    const double p = ((double)c.x * c.x + (double)c.y * c.y) * amp2 / (w2 * w2) - shot;
    const double wt = (kx > 0 && 2 * kx < n) ? 2.0 : 1.0;
    atomicAdd(&sh[b], wt);
    atomicAdd(&sh[nb + b], wt * p);
    atomicAdd(&sh[2 * nb + b], wt * km);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * nb; i += PK_NT) part[(long)blockIdx.x * 3 * nb + i] = sh[i];
}

// fixed-order sum of the blocks' partials
__global__ __launch_bounds__(PK_NT) void pk_reduce_kernel(const double* __restrict__ part, int nblocks, int len,
                                                          double* __restrict__ out) {
  const int i = blockIdx.x * PK_NT + threadIdx.x;
  if (i >= len) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += part[(long)b * len + i];
  out[i] = s;
}

int pk_blocks(int n, size_t scratch_bytes) {
  const long total = (long)n * n * (n / 2 + 1);
  const long row = 3L * (n / 2 + 1) * 8;
  long nb = (total + 4 * PK_NT - 1) / (4 * PK_NT);
  nb = nb < 1024 ? nb : 1024;
  const long fit = (long)(scratch_bytes / row) - 1;  // one row stays free for the result
  nb = nb < fit ? nb : fit;
  return nb < 1 ? 1 : (int)nb;
}

template <typename T>
void launch_power_spectrum(const cplx<T>* spec, int n, int nhp, double amp2, double shot, int nblocks, double* scratch,
                           hipStream_t st) {
  const long total = (long)n * n * (n / 2 + 1);
  const long per_block = (total + nblocks - 1) / nblocks;
  const int len = 3 * (n / 2 + 1);
  hipLaunchKernelGGL((pk_bin_kernel<T>), dim3(nblocks), dim3(PK_NT), len * sizeof(double), st, spec, n, nhp, amp2,
                     shot, per_block, scratch);
  hipLaunchKernelGGL(pk_reduce_kernel, dim3((len + PK_NT - 1) / PK_NT), dim3(PK_NT), 0, st, scratch, nblocks, len,
                     scratch + (long)nblocks * len);
}

template void launch_power_spectrum<float>(const cplx<float>*, int, int, double, double, int, double*, hipStream_t);
template void launch_power_spectrum<double>(const cplx<double>*, int, int, double, double, int, double*, hipStream_t);

}  // namespace gpm
