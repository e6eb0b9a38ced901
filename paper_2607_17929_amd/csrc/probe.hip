// Achievable-bandwidth probe: a plain device copy, one 16-byte element per thread over a grid that
// covers the buffer, with non-temporal loads and stores (streaming data, not to be kept in the caches),
// timed with events on the caller's stream.  Of the copy forms measured on the MI355X (grid-stride
// loops with 4, 8 or 16 elements per thread, with and without the non-temporal hint) this one moved
// the most bytes (6.4 TB/s read + write on 2 GiB); it is the practical ceiling the PM kernels' HBM
// rates are compared against beside the nominal peak.
#include <hip/hip_runtime.h>

#include "pm.h"

namespace {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));
constexpr int CP_NT = 256;

__global__ __launch_bounds__(CP_NT) void copy_probe_kernel(const v4u* __restrict__ src, v4u* __restrict__ dst,
                                                           long n16) {
  const long i = (long)blockIdx.x * CP_NT + threadIdx.x;
  if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

extern "C" pm_status pm_copy_probe(const void* d_src, void* d_dst, size_t bytes, int reps, void* hip_stream,
                                   double* ms_per_copy) {
  if (!d_src || !d_dst || !ms_per_copy || reps < 1 || bytes == 0 || bytes % 16 != 0 ||
      ((uintptr_t)d_src % 16) != 0 || ((uintptr_t)d_dst % 16) != 0)
    return PM_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const long n16 = (long)(bytes / 16);
  const long blocks = (n16 + CP_NT - 1) / CP_NT;
  if (blocks > 0x7fffffffL) return PM_ERANGE;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return PM_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return PM_EHIP;
  }
  const v4u* s = reinterpret_cast<const v4u*>(d_src);
  v4u* d = reinterpret_cast<v4u*>(d_dst);
  hipLaunchKernelGGL(copy_probe_kernel, dim3((unsigned)blocks), dim3(CP_NT), 0, st, s, d, n16);  // warm-up
  (void)hipEventRecord(e0, st);
  for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(copy_probe_kernel, dim3((unsigned)blocks), dim3(CP_NT), 0, st, s, d, n16);
  (void)hipEventRecord(e1, st);
  pm_status status = PM_OK;
  float ms = 0.f;
  if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
      hipGetLastError() != hipSuccess)
    status = PM_EHIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status == PM_OK) *ms_per_copy = (double)ms / reps;
  return status;
}
