// 3D real-to-complex FFT entry point that allocates nothing: the variant of pm_debug_fft without a
// context, for callers that cannot allocate device memory (code under HIP graph capture, tight
// serving loops).  Its scratch -- the padded half spectrum the column passes work in and the twiddle
// table -- lives in one file-scope device array of fixed size, which each GPU the library runs on
// holds until the process ends.
#include <math.h>

#include <mutex>

#include "kernels.h"
#include "pm.h"

using namespace gpm;

namespace {

constexpr size_t kScratchBytes = (size_t)PM_FFT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {nullptr};

// the device address of this device's copy of the scratch array (looked up once per device, with the
// device current); null if the lookup failed
void* scratch_address(int dev) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

// exp(-2 pi i j / n) in FP64, stored in the precision of the transform
template <typename T>
__global__ __launch_bounds__(256) void twiddle_kernel(cplx<T>* tw, int n) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  double s, c;
  sincos(-2.0 * M_PI * (double)j / (double)n, &s, &c);
  tw[j] = mk<T>((T)c, (T)s);
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

template <typename T>
pm_status run_fft(const void* d_in, void* d_out, int n, int direction, hipStream_t st, unsigned char* base) {
  const int nhp = (n / 2 + 1 + 15) / 16 * 16;
  cplx<T>* spec = reinterpret_cast<cplx<T>*>(base);
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(base + align256((size_t)n * n * nhp * sizeof(cplx<T>)));
  hipLaunchKernelGGL((twiddle_kernel<T>), dim3((n + 255) / 256), dim3(256), 0, st, tw, n);
  if (direction == 1) {
    SrcArgsH<T> s;
    s.raw = reinterpret_cast<const T*>(d_in);
    fft_forward<T>(s, MODE_RAW, n, nhp, spec, 1, tw, st);
    launch_copy_unpad<T>(spec, n, nhp, reinterpret_cast<cplx<T>*>(d_out), false, st);
  } else {
    launch_copy_unpad<T>(spec, n, nhp, const_cast<cplx<T>*>(reinterpret_cast<const cplx<T>*>(d_in)), true, st);
    T* out[1] = {reinterpret_cast<T*>(d_out)};
    fft_inverse<T>(n, nhp, spec, 1, out, 1.0 / ((double)n * n * n), tw, st);
  }
  return hipGetLastError() == hipSuccess ? PM_OK : PM_EHIP;
}

}  // namespace

extern "C" size_t pm_fft_noalloc_scratch_bytes(int n_mesh, int precision) {
  if (n_mesh < 16 || n_mesh > 1024 || (n_mesh & (n_mesh - 1)) != 0) return 0;
  if (precision != PM_FP32 && precision != PM_FP64) return 0;
  const size_t rs = precision == PM_FP64 ? 8 : 4;
  const size_t nhp = (size_t)(n_mesh / 2 + 1 + 15) / 16 * 16;
  return align256((size_t)n_mesh * n_mesh * nhp * 2 * rs) + (size_t)n_mesh * 2 * rs;
}

extern "C" pm_status pm_fft_noalloc(const void* d_in, void* d_out, int n_mesh, int precision, int direction,
                                    void* hip_stream) {
  if (!d_in || !d_out || (direction != 1 && direction != -1)) return PM_EINVAL;
  const size_t need = pm_fft_noalloc_scratch_bytes(n_mesh, precision);
  if (need == 0) return PM_EINVAL;
  if (need > kScratchBytes) return PM_ERANGE;  // the mesh's padded spectrum does not fit the scratch array
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PM_EHIP;
  unsigned char* base = reinterpret_cast<unsigned char*>(scratch_address(dev));
  if (!base) return PM_EHIP;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  return precision == PM_FP64 ? run_fft<double>(d_in, d_out, n_mesh, direction, st, base)
                              : run_fft<float>(d_in, d_out, n_mesh, direction, st, base);
}
