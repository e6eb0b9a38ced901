// Shared device helpers for the PM library (complex arithmetic, small DFTs, indexing).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpm {

template <typename T> struct cplx { T x, y; };

template <typename T> __device__ __forceinline__ cplx<T> mk(T a, T b) { cplx<T> c; c.x = a; c.y = b; return c; }
template <typename T> __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T> __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T> __device__ __forceinline__ cplx<T> conj(cplx<T> a) { return mk(a.x, -a.y); }
template <typename T> __device__ __forceinline__ cplx<T> scale(cplx<T> a, T s) { return mk(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV> __device__ __forceinline__ cplx<T> mul_mi(cplx<T> a) {
  return INV ? mk(-a.y, a.x) : mk(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// In-register DFTs of length 2, 4, 8.  Forward: X_k = sum_n x_n exp(-2 pi i nk/R);
// inverse: the conjugate kernel (no scaling).  Outputs in natural order.
// ---------------------------------------------------------------------------
template <typename T, bool INV> __device__ __forceinline__ void dft2(cplx<T>* v) {
  cplx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename T, bool INV> __device__ __forceinline__ void dft4(cplx<T>* v) {
  cplx<T> s02 = v[0] + v[2], d02 = v[0] - v[2];
  cplx<T> s13 = v[1] + v[3], d13 = mul_mi<T, INV>(v[1] - v[3]);
  v[0] = s02 + s13;
  v[2] = s02 - s13;
  v[1] = d02 + d13;
  v[3] = d02 - d13;
}

template <typename T, bool INV> __device__ __forceinline__ void dft8(cplx<T>* v) {
  // split into even outputs (DFT4 of a_n = x_n + x_{n+4}) and odd outputs
  // (DFT4 of b_n = (x_n - x_{n+4}) w8^n), w8 = exp(-+ i pi / 4)
  const T h = (T)0.70710678118654752440;
  cplx<T> a[4], b[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    a[n] = v[n] + v[n + 4];
    b[n] = v[n] - v[n + 4];
  }
  // b1 *= w8, b2 *= w8^2 = -+i, b3 *= w8^3
  {
    cplx<T> t = b[1];
    b[1] = INV ? mk(h * (t.x - t.y), h * (t.x + t.y)) : mk(h * (t.x + t.y), h * (t.y - t.x));
    b[2] = mul_mi<T, INV>(b[2]);
    t = b[3];
    b[3] = INV ? mk(-h * (t.x + t.y), h * (t.x - t.y)) : mk(h * (t.y - t.x), -h * (t.x + t.y));
  }
  dft4<T, INV>(a);
  dft4<T, INV>(b);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[2 * k] = a[k];
    v[2 * k + 1] = b[k];
  }
}

template <typename T, int R, bool INV> __device__ __forceinline__ void dftR(cplx<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else dft8<T, INV>(v);
}

// radix of stage s for a length-M transform: eights first, then a 4 or 2
__host__ __device__ constexpr int ilog2c(int m) { return m <= 1 ? 0 : 1 + ilog2c(m / 2); }
__host__ __device__ constexpr int nstages(int m) { return (ilog2c(m) + 2) / 3; }
__host__ __device__ constexpr int stage_radix(int m, int s) {
  // number of full radix-8 stages = log2(m) / 3, the last stage takes the rest
  return (s < ilog2c(m) / 3) ? 8 : (ilog2c(m) % 3 == 1 ? 2 : (ilog2c(m) % 3 == 2 ? 4 : 8));
}
__host__ __device__ constexpr int stage_ns(int m, int s) {
  return s == 0 ? 1 : stage_ns(m, s - 1) * stage_radix(m, s - 1);
}

__device__ __forceinline__ int wrapi(int i, int n) { return i & (n - 1); }

// four values read or written as one aligned LDS access
template <typename T> struct alignas(4 * sizeof(T)) V4 { T x, y, z, w; };

// Reciprocal and reciprocal square root: the FP32 path uses the hardware
// instructions (about 1 ulp), the FP64 path the correctly rounded operations.
template <typename T> __device__ __forceinline__ T rcp(T x) { return (T)1 / x; }
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <typename T> __device__ __forceinline__ T rsqrt_(T x) { return (T)1 / sqrt(x); }
template <> __device__ __forceinline__ float rsqrt_<float>(float x) { return __builtin_amdgcn_rsqf(x); }

// Workgroups of a launch go to the 8 XCDs in turn (workgroup b to XCD b mod 8),
// and each XCD has its own L2.  xcd_remap turns the hardware index into a
// logical one under which every XCD walks one contiguous range, so that
// neighbouring workgroups -- which share halo data or output cache lines --
// meet in the same L2.  A bijection of [0, nb) for any nb.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb) {
  constexpr uint32_t NX = 8;
  const uint32_t q = nb / NX, r = nb % NX, x = b % NX;
  return x * q + min(x, r) + b / NX;
}

// the logical 3D workgroup coordinate of a 3D launch (x fastest)
__device__ __forceinline__ void xcd_block3(int& bx, int& by, int& bz) {
  const uint32_t gx = gridDim.x, gy = gridDim.y;
  const uint32_t b = (blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x;
  const uint32_t l = xcd_remap(b, gx * gy * gridDim.z);
  bx = (int)(l % gx);
  by = (int)((l / gx) % gy);
  bz = (int)(l / (gx * gy));
}

}  // namespace gpm
