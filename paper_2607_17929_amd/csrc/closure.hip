// Learned force closure: a 3-layer 3x3x3 convolutional network on the mesh.
//
// Not part of the paper's method.  The network maps fields of the particle-mesh
// solution (density contrast, gradient of phi) to a correction of the gathered
// force; it is trained on pairs of the same particles' forces from a mesh and a
// mesh of twice the resolution.  conv(4->16)-ReLU-conv(16->16)-ReLU-conv(16->3),
// periodic padding, taps d in {-1,0,1}^3 (cross-correlation).
//
// Every layer runs as a 16 -> 16 channel convolution (the 4 input and 3 output
// channels are zero-padded) on channels-last bfloat16 activations
// [z][y][x][16] with FP32 accumulation on the matrix cores: an implicit GEMM
// whose M dimension is a row of 16 points along x, N the 16 output channels and
// K = 2 taps x 16 input channels per v_mfma_f32_16x16x32_bf16.  A workgroup
// computes a 16 x 8 x 4 block of points from an LDS copy of its input block
// plus a one-point margin.  The backward pass with respect to the input is the
// same kernel with flipped, transposed weights and a ReLU mask; the weight
// gradient is a second implicit GEMM on the matrix cores (K = points), its
// per-workgroup FP32 partials reduced in FP64 in a fixed order.  The training
// residual, its mean square and the augmentation by cube symmetries are
// kernels here too, so a training step is library calls only.
#include "kernels.h"

namespace gpm {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// round-to-nearest-even float -> bfloat16 bits
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

constexpr int CV_TX = 16, CV_TY = 8, CV_TZ = 4, CV_NT = 256;
constexpr int CV_HX = CV_TX + 2, CV_HY = CV_TY + 2, CV_HZ = CV_TZ + 2;
constexpr int CV_HP = CV_HX * CV_HY * CV_HZ;  // halo points
constexpr int CV_KSTEPS = 14;                 // ceil(27 taps / 2)

__device__ __forceinline__ int tap_dz(int t) { return t / 9 - 1; }
__device__ __forceinline__ int tap_dy(int t) { return (t / 3) % 3 - 1; }
__device__ __forceinline__ int tap_dx(int t) { return t % 3 - 1; }

// Load the input block plus margin into LDS: [hz][hy][hx][16] bfloat16, 16-byte chunks.
__device__ __forceinline__ void load_halo(const uint16_t* __restrict__ in, int n, int x0, int y0, int z0,
                                          uint4* __restrict__ lds) {
  const int m = n - 1;
  const long nn = (long)n * n;
  for (int q = threadIdx.x; q < CV_HP * 2; q += CV_NT) {
    const int pt = q >> 1, half = q & 1;
    const int hx = pt % CV_HX, hy = (pt / CV_HX) % CV_HY, hz = pt / (CV_HX * CV_HY);
    const long g = (long)((z0 - 1 + hz) & m) * nn + (long)((y0 - 1 + hy) & m) * n + ((x0 - 1 + hx) & m);
    lds[q] = reinterpret_cast<const uint4*>(in + g * 16)[half];
  }
}

// mode: 0 = relu(conv + bias) -> bf16 [p][16]; 1 = (conv + bias)[0..2] * scale -> FP32 SoA [3][n^3];
//       2 = conv * (mask > 0) -> bf16 [p][16] (input gradient through a ReLU)
template <int MODE>
__global__ __launch_bounds__(CV_NT) void conv16_kernel(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w,
                                                       const float* __restrict__ bias, int n, void* out,
                                                       const uint16_t* __restrict__ mask, const float* scale_ptr) {
  __shared__ uint4 tile[CV_HP * 2];
  const int x0 = blockIdx.x * CV_TX, y0 = blockIdx.y * CV_TY, z0 = blockIdx.z * CV_TZ;
  load_halo(in, n, x0, y0, z0, tile);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  // B fragments (weights, [tap][out][in] bfloat16) for the 14 K-steps, kept in registers
  v8bf bfrag[CV_KSTEPS];
#pragma unroll
  for (int s = 0; s < CV_KSTEPS; ++s) {
    const int t = 2 * s + (grp >> 1);
    uint4 v = make_uint4(0, 0, 0, 0);
    if (t < 27) v = *reinterpret_cast<const uint4*>(w + ((t * 16 + col) * 16 + 8 * (grp & 1)));
    bfrag[s] = __builtin_bit_cast(v8bf, v);
  }
  __syncthreads();
  const long n3 = (long)n * n * n;
  const float scale = (MODE == 1 && scale_ptr) ? scale_ptr[0] : 1.0f;
  const float bco = bias ? bias[col] : 0.0f;
  // each wave computes 8 rows of 16 points
  for (int r = wave; r < CV_TY * CV_TZ; r += CV_NT / 64) {
    const int ly = r % CV_TY, lz = r / CV_TY;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < CV_KSTEPS; ++s) {
      const int t = 2 * s + (grp >> 1);
      uint4 av = make_uint4(0, 0, 0, 0);
      if (t < 27) {
        // A: point x = col of this row, shifted by the tap; 8 input channels
        const int hx = col + 1 + tap_dx(t), hy = ly + 1 + tap_dy(t), hz = lz + 1 + tap_dz(t);
        av = tile[((hz * CV_HY + hy) * CV_HX + hx) * 2 + (grp & 1)];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, av), bfrag[s], acc, 0, 0, 0);
    }
    // D: lane holds rows (points) 4*grp + j of column (output channel) col
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int px = 4 * grp + j;
      const long p = ((long)(z0 + lz) * n + (y0 + ly)) * n + (x0 + px);
      const float v = acc[j] + bco;
      if constexpr (MODE == 0) {
        reinterpret_cast<uint16_t*>(out)[p * 16 + col] = f2bf(fmaxf(v, 0.0f));
      } else if constexpr (MODE == 1) {
        if (col < 3) reinterpret_cast<float*>(out)[col * n3 + p] = v * scale;
      } else {
        const bool on = bf2f(mask[p * 16 + col]) > 0.0f;
        reinterpret_cast<uint16_t*>(out)[p * 16 + col] = f2bf(on ? acc[j] : 0.0f);
      }
    }
  }
}

// Weight gradient of one layer on the matrix cores: for each tap t,
// dW_t[co][ci] = sum_p dy[p][co] x[p + d_t][ci] is a 16 x 16 GEMM with K running over the
// points.  One MFMA takes 32 points (two x-rows of a 16 x 8 x 4 tile): A[co][k] = dy[p_k][co],
// B[k][ci] = x[p_k + d_t][ci].  Both operands need 8 consecutive points per lane for one
// channel, so the tile is transposed into LDS channel-major ([ci][hz][hy][hx] with rows of
// WG_ROW elements, [co][row][lx] for dy); the x-shift of a tap is then a funnel shift of
// two aligned words.  Wave w owns taps w, w + 4, ..., and wave 3's spare slot accumulates the
// bias gradient (B = ones).  A workgroup walks tiles blockIdx.x, + gridDim.x, ... and writes
// one FP32 partial; the partials are summed in a fixed order in FP64.
constexpr int WG_ROW = 24;                              // LDS row: 18 halo points + pad, 16-byte aligned
constexpr int WG_CI = CV_HZ * CV_HY * WG_ROW + 8;       // channel stride (pad spreads the banks)
constexpr int WG_CO = CV_TX * CV_TY * CV_TZ + 8;        // dy channel stride
constexpr int WG_PART = 27 * 256 + 16;                  // one partial: [t][co][ci] then the bias [co]
constexpr int WG_GRID = 512;                            // workgroups (partials) at most

__global__ __launch_bounds__(CV_NT) void conv16_wgrad_kernel(const uint16_t* __restrict__ x,
                                                             const uint16_t* __restrict__ dy, int n, long ntiles,
                                                             float* __restrict__ part) {
  __shared__ __align__(16) uint16_t xt[16 * WG_CI];
  __shared__ __align__(16) uint16_t dyt[16 * WG_CO];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int ntx = n / CV_TX, nty = n / CV_TY;
  const int m = n - 1;
  const long nn = (long)n * n;
  v4f acc[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
  const v8bf ones = __builtin_bit_cast(v8bf, make_uint4(0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u));
  for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int x0 = (int)(tile % ntx) * CV_TX, y0 = (int)((tile / ntx) % nty) * CV_TY;
    const int z0 = (int)(tile / ((long)ntx * nty)) * CV_TZ;
    __syncthreads();  // the previous tile's operands are consumed
    for (int q = threadIdx.x; q < CV_HP * 2; q += CV_NT) {
      const int pt = q >> 1, half = q & 1;
      const int hx = pt % CV_HX, hy = (pt / CV_HX) % CV_HY, hz = pt / (CV_HX * CV_HY);
      const long g = (long)((z0 - 1 + hz) & m) * nn + (long)((y0 - 1 + hy) & m) * n + ((x0 - 1 + hx) & m);
      const uint4 v = reinterpret_cast<const uint4*>(x + g * 16)[half];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
      uint16_t* d = xt + (8 * half) * WG_CI + (hz * CV_HY + hy) * WG_ROW + hx;
#pragma unroll
      for (int c = 0; c < 8; ++c) d[c * WG_CI] = (uint16_t)(w[c >> 1] >> (16 * (c & 1)));
    }
    for (int q = threadIdx.x; q < CV_TX * CV_TY * CV_TZ * 2; q += CV_NT) {
      const int pt = q >> 1, half = q & 1;
      const int lx = pt % CV_TX, row = pt / CV_TX;  // row = ly + 8 lz
      const long g = ((long)(z0 + row / CV_TY) * n + (y0 + row % CV_TY)) * n + (x0 + lx);
      const uint4 v = reinterpret_cast<const uint4*>(dy + g * 16)[half];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
      uint16_t* d = dyt + (8 * half) * WG_CO + pt;
#pragma unroll
      for (int c = 0; c < 8; ++c) d[c * WG_CO] = (uint16_t)(w[c >> 1] >> (16 * (c & 1)));
    }
    __syncthreads();
    // lane (col, grp) of K-step s: points lx = 8 (grp & 1) + e, e < 8, of row 2 s + (grp >> 1)
    const int xb = 8 * (grp & 1);
    for (int s = 0; s < CV_TY * CV_TZ / 2; ++s) {
      const int row = 2 * s + (grp >> 1);
      const int ly = row % CV_TY, lz = row / CV_TY;
      const v8bf a = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(dyt + col * WG_CO + row * CV_TX + xb));
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        const int t = wave + 4 * j;
        if (t < 27) {
          const int hz = lz + 1 + tap_dz(t), hy = ly + 1 + tap_dy(t), dx = tap_dx(t);
          const uint16_t* r = xt + col * WG_CI + (hz * CV_HY + hy) * WG_ROW + xb;
          // halo points xb + 1 + dx + e: from the aligned words at xb .. xb + 9
          const uint4 w = *reinterpret_cast<const uint4*>(r);
          uint4 b;
          if (dx < 0) {
            b = w;
          } else {
            const uint32_t w4 = *reinterpret_cast<const uint32_t*>(r + 8);
            if (dx > 0) b = make_uint4(w.y, w.z, w.w, w4);
            else b = make_uint4(__builtin_amdgcn_alignbit(w.y, w.x, 16), __builtin_amdgcn_alignbit(w.z, w.y, 16),
                                __builtin_amdgcn_alignbit(w.w, w.z, 16), __builtin_amdgcn_alignbit(w4, w.w, 16));
          }
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(v8bf, b), acc[j], 0, 0, 0);
        } else {
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, ones, acc[j], 0, 0, 0);
        }
      }
    }
  }
  // D: lane holds co = 4 grp + r of column ci = col
  float* o = part + (long)blockIdx.x * WG_PART;
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const int t = wave + 4 * j;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int co = 4 * grp + r;
      if (t < 27) o[(t * 16 + co) * 16 + col] = acc[j][r];
      else if (col == 0) o[27 * 256 + co] = acc[j][r];
    }
  }
}

// sum the partials in a fixed order (FP64) and scatter into the flat parameter-gradient layout
// W[co][ci][27] b[co] of layer (ci_n -> co_n) at offset off; 64 entries per workgroup, each wave
// adds a contiguous quarter of the partials and the quarters are combined in order
__global__ __launch_bounds__(256) void wgrad_reduce_kernel(const float* __restrict__ part, int nblk, int ci_n, int co_n,
                                                           float* __restrict__ grad, long off) {
  __shared__ double q[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  const int lo = wave * nblk / 4, hi = (wave + 1) * nblk / 4;
  double s = 0.0;
  if (e < WG_PART)
    for (int b = lo; b < hi; ++b) s += (double)part[(long)b * WG_PART + e];
  q[wave][lane] = s;
  __syncthreads();
  if (wave != 0 || e >= WG_PART) return;
  s = ((q[0][lane] + q[1][lane]) + q[2][lane]) + q[3][lane];
  if (e < 27 * 256) {
    const int t = e / 256, co = (e / 16) % 16, ci = e % 16;
    if (co < co_n && ci < ci_n) grad[off + ((long)co * ci_n + ci) * 27 + t] = (float)s;
  } else {
    const int co = e - 27 * 256;
    if (co < co_n) grad[off + (long)co_n * ci_n * 27 + co] = (float)s;
  }
}

// flat FP32 parameters -> bf16 forward weights [L][t][co][ci], backward-data weights
// [L][t'][ci][co] (t' = 26 - t), FP32 biases [L][16]; padded channels are zero
__global__ __launch_bounds__(256) void pack_weights_kernel(const float* __restrict__ p, uint16_t* wf, uint16_t* wb,
                                                           float* bias) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;  // over 3 * 27 * 256
  const int cis[3] = {4, 16, 16}, cos_[3] = {16, 16, 3};
  const long offs[3] = {0, 16 * 4 * 27 + 16, 16 * 4 * 27 + 16 + 16 * 16 * 27 + 16};
  if (e < 3 * 16) {
    const int L = e / 16, co = e % 16;
    bias[e] = co < cos_[L] ? p[offs[L] + (long)cos_[L] * cis[L] * 27 + co] : 0.f;
  }
  if (e >= 3 * 27 * 256) return;
  const int L = e / (27 * 256), r = e % (27 * 256);
  const int t = r / 256, a = (r / 16) % 16, b = r % 16;
  // forward: wf[L][t][co = a][ci = b]
  float vf = 0.f;
  if (a < cos_[L] && b < cis[L]) vf = p[offs[L] + ((long)a * cis[L] + b) * 27 + t];
  wf[e] = f2bf(vf);
  // backward data: wb[L][t][ci = a][co = b] = W[co][ci][26 - t]
  float vb = 0.f;
  if (b < cos_[L] && a < cis[L]) vb = p[offs[L] + ((long)b * cis[L] + a) * 27 + (26 - t)];
  wb[e] = f2bf(vb);
}

// Adam on the FP32 master parameters (bias-corrected)
// (1 - beta) is passed separately: forming it in FP32 from beta = 0.999f would cost 5e-5 relative
__global__ __launch_bounds__(256) void adam_kernel(float* p, float* m, float* v, const float* g, int np, float lr,
                                                   float b1, float b2, float omb1, float omb2, float eps, float c1,
                                                   float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float vi = b2 * v[i] + omb2 * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// inputs: channel 0 = sign(delta) log(1 + |delta|), channels 1..3 = grad phi / rms|grad phi|
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void gradsq_partial_kernel(const T* __restrict__ phi, int n, double* part) {
  __shared__ double red[256];
  const long n3 = (long)n * n * n;
  const int m = n - 1;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n3; i += (long)gridDim.x * 256) {
    const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((long)n * n));
    const long nn = (long)n * n;
    const double hn = 0.5 * n;
    const double gx = ((double)phi[z * nn + y * n + ((x + 1) & m)] - (double)phi[z * nn + y * n + ((x - 1) & m)]) * hn;
    const double gy = ((double)phi[z * nn + ((y + 1) & m) * n + x] - (double)phi[z * nn + ((y - 1) & m) * n + x]) * hn;
    const double gz = ((double)phi[((z + 1) & m) * nn + y * n + x] - (double)phi[((z - 1) & m) * nn + y * n + x]) * hn;
    acc += gx * gx + gy * gy + gz * gz;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// scal[0] <- rms |grad phi| (FP32), from the partials
__global__ void gradsq_final_kernel(const double* part, int nb, long n3, float* rms) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) rms[0] = (float)sqrt(red[0] / (double)n3);
}

template <typename T>
__global__ __launch_bounds__(256) void features_kernel(const T* __restrict__ n00, const T* __restrict__ phi, int n,
                                                       const double* __restrict__ n00_sum, const float* __restrict__ rms,
                                                       uint16_t* __restrict__ out) {
  const long n3 = (long)n * n * n;
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n3) return;
  const int m = n - 1;
  const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((long)n * n));
  const long nn = (long)n * n;
  const float hn = 0.5f * n;
  const float mean = (float)(n00_sum[0] / (double)n3);
  const float delta = (float)n00[i] / mean - 1.0f;
  const float s = copysignf(log1pf(fabsf(delta)), delta);
  const float ir = 1.0f / rms[0];
  const float gx = (float)(phi[z * nn + y * n + ((x + 1) & m)] - phi[z * nn + y * n + ((x - 1) & m)]) * hn * ir;
  const float gy = (float)(phi[z * nn + ((y + 1) & m) * n + x] - phi[z * nn + ((y - 1) & m) * n + x]) * hn * ir;
  const float gz = (float)(phi[((z + 1) & m) * nn + y * n + x] - phi[((z - 1) & m) * nn + y * n + x]) * hn * ir;
  uint4 a = make_uint4((uint32_t)f2bf(s) | ((uint32_t)f2bf(gx) << 16), (uint32_t)f2bf(gy) | ((uint32_t)f2bf(gz) << 16), 0u, 0u);
  uint4* o = reinterpret_cast<uint4*>(out + i * 16);
  o[0] = a;
  o[1] = make_uint4(0u, 0u, 0u, 0u);
}

// ---------------------------------------------------------------------------
// particle-side helpers: CIC gather of a 3-component FP32 SoA field and its adjoint
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cic(double x, int n, int& i0, int& i1, float& w0, float& w1) {
  const double s = x * (double)n;
  const double fl = floor(s);
  const float f = (float)(s - fl);
  i0 = ((int)fl) & (n - 1);
  i1 = (i0 + 1) & (n - 1);
  w0 = 1.0f - f;
  w1 = f;
}

// CIC interpolation of the 3-component FP32 SoA field f at particle i
template <typename T>
__device__ __forceinline__ void gather3_at(const Particles<T>& p, long i, int n, const float* __restrict__ f,
                                           float v[3]) {
  int x0, x1, y0, y1, z0, z1;
  float wx0, wx1, wy0, wy1, wz0, wz1;
  cic(p.px[i], n, x0, x1, wx0, wx1);
  cic(p.py[i], n, y0, y1, wy0, wy1);
  cic(p.pz[i], n, z0, z1, wz0, wz1);
  const long nn = (long)n * n, n3 = nn * n;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float* g = f + c * n3;
    v[c] = wz0 * (wy0 * (wx0 * g[z0 * nn + y0 * n + x0] + wx1 * g[z0 * nn + y0 * n + x1]) +
                  wy1 * (wx0 * g[z0 * nn + y1 * n + x0] + wx1 * g[z0 * nn + y1 * n + x1])) +
           wz1 * (wy0 * (wx0 * g[z1 * nn + y0 * n + x0] + wx1 * g[z1 * nn + y0 * n + x1]) +
                  wy1 * (wx0 * g[z1 * nn + y1 * n + x0] + wx1 * g[z1 * nn + y1 * n + x1]));
  }
}

template <typename T>
__global__ __launch_bounds__(256) void gather3_kernel(Particles<T> p, long np, int n, const float* __restrict__ f,
                                                      float* __restrict__ out) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  float v[3];
  gather3_at(p, i, n, f, v);
  const long id = p.id[i];
  for (int c = 0; c < 3; ++c) out[3 * id + c] = v[c];
}

// Training residual: pred = gathered network output, r = pred - target (FP32, identifier order),
// dpred = gscale r, and FP64 per-workgroup sums of |r|^2 and |target|^2 (fixed grid, fixed order).
constexpr int LOSS_BLOCKS = 512;
template <typename T>
__global__ __launch_bounds__(256) void loss3_kernel(Particles<T> p, long np, int n, const float* __restrict__ f,
                                                    const float* __restrict__ target, float gscale,
                                                    float* __restrict__ dpred, double* __restrict__ part) {
  __shared__ double red[2][256];
  double e2 = 0.0, t2 = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < np; i += (long)gridDim.x * 256) {
    float v[3];
    gather3_at(p, i, n, f, v);
    const long id = p.id[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float tg = target[3 * id + c];
      const float r = v[c] - tg;
      dpred[3 * id + c] = r * gscale;
      e2 += (double)r * (double)r;
      t2 += (double)tg * (double)tg;
    }
  }
  red[0][threadIdx.x] = e2;
  red[1][threadIdx.x] = t2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
}

// out[0] = mean |r|^2, out[1] = mean |target|^2 over the 3 np components
__global__ __launch_bounds__(256) void loss3_final_kernel(const double* __restrict__ part, int nb, double inv_count,
                                                          double* __restrict__ out) {
  __shared__ double red[2][256];
  double e2 = 0.0, t2 = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    e2 += part[2 * b];
    t2 += part[2 * b + 1];
  }
  red[0][threadIdx.x] = e2;
  red[1][threadIdx.x] = t2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0][0] * inv_count;
    out[1] = red[1][0] * inv_count;
  }
}

// One of the 48 symmetries of the periodic unit cube on particle data: component d of the result
// is component perm[d] of the input, reflected (x -> 1 - x, wrapped into [0, 1)) for positions and
// negated for the two vector fields where flip bit d is set.  Each thread reads its particle before
// writing it, so the outputs may alias the inputs.
__global__ __launch_bounds__(256) void cube_symmetry_kernel(long np, int p0, int p1, int p2, int flip,
                                                            const double* pos, const float* u, const float* v,
                                                            double* pos_out, float* u_out, float* v_out) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  const int perm[3] = {p0, p1, p2};
  double x[3];
  float a[3], b[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    x[d] = pos[3 * i + perm[d]];
    a[d] = u[3 * i + perm[d]];
    b[d] = v[3 * i + perm[d]];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const bool f = (flip >> d) & 1;
    double y = x[d];
    if (f) {
      y = 1.0 - y;
      if (y >= 1.0) y -= 1.0;
    }
    pos_out[3 * i + d] = y;
    u_out[3 * i + d] = f ? -a[d] : a[d];
    v_out[3 * i + d] = f ? -b[d] : b[d];
  }
}

// adjoint of gather3: FP32 atomics into a zeroed SoA field (training sizes only)
template <typename T>
__global__ __launch_bounds__(256) void gather3_adjoint_kernel(Particles<T> p, long np, int n,
                                                              const float* __restrict__ vals, float* __restrict__ f) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  int x0, x1, y0, y1, z0, z1;
  float wx0, wx1, wy0, wy1, wz0, wz1;
  cic(p.px[i], n, x0, x1, wx0, wx1);
  cic(p.py[i], n, y0, y1, wy0, wy1);
  cic(p.pz[i], n, z0, z1, wz0, wz1);
  const long nn = (long)n * n, n3 = nn * n;
  const long id = p.id[i];
  const int zs[2] = {z0, z1}, ys[2] = {y0, y1}, xs[2] = {x0, x1};
  const float wz[2] = {wz0, wz1}, wy[2] = {wy0, wy1}, wx[2] = {wx0, wx1};
  for (int c = 0; c < 3; ++c) {
    const float v = vals[3 * id + c];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int d = 0; d < 2; ++d)
          atomicAdd(&f[c * n3 + zs[a] * nn + ys[b] * n + xs[d]], v * wz[a] * wy[b] * wx[d]);
  }
}

// FP32 SoA [3][n^3] -> bfloat16 [p][16] (channels 3..15 zero)
__global__ __launch_bounds__(256) void soa3_to_bf16_kernel(const float* __restrict__ f, long n3, uint16_t* out) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n3) return;
  uint4 a = make_uint4((uint32_t)f2bf(f[i]) | ((uint32_t)f2bf(f[n3 + i]) << 16), (uint32_t)f2bf(f[2 * n3 + i]), 0u, 0u);
  uint4* o = reinterpret_cast<uint4*>(out + i * 16);
  o[0] = a;
  o[1] = make_uint4(0u, 0u, 0u, 0u);
}

// gradient of phi (centred differences, CIC-interpolated) at the particles, identifier order
template <typename T>
__global__ __launch_bounds__(256) void gather_grad_phi_kernel(Particles<T> p, long np, int n, const T* __restrict__ phi,
                                                              T* __restrict__ out) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  const int m = n - 1;
  const long nn = (long)n * n;
  int ix[2], iy[2], iz[2];
  T wx[2], wy[2], wz[2];
  {
    const double sx = p.px[i] * (double)n, sy = p.py[i] * (double)n, sz = p.pz[i] * (double)n;
    const double fx = floor(sx), fy = floor(sy), fz = floor(sz);
    ix[0] = ((int)fx) & m; iy[0] = ((int)fy) & m; iz[0] = ((int)fz) & m;
    ix[1] = (ix[0] + 1) & m; iy[1] = (iy[0] + 1) & m; iz[1] = (iz[0] + 1) & m;
    wx[1] = (T)(sx - fx); wy[1] = (T)(sy - fy); wz[1] = (T)(sz - fz);
    wx[0] = (T)1 - wx[1]; wy[0] = (T)1 - wy[1]; wz[0] = (T)1 - wz[1];
  }
  T g[3] = {0, 0, 0};
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int c = 0; c < 2; ++c) {
        const int z = iz[a], y = iy[b], x = ix[c];
        const T w = wz[a] * wy[b] * wx[c];
        g[0] += w * (phi[z * nn + y * n + ((x + 1) & m)] - phi[z * nn + y * n + ((x - 1) & m)]);
        g[1] += w * (phi[z * nn + ((y + 1) & m) * n + x] - phi[z * nn + ((y - 1) & m) * n + x]);
        g[2] += w * (phi[((z + 1) & m) * nn + y * n + x] - phi[((z - 1) & m) * nn + y * n + x]);
      }
  const long id = p.id[i];
  const T hn = (T)(0.5 * n);
  for (int d = 0; d < 3; ++d) out[3 * id + d] = g[d] * hn;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
void closure_pack(const float* params, uint16_t* wf, uint16_t* wb, float* bias, hipStream_t st) {
  hipLaunchKernelGGL(pack_weights_kernel, dim3((3 * 27 * 256 + 255) / 256), dim3(256), 0, st, params, wf, wb, bias);
}

void closure_conv(const uint16_t* in, const uint16_t* w, const float* bias, int n, int mode, void* out,
                  const uint16_t* mask, const float* scale, hipStream_t st) {
  dim3 grid(n / CV_TX, n / CV_TY, n / CV_TZ);
  if (mode == 0)
    hipLaunchKernelGGL((conv16_kernel<0>), grid, dim3(CV_NT), 0, st, in, w, bias, n, out, mask, scale);
  else if (mode == 1)
    hipLaunchKernelGGL((conv16_kernel<1>), grid, dim3(CV_NT), 0, st, in, w, bias, n, out, mask, scale);
  else
    hipLaunchKernelGGL((conv16_kernel<2>), grid, dim3(CV_NT), 0, st, in, w, bias, n, out, mask, scale);
}

static long closure_wgrad_tiles(int n) { return (long)(n / CV_TX) * (n / CV_TY) * (n / CV_TZ); }
// workgroups of the weight-gradient kernel: every workgroup takes at least two tiles (so that the
// tile walk runs at every size), at most WG_GRID workgroups
static int closure_wgrad_grid(int n) {
  const long h = closure_wgrad_tiles(n) / 2;
  return (int)(h < 1 ? 1 : (h < WG_GRID ? h : WG_GRID));
}
long closure_wgrad_part_bytes(int n) { return (long)closure_wgrad_grid(n) * WG_PART * 4; }

void closure_wgrad(const uint16_t* x, const uint16_t* dy, int n, float* part, int ci_n, int co_n, float* grad,
                   long off, hipStream_t st) {
  const long tiles = closure_wgrad_tiles(n);
  const int grid = closure_wgrad_grid(n);
  hipLaunchKernelGGL(conv16_wgrad_kernel, dim3(grid), dim3(CV_NT), 0, st, x, dy, n, tiles, part);
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((WG_PART + 63) / 64), dim3(256), 0, st, part, grid, ci_n, co_n, grad,
                     off);
}

void closure_adam(float* p, float* m, float* v, const float* g, int np, double lr, int step, hipStream_t st) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - pow(b1, step)), c2 = (float)(1.0 - pow(b2, step));
  hipLaunchKernelGGL(adam_kernel, dim3((np + 255) / 256), dim3(256), 0, st, p, m, v, g, np, (float)lr, (float)b1,
                     (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, c1, c2);
}

template <typename T>
void closure_features(const T* n00, const T* phi, int n, const double* n00_sum, double* part, float* rms,
                      uint16_t* out, hipStream_t st) {
  const long n3 = (long)n * n * n;
  const int nb = 512;
  hipLaunchKernelGGL((gradsq_partial_kernel<T>), dim3(nb), dim3(256), 0, st, phi, n, part);
  hipLaunchKernelGGL(gradsq_final_kernel, dim3(1), dim3(256), 0, st, part, nb, n3, rms);
  hipLaunchKernelGGL((features_kernel<T>), dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, n00, phi, n, n00_sum,
                     rms, out);
}

template <typename T>
void closure_gather3(const Particles<T>& p, long np, int n, const float* f, float* out, hipStream_t st) {
  hipLaunchKernelGGL((gather3_kernel<T>), dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, p, np, n, f, out);
}

template <typename T>
void closure_loss3(const Particles<T>& p, long np, int n, const float* f, const float* target, float* dpred,
                   double* part, double* out, hipStream_t st) {
  const long want = (np + 255) / 256;
  const int nb = (int)(want < LOSS_BLOCKS ? (want > 0 ? want : 1) : LOSS_BLOCKS);
  const float gscale = (float)(2.0 / (3.0 * (double)np));
  hipLaunchKernelGGL((loss3_kernel<T>), dim3(nb), dim3(256), 0, st, p, np, n, f, target, gscale, dpred, part);
  hipLaunchKernelGGL(loss3_final_kernel, dim3(1), dim3(256), 0, st, part, nb, 1.0 / (3.0 * (double)np), out);
}

void closure_cube_symmetry(long np, const int perm[3], int flip, const double* pos, const float* u, const float* v,
                           double* pos_out, float* u_out, float* v_out, hipStream_t st) {
  hipLaunchKernelGGL(cube_symmetry_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, np, perm[0], perm[1],
                     perm[2], flip, pos, u, v, pos_out, u_out, v_out);
}

template <typename T>
void closure_gather3_adjoint(const Particles<T>& p, long np, int n, const float* vals, float* f, hipStream_t st) {
  hipLaunchKernelGGL((gather3_adjoint_kernel<T>), dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, p, np, n, vals,
                     f);
}

void closure_soa3_to_bf16(const float* f, long n3, uint16_t* out, hipStream_t st) {
  hipLaunchKernelGGL(soa3_to_bf16_kernel, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, f, n3, out);
}

template <typename T>
void gather_grad_phi(const Particles<T>& p, long np, int n, const T* phi, T* out, hipStream_t st) {
  hipLaunchKernelGGL((gather_grad_phi_kernel<T>), dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, p, np, n, phi,
                     out);
}

#define GPM_CL_INST(T)                                                                                          \
  template void closure_features<T>(const T*, const T*, int, const double*, double*, float*, uint16_t*, hipStream_t); \
  template void closure_gather3<T>(const Particles<T>&, long, int, const float*, float*, hipStream_t);          \
  template void closure_gather3_adjoint<T>(const Particles<T>&, long, int, const float*, float*, hipStream_t);  \
  template void closure_loss3<T>(const Particles<T>&, long, int, const float*, const float*, float*, double*,     \
                                 double*, hipStream_t);                                                          \
  template void gather_grad_phi<T>(const Particles<T>&, long, int, const T*, T*, hipStream_t);
GPM_CL_INST(float)
GPM_CL_INST(double)

}  // namespace gpm
