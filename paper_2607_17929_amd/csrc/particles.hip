// Particle kernels: ingest, CIC deposit, gather + kick + drift, counting sort by cell.
//
// The particle store is a structure of arrays (x, y, z in FP64; u_x, u_y, u_z
// and the identifier) kept sorted by mesh cell in row-major order
// key = (iz n + iy) n + ix, so that the particles of one x-row of cells are
// contiguous and ordered along x, as in the paper's particle handler
// (Sec. 2.1).  cell_start[key] .. cell_start[key + 1] is the range of a cell.
#include "kernels.h"

namespace gpm {

__device__ __forceinline__ void cell_of(double x, int n, int& i, double& f) {
  // n is a power of two, so x * n is exact in FP64
  const double s = x * (double)n;
  const double fl = floor(s);
  f = s - fl;
  i = ((int)fl) & (n - 1);
}

__device__ __forceinline__ double wrap01(double x) {
  double y = x - floor(x);
  return (y >= 1.0) ? 0.0 : y;
}

__device__ __forceinline__ uint32_t cell_key(double x, double y, double z, int n) {
  int ix, iy, iz;
  double f;
  cell_of(x, n, ix, f);
  cell_of(y, n, iy, f);
  cell_of(z, n, iz, f);
  return ((uint32_t)iz * (uint32_t)n + (uint32_t)iy) * (uint32_t)n + (uint32_t)ix;
}

// ---------------------------------------------------------------------------
// ingest: [n][3] inputs -> SoA, wrap, validate, key and rank within the cell
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void ingest_kernel(const double* pos, const T* u, const uint32_t* ids, long np,
                                                     Particles<T> out, int nmesh, uint32_t* key, uint32_t* rank,
                                                     uint32_t* cnt, int* err) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
  T ux = u[3 * i], uy = u[3 * i + 1], uz = u[3 * i + 2];
  if (!(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(ux) && isfinite(uy) && isfinite(uz))) {
    atomicOr(err, 1);
    x = y = z = 0.0;
    ux = uy = uz = (T)0;
  }
  x = wrap01(x); y = wrap01(y); z = wrap01(z);
  uint32_t id = ids ? ids[i] : (uint32_t)i;
  if ((long)id >= np) {
    atomicOr(err, 2);
    id = 0;
  }
  out.px[i] = x; out.py[i] = y; out.pz[i] = z;
  out.ux[i] = ux; out.uy[i] = uy; out.uz[i] = uz;
  out.id[i] = id;
  const uint32_t k = cell_key(x, y, z, nmesh);
  key[i] = k;
  rank[i] = atomicAdd(&cnt[k], 1u);
}

template <typename T>
void launch_ingest(const double* pos_aos, const T* u_aos, const uint32_t* ids, long n, Particles<T> out, int nmesh,
                   uint32_t* key, uint32_t* rank, uint32_t* cnt, int* err, hipStream_t st) {
  hipLaunchKernelGGL((ingest_kernel<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pos_aos, u_aos, ids, n,
                     out, nmesh, key, rank, cnt, err);
}

// ---------------------------------------------------------------------------
// CIC deposit, owner computes: one workgroup owns a TX x TY x TZ block of
// vertices, accumulates in LDS every particle of the (TX+1)(TY+1)(TZ+1) cells
// that touch it (found through cell_start: each cell row is two contiguous
// particle ranges), and writes its block once with plain stores.  No global
// atomics and no zero-fill of the mesh are needed.
// ---------------------------------------------------------------------------
constexpr int DEP_TX = 16, DEP_TY = 8, DEP_TZ = 8, DEP_NT = 256;
constexpr int DEP_MAXSEG = 2 * (DEP_TY + 1) * (DEP_TZ + 1);

template <typename T, int NC, bool REL>
__global__ __launch_bounds__(DEP_NT) void deposit_kernel(Particles<T> p, const uint32_t* __restrict__ cell_start, int n,
                                                         T a, T* __restrict__ dep, double* __restrict__ esum) {
  extern __shared__ __align__(16) unsigned char dsm[];
  T* acc = reinterpret_cast<T*>(dsm);  // [NC][TZ][TY][TX]
  __shared__ uint32_t seg_begin[DEP_MAXSEG];
  __shared__ uint32_t seg_off[DEP_MAXSEG + 1];
  __shared__ unsigned char seg_own[DEP_MAXSEG];
  __shared__ double red[DEP_NT];
  const int TX = min(DEP_TX, n), TY = min(DEP_TY, n), TZ = min(DEP_TZ, n);
  const int nv = TX * TY * TZ;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
  const int tid = threadIdx.x;
  const int m = n - 1;
  for (int i = tid; i < NC * nv; i += DEP_NT) acc[i] = (T)0;
  // segment table: rows (cy, cz) of cells touching the block
  const int ry = (TY == n) ? TY : TY + 1, ry0 = (TY == n) ? y0 : y0 - 1;
  const int rz = (TZ == n) ? TZ : TZ + 1, rz0 = (TZ == n) ? z0 : z0 - 1;
  const bool halo_x = (TX != n);
  const int nrow = ry * rz;
  const int nseg = nrow * 2;
  if (tid < nseg) {
    const int row = tid >> 1, part = tid & 1;
    const int cy = (ry0 + row % ry) & m, cz = (rz0 + row / ry) & m;
    const uint32_t rowbase = ((uint32_t)cz * n + cy) * (uint32_t)n;
    uint32_t b, e;
    if (part == 0) {  // the halo cell x0 - 1
      if (halo_x) {
        const uint32_t c = rowbase + ((x0 - 1) & m);
        b = cell_start[c];
        e = cell_start[c + 1];
      } else {
        b = e = 0;
      }
    } else {  // cells x0 .. x0 + TX - 1
      b = cell_start[rowbase + x0];
      e = cell_start[rowbase + x0 + TX];
    }
    seg_begin[tid] = b;
    seg_off[tid + 1] = e - b;
    // particles of the block's own cells are counted once in the FP64 energy sum
    const bool own_y = (ry == TY) || (row % ry) != 0;
    const bool own_z = (rz == TZ) || (row / ry) != 0;
    seg_own[tid] = (part == 1 && own_y && own_z) ? 1 : 0;
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t s = 0;
    seg_off[0] = 0;
    for (int i = 1; i <= nseg; ++i) {
      s += seg_off[i];
      seg_off[i] = s;
    }
  }
  __syncthreads();
  const uint32_t total = seg_off[nseg];
  const double ad = (double)a;
  double e_own = 0.0;
  for (uint32_t i = tid; i < total; i += DEP_NT) {
    // segment containing flattened index i
    int lo = 0, hi = nseg;  // seg_off[lo] <= i < seg_off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (seg_off[mid] <= i) lo = mid; else hi = mid;
    }
    const uint32_t pi = seg_begin[lo] + (i - seg_off[lo]);
    int ix, iy, iz;
    double fxd, fyd, fzd;
    cell_of(p.px[pi], n, ix, fxd);
    cell_of(p.py[pi], n, iy, fyd);
    cell_of(p.pz[pi], n, iz, fzd);
    const T fx = (T)fxd, fy = (T)fyd, fz = (T)fzd;
    T q[NC];
    if constexpr (NC == 1) {
      q[0] = a;
    } else {
      const T ux = p.ux[pi], uy = p.uy[pi], uz = p.uz[pi];
      const T e = REL ? sqrt(a * a + ux * ux + uy * uy + uz * uz) : a;
      const T ie = (T)1 / e;
      q[0] = e; q[1] = ux; q[2] = uy; q[3] = uz;
      q[4] = ux * ux * ie; q[5] = ux * uy * ie; q[6] = ux * uz * ie;
      q[7] = uy * uy * ie; q[8] = uy * uz * ie; q[9] = uz * uz * ie;
      if (seg_own[lo]) {
        const double dx = ux, dy = uy, dz = uz;
        e_own += REL ? sqrt(ad * ad + dx * dx + dy * dy + dz * dz) : ad;
      }
    }
    const T wx[2] = {(T)1 - fx, fx}, wy[2] = {(T)1 - fy, fy}, wz[2] = {(T)1 - fz, fz};
#pragma unroll
    for (int cz = 0; cz < 2; ++cz) {
      const int lz = (iz + cz - z0) & m;
      if (lz >= TZ) continue;
#pragma unroll
      for (int cy = 0; cy < 2; ++cy) {
        const int ly = (iy + cy - y0) & m;
        if (ly >= TY) continue;
        const T wyz = wy[cy] * wz[cz];
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
          const int lx = (ix + cx - x0) & m;
          if (lx >= TX) continue;
          const T w = wx[cx] * wyz;
          const int v = (lz * TY + ly) * TX + lx;
#pragma unroll
          for (int c = 0; c < NC; ++c) atomicAdd(&acc[c * nv + v], w * q[c]);
        }
      }
    }
  }
  if (esum) {
    red[tid] = e_own;
    __syncthreads();
    for (int w = DEP_NT / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) esum[(blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
  }
  __syncthreads();
  const long n3 = (long)n * n * n;
  for (int i = tid; i < NC * nv; i += DEP_NT) {
    const int c = i / nv, v = i % nv;
    const int lx = v % TX, ly = (v / TX) % TY, lz = v / (TX * TY);
    dep[c * n3 + ((long)(z0 + lz) * n + (y0 + ly)) * n + (x0 + lx)] = acc[i];
  }
}

template <typename T>
void launch_deposit(const Particles<T>& p, const uint32_t* cell_start, int n, int ncomp, bool relativistic, double a,
                    T* dep, double* esum_part, double* esum, hipStream_t st) {
  const int TX = n < DEP_TX ? n : DEP_TX, TY = n < DEP_TY ? n : DEP_TY, TZ = n < DEP_TZ ? n : DEP_TZ;
  dim3 grid(n / TX, n / TY, n / TZ);
  const size_t shm = (size_t)ncomp * TX * TY * TZ * sizeof(T);
  // the FP64 accumulator (80 KB) exceeds the default dynamic LDS limit
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&deposit_kernel<T, 1, false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&deposit_kernel<T, 10, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&deposit_kernel<T, 10, false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (ncomp == 1) {
    hipLaunchKernelGGL((deposit_kernel<T, 1, false>), grid, dim3(DEP_NT), shm, st, p, cell_start, n, (T)a, dep,
                       (double*)nullptr);
    return;
  }
  if (relativistic)
    hipLaunchKernelGGL((deposit_kernel<T, 10, true>), grid, dim3(DEP_NT), shm, st, p, cell_start, n, (T)a, dep,
                       esum_part);
  else
    hipLaunchKernelGGL((deposit_kernel<T, 10, false>), grid, dim3(DEP_NT), shm, st, p, cell_start, n, (T)a, dep,
                       esum_part);
  launch_sum_f64(esum_part, (long)grid.x * grid.y * grid.z, esum, st);
}

// ---------------------------------------------------------------------------
// gather + kick + drift + new key.  Fields at x^n, CIC-interpolated together
// with their centred-difference gradients (the interpolation of the vertex
// gradients, written out per corner).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void gather_one(const T* __restrict__ f, const long* zo, const long* yo, const int* xo,
                                           const T* wx, const T* wy, const T* wz, T half_n, T& val, T* g) {
  T v = 0, gx = 0, gy = 0, gz = 0;
#pragma unroll
  for (int cz = 0; cz < 2; ++cz) {
#pragma unroll
    for (int cy = 0; cy < 2; ++cy) {
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) {
        const T w = wx[cx] * wy[cy] * wz[cz];
        const int X = cx + 1, Y = cy + 1, Z = cz + 1;
        const long zy = zo[Z] + yo[Y];
        v += w * f[zy + xo[X]];
        gx += w * (f[zy + xo[X + 1]] - f[zy + xo[X - 1]]);
        gy += w * (f[zo[Z] + yo[Y + 1] + xo[X]] - f[zo[Z] + yo[Y - 1] + xo[X]]);
        gz += w * (f[zo[Z + 1] + yo[Y] + xo[X]] - f[zo[Z - 1] + yo[Y] + xo[X]]);
      }
    }
  }
  val = v;
  g[0] = gx * half_n;
  g[1] = gy * half_n;
  g[2] = gz * half_n;
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void kick_drift_kernel(Particles<T> p, long np, int n, GatherArgs<T> ga,
                                                         uint32_t* key, uint32_t* rank, uint32_t* cnt, int* err) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int m = n - 1;
  double x = p.px[i], y = p.py[i], z = p.pz[i];
  int ix, iy, iz;
  double fxd, fyd, fzd;
  cell_of(x, n, ix, fxd);
  cell_of(y, n, iy, fyd);
  cell_of(z, n, iz, fzd);
  const T wx[2] = {(T)1 - (T)fxd, (T)fxd}, wy[2] = {(T)1 - (T)fyd, (T)fyd}, wz[2] = {(T)1 - (T)fzd, (T)fzd};
  const long nn = (long)n * n;
  const long zo[4] = {((iz - 1) & m) * nn, iz * nn, ((iz + 1) & m) * nn, ((iz + 2) & m) * nn};
  const long yo[4] = {(long)((iy - 1) & m) * n, (long)iy * n, (long)((iy + 1) & m) * n, (long)((iy + 2) & m) * n};
  const int xo[4] = {(ix - 1) & m, ix, (ix + 1) & m, (ix + 2) & m};
  const T hn = (T)(0.5 * n);
  T phi_p, gphi[3];
  gather_one(ga.phi, zo, yo, xo, wx, wy, wz, hn, phi_p, gphi);
  T ux = p.ux[i], uy = p.uy[i], uz = p.uz[i];
  const T dt = (T)ga.dtau;
  const T a = (T)ga.a, ah = (T)ga.a_half;
  T vx, vy, vz;
  if constexpr (MODE == MODE_NEWTONIAN) {
    ux -= dt * a * gphi[0];
    uy -= dt * a * gphi[1];
    uz -= dt * a * gphi[2];
    const T ia = (T)1 / ah;
    vx = ux * ia; vy = uy * ia; vz = uz * ia;
  } else {
    T chi_p, gchi[3];
    gather_one(ga.chi, zo, yo, xo, wx, wy, wz, hn, chi_p, gchi);
    const T u2 = ux * ux + uy * uy + uz * uz;
    const T e = sqrt(a * a + u2);
    const T cphi = -(a * a + (T)2 * u2) / e;
    T fx = cphi * gphi[0] + e * gchi[0];
    T fy = cphi * gphi[1] + e * gchi[1];
    T fz = cphi * gphi[2] + e * gchi[2];
    T B[3] = {0, 0, 0};
    if constexpr (MODE == MODE_FULL) {
      T gb[3][3];  // gb[j][i] = d_i B_j
      gather_one(ga.bx, zo, yo, xo, wx, wy, wz, hn, B[0], gb[0]);
      gather_one(ga.by, zo, yo, xo, wx, wy, wz, hn, B[1], gb[1]);
      gather_one(ga.bz, zo, yo, xo, wx, wy, wz, hn, B[2], gb[2]);
      fx -= ux * gb[0][0] + uy * gb[1][0] + uz * gb[2][0];
      fy -= ux * gb[0][1] + uy * gb[1][1] + uz * gb[2][1];
      fz -= ux * gb[0][2] + uy * gb[1][2] + uz * gb[2][2];
    }
    ux += dt * fx;
    uy += dt * fy;
    uz += dt * fz;
    const T v2 = ux * ux + uy * uy + uz * uz;
    const T eh2 = ah * ah + v2;
    const T ieh = (T)1 / sqrt(eh2);
    const T fac = ((T)1 + ((T)3 - v2 / eh2) * phi_p - chi_p) * ieh;
    vx = ux * fac + B[0];
    vy = uy * fac + B[1];
    vz = uz * fac + B[2];
  }
  x += ga.dtau * (double)vx;
  y += ga.dtau * (double)vy;
  z += ga.dtau * (double)vz;
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
    atomicOr(err, 1);
    x = y = z = 0.0;
  }
  x = wrap01(x); y = wrap01(y); z = wrap01(z);
  p.px[i] = x; p.py[i] = y; p.pz[i] = z;
  p.ux[i] = ux; p.uy[i] = uy; p.uz[i] = uz;
  const uint32_t k = cell_key(x, y, z, n);
  key[i] = k;
  rank[i] = atomicAdd(&cnt[k], 1u);
}

template <typename T>
void launch_kick_drift(const Particles<T>& p, long np, int n, const GatherArgs<T>& g, uint32_t* key, uint32_t* rank,
                       uint32_t* cnt, int* err, hipStream_t st) {
  dim3 grid((unsigned)((np + 255) / 256));
  if (g.mode == MODE_NEWTONIAN)
    hipLaunchKernelGGL((kick_drift_kernel<T, MODE_NEWTONIAN>), grid, dim3(256), 0, st, p, np, n, g, key, rank, cnt, err);
  else if (g.mode == MODE_SCALAR)
    hipLaunchKernelGGL((kick_drift_kernel<T, MODE_SCALAR>), grid, dim3(256), 0, st, p, np, n, g, key, rank, cnt, err);
  else
    hipLaunchKernelGGL((kick_drift_kernel<T, MODE_FULL>), grid, dim3(256), 0, st, p, np, n, g, key, rank, cnt, err);
}

// ---------------------------------------------------------------------------
// exclusive scan of the per-cell counts -> cell_start (n^3 + 1 entries);
// the counts are reset to zero for the next histogram.
// ---------------------------------------------------------------------------
constexpr int SCAN_NT = 256, SCAN_PER = 16, SCAN_CHUNK = SCAN_NT * SCAN_PER;

size_t scan_block_sums_count(long ncell) { return (size_t)((ncell + SCAN_CHUNK - 1) / SCAN_CHUNK); }

__global__ __launch_bounds__(SCAN_NT) void scan_reduce_kernel(const uint32_t* cnt, long ncell, uint32_t* bsum) {
  __shared__ uint32_t red[SCAN_NT];
  const long base = (long)blockIdx.x * SCAN_CHUNK + (long)threadIdx.x * SCAN_PER;
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j)
    if (base + j < ncell) s += cnt[base + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = SCAN_NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// single workgroup: exclusive scan of the block sums in place
__global__ __launch_bounds__(1024) void scan_blocks_kernel(uint32_t* bsum, long nb) {
  __shared__ uint32_t part[1024];
  const long per = (nb + 1023) / 1024;
  const long b0 = threadIdx.x * per;
  uint32_t s = 0;
  for (long j = 0; j < per; ++j)
    if (b0 + j < nb) s += bsum[b0 + j];
  part[threadIdx.x] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan of the 1024 partial sums
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t v = (threadIdx.x >= (unsigned)off) ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = (threadIdx.x == 0) ? 0u : part[threadIdx.x - 1];
  for (long j = 0; j < per; ++j) {
    if (b0 + j < nb) {
      const uint32_t v = bsum[b0 + j];
      bsum[b0 + j] = run;
      run += v;
    }
  }
}

__global__ __launch_bounds__(SCAN_NT) void scan_apply_kernel(uint32_t* cnt, long ncell, const uint32_t* boff,
                                                             uint32_t* cell_start) {
  __shared__ uint32_t part[SCAN_NT];
  const long base = (long)blockIdx.x * SCAN_CHUNK + (long)threadIdx.x * SCAN_PER;
  uint32_t v[SCAN_PER];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    v[j] = (base + j < ncell) ? cnt[base + j] : 0u;
    s += v[j];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < SCAN_NT; off <<= 1) {
    const uint32_t t = (threadIdx.x >= (unsigned)off) ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  uint32_t run = boff[blockIdx.x] + ((threadIdx.x == 0) ? 0u : part[threadIdx.x - 1]);
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    if (base + j < ncell) {
      cell_start[base + j] = run;
      cnt[base + j] = 0u;
      run += v[j];
      if (base + j == ncell - 1) cell_start[ncell] = run;
    }
  }
}

void launch_scan(uint32_t* cnt, uint32_t* cell_start, long ncell, uint32_t* block_sums, hipStream_t st) {
  const long nb = (long)scan_block_sums_count(ncell);
  hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(SCAN_NT), 0, st, cnt, ncell, block_sums);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(1024), 0, st, block_sums, nb);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(SCAN_NT), 0, st, cnt, ncell, block_sums, cell_start);
}

// ---------------------------------------------------------------------------
// scatter into the other buffer at cell_start[key] + rank
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void scatter_kernel(Particles<T> s, Particles<T> d, long np,
                                                      const uint32_t* __restrict__ key, const uint32_t* __restrict__ rank,
                                                      const uint32_t* __restrict__ cell_start) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const long j = (long)cell_start[key[i]] + rank[i];
  d.px[j] = s.px[i]; d.py[j] = s.py[i]; d.pz[j] = s.pz[i];
  d.ux[j] = s.ux[i]; d.uy[j] = s.uy[i]; d.uz[j] = s.uz[i];
  d.id[j] = s.id[i];
}

template <typename T>
void launch_scatter(const Particles<T>& src, Particles<T> dst, long np, const uint32_t* key, const uint32_t* rank,
                    const uint32_t* cell_start, hipStream_t st) {
  hipLaunchKernelGGL((scatter_kernel<T>), dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, src, dst, np, key, rank,
                     cell_start);
}

// ---------------------------------------------------------------------------
// export in identifier order as [n][3] arrays
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void export_kernel(Particles<T> p, long np, double* pos, T* u, uint32_t* ids) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const long d = p.id[i];
  if (pos) { pos[3 * d] = p.px[i]; pos[3 * d + 1] = p.py[i]; pos[3 * d + 2] = p.pz[i]; }
  if (u) { u[3 * d] = p.ux[i]; u[3 * d + 1] = p.uy[i]; u[3 * d + 2] = p.uz[i]; }
  if (ids) ids[d] = (uint32_t)d;
}

template <typename T>
void launch_export(const Particles<T>& p, long np, double* pos_aos, T* u_aos, uint32_t* ids, hipStream_t st) {
  hipLaunchKernelGGL((export_kernel<T>), dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, p, np, pos_aos, u_aos,
                     ids);
}

// ---------------------------------------------------------------------------
// padded <-> dense half spectrum copies (diagnostic FFT entry point)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void copy_unpad_kernel(const cplx<T>* a, int n, int nhp, cplx<T>* b, bool to_padded) {
  const int nh = n / 2 + 1;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)n * n * nh) return;
  const int kx = (int)(t % nh);
  const long row = t / nh;
  if (to_padded) {
    const_cast<cplx<T>*>(a)[row * nhp + kx] = b[t];
  } else {
    b[t] = a[row * nhp + kx];
  }
}

template <typename T>
void launch_copy_unpad(const cplx<T>* spec, int n, int nhp, cplx<T>* out, bool to_padded, hipStream_t st) {
  const long total = (long)n * n * (n / 2 + 1);
  hipLaunchKernelGGL((copy_unpad_kernel<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, spec, n, nhp, out,
                     to_padded);
}

#define GPM_INST(T)                                                                                                   \
  template void launch_ingest<T>(const double*, const T*, const uint32_t*, long, Particles<T>, int, uint32_t*,         \
                                 uint32_t*, uint32_t*, int*, hipStream_t);                                             \
  template void launch_deposit<T>(const Particles<T>&, const uint32_t*, int, int, bool, double, T*, double*, double*, \
                                  hipStream_t);                                                                       \
  template void launch_kick_drift<T>(const Particles<T>&, long, int, const GatherArgs<T>&, uint32_t*, uint32_t*,       \
                                     uint32_t*, int*, hipStream_t);                                                    \
  template void launch_scatter<T>(const Particles<T>&, Particles<T>, long, const uint32_t*, const uint32_t*,           \
                                  const uint32_t*, hipStream_t);                                                       \
  template void launch_export<T>(const Particles<T>&, long, double*, T*, uint32_t*, hipStream_t);                      \
  template void launch_copy_unpad<T>(const cplx<T>*, int, int, cplx<T>*, bool, hipStream_t);
GPM_INST(float)
GPM_INST(double)

}  // namespace gpm
