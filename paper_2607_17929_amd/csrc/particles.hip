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
// ingest: [n][3] inputs -> SoA, wrap, validate, rank within the cell
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void ingest_kernel(const double* pos, const T* u, const uint32_t* ids, long np,
                                                     Particles<T> out, int nmesh, uint32_t* rank, uint32_t* cnt,
                                                     int* err) {
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
  rank[i] = atomicAdd(&cnt[k], 1u);
}

template <typename T>
void launch_ingest(const double* pos_aos, const T* u_aos, const uint32_t* ids, long n, Particles<T> out, int nmesh,
                   uint32_t* rank, uint32_t* cnt, int* err, hipStream_t st) {
  hipLaunchKernelGGL((ingest_kernel<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pos_aos, u_aos, ids, n,
                     out, nmesh, rank, cnt, err);
}

// ---------------------------------------------------------------------------
// CIC deposit without atomics, streamed along z.  A workgroup owns a column of
// TX x TY vertices (x, y) over zb vertex planes and walks the cell planes
// z0 - 1 .. z0 + zb - 1 in order.  The particles of one cell plane that touch
// the column -- TY + 1 cell rows, each the halo cell x0 - 1 and the cells
// x0 .. x0 + TX - 1, i.e. two contiguous ranges of the cell-sorted store -- are
// staged in LDS (cell fractions, energy, momentum and the stresses u_i u_j / e),
// and each thread, owning one vertex column, sums the contributions of the
// particles of its 4 cells of the plane in one loop over both cell rows:
// weight (1 - f_z) to the vertex on the plane's lower face, f_z to the one on
// its upper face.  A vertex plane is complete after the cell planes below and
// above it and is stored then, so every cell plane is read once per column.
// While a plane is summed, the particles of the next plane are being loaded
// into registers and the cell offsets of the plane after the next one too (row
// offsets of the staged lists are scanned in LDS, three planes in flight).
// Only cell_start and the particle arrays are read; each vertex is written once.
// ---------------------------------------------------------------------------
constexpr int DEP_NT = 256;                  // one vertex column per thread
template <typename T> constexpr int dep_cap() { return sizeof(T) == 4 ? 512 : 256; }  // staged particles per chunk
constexpr int DEP_ZB = 16;                   // vertex planes per workgroup (fewer on small meshes)

__host__ __device__ constexpr int dep_tx(int n) { return n >= 32 ? 32 : 16; }

// exclusive prefix of c over the first wave's lanes (R <= 64 rows): off[0] = 0, off[r + 1] = sum_{q <= r} c_q
template <int R>
__device__ __forceinline__ void wave_row_offsets(uint32_t c, uint32_t* off) {
  const int lane = threadIdx.x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(c, d);
    if (lane >= d) c += t;
  }
  if (lane < R) off[lane + 1] = c;
  if (lane == 0) off[0] = 0;
}

// largest r in [0, R) with off[r] <= i, for a non-decreasing off with off[0] = 0 <= i (R <= 64)
template <int R>
__device__ __forceinline__ int row_of(const uint32_t* off, uint32_t i) {
  int lo = 0;
#pragma unroll
  for (int step = 32; step > 0; step >>= 1)
    if (step < R && lo + step < R && off[lo + step] <= i) lo += step;
  return lo;
}

// One particle in registers (loaded for the next plane while the current one is summed).
template <typename T>
struct DepPart {
  double x, y, z;
  T ux, uy, uz;
};

template <typename T, int NC, bool REL, int TX>
__global__ __launch_bounds__(DEP_NT) void deposit_kernel(Particles<T> p, const uint32_t* __restrict__ cell_start, int n,
                                                         int zb, T a, double a64, T w, double wd, int accumulate,
                                                         T* __restrict__ dep, double* __restrict__ esum) {
  constexpr int TY = DEP_NT / TX, ROWS = TY + 1, RW = TX + 3;  // raw offsets per row: halo start/end, x0 .. x0 + TX
  constexpr int CAP = dep_cap<T>(), SPT = CAP / DEP_NT;
  constexpr int NQ = (ROWS * RW + DEP_NT - 1) / DEP_NT;
  constexpr int N4 = NC < 4 ? NC : 4, N6 = NC > 4 ? NC - 4 : 1;
  constexpr int WX = TX >= 16 ? 16 : TX, WY = 64 / WX;         // a wave's vertex columns: WX x WY
  static_assert(ROWS <= 64 && CAP % DEP_NT == 0 && TX % WX == 0 && TY % WY == 0, "tile shape");
  constexpr int C4 = NC > 1 ? CAP : 1;
  __shared__ V4<T> sfr[CAP];                  // f_x, f_y, f_z, -
  __shared__ V4<T> sq[C4], ss[C4];            // (e, u_x, u_y, u_z), (u_x u_x, u_x u_y, u_x u_z, u_y u_y) / e
  __shared__ T ss2[C4][2];                    // (u_y u_z, u_z u_z) / e
  __shared__ uint32_t raw[3][ROWS][RW];       // cell offsets of the planes in flight (plane mod 3)
  __shared__ uint32_t roff[3][ROWS + 1];      // staged offset of each row
  __shared__ double red[DEP_NT / 64];
  const int m = n - 1;
  int bx, by, bz;
  xcd_block3(bx, by, bz);
  const int x0 = bx * TX, y0 = by * TY, zs = bz * zb;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // waves of WX x WY vertex columns (the clustered occupancy is less uneven over squarer patches)
  const int lvx = (wave % (TX / WX)) * WX + lane % WX, lvy = (wave / (TX / WX)) * WY + lane / WX;
  const long nn = (long)n * n, n3 = nn * n;

  // raw cell offsets of cell plane cz: row r is cell row y0 - 1 + r; entry 0/1 = start/end of the
  // halo cell x0 - 1, entry 2 + j = start of cell x0 + j (j = 0 .. TX)
  auto load_raw = [&](int cz, uint32_t* v) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const int q = tid + k * DEP_NT;
      if (q < ROWS * RW) {
        const int r = q / RW, j = q - r * RW;
        const uint32_t rb = ((uint32_t)(cz & m) * (uint32_t)n + (uint32_t)((y0 - 1 + r) & m)) * (uint32_t)n;
        const uint32_t hc = rb + (uint32_t)((x0 - 1) & m);
        v[k] = cell_start[j == 0 ? hc : (j == 1 ? hc + 1 : rb + x0 + (j - 2))];
      }
    }
  };
  auto store_raw = [&](int b, const uint32_t* v) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const int q = tid + k * DEP_NT;
      if (q < ROWS * RW) raw[b][q / RW][q % RW] = v[k];
    }
  };
  // staged offsets of the rows of the plane in buffer b (first wave)
  auto scan_rows = [&](int b) {
    if (tid < 64) {
      uint32_t c = 0;
      if (tid < ROWS) c = (raw[b][tid][1] - raw[b][tid][0]) + (raw[b][tid][2 + TX] - raw[b][tid][2]);
      wave_row_offsets<ROWS>(c, roff[b]);
    }
  };
  // global index of staged particle i of the plane in buffer b; own: in a cell of this column
  auto source_of = [&](int b, uint32_t i, bool& own) {
    const int r = row_of<ROWS + 1>(roff[b], i);
    const uint32_t k = i - roff[b][r];
    const uint32_t hs = raw[b][r][0], hn = raw[b][r][1] - hs;
    own = r > 0 && k >= hn;
    return k < hn ? hs + k : raw[b][r][2] + (k - hn);
  };
  auto load_part = [&](uint32_t g, DepPart<T>& d) {
    d.x = p.px[g]; d.y = p.py[g]; d.z = p.pz[g];
    if constexpr (NC > 1) { d.ux = p.ux[g]; d.uy = p.uy[g]; d.uz = p.uz[g]; }
  };
  double e_own = 0.0;
  auto stage = [&](uint32_t l, const DepPart<T>& d, bool own) {
    const double sx = d.x * (double)n, sy = d.y * (double)n, sz = d.z * (double)n;
    V4<T> fr;
    fr.x = (T)(sx - floor(sx));
    fr.y = (T)(sy - floor(sy));
    fr.z = (T)(sz - floor(sz));
    fr.w = (T)0;
    sfr[l] = fr;
    if constexpr (NC > 1) {
      const T vx = d.ux, vy = d.uy, vz = d.uz;
      const T u2 = vx * vx + vy * vy + vz * vz;
      const T e = REL ? sqrt(a * a + u2) : a;
      const T ie = rcp(e);
      V4<T> q, t;
      q.x = e; q.y = vx; q.z = vy; q.w = vz;
      const T ix = vx * ie, iy = vy * ie;
      t.x = ix * vx; t.y = ix * vy; t.z = ix * vz; t.w = iy * vy;
      sq[l] = q;
      ss[l] = t;
      ss2[l][0] = iy * vz;
      ss2[l][1] = vz * ie * vz;
      // FP64 sum over the particles of this column's own cells (the homogeneous source of phi is its
      // small difference from the background, so e is formed from the momenta in FP64 here)
      if (own) {
        const double dx = vx, dy = vy, dz = vz;
        e_own += REL ? sqrt(a64 * a64 + dx * dx + dy * dy + dz * dz) : a64;
      }
    }
  };

  // sums of the vertex on the current plane's lower face (lo) and upper face (hi): n00 and n0i in FP64
  // (each product w q in T), the stresses in T.  The lagged time derivative of phi is the change
  // between two solves, which would otherwise carry the independent rounding of two FP32 sums over a
  // crowded cell amplified by |phi| / |phi_n - phi_{n-1}|.
  double lo4[N4], hi4[N4];
  T lo6[N6], hi6[N6];
#pragma unroll
  for (int c = 0; c < N4; ++c) lo4[c] = hi4[c] = 0.0;
#pragma unroll
  for (int c = 0; c < N6; ++c) lo6[c] = hi6[c] = (T)0;

  // sum the staged particles [c0, c1) of the plane in buffer b: the thread's cells are, in the cell
  // rows lvy (below the vertex: weight f_y) and lvy + 1 (1 - f_y), the local cells lvx (x0 + lvx - 1,
  // weight f_x) and lvx + 1 (1 - f_x), one contiguous staged range per row
  auto accumulate_chunk = [&](int b, uint32_t c0, uint32_t c1) {
    uint32_t beg[2], spl[2], len[2];
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
      const int r = lvy + dy;
      const uint32_t* rr = raw[b][r];
      const uint32_t hn = rr[1] - rr[0], m0 = rr[2], ro = roff[b][r];
      const uint32_t s0 = ro + (lvx == 0 ? 0u : hn + (rr[1 + lvx] - m0));
      const uint32_t s1 = ro + hn + (rr[2 + lvx] - m0);
      const uint32_t s2 = ro + hn + (rr[3 + lvx] - m0);
      const uint32_t bb = max(s0, c0), ee = min(s2, c1);
      beg[dy] = bb - c0;
      spl[dy] = s1 > c0 ? s1 - c0 : 0u;
      len[dy] = ee > bb ? ee - bb : 0u;
    }
    const uint32_t tot = len[0] + len[1];
    for (uint32_t j = 0; j < tot; ++j) {
      const bool r1 = j >= len[0];
      const uint32_t l = r1 ? beg[1] + (j - len[0]) : beg[0] + j;
      const V4<T> fr = sfr[l];
      const T wx = l < (r1 ? spl[1] : spl[0]) ? fr.x : (T)1 - fr.x;
      const T wy = r1 ? (T)1 - fr.y : fr.y;
      const T wxy = wx * wy;
      const T wh = wxy * fr.z, wl = wxy - wh;  // f_z and (1 - f_z) shares
      if constexpr (NC == 1) {
        lo4[0] += (double)(wl * a);
        hi4[0] += (double)(wh * a);
      } else {
        const V4<T> q = sq[l], t = ss[l];
        const T t4 = ss2[l][0], t5 = ss2[l][1];
        const double dl = (double)wl, dh = (double)wh;
        const double q0 = (double)q.x, q1 = (double)q.y, q2 = (double)q.z, q3 = (double)q.w;
        lo4[0] = fma(dl, q0, lo4[0]); lo4[1] = fma(dl, q1, lo4[1]);
        lo4[2] = fma(dl, q2, lo4[2]); lo4[3] = fma(dl, q3, lo4[3]);
        hi4[0] = fma(dh, q0, hi4[0]); hi4[1] = fma(dh, q1, hi4[1]);
        hi4[2] = fma(dh, q2, hi4[2]); hi4[3] = fma(dh, q3, hi4[3]);
        lo6[0] += wl * t.x; lo6[1] += wl * t.y; lo6[2] += wl * t.z;
        lo6[3] += wl * t.w; lo6[4] += wl * t4; lo6[5] += wl * t5;
        hi6[0] += wh * t.x; hi6[1] += wh * t.y; hi6[2] += wh * t.z;
        hi6[3] += wh * t.w; hi6[4] += wh * t4; hi6[5] += wh * t5;
      }
    }
  };

  // prologue: offsets of the first three planes, row offsets of the first two, the first plane's
  // particles in flight
  {
    uint32_t v[NQ];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      if (q <= zb) {
        load_raw(zs - 1 + q, v);
        store_raw(q, v);
      }
    }
  }
  __syncthreads();
  scan_rows(0);
  scan_rows(1);
  __syncthreads();
  DepPart<T> pr[SPT];
  bool pown[SPT];
  {
    const uint32_t lim = min(roff[0][ROWS], (uint32_t)CAP);
#pragma unroll
    for (int s2 = 0; s2 < SPT; ++s2) {
      const uint32_t i = tid + s2 * DEP_NT;
      if (i < lim) {
        bool own;
        load_part(source_of(0, i, own), pr[s2]);
      }
      pown[s2] = false;  // the first plane is below the column's own cells
    }
  }
  uint32_t rnext[NQ];
  for (int P = 0; P <= zb; ++P) {
    const int b = P % 3, b1 = (P + 1) % 3, b2 = (P + 2) % 3;
    const int cz = zs - 1 + P;
    const uint32_t total = roff[b][ROWS];
    // 1. the prefetched first chunk of this plane into LDS
    {
      const uint32_t lim = min(total, (uint32_t)CAP);
#pragma unroll
      for (int s2 = 0; s2 < SPT; ++s2) {
        const uint32_t i = tid + s2 * DEP_NT;
        if (i < lim) stage(i, pr[s2], pown[s2]);
      }
    }
    __syncthreads();
    // 2. requests for the next planes: particles of plane P + 1, cell offsets of plane P + 3
    if (P + 1 <= zb) {
      const uint32_t lim = min(roff[b1][ROWS], (uint32_t)CAP);
#pragma unroll
      for (int s2 = 0; s2 < SPT; ++s2) {
        const uint32_t i = tid + s2 * DEP_NT;
        pown[s2] = false;
        if (i < lim) load_part(source_of(b1, i, pown[s2]), pr[s2]);
      }
    }
    if (P + 3 <= zb) load_raw(cz + 3, rnext);
    // 3. sum this plane: (1 - f_z) to vertex plane cz, f_z to vertex plane cz + 1 (the first plane's
    //    lower-face sums and the last plane's upper-face sums belong to other columns and are dropped)
    accumulate_chunk(b, 0, min(total, (uint32_t)CAP));
    for (uint32_t c0 = CAP; c0 < total; c0 += CAP) {
      // a crowded plane: further chunks loaded and summed in turn
      const uint32_t c1 = min(total, c0 + (uint32_t)CAP);
      __syncthreads();
#pragma unroll
      for (int s2 = 0; s2 < SPT; ++s2) {
        const uint32_t i = c0 + tid + s2 * DEP_NT;
        if (i < c1) {
          bool own;
          DepPart<T> d;
          load_part(source_of(b, i, own), d);
          stage(i - c0, d, own && P > 0);
        }
      }
      __syncthreads();
      accumulate_chunk(b, c0, c1);
    }
    // 4. vertex plane cz is complete: store it and move the upper-face sums down
    if (P > 0) {
      const long o = ((long)cz * n + (y0 + lvy)) * n + (x0 + lvx);
      if (accumulate) {
        // a further species: its sums, weighted by its particle mass over the first species', are added
#pragma unroll
        for (int c = 0; c < N4; ++c) dep[c * n3 + o] = (T)((double)dep[c * n3 + o] + wd * lo4[c]);
#pragma unroll
        for (int c = 4; c < NC; ++c) dep[c * n3 + o] += w * lo6[c - 4];
      } else {
#pragma unroll
        for (int c = 0; c < N4; ++c) dep[c * n3 + o] = (T)lo4[c];
#pragma unroll
        for (int c = 4; c < NC; ++c) dep[c * n3 + o] = lo6[c - 4];
      }
    }
#pragma unroll
    for (int c = 0; c < N4; ++c) { lo4[c] = hi4[c]; hi4[c] = 0.0; }
#pragma unroll
    for (int c = 0; c < N6; ++c) { lo6[c] = hi6[c]; hi6[c] = (T)0; }
    __syncthreads();
    // 5. row offsets of plane P + 2; the cell offsets of plane P + 3 replace this plane's
    if (P + 2 <= zb) scan_rows(b2);
    if (P + 3 <= zb) store_raw(b, rnext);
  }
  if (esum) {
    // fixed-order reduction: within each wave, then the waves' sums in order
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) e_own += __shfl_down(e_own, d);
    if (lane == 0) red[wave] = e_own;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < DEP_NT / 64; ++w2) t += red[w2];
      esum[(bz * gridDim.y + by) * gridDim.x + bx] = wd * t;
    }
  }
}

static int dep_zb(int n) { return n < DEP_ZB ? n : DEP_ZB; }

int deposit_blocks(int n) {
  const int tx = dep_tx(n), ty = DEP_NT / tx;
  return (n / tx) * (n / ty) * (n / dep_zb(n));
}

template <typename T, int TX>
static void launch_deposit_tx(const Particles<T>& p, const uint32_t* cell_start, int n, int ncomp, bool relativistic,
                              double a, double weight, bool accumulate, T* dep, double* esum_part, hipStream_t st) {
  constexpr int TY = DEP_NT / TX;
  const int zb = dep_zb(n);
  dim3 grid(n / TX, n / TY, n / zb);
  const int acc = accumulate ? 1 : 0;
  if (ncomp == 1) {
    hipLaunchKernelGGL((deposit_kernel<T, 1, false, TX>), grid, dim3(DEP_NT), 0, st, p, cell_start, n, zb, (T)a, a,
                       (T)weight, weight, acc, dep, (double*)nullptr);
    return;
  }
  if (relativistic)
    hipLaunchKernelGGL((deposit_kernel<T, 10, true, TX>), grid, dim3(DEP_NT), 0, st, p, cell_start, n, zb, (T)a, a,
                       (T)weight, weight, acc, dep, esum_part);
  else
    hipLaunchKernelGGL((deposit_kernel<T, 10, false, TX>), grid, dim3(DEP_NT), 0, st, p, cell_start, n, zb, (T)a, a,
                       (T)weight, weight, acc, dep, esum_part);
}

template <typename T>
void launch_deposit(const Particles<T>& p, const uint32_t* cell_start, int n, int ncomp, bool relativistic, double a,
                    double weight, bool accumulate, T* dep, double* esum_part, hipStream_t st) {
  if (dep_tx(n) == 32)
    launch_deposit_tx<T, 32>(p, cell_start, n, ncomp, relativistic, a, weight, accumulate, dep, esum_part, st);
  else
    launch_deposit_tx<T, 16>(p, cell_start, n, ncomp, relativistic, a, weight, accumulate, dep, esum_part, st);
}

// ---------------------------------------------------------------------------
// gather + kick + drift + rank in the new cell.  A workgroup takes the particles of a
// TX x TY x TZ block of cells (TY*TZ contiguous row ranges of the sorted
// store) and first copies the fields it needs -- the block's vertices plus a
// margin of one below and two above, enough for the centred differences at
// the 8 corners of every cell -- into LDS.  Each particle then interpolates
// phi, chi, B and their centred-difference gradients from LDS (the CIC
// interpolation of the vertex gradients, written out per corner), kicks, drifts
// and takes its rank inside its new cell (the sort recomputes the cell from
// the stored position).
// ---------------------------------------------------------------------------
// Blocks are TX x TY x TZ cells with TX = 32 (16 on a 16^3 mesh): rows of 32 cells keep the
// row segments of the 4-byte particle arrays at whole 128-byte lines more often.  FP32: 32x4x8
// cells and 512 threads (the field tile is 2.6 values per cell of the block).  FP64: 32x2x4 cells
// and 256 threads: its 152 VGPRs allow 12 waves per CU, three such workgroups (measured at 512^3:
// 8.5 ms against 9.6 ms for 32x4x8 with 512 threads, whose 108 KB tile holds one per CU).
template <typename T> struct KdShape { static constexpr int TY = 4, TZ = 8, NT = 512; };
template <> struct KdShape<double> { static constexpr int TY = 2, TZ = 4, NT = 256; };
template <typename T, int TX> struct KdTile {
  static constexpr int GX = TX + 3, GY = KdShape<T>::TY + 3, GZ = KdShape<T>::TZ + 3, G = GX * GY * GZ;
};

template <typename T, int GX, int GY>
__device__ __forceinline__ void gather_lds(const T* __restrict__ f, int zo0, int yo0, int xo0, const T* wx, const T* wy,
                                           const T* wz, T half_n, T& val, T* g) {
  // f: LDS tile with x stride 1, y stride GX, z stride GX*GY whose index 0 is the vertex one
  // below the block in every axis; (xo0, yo0, zo0) = the particle's cell relative to the block, so the
  // cell's lower corner is tile index (xo0 + 1, yo0 + 1, zo0 + 1)
  T v = 0, gx = 0, gy = 0, gz = 0;
  constexpr int SY = GX, SZ = GX * GY;
#pragma unroll
  for (int cz = 0; cz < 2; ++cz) {
#pragma unroll
    for (int cy = 0; cy < 2; ++cy) {
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) {
        const T w = wx[cx] * wy[cy] * wz[cz];
        const int b = (zo0 + cz + 1) * SZ + (yo0 + cy + 1) * SY + (xo0 + cx + 1);
        v += w * f[b];
        gx += w * (f[b + 1] - f[b - 1]);
        gy += w * (f[b + SY] - f[b - SY]);
        gz += w * (f[b + SZ] - f[b - SZ]);
      }
    }
  }
  val = v;
  g[0] = gx * half_n;
  g[1] = gy * half_n;
  g[2] = gz * half_n;
}

// Rank of a particle among those that reach the same cell.  The store is
// sorted by cell and few particles change cell in a step, so equal keys mostly
// sit in consecutive lanes: each such run of the wave takes its slots with one
// atomicAdd of its length (one per run instead of one per particle, which
// serialises on the counter of a crowded cell).  Call with the active lanes in
// lockstep; every key gets a distinct rank in [0, final count of its cell).
__device__ __forceinline__ uint32_t rank_in_cell(uint32_t* cnt, uint32_t k) {
  const int lane = (int)__lane_id();
  const uint64_t act = __ballot(1);
  const uint32_t kp = __shfl_up(k, 1);
  const bool joins_prev = lane > 0 && ((act >> (lane - 1)) & 1ull) && kp == k;
  const uint64_t heads = __ballot(!joins_prev);
  const uint64_t upto = (2ull << lane) - 1ull;  // lanes 0 .. lane (all ones for lane 63)
  const int head = 63 - __clzll((long long)(heads & upto));
  const uint64_t after = (heads | ~act) & ~upto;  // run boundaries above this lane
  const int next = after ? __ffsll((long long)after) - 1 : 64;
  uint32_t base = 0;
  if (head == lane) base = atomicAdd(&cnt[k], (uint32_t)(next - head));
  base = __shfl(base, head);
  return base + (uint32_t)(lane - head);
}

template <typename T, int MODE, int TX>
__global__ __launch_bounds__(KdShape<T>::NT) void kick_drift_kernel(Particles<T> p,
                                                                    const uint32_t* __restrict__ cell_start, int n,
                                                                    GatherArgs<T> ga, uint32_t* rank, uint32_t* cnt,
                                                                    int* err) {
  constexpr int KD_TY = KdShape<T>::TY, KD_TZ = KdShape<T>::TZ, KD_NT = KdShape<T>::NT;
  constexpr int NF = MODE == MODE_FULL ? 5 : (MODE == MODE_SCALAR ? 2 : 1);
  constexpr int NR = KD_TY * KD_TZ;                   // particle rows of the block
  constexpr int KD_GX = KdTile<T, TX>::GX, KD_GY = KdTile<T, TX>::GY, KD_G = KdTile<T, TX>::G;
  constexpr int NTL = (KD_G + KD_NT - 1) / KD_NT;     // tile entries per thread and field
  static_assert(NR <= 64, "row scan in one wave");
  __shared__ T tile[NF][KD_G];
  __shared__ uint32_t rbeg[NR], roff[NR + 1];
  const int m = n - 1;
  int bx, by, bz;
  xcd_block3(bx, by, bz);
  const int x0 = bx * TX, y0 = by * KD_TY, z0 = bz * KD_TZ;
  const int tid = threadIdx.x;
  const long nn = (long)n * n;
  // field tile with periodic wrap: local (gx, gy, gz) <-> global (x0 - 1 + gx, ...), x fastest;
  // every read of the thread is issued before the first is used
  const T* src[5] = {ga.phi, ga.chi, ga.bx, ga.by, ga.bz};
  T tv[NF][NTL];
#pragma unroll
  for (int k = 0; k < NTL; ++k) {
    const int q = tid + k * KD_NT;
    if (q < KD_G) {
      const int gx = q % KD_GX, row = q / KD_GX;
      const int gy = row % KD_GY, gz = row / KD_GY;
      const long o = (long)((z0 - 1 + gz) & m) * nn + (long)((y0 - 1 + gy) & m) * n + ((x0 - 1 + gx) & m);
#pragma unroll
      for (int f = 0; f < NF; ++f) tv[f][k] = src[f][o];
    }
  }
  // particle rows of the block: start of each row in the sorted store and the prefix of their lengths
  if (tid < 64) {
    uint32_t c = 0;
    if (tid < NR) {
      const int ly = tid % KD_TY, lz = tid / KD_TY;
      const long rb = ((long)(z0 + lz) * n + (y0 + ly)) * n;
      const uint32_t b = cell_start[rb + x0], e = cell_start[rb + x0 + TX];
      rbeg[tid] = b;
      c = e - b;
    }
    wave_row_offsets<NR>(c, roff);
  }
#pragma unroll
  for (int k = 0; k < NTL; ++k) {
    const int q = tid + k * KD_NT;
    if (q < KD_G) {
#pragma unroll
      for (int f = 0; f < NF; ++f) tile[f][q] = tv[f][k];
    }
  }
  __syncthreads();
  const uint32_t total = roff[NR];
  const T hn = (T)(0.5 * n);
  const T dt = (T)ga.dtau;
  const T a = (T)ga.a, ah = (T)ga.a_half;
  // each thread takes particles tid, tid + KD_NT, ...; the next one's state is read while the
  // current one is processed
  uint32_t pin = 0;
  double xn = 0.0, yn = 0.0, zn = 0.0;
  T uxn = 0, uyn = 0, uzn = 0;
  if ((uint32_t)tid < total) {
    const int r = row_of<NR>(roff, tid);
    pin = rbeg[r] + (tid - roff[r]);
    xn = p.px[pin]; yn = p.py[pin]; zn = p.pz[pin];
    uxn = p.ux[pin]; uyn = p.uy[pin]; uzn = p.uz[pin];
  }
  for (uint32_t i = tid; i < total; i += KD_NT) {
    const uint32_t pi = pin;
    double x = xn, y = yn, z = zn;
    T ux = uxn, uy = uyn, uz = uzn;
    const uint32_t inx = i + KD_NT;
    if (inx < total) {
      const int r = row_of<NR>(roff, inx);
      pin = rbeg[r] + (inx - roff[r]);
      xn = p.px[pin]; yn = p.py[pin]; zn = p.pz[pin];
      uxn = p.ux[pin]; uyn = p.uy[pin]; uzn = p.uz[pin];
    }
    int ix, iy, iz;
    double fxd, fyd, fzd;
    cell_of(x, n, ix, fxd);
    cell_of(y, n, iy, fyd);
    cell_of(z, n, iz, fzd);
    const T wx[2] = {(T)1 - (T)fxd, (T)fxd}, wy[2] = {(T)1 - (T)fyd, (T)fyd}, wz[2] = {(T)1 - (T)fzd, (T)fzd};
    const int lx = ix - x0, ly = iy - y0, lz = iz - z0;  // in [0, T*) by construction of the rows
    T phi_p, gphi[3];
    gather_lds<T, KD_GX, KD_GY>(tile[0], lz, ly, lx, wx, wy, wz, hn, phi_p, gphi);
    if (ga.corr) {
      // learned closure: CIC-interpolated correction to grad phi
      const long n3 = nn * n;
      const int xs[2] = {ix, (ix + 1) & m}, ys[2] = {iy, (iy + 1) & m}, zs[2] = {iz, (iz + 1) & m};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float* g = ga.corr + c * n3;
        T acc = 0;
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
          for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
            for (int d2 = 0; d2 < 2; ++d2)
              acc += wz[a2] * wy[b2] * wx[d2] * (T)g[zs[a2] * nn + (long)ys[b2] * n + xs[d2]];
        gphi[c] += acc;
      }
    }
    T vx, vy, vz;
    if constexpr (MODE == MODE_NEWTONIAN) {
      ux -= dt * a * gphi[0];
      uy -= dt * a * gphi[1];
      uz -= dt * a * gphi[2];
      const T ia = rcp(ah);
      vx = ux * ia; vy = uy * ia; vz = uz * ia;
    } else {
      T chi_p, gchi[3];
      gather_lds<T, KD_GX, KD_GY>(tile[1], lz, ly, lx, wx, wy, wz, hn, chi_p, gchi);
      const T u2 = ux * ux + uy * uy + uz * uz;
      const T ie = rsqrt_(a * a + u2);
      const T e = (a * a + u2) * ie;
      const T cphi = -(a * a + (T)2 * u2) * ie;
      T fx = cphi * gphi[0] + e * gchi[0];
      T fy = cphi * gphi[1] + e * gchi[1];
      T fz = cphi * gphi[2] + e * gchi[2];
      T B[3] = {0, 0, 0};
      if constexpr (MODE == MODE_FULL) {
        T gb[3][3];  // gb[j][i] = d_i B_j
        gather_lds<T, KD_GX, KD_GY>(tile[2 % NF], lz, ly, lx, wx, wy, wz, hn, B[0], gb[0]);
        gather_lds<T, KD_GX, KD_GY>(tile[3 % NF], lz, ly, lx, wx, wy, wz, hn, B[1], gb[1]);
        gather_lds<T, KD_GX, KD_GY>(tile[4 % NF], lz, ly, lx, wx, wy, wz, hn, B[2], gb[2]);
        fx -= ux * gb[0][0] + uy * gb[1][0] + uz * gb[2][0];
        fy -= ux * gb[0][1] + uy * gb[1][1] + uz * gb[2][1];
        fz -= ux * gb[0][2] + uy * gb[1][2] + uz * gb[2][2];
      }
      ux += dt * fx;
      uy += dt * fy;
      uz += dt * fz;
      const T v2 = ux * ux + uy * uy + uz * uz;
      const T eh2 = ah * ah + v2;
      const T ieh = rsqrt_(eh2);
      const T fac = ((T)1 + ((T)3 - v2 * ieh * ieh) * phi_p - chi_p) * ieh;
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
    p.px[pi] = x; p.py[pi] = y; p.pz[pi] = z;
    p.ux[pi] = ux; p.uy[pi] = uy; p.uz[pi] = uz;
    rank[pi] = rank_in_cell(cnt, cell_key(x, y, z, n));
  }
}

template <typename T, int TX>
static void launch_kick_drift_tx(const Particles<T>& p, int n, const uint32_t* cell_start, const GatherArgs<T>& g,
                                 uint32_t* rank, uint32_t* cnt, int* err, hipStream_t st) {
  constexpr int KD_NT = KdShape<T>::NT;
  dim3 grid(n / TX, n / KdShape<T>::TY, n / KdShape<T>::TZ);
  if (g.mode == MODE_NEWTONIAN)
    hipLaunchKernelGGL((kick_drift_kernel<T, MODE_NEWTONIAN, TX>), grid, dim3(KD_NT), 0, st, p, cell_start, n, g, rank,
                       cnt, err);
  else if (g.mode == MODE_SCALAR)
    hipLaunchKernelGGL((kick_drift_kernel<T, MODE_SCALAR, TX>), grid, dim3(KD_NT), 0, st, p, cell_start, n, g, rank,
                       cnt, err);
  else
    hipLaunchKernelGGL((kick_drift_kernel<T, MODE_FULL, TX>), grid, dim3(KD_NT), 0, st, p, cell_start, n, g, rank, cnt,
                       err);
}

template <typename T>
void launch_kick_drift(const Particles<T>& p, long np, int n, const uint32_t* cell_start, const GatherArgs<T>& g,
                       uint32_t* rank, uint32_t* cnt, int* err, hipStream_t st) {
  (void)np;
  if (n >= 32)
    launch_kick_drift_tx<T, 32>(p, n, cell_start, g, rank, cnt, err, st);
  else
    launch_kick_drift_tx<T, 16>(p, n, cell_start, g, rank, cnt, err, st);
}

// ---------------------------------------------------------------------------
// exclusive scan of the per-cell counts -> cell_start (n^3 + 1 entries);
// the counts are reset to zero for the next histogram.
// ---------------------------------------------------------------------------
constexpr int SCAN_NT = 256, SCAN_PER = 16, SCAN_CHUNK = SCAN_NT * SCAN_PER;

size_t scan_block_sums_count(long ncell) { return (size_t)((ncell + SCAN_CHUNK - 1) / SCAN_CHUNK); }

// block sums; the order inside a block does not matter, so loads are striped (coalesced)
__global__ __launch_bounds__(SCAN_NT) void scan_reduce_kernel(const uint32_t* cnt, long ncell, uint32_t* bsum) {
  __shared__ uint32_t red[SCAN_NT];
  const long base = (long)blockIdx.x * SCAN_CHUNK + threadIdx.x;
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    const long i = base + (long)j * SCAN_NT;
    if (i < ncell) s += cnt[i];
  }
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

// exclusive scan of one chunk: striped coalesced loads into LDS, per-thread scan of 16
// consecutive values (padded LDS rows), block scan of the thread totals, striped stores
__global__ __launch_bounds__(SCAN_NT) void scan_apply_kernel(uint32_t* cnt, long ncell, const uint32_t* boff,
                                                             uint32_t* cell_start) {
  constexpr int PAD = SCAN_PER + 1;
  __shared__ uint32_t buf[SCAN_NT * PAD];
  __shared__ uint32_t part[SCAN_NT];
  const long base = (long)blockIdx.x * SCAN_CHUNK;
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    const int q = t + j * SCAN_NT;  // element of the chunk
    const long i = base + q;
    buf[(q / SCAN_PER) * PAD + q % SCAN_PER] = (i < ncell) ? cnt[i] : 0u;
    if (i < ncell) cnt[i] = 0u;
  }
  __syncthreads();
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) s += buf[t * PAD + j];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < SCAN_NT; off <<= 1) {
    const uint32_t v = (t >= off) ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = boff[blockIdx.x] + ((t == 0) ? 0u : part[t - 1]);
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    const uint32_t v = buf[t * PAD + j];
    buf[t * PAD + j] = run;
    run += v;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    const int q = t + j * SCAN_NT;
    const long i = base + q;
    if (i < ncell) cell_start[i] = buf[(q / SCAN_PER) * PAD + q % SCAN_PER];
  }
  if (base + SCAN_CHUNK >= ncell && t == SCAN_NT - 1) {
    // the last block also writes the total at cell_start[ncell]
    cell_start[ncell] = boff[blockIdx.x] + part[SCAN_NT - 1];
  }
}

void launch_scan(uint32_t* cnt, uint32_t* cell_start, long ncell, uint32_t* block_sums, hipStream_t st) {
  const long nb = (long)scan_block_sums_count(ncell);
  hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(SCAN_NT), 0, st, cnt, ncell, block_sums);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(1024), 0, st, block_sums, nb);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(SCAN_NT), 0, st, cnt, ncell, block_sums, cell_start);
}

// ---------------------------------------------------------------------------
// scatter into the other buffer at cell_start[cell] + rank; the cell is
// recomputed from the stored position exactly as the kick/drift computed it
// ---------------------------------------------------------------------------
constexpr int SC_PER = 2;  // particles per thread: independent load chains in flight (2 measured best of 2, 4, 8)

template <typename T>
__global__ __launch_bounds__(256) void scatter_kernel(Particles<T> s, Particles<T> d, long np, int nmesh,
                                                      const uint32_t* __restrict__ rank,
                                                      const uint32_t* __restrict__ cell_start) {
  const long base = (long)xcd_remap(blockIdx.x, gridDim.x) * (256 * SC_PER) + threadIdx.x;
  // every read that does not depend on the destination is issued first
  uint32_t r[SC_PER], id[SC_PER];
  double x[SC_PER], y[SC_PER], z[SC_PER];
  T ux[SC_PER], uy[SC_PER], uz[SC_PER];
#pragma unroll
  for (int q = 0; q < SC_PER; ++q) {
    const long i = base + q * 256;
    if (i < np) {
      r[q] = rank[i];
      x[q] = s.px[i]; y[q] = s.py[i]; z[q] = s.pz[i];
      ux[q] = s.ux[i]; uy[q] = s.uy[i]; uz[q] = s.uz[i];
      id[q] = s.id[i];
    }
  }
  long j[SC_PER];
#pragma unroll
  for (int q = 0; q < SC_PER; ++q)
    j[q] = (base + q * 256 < np) ? (long)cell_start[cell_key(x[q], y[q], z[q], nmesh)] + r[q] : 0;
#pragma unroll
  for (int q = 0; q < SC_PER; ++q) {
    if (base + q * 256 < np) {
      d.px[j[q]] = x[q]; d.py[j[q]] = y[q]; d.pz[j[q]] = z[q];
      d.ux[j[q]] = ux[q]; d.uy[j[q]] = uy[q]; d.uz[j[q]] = uz[q];
      d.id[j[q]] = id[q];
    }
  }
}

template <typename T>
void launch_scatter(const Particles<T>& src, Particles<T> dst, long np, int nmesh, const uint32_t* rank,
                    const uint32_t* cell_start, hipStream_t st) {
  const long per_block = 256 * SC_PER;
  hipLaunchKernelGGL((scatter_kernel<T>), dim3((unsigned)((np + per_block - 1) / per_block)), dim3(256), 0, st, src, dst,
                     np, nmesh, rank, cell_start);
}

// ---------------------------------------------------------------------------
// deterministic order inside each cell: after the counting sort the particles of
// a cell sit in the order in which atomic counters handed out their ranks; this
// pass moves each particle to cell_start[cell] + (number of particles of its cell
// with a smaller identifier), so the store -- and every sum over it -- no longer
// depends on that order (identifiers are unique)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void order_by_id_kernel(Particles<T> s, Particles<T> d, long np, int nmesh,
                                                          const uint32_t* __restrict__ cell_start) {
  const long i = (long)xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (i >= np) return;
  const double x = s.px[i], y = s.py[i], z = s.pz[i];
  const T ux = s.ux[i], uy = s.uy[i], uz = s.uz[i];
  const uint32_t id = s.id[i];
  const uint32_t k = cell_key(x, y, z, nmesh);
  const uint32_t b = cell_start[k], e = cell_start[k + 1];
  uint32_t r = 0;
  for (uint32_t j = b; j < e; ++j) r += s.id[j] < id ? 1u : 0u;
  const long o = (long)b + r;
  d.px[o] = x; d.py[o] = y; d.pz[o] = z;
  d.ux[o] = ux; d.uy[o] = uy; d.uz[o] = uz;
  d.id[o] = id;
}

template <typename T>
void launch_order_by_id(const Particles<T>& src, Particles<T> dst, long np, int nmesh, const uint32_t* cell_start,
                        hipStream_t st) {
  hipLaunchKernelGGL((order_by_id_kernel<T>), dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, src, dst, np, nmesh,
                     cell_start);
}

// ---------------------------------------------------------------------------
// consistency check of a restored store (checkpoint bodies are not trusted):
// cell_start[0] = 0, cell_start[n^3] = np, non-decreasing; every particle has
// finite momenta, a position in [0, 1), an identifier < np, and sits inside the
// range of the cell its position falls in.  Any failure sets bit 4 of err.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void check_offsets_kernel(const uint32_t* cell_start, long ncell, long np, int* err) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > ncell) return;
  bool bad = false;
  if (c == 0) bad = cell_start[0] != 0u;
  if (c == ncell) bad = bad || (long)cell_start[ncell] != np;
  if (c < ncell) bad = bad || cell_start[c] > cell_start[c + 1];
  if (bad) atomicOr(err, 4);
}

template <typename T>
__global__ __launch_bounds__(256) void check_store_kernel(Particles<T> p, long np, int nmesh,
                                                          const uint32_t* cell_start, int* err) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const double x = p.px[i], y = p.py[i], z = p.pz[i];
  const T ux = p.ux[i], uy = p.uy[i], uz = p.uz[i];
  bool ok = isfinite(ux) && isfinite(uy) && isfinite(uz);
  ok = ok && x >= 0.0 && x < 1.0 && y >= 0.0 && y < 1.0 && z >= 0.0 && z < 1.0;  // false for NaN
  ok = ok && (long)p.id[i] < np;
  if (ok) {
    const uint32_t k = cell_key(x, y, z, nmesh);
    ok = (long)cell_start[k] <= i && i < (long)cell_start[k + 1];
  }
  if (!ok) atomicOr(err, 4);
}

template <typename T>
void launch_check_store(const Particles<T>& p, long np, int nmesh, const uint32_t* cell_start, int* err,
                        hipStream_t st) {
  const long ncell = (long)nmesh * nmesh * nmesh;
  hipLaunchKernelGGL(check_offsets_kernel, dim3((unsigned)((ncell + 1 + 255) / 256)), dim3(256), 0, st, cell_start,
                     ncell, np, err);
  hipLaunchKernelGGL((check_store_kernel<T>), dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, p, np, nmesh,
                     cell_start, err);
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
                                 uint32_t*, int*, hipStream_t);                                                        \
  template void launch_deposit<T>(const Particles<T>&, const uint32_t*, int, int, bool, double, double, bool, T*,     \
                                  double*, hipStream_t);                                                              \
  template void launch_kick_drift<T>(const Particles<T>&, long, int, const uint32_t*, const GatherArgs<T>&, uint32_t*, \
                                     uint32_t*, int*, hipStream_t);                                                    \
  template void launch_scatter<T>(const Particles<T>&, Particles<T>, long, int, const uint32_t*, const uint32_t*,      \
                                  hipStream_t);                                                                        \
  template void launch_export<T>(const Particles<T>&, long, double*, T*, uint32_t*, hipStream_t);                      \
  template void launch_check_store<T>(const Particles<T>&, long, int, const uint32_t*, int*, hipStream_t);            \
  template void launch_order_by_id<T>(const Particles<T>&, Particles<T>, long, int, const uint32_t*, hipStream_t);     \
  template void launch_copy_unpad<T>(const cplx<T>*, int, int, cplx<T>*, bool, hipStream_t);
GPM_INST(float)
GPM_INST(double)

}  // namespace gpm
