// Batched complex FFTs of LDS-resident column tiles (shared by the column passes and the
// fused Fourier-space kernel).
//
// A tile holds C columns of N complex values as [element][column].  Each 1D
// FFT is a Stockham auto-sort radix-8/4/2 transform done in place: every
// thread loads its butterflies' inputs into registers, the workgroup
// synchronises, and the results are written back, so one tile buffer
// suffices.  The first stage may read its inputs straight from global memory
// (column j of element e at gin[e * esin + j]) and the last stage may write
// straight to global memory (gout[e * esout + j]).
#pragma once

#include "common.h"

namespace gpm {

// One stage.  Job j -> column j % C (fastest, so a wave touches consecutive
// words), butterfly index j / C.
// IX: index type of the global offsets (32-bit unless the arrays exceed 2^32 elements).
// TWPOW: read one twiddle W^k per butterfly and form W^(r k), r = 2 .. R-1, by products (for a
// table in global memory: one load instead of R - 1; at most three roundings deep).
// NTG: the global reads and writes carry the non-temporal hint (streamed data that is not read again
// soon; measured faster for the plain column passes, slower for the fused Fourier-space kernel).
template <typename T, int R, bool INV>
__device__ __forceinline__ void twiddle_pow(cplx<T>* v, cplx<T> w1) {
  cplx<T> w[8];
  w[1] = w1;
  if (R > 2) { w[2] = cmul(w1, w1); w[3] = cmul(w[2], w1); }
  if (R > 4) { w[4] = cmul(w[2], w[2]); w[5] = cmul(w[4], w1); w[6] = cmul(w[3], w[3]); w[7] = cmul(w[4], w[3]); }
#pragma unroll
  for (int r = 1; r < R; ++r) v[r] = INV ? cmulc(v[r], w[r]) : cmul(v[r], w[r]);
}

template <typename T>
__device__ __forceinline__ cplx<T> load_nt(const cplx<T>* p) {
  const T* q = reinterpret_cast<const T*>(p);
  return mk<T>(__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1));
}
template <typename T>
__device__ __forceinline__ void store_nt(cplx<T>* p, cplx<T> v) {
  T* q = reinterpret_cast<T*>(p);
  __builtin_nontemporal_store(v.x, q);
  __builtin_nontemporal_store(v.y, q + 1);
}

template <typename T, int N, int C, int NT, int S, bool INV, bool FROM_G, bool TO_G, typename IX, bool TWPOW = false,
          bool NTG = false>
__device__ __forceinline__ void col_stage(cplx<T>* sm, const cplx<T>* gin, IX esin, cplx<T>* gout, IX esout,
                                          const cplx<T>* stw) {
  constexpr int R = stage_radix(N, S);
  constexpr int NS = stage_ns(N, S);
  constexpr int J = N * C / R;
  constexpr int PER = (J + NT - 1) / NT;
  const int tid = threadIdx.x;
  cplx<T> v[PER][R];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int job = tid + p * NT;
    if (J % NT == 0 || job < J) {
      const int col = job % C, i = job / C;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = i + r * (N / R);
        if (FROM_G) {
          v[p][r] = NTG ? load_nt(gin + ((IX)e * esin + (IX)col)) : gin[(IX)e * esin + (IX)col];
        } else {
          v[p][r] = sm[e * C + col];
        }
      }
    }
  }
  if (!FROM_G) __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int job = tid + p * NT;
    if (J % NT == 0 || job < J) {
      const int col = job % C, i = job / C;
      const int k = i % NS;
      if (NS > 1) {
        if constexpr (TWPOW) {
          twiddle_pow<T, R, INV>(v[p], stw[k * (N / (NS * R))]);
        } else {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            const cplx<T> w = stw[(r * k) * (N / (NS * R))];
            v[p][r] = INV ? cmulc(v[p][r], w) : cmul(v[p][r], w);
          }
        }
      }
      dftR<T, R, INV>(v[p]);
      const int j0 = (i / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = j0 + r * NS;
        if (TO_G) {
          if (NTG) store_nt(gout + ((IX)e * esout + (IX)col), v[p][r]);
          else gout[(IX)e * esout + (IX)col] = v[p][r];
        } else {
          sm[e * C + col] = v[p][r];
        }
      }
    }
  }
  if (!TO_G) __syncthreads();
}

// All stages of the transform; GIN / GOUT: the first stage reads global memory, the last
// stage writes global memory (otherwise the tile starts / ends in LDS).
template <typename T, int N, int C, int NT, int S, bool INV, bool GIN, bool GOUT, typename IX, bool TWPOW = false,
          bool NTG = false>
__device__ __forceinline__ void col_stages(cplx<T>* sm, const cplx<T>* gin, IX esin, cplx<T>* gout, IX esout,
                                           const cplx<T>* stw) {
  constexpr int NSTG = nstages(N);
  if constexpr (S < NSTG) {
    col_stage<T, N, C, NT, S, INV, GIN && S == 0, GOUT && S == NSTG - 1, IX, TWPOW, NTG>(sm, gin, esin, gout, esout,
                                                                                          stw);
    col_stages<T, N, C, NT, S + 1, INV, GIN, GOUT, IX, TWPOW, NTG>(sm, gin, esin, gout, esout, stw);
  }
}

}  // namespace gpm
