// Host-side declarations of the PM kernels' launchers (one header for all .hip units).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace gpm {

// source assembly modes of the forward pass X (MODE_FULLP: full physics with B from the vector part
// of the space-space equation -- the sources are those of MODE_SCALAR, the solve adds B and h)
enum { MODE_RAW = 0, MODE_NEWTONIAN = 1, MODE_SCALAR = 2, MODE_FULL = 3, MODE_FULLP = 4 };
__host__ __device__ constexpr int mode_nsrc(int mode) {
  return mode == MODE_FULL ? 10 : ((mode == MODE_SCALAR || mode == MODE_FULLP) ? 7 : 1);
}

// host-side (FP64) arguments of the forward transform with source assembly
template <typename T>
struct SrcArgsH {
  const T* dep = nullptr;
  const T* phi1 = nullptr;
  const T* dphi1 = nullptr;  // increment phi_{n-1} - phi_{n-2} of the lagged solve
  const T* chi1 = nullptr;
  const T* raw = nullptr;
  double* rowsum = nullptr;
  double kap = 0, ebar = 0, hc = 0, inv_dt = 0, inv_dtl = 0;
  int incr = 0;              // source of the increment phi_n - phi_{n-1} instead of phi_n
};

// ---- fft.hip ----
// Half spectra of several components are component-interleaved: [z][y][kx][c], rows of nhp kx.
// pass X forward with source assembly: spec gets mode_nsrc(mode) interleaved components
template <typename T>
void fft_r2c_x(const SrcArgsH<T>& a, int mode, int n, int nhp, cplx<T>* spec, const cplx<T>* tw, hipStream_t st);
// column passes over ncomp separate arrays of rows of nhp complex values (an interleaved spectrum
// of c components is one array with rows of c * nhp values)
template <typename T>
void fft_cols(int n, int nhp, cplx<T>* spec, int ncomp, bool inv, bool along_z, const cplx<T>* tw, hipStream_t st);
// pass X inverse of nout interleaved components into separate real arrays; with base0 non-null,
// component 0 is an increment: outp[0] = base0 + value, and the value itself goes to delta0
template <typename T>
void fft_c2r_x(int n, int nhp, const cplx<T>* spec, int nout, T* const* outp, double out_scale, const cplx<T>* tw,
               hipStream_t st, const T* base0 = nullptr, T* delta0 = nullptr);
template <typename T>
void fft_forward(const SrcArgsH<T>& a, int mode, int n, int nhp, cplx<T>* spec, int ncomp, const cplx<T>* tw,
                 hipStream_t st);
template <typename T>
void fft_inverse(int n, int nhp, cplx<T>* spec, int nout, T* const* outp, double out_scale, const cplx<T>* tw,
                 hipStream_t st);

// ---- solve.hip ----
// solution components of a solve: phi | phi, chi | phi, chi, B_x, B_y, B_z
__host__ __device__ constexpr int mode_nout(int mode) {
  return (mode == MODE_FULL || mode == MODE_FULLP) ? 5 : (mode == MODE_SCALAR ? 2 : 1);
}
// record index of mode (kx, ky, kz) in the per-mode state arrays (tensor and parabolic B):
// [ky][kx][kz], so that the modes of one ky and a few kx (one workgroup of the Fourier-space
// kernel) are one contiguous block
__host__ __device__ inline long state_index(int n, int nhp, int kx, int ky, int kz) {
  return ((long)ky * nhp + kx) * n + kz;
}

template <typename T>
struct SolveArgs {
  const cplx<T>* spec;  // [z][y][kx][NS] sources after passes X and Y (component-interleaved)
  cplx<T>* out;         // [z][y][kx][NOUT] solutions (phi, chi, B) before the inverse passes Y and X
  int n, nhp;
  int mode;             // MODE_NEWTONIAN / MODE_SCALAR / MODE_FULL / MODE_FULLP
  const T* kt;          // kt[m] = 2 n sin(pi m_signed / n), m = 0 .. n-1
  const cplx<T>* tw;    // exp(-2 pi i j / n), j = 0 .. n-1
  double hc, inv_dt, ebar, inv_n3;
  // FP64 homogeneous mode of the phi source: dc[0] = mesh sum of every term but E - ebar,
  // dc[2] = sum over particles of e; k = 0 source = dc[0] + kap_a2 dc[2] - n3 ebar
  const double* dc;
  double kap_a2, n3_ebar;
  double* phibar_out; // FP64 mean of the new phi (may be null)
  int incr;           // the phi source is that of the increment phi_n - phi_{n-1}: the FP64 mean
                      // of the solution is added to the previous mean in phibar_out
  // tensor state: records (h+, hx, pi+, pix) of the polarisation amplitudes and their
  // time derivatives at state_index
  cplx<T>* hst;
  int tensor_op;      // 0: none, 1: reset to zero, 2: Crank-Nicolson step
  double dtau, hc_half;
  // parabolic B state: records a^2 (B_x, B_y, B_z)(k) at state_index (unnormalised like the sources)
  cplx<T>* a2b;
  int b_op;           // MODE_FULL: 1 = also store a^2 B of the elliptic solution; MODE_FULLP: step
  double a2_now, a2_mid;
};
// z transform + solves + inverse z transform (one fused kernel)
template <typename T> void launch_solve(const SolveArgs<T>& a, hipStream_t st);
// rebuild the six h_ij half spectra [q][z][y][kx] (stride comp_stride) from the tensor state (diagnostic)
template <typename T>
void launch_tensor_components(cplx<T>* spec, long comp_stride, int n, int nhp, const T* kt, const cplx<T>* hst,
                              hipStream_t st);
// FP64 sum of count values into out[0]; out[8 .. 8 + 512) is used as scratch
void launch_sum_f64(const double* in, long count, double* out, hipStream_t st);
void launch_sum_as_f64(const float* in, long count, double* out, hipStream_t st);

// ---- pk.hip ----
// blocks of the binning pass whose partials ((blocks + 1) rows of 3 (n/2 + 1) doubles) fit in scratch_bytes
int pk_blocks(int n, size_t scratch_bytes);
// shell sums [modes | P | |m|] of the power spectrum of a count field's half spectrum, written to
// scratch + nblocks * 3 (n/2 + 1); amp2 = L^3 / N_p^2, shot = L^3 / N_p (or 0)
template <typename T>
void launch_power_spectrum(const cplx<T>* spec, int n, int nhp, double amp2, double shot, int nblocks, double* scratch,
                           hipStream_t st);

// ---- particles.hip ----
template <typename T>
struct Particles {
  double* px; double* py; double* pz;  // SoA positions
  T* ux; T* uy; T* uz;                 // SoA momenta
  uint32_t* id;
};

template <typename T>
void launch_ingest(const double* pos_aos, const T* u_aos, const uint32_t* ids, long n, Particles<T> out, int nmesh,
                   uint32_t* rank, uint32_t* cnt, int* err, hipStream_t st);
// CIC deposit of one species: stores the sums (accumulate = false) or adds weight x the sums
// (accumulate = true, a further species of particle mass weight x the first's); writes one FP64
// energy partial (weight x the sum of e over the block's own cells) per block to esum_part
int deposit_blocks(int n);
template <typename T>
void launch_deposit(const Particles<T>& p, const uint32_t* cell_start, int n, int ncomp, bool relativistic, double a,
                    double weight, bool accumulate, T* dep, double* esum_part, hipStream_t st);
template <typename T>
struct GatherArgs {
  const T* phi; const T* chi; const T* bx; const T* by; const T* bz;
  const float* corr;  // closure correction to grad phi, FP32 SoA [3][n^3] (null: none)
  int mode;
  double dtau, a, a_half;
};
template <typename T>
void launch_kick_drift(const Particles<T>& p, long np, int n, const uint32_t* cell_start, const GatherArgs<T>& g,
                       uint32_t* rank, uint32_t* cnt, int* err, hipStream_t st);
void launch_scan(uint32_t* cnt, uint32_t* cell_start, long ncell, uint32_t* block_sums, hipStream_t st);
size_t scan_block_sums_count(long ncell);
template <typename T>
void launch_scatter(const Particles<T>& src, Particles<T> dst, long np, int nmesh, const uint32_t* rank,
                    const uint32_t* cell_start, hipStream_t st);
// move each particle of the cell-sorted src to cell_start[cell] + (particles of its cell with a smaller
// identifier) in dst: an in-cell order that does not depend on the order of the sort's atomic ranks
template <typename T>
void launch_order_by_id(const Particles<T>& src, Particles<T> dst, long np, int nmesh, const uint32_t* cell_start,
                        hipStream_t st);
// bit 4 of err unless the store and its cell offsets are consistent (used on restored checkpoints)
template <typename T>
void launch_check_store(const Particles<T>& p, long np, int nmesh, const uint32_t* cell_start, int* err,
                        hipStream_t st);
template <typename T>
void launch_export(const Particles<T>& p, long np, double* pos_aos, T* u_aos, uint32_t* ids, hipStream_t st);
template <typename T>
void launch_copy_unpad(const cplx<T>* spec, int n, int nhp, cplx<T>* out, bool to_padded, hipStream_t st);

// ---- closure.hip ----
void closure_pack(const float* params, uint16_t* wf, uint16_t* wb, float* bias, hipStream_t st);
void closure_conv(const uint16_t* in, const uint16_t* w, const float* bias, int n, int mode, void* out,
                  const uint16_t* mask, const float* scale, hipStream_t st);
long closure_wgrad_part_bytes(int n);  // weight-gradient partials of one layer (bytes)
void closure_wgrad(const uint16_t* x, const uint16_t* dy, int n, float* part, int ci_n, int co_n, float* grad,
                   long off, hipStream_t st);
void closure_adam(float* p, float* m, float* v, const float* g, int np, double lr, int step, hipStream_t st);
template <typename T>
void closure_features(const T* n00, const T* phi, int n, const double* n00_sum, double* part, float* rms,
                      uint16_t* out, hipStream_t st);
template <typename T>
void closure_gather3(const Particles<T>& p, long np, int n, const float* f, float* out, hipStream_t st);
template <typename T>
void closure_gather3_adjoint(const Particles<T>& p, long np, int n, const float* vals, float* f, hipStream_t st);
// pred - target at the particles: dpred = 2 (pred - target) / (3 np), out[0] = mean |pred - target|^2,
// out[1] = mean |target|^2 (FP64); part holds 2 x 512 doubles of scratch
template <typename T>
void closure_loss3(const Particles<T>& p, long np, int n, const float* f, const float* target, float* dpred,
                   double* part, double* out, hipStream_t st);
void closure_cube_symmetry(long np, const int perm[3], int flip, const double* pos, const float* u, const float* v,
                           double* pos_out, float* u_out, float* v_out, hipStream_t st);
void closure_soa3_to_bf16(const float* f, long n3, uint16_t* out, hipStream_t st);
template <typename T>
void gather_grad_phi(const Particles<T>& p, long np, int n, const T* phi, T* out, hipStream_t st);

}  // namespace gpm
