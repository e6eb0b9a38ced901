/*
 * pm.h -- C ABI of the MI355X (gfx950) relativistic particle-mesh step.
 *
 * The library implements one step of the particle-mesh (PM) method of
 * Adamek & Christiansen, "gevolution 2.0" (arXiv:2607.17929):
 *   (1) cloud-in-cell deposit of the particle stress-energy T00, T0i, Tij
 *       (Sec. 3.1, Eqs. 11-13; the projection of Sec. 2.1),
 *   (2) 3D real-to-complex FFTs and Fourier-space solves for phi (Hamiltonian
 *       constraint, Eq. 4), chi = phi - psi and h_ij (trace-free space-space
 *       equation, Eq. 5) and B_i (momentum constraint, Eq. 6),
 *   (3) cloud-in-cell gather of the metric and the geodesic kick and drift
 *       (Eqs. 8-10 expanded to first order in phi, psi and B, h neglected),
 *       followed by a re-sort of the particles by mesh cell (Sec. 2.1).
 * All work runs in HIP kernels on one GPU, enqueued on the caller's stream.
 *
 * Units: the box side is 1 and c = 1.  Positions are in [0, 1); momenta are
 * the canonical momentum per unit mass u = q/m; conformal time tau is in units
 * of box/c.  The background is Einstein-de Sitter: a = (H0 tau / 2)^2 with
 * H0 = box_mpch / 2997.92458.  Mesh arrays are [z][y][x] with x fastest,
 * n_mesh^3 vertices at x_v = v / n_mesh.
 *
 * Memory ownership: the caller allocates one device workspace of the size
 * pm_query_workspace() reports and owns it; the library carves all its device
 * buffers out of it and never allocates device memory itself.  Host pointers
 * passed in are only read (or written) during the call.  pm_ctx is an opaque
 * host object owned by the library until pm_destroy().
 *
 * Ordering and errors: every call enqueues work on the context's stream and
 * returns without waiting, except calls that write to host memory, which
 * synchronise the stream.  Functions return pm_status (0 = success, negative =
 * error) and never throw.  A failed HIP call or a non-finite particle
 * coordinate found on the device is reported as PM_EHIP / PM_ENAN by the next
 * synchronising call and is sticky until pm_init_particles() or
 * pm_set_state().  One context must not be used from two threads at once.
 */
#ifndef PM_H
#define PM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pm_status {
  PM_OK = 0,
  PM_EINVAL = -1,      /* bad argument (null pointer, size, id out of range) */
  PM_EWORKSPACE = -2,  /* workspace null, too small or misaligned (256 B) */
  PM_EHIP = -3,        /* a HIP runtime call failed */
  PM_ENAN = -4,        /* non-finite particle data detected on the device */
  PM_ESTATE = -5,      /* call out of order (e.g. solve before deposit) */
  PM_ERANGE = -6,      /* size outside the supported range */
  PM_EUNSUPPORTED = -7 /* option not built into this library */
} pm_status;

/* arithmetic of fields, FFTs, deposit and momenta; positions are always FP64 */
enum { PM_FP32 = 0, PM_FP64 = 1 };

/* physics: which metric components are solved for and act on particles */
enum {
  PM_NEWTONIAN = 0, /* Newtonian limit (Sec. 3.2): lap psi = 4 pi G a^2 delta rho, phi = psi */
  PM_SCALAR = 1,    /* phi and chi (psi = phi - chi) */
  PM_FULL = 2       /* phi, chi, B_i (elliptic, Eq. 6, or parabolic, see PM_FLAG_B_PARABOLIC) and h_ij
                       (Eq. 5, not fed back) */
};

enum {
  PM_FLAG_TIMINGS = 1u,    /* record per-stage device times (pm_get_timings) */
  PM_FLAG_CLOSURE = 2u,    /* reserve workspace for the learned closure (pm_closure_*) */
  /* With PM_FULL: B_i from the vector part of the trace-free space-space equation (Sec. 3.1,
   * Eq. 5), d_tau(a^2 B_j) = -i a^2 w_j / |kt| with w the spin-1 part of its source, integrated
   * with a^2 at the midpoint of each step and started from the momentum constraint (Eq. 6) at the
   * quasi-static start.  Later steps need 7 forward and 5 inverse transforms instead of 10 and 5
   * (the paper's benchmark configuration, Sec. 4.1).  Ignored for other physics. */
  PM_FLAG_B_PARABOLIC = 4u,
  /* Deterministic runs: after every sort by cell, the particles of each cell are put in identifier
   * order (one more pass over the particles), so that the order of the atomic counters the sort
   * ranks with no longer reaches the sums over a cell; two runs from the same inputs, and a run
   * restarted from pm_get_state / pm_set_state, then give bitwise identical particles and fields. */
  PM_FLAG_DETERMINISTIC = 8u
};

/* field identifiers for pm_get_field / pm_set_field (real space, [z][y][x]) */
enum {
  PM_FIELD_N00 = 0, /* deposit sum W e, e = sqrt(a^2 + u^2) (Newtonian: a) */
  PM_FIELD_N0X = 1, PM_FIELD_N0Y = 2, PM_FIELD_N0Z = 3, /* sum W u_i */
  PM_FIELD_NXX = 4, PM_FIELD_NXY = 5, PM_FIELD_NXZ = 6, /* sum W u_i u_j / e */
  PM_FIELD_NYY = 7, PM_FIELD_NYZ = 8, PM_FIELD_NZZ = 9,
  PM_FIELD_PHI = 10,      /* latest phi (after a solve: phi_n) */
  PM_FIELD_CHI = 11,      /* latest chi */
  PM_FIELD_BX = 12, PM_FIELD_BY = 13, PM_FIELD_BZ = 14,
  PM_FIELD_PHI_PREV = 15, /* phi of the solve before the latest one */
  PM_FIELD_HXX = 16, PM_FIELD_HXY = 17, PM_FIELD_HXZ = 18, /* h_ij, get only */
  PM_FIELD_HYY = 19, PM_FIELD_HYZ = 20, PM_FIELD_HZZ = 21,
  PM_FIELD_COUNT = 22
};

/* timed stages (PM_FLAG_TIMINGS): each is one kernel or a pair of kernels of one kind */
enum {
  PM_STAGE_DEPOSIT = 0,    /* CIC deposit (+ FP64 energy sum) */
  PM_STAGE_FFT_X_FWD = 1,  /* source assembly + R2C along x */
  PM_STAGE_FFT_Y_FWD = 2,  /* complex FFTs along y */
  PM_STAGE_KSPACE = 3,     /* complex FFTs along z, Fourier-space solves, inverse FFTs along z (one kernel) */
  PM_STAGE_FFT_Y_INV = 4,  /* inverse complex FFTs along y */
  PM_STAGE_FFT_X_INV = 5,  /* C2R along x */
  PM_STAGE_KICK_DRIFT = 6, /* gather + kick + drift + cell key */
  PM_STAGE_SORT = 7,       /* counting sort: scan + scatter */
  PM_NSTAGES = 8
};

typedef struct pm_config {
  int32_t n_mesh;       /* N: power of two, 16 .. 1024 */
  int32_t precision;    /* PM_FP32 or PM_FP64 */
  int64_t n_particles;  /* number of particles, 1 .. 2^31 - 1 */
  double box_mpch;      /* box side in Mpc/h (sets H0 in box units) */
  int32_t physics;      /* PM_NEWTONIAN, PM_SCALAR or PM_FULL */
  uint32_t flags;       /* PM_FLAG_* */
  /* Optional second particle species of another particle mass (e.g. a hot,
   * neutrino-like set; Sec. 3.1: the stress-energy sums run over all particles,
   * each with its own mass, and the update keeps momenta non-perturbative).
   * n_particles_2 = 0 (and mass_fraction_2 = 0): none.  Otherwise the species
   * holds n_particles_2 (1 .. 2^31 - 1) particles carrying the fraction
   * 0 < mass_fraction_2 < 1 of the total rest mass (species 1 carries the rest;
   * the background stays Einstein-de Sitter).  Both species deposit into the
   * same fields, species 2 weighted by its particle mass over species 1's, and
   * both take the same kick and drift.  P(k) and the closure's grad-phi gather
   * use species 1. */
  int64_t n_particles_2;
  double mass_fraction_2;
} pm_config;

typedef struct pm_ctx pm_ctx;

/* Device workspace (bytes) that pm_create needs for this configuration. */
pm_status pm_query_workspace(const pm_config* cfg, size_t* bytes);

/* Create a context on the current HIP device.  d_workspace: device pointer,
 * 256-byte aligned, at least pm_query_workspace bytes, owned by the caller and
 * kept alive until pm_destroy.  hip_stream: a hipStream_t (NULL = default). */
pm_status pm_create(const pm_config* cfg, void* d_workspace, size_t bytes, void* hip_stream, pm_ctx** out);
pm_status pm_destroy(pm_ctx* ctx);

/* Load particles and reset the time-stepping state.
 * pos: [n][3] doubles (x, y, z), wrapped into [0, 1) on the device.
 * u:   [n][3] momenta per unit mass in the context precision (float or double).
 * ids: [n] identifiers forming a permutation of 0..n-1, or NULL for 0..n-1
 *      (an identifier >= n is reported as PM_EINVAL by the next synchronising
 *      call; repeated identifiers are not detected and leave the outputs in
 *      identifier order undefined).
 * n must equal cfg.n_particles.  tau0 > 0 is the conformal time of pos (u is
 * at tau0 - dtau/2, the leapfrog's half step).  src_on_device: pointers are
 * device (1) or host (0) memory. */
pm_status pm_init_particles(pm_ctx* ctx, const double* pos, const void* u, const uint32_t* ids, int64_t n,
                            double tau0, int src_on_device);

/* Load the second species (same conventions as pm_init_particles; n must equal
 * cfg.n_particles_2; ids a permutation of 0..n-1 or NULL).  Call after
 * pm_init_particles (which takes the start time and unloads the second species);
 * PM_EINVAL if the configuration has no second species.  pm_deposit returns
 * PM_ESTATE while a configured second species is not loaded. */
pm_status pm_init_particles_2(pm_ctx* ctx, const double* pos, const void* u, const uint32_t* ids, int64_t n,
                              int src_on_device);

/* Stage 1: CIC deposit of e, u_i and u_i u_j / e at a(tau) (Sec. 3.1, Eqs. 11-13). */
pm_status pm_deposit(pm_ctx* ctx);

/* Stage 2: metric solve at the current tau from the last deposit.
 * dtau_prev > 0: tau - tau_prev of the previous solve (semi-implicit time
 * derivative, non-linear terms lagged, Sec. 3.1); dtau_prev <= 0: quasi-static
 * start (two predictor-corrector passes). Requires a preceding pm_deposit. */
pm_status pm_solve_metric(pm_ctx* ctx, double dtau_prev);

/* Stage 3: gather + kick (u to tau + dtau/2) + drift (x to tau + dtau) + re-sort;
 * tau += dtau.  Requires a preceding pm_solve_metric.  dtau > 0. */
pm_status pm_update_particles(pm_ctx* ctx, double dtau);

/* One whole step: deposit, solve (dtau_prev = the previous step's dtau, or a
 * quasi-static solve on the first step after pm_init_particles), update. */
pm_status pm_step(pm_ctx* ctx, double dtau);

/* Copy a real-space field ([z][y][x], n_mesh^3 values of the context precision).  The h_ij
 * components are rebuilt from the per-mode tensor state through the spectrum buffers; no field of
 * the time-stepping state (the deposit included) is touched, so this may be called between any
 * two stages. */
pm_status pm_get_field(pm_ctx* ctx, int field_id, void* dst, int dst_on_device);
/* Overwrite a field (deposit components, PHI, CHI, B*, PHI_PREV); for tests and
 * for the closure. Setting a deposit component marks the deposit as done. */
pm_status pm_set_field(pm_ctx* ctx, int field_id, const void* src, int src_on_device);

/* Particles in identifier order: pos [n][3] doubles, u [n][3] context precision,
 * ids [n] (may be NULL; any of pos/u may be NULL). */
pm_status pm_get_particles(pm_ctx* ctx, double* pos, void* u, uint32_t* ids, int dst_on_device);

/* The second species in identifier order (as pm_get_particles). */
pm_status pm_get_particles_2(pm_ctx* ctx, double* pos, void* u, uint32_t* ids, int dst_on_device);

/* Conservation diagnostics in FP64 (a per-step log for the caller; synchronises):
 * out[0] = sum over particles of e = sqrt(a^2 + u^2) at the last pm_deposit (the
 *          homogeneous mode's energy sum; species 2 weighted by m_2/m_1),
 * out[1] = mean phi of the last pm_solve_metric (the FP64 homogeneous mode),
 * out[2..4] = total momentum per unit mass of species 1, sum of u_i over the
 *          particles as they are now (species 2 weighted by m_2/m_1).
 * out[0] and out[1] are 0 before the first deposit / solve and with Newtonian
 * physics (which solves without the FP64 homogeneous mode).
 * n: entries of out to write (1 .. 5). */
pm_status pm_diagnostics(pm_ctx* ctx, double* out, int n);

/* Current conformal time, scale factor and number of completed steps. */
pm_status pm_get_time(pm_ctx* ctx, double* tau, double* a, int64_t* steps);

/* Background of a configuration (host only): a(tau) and H_conf(tau) = d ln a / d tau. */
pm_status pm_background(const pm_config* cfg, double tau, double* a, double* hconf);
/* Conformal time at which the scale factor equals a. */
pm_status pm_tau_of_a(const pm_config* cfg, double a, double* tau);

/* Device milliseconds spent in each stage (ms[i]) and the number of times it ran
 * (calls[i], may be NULL) since the previous pm_get_timings call or context
 * creation; resets both.  Needs PM_FLAG_TIMINGS.  Synchronises the stream. */
pm_status pm_get_timings(pm_ctx* ctx, double* ms, int64_t* calls, int n);

/* Wait for the context's stream and report sticky device errors. */
pm_status pm_sync(pm_ctx* ctx);

/* Diagnostic: 3D real-to-complex FFT of a device array with the library's own
 * kernels.  direction +1: in = real [z][y][x] (n^3), out = complex [z][y][kx]
 * (n^2 (n/2+1) interleaved re,im), unnormalised.  direction -1: in = that
 * half spectrum, out = real, scaled by 1/n^3.  Both device pointers, context
 * precision; uses the context's spectrum buffer as scratch. */
pm_status pm_debug_fft(pm_ctx* ctx, const void* d_in, void* d_out, int direction);

/* Shell-averaged matter power spectrum of the current particles on the context's
 * mesh (evaluation of results, not part of a step; Sec. 4.1 computes spectra on the
 * fly, Sec. 4.4 compares them): CIC count field, forward FFT, division by the CIC
 * window prod_d sinc^2(pi m_d / n), |delta_k|^2 L^3 / n^6 minus the Poisson shot
 * noise L^3 / N_p when subtract_shot_noise != 0, averaged over shells of width
 * k_f = 2 pi / L, shell b = round(|m|) for b = 1 .. n/2.  Writes n/2 + 1 host
 * values to each of k_out (mean |k| of the shell, h/Mpc), p_out ((Mpc/h)^3) and
 * modes_out (modes in the shell; entry 0 and empty shells are 0).  Uses the
 * spectrum buffers as scratch, which hold nothing between a solve and the next
 * one, so it may be called between any two stages; synchronises the stream. */
pm_status pm_power_spectrum(pm_ctx* ctx, int subtract_shot_noise, double* k_out, double* p_out, double* modes_out);

/* Checkpoint and restart.  The paper writes particle and metric snapshots
 * (Sec. 4.1) but does not describe a restart; this pair saves and restores
 * everything the next steps depend on: the particles in their sorted order,
 * the cell offsets of the sort, phi of the latest and the previous solve, chi,
 * B_i, the tensor state (h and its time derivative, two polarisations, Sec. 3.1),
 * the parabolic a^2 B state, the second species' particles and cell offsets,
 * the FP64 homogeneous-mode scalars, tau, the step
 * counter, the last two time steps, the call-order state and, between
 * pm_deposit and pm_solve_metric, the deposit.  Not included: the closure's
 * parameters and its enable switch (bind them again after a restore).
 * pm_get_state: blob NULL -> *bytes = the size the current state needs (it
 * grows by the deposit between pm_deposit and pm_solve_metric).  Otherwise
 * *bytes is the capacity of blob (PM_EINVAL, with *bytes set to the size, if it
 * is too small); on success *bytes is the size written.  The blob is an opaque
 * byte image for a context of the same n_mesh, precision, physics, B route and
 * n_particles.  dst_on_device / src_on_device: the blob is device (1) or host (0)
 * memory; either way both calls synchronise the stream before they return.
 * pm_set_state validates the header (PM_EINVAL for a blob of another
 * configuration, truncated or corrupt) and then the body on the device: the cell
 * offsets must start at 0, end at the particle count and never decrease, and every
 * particle must have finite momenta, a position in [0, 1), an identifier below the
 * particle count and sit inside the offsets' range of the cell its position falls
 * in (PM_EINVAL otherwise, and the context then holds no particles until the next
 * pm_init_particles or successful pm_set_state; repeated identifiers are not
 * detected).  On success it clears a sticky device error and leaves the context as
 * it was when the blob was taken.  The run after a restore agrees with the
 * uninterrupted run bit for bit under PM_FLAG_DETERMINISTIC, otherwise to rounding
 * (particles inside a cell are then ordered by the sort's atomic counters, so sums
 * over a cell's particles may round differently from run to run). */
pm_status pm_get_state(pm_ctx* ctx, void* blob, size_t* bytes, int dst_on_device);
pm_status pm_set_state(pm_ctx* ctx, const void* blob, size_t bytes, int src_on_device);

/* Gradient of phi (centred differences, CIC-interpolated, as used by the kick)
 * at every particle, [n][3] in identifier order, context precision. */
pm_status pm_gather_grad_phi(pm_ctx* ctx, void* out, int dst_on_device);

/* ---- learned force closure (an addition to the paper's method) --------------
 * A 3-layer convolutional network on the mesh, conv(4->16)-ReLU-conv(16->16)-
 * ReLU-conv(16->3) with 3x3x3 periodic kernels, bfloat16 weights and
 * activations with FP32 accumulation, predicts a correction to grad phi from
 * sign(delta) log(1+|delta|) (delta from the last deposit's n00) and
 * grad phi / rms|grad phi|; the output is in units of rms|grad phi|.  When
 * enabled, pm_update_particles adds the CIC-interpolated, rescaled output to
 * the gathered grad phi.  Needs PM_FLAG_CLOSURE; training needs n_mesh <= 256.
 * Parameters: one FP32 vector of PM_CLOSURE_NPARAM values laid out as
 * W1[16][4][27] b1[16] W2[16][16][27] b2[16] W3[3][16][27] b3[3], tap index
 * 9 (dz+1) + 3 (dy+1) + (dx+1), y[co](p) = b[co] + sum W[co][ci][t] x[ci](p + d_t). */
enum { PM_CLOSURE_NPARAM = 9971 };
pm_status pm_closure_set_params(pm_ctx* ctx, const float* params, int src_on_device);
pm_status pm_closure_enable(pm_ctx* ctx, int on);
/* Run the network on the current deposit and phi (after pm_solve_metric); output kept in the
 * context; scaled = 1 multiplies by rms|grad phi| (force units). */
pm_status pm_closure_forward(pm_ctx* ctx, int scaled);
/* rms|grad phi| of the last pm_closure_forward (the output's unit); synchronises. */
pm_status pm_closure_scale(pm_ctx* ctx, double* rms);
/* Network output at the particles, [n][3] FP32, identifier order. */
pm_status pm_closure_gather(pm_ctx* ctx, float* out, int dst_on_device);
/* Gradient of sum_p dpred_p . out_p with respect to the parameters (device pointers:
 * d_dpred [n][3] in identifier order, d_grad [PM_CLOSURE_NPARAM], overwritten), using the
 * activations of the last pm_closure_forward. */
pm_status pm_closure_backward(pm_ctx* ctx, const float* d_dpred, float* d_grad);
/* Training residual of the last pm_closure_forward against d_target ([n][3] FP32, identifier
 * order, device): r = out_p - target_p at every particle; writes d_dpred[n][3] = 2 r / (3 n),
 * the gradient of the mean-squared error that pm_closure_backward takes (device, may not alias
 * d_target), and, when loss is not NULL, loss[0] = mean |r|^2 and loss[1] = mean |target|^2 over
 * the 3 n components (FP64, fixed summation order; synchronises).  PM_ESTATE before a forward
 * pass or without particles. */
pm_status pm_closure_loss(pm_ctx* ctx, const float* d_target, float* d_dpred, double* loss);
/* Augmentation of training data by the 48 symmetries of the periodic cube (the mesh, CIC and the
 * centred differences map onto themselves): for n particles, component d of the outputs is
 * component perm[d] of the inputs ([n][3] device arrays: positions FP64 in [0,1), two FP32
 * vector fields such as momenta and force differences), and where bit d of flip (0..7) is set
 * the position is reflected (x -> 1 - x, wrapped into [0,1)) and both vectors negated.  Outputs
 * may alias the inputs.  Runs on the context's stream; PM_EINVAL if perm is not a permutation. */
pm_status pm_cube_symmetry(pm_ctx* ctx, long n, const int* perm, int flip, const double* d_pos, const float* d_u,
                           const float* d_v, double* d_pos_out, float* d_u_out, float* d_v_out);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step >= 1) on FP32
 * device vectors, then the context's bfloat16 weights are refreshed from d_params. */
pm_status pm_closure_adam(pm_ctx* ctx, float* d_params, float* d_m, float* d_v, const float* d_grad, int step,
                          double lr);

/* Measurement helper (Sec. 4 reports step times; the HBM rates of the kernels here are judged
 * against the device's own sustainable rate): copies `bytes` (a multiple of 16, both pointers device
 * memory aligned to 16 bytes) from d_src to d_dst with a plain copy kernel (one 16-byte element per
 * thread, non-temporal loads and stores), once to warm
 * up and then `reps` times on hip_stream, and writes the average milliseconds of one copy to
 * ms_per_copy.  The copy moves 2 x bytes through HBM.  Synchronises the stream; needs no context. */
pm_status pm_copy_probe(const void* d_src, void* d_dst, size_t bytes, int reps, void* hip_stream, double* ms_per_copy);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops):
 * the 3D real-to-complex FFT of pm_debug_fft without a context.  Its scratch (the padded half spectrum
 * and the twiddle table, pm_fft_noalloc_scratch_bytes) lives in one fixed device array of
 * PM_FFT_NOALLOC_SCRATCH_BYTES that each GPU holds until the process ends: meshes up to 128^3 in either
 * precision fit, larger ones return PM_ERANGE.  It calls no allocation routine; the array's device
 * address is looked up once per device on the first call made with that device current.
 * direction +1: d_in = real [z][y][x] (n^3 values), d_out = complex [z][y][kx] (n^2 (n/2+1) interleaved
 * re, im), unnormalised; -1: d_in = that half spectrum, d_out = real, scaled by 1/n^3.  Both device
 * pointers of the given precision (PM_FP32 / PM_FP64); enqueued on hip_stream, no synchronisation.
 * Every call on one GPU uses that GPU's one array, so calls that overlap on a GPU (two streams, two
 * threads) race and must be ordered by the caller.  PM_EINVAL for null pointers, a bad direction or a
 * mesh that is not a power of two in 16 .. 1024; PM_EHIP if the array's address cannot be found. */
enum { PM_FFT_NOALLOC_SCRATCH_BYTES = 24 << 20 };
size_t pm_fft_noalloc_scratch_bytes(int n_mesh, int precision); /* 0 for an invalid mesh or precision */
pm_status pm_fft_noalloc(const void* d_in, void* d_out, int n_mesh, int precision, int direction, void* hip_stream);

const char* pm_status_string(pm_status s);
/* Last error message recorded on this context (never NULL). */
const char* pm_last_error(pm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* PM_H */
