// C ABI of the PM library: context, workspace carving, the three stages and the getters.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "pm.h"
#include "kernels.h"

using namespace gpm;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kSkew = 5 * 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int mode_of(int physics) {
  return physics == PM_NEWTONIAN ? MODE_NEWTONIAN : (physics == PM_SCALAR ? MODE_SCALAR : MODE_FULL);
}

bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }

// byte offsets of every device buffer inside the workspace
struct Layout {
  size_t pos[2], mom[2], ids[2], rank, cnt, cell_start, bsum;
  // second particle species (zero offsets without one)
  size_t pos2[2], mom2[2], ids2[2], rank2, cnt2, cell_start2;
  size_t dep, part, phi[3], chi, b[3], spec, spec_out, hst, a2b, tw, kt, rowsum, scal, err;
  // learned closure (PM_FLAG_CLOSURE): activations, gradients, packed weights, partials
  size_t cl_act[3], cl_dact[3], cl_corr, cl_dcorr, cl_wf, cl_wb, cl_bias, cl_part, cl_scal;
  bool closure, cl_train;
  size_t total;
  int ndep, nsrc, nout, nhp;
  long spec_comp;
};

Layout make_layout(const pm_config& c) {
  Layout L;
  memset(&L, 0, sizeof(L));
  const long n = c.n_mesh, n3 = n * n * n, np = c.n_particles;
  const size_t rs = c.precision == PM_FP64 ? 8 : 4;
  const int mode = mode_of(c.physics);
  L.ndep = mode == MODE_NEWTONIAN ? 1 : 10;
  L.nsrc = mode_nsrc(mode);
  L.nout = mode == MODE_FULL ? 5 : (mode == MODE_SCALAR ? 2 : 1);
  L.nhp = (int)((n / 2 + 1 + 15) / 16 * 16);
  L.spec_comp = n * n * (long)L.nhp;
  const int nspec = L.nsrc < 6 && mode == MODE_FULL ? 6 : (L.nsrc < 1 ? 1 : L.nsrc);
  size_t o = 0;
  // every buffer (and every component inside the particle blocks) starts kSkew bytes further
  // from a large power-of-two boundary than the previous one, so that the same index in
  // different arrays does not fall on the same HBM channel
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes) + kSkew; return r; };
  for (int b = 0; b < 2; ++b) {
    L.pos[b] = take(3 * np * 8 + 2 * kSkew);
    L.mom[b] = take(3 * np * rs + 2 * kSkew);
    L.ids[b] = take(np * 4);
  }
  L.rank = take(np * 4);
  L.cnt = take(n3 * 4);
  L.cell_start = take((n3 + 1) * 4);
  const long np2 = c.n_particles_2;
  if (np2 > 0) {
    for (int b = 0; b < 2; ++b) {
      L.pos2[b] = take(3 * np2 * 8 + 2 * kSkew);
      L.mom2[b] = take(3 * np2 * rs + 2 * kSkew);
      L.ids2[b] = take(np2 * 4);
    }
    L.rank2 = take(np2 * 4);
    L.cnt2 = take(n3 * 4);
    L.cell_start2 = take((n3 + 1) * 4);
  }
  L.bsum = take(scan_block_sums_count(n3) * 4 + 64);
  L.dep = take(L.ndep * n3 * rs);
  // one FP64 energy partial per deposit block and species
  L.part = take(((size_t)deposit_blocks((int)n) * (np2 > 0 ? 2 : 1) + 64) * 8);
  for (int i = 0; i < 3; ++i) L.phi[i] = take(n3 * rs);
  L.chi = mode != MODE_NEWTONIAN ? take(n3 * rs) : 0;
  for (int i = 0; i < 3; ++i) L.b[i] = mode == MODE_FULL ? take(n3 * rs) : 0;
  // sources (component-interleaved half spectra) and the solutions of the Fourier-space kernel
  L.spec = take((size_t)nspec * L.spec_comp * 2 * rs);
  L.spec_out = take((size_t)L.nout * L.spec_comp * 2 * rs);
  // per-mode state: tensor records of 4 and parabolic-B records of 3 complex values
  L.hst = mode == MODE_FULL ? take(4 * L.spec_comp * 2 * rs) : 0;
  const bool parabolic = mode == MODE_FULL && (c.flags & PM_FLAG_B_PARABOLIC) != 0;
  L.a2b = parabolic ? take(3 * L.spec_comp * 2 * rs) : 0;
  L.tw = take(n * 2 * rs);
  L.kt = take(n * rs);
  L.rowsum = take(n * n * 8);
  L.scal = take(1024 * 8);  // FP64 scalars [0..8) and reduction scratch [8..1024)
  L.closure = (c.flags & PM_FLAG_CLOSURE) != 0;
  if (L.closure) {
    for (int i = 0; i < 3; ++i) L.cl_act[i] = take(n3 * 32);
    L.cl_corr = take(3 * n3 * 4);
    L.cl_wf = take(3 * 27 * 256 * 2);
    L.cl_wb = take(3 * 27 * 256 * 2);
    L.cl_bias = take(3 * 16 * 4);
    L.cl_scal = take(2048 * 8);  // [0..528) features, [4..6) loss, [1024..2048) loss partials
    // training buffers only on meshes up to 256^3 (the back-propagated activations grow with n^3)
    L.cl_train = n <= 256;
    if (L.cl_train) {
      for (int i = 0; i < 3; ++i) L.cl_dact[i] = take(n3 * 32);
      L.cl_dcorr = take(3 * n3 * 4);
      L.cl_part = take((size_t)closure_wgrad_part_bytes(n));
    }
  }
  L.err = take(64);
  L.total = o;
  return L;
}

pm_status check_config(const pm_config* c) {
  if (!c) return PM_EINVAL;
  if (!is_pow2(c->n_mesh) || c->n_mesh < 16 || c->n_mesh > 1024) return PM_ERANGE;
  if (c->precision != PM_FP32 && c->precision != PM_FP64) return PM_EINVAL;
  if (c->physics < PM_NEWTONIAN || c->physics > PM_FULL) return PM_EINVAL;
  if (c->n_particles < 1 || c->n_particles > 2147483647LL) return PM_ERANGE;
  if (c->n_particles_2 < 0 || c->n_particles_2 > 2147483647LL) return PM_ERANGE;
  if (c->n_particles_2 > 0 ? !(c->mass_fraction_2 > 0.0 && c->mass_fraction_2 < 1.0) : c->mass_fraction_2 != 0.0)
    return PM_EINVAL;
  if (!(c->box_mpch > 0) || !isfinite(c->box_mpch)) return PM_EINVAL;
  return PM_OK;
}

__global__ void zero_bytes_kernel(unsigned char* p, size_t bytes) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < bytes) p[i] = 0;
}

// p must be 16-byte aligned
__global__ void zero_kernel(unsigned char* p, size_t bytes) {
  const size_t i = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * 16;
  if (i + 16 <= bytes) {
    *reinterpret_cast<uint4*>(p + i) = make_uint4(0, 0, 0, 0);
  } else {
    for (size_t j = i; j < bytes; ++j) p[j] = 0;
  }
}

}  // namespace

struct pm_ctx {
  pm_config cfg;
  Layout L;
  int n = 0, mode = 0;
  long n3 = 0, np = 0, np2 = 0;
  int cur2 = 0;                // particle buffer holding the sorted second species
  bool have_particles2 = false;
  size_t rs = 4;
  hipStream_t st = nullptr;
  unsigned char* ws = nullptr;
  int cur = 0;                // particle buffer holding the sorted particles
  int i_phi = 0, i_prev = 1;  // phi slots: latest, previous
  double tau = 0, last_step = 0, dtau_last = 0;
  int64_t steps = 0;
  bool have_particles = false, deposited = false, solved = false, solved_once = false;
  bool cl_params = false, cl_on = false, cl_forwarded = false;
  int sticky = 0;
  std::string last_error;
  // per-stage event pairs recorded since the last pm_get_timings (pool reused)
  static constexpr int kEvCap = 256;
  std::vector<hipEvent_t> ev0[PM_NSTAGES], ev1[PM_NSTAGES];
  int ev_n[PM_NSTAGES] = {0};
  double ev_ms[PM_NSTAGES] = {0};
  int64_t ev_calls[PM_NSTAGES] = {0};

  template <typename X> X* at(size_t off) { return reinterpret_cast<X*>(ws + off); }
  double h0() const { return cfg.box_mpch / 2997.92458; }
  double a_of(double t) const { const double x = 0.5 * h0() * t; return x * x; }
  double hc_of(double t) const { return 2.0 / t; }
  double ebar(double a) const { return 1.5 * h0() * h0() / a; }
  // 4 pi G m_1 / dx^3: species 1 carries the fraction 1 - f of the rest mass
  double kappa() const { return 1.5 * h0() * h0() * (double)n3 * (1.0 - cfg.mass_fraction_2) / (double)np; }
  // particle mass of species 2 over that of species 1
  double weight2() const {
    const double f = cfg.mass_fraction_2;
    return np2 > 0 ? (f / (double)np2) / ((1.0 - f) / (double)np) : 0.0;
  }

  pm_status fail(pm_status s, const char* msg) {
    last_error = msg;
    return s;
  }
  pm_status hip_check(const char* where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      sticky = PM_EHIP;
      last_error = std::string(where) + ": " + hipGetErrorString(e);
      return PM_EHIP;
    }
    return PM_OK;
  }
  void zero(size_t off, size_t bytes) {
    const size_t nthr = (bytes + 15) / 16;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, st, ws + off, bytes);
  }
  // any alignment, small sizes
  void zero_bytes(unsigned char* p, size_t bytes) {
    hipLaunchKernelGGL(zero_bytes_kernel, dim3((unsigned)((bytes + 255) / 256)), dim3(256), 0, st, p, bytes);
  }
  void drain_events() {
    (void)hipStreamSynchronize(st);
    for (int s = 0; s < PM_NSTAGES; ++s) {
      for (int i = 0; i < ev_n[s]; ++i) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, ev0[s][i], ev1[s][i]) == hipSuccess) ev_ms[s] += t;
      }
      ev_calls[s] += ev_n[s];
      ev_n[s] = 0;
    }
  }
  void stage_begin(int s) {
    if (!(cfg.flags & PM_FLAG_TIMINGS)) return;
    if (ev_n[s] == kEvCap) drain_events();
    if ((int)ev0[s].size() <= ev_n[s]) {
      hipEvent_t a, b;
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&b);
      ev0[s].push_back(a);
      ev1[s].push_back(b);
    }
    (void)hipEventRecord(ev0[s][ev_n[s]], st);
  }
  void stage_end(int s) {
    if (!(cfg.flags & PM_FLAG_TIMINGS)) return;
    (void)hipEventRecord(ev1[s][ev_n[s]], st);
    ev_n[s] += 1;
  }

  template <typename T> Particles<T> parts_at(size_t pos, size_t mom, size_t ids, long cnt) {
    Particles<T> p;
    double* pb = at<double>(pos);
    T* mb = at<T>(mom);
    const long sd = (long)(kSkew / sizeof(double)), st_ = (long)(kSkew / sizeof(T));
    p.px = pb; p.py = pb + cnt + sd; p.pz = pb + 2 * (cnt + sd);
    p.ux = mb; p.uy = mb + cnt + st_; p.uz = mb + 2 * (cnt + st_);
    p.id = at<uint32_t>(ids);
    return p;
  }
  template <typename T> Particles<T> parts(int b) { return parts_at<T>(L.pos[b], L.mom[b], L.ids[b], np); }
  template <typename T> Particles<T> parts2(int b) { return parts_at<T>(L.pos2[b], L.mom2[b], L.ids2[b], np2); }
  void* field_ptr(int id) {
    if (id >= PM_FIELD_N00 && id <= PM_FIELD_NZZ) {
      if (id >= L.ndep) return nullptr;
      return ws + L.dep + (size_t)id * n3 * rs;
    }
    switch (id) {
      case PM_FIELD_PHI: return ws + L.phi[i_phi];
      case PM_FIELD_PHI_PREV: return ws + L.phi[i_prev];
      case PM_FIELD_CHI: return L.chi ? ws + L.chi : nullptr;
      case PM_FIELD_BX: return L.b[0] ? ws + L.b[0] : nullptr;
      case PM_FIELD_BY: return L.b[1] ? ws + L.b[1] : nullptr;
      case PM_FIELD_BZ: return L.b[2] ? ws + L.b[2] : nullptr;
      default: return nullptr;
    }
  }
};

namespace {

template <typename T>
void upload_tables(pm_ctx* c) {
  const int n = c->n;
  std::vector<T> tw(2 * n), kt(n);
  for (int j = 0; j < n; ++j) {
    const double ang = -2.0 * M_PI * (double)j / (double)n;
    tw[2 * j] = (T)cos(ang);
    tw[2 * j + 1] = (T)sin(ang);
    const int ms = j <= n / 2 ? j : j - n;
    kt[j] = (T)(2.0 * n * sin(M_PI * (double)ms / (double)n));
  }
  hipMemcpy(c->ws + c->L.tw, tw.data(), tw.size() * sizeof(T), hipMemcpyHostToDevice);
  hipMemcpy(c->ws + c->L.kt, kt.data(), kt.size() * sizeof(T), hipMemcpyHostToDevice);
}

// one forward transform + solve + inverse transform
// smode: the solve's mode (c->mode, or MODE_FULLP for a parabolic-B step); b_op as in SolveArgs
// incr: solve for the increment phi_n - phi_{n-1} (phi1 = phi_{n-1}); phi_out then gets phi1 plus the
// increment and delta_out the increment itself
template <typename T>
void solve_pass(pm_ctx* c, const T* phi1, const T* dphi1, const T* chi1, double inv_dt, double inv_dtl, T* phi_out,
                int tensor_op, double dtau, double hc_half, int smode, int b_op, int incr = 0, T* delta_out = nullptr) {
  const Layout& L = c->L;
  const int nsrc = mode_nsrc(smode);
  const double a = c->a_of(c->tau), hc = c->hc_of(c->tau), eb = c->ebar(a);
  SrcArgsH<T> s;
  s.dep = c->at<T>(L.dep);
  s.phi1 = phi1; s.dphi1 = dphi1; s.chi1 = chi1;
  s.incr = incr;
  s.rowsum = c->mode == MODE_NEWTONIAN ? nullptr : c->at<double>(L.rowsum);
  s.kap = c->kappa() / (a * a);
  s.ebar = eb; s.hc = hc; s.inv_dt = inv_dt; s.inv_dtl = inv_dtl;
  cplx<T>* spec = c->at<cplx<T>>(L.spec);
  cplx<T>* spec_out = c->at<cplx<T>>(L.spec_out);
  const cplx<T>* tw = c->at<cplx<T>>(L.tw);
  c->stage_begin(PM_STAGE_FFT_X_FWD);
  fft_r2c_x<T>(s, smode == MODE_FULLP ? MODE_SCALAR : smode, c->n, L.nhp, spec, tw, c->st);
  c->stage_end(PM_STAGE_FFT_X_FWD);
  c->stage_begin(PM_STAGE_FFT_Y_FWD);
  fft_cols<T>(c->n, L.nhp * nsrc, spec, 1, false, false, tw, c->st);
  c->stage_end(PM_STAGE_FFT_Y_FWD);
  double* dc = c->at<double>(L.scal);
  c->stage_begin(PM_STAGE_KSPACE);
  if (c->mode != MODE_NEWTONIAN) launch_sum_f64(s.rowsum, (long)c->n * c->n, dc, c->st);
  SolveArgs<T> sa;
  sa.spec = spec; sa.out = spec_out; sa.n = c->n; sa.nhp = L.nhp; sa.mode = smode;
  sa.kt = c->at<T>(L.kt);
  sa.tw = tw;
  sa.hc = hc; sa.inv_dt = inv_dt; sa.ebar = eb; sa.inv_n3 = 1.0 / (double)c->n3;
  sa.dc = c->mode == MODE_NEWTONIAN ? nullptr : dc;
  sa.kap_a2 = c->kappa() / (a * a);
  sa.n3_ebar = (double)c->n3 * eb;
  sa.phibar_out = dc + 1;
  sa.incr = incr;
  sa.hst = L.hst ? c->at<cplx<T>>(L.hst) : nullptr;
  sa.tensor_op = c->mode == MODE_FULL ? tensor_op : 0;
  sa.dtau = dtau; sa.hc_half = hc_half;
  sa.a2b = L.a2b ? c->at<cplx<T>>(L.a2b) : nullptr;
  sa.b_op = L.a2b ? b_op : 0;
  sa.a2_now = a * a;
  const double am = c->a_of(c->tau - 0.5 * dtau);
  sa.a2_mid = am * am;
  launch_solve<T>(sa, c->st);
  c->stage_end(PM_STAGE_KSPACE);
  T* outs[8] = {phi_out, c->mode != MODE_NEWTONIAN ? c->at<T>(L.chi) : nullptr, nullptr, nullptr, nullptr,
                nullptr, nullptr, nullptr};
  if (c->mode == MODE_FULL)
    for (int i = 0; i < 3; ++i) outs[2 + i] = c->at<T>(L.b[i]);
  c->stage_begin(PM_STAGE_FFT_Y_INV);
  fft_cols<T>(c->n, L.nhp * L.nout, spec_out, 1, true, false, tw, c->st);
  c->stage_end(PM_STAGE_FFT_Y_INV);
  c->stage_begin(PM_STAGE_FFT_X_INV);
  fft_c2r_x<T>(c->n, L.nhp, spec_out, L.nout, outs, 1.0, tw, c->st, incr ? phi1 : nullptr, delta_out);
  c->stage_end(PM_STAGE_FFT_X_INV);
}

template <typename T>
pm_status do_solve(pm_ctx* c, double dtau_prev) {
  const Layout& L = c->L;
  auto slot = [&](int i) { return c->at<T>(L.phi[i]); };
  const T* chi = c->mode != MODE_NEWTONIAN ? c->at<T>(L.chi) : nullptr;
  if (c->mode == MODE_NEWTONIAN) {
    const int i_new = 3 - c->i_phi - c->i_prev;
    solve_pass<T>(c, nullptr, nullptr, nullptr, 0, 0, slot(i_new), 0, 0, 0, c->mode, 0);
    c->i_prev = c->i_phi;
    c->i_phi = i_new;
  } else if (dtau_prev <= 0) {
    // quasi-static start: two passes from phi = chi = 0, no time derivatives; the slots end as
    // latest = previous = the second pass's phi and a zero increment (the third slot)
    const int sa = 0, sb = 1, sc = 2;
    // (the parabolic B route starts from the momentum constraint's B of the second pass)
    c->zero(L.phi[sc], c->n3 * sizeof(T));
    solve_pass<T>(c, nullptr, nullptr, nullptr, 0, 0, slot(sa), 1, 0, 0, c->mode, 0);
    solve_pass<T>(c, slot(sa), slot(sc), chi, 0, 0, slot(sb), 1, 0, 0, c->mode, 1);
    hipMemcpyAsync(slot(sc), slot(sb), c->n3 * sizeof(T), hipMemcpyDeviceToDevice, c->st);
    c->zero(L.phi[sa], c->n3 * sizeof(T));
    c->i_phi = sb;
    c->i_prev = sc;
    c->dtau_last = 0;
  } else {
    // semi-implicit step solved for the increment: phi_{n-2} is no longer needed, so phi_n takes
    // its slot; the increment slot holds phi_{n-1} - phi_{n-2} (read by the source assembly for the
    // lagged time derivative) and then phi_n - phi_{n-1}
    const int i_new = c->i_prev, i_d = 3 - c->i_phi - c->i_prev;
    const double inv_dtl = c->dtau_last > 0 ? 1.0 / c->dtau_last : 0.0;
    const double hc_half = c->hc_of(c->tau - 0.5 * dtau_prev);
    const int smode = (c->mode == MODE_FULL && c->L.a2b) ? MODE_FULLP : c->mode;
    solve_pass<T>(c, slot(c->i_phi), slot(i_d), chi, 1.0 / dtau_prev, inv_dtl, slot(i_new), 2, dtau_prev,
                  hc_half, smode, 2, 1, slot(i_d));
    c->i_prev = c->i_phi;
    c->i_phi = i_new;
    c->dtau_last = dtau_prev;
  }
  return c->hip_check("solve");
}

// counting sort by cell; with PM_FLAG_DETERMINISTIC the particles of each cell are then put in
// identifier order, so that the store and every sum over it are the same from run to run
template <typename T>
void sort_particles(pm_ctx* c) {
  const Layout& L = c->L;
  launch_scan(c->at<uint32_t>(L.cnt), c->at<uint32_t>(L.cell_start), c->n3, c->at<uint32_t>(L.bsum), c->st);
  launch_scatter<T>(c->parts<T>(c->cur), c->parts<T>(1 - c->cur), c->np, c->n, c->at<uint32_t>(L.rank),
                    c->at<uint32_t>(L.cell_start), c->st);
  c->cur = 1 - c->cur;
  if (c->cfg.flags & PM_FLAG_DETERMINISTIC) {
    launch_order_by_id<T>(c->parts<T>(c->cur), c->parts<T>(1 - c->cur), c->np, c->n, c->at<uint32_t>(L.cell_start),
                          c->st);
    c->cur = 1 - c->cur;
  }
}

template <typename T>
void sort_particles2(pm_ctx* c) {
  const Layout& L = c->L;
  launch_scan(c->at<uint32_t>(L.cnt2), c->at<uint32_t>(L.cell_start2), c->n3, c->at<uint32_t>(L.bsum), c->st);
  launch_scatter<T>(c->parts2<T>(c->cur2), c->parts2<T>(1 - c->cur2), c->np2, c->n, c->at<uint32_t>(L.rank2),
                    c->at<uint32_t>(L.cell_start2), c->st);
  c->cur2 = 1 - c->cur2;
  if (c->cfg.flags & PM_FLAG_DETERMINISTIC) {
    launch_order_by_id<T>(c->parts2<T>(c->cur2), c->parts2<T>(1 - c->cur2), c->np2, c->n,
                          c->at<uint32_t>(L.cell_start2), c->st);
    c->cur2 = 1 - c->cur2;
  }
}

template <typename T>
pm_status do_init(pm_ctx* c, const double* pos, const void* u, const uint32_t* ids, int on_device) {
  const Layout& L = c->L;
  const long np = c->np;
  // staging for host data: the second particle buffer
  const double* dpos = pos;
  const T* du = reinterpret_cast<const T*>(u);
  const uint32_t* dids = ids;
  if (!on_device) {
    double* sp = c->at<double>(L.pos[1]);
    T* su = c->at<T>(L.mom[1]);
    uint32_t* si = c->at<uint32_t>(L.ids[1]);
    hipMemcpyAsync(sp, pos, 3 * np * sizeof(double), hipMemcpyHostToDevice, c->st);
    hipMemcpyAsync(su, u, 3 * np * sizeof(T), hipMemcpyHostToDevice, c->st);
    if (ids) hipMemcpyAsync(si, ids, np * sizeof(uint32_t), hipMemcpyHostToDevice, c->st);
    dpos = sp; du = su; dids = ids ? si : nullptr;
  }
  // clear counts, error flag, FP64 scalars, fields and tensor state
  c->zero(L.cnt, c->n3 * 4);
  c->zero(L.err, 64);
  c->zero(L.scal, 8 * 8);
  for (int i = 0; i < 3; ++i) c->zero(L.phi[i], c->n3 * c->rs);
  if (L.chi) c->zero(L.chi, c->n3 * c->rs);
  for (int i = 0; i < 3; ++i)
    if (L.b[i]) c->zero(L.b[i], c->n3 * c->rs);
  if (L.hst) c->zero(L.hst, 4 * L.spec_comp * 2 * c->rs);
  if (L.a2b) c->zero(L.a2b, 3 * L.spec_comp * 2 * c->rs);
  Particles<T> p0 = c->parts<T>(0);
  launch_ingest<T>(dpos, du, dids, np, p0, c->n, c->at<uint32_t>(L.rank), c->at<uint32_t>(L.cnt),
                   c->at<int>(L.err), c->st);
  c->cur = 0;
  sort_particles<T>(c);
  if (!on_device) hipStreamSynchronize(c->st);  // host buffers may be released after return
  return c->hip_check("init_particles");
}

// the second species: ingest (positions wrapped, identifiers checked) and sort by cell
template <typename T>
pm_status do_init2(pm_ctx* c, const double* pos, const void* u, const uint32_t* ids, int on_device) {
  const Layout& L = c->L;
  const long np = c->np2;
  const double* dpos = pos;
  const T* du = reinterpret_cast<const T*>(u);
  const uint32_t* dids = ids;
  if (!on_device) {
    double* sp = c->at<double>(L.pos2[1]);
    T* su = c->at<T>(L.mom2[1]);
    uint32_t* si = c->at<uint32_t>(L.ids2[1]);
    hipMemcpyAsync(sp, pos, 3 * np * sizeof(double), hipMemcpyHostToDevice, c->st);
    hipMemcpyAsync(su, u, 3 * np * sizeof(T), hipMemcpyHostToDevice, c->st);
    if (ids) hipMemcpyAsync(si, ids, np * sizeof(uint32_t), hipMemcpyHostToDevice, c->st);
    dpos = sp; du = su; dids = ids ? si : nullptr;
  }
  c->zero(L.cnt2, c->n3 * 4);
  launch_ingest<T>(dpos, du, dids, np, c->parts2<T>(0), c->n, c->at<uint32_t>(L.rank2), c->at<uint32_t>(L.cnt2),
                   c->at<int>(L.err), c->st);
  c->cur2 = 0;
  sort_particles2<T>(c);
  if (!on_device) hipStreamSynchronize(c->st);
  return c->hip_check("init_particles_2");
}

// features of the last deposit (n00) and the latest phi -> three convolutions -> FP32 SoA output
// (scaled by rms |grad phi| when `scaled`, i.e. in force units)
template <typename T>
void closure_forward_impl(pm_ctx* c, bool scaled) {
  const Layout& L = c->L;
  double* cs = c->at<double>(L.cl_scal);
  float* rms = reinterpret_cast<float*>(cs + 1);
  // FP64 sum of n00 into cs[0], partials in cs[8..]
  if (c->cfg.precision == PM_FP64) launch_sum_f64(c->at<double>(L.dep), c->n3, cs, c->st);
  else launch_sum_as_f64(c->at<float>(L.dep), c->n3, cs, c->st);
  uint16_t* a0 = c->at<uint16_t>(L.cl_act[0]);
  uint16_t* a1 = c->at<uint16_t>(L.cl_act[1]);
  uint16_t* a2 = c->at<uint16_t>(L.cl_act[2]);
  closure_features<T>(c->at<T>(L.dep), c->at<T>(L.phi[c->i_phi]), c->n, cs, cs + 16, rms, a0, c->st);
  const uint16_t* wf = c->at<uint16_t>(L.cl_wf);
  const float* bias = c->at<float>(L.cl_bias);
  closure_conv(a0, wf, bias, c->n, 0, a1, nullptr, nullptr, c->st);
  closure_conv(a1, wf + 27 * 256, bias + 16, c->n, 0, a2, nullptr, nullptr, c->st);
  closure_conv(a2, wf + 2 * 27 * 256, bias + 32, c->n, 1, c->at<float>(L.cl_corr), nullptr, scaled ? rms : nullptr,
               c->st);
  c->cl_forwarded = true;
}

template <typename T>
pm_status do_update(pm_ctx* c, double dtau) {
  const Layout& L = c->L;
  GatherArgs<T> g;
  g.phi = c->at<T>(L.phi[c->i_phi]);
  g.chi = L.chi ? c->at<T>(L.chi) : nullptr;
  g.bx = L.b[0] ? c->at<T>(L.b[0]) : nullptr;
  g.by = L.b[1] ? c->at<T>(L.b[1]) : nullptr;
  g.bz = L.b[2] ? c->at<T>(L.b[2]) : nullptr;
  g.corr = nullptr;
  if (c->cl_on) {
    closure_forward_impl<T>(c, true);
    g.corr = c->at<float>(L.cl_corr);
  }
  g.mode = c->mode;
  g.dtau = dtau;
  g.a = c->a_of(c->tau);
  g.a_half = c->a_of(c->tau + 0.5 * dtau);
  c->stage_begin(PM_STAGE_KICK_DRIFT);
  launch_kick_drift<T>(c->parts<T>(c->cur), c->np, c->n, c->at<uint32_t>(L.cell_start), g, c->at<uint32_t>(L.rank),
                       c->at<uint32_t>(L.cnt), c->at<int>(L.err), c->st);
  if (c->np2 > 0)  // the second species: the same update (per unit mass) in the same fields
    launch_kick_drift<T>(c->parts2<T>(c->cur2), c->np2, c->n, c->at<uint32_t>(L.cell_start2), g,
                         c->at<uint32_t>(L.rank2), c->at<uint32_t>(L.cnt2), c->at<int>(L.err), c->st);
  c->stage_end(PM_STAGE_KICK_DRIFT);
  c->stage_begin(PM_STAGE_SORT);
  sort_particles<T>(c);
  if (c->np2 > 0) sort_particles2<T>(c);
  c->stage_end(PM_STAGE_SORT);
  c->tau += dtau;
  c->steps += 1;
  return c->hip_check("update_particles");
}

pm_status read_sticky(pm_ctx* c) {
  if (c->sticky) return (pm_status)c->sticky;
  int err = 0;
  if (hipMemcpy(&err, c->ws + c->L.err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
    c->sticky = PM_EHIP;
    c->last_error = "reading the device error flag failed";
    return PM_EHIP;
  }
  if (err & 1) { c->sticky = PM_ENAN; c->last_error = "non-finite particle coordinate or momentum"; }
  else if (err & 2) { c->sticky = PM_EINVAL; c->last_error = "particle identifier out of range"; }
  return (pm_status)c->sticky;
}

#define DISPATCH(c, F, ...) ((c)->cfg.precision == PM_FP64 ? F<double>(__VA_ARGS__) : F<float>(__VA_ARGS__))

}  // namespace

extern "C" {

pm_status pm_query_workspace(const pm_config* cfg, size_t* bytes) {
  pm_status s = check_config(cfg);
  if (s != PM_OK) return s;
  if (!bytes) return PM_EINVAL;
  *bytes = make_layout(*cfg).total;
  return PM_OK;
}

pm_status pm_create(const pm_config* cfg, void* d_workspace, size_t bytes, void* hip_stream, pm_ctx** out) {
  pm_status s = check_config(cfg);
  if (s != PM_OK) return s;
  if (!out) return PM_EINVAL;
  *out = nullptr;
  Layout L = make_layout(*cfg);
  if (!d_workspace || bytes < L.total || ((uintptr_t)d_workspace % kAlign) != 0) return PM_EWORKSPACE;
  pm_ctx* c = new (std::nothrow) pm_ctx();
  if (!c) return PM_EINVAL;
  c->cfg = *cfg;
  c->L = L;
  c->n = cfg->n_mesh;
  c->n3 = (long)c->n * c->n * c->n;
  c->np = cfg->n_particles;
  c->np2 = cfg->n_particles_2;
  c->mode = mode_of(cfg->physics);
  c->rs = cfg->precision == PM_FP64 ? 8 : 4;
  c->st = reinterpret_cast<hipStream_t>(hip_stream);
  c->ws = reinterpret_cast<unsigned char*>(d_workspace);
  if (cfg->precision == PM_FP64) upload_tables<double>(c); else upload_tables<float>(c);
  if (c->hip_check("create") != PM_OK) {
    delete c;
    return PM_EHIP;
  }
  *out = c;
  return PM_OK;
}

pm_status pm_destroy(pm_ctx* c) {
  if (!c) return PM_EINVAL;
  hipStreamSynchronize(c->st);
  for (int i = 0; i < PM_NSTAGES; ++i) {
    for (auto e : c->ev0[i]) (void)hipEventDestroy(e);
    for (auto e : c->ev1[i]) (void)hipEventDestroy(e);
  }
  delete c;
  return PM_OK;
}

pm_status pm_init_particles(pm_ctx* c, const double* pos, const void* u, const uint32_t* ids, int64_t n, double tau0,
                            int src_on_device) {
  if (!c || !pos || !u) return PM_EINVAL;
  if (n != c->np) return c->fail(PM_EINVAL, "n differs from the configured particle count");
  if (!(tau0 > 0) || !isfinite(tau0)) return c->fail(PM_EINVAL, "tau0 must be positive");
  c->sticky = 0;
  c->tau = tau0;
  c->steps = 0;
  c->last_step = 0;
  c->dtau_last = 0;
  c->i_phi = 0;
  c->i_prev = 1;
  c->deposited = c->solved = c->solved_once = false;
  c->have_particles2 = false;  // a second species is loaded again for the new start
  pm_status s = DISPATCH(c, do_init, c, pos, u, ids, src_on_device);
  if (s != PM_OK) return s;
  c->have_particles = true;
  return PM_OK;
}

pm_status pm_deposit(pm_ctx* c) {
  if (!c) return PM_EINVAL;
  if (!c->have_particles) return c->fail(PM_ESTATE, "deposit before init_particles");
  if (c->sticky) return (pm_status)c->sticky;
  if (c->np2 > 0 && !c->have_particles2) return c->fail(PM_ESTATE, "deposit before init_particles_2");
  const double a = c->a_of(c->tau);
  const Layout& L = c->L;
  const bool rel = c->mode != MODE_NEWTONIAN;
  const long nb = deposit_blocks(c->n);
  double* part = c->at<double>(L.part);
  c->stage_begin(PM_STAGE_DEPOSIT);
  if (c->cfg.precision == PM_FP64) {
    launch_deposit<double>(c->parts<double>(c->cur), c->at<uint32_t>(L.cell_start), c->n, L.ndep, rel, a, 1.0, false,
                           c->at<double>(L.dep), part, c->st);
    if (c->np2 > 0)
      launch_deposit<double>(c->parts2<double>(c->cur2), c->at<uint32_t>(L.cell_start2), c->n, L.ndep, rel, a,
                             c->weight2(), true, c->at<double>(L.dep), part + nb, c->st);
  } else {
    launch_deposit<float>(c->parts<float>(c->cur), c->at<uint32_t>(L.cell_start), c->n, L.ndep, rel, a, 1.0, false,
                          c->at<float>(L.dep), part, c->st);
    if (c->np2 > 0)
      launch_deposit<float>(c->parts2<float>(c->cur2), c->at<uint32_t>(L.cell_start2), c->n, L.ndep, rel, a,
                            c->weight2(), true, c->at<float>(L.dep), part + nb, c->st);
  }
  // FP64 sum over particles of e (species 2 weighted by its mass ratio), fixed order
  if (L.ndep > 1) launch_sum_f64(part, nb * (c->np2 > 0 ? 2 : 1), c->at<double>(L.scal) + 2, c->st);
  c->stage_end(PM_STAGE_DEPOSIT);
  c->deposited = true;
  return c->hip_check("deposit");
}

pm_status pm_solve_metric(pm_ctx* c, double dtau_prev) {
  if (!c) return PM_EINVAL;
  if (!c->deposited) return c->fail(PM_ESTATE, "solve_metric needs a preceding deposit");
  if (c->sticky) return (pm_status)c->sticky;
  if (!isfinite(dtau_prev)) return c->fail(PM_EINVAL, "dtau_prev must be finite");
  if (dtau_prev >= c->tau) return c->fail(PM_EINVAL, "dtau_prev must be smaller than tau");
  pm_status s = DISPATCH(c, do_solve, c, dtau_prev);
  if (s != PM_OK) return s;
  c->deposited = false;
  c->solved = true;
  c->solved_once = true;
  return PM_OK;
}

pm_status pm_update_particles(pm_ctx* c, double dtau) {
  if (!c) return PM_EINVAL;
  if (!c->solved) return c->fail(PM_ESTATE, "update_particles needs a preceding solve_metric");
  if (c->sticky) return (pm_status)c->sticky;
  if (!(dtau > 0) || !isfinite(dtau)) return c->fail(PM_EINVAL, "dtau must be positive");
  pm_status s = DISPATCH(c, do_update, c, dtau);
  if (s != PM_OK) return s;
  c->solved = false;
  c->last_step = dtau;
  return PM_OK;
}

pm_status pm_step(pm_ctx* c, double dtau) {
  if (!c) return PM_EINVAL;
  if (!(dtau > 0) || !isfinite(dtau)) return c->fail(PM_EINVAL, "dtau must be positive");
  const double dtau_prev = c->solved_once ? c->last_step : 0.0;
  pm_status s = pm_deposit(c);
  if (s != PM_OK) return s;
  s = pm_solve_metric(c, dtau_prev);
  if (s != PM_OK) return s;
  return pm_update_particles(c, dtau);
}

pm_status pm_get_field(pm_ctx* c, int id, void* dst, int dst_on_device) {
  if (!c || !dst) return PM_EINVAL;
  if (id < 0 || id >= PM_FIELD_COUNT) return c->fail(PM_EINVAL, "unknown field id");
  const size_t bytes = c->n3 * c->rs;
  const void* src = nullptr;
  if (id >= PM_FIELD_HXX && id <= PM_FIELD_HZZ) {
    if (c->mode != MODE_FULL) return c->fail(PM_EINVAL, "h_ij needs PM_FULL physics");
    // rebuild the six components into the spectrum buffer and transform the requested one
    const int comp = id - PM_FIELD_HXX;
    const Layout& L = c->L;
    // (the real result goes to the solutions' spectrum buffer, which holds nothing between solves;
    // the deposit, which the closure reads after a solve, stays untouched)
    if (c->cfg.precision == PM_FP64) {
      cplx<double>* spec = c->at<cplx<double>>(L.spec);
      launch_tensor_components<double>(spec, L.spec_comp, c->n, L.nhp, c->at<double>(L.kt),
                                       c->at<cplx<double>>(L.hst), c->st);
      double* out[1] = {c->at<double>(L.spec_out)};
      fft_inverse<double>(c->n, L.nhp, spec + comp * L.spec_comp, 1, out, 1.0 / c->n3, c->at<cplx<double>>(L.tw), c->st);
    } else {
      cplx<float>* spec = c->at<cplx<float>>(L.spec);
      launch_tensor_components<float>(spec, L.spec_comp, c->n, L.nhp, c->at<float>(L.kt), c->at<cplx<float>>(L.hst),
                                      c->st);
      float* out[1] = {c->at<float>(L.spec_out)};
      fft_inverse<float>(c->n, L.nhp, spec + comp * L.spec_comp, 1, out, 1.0 / c->n3, c->at<cplx<float>>(L.tw), c->st);
    }
    src = c->ws + L.spec_out;
  } else {
    src = c->field_ptr(id);
    if (!src) return c->fail(PM_EINVAL, "field not present for this physics");
  }
  if (dst_on_device) {
    hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->st);
  } else {
    hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->st);
    hipStreamSynchronize(c->st);
  }
  pm_status s = c->hip_check("get_field");
  if (s != PM_OK) return s;
  return dst_on_device ? PM_OK : read_sticky(c);
}

pm_status pm_set_field(pm_ctx* c, int id, const void* src, int src_on_device) {
  if (!c || !src) return PM_EINVAL;
  if (id < 0 || id >= PM_FIELD_HXX) return c->fail(PM_EINVAL, "field cannot be set");
  void* dst = c->field_ptr(id);
  if (!dst) return c->fail(PM_EINVAL, "field not present for this physics");
  hipMemcpyAsync(dst, src, c->n3 * c->rs, src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->st);
  if (!src_on_device) hipStreamSynchronize(c->st);
  if (id == PM_FIELD_N00 && c->mode != MODE_NEWTONIAN) {
    // the homogeneous mode then comes from the mesh: sum of n00 in FP64
    if (c->cfg.precision == PM_FP64)
      launch_sum_f64(c->at<double>(c->L.dep), c->n3, c->at<double>(c->L.scal) + 2, c->st);
    else
      launch_sum_as_f64(c->at<float>(c->L.dep), c->n3, c->at<double>(c->L.scal) + 2, c->st);
  }
  if (id <= PM_FIELD_NZZ) c->deposited = true;
  else if (id != PM_FIELD_PHI_PREV) c->solved = true;
  return c->hip_check("set_field");
}

pm_status pm_get_particles(pm_ctx* c, double* pos, void* u, uint32_t* ids, int dst_on_device) {
  if (!c) return PM_EINVAL;
  if (!c->have_particles) return c->fail(PM_ESTATE, "no particles");
  const Layout& L = c->L;
  const long np = c->np;
  const int other = 1 - c->cur;
  double* sp = dst_on_device ? pos : (pos ? c->at<double>(L.pos[other]) : nullptr);
  void* su = dst_on_device ? u : (u ? (void*)(c->ws + L.mom[other]) : nullptr);
  uint32_t* si = dst_on_device ? ids : (ids ? c->at<uint32_t>(L.ids[other]) : nullptr);
  if (c->cfg.precision == PM_FP64)
    launch_export<double>(c->parts<double>(c->cur), np, sp, reinterpret_cast<double*>(su), si, c->st);
  else
    launch_export<float>(c->parts<float>(c->cur), np, sp, reinterpret_cast<float*>(su), si, c->st);
  if (!dst_on_device) {
    if (pos) hipMemcpyAsync(pos, sp, 3 * np * sizeof(double), hipMemcpyDeviceToHost, c->st);
    if (u) hipMemcpyAsync(u, su, 3 * np * c->rs, hipMemcpyDeviceToHost, c->st);
    if (ids) hipMemcpyAsync(ids, si, np * sizeof(uint32_t), hipMemcpyDeviceToHost, c->st);
    hipStreamSynchronize(c->st);
  }
  pm_status s = c->hip_check("get_particles");
  if (s != PM_OK) return s;
  return dst_on_device ? PM_OK : read_sticky(c);
}

pm_status pm_init_particles_2(pm_ctx* c, const double* pos, const void* u, const uint32_t* ids, int64_t n,
                              int src_on_device) {
  if (!c || !pos || !u) return PM_EINVAL;
  if (c->np2 == 0) return c->fail(PM_EINVAL, "the configuration has no second species");
  if (n != c->np2) return c->fail(PM_EINVAL, "n differs from the configured count of the second species");
  if (!c->have_particles) return c->fail(PM_ESTATE, "init_particles_2 before init_particles");
  if (c->sticky) return (pm_status)c->sticky;
  pm_status s = DISPATCH(c, do_init2, c, pos, u, ids, src_on_device);
  if (s != PM_OK) return s;
  c->have_particles2 = true;
  c->deposited = c->solved = false;
  return PM_OK;
}

pm_status pm_get_particles_2(pm_ctx* c, double* pos, void* u, uint32_t* ids, int dst_on_device) {
  if (!c) return PM_EINVAL;
  if (c->np2 == 0 || !c->have_particles2) return c->fail(PM_ESTATE, "no second species loaded");
  const Layout& L = c->L;
  const long np = c->np2;
  const int other = 1 - c->cur2;
  double* sp = dst_on_device ? pos : (pos ? c->at<double>(L.pos2[other]) : nullptr);
  void* su = dst_on_device ? u : (u ? (void*)(c->ws + L.mom2[other]) : nullptr);
  uint32_t* si = dst_on_device ? ids : (ids ? c->at<uint32_t>(L.ids2[other]) : nullptr);
  if (c->cfg.precision == PM_FP64)
    launch_export<double>(c->parts2<double>(c->cur2), np, sp, reinterpret_cast<double*>(su), si, c->st);
  else
    launch_export<float>(c->parts2<float>(c->cur2), np, sp, reinterpret_cast<float*>(su), si, c->st);
  if (!dst_on_device) {
    if (pos) hipMemcpyAsync(pos, sp, 3 * np * sizeof(double), hipMemcpyDeviceToHost, c->st);
    if (u) hipMemcpyAsync(u, su, 3 * np * c->rs, hipMemcpyDeviceToHost, c->st);
    if (ids) hipMemcpyAsync(ids, si, np * sizeof(uint32_t), hipMemcpyDeviceToHost, c->st);
    hipStreamSynchronize(c->st);
  }
  pm_status s = c->hip_check("get_particles_2");
  if (s != PM_OK) return s;
  return dst_on_device ? PM_OK : read_sticky(c);
}

pm_status pm_diagnostics(pm_ctx* c, double* out, int n) {
  if (!c || !out || n < 1) return PM_EINVAL;
  if (!c->have_particles || (c->np2 > 0 && !c->have_particles2)) return c->fail(PM_ESTATE, "no particles");
  if (c->sticky) return (pm_status)c->sticky;
  double* sc = c->at<double>(c->L.scal);
  // total momentum per unit mass of species 1: FP64 sums of the SoA momenta (scalars 3..5 for species 1,
  // then 3..5 again for species 2 after species 1's were read)
  double mom[3] = {0, 0, 0};
  for (int s = 0; s < (c->np2 > 0 ? 2 : 1); ++s) {
    const double w = s == 0 ? 1.0 : c->weight2();
    for (int d = 0; d < 3; ++d) {
      if (c->cfg.precision == PM_FP64) {
        const Particles<double> p = s == 0 ? c->parts<double>(c->cur) : c->parts2<double>(c->cur2);
        const double* u = d == 0 ? p.ux : (d == 1 ? p.uy : p.uz);
        launch_sum_f64(u, s == 0 ? c->np : c->np2, sc + 3 + d, c->st);
      } else {
        const Particles<float> p = s == 0 ? c->parts<float>(c->cur) : c->parts2<float>(c->cur2);
        const float* u = d == 0 ? p.ux : (d == 1 ? p.uy : p.uz);
        launch_sum_as_f64(u, s == 0 ? c->np : c->np2, sc + 3 + d, c->st);
      }
    }
    double h[6];
    if (hipMemcpyAsync(h, sc, 6 * sizeof(double), hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess)
      return c->fail(PM_EHIP, "reading the diagnostics failed");
    for (int d = 0; d < 3; ++d) mom[d] += w * h[3 + d];
    if (s == 0) {
      const double v[5] = {h[2], h[1], 0, 0, 0};
      for (int i = 0; i < n && i < 2; ++i) out[i] = v[i];
    }
  }
  for (int i = 2; i < n && i < 5; ++i) out[i] = mom[i - 2];
  pm_status st = c->hip_check("diagnostics");
  if (st != PM_OK) return st;
  return read_sticky(c);
}

pm_status pm_get_time(pm_ctx* c, double* tau, double* a, int64_t* steps) {
  if (!c) return PM_EINVAL;
  if (tau) *tau = c->tau;
  if (a) *a = c->a_of(c->tau);
  if (steps) *steps = c->steps;
  return PM_OK;
}

pm_status pm_background(const pm_config* cfg, double tau, double* a, double* hconf) {
  if (!cfg || !(cfg->box_mpch > 0) || !(tau > 0)) return PM_EINVAL;
  const double h0 = cfg->box_mpch / 2997.92458;
  const double x = 0.5 * h0 * tau;
  if (a) *a = x * x;
  if (hconf) *hconf = 2.0 / tau;
  return PM_OK;
}

pm_status pm_tau_of_a(const pm_config* cfg, double a, double* tau) {
  if (!cfg || !(cfg->box_mpch > 0) || !(a > 0) || !tau) return PM_EINVAL;
  *tau = 2.0 * sqrt(a) / (cfg->box_mpch / 2997.92458);
  return PM_OK;
}

pm_status pm_get_timings(pm_ctx* c, double* ms, int64_t* calls, int n) {
  if (!c || !ms) return PM_EINVAL;
  if (!(c->cfg.flags & PM_FLAG_TIMINGS)) return c->fail(PM_EUNSUPPORTED, "context created without PM_FLAG_TIMINGS");
  c->drain_events();
  for (int i = 0; i < n && i < PM_NSTAGES; ++i) {
    ms[i] = c->ev_ms[i];
    if (calls) calls[i] = c->ev_calls[i];
  }
  for (int i = 0; i < PM_NSTAGES; ++i) {
    c->ev_ms[i] = 0;
    c->ev_calls[i] = 0;
  }
  return c->hip_check("get_timings");
}

pm_status pm_sync(pm_ctx* c) {
  if (!c) return PM_EINVAL;
  if (hipStreamSynchronize(c->st) != hipSuccess) {
    c->sticky = PM_EHIP;
    c->last_error = "stream synchronisation failed";
    return PM_EHIP;
  }
  pm_status s = c->hip_check("sync");
  if (s != PM_OK) return s;
  return read_sticky(c);
}

pm_status pm_debug_fft(pm_ctx* c, const void* d_in, void* d_out, int direction) {
  if (!c || !d_in || !d_out) return PM_EINVAL;
  if (direction != 1 && direction != -1) return PM_EINVAL;
  const Layout& L = c->L;
  if (c->cfg.precision == PM_FP64) {
    cplx<double>* spec = c->at<cplx<double>>(L.spec);
    if (direction == 1) {
      SrcArgsH<double> s;
      s.raw = reinterpret_cast<const double*>(d_in);
      fft_forward<double>(s, MODE_RAW, c->n, L.nhp, spec, 1, c->at<cplx<double>>(L.tw), c->st);
      launch_copy_unpad<double>(spec, c->n, L.nhp, reinterpret_cast<cplx<double>*>(d_out), false, c->st);
    } else {
      launch_copy_unpad<double>(spec, c->n, L.nhp, const_cast<cplx<double>*>(reinterpret_cast<const cplx<double>*>(d_in)),
                                true, c->st);
      double* out[1] = {reinterpret_cast<double*>(d_out)};
      fft_inverse<double>(c->n, L.nhp, spec, 1, out, 1.0 / c->n3, c->at<cplx<double>>(L.tw), c->st);
    }
  } else {
    cplx<float>* spec = c->at<cplx<float>>(L.spec);
    if (direction == 1) {
      SrcArgsH<float> s;
      s.raw = reinterpret_cast<const float*>(d_in);
      fft_forward<float>(s, MODE_RAW, c->n, L.nhp, spec, 1, c->at<cplx<float>>(L.tw), c->st);
      launch_copy_unpad<float>(spec, c->n, L.nhp, reinterpret_cast<cplx<float>*>(d_out), false, c->st);
    } else {
      launch_copy_unpad<float>(spec, c->n, L.nhp, const_cast<cplx<float>*>(reinterpret_cast<const cplx<float>*>(d_in)),
                               true, c->st);
      float* out[1] = {reinterpret_cast<float*>(d_out)};
      fft_inverse<float>(c->n, L.nhp, spec, 1, out, 1.0 / c->n3, c->at<cplx<float>>(L.tw), c->st);
    }
  }
  return c->hip_check("debug_fft");
}

}  // extern "C"

namespace {
template <typename T>
pm_status do_power_spectrum(pm_ctx* c, int subtract, double* k_out, double* p_out, double* modes_out) {
  const Layout& L = c->L;
  // the count field lives in the solutions' spectrum buffer (free between solves; at least n^3
  // values), so that the deposit and the fields of the time-stepping state stay untouched
  T* cnt = c->at<T>(L.spec_out);
  launch_deposit<T>(c->parts<T>(c->cur), c->at<uint32_t>(L.cell_start), c->n, 1, false, 1.0, 1.0, false, cnt, nullptr,
                    c->st);
  SrcArgsH<T> s;
  s.raw = cnt;
  cplx<T>* spec = c->at<cplx<T>>(L.spec);
  fft_forward<T>(s, MODE_RAW, c->n, L.nhp, spec, 1, c->at<cplx<T>>(L.tw), c->st);
  // the count field has been transformed: its buffer holds the partials and the result
  const size_t scratch = (size_t)L.nout * L.spec_comp * 2 * c->rs;
  const int nblocks = pk_blocks(c->n, scratch);
  const int nb = c->n / 2 + 1;
  double* part = reinterpret_cast<double*>(cnt);
  const double box3 = 1.0;  // box units: P in units of L^3, converted below
  launch_power_spectrum<T>(spec, c->n, L.nhp, box3 / ((double)c->np * (double)c->np), subtract ? box3 / (double)c->np : 0.0,
                           nblocks, part, c->st);
  std::vector<double> h(3 * nb);
  (void)hipMemcpyAsync(h.data(), part + (long)nblocks * 3 * nb, 3 * nb * sizeof(double), hipMemcpyDeviceToHost, c->st);
  (void)hipStreamSynchronize(c->st);
  const double Lb = c->cfg.box_mpch, kf = 2.0 * M_PI / Lb;
  for (int b = 0; b < nb; ++b) {
    const double m = h[b];
    modes_out[b] = m;
    p_out[b] = m > 0 ? h[nb + b] / m * Lb * Lb * Lb : 0.0;
    k_out[b] = m > 0 ? h[2 * nb + b] / m * kf : 0.0;
  }
  return c->hip_check("power_spectrum");
}
}  // namespace

extern "C" {

pm_status pm_power_spectrum(pm_ctx* c, int subtract_shot_noise, double* k_out, double* p_out, double* modes_out) {
  if (!c || !k_out || !p_out || !modes_out) return PM_EINVAL;
  if (!c->have_particles) return c->fail(PM_ESTATE, "no particles");
  pm_status s = DISPATCH(c, do_power_spectrum, c, subtract_shot_noise, k_out, p_out, modes_out);
  if (s != PM_OK) return s;
  return read_sticky(c);
}

}  // extern "C"

// ---- checkpoint of the time-stepping state ---------------------------------------------------
namespace {

constexpr uint64_t kStateMagic = 0x31455441545347ULL;  // "GSTATE1" (little-endian bytes)
constexpr uint32_t kStateVersion = 3;
constexpr size_t kStateHeader = 1024;
constexpr int kStateMaxSec = 32;

struct StateHeader {
  uint64_t magic;
  uint32_t version, nsec;
  int32_t n_mesh, precision, physics, parabolic;
  int64_t n_particles;
  double tau, last_step, dtau_last;
  int64_t steps;
  int32_t deposited, solved, solved_once, pad;
  int64_t n_particles_2;
  double mass_fraction_2;
  uint64_t total;
  uint64_t off[kStateMaxSec], bytes[kStateMaxSec];
};
static_assert(sizeof(StateHeader) <= kStateHeader, "state header too large");

// workspace regions that make up the state: the sorted particles (buffer `cur`), the cell offsets
// of the sort, phi of the latest and the previous solve and the latest solve's increment, chi, B,
// the tensor and parabolic-B spectra, the FP64 scalars and, between a deposit and its solve, the
// deposit
int state_sections(const pm_ctx* c, int cur, int cur2, int i_phi, int i_prev, bool with_dep, size_t* ws_off,
                   size_t* bytes) {
  const Layout& L = c->L;
  const long np = c->np, n3 = c->n3;
  const size_t rs = c->rs;
  int k = 0;
  auto add = [&](size_t off, size_t b) { ws_off[k] = off; bytes[k] = b; ++k; };
  add(L.pos[cur], 3 * np * 8 + 2 * kSkew);
  add(L.mom[cur], 3 * np * rs + 2 * kSkew);
  add(L.ids[cur], np * 4);
  add(L.cell_start, (n3 + 1) * 4);
  if (c->np2 > 0) {
    const long np2 = c->np2;
    add(L.pos2[cur2], 3 * np2 * 8 + 2 * kSkew);
    add(L.mom2[cur2], 3 * np2 * rs + 2 * kSkew);
    add(L.ids2[cur2], np2 * 4);
    add(L.cell_start2, (n3 + 1) * 4);
  }
  add(L.phi[i_phi], n3 * rs);
  add(L.phi[i_prev], n3 * rs);
  if (c->mode != MODE_NEWTONIAN) add(L.phi[3 - i_phi - i_prev], n3 * rs);  // increment of the latest solve
  if (L.chi) add(L.chi, n3 * rs);
  for (int i = 0; i < 3; ++i)
    if (L.b[i]) add(L.b[i], n3 * rs);
  if (L.hst) add(L.hst, 4 * L.spec_comp * 2 * rs);
  if (L.a2b) add(L.a2b, 3 * L.spec_comp * 2 * rs);
  add(L.scal, 8 * 8);
  if (with_dep) add(L.dep, (size_t)L.ndep * n3 * rs);
  return k;
}

size_t state_blob_offsets(int nsec, const size_t* bytes, uint64_t* off) {
  size_t o = kStateHeader;
  for (int i = 0; i < nsec; ++i) {
    off[i] = o;
    o = align_up(o + bytes[i]);
  }
  return o;
}

}  // namespace

extern "C" {

pm_status pm_get_state(pm_ctx* c, void* blob, size_t* bytes, int dst_on_device) {
  if (!c || !bytes) return PM_EINVAL;
  if (!c->have_particles) return c->fail(PM_ESTATE, "no particles");
  if (c->np2 > 0 && !c->have_particles2) return c->fail(PM_ESTATE, "no second species loaded");
  if (c->sticky) return (pm_status)c->sticky;
  size_t ws_off[kStateMaxSec], sb[kStateMaxSec];
  const int nsec = state_sections(c, c->cur, c->cur2, c->i_phi, c->i_prev, c->deposited, ws_off, sb);
  StateHeader h;
  memset(&h, 0, sizeof(h));
  const size_t total = state_blob_offsets(nsec, sb, h.off);
  if (!blob) {
    *bytes = total;
    return PM_OK;
  }
  if (*bytes < total) {
    *bytes = total;
    return c->fail(PM_EINVAL, "state buffer too small");
  }
  h.magic = kStateMagic;
  h.version = kStateVersion;
  h.nsec = (uint32_t)nsec;
  h.n_mesh = c->n;
  h.precision = c->cfg.precision;
  h.physics = c->cfg.physics;
  h.parabolic = c->L.a2b ? 1 : 0;
  h.n_particles = c->np;
  h.n_particles_2 = c->np2;
  h.mass_fraction_2 = c->cfg.mass_fraction_2;
  h.tau = c->tau;
  h.last_step = c->last_step;
  h.dtau_last = c->dtau_last;
  h.steps = c->steps;
  h.deposited = c->deposited;
  h.solved = c->solved;
  h.solved_once = c->solved_once;
  h.total = total;
  for (int i = 0; i < nsec; ++i) h.bytes[i] = sb[i];
  unsigned char* dst = reinterpret_cast<unsigned char*>(blob);
  const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  // the whole header block, zero beyond the struct
  std::vector<unsigned char> head(kStateHeader, 0);
  memcpy(head.data(), &h, sizeof(h));
  if (dst_on_device)
    (void)hipMemcpyAsync(dst, head.data(), kStateHeader, hipMemcpyHostToDevice, c->st);
  else
    memcpy(dst, head.data(), kStateHeader);
  for (int i = 0; i < nsec; ++i) {
    (void)hipMemcpyAsync(dst + h.off[i], c->ws + ws_off[i], sb[i], kind, c->st);
    // zero the alignment gap after the section, so that equal states give equal blobs
    const size_t end = h.off[i] + sb[i], next = i + 1 < nsec ? h.off[i + 1] : total;
    if (next > end) {
      if (dst_on_device) c->zero_bytes(dst + end, next - end);
      else memset(dst + end, 0, next - end);
    }
  }
  // the header copy reads host memory of this frame: wait for it (and for host destinations)
  (void)hipStreamSynchronize(c->st);
  *bytes = total;
  pm_status s = c->hip_check("get_state");
  if (s != PM_OK) return s;
  return read_sticky(c);
}

pm_status pm_set_state(pm_ctx* c, const void* blob, size_t bytes, int src_on_device) {
  if (!c || !blob) return PM_EINVAL;
  if (bytes < kStateHeader) return c->fail(PM_EINVAL, "state blob too small");
  StateHeader h;
  if (src_on_device) {
    if (hipMemcpyAsync(&h, blob, sizeof(h), hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess)
      return c->fail(PM_EHIP, "reading the state header failed");
  } else {
    memcpy(&h, blob, sizeof(h));
  }
  if (h.magic != kStateMagic || h.version != kStateVersion) return c->fail(PM_EINVAL, "not a state blob");
  if (h.n_mesh != c->n || h.precision != c->cfg.precision || h.physics != c->cfg.physics ||
      h.parabolic != (c->L.a2b ? 1 : 0) || h.n_particles != c->np || h.n_particles_2 != c->np2 ||
      h.mass_fraction_2 != c->cfg.mass_fraction_2)
    return c->fail(PM_EINVAL, "state blob of another configuration");
  if (!(h.tau > 0) || !isfinite(h.tau) || h.steps < 0 || h.total > bytes)
    return c->fail(PM_EINVAL, "corrupt state header");
  // restore into particle buffer 0 and phi slots 0 (latest), 1 (previous) and 2 (increment)
  size_t ws_off[kStateMaxSec], sb[kStateMaxSec];
  uint64_t off[kStateMaxSec];
  const int nsec = state_sections(c, 0, 0, 0, 1, h.deposited != 0, ws_off, sb);
  const size_t total = state_blob_offsets(nsec, sb, off);
  if ((int)h.nsec != nsec || h.total != total) return c->fail(PM_EINVAL, "corrupt state header");
  for (int i = 0; i < nsec; ++i)
    if (h.off[i] != off[i] || h.bytes[i] != sb[i]) return c->fail(PM_EINVAL, "corrupt state header");
  const unsigned char* src = reinterpret_cast<const unsigned char*>(blob);
  const hipMemcpyKind kind = src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  for (int i = 0; i < nsec; ++i) (void)hipMemcpyAsync(c->ws + ws_off[i], src + off[i], sb[i], kind, c->st);
  // the per-cell counters are zero between sorts; the device error flag starts clear
  c->zero(c->L.cnt, c->n3 * 4);
  if (c->np2 > 0) c->zero(c->L.cnt2, c->n3 * 4);
  c->zero(c->L.err, 64);
  // the body is not trusted: the kernels index LDS tiles and ranges by the cell offsets and the
  // positions, so both are checked against each other before the context may run on them
  int* err = c->at<int>(c->L.err);
  if (c->cfg.precision == PM_FP64) {
    launch_check_store<double>(c->parts<double>(0), c->np, c->n, c->at<uint32_t>(c->L.cell_start), err, c->st);
    if (c->np2 > 0)
      launch_check_store<double>(c->parts2<double>(0), c->np2, c->n, c->at<uint32_t>(c->L.cell_start2), err, c->st);
  } else {
    launch_check_store<float>(c->parts<float>(0), c->np, c->n, c->at<uint32_t>(c->L.cell_start), err, c->st);
    if (c->np2 > 0)
      launch_check_store<float>(c->parts2<float>(0), c->np2, c->n, c->at<uint32_t>(c->L.cell_start2), err, c->st);
  }
  int flag = 0;
  if (hipMemcpyAsync(&flag, err, sizeof(int), hipMemcpyDeviceToHost, c->st) != hipSuccess ||
      hipStreamSynchronize(c->st) != hipSuccess) {
    c->have_particles = c->have_particles2 = false;
    c->deposited = c->solved = false;
    return c->fail(PM_EHIP, "checking the restored state failed");
  }
  if (flag & 4) {
    // nothing of the blob may be used: the context has no particles until the next load or restore
    c->zero(c->L.err, 64);
    c->have_particles = c->have_particles2 = false;
    c->deposited = c->solved = c->solved_once = false;
    return c->fail(PM_EINVAL, "state blob body inconsistent (cell offsets, positions or identifiers)");
  }
  c->cur = 0;
  c->cur2 = 0;
  c->have_particles2 = c->np2 > 0;
  c->i_phi = 0;
  c->i_prev = 1;
  c->tau = h.tau;
  c->last_step = h.last_step;
  c->dtau_last = h.dtau_last;
  c->steps = h.steps;
  c->deposited = h.deposited != 0;
  c->solved = h.solved != 0;
  c->solved_once = h.solved_once != 0;
  c->have_particles = true;
  c->cl_forwarded = false;
  c->sticky = 0;
  c->last_error.clear();
  return c->hip_check("set_state");
}

pm_status pm_gather_grad_phi(pm_ctx* c, void* out, int dst_on_device) {
  if (!c || !out) return PM_EINVAL;
  if (!c->have_particles) return c->fail(PM_ESTATE, "no particles");
  const Layout& L = c->L;
  const long np = c->np;
  const int other = 1 - c->cur;
  void* dst = dst_on_device ? out : (void*)(c->ws + L.pos[other]);  // 3 np values fit the FP64 position block
  if (c->cfg.precision == PM_FP64)
    gather_grad_phi<double>(c->parts<double>(c->cur), np, c->n, c->at<double>(L.phi[c->i_phi]),
                            reinterpret_cast<double*>(dst), c->st);
  else
    gather_grad_phi<float>(c->parts<float>(c->cur), np, c->n, c->at<float>(L.phi[c->i_phi]),
                           reinterpret_cast<float*>(dst), c->st);
  if (!dst_on_device) {
    (void)hipMemcpyAsync(out, dst, 3 * np * c->rs, hipMemcpyDeviceToHost, c->st);
    (void)hipStreamSynchronize(c->st);
  }
  return c->hip_check("gather_grad_phi");
}

static pm_status closure_ready(pm_ctx* c, bool params) {
  if (!c) return PM_EINVAL;
  if (!c->L.closure) return c->fail(PM_EUNSUPPORTED, "context created without PM_FLAG_CLOSURE");
  if (params && !c->cl_params) return c->fail(PM_ESTATE, "closure parameters not set");
  return PM_OK;
}

pm_status pm_closure_set_params(pm_ctx* c, const float* params, int src_on_device) {
  pm_status s = closure_ready(c, false);
  if (s != PM_OK) return s;
  if (!params) return PM_EINVAL;
  const Layout& L = c->L;
  const float* src = params;
  if (!src_on_device) {
    // stage through the closure's output buffer (3 n^3 floats >= 49152 bytes for n >= 16, more than
    // the parameters need); its contents are stale afterwards, so a new forward pass is required
    static_assert(3 * 16 * 16 * 16 >= PM_CLOSURE_NPARAM, "staging buffer too small");
    float* dst = c->at<float>(L.cl_corr);
    (void)hipMemcpyAsync(dst, params, PM_CLOSURE_NPARAM * sizeof(float), hipMemcpyHostToDevice, c->st);
    src = dst;
    c->cl_forwarded = false;
  }
  closure_pack(src, c->at<uint16_t>(L.cl_wf), c->at<uint16_t>(L.cl_wb), c->at<float>(L.cl_bias), c->st);
  if (!src_on_device) (void)hipStreamSynchronize(c->st);
  c->cl_params = true;
  return c->hip_check("closure_set_params");
}

pm_status pm_closure_enable(pm_ctx* c, int on) {
  pm_status s = closure_ready(c, on != 0);
  if (s != PM_OK) return s;
  c->cl_on = on != 0;
  return PM_OK;
}

pm_status pm_closure_forward(pm_ctx* c, int scaled) {
  pm_status s = closure_ready(c, true);
  if (s != PM_OK) return s;
  if (!c->solved) return c->fail(PM_ESTATE, "closure_forward needs a deposit and a metric solve");
  if (c->cfg.precision == PM_FP64) closure_forward_impl<double>(c, scaled != 0);
  else closure_forward_impl<float>(c, scaled != 0);
  return c->hip_check("closure_forward");
}

pm_status pm_closure_scale(pm_ctx* c, double* rms) {
  pm_status s = closure_ready(c, true);
  if (s != PM_OK) return s;
  if (!rms) return PM_EINVAL;
  if (!c->cl_forwarded) return c->fail(PM_ESTATE, "closure_scale needs closure_forward");
  float v = 0.f;
  (void)hipStreamSynchronize(c->st);
  if (hipMemcpy(&v, c->at<double>(c->L.cl_scal) + 1, sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return c->fail(PM_EHIP, "reading the closure scale failed");
  *rms = v;
  return PM_OK;
}

pm_status pm_closure_gather(pm_ctx* c, float* out, int dst_on_device) {
  pm_status s = closure_ready(c, true);
  if (s != PM_OK) return s;
  if (!out) return PM_EINVAL;
  if (!c->cl_forwarded) return c->fail(PM_ESTATE, "closure_gather needs closure_forward");
  const Layout& L = c->L;
  const long np = c->np;
  float* dst = dst_on_device ? out : reinterpret_cast<float*>(c->ws + L.pos[1 - c->cur]);
  if (c->cfg.precision == PM_FP64)
    closure_gather3<double>(c->parts<double>(c->cur), np, c->n, c->at<float>(L.cl_corr), dst, c->st);
  else
    closure_gather3<float>(c->parts<float>(c->cur), np, c->n, c->at<float>(L.cl_corr), dst, c->st);
  if (!dst_on_device) {
    (void)hipMemcpyAsync(out, dst, 3 * np * sizeof(float), hipMemcpyDeviceToHost, c->st);
    (void)hipStreamSynchronize(c->st);
  }
  return c->hip_check("closure_gather");
}

pm_status pm_closure_backward(pm_ctx* c, const float* d_dpred, float* d_grad) {
  pm_status s = closure_ready(c, true);
  if (s != PM_OK) return s;
  if (!d_dpred || !d_grad) return PM_EINVAL;
  const Layout& L = c->L;
  if (!L.cl_train) return c->fail(PM_EUNSUPPORTED, "closure training needs n_mesh <= 256");
  if (!c->cl_forwarded) return c->fail(PM_ESTATE, "closure_backward needs closure_forward");
  const int n = c->n;
  float* dcorr = c->at<float>(L.cl_dcorr);
  c->zero(L.cl_dcorr, 3 * c->n3 * 4);
  if (c->cfg.precision == PM_FP64)
    closure_gather3_adjoint<double>(c->parts<double>(c->cur), c->np, n, d_dpred, dcorr, c->st);
  else
    closure_gather3_adjoint<float>(c->parts<float>(c->cur), c->np, n, d_dpred, dcorr, c->st);
  uint16_t* d3 = c->at<uint16_t>(L.cl_dact[2]);
  uint16_t* d2 = c->at<uint16_t>(L.cl_dact[1]);
  uint16_t* d1 = c->at<uint16_t>(L.cl_dact[0]);
  const uint16_t* a0 = c->at<uint16_t>(L.cl_act[0]);
  const uint16_t* a1 = c->at<uint16_t>(L.cl_act[1]);
  const uint16_t* a2 = c->at<uint16_t>(L.cl_act[2]);
  const uint16_t* wb = c->at<uint16_t>(L.cl_wb);
  float* part = c->at<float>(L.cl_part);
  closure_soa3_to_bf16(dcorr, c->n3, d3, c->st);
  const long off2 = 16 * 4 * 27 + 16, off3 = off2 + 16 * 16 * 27 + 16;
  closure_wgrad(a2, d3, n, part, 16, 3, d_grad, off3, c->st);
  closure_conv(d3, wb + 2 * 27 * 256, nullptr, n, 2, d2, a2, nullptr, c->st);
  closure_wgrad(a1, d2, n, part, 16, 16, d_grad, off2, c->st);
  closure_conv(d2, wb + 27 * 256, nullptr, n, 2, d1, a1, nullptr, c->st);
  closure_wgrad(a0, d1, n, part, 4, 16, d_grad, 0, c->st);
  return c->hip_check("closure_backward");
}

pm_status pm_closure_loss(pm_ctx* c, const float* d_target, float* d_dpred, double* loss) {
  pm_status s = closure_ready(c, true);
  if (s != PM_OK) return s;
  if (!d_target || !d_dpred) return PM_EINVAL;
  if (!c->cl_forwarded) return c->fail(PM_ESTATE, "closure_loss needs closure_forward");
  if (c->np < 1) return c->fail(PM_ESTATE, "closure_loss needs particles");
  const Layout& L = c->L;
  double* cs = c->at<double>(L.cl_scal);
  if (c->cfg.precision == PM_FP64)
    closure_loss3<double>(c->parts<double>(c->cur), c->np, c->n, c->at<float>(L.cl_corr), d_target, d_dpred, cs + 1024,
                          cs + 4, c->st);
  else
    closure_loss3<float>(c->parts<float>(c->cur), c->np, c->n, c->at<float>(L.cl_corr), d_target, d_dpred, cs + 1024,
                         cs + 4, c->st);
  if (loss) {
    if (hipMemcpyAsync(loss, cs + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess)
      return c->fail(PM_EHIP, "reading the closure loss failed");
  }
  return c->hip_check("closure_loss");
}

pm_status pm_cube_symmetry(pm_ctx* c, long n, const int* perm, int flip, const double* d_pos, const float* d_u,
                           const float* d_v, double* d_pos_out, float* d_u_out, float* d_v_out) {
  if (!c) return PM_EINVAL;
  if (!perm || n < 0 || flip < 0 || flip > 7) return c->fail(PM_EINVAL, "cube_symmetry: bad arguments");
  bool seen[3] = {false, false, false};
  for (int d = 0; d < 3; ++d) {
    if (perm[d] < 0 || perm[d] > 2 || seen[perm[d]])
      return c->fail(PM_EINVAL, "cube_symmetry: perm must be a permutation of 0, 1, 2");
    seen[perm[d]] = true;
  }
  if (n == 0) return PM_OK;
  if (!d_pos || !d_u || !d_v || !d_pos_out || !d_u_out || !d_v_out) return PM_EINVAL;
  closure_cube_symmetry(n, perm, flip, d_pos, d_u, d_v, d_pos_out, d_u_out, d_v_out, c->st);
  return c->hip_check("cube_symmetry");
}

pm_status pm_closure_adam(pm_ctx* c, float* d_params, float* d_m, float* d_v, const float* d_grad, int step,
                          double lr) {
  pm_status s = closure_ready(c, false);
  if (s != PM_OK) return s;
  if (!d_params || !d_m || !d_v || !d_grad || step < 1 || !(lr > 0)) return PM_EINVAL;
  closure_adam(d_params, d_m, d_v, d_grad, PM_CLOSURE_NPARAM, lr, step, c->st);
  closure_pack(d_params, c->at<uint16_t>(c->L.cl_wf), c->at<uint16_t>(c->L.cl_wb), c->at<float>(c->L.cl_bias), c->st);
  c->cl_params = true;
  return c->hip_check("closure_adam");
}

const char* pm_status_string(pm_status s) {
  switch (s) {
    case PM_OK: return "ok";
    case PM_EINVAL: return "invalid argument";
    case PM_EWORKSPACE: return "workspace missing, too small or misaligned";
    case PM_EHIP: return "HIP runtime error";
    case PM_ENAN: return "non-finite particle data";
    case PM_ESTATE: return "call out of order";
    case PM_ERANGE: return "size out of supported range";
    case PM_EUNSUPPORTED: return "unsupported option";
    default: return "unknown status";
  }
}

const char* pm_last_error(pm_ctx* c) {
  if (!c) return "null context";
  return c->last_error.c_str();
}

}  // extern "C"
