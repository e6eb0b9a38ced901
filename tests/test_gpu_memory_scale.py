"""Memory-scale run: 1024^3 particles on a 1024^3 mesh, box 4096 Mpc/h, the benchmark's spectrum, Zel'dovich
start at a = 0.1, FP32 fields with FP64 positions, full physics (about 234 GB of the 288 GB of HBM).

The oracle cannot run the whole step at this size (its FP64 state alone exceeds the host), and the FP64
GPU path needs about 395 GB, so the checks are on outputs the oracle gives one by one and on invariants:
* FFT: 12 sampled Fourier coefficients of a seeded 1024^3 field against the DFT sum written out (the
  1024-point transforms of every pass);
* deposit: every vertex of two 16^3 regions (the densest cell's and a random one) against the oracle's
  CIC sums of the particles around them; CIC partition of unity (sum of n00 = sum of the particle
  energies, sum of n0i = sum of the momenta);
* gather + kick + drift: for 8192 sampled particles, the oracle's update on the GPU's own 1024^3 fields
  after the start-up solve (gradients evaluated at the vertices the particles need), against the GPU's;
* finite fields and positions after three steps.  The per-stage times of the last step are printed.

The checks of the run share one context (a module fixture, in file order; each also runs alone), so
that none of them takes more than about two minutes.
"""
import gc

import numpy as np
import pytest

from oracle import pm as opm
from synth import spectrum_power_law_m2, zeldovich_particles
from synth.ics import eds_a_of_tau
from tests.helpers import periodic_max_dx, rel_l2
from tests.test_gpu_fullsize import DEP, _region_deposit

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N = 1024
BOX = 4096.0


def _say(msg):
    print(msg, flush=True)


def _release():
    gc.collect()
    torch.cuda.empty_cache()


def test_fft_1024_sampled_modes():
    from paper_2607_17929_amd import PMContext
    _release()
    _say("fft 1024 fp32, sampled modes")
    r = np.random.default_rng(8)
    f = r.standard_normal((N, N, N), dtype=np.float32)
    ctx = PMContext(N, 1, BOX, physics="newtonian", precision="fp32")
    spec = ctx.debug_fft(torch.from_numpy(f).cuda(), 1).cpu().numpy()
    del ctx
    _release()
    modes = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (3, 17, 1023), (512, 0, 0), (512, 512, 512),
             (100, 1023, 3), (17, 600, 900), (511, 1, 1022), (256, 768, 128), (5, 5, 5)]
    x = np.arange(N)
    ex = np.exp(-2j * np.pi * np.outer(x, [m[0] for m in modes]) / N)
    f2 = f.reshape(-1, N).astype(np.float64)
    gx = (f2 @ ex.real + 1j * (f2 @ ex.imag)).reshape(N, N, len(modes))
    scale = np.sqrt(np.sum(f2 * f2))
    del f2
    for j, (kx, ky, kz) in enumerate(modes):
        ref = np.exp(-2j * np.pi * kz * x / N) @ (gx[:, :, j] @ np.exp(-2j * np.pi * ky * x / N))
        err = abs(spec[kz, ky, kx].astype(np.complex128) - ref) / scale
        assert err < 1e-5, ((kx, ky, kz), err)


class _Run:
    """The 1024^3 run shared by the tests below (the workspace takes 256 GB of the device)."""

    def __init__(self):
        self.ctx = None
        self.stage = "none"
        self.bg = opm.Background(BOX)
        self.tau = self.bg.tau(0.1)
        self.dtau = 0.01 * self.tau

    def ensure(self):
        if self.ctx is not None:
            return
        from paper_2607_17929_amd import PMContext
        # release what earlier tests left in the caching allocator
        _release()
        props = torch.cuda.get_device_properties(0)
        _say(f"device memory {props.total_memory / 1e9:.0f} GB")
        _say("building the 1024^3 input")
        self.pos, u = zeldovich_particles(N, 4, spectrum_power_law_m2, BOX, 0.2, 0.02, 0.1,
                                          eds_a_of_tau(self.tau - 0.5 * self.dtau, BOX))
        self.u32 = u.astype(np.float32)
        del u
        self.ctx = PMContext(N, N ** 3, BOX, physics="full", precision="fp32", timings=True)
        _say(f"workspace {self.ctx.ws_bytes / 1e9:.1f} GB")
        self.ctx.init_particles(self.pos, self.u32, self.tau)
        self.stage = "init"


@pytest.fixture(scope="module")
def run1024():
    r = _Run()
    yield r
    del r
    gc.collect()
    _release()


def test_memory_scale_1024_input(run1024):
    """The full-size input: 1024^3 particles in [0, 1), rms distance from their lattice sites 1.0 cell (0.2
    cells at a = 0.02 grown to a = 0.1), finite momenta; the library takes them (init_particles)."""
    r = run1024
    r.ensure()
    assert r.pos.shape == (N ** 3, 3) and float(r.pos.min()) >= 0.0 and float(r.pos.max()) < 1.0
    assert bool(np.isfinite(r.u32).all())
    q = ((np.arange(N) + 0.5) / N)
    sample = np.random.default_rng(5).choice(N ** 3, 1 << 20, replace=False)
    lat = np.stack([q[sample % N], q[(sample // N) % N], q[sample // (N * N)]], axis=1)
    d = (r.pos[sample] - lat + 0.5) % 1.0 - 0.5
    rms = float(np.sqrt(np.mean(np.sum(d * d, axis=1)))) * N
    _say(f"rms displacement {rms:.3f} cells")
    assert abs(rms - 1.0) < 0.02


def _region_particles(pos, z0, y0, x0, R):
    """The particles whose cell touches the vertices [z0, z0 + R) x ... (cells z0 - 1 .. z0 + R - 1 per axis)."""
    sel = np.ones(pos.shape[0], dtype=bool)
    for ax, o in ((2, z0), (1, y0), (0, x0)):
        c = np.floor(pos[:, ax] * N).astype(np.int64)
        sel &= (c - (o - 1)) % N < R + 1
    return np.nonzero(sel)[0]


def test_memory_scale_1024_deposit(run1024):
    """CIC partition of unity over the whole mesh and every vertex of two 16^3 regions (the densest
    cell's and a random one) against the oracle's CIC sums of the particles around them."""
    r = run1024
    r.ensure()
    ctx = r.ctx
    ctx.deposit()
    a = r.bg.a(r.tau)
    e_sum = float(np.sum(np.sqrt(a * a + np.sum(r.u32.astype(np.float64) ** 2, axis=1))))
    u_sum = r.u32.astype(np.float64).sum(axis=0)
    n00 = ctx.get_field("n00", device=True)
    tot = float(torch.sum(n00, dtype=torch.float64))
    del n00
    _say(f"sum n00 {tot:.9e} vs sum e {e_sum:.9e}")
    assert abs(tot - e_sum) < 1e-6 * e_sum
    for i, c in enumerate(("n0x", "n0y", "n0z")):
        f = ctx.get_field(c, device=True)
        s = float(torch.sum(f, dtype=torch.float64))
        del f
        assert abs(s - u_sum[i]) < 1e-5 * (abs(u_sum[i]) + 1e-6 * e_sum), (c, s, u_sum[i])
    # the densest cell: one pass over the particles' cell keys
    key = np.floor(r.pos[:, 0] * N).astype(np.int64)
    key += N * np.floor(r.pos[:, 1] * N).astype(np.int64)
    key += N * N * np.floor(r.pos[:, 2] * N).astype(np.int64)
    dense = int(np.argmax(np.bincount(key, minlength=N ** 3)))
    del key
    dz, dy, dx = dense // (N * N), (dense // N) % N, dense % N
    R = 16
    rg = np.random.default_rng(12)
    regions = [((dz - R // 2) % N, (dy - R // 2) % N, (dx - R // 2) % N), tuple(int(v) for v in rg.integers(0, N, 3))]
    for (z0, y0, x0) in regions:
        idx = _region_particles(r.pos, z0, y0, x0, R)
        ref = _region_deposit(r.pos[idx], r.u32[idx].astype(np.float64), a, z0, y0, x0, R, n=N)
        zi, yi, xi = (np.arange(z0, z0 + R) % N, np.arange(y0, y0 + R) % N, np.arange(x0, x0 + R) % N)
        for c, name in enumerate(DEP):
            f = ctx.get_field(name, device=True)
            got = f[torch.tensor(zi)][:, torch.tensor(yi)][:, :, torch.tensor(xi)].cpu().numpy().astype(np.float64)
            del f
            err = rel_l2(got, ref[c])
            assert err < 2e-6, ((z0, y0, x0), name, err)
        _say(f"  deposit region {(z0, y0, x0)} ({idx.size} particles) matches")
    r.stage = "deposited"


def test_memory_scale_1024_update(run1024):
    """The start-up solve, then the update of 8192 sampled particles against the oracle's on the same fields."""
    r = run1024
    r.ensure()
    ctx = r.ctx
    if r.stage != "deposited":
        ctx.deposit()
    r.pos = r.u32 = None
    gc.collect()
    ctx.solve_metric(0.0)
    fields = {k: ctx.get_field(k) for k in ("phi", "chi", "bx", "by", "bz")}
    p0, u0 = ctx.get_particles()
    sample = np.random.default_rng(78).choice(N ** 3, 8192, replace=False)
    p0, u0 = p0[sample].copy(), u0[sample].astype(np.float64)
    gc.collect()
    ctx.update_particles(r.dtau)
    p1, u1 = ctx.get_particles()
    p1, u1 = p1[sample].copy(), u1[sample].astype(np.float64)
    gc.collect()
    # the oracle's kick and drift (the equations of its update) on gathered values whose centred
    # differences are evaluated at the vertices the sampled particles need
    g = opm.gathered_pointwise(fields["phi"], fields["chi"], [fields["bx"], fields["by"], fields["bz"]], p0, N)
    del fields
    gc.collect()
    p_ref, u_ref = opm.kick_drift(g, p0, u0, r.bg.a(r.tau), r.bg.a(r.tau + 0.5 * r.dtau), r.dtau, opm.FULL)
    dxm = periodic_max_dx(p1, p_ref, N)
    du = rel_l2(u1, u_ref)
    _say(f"  sampled update: max |dx| {dxm:.2e} cells, u rel-L2 {du:.2e}, largest move "
         f"{periodic_max_dx(p1, p0, N):.2f} cells")
    assert dxm < 1e-4 and du < 1e-5
    r.stage = "updated"


def test_memory_scale_1024_steps(run1024):
    """Three more steps (the last one timed per stage); fields and positions stay finite."""
    r = run1024
    r.ensure()
    ctx = r.ctx
    for _ in range(2):
        ctx.step(r.dtau)
    ctx.sync()
    ctx.timings()  # time the next step alone
    ctx.step(r.dtau)
    ctx.sync()
    st = ctx.timings()
    per = {k: v[0] / v[1] for k, v in st.items() if v[1]}
    total = sum(v[0] for v in st.values())
    _say("stage ms per launch: " + ", ".join(f"{k} {v:.2f}" for k, v in per.items()) + f"; step {total:.1f} ms")
    for c in ("phi", "chi", "bx"):
        f = ctx.get_field(c, device=True)
        assert bool(torch.isfinite(f).all()), c
        del f
    p, _ = ctx.get_particles()
    assert bool(np.isfinite(p).all()) and float(p.min()) >= 0.0 and float(p.max()) < 1.0
