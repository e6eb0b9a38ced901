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


def test_memory_scale_1024():
    from paper_2607_17929_amd import PMContext
    # release what earlier tests left in the caching allocator: the workspace needs 234 GB
    _release()
    props = torch.cuda.get_device_properties(0)
    _say(f"device memory {props.total_memory / 1e9:.0f} GB")
    bg = opm.Background(BOX)
    tau = bg.tau(0.1)
    dtau = 0.01 * tau
    _say("building the 1024^3 input")
    pos, u = zeldovich_particles(N, 4, spectrum_power_law_m2, BOX, 0.2, 0.02, 0.1, eds_a_of_tau(tau - 0.5 * dtau, BOX))
    u32 = u.astype(np.float32)
    del u
    ctx = PMContext(N, N ** 3, BOX, physics="full", precision="fp32", timings=True)
    _say(f"workspace {ctx.ws_bytes / 1e9:.1f} GB")
    ctx.init_particles(pos, u32, tau)
    ctx.deposit()
    a = bg.a(tau)
    u64 = u32.astype(np.float64)
    e_sum = float(np.sum(np.sqrt(a * a + np.sum(u64 * u64, axis=1))))
    u_sum = u64.sum(axis=0)
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
    # two 16^3 regions of the deposit, vertex by vertex
    base, _ = opm.cic_cells(pos, N)
    key = (base[:, 2] * N + base[:, 1]) * N + base[:, 0]
    del base
    counts = np.bincount(key, minlength=N ** 3)
    del key
    dense = int(np.argmax(counts))
    del counts
    dz, dy, dx = dense // (N * N), (dense // N) % N, dense % N
    R = 16
    r = np.random.default_rng(12)
    regions = [((dz - R // 2) % N, (dy - R // 2) % N, (dx - R // 2) % N), tuple(int(v) for v in r.integers(0, N, 3))]
    for (z0, y0, x0) in regions:
        ref = _region_deposit(pos, u64, a, z0, y0, x0, R, n=N)
        zi, yi, xi = (np.arange(z0, z0 + R) % N, np.arange(y0, y0 + R) % N, np.arange(x0, x0 + R) % N)
        for c, name in enumerate(DEP):
            f = ctx.get_field(name, device=True)
            got = f[torch.tensor(zi)][:, torch.tensor(yi)][:, :, torch.tensor(xi)].cpu().numpy().astype(np.float64)
            del f
            err = rel_l2(got, ref[c])
            assert err < 2e-6, ((z0, y0, x0), name, err)
        _say(f"  deposit region {(z0, y0, x0)} matches")
    del pos, u64, u32
    gc.collect()
    # the start-up solve, then the update of 8192 sampled particles against the oracle's on the same fields
    ctx.solve_metric(0.0)
    fields = {k: ctx.get_field(k) for k in ("phi", "chi", "bx", "by", "bz")}
    p0, u0 = ctx.get_particles()
    sample = np.random.default_rng(78).choice(N ** 3, 8192, replace=False)
    p0, u0 = p0[sample].copy(), u0[sample].astype(np.float64)
    gc.collect()
    ctx.update_particles(dtau)
    p1, u1 = ctx.get_particles()
    p1, u1 = p1[sample].copy(), u1[sample].astype(np.float64)
    gc.collect()
    # the oracle's kick and drift (the equations of its update) on gathered values whose centred
    # differences are evaluated at the vertices the sampled particles need
    g = opm.gathered_pointwise(fields["phi"], fields["chi"], [fields["bx"], fields["by"], fields["bz"]], p0, N)
    del fields
    gc.collect()
    p_ref, u_ref = opm.kick_drift(g, p0, u0, bg.a(tau), bg.a(tau + 0.5 * dtau), dtau, opm.FULL)
    dxm = periodic_max_dx(p1, p_ref, N)
    du = rel_l2(u1, u_ref)
    _say(f"  sampled update: max |dx| {dxm:.2e} cells, u rel-L2 {du:.2e}, largest move "
         f"{periodic_max_dx(p1, p0, N):.2f} cells")
    assert dxm < 1e-4 and du < 1e-5
    for _ in range(2):
        ctx.step(dtau)
    ctx.sync()
    ctx.timings()  # time the next step alone
    ctx.step(dtau)
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
    del ctx, p
    _release()
