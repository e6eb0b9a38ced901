"""Conservation diagnostics through the C ABI (pm_diagnostics).

* Newtonian PM with CIC assignment, CIC interpolation and centred differences exerts no net force
  (the Green's function is symmetric and the difference operator antisymmetric), so the total momentum
  of the particles is conserved to rounding over 10 FP64 steps (a scheme with a self-force would move
  it by dtau a sum|grad phi| per step).
* The energy sum of the last deposit equals the FP64 sum of sqrt(a^2 + u^2) over the particles at
  that time; a second species enters weighted by its mass ratio, in the momentum too.
"""
import numpy as np
import pytest

from oracle import pm as opm
from synth import config_particles

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ctx(n, n_p, box, physics, precision, n2=0, f2=0.0):
    from paper_2607_17929_amd import PMContext
    return PMContext(n, n_p, box, physics=physics, precision=precision, n_particles_2=n2, mass_fraction_2=f2)


def test_newtonian_total_momentum_is_conserved():
    pos, u, tau0, dtau = config_particles("zeldovich_32_scalar_fp64")
    ctx = _ctx(32, pos.shape[0], 320.0, "newtonian", "fp64")
    ctx.init_particles(pos, u, tau0)
    p0 = np.array(ctx.diagnostics()["momentum"])
    assert np.allclose(p0, u.sum(axis=0), rtol=0, atol=1e-13 * np.abs(u).sum())
    scale = 0.0
    for _ in range(10):
        ctx.step(dtau)
        _, uu = ctx.get_particles()
        scale = max(scale, float(np.abs(uu - u).sum()))  # accumulated momentum changes of the particles
    d = ctx.diagnostics()
    p1 = np.array(d["momentum"])
    assert scale > 0
    assert np.max(np.abs(p1 - p0)) < 1e-10 * scale, (p1 - p0, scale)
    assert d["energy_sum"] == 0.0 and d["phi_mean"] == 0.0  # no FP64 homogeneous mode in the Newtonian limit


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_energy_sum_and_two_species_momentum(precision):
    pos, u, tau0, dtau = config_particles("zeldovich_32_scalar_fp64")
    r = np.random.default_rng(5)
    p2, u2 = r.random((999, 3)), r.normal(0.0, 0.05, (999, 3))
    f2 = 0.1
    ctx = _ctx(32, pos.shape[0], 320.0, "full", precision, 999, f2)
    dt = ctx.np_dtype
    ctx.init_particles(pos, u.astype(dt), tau0)
    ctx.init_particles_2(p2, u2.astype(dt))
    ctx.step(dtau)
    ctx.deposit()
    a = opm.Background(320.0).a(ctx.time()[0])
    _, ua = ctx.get_particles()
    _, ub = ctx.get_particles_2()
    ua, ub = ua.astype(np.float64), ub.astype(np.float64)
    w = (f2 / 999) / ((1 - f2) / pos.shape[0])
    e = np.sqrt(a * a + (ua * ua).sum(axis=1)).sum() + w * np.sqrt(a * a + (ub * ub).sum(axis=1)).sum()
    d = ctx.diagnostics()
    assert abs(d["energy_sum"] - e) < 1e-12 * e
    mom = ua.sum(axis=0) + w * ub.sum(axis=0)
    assert np.allclose(d["momentum"], mom, rtol=0, atol=1e-12 * (np.abs(ua).sum() + w * np.abs(ub).sum()))
    assert d["phi_mean"] != 0.0


def test_copy_probe_copies_every_byte():
    """The bandwidth probe is a copy: random bytes of a size that is no power of two (16 x 1000003) arrive
    unchanged, and the reported time is positive."""
    import ctypes as C

    from paper_2607_17929_amd import _lib as L
    lib = L.load()
    nb = 16 * 1000003
    src = torch.randint(0, 256, (nb,), dtype=torch.uint8, generator=torch.Generator().manual_seed(5)).cuda()
    dst = torch.zeros_like(src)
    ms = C.c_double()
    st = torch.cuda.current_stream()
    assert lib.pm_copy_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nb, 3, C.c_void_p(st.cuda_stream),
                             C.byref(ms)) == L.PM_OK
    assert torch.equal(src, dst) and ms.value > 0
