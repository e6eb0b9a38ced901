"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on identical seeded inputs.

Tolerances: FP64 path 1e-10 relative L2 per field and 1e-9 mesh spacings on
positions; FP32 path 1e-5 relative L2 per field and 1e-4 mesh spacings on
positions after 10 steps.
"""
import math
import sys

import numpy as np
import pytest

from oracle import pm as opm
from synth import config_particles, lattice_positions
from tests.helpers import FIELD_LINF, gpu_fields, oracle_fields, periodic_max_dx, rel_l2, rel_linf

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ctx(n, n_p, box, physics, precision, timings=False, b_route="elliptic"):
    from paper_2607_17929_amd import PMContext
    return PMContext(n, n_p, box, physics=physics, precision=precision, timings=timings, b_route=b_route)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


FIELD_TOL = {"fp64": 1e-10, "fp32": 1e-5}
POS_TOL = {"fp64": 1e-9, "fp32": 1e-4}


# ---------------------------------------------------------------------------
# FFT
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [16, 32, 64, 128])
def test_fft_against_oracle(n, precision):
    _say(f"fft n={n} {precision}")
    ctx = _ctx(n, 8, 100.0, "full", precision)
    r = np.random.default_rng(n)
    f = r.standard_normal((n, n, n))
    dt = torch.float64 if precision == "fp64" else torch.float32
    fk = ctx.debug_fft(torch.tensor(f, dtype=dt, device="cuda"), 1).cpu().numpy()
    ref = opm.fft3(f.astype(np.float32 if precision == "fp32" else np.float64).astype(np.float64))
    tol = 1e-13 if precision == "fp64" else 3e-7
    assert rel_l2(fk.real, ref.real) < tol * math.log2(n) and rel_l2(fk.imag, ref.imag) < tol * math.log2(n)
    # inverse of the oracle spectrum
    back = ctx.debug_fft(torch.tensor(ref, device="cuda"), -1).cpu().numpy()
    assert rel_l2(back, f) < tol * math.log2(n)


# ---------------------------------------------------------------------------
# deposit
# ---------------------------------------------------------------------------

def _random_particles(n_p, seed, umax):
    r = np.random.default_rng(seed)
    return r.random((n_p, 3)), (r.random((n_p, 3)) - 0.5) * 2 * umax


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["zeldovich_32", "random_ragged", "clustered", "single"])
def test_deposit_parity(case, precision):
    _say(f"deposit {case} {precision}")
    box = 320.0
    if case == "zeldovich_32":
        pos, u, tau0, _ = config_particles("zeldovich_32_scalar_fp64")
        n = 32
    elif case == "random_ragged":
        n = 32
        pos, u = _random_particles(7919, 5, 0.01)
        tau0 = 40.0
    elif case == "clustered":
        # most particles in a handful of cells, some exactly on cell faces
        n = 64
        r = np.random.default_rng(6)
        centers = r.random((5, 3))
        pos = (centers[r.integers(0, 5, 20000)] + 0.3 / n * r.standard_normal((20000, 3))) % 1.0
        pos[:50, 0] = np.floor(pos[:50, 0] * n) / n
        u = 0.02 * r.standard_normal((20000, 3))
        tau0 = 40.0
    else:
        n = 16
        pos = np.array([[0.999999, 0.0, 0.5]])
        u = np.array([[0.01, -0.02, 0.03]])
        tau0 = 40.0
    ctx = _ctx(n, pos.shape[0], box, "full", precision)
    ctx.init_particles(pos, u.astype(ctx.np_dtype), tau0)
    ctx.deposit()
    a = opm.Background(box).a(tau0)
    u_eff = u.astype(ctx.np_dtype).astype(np.float64)
    ref = opm.deposit(pos, u_eff, a, n)
    names = ["n00", "n0x", "n0y", "n0z", "nxx", "nxy", "nxz", "nyy", "nyz", "nzz"]
    tol = 1e-13 if precision == "fp64" else 2e-6
    for c, name in enumerate(names):
        g = ctx.get_field(name)
        assert rel_l2(g, ref[c]) < tol, (name, rel_l2(g, ref[c]))


# ---------------------------------------------------------------------------
# whole steps
# ---------------------------------------------------------------------------

def _run_both(n, box, physics, precision, pos, u, tau0, dtaus, check_every=False, b_route="elliptic"):
    ctx = _ctx(n, pos.shape[0], box, physics, precision, b_route=b_route)
    u_in = u.astype(ctx.np_dtype)
    ctx.init_particles(pos, u_in, tau0)
    sim = opm.OracleSim(n=n, box_mpch=box, physics=physics, pos=pos, u=u_in.astype(np.float64), tau=tau0,
                        b_route=b_route)
    worst, worst_max = {}, {}
    for i, dt in enumerate(dtaus):
        ctx.step(dt)
        sim.step(dt)
        if check_every or i == len(dtaus) - 1:
            gf = gpu_fields(ctx, physics)
            of = oracle_fields(sim, physics)
            for k in gf:
                worst[k] = max(worst.get(k, 0.0), rel_l2(gf[k], of[k]))
                worst_max[k] = max(worst_max.get(k, 0.0), rel_linf(gf[k], of[k]))
    _say("  rel-max", {k: f"{v:.1e}" for k, v in worst_max.items()})
    for k, v in worst_max.items():
        assert v < FIELD_LINF[precision], (k, "rel-max", v)
    gp, gu = ctx.get_particles()
    op, ou = sim.particles_by_id()
    return worst, periodic_max_dx(gp, op, n), rel_l2(gu, ou), ctx, sim


def test_zeldovich_32_fp64_scalar_ten_steps():
    """32^3 particles and mesh, FP64, scalar physics, 10 steps a = 0.02 -> 0.05."""
    _say("zeldovich 32^3 fp64 scalar 10 steps")
    pos, u, tau0, dtau = config_particles("zeldovich_32_scalar_fp64")
    worst, dxmax, urel, ctx, sim = _run_both(32, 320.0, "scalar", "fp64", pos, u, tau0, [dtau] * 10, check_every=True)
    _say(worst, dxmax, urel)
    for k, v in worst.items():
        assert v < FIELD_TOL["fp64"], (k, v)
    assert dxmax < POS_TOL["fp64"]
    assert urel < 1e-10
    tau, a, steps = ctx.time()
    assert steps == 10 and abs(a - 0.05) < 1e-12


@pytest.mark.parametrize("physics", ["newtonian", "full"])
def test_fp64_step_parity_physics(physics):
    _say(f"fp64 {physics}")
    pos, u, tau0, dtau = config_particles("zeldovich_32_scalar_fp64")
    worst, dxmax, urel, *_ = _run_both(32, 320.0, physics, "fp64", pos, u, tau0, [dtau] * 4, check_every=True)
    _say(worst, dxmax, urel)
    for k, v in worst.items():
        assert v < FIELD_TOL["fp64"], (k, v)
    assert dxmax < POS_TOL["fp64"]


@pytest.mark.parametrize("physics", ["scalar", "full"])
def test_fp32_ten_steps(physics):
    """FP32 fields/momenta, FP64 positions: 10 steps on the 32^3 workload's initial conditions (box 320 Mpc/h,
    k^-2 spectrum, Zel'dovich start at a = 0.02)."""
    _say(f"fp32 {physics} 10 steps")
    pos, u, tau0, dtau = config_particles("zeldovich_32_scalar_fp64")
    worst, dxmax, urel, *_ = _run_both(32, 320.0, physics, "fp32", pos, u, tau0, [dtau] * 10)
    _say(worst, dxmax, urel)
    for k, v in worst.items():
        assert v < FIELD_TOL["fp32"], (k, v)
    assert dxmax < POS_TOL["fp32"]


def test_fp32_full_ktk_spectrum_64():
    """The 256^3 full-physics workload's k T(k) spectrum and physics at a reduced 64^3 size, started at
    a = 0.1 (several tiles, all passes)."""
    _say("fp32 k T(k) spectrum 64^3")
    pos, u, tau0, dtau = config_particles("ktk_256_full", n=64)
    box = 1024.0 * 64 / 256
    worst, dxmax, urel, *_ = _run_both(64, box, "full", "fp32", pos, u, tau0, [dtau] * 10)
    _say(worst, dxmax, urel)
    for k, v in worst.items():
        assert v < FIELD_TOL["fp32"], (k, v)
    assert dxmax < POS_TOL["fp32"]


def test_ragged_particle_count_and_mesh():
    """Particle count unrelated to the mesh (7919 on 32^3), FP64 full physics, explicit stage calls."""
    _say("ragged")
    pos, u = _random_particles(7919, 17, 0.003)
    tau0, box, n = 40.0, 320.0, 32
    ctx = _ctx(n, pos.shape[0], box, "full", "fp64")
    ctx.init_particles(pos, u, tau0)
    sim = opm.OracleSim(n=n, box_mpch=box, physics="full", pos=pos, u=u, tau=tau0)
    for dtau_prev, dtau in [(0.0, 0.3), (0.3, 0.25), (0.25, 0.25)]:
        ctx.deposit(); ctx.solve_metric(dtau_prev); ctx.update_particles(dtau)
        sim.deposit(); sim.solve(dtau_prev); sim.update(dtau)
    gf, of = gpu_fields(ctx, "full"), oracle_fields(sim, "full")
    for k in gf:
        assert rel_l2(gf[k], of[k]) < FIELD_TOL["fp64"], (k, rel_l2(gf[k], of[k]))
    gp, _ = ctx.get_particles()
    op, _ = sim.particles_by_id()
    assert periodic_max_dx(gp, op, n) < POS_TOL["fp64"]


def test_call_order_is_enforced():
    from paper_2607_17929_amd import PMError
    ctx = _ctx(16, 64, 100.0, "scalar", "fp32")
    with pytest.raises(PMError):
        ctx.deposit()
    ctx.init_particles(lattice_positions(4), np.zeros((64, 3), np.float32), 10.0)
    with pytest.raises(PMError):
        ctx.solve_metric(0.0)
    with pytest.raises(PMError):
        ctx.update_particles(0.1)
    ctx.deposit()
    ctx.solve_metric(0.0)
    ctx.update_particles(0.1)


def test_nan_particles_are_reported():
    from paper_2607_17929_amd import PMError
    ctx = _ctx(16, 64, 100.0, "scalar", "fp32")
    pos = lattice_positions(4)
    pos[3, 1] = np.nan
    ctx.init_particles(pos, np.zeros((64, 3), np.float32), 10.0)
    with pytest.raises(PMError):
        ctx.sync()


def test_ingest_wraps_positions_and_checks_identifiers():
    """Positions outside [0, 1) are wrapped exactly as x - floor(x) with 1.0 mapped to 0.0 (bit for
    bit against the oracle's wrap), and an identifier out of range is reported by the next
    synchronising call until particles are loaded again."""
    from paper_2607_17929_amd import PMError
    _say("ingest: wrap and identifier checks")
    r = np.random.default_rng(31)
    n_p = 1000
    pos = r.uniform(-2.0, 3.0, (n_p, 3))
    pos[:8, 0] = [1.0, -1.0, 0.0, -0.0, 2.0, -1e-17, 1.0 - 2.0 ** -53, 3.0 - 2.0 ** -51]
    u = r.standard_normal((n_p, 3)) * 1e-3
    ctx = _ctx(16, n_p, 100.0, "scalar", "fp64")
    ctx.init_particles(pos, u, 10.0)
    gp, gu = ctx.get_particles()
    want = opm.wrap_positions(pos.copy())
    assert np.all((gp >= 0.0) & (gp < 1.0))
    assert np.array_equal(gp.view(np.uint64), want.view(np.uint64))
    assert np.array_equal(gu, u)
    ids = np.arange(n_p, dtype=np.uint32)
    ids[17] = n_p
    ctx.init_particles(pos, u, 10.0, ids=ids)
    with pytest.raises(PMError) as e:
        ctx.sync()
    assert e.value.status == -1
    ctx.init_particles(pos, u, 10.0)
    ctx.sync()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_parabolic_b_route(precision):
    """Full physics with B integrated from the vector part of the space-space equation (12 FFTs per step)."""
    _say(f"{precision} full, parabolic B")
    pos, u, tau0, dtau = config_particles("zeldovich_32_scalar_fp64")
    steps = 4 if precision == "fp64" else 10
    worst, dxmax, urel, *_ = _run_both(32, 320.0, "full", precision, pos, u, tau0, [dtau] * steps,
                                       check_every=precision == "fp64", b_route="parabolic")
    _say(worst, dxmax, urel)
    for k, v in worst.items():
        assert v < FIELD_TOL[precision], (k, v)
    assert dxmax < POS_TOL[precision]


def test_full_parabolic_b_route_ktk_spectrum_64():
    """The parabolic route on the k T(k) spectrum of the 256^3 full-physics workload at 64^3 (several
    tiles), FP32, 10 steps."""
    _say("fp32 k T(k) spectrum 64^3 parabolic B")
    pos, u, tau0, dtau = config_particles("ktk_256_full", n=64)
    box = 1024.0 * 64 / 256
    worst, dxmax, urel, *_ = _run_both(64, box, "full", "fp32", pos, u, tau0, [dtau] * 10, b_route="parabolic")
    _say(worst, dxmax, urel)
    for k, v in worst.items():
        assert v < FIELD_TOL["fp32"], (k, v)
    assert dxmax < POS_TOL["fp32"]


@pytest.mark.parametrize("b_route", ["elliptic", "parabolic"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["one_particle", "one_cell"])
def test_degenerate_inputs_full_steps(case, precision, b_route):
    """Whole full-physics steps on a 16^3 mesh for one particle, and for 1000 particles that all start
    in one cell (one crowded row, every rank in one counter), against the oracle, both precisions at
    their bars with either B route.  In the one-cell case the transverse momentum source of the
    elliptic route is dominated by -phidot d_i psi, and phidot is the change of phi between two solves,
    about 2 % of phi (kappa = |phi| / |phi - phi_prev| is about 50): the FP32 path meets the bar because
    it solves for that change itself and sums the energy and momentum deposits in FP64."""
    _say(f"degenerate {case} {precision} {b_route}")
    r = np.random.default_rng(41)
    n, box = 16, 160.0
    if case == "one_particle":
        pos = np.array([[0.3, 0.71, 0.999]])
        u = np.array([[1e-3, -2e-3, 5e-4]])
    else:
        pos = (np.array([5.0, 9.0, 2.0]) + r.random((1000, 3))) / n
        u = r.normal(0.0, 1e-3, (1000, 3))
    tau0 = opm.Background(box).tau(0.05)
    worst, dxmax, urel, _, sim = _run_both(n, box, "full", precision, pos, u, tau0, [0.02 * tau0] * 3,
                                           check_every=True, b_route=b_route)
    kappa = np.linalg.norm(sim.phi) / np.linalg.norm(sim.phi - sim.phi_prev)
    _say(worst, dxmax, urel, f"kappa {kappa:.1f}")
    for k, v in worst.items():
        assert v < FIELD_TOL[precision], (k, v)
    assert dxmax < POS_TOL[precision]
    assert urel < (1e-10 if precision == "fp64" else FIELD_TOL["fp32"])
