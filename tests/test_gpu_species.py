"""A second particle species through the C ABI (pm_init_particles_2 / pm_get_particles_2).

* Parity with the oracle: the 32^3 workload's Zel'dovich set (box 320 Mpc/h) as species 1 plus a hot species (|u| = 2a in random
  directions, speeds near 0.9 c, a ragged count of 5003 particles) carrying 10 % of the rest mass:
  FP64 full and scalar physics 4 steps at the FP64 bar; FP32 full physics with parabolic B 10 steps
  at the FP32 bar; fields and both species' positions.
* Splitting one species into two halves with half of the mass each reproduces the one-species GPU
  run (the deposit's order of summation differs, so to rounding).
* Call order and argument checks; a checkpoint carries the second species.
"""
import numpy as np
import pytest

from oracle import pm as opm
from synth import config_particles
from tests.helpers import gpu_fields, oracle_fields, periodic_max_dx, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FIELD_TOL = {"fp64": 1e-10, "fp32": 1e-5}
POS_TOL = {"fp64": 1e-9, "fp32": 1e-4}


def _say(msg):
    print(msg, flush=True)


def _ctx(n, n_p, box, physics, precision, n2=0, f2=0.0, b_route="elliptic"):
    from paper_2607_17929_amd import PMContext
    return PMContext(n, n_p, box, physics=physics, precision=precision, b_route=b_route, n_particles_2=n2,
                     mass_fraction_2=f2)


def _hot_species(n2, a, seed=29):
    r = np.random.default_rng(seed)
    d = r.normal(size=(n2, 3))
    return r.random((n2, 3)), 2.0 * a * d / np.linalg.norm(d, axis=1)[:, None]


@pytest.mark.parametrize("precision,physics,steps,b_route", [("fp64", "full", 4, "elliptic"),
                                                             ("fp64", "scalar", 4, "elliptic"),
                                                             ("fp32", "full", 10, "parabolic")])
def test_hot_second_species_matches_oracle(precision, physics, steps, b_route):
    _say(f"two species {precision} {physics} {b_route}")
    pos, u, tau0, dtau = config_particles("zeldovich_32_scalar_fp64")
    n, box, f2, n2 = 32, 320.0, 0.1, 5003
    bg = opm.Background(box)
    pos2, u2 = _hot_species(n2, bg.a(tau0 - 0.5 * dtau))
    ctx = _ctx(n, pos.shape[0], box, physics, precision, n2, f2, b_route)
    dt = ctx.np_dtype
    ctx.init_particles(pos, u.astype(dt), tau0)
    ctx.init_particles_2(pos2, u2.astype(dt))
    sim = opm.OracleSim(n=n, box_mpch=box, physics=physics, pos=pos, u=u.astype(dt).astype(np.float64), tau=tau0,
                        b_route=b_route, pos2=pos2, u2=u2.astype(dt).astype(np.float64), mass_fraction2=f2)
    worst = {}
    for i in range(steps):
        ctx.step(dtau)
        sim.step(dtau)
        if precision == "fp64" or i == steps - 1:
            gf, of = gpu_fields(ctx, physics), oracle_fields(sim, physics)
            for k in gf:
                worst[k] = max(worst.get(k, 0.0), rel_l2(gf[k], of[k]))
    _say(f"  fields {worst}")
    for k, v in worst.items():
        assert v < FIELD_TOL[precision], (k, v)
    gp, _ = ctx.get_particles()
    op, _ = sim.particles_by_id()
    assert periodic_max_dx(gp, op, n) < POS_TOL[precision]
    gp2, gu2 = ctx.get_particles_2()
    op2, ou2 = sim.species2()
    dx2 = periodic_max_dx(gp2, op2, n)
    _say(f"  species 2: max |dx| {dx2:.2e} cells, |u| rel {rel_l2(gu2, ou2):.2e}")
    assert dx2 < POS_TOL[precision]
    assert rel_l2(gu2, ou2) < FIELD_TOL[precision]
    # the hot species moves several cells per step
    assert np.max(np.abs(((gp2 - pos2) + 0.5) % 1.0 - 0.5)) * n > 3


def test_split_species_reproduces_one_species():
    _say("two species: split invariance")
    pos, u, tau0, dtau = config_particles("zeldovich_32_scalar_fp64")
    n, box = 32, 320.0
    one = _ctx(n, pos.shape[0], box, "full", "fp64")
    one.init_particles(pos, u, tau0)
    h = pos.shape[0] // 2
    two = _ctx(n, h, box, "full", "fp64", pos.shape[0] - h, 0.5)
    two.init_particles(pos[:h], u[:h], tau0)
    two.init_particles_2(pos[h:], u[h:])
    for _ in range(4):
        one.step(dtau)
        two.step(dtau)
    f1, f2 = gpu_fields(one, "full"), gpu_fields(two, "full")
    for k in f1:
        assert rel_l2(f2[k], f1[k]) < 1e-12, (k, rel_l2(f2[k], f1[k]))
    p1, _ = one.get_particles()
    pa, _ = two.get_particles()
    pb, _ = two.get_particles_2()
    assert periodic_max_dx(np.concatenate([pa, pb]), p1, n) < 1e-11


def test_second_species_call_order_and_arguments():
    from paper_2607_17929_amd import PMError
    _say("two species: argument checks")
    pos, u, tau0, dtau = config_particles("zeldovich_32_scalar_fp64")
    ctx = _ctx(32, pos.shape[0], 320.0, "scalar", "fp64", 100, 0.05)
    p2, u2 = _hot_species(100, 0.02)
    with pytest.raises(PMError) as e:
        ctx.init_particles_2(p2, u2)  # before the first species
    assert e.value.status == -5
    ctx.init_particles(pos, u, tau0)
    with pytest.raises(PMError) as e:
        ctx.deposit()  # second species not loaded
    assert e.value.status == -5
    with pytest.raises(PMError):
        ctx.init_particles_2(p2[:50], u2[:50])  # wrong count
    ctx.init_particles_2(p2, u2)
    ctx.step(dtau)
    single = _ctx(32, pos.shape[0], 320.0, "scalar", "fp64")
    single.init_particles(pos, u, tau0)
    with pytest.raises(PMError) as e:
        single.init_particles_2(p2, u2)  # no second species configured
    assert e.value.status == -1
    with pytest.raises(PMError):
        _ctx(32, pos.shape[0], 320.0, "scalar", "fp64", 100, 0.0)  # a second species needs 0 < f < 1
    with pytest.raises(PMError):
        _ctx(32, pos.shape[0], 320.0, "scalar", "fp64", 0, 0.1)  # a fraction without a species


def test_checkpoint_carries_the_second_species():
    _say("two species: checkpoint")
    pos, u, tau0, dtau = config_particles("zeldovich_32_scalar_fp64")
    p2, u2 = _hot_species(777, 0.02)
    a = _ctx(32, pos.shape[0], 320.0, "scalar", "fp64", 777, 0.1)
    a.init_particles(pos, u, tau0)
    a.init_particles_2(p2, u2)
    for _ in range(2):
        a.step(dtau)
    blob = a.get_state()
    for _ in range(3):
        a.step(dtau)
    b = _ctx(32, pos.shape[0], 320.0, "scalar", "fp64", 777, 0.1)
    b.set_state(blob)
    for _ in range(3):
        b.step(dtau)
    fa, fb = gpu_fields(a, "scalar"), gpu_fields(b, "scalar")
    for k in fa:
        assert rel_l2(fb[k], fa[k]) < 1e-11, k
    qa, _ = a.get_particles_2()
    qb, _ = b.get_particles_2()
    assert periodic_max_dx(qa, qb, 32) < 1e-10
