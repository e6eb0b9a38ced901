"""Element-by-element parity at the full size of the 256^3 full-physics workload: 256^3 particles on a
256^3 mesh, box 1024 Mpc/h, the k T(k) spectrum (seed 2), Zel'dovich start at a = 0.1, dtau = 0.01 tau;
the quasi-static start step and one semi-implicit step (time derivatives, lagged fields, the first
Crank-Nicolson step of h), against the FP64 oracle on the same inputs.

Bars: the FP32 path 1e-5 relative L2 per field (phi, chi, B, the six h_ij) and 1e-4 mesh spacings on
positions; the FP64 path 1e-10 and 1e-9.  The oracle takes about a minute per run here.
"""
import numpy as np
import pytest

from oracle import pm as opm
from synth import config_particles
from tests.helpers import gpu_fields, oracle_fields, periodic_max_dx, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {"fp32": (1e-5, 1e-4), "fp64": (1e-10, 1e-9)}


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_ktk_256_full_two_steps_against_oracle(precision):
    from paper_2607_17929_amd import PMContext
    pos, u, tau0, dtau = config_particles("ktk_256_full")
    n, box = 256, 1024.0
    ctx = PMContext(n, pos.shape[0], box, physics="full", precision=precision)
    u_in = u.astype(ctx.np_dtype)
    ctx.init_particles(pos, u_in, tau0)
    sim = opm.OracleSim(n=n, box_mpch=box, physics="full", pos=pos, u=u_in.astype(np.float64), tau=tau0)
    del u
    for i in range(2):
        _say(f"256^3 full physics {precision}: step {i + 1}")
        ctx.step(dtau)
        sim.step(dtau)
    gf, of = gpu_fields(ctx, "full"), oracle_fields(sim, "full")
    ftol, ptol = TOL[precision]
    errs = {k: rel_l2(gf[k], of[k]) for k in gf}
    _say("  " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v < ftol, (k, v)
    gp, gu = ctx.get_particles()
    op, ou = sim.particles_by_id()
    dx = periodic_max_dx(gp, op, n)
    _say(f"  max |dx| {dx:.2e} cells, u rel-L2 {rel_l2(gu, ou):.2e}")
    assert dx < ptol
    assert rel_l2(gu, ou) < ftol
    assert ctx.time()[2] == 2
