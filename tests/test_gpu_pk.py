"""The library's power-spectrum estimator (pm_power_spectrum) against the oracle's (oracle.pk) on the
same particles: shells, mode counts and k exactly (up to rounding), P to the precision's tolerance."""
import numpy as np
import pytest

from oracle import pk
from synth import config_particles

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _both(pos, m, box, precision, shot):
    from paper_2607_17929_amd import PMContext
    ctx = PMContext(m, pos.shape[0], box, physics="newtonian", precision=precision)
    ctx.init_particles(pos, np.zeros_like(pos, dtype=ctx.np_dtype), 1.0)
    return ctx.power_spectrum(subtract_shot_noise=shot), pk.power_spectrum(pos, m, box, subtract_shot_noise=shot)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["zeldovich_32", "poisson_64"])
def test_power_spectrum_matches_oracle(precision, case):
    print("pk", precision, case, flush=True)
    if case == "zeldovich_32":
        pos, _, _, _ = config_particles("zeldovich_32_scalar_fp64")
        m, box = 32, 320.0
    else:
        pos = np.random.default_rng(12).random((100003, 3))
        m, box = 64, 250.0
    for shot in (True, False):
        (k, p, c), (k0, p0, c0) = _both(pos, m, box, precision, shot)
        assert np.array_equal(c, c0)
        assert np.max(np.abs(k / k0 - 1)) < 1e-12
        tol = 1e-10 if precision == "fp64" else 1e-5
        assert np.max(np.abs(p - p0)) < tol * np.max(np.abs(p0)), np.max(np.abs(p - p0)) / np.max(np.abs(p0))
