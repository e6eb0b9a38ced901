"""Host pins of the oracle's training helpers: the cube symmetries used to augment closure training data
(they commute with the 1x force of the oracle and are 48 distinct maps) and the particle MSE and its
gradient (finite differences). CPU only."""
import itertools

import numpy as np
import pytest

from oracle import cnn
from oracle import pm as opm


def _flip(signs):
    return sum(1 << d for d in range(3) if signs[d] < 0)


@pytest.mark.parametrize("perm,signs", [((0, 1, 2), (1, 1, -1)), ((2, 0, 1), (1, -1, 1)), ((1, 0, 2), (-1, -1, 1))])
def test_cube_symmetry_commutes_with_the_1x_force(perm, signs):
    n = 16
    r = np.random.default_rng(4)
    pos = r.random((300, 3))
    u = 1e-3 * r.standard_normal((300, 3))
    tau = 40.0

    def force(p, v):
        sim = opm.OracleSim(n=n, box_mpch=320.0, physics="scalar", pos=p, u=v, tau=tau)
        sim.deposit()
        sim.solve(0.0)
        return opm.interpolate(opm.grad(sim.phi, n), opm.wrap_positions(p.copy()), n).T

    g = force(pos, u)
    tp, tu, tg = cnn.cube_symmetry(pos, u, g, perm, _flip(signs))
    g2 = force(tp, tu)
    assert np.max(np.abs(g2 - tg)) < 1e-10 * np.max(np.abs(g))


def test_cube_symmetries_are_48_distinct_maps():
    x = np.array([[0.1, 0.2, 0.4], [0.0, 0.5, 0.75]])
    seen = set()
    for perm in itertools.permutations(range(3)):
        for flip in range(8):
            p, _, _ = cnn.cube_symmetry(x, x, x, perm, flip)
            assert np.all((p >= 0.0) & (p < 1.0))
            seen.add(tuple(np.round(p[0], 12)))
    assert len(seen) == 48


def test_mse_gradient_by_finite_differences():
    r = np.random.default_rng(6)
    pred, target = r.standard_normal((50, 3)), r.standard_normal((50, 3))
    loss, tms, g = cnn.mse_loss(pred, target)
    assert abs(tms - np.sum(target ** 2) / 150) < 1e-14
    h = 1e-6
    for (i, c) in [(0, 0), (7, 2), (49, 1)]:
        p = pred.copy()
        p[i, c] += h
        lp = cnn.mse_loss(p, target)[0]
        p[i, c] -= 2 * h
        lm = cnn.mse_loss(p, target)[0]
        assert abs((lp - lm) / (2 * h) - g[i, c]) < 1e-8
