"""Host checks of the closure driver's data augmentation against the oracle (CPU only)."""
import itertools

import numpy as np
import pytest

from oracle import pm as opm

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("perm,signs", [((0, 1, 2), (1, 1, -1)), ((2, 0, 1), (1, -1, 1)), ((1, 0, 2), (-1, -1, 1))])
def test_cube_symmetry_commutes_with_the_1x_force(perm, signs):
    from paper_2607_17929_amd.closure import cube_symmetry
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
    tp, tu, tg = cube_symmetry(torch.tensor(pos), torch.tensor(u), torch.tensor(g), perm, signs)
    g2 = force(tp.numpy(), tu.numpy())
    assert np.max(np.abs(g2 - tg.numpy())) < 1e-10 * np.max(np.abs(g))


def test_cube_symmetries_are_48_distinct_maps():
    from paper_2607_17929_amd.closure import cube_symmetry
    x = torch.tensor([[0.1, 0.2, 0.4]], dtype=torch.float64)
    seen = set()
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((-1.0, 1.0), repeat=3):
            p, _, _ = cube_symmetry(x, x.float(), x.float(), perm, signs)
            seen.add(tuple(np.round(p.numpy()[0], 12)))
    assert len(seen) == 48
