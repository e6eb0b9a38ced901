"""Pins of the power-spectrum estimator (oracle.pk)."""
import numpy as np

from oracle import pk
from synth import gaussian_displacement, lattice_positions


def test_p17_poisson_particles_have_no_excess_power_at_low_k():
    r = np.random.default_rng(4)
    n_p, m, L = 40000, 32, 100.0
    pos = r.random((n_p, 3))
    k, p, cnt = pk.power_spectrum(pos, m, L)
    shot = L ** 3 / n_p
    low = k < 0.25 * np.pi * m / L
    # shot-noise-subtracted power is zero within the sampling error of each bin
    sig = shot / np.sqrt(cnt[low] / 2.0)
    assert np.all(np.abs(p[low]) < 5 * sig)
    k2, p2, _ = pk.power_spectrum(pos, m, L, subtract_shot_noise=False)
    assert np.all(np.abs(p2[low] / shot - 1) < 5 / np.sqrt(cnt[low] / 2.0))


def test_p17_unperturbed_lattice_has_zero_power_and_single_mode_one_bin():
    n, L = 16, 64.0
    q = lattice_positions(n)
    k, p, _ = pk.power_spectrum(q, n, L, subtract_shot_noise=False)
    assert np.max(np.abs(p)) < 1e-20
    # small displacement wave along y with mode 3: only bin 3 carries power
    amp = 1e-4 / n
    pos = q.copy()
    pos[:, 1] += amp * np.sin(2 * np.pi * 3 * q[:, 1])
    k, p, _ = pk.power_spectrum(pos, n, L, subtract_shot_noise=False)
    kf = 2 * np.pi / L
    b = np.rint(k / kf).astype(int)
    assert np.argmax(p) == np.where(b == 3)[0][0]
    assert np.all(p[b != 3] < 1e-8 * p[b == 3].max())


def test_p17_gaussian_field_recovers_input_shape():
    """Linear Zel'dovich displacement of a lattice: P(k) follows the input spectrum at low k."""
    n, L = 64, 256.0
    spec = lambda k: k ** -1.0  # noqa: E731
    psi = gaussian_displacement(n, 9, spec, L, rms_cells=0.02)
    pos = lattice_positions(n) + psi.reshape(3, -1).T
    pos -= np.floor(pos)
    k, p, cnt = pk.power_spectrum(pos, n, L, subtract_shot_noise=False)
    sel = (k > 0.05) & (k < 0.15 * np.pi * n / L)
    ratio = p[sel] / spec(k[sel])
    ratio /= np.median(ratio)
    assert np.all(np.abs(ratio - 1) < 4 / np.sqrt(cnt[sel] / 2.0) + 0.03)
