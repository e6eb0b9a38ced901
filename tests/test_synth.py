"""Host checks of the seeded input generator (no GPU): the properties every parity case and the
benchmark rely on, each checked against its definition rather than against the generator's code."""
import math

import numpy as np
import pytest

from synth import lattice_positions, plane_wave_particles, spectrum_k_transfer, spectrum_power_law_m2
from synth import zeldovich_particles
from synth.ics import eds_a_of_tau, eds_hubble0, eds_tau_of_a, gaussian_displacement


def test_lattice_is_cell_centred_and_x_fastest():
    n = 4
    q = lattice_positions(n)
    assert q.shape == (n ** 3, 3)
    assert np.allclose(q[0], [0.125, 0.125, 0.125])
    assert np.allclose(q[1], [0.375, 0.125, 0.125])  # x fastest
    assert np.allclose(q[n], [0.125, 0.375, 0.125])
    assert np.allclose(q[n * n], [0.125, 0.125, 0.375])


def test_eds_background_round_trip_and_growth_rate():
    box = 2048.0
    for a in (0.02, 0.1, 0.5, 1.0):
        tau = eds_tau_of_a(a, box)
        assert abs(eds_a_of_tau(tau, box) - a) < 1e-15 * a
    # a = 1 at tau = 2 / H0, and H_conf = a'/a = 2 / tau
    h0 = eds_hubble0(box)
    assert abs(eds_a_of_tau(2.0 / h0, box) - 1.0) < 1e-15
    tau, e = 3.0, 1e-6
    dlna = (math.log(eds_a_of_tau(tau + e, box)) - math.log(eds_a_of_tau(tau - e, box))) / (2 * e)
    assert abs(dlna - 2.0 / tau) < 1e-8


@pytest.mark.parametrize("spectrum", [spectrum_power_law_m2, spectrum_k_transfer])
def test_displacement_is_seeded_longitudinal_band_limited_and_normalised(spectrum):
    n, box = 16, 320.0
    psi = gaussian_displacement(n, 5, spectrum, box, 0.2)
    assert np.array_equal(psi, gaussian_displacement(n, 5, spectrum, box, 0.2))
    assert not np.allclose(psi, gaussian_displacement(n, 6, spectrum, box, 0.2))
    # rms |Psi| = 0.2 lattice spacings
    assert abs(math.sqrt(np.mean(np.sum(psi ** 2, axis=0))) * n - 0.2) < 1e-12
    pk = [np.fft.fftn(psi[d]) for d in range(3)]
    m = np.fft.fftfreq(n, d=1.0 / n)
    kz, ky, kx = np.meshgrid(m, m, m, indexing="ij")
    kvec = (kx, ky, kz)
    # longitudinal: k x Psi(k) = 0 (a displacement of a potential flow)
    for i, j in ((0, 1), (1, 2), (2, 0)):
        cross = kvec[i] * pk[j] - kvec[j] * pk[i]
        assert np.max(np.abs(cross)) < 1e-10 * np.max(np.abs(pk[0]))
    # no power at k = 0 and none at or beyond the Nyquist wavenumber (spherical cut)
    kmag = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    power = sum(np.abs(p) ** 2 for p in pk)
    assert np.max(power[kmag >= n / 2]) < 1e-20 * np.max(power)
    assert power[0, 0, 0] < 1e-20 * np.max(power)


def test_zeldovich_positions_and_momenta_follow_the_growing_mode():
    n, box, a_ref = 16, 320.0, 0.02
    a_pos, a_vel = 0.05, 0.049
    pos, u = zeldovich_particles(n, 3, spectrum_power_law_m2, box, 0.2, a_ref, a_pos, a_vel)
    q = lattice_positions(n)
    d = pos - q
    d -= np.round(d)
    # displacement grows as D = a / a_ref: rms 0.2 * 2.5 = 0.5 cells
    assert abs(math.sqrt(np.mean(np.sum(d ** 2, axis=1))) * n - 0.2 * a_pos / a_ref) < 1e-9
    # v = H_conf(a_vel) D(a_vel) Psi and u = a v / sqrt(1 - v^2)
    psi = d / (a_pos / a_ref)
    v = (eds_hubble0(box) / math.sqrt(a_vel)) * (a_vel / a_ref) * psi
    want = a_vel * v / np.sqrt(1.0 - np.sum(v * v, axis=1, keepdims=True))
    assert np.max(np.abs(u - want)) < 1e-9 * np.max(np.abs(want))
    assert np.all((pos >= 0.0) & (pos < 1.0))


def test_plane_wave_particles():
    pos, u = plane_wave_particles(8, 8, 1e-3, 2e-4, mode=2, axis=1)
    q = lattice_positions(8)
    s = np.sin(2 * np.pi * 2 * q[:, 1])
    d = pos[:, 1] - q[:, 1]
    d -= np.round(d)
    assert np.allclose(d, 1e-3 * s, atol=1e-15)
    assert np.array_equal(pos[:, 0], q[:, 0]) and np.array_equal(pos[:, 2], q[:, 2])
    assert np.allclose(u[:, 1], 2e-4 * s) and not u[:, 0].any() and not u[:, 2].any()
