"""Seeded particle sets for the relativistic particle-mesh step.

Units: the box side is 1 and c = 1, so positions live in [0, 1) and
velocities are fractions of c.  Particle arrays are ordered with x fastest:
particle index = (z*n + y)*n + x for the unperturbed lattice site (x, y, z).

Everything here is input construction.  The Zel'dovich approximation used to
displace the lattice is the standard first-order Lagrangian initial
condition, not part of the particle-mesh step, and it needs the
Einstein-de Sitter expansion law only to turn displacements into velocities.
"""
from __future__ import annotations

import math
from typing import Callable

import numpy as np
import scipy.fft as sfft

_WORKERS = max(1, min(16, (len(__import__("os").sched_getaffinity(0)))))

# speed of light in km/s divided by 100: H0 * (box in Mpc/h) / c = box / 2997.92458
_C_OVER_100 = 2997.92458


def eds_hubble0(box_mpch: float) -> float:
    """Hubble rate today in units of c / (box side), for h-scaled box sizes."""
    return box_mpch / _C_OVER_100


def eds_a_of_tau(tau: float, box_mpch: float) -> float:
    """Scale factor of an Einstein-de Sitter universe at conformal time tau."""
    h0 = eds_hubble0(box_mpch)
    return (0.5 * h0 * tau) ** 2


def eds_tau_of_a(a: float, box_mpch: float) -> float:
    """Conformal time (units of box/c) of an Einstein-de Sitter universe at scale factor a."""
    return 2.0 * math.sqrt(a) / eds_hubble0(box_mpch)


# --------------------------------------------------------------------------
# spectra (arbitrary normalisation; the amplitude is fixed by an rms rule)
# --------------------------------------------------------------------------

def spectrum_power_law_m2(k: np.ndarray) -> np.ndarray:
    """P(k) proportional to k^-2 (k in h/Mpc)."""
    out = np.zeros_like(k)
    nz = k > 0
    out[nz] = k[nz] ** -2.0
    return out


def spectrum_k_transfer(k: np.ndarray, k0: float = 0.02) -> np.ndarray:
    """P(k) proportional to k * T(k) with T(k) = (1 + (k/k0)^2)^-2 (k, k0 in h/Mpc)."""
    return k * (1.0 + (k / k0) ** 2) ** -2.0


# --------------------------------------------------------------------------
# lattices and Gaussian fields
# --------------------------------------------------------------------------

def lattice_positions(n: int) -> np.ndarray:
    """Cell-centred lattice (j + 1/2)/n, shape (n^3, 3), columns (x, y, z), x fastest."""
    c = (np.arange(n, dtype=np.float64) + 0.5) / n
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def gaussian_displacement(n: int, seed: int, spectrum: Callable[[np.ndarray], np.ndarray],
                          box_mpch: float, rms_cells: float) -> np.ndarray:
    """Zel'dovich displacement field of a seeded Gaussian density field.

    White noise from numpy's PCG64 generator (``default_rng(seed)``) is drawn
    on the n^3 lattice in [z][y][x] order and coloured by sqrt(P(|k|)); modes
    with |k| at or above the Nyquist wavenumber pi*n/L are removed (spherical
    cut) and so is k = 0.  The displacement is Psi(k) = i k delta(k) / |k|^2,
    so that delta = -div Psi, using the continuous wavevector.  The result is
    scaled so that the 3D rms of |Psi| equals ``rms_cells`` lattice spacings.

    Returns an array of shape (3, n, n, n) [component x,y,z][z][y][x] in box units.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    wk = sfft.rfftn(w, workers=_WORKERS)
    del w
    kf = 2.0 * np.pi / box_mpch
    m_full = np.fft.fftfreq(n, d=1.0 / n)
    m_half = np.arange(n // 2 + 1, dtype=np.float64)
    kz = (kf * m_full)[:, None, None]
    ky = (kf * m_full)[None, :, None]
    kx = (kf * m_half)[None, None, :]
    kmag = np.sqrt(kx * kx + ky * ky + kz * kz)
    k_nyq = np.pi * n / box_mpch
    amp = np.where((kmag > 0) & (kmag < k_nyq), np.sqrt(np.maximum(spectrum(np.where(kmag > 0, kmag, 1.0)), 0.0)), 0.0)
    dk = wk * amp
    del wk, amp
    inv_k2 = np.where(kmag > 0, 1.0 / np.where(kmag > 0, kmag * kmag, 1.0), 0.0)
    del kmag
    psi = np.empty((3, n, n, n), dtype=np.float64)
    for d, kd in enumerate((kx, ky, kz)):
        psi[d] = sfft.irfftn(1j * kd * dk * inv_k2, s=(n, n, n), workers=_WORKERS)
    rms = math.sqrt(float(np.mean(np.sum(psi * psi, axis=0))))
    if rms > 0:
        psi *= (rms_cells / n) / rms
    return psi


def _wrap(x: np.ndarray) -> np.ndarray:
    y = x - np.floor(x)
    y[y >= 1.0] = 0.0
    return y


def zeldovich_particles(n: int, seed: int, spectrum: Callable[[np.ndarray], np.ndarray],
                        box_mpch: float, rms_cells: float, a_ref: float,
                        a_pos: float, a_vel: float):
    """Zel'dovich initial conditions in Einstein-de Sitter (growth factor D = a / a_ref).

    Positions are the lattice displaced by D(a_pos) * Psi; the momenta per unit
    mass u = a v / sqrt(1 - v^2) use the velocity v = H_conf D Psi evaluated at
    a_vel (the leapfrog's half-step-earlier time level).  ``rms_cells`` is the rms
    displacement at a_ref, in lattice spacings.

    Returns (pos (n^3,3) float64 in [0,1), u (n^3,3) float64).
    """
    psi = gaussian_displacement(n, seed, spectrum, box_mpch, rms_cells)
    psi = psi.reshape(3, -1).T.copy()
    q = lattice_positions(n)
    pos = _wrap(q + (a_pos / a_ref) * psi)
    hc = eds_hubble0(box_mpch) / math.sqrt(a_vel)
    v = hc * (a_vel / a_ref) * psi
    v2 = np.sum(v * v, axis=1, keepdims=True)
    u = a_vel * v / np.sqrt(1.0 - v2)
    return pos, u


def plane_wave_particles(n: int, n_p: int, amp_disp: float, amp_mom: float, mode: int = 1, axis: int = 0):
    """One particle per cell at cell centres, displaced by a single sine wave.

    The particle at lattice coordinate q along ``axis`` is moved by
    amp_disp * sin(k q) along that axis and given momentum amp_mom * sin(k q)
    along the same axis, with k = 2*pi*mode (box units).  ``amp_disp`` is in
    box units.  ``n`` is unused except for validation (kept for symmetry with
    the mesh size); the lattice has n_p^3 particles.
    """
    del n
    q = lattice_positions(n_p)
    k = 2.0 * np.pi * mode
    s = np.sin(k * q[:, axis])
    pos = q.copy()
    pos[:, axis] += amp_disp * s
    pos = _wrap(pos)
    u = np.zeros_like(q)
    u[:, axis] = amp_mom * s
    return pos, u


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

CONFIGS = {
    # 32^3 particles and mesh, FP64, scalar (phi, chi) physics, 10 steps a = 0.02 -> 0.05
    "zeldovich_32_scalar_fp64": dict(n=32, box=320.0, spectrum=spectrum_power_law_m2, rms_cells=0.2,
                              a_ref=0.02, a_init=0.02, a_end=0.05, steps=10, physics="scalar",
                              precision="fp64", seed=1),
    # 256^3 full scalar+vector+tensor, FP32 fields, start at a = 0.1, steps of 1% in tau
    "ktk_256_full": dict(n=256, box=1024.0, spectrum=spectrum_k_transfer, rms_cells=0.2,
                        a_ref=0.02, a_init=0.1, a_end=None, steps=None, physics="full",
                        precision="fp32", seed=2),
    # 512^3 clustered: k^-2 spectrum from a = 0.02, evolved to a = 0.5 in 100 uniform-tau steps
    "clustered_512": dict(n=512, box=2048.0, spectrum=spectrum_power_law_m2, rms_cells=0.2,
                             a_ref=0.02, a_init=0.02, a_end=0.5, steps=100, physics="full",
                             precision="fp32", seed=3),
    # 1024^3 memory scale, Zel'dovich at a = 0.1
    "memory_1024": dict(n=1024, box=4096.0, spectrum=spectrum_power_law_m2, rms_cells=0.2,
                           a_ref=0.02, a_init=0.1, a_end=None, steps=None, physics="full",
                           precision="fp32", seed=4),
}


def config_particles(name: str, n: int | None = None, dtau0_frac: float = 0.01, a_init: float | None = None):
    """Initial particles of a named workload (optionally at a reduced lattice size n).

    The velocity time level is tau_0 - dtau_0/2 with dtau_0 = dtau0_frac * tau_0,
    unless the workload is a fixed uniform-tau schedule (then dtau_0 follows it).
    Returns (pos, u, tau0, dtau0).
    """
    c = CONFIGS[name]
    n = c["n"] if n is None else n
    box = c["box"] * (n / c["n"])  # keep the cell size fixed when shrinking
    a0 = c["a_init"] if a_init is None else a_init
    tau0 = eds_tau_of_a(a0, box)
    if c["steps"] and c["a_end"]:
        dtau0 = (eds_tau_of_a(c["a_end"], box) - tau0) / c["steps"]
    else:
        dtau0 = dtau0_frac * tau0
    a_vel = eds_a_of_tau(tau0 - 0.5 * dtau0, box)
    pos, u = zeldovich_particles(n, c["seed"], c["spectrum"], box, c["rms_cells"], c["a_ref"], a0, a_vel)
    return pos, u, tau0, dtau0
