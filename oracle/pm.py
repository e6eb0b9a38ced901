"""FP64 CPU oracle of the relativistic particle-mesh step (TEST INFRASTRUCTURE).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
use this module.  It follows the method of Adamek & Christiansen,
"gevolution 2.0" (arXiv:2607.17929), Sec. 3, step by step in float64 with
numpy/scipy; it is deliberately plain (no blocking, no fusion) so that each
line can be checked against the equations by eye.

Conventions (readings of the paper where it is silent):
  * box side L = 1, c = 1; mesh of n^3 vertices at x_v = v/n, periodic;
    arrays are indexed [z][y][x] with x fastest (the paper's fast index, Sec. 2);
  * Einstein-de Sitter background: a = (H0 tau / 2)^2, H_conf = 2/tau,
    4 pi G a^2 rho_bar = (3/2) H0^2 / a;
  * equal-mass particles carrying u = q/m; 4 pi G m N_p = (3/2) H0^2; an optional
    second species of another particle mass carries a fraction f of the rest mass
    (4 pi G m_2 N_2 = (3/2) H0^2 f) and enters the deposit weighted by m_2 / m_1;
  * cloud-in-cell (CIC) assignment and interpolation (Sec. 3.1, below Eq. 13);
  * 7-point Laplacian (symbol -kt^2, kt_d = 2 n sin(pi m_d / n)) and centred
    differences for gradients; projectors use kt_d;
  * forward FFT unnormalised, inverse scaled by 1/n^3 (numpy's convention).

Pins: the quadratic gradient products in the trace-free source and the gradient
term of the Hamiltonian remainder are checked against an exact solution of general
relativity (the exterior Schwarzschild metric in isotropic coordinates); the whole
remainder through fixed points of the lagged equation that must satisfy Eq. 4
pointwise; the momentum source's time-derivative term -phidot d_i psi through an
evolution solve on single-wave lagged fields (B in closed form by product-to-sum)
and its metric factor exp(psi + 3 phi) through uniform offsets of phi and chi.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np
import scipy.fft as sfft

def _host_threads() -> int:
    """Threads for the library FFTs: the cores this process may run on, capped by OMP_NUM_THREADS when
    it is set (the share of the host's cores that belongs to this process)."""
    n = len(os.sched_getaffinity(0))
    try:
        cap = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        cap = 0
    return max(1, min(n, cap) if cap > 0 else n)


_WORKERS = _host_threads()

NEWTONIAN, SCALAR, FULL = "newtonian", "scalar", "full"

# symmetric tensor component order used everywhere: xx, xy, xz, yy, yz, zz
SYM = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))
SYM_INDEX = {p: s for s, p in enumerate(SYM)}
SYM_INDEX.update({(j, i): s for (i, j), s in list(SYM_INDEX.items())})


# ---------------------------------------------------------------------------
# Background (EdS reading of the scale factor the paper introduces in Sec. 3.1)
# ---------------------------------------------------------------------------

@dataclass
class Background:
    box_mpch: float

    @property
    def h0(self) -> float:
        """H0 in units of c / L for a box of L Mpc/h."""
        return self.box_mpch / 2997.92458

    def a(self, tau: float) -> float:
        return (0.5 * self.h0 * tau) ** 2

    def hconf(self, tau: float) -> float:
        """Conformal Hubble rate H = d ln a / d tau."""
        return 2.0 / tau

    def tau(self, a: float) -> float:
        return 2.0 * math.sqrt(a) / self.h0

    def ebar(self, a: float) -> float:
        """4 pi G a^2 rho_bar (Friedmann equation, EdS): (3/2) H0^2 / a."""
        return 1.5 * self.h0 ** 2 / a

    def kappa(self, n: int, n_p: int, mass_fraction: float = 1.0) -> float:
        """4 pi G m / dx^3 for N_p equal masses m carrying the fraction `mass_fraction` of the total
        rest mass, the total fixed by the Friedmann equation: 4 pi G m N_p = (3/2) H0^2 mass_fraction."""
        return 1.5 * self.h0 ** 2 * n ** 3 * mass_fraction / n_p


# ---------------------------------------------------------------------------
# Mesh helpers
# ---------------------------------------------------------------------------

def fft3(f: np.ndarray) -> np.ndarray:
    """Forward 3D real-to-complex DFT of an [z][y][x] array (unnormalised)."""
    return sfft.rfftn(f, workers=_WORKERS)


def ifft3(fk: np.ndarray, n: int) -> np.ndarray:
    """Inverse of fft3 (scaled by 1/n^3)."""
    return sfft.irfftn(fk, s=(n, n, n), workers=_WORKERS)


def lattice_symbols(n: int):
    """kt_d = (2/dx) sin(k_d dx/2) on the half spectrum, as broadcastable (x, y, z) arrays.

    k_d = 2 pi m_d with m_d the signed mode index; the 7-point Laplacian has
    symbol -(kt_x^2 + kt_y^2 + kt_z^2).
    """
    m_full = np.fft.fftfreq(n, d=1.0 / n)
    m_half = np.arange(n // 2 + 1, dtype=np.float64)
    ktx = (2.0 * n * np.sin(np.pi * m_half / n))[None, None, :]
    kty = (2.0 * n * np.sin(np.pi * m_full / n))[None, :, None]
    ktz = (2.0 * n * np.sin(np.pi * m_full / n))[:, None, None]
    return ktx, kty, ktz


def grad(f: np.ndarray, n: int):
    """Centred second-order differences (f[i+1] - f[i-1]) / (2 dx) along x, y, z."""
    h = 0.5 * n
    return [
        (np.roll(f, -1, axis=2) - np.roll(f, 1, axis=2)) * h,
        (np.roll(f, -1, axis=1) - np.roll(f, 1, axis=1)) * h,
        (np.roll(f, -1, axis=0) - np.roll(f, 1, axis=0)) * h,
    ]


def laplacian7(f: np.ndarray, n: int) -> np.ndarray:
    """Real-space 7-point Laplacian (used by tests, independent of the FFT)."""
    out = -6.0 * f
    for ax in range(3):
        out = out + np.roll(f, 1, axis=ax) + np.roll(f, -1, axis=ax)
    return out * (n * n)


# ---------------------------------------------------------------------------
# CIC weights, deposit (Sec. 3.1, Eqs. 11-13) and interpolation
# ---------------------------------------------------------------------------

def cic_cells(pos: np.ndarray, n: int):
    """Base vertex index (floor(x n) mod n) and fraction, per particle and axis."""
    s = pos * n
    fl = np.floor(s)
    frac = s - fl
    base = fl.astype(np.int64) % n
    return base, frac


def _corners(pos: np.ndarray, n: int):
    """Yield (flat vertex index, CIC weight) for the 8 corners of each particle's cell."""
    base, frac = cic_cells(pos, n)
    for cz in (0, 1):
        wz = frac[:, 2] if cz else 1.0 - frac[:, 2]
        iz = (base[:, 2] + cz) % n
        for cy in (0, 1):
            wy = frac[:, 1] if cy else 1.0 - frac[:, 1]
            iy = (base[:, 1] + cy) % n
            for cx in (0, 1):
                wx = frac[:, 0] if cx else 1.0 - frac[:, 0]
                ix = (base[:, 0] + cx) % n
                yield (iz * n + iy) * n + ix, wx * wy * wz


def deposit_quantities(u: np.ndarray, a: float, relativistic: bool = True) -> np.ndarray:
    """Per-particle quantities deposited on the mesh, shape (10, N_p).

    Rows: e, u_x, u_y, u_z, then u_i u_j / e for (ij) in xx, xy, xz, yy, yz, zz,
    where e = sqrt(a^2 + |u|^2) is the particle energy per unit mass times a
    (the square root in Eqs. 11 and 13 with the metric factor exp(2 phi) inside it
    dropped at this order).  In the Newtonian limit (Sec. 3.2) e is replaced by a.
    """
    if relativistic:
        e = np.sqrt(a * a + np.sum(u * u, axis=1))
    else:
        e = np.full(u.shape[0], float(a))
    q = [e, u[:, 0], u[:, 1], u[:, 2]]
    for i, j in SYM:
        q.append(u[:, i] * u[:, j] / e)
    return np.stack(q)


def deposit(pos: np.ndarray, u: np.ndarray, a: float, n: int, relativistic: bool = True,
            ncomp: int = 10) -> np.ndarray:
    """CIC deposit of n00 = sum W e, n0i = sum W u_i, nij = sum W u_i u_j / e.

    Returns an array (ncomp, n, n, n) [comp][z][y][x]; ncomp = 1 deposits n00 only.
    """
    q = deposit_quantities(u, a, relativistic)[:ncomp]
    out = np.zeros((ncomp, n ** 3))
    for idx, w in _corners(pos, n):
        for c in range(ncomp):
            out[c] += np.bincount(idx, weights=w * q[c], minlength=n ** 3)
    return out.reshape(ncomp, n, n, n)


def interpolate(fields, pos: np.ndarray, n: int) -> np.ndarray:
    """CIC interpolation of a list of [z][y][x] fields to particle positions -> (len(fields), N_p)."""
    flat = [f.reshape(-1) for f in fields]
    out = np.zeros((len(flat), pos.shape[0]))
    for idx, w in _corners(pos, n):
        for c, f in enumerate(flat):
            out[c] += w * f[idx]
    return out


def interpolate_with_gradients(fields, pos: np.ndarray, n: int) -> np.ndarray:
    """CIC interpolation, at the given positions, of each field and of its centred-difference gradient
    (f[v + e_d] - f[v - e_d]) / (2 dx), the differences evaluated only at the corner vertices the
    particles need (the same quantities as interpolating the full arrays of grad(f), without forming
    them).  Returns (len(fields), 4, N_p): value, d/dx, d/dy, d/dz."""
    flat = [np.asarray(f).reshape(-1) for f in fields]
    out = np.zeros((len(flat), 4, pos.shape[0]))
    h = 0.5 * n
    for idx, w in _corners(pos, n):
        iz, iy, ix = idx // (n * n), (idx // n) % n, idx % n
        nb = []
        for d, (dz, dy, dx) in enumerate(((0, 0, 1), (0, 1, 0), (1, 0, 0))):
            up = (((iz + dz) % n) * n + (iy + dy) % n) * n + (ix + dx) % n
            dn = (((iz - dz) % n) * n + (iy - dy) % n) * n + (ix - dx) % n
            nb.append((up, dn))
        for c, f in enumerate(flat):
            out[c, 0] += w * f[idx]
            for d, (up, dn) in enumerate(nb):
                out[c, 1 + d] += w * (f[up].astype(np.float64) - f[dn]) * h
    return out


def wrap_positions(x: np.ndarray) -> np.ndarray:
    """Periodic wrap into [0, 1); a result of exactly 1.0 maps to 0.0."""
    y = x - np.floor(x)
    y[y >= 1.0] = 0.0
    return y


# ---------------------------------------------------------------------------
# Metric solves (Sec. 3.1)
# ---------------------------------------------------------------------------

def expm1_minus_x(x: np.ndarray) -> np.ndarray:
    """exp(x) - 1 - x."""
    return np.expm1(x) - x


def hamiltonian_remainder(E, ebar, hconf, phi, chi, phidot, grad_phi):
    """Non-linear remainder R of the Hamiltonian constraint (Eq. 4 divided by exp(2 phi)).

    With psi = phi - chi and w = 2 phi - chi the constraint reads
        F = lap phi - |grad phi|^2/2 + (3/2)(H - phidot)^2 exp(-2w) - E exp(phi) = 0,
    whose linear part about phi = chi = phidot = 0 is
        lap phi - 3 H phidot - 6 H^2 phi + 3 H^2 chi - ebar phi - (E - ebar)
    (using (3/2) H^2 = ebar).  R collects everything else, so that F = 0 is
        lap phi - 3 H phidot - (6 H^2 + ebar) phi + 3 H^2 chi = (E - ebar) + R.
    """
    w = 2.0 * phi - chi
    g2 = grad_phi[0] ** 2 + grad_phi[1] ** 2 + grad_phi[2] ** 2
    return (0.5 * g2 + (E - ebar) * phi + E * expm1_minus_x(phi)
            - 1.5 * ((hconf - phidot) ** 2 * (np.expm1(-2.0 * w) + 2.0 * w)
                     + 2.0 * w * (2.0 * hconf * phidot - phidot ** 2) + phidot ** 2))


def traceless_source(K, phi, chi, gphi, gchi):
    """Sigma_ij = 4 exp(3 phi) K_ij + 4 d_i phi d_j phi - 4 (d_i phi d_j chi + d_i chi d_j phi) + 2 d_i chi d_j chi.

    This is the right-hand side of Eq. 5 (trace-free space-space equation) with
    16 pi G T_ij = 4 exp(3 phi) K_ij and the quadratic gradient terms of the
    bracket moved to the source, using psi = phi - chi.  Only the trace-free
    part of Sigma enters the solves.
    """
    e3 = np.exp(3.0 * phi)
    out = []
    for s, (i, j) in enumerate(SYM):
        out.append(4.0 * e3 * K[s] + 4.0 * gphi[i] * gphi[j]
                   - 4.0 * (gphi[i] * gchi[j] + gchi[i] * gphi[j]) + 2.0 * gchi[i] * gchi[j])
    return out


def momentum_source(J, phi, chi, phidot, gphi, gchi):
    """S_i = exp(psi + 3 phi) J_i - phidot d_i psi (Eq. 6; pure gradients dropped, they vanish under the projector)."""
    psi = phi - chi
    ef = np.exp(psi + 3.0 * phi)
    return [ef * J[i] - phidot * (gphi[i] - gchi[i]) for i in range(3)]


def nyquist_mask(n: int) -> np.ndarray:
    """1 on the half spectrum except on the Nyquist planes (any |m_d| = n/2), where it is 0.

    The scalar, vector and tensor projections contain factors such as
    kt_x kt_y that are odd in one component.  On a Nyquist plane k_d and -k_d
    are the same lattice mode, so such a factor has no well-defined sign there;
    chi, B and h are therefore given no Nyquist-plane modes (phi, whose symbol
    kt^2 is even, keeps them).
    """
    h = n // 2
    m = np.arange(n)
    ny = (m == h)
    mx = (np.arange(n // 2 + 1) == h)
    bad = ny[:, None, None] | ny[None, :, None] | mx[None, None, :]
    return np.where(bad, 0.0, 1.0)


def chi_from_sigma(sig_k, kt, n):
    """Scalar part of Eq. 5: chi(k) = -(3 / (4 kt^4)) (kt_i kt_j Sigma_ij - kt^2 Sigma_ii / 3); chi(0) = 0."""
    ktx, kty, ktz = kt
    k = (ktx, kty, ktz)
    k2 = ktx ** 2 + kty ** 2 + ktz ** 2
    contr = 0.0
    for s, (i, j) in enumerate(SYM):
        mult = 1.0 if i == j else 2.0
        contr = contr + mult * k[i] * k[j] * sig_k[s]
    trace = sig_k[0] + sig_k[3] + sig_k[5]
    with np.errstate(divide="ignore", invalid="ignore"):
        chik = -(3.0 / (4.0 * k2 * k2)) * (contr - k2 * trace / 3.0)
    chik = np.where(k2 > 0, chik, 0.0)
    return chik


def b_from_momentum(s_k, kt):
    """Eq. 6 after the spin-1 projector: B_i(k) = (4 / kt^2) (delta_ij - kt_i kt_j / kt^2) S_j(k); B(0) = 0."""
    k = kt
    k2 = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
    safe = np.where(k2 > 0, k2, 1.0)
    kdots = (k[0] * s_k[0] + k[1] * s_k[1] + k[2] * s_k[2]) / safe
    return [np.where(k2 > 0, 4.0 / safe * (s_k[i] - k[i] * kdots), 0.0) for i in range(3)]


def vector_source(sig_k, kt):
    """Vector part of the trace-free source: w_j = P_jl khat_m Sigma_lm with P = delta - khat khat.

    The spin-1 part of Sigma is khat_i w_j + khat_j w_i, and w = 0 at k = 0.
    """
    k = kt
    k2 = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
    kn = np.sqrt(np.where(k2 > 0, k2, 1.0))
    kh = [k[i] / kn for i in range(3)]
    v = [sum(sig_k[SYM_INDEX[(l, m)]] * kh[m] for m in range(3)) for l in range(3)]
    kv = kh[0] * v[0] + kh[1] * v[1] + kh[2] * v[2]
    return [np.where(k2 > 0, v[j] - kh[j] * kv, 0.0) for j in range(3)]


def b_parabolic_step(a2b_k, w, kt, dtau, a_mid):
    """Vector part of Eq. 5: (d_tau + 2 H)(i kt_i B_j + i kt_j B_i) = khat_i w_j + khat_j w_i.

    With B transverse this is d_tau (a^2 B_j) = -i a^2 w_j / |kt|; one step from
    tau - dtau to tau with a^2 at the midpoint.  State and result: a^2 B(k).
    """
    k2 = kt[0] ** 2 + kt[1] ** 2 + kt[2] ** 2
    kn = np.sqrt(np.where(k2 > 0, k2, 1.0))
    return [np.where(k2 > 0, a2b_k[j] + dtau * a_mid * a_mid * (-1j) * w[j] / kn, 0.0) for j in range(3)]


def tt_project(sig_k, kt):
    """Lambda^TT_{ij,kl} Sigma_kl = P_ik P_jl Sigma_kl - P_ij P_kl Sigma_kl / 2, P = delta - kt kt / kt^2."""
    k = kt
    k2 = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
    safe = np.where(k2 > 0, k2, 1.0)

    def P(i, j):
        return (1.0 if i == j else 0.0) - k[i] * k[j] / safe

    def S(i, j):
        return sig_k[SYM_INDEX[(i, j)]]

    # PS P (full contraction), trace part
    trPS = sum(P(k_, l) * S(l, k_) for k_ in range(3) for l in range(3))
    out = []
    for i, j in SYM:
        acc = 0.0
        for k_ in range(3):
            for l in range(3):
                acc = acc + P(i, k_) * P(j, l) * S(k_, l)
        acc = acc - 0.5 * P(i, j) * trPS
        out.append(np.where(k2 > 0, acc, 0.0))
    return out


def crank_nicolson_tensor(h, pi, src, k2, dtau, hconf_half):
    """One Crank-Nicolson step of h'' + 2 H h' + kt^2 h = src per mode (state h, pi = h').

        h+ - h   = dtau/2 (pi+ + pi)
        pi+ - pi = dtau src - dtau/2 kt^2 (h+ + h) - dtau H (pi+ + pi)
    solved in closed form.
    """
    d = dtau
    q = 0.25 * d * d * k2
    pin = (pi * (1.0 - q - d * hconf_half) + d * src - d * k2 * h) / (1.0 + q + d * hconf_half)
    hn = h + 0.5 * d * (pin + pi)
    return hn, pin


# ---------------------------------------------------------------------------
# The simulation state and the three stages of a step
# ---------------------------------------------------------------------------

@dataclass
class OracleSim:
    """FP64 particle-mesh simulation with the same call sequence as the C library.

    deposit() -> solve(dtau_prev) -> update(dtau); step(dtau) chains them, with
    dtau_prev = 0 (quasi-static solve) on the first step.
    """
    n: int
    box_mpch: float
    physics: str
    pos: np.ndarray
    u: np.ndarray
    tau: float
    ids: np.ndarray = None
    b_route: str = "elliptic"  # full physics: B from Eq. 6 ("elliptic") or from the vector part of Eq. 5
    # optional second particle species (its own particle mass, e.g. a hot, neutrino-like set):
    # positions, momenta per unit mass and the fraction of the total rest mass it carries
    pos2: np.ndarray = None
    u2: np.ndarray = None
    mass_fraction2: float = 0.0
    bg: Background = field(init=False)

    def __post_init__(self):
        self.bg = Background(self.box_mpch)
        self.pos = np.array(self.pos, dtype=np.float64)
        self.u = np.array(self.u, dtype=np.float64)
        if self.ids is None:
            self.ids = np.arange(self.pos.shape[0], dtype=np.int64)
        if self.pos2 is not None:
            self.pos2 = np.array(self.pos2, dtype=np.float64)
            self.u2 = np.array(self.u2, dtype=np.float64)
            if not 0.0 < self.mass_fraction2 < 1.0:
                raise ValueError("a second species needs 0 < mass_fraction2 < 1")
        elif self.mass_fraction2 != 0.0:
            raise ValueError("mass_fraction2 without a second species")
        n = self.n
        z = np.zeros((n, n, n))
        self.dep = None
        self.phi = z.copy()       # phi_{n-1} after a solve is the latest solution
        self.phi_prev = z.copy()  # phi_{n-2}
        self.chi = z.copy()
        self.B = [z.copy(), z.copy(), z.copy()]
        self.dtau_last = 0.0      # tau_{n-1} - tau_{n-2} (0: no time derivative yet)
        self.solved_once = False
        hk0 = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
        self.h_k = [hk0.copy() for _ in range(6)]   # 6-component tensor spectrum and its time derivative
        self.pi_k = [hk0.copy() for _ in range(6)]
        self.a2B_k = [hk0.copy() for _ in range(3)]  # a^2 B(k), the state of the parabolic B route
        self.last_sigma_k = None
        if self.b_route not in ("elliptic", "parabolic"):
            raise ValueError("b_route must be 'elliptic' or 'parabolic'")

    @property
    def n_p(self) -> int:
        return self.pos.shape[0]

    @property
    def n_p2(self) -> int:
        return 0 if self.pos2 is None else self.pos2.shape[0]

    def species_weight(self) -> float:
        """Particle mass of species 2 over that of species 1: (f / N_2) / ((1 - f) / N_1)."""
        f = self.mass_fraction2
        return (f / self.n_p2) / ((1.0 - f) / self.n_p)

    def kappa(self) -> float:
        """4 pi G m_1 / dx^3: species 1 carries the fraction 1 - f of the rest mass."""
        return self.bg.kappa(self.n, self.n_p, 1.0 - self.mass_fraction2)

    # -- stage 1 ----------------------------------------------------------
    def deposit(self):
        """The stress-energy sums run over the particles of every species, each weighted by its
        mass (Sec. 3.1, the sums over particles below Eq. 10); the deposit is kept in units of the
        species-1 particle mass: dep = dep_1 + (m_2 / m_1) dep_2."""
        a = self.bg.a(self.tau)
        rel = self.physics != NEWTONIAN
        nc = 10 if rel else 1
        self.dep = deposit(self.pos, self.u, a, self.n, relativistic=rel, ncomp=nc)
        if self.pos2 is not None:
            self.dep = self.dep + self.species_weight() * deposit(self.pos2, self.u2, a, self.n, relativistic=rel,
                                                                  ncomp=nc)
        return self.dep

    # -- stage 2 ----------------------------------------------------------
    def _sources(self, phi1, chi1, phidot):
        """Mesh sources from the deposit and the lagged fields (metric factors applied mesh-side)."""
        n = self.n
        a = self.bg.a(self.tau)
        kap = self.kappa() / (a * a)
        E = kap * self.dep[0]
        J = [kap * self.dep[1 + i] for i in range(3)]
        K = [kap * self.dep[4 + s] for s in range(6)]
        gphi = grad(phi1, n)
        gchi = grad(chi1, n)
        return E, J, K, gphi, gchi

    def _solve_once(self, phi1, chi1, phidot, inv_dtau, elliptic_b=True):
        n = self.n
        a = self.bg.a(self.tau)
        hc = self.bg.hconf(self.tau)
        eb = self.bg.ebar(a)
        E, J, K, gphi, gchi = self._sources(phi1, chi1, phidot)
        R = hamiltonian_remainder(E, eb, hc, phi1, chi1, phidot, gphi)
        rhs = (E - eb) - 3.0 * hc * inv_dtau * phi1 - 3.0 * hc * hc * chi1 + R
        kt = lattice_symbols(n)
        k2 = kt[0] ** 2 + kt[1] ** 2 + kt[2] ** 2
        denom = -k2 - 3.0 * hc * inv_dtau - 6.0 * hc * hc - eb
        phi = ifft3(fft3(rhs) / denom, n)
        sig = traceless_source(K, phi1, chi1, gphi, gchi)
        nyq = nyquist_mask(n)
        sig_k = [fft3(s) * nyq for s in sig]
        chi = ifft3(chi_from_sigma(sig_k, kt, n), n)
        B = None
        self._B_k = None
        if self.physics == FULL and elliptic_b:
            S = momentum_source(J, phi1, chi1, phidot, gphi, gchi)
            self._B_k = b_from_momentum([fft3(s) * nyq for s in S], kt)
            B = [ifft3(bk, n) for bk in self._B_k]
        return phi, chi, B, sig_k

    def solve(self, dtau_prev: float):
        """Metric solve at the current time.

        dtau_prev > 0: semi-implicit step with the time derivative
        (phi_n - phi_{n-1}) / dtau_prev treated implicitly and every non-linear
        term lagged to the previous solution (Sec. 3.1: the previous step's
        solution is a sufficient initial guess, no iterations).
        dtau_prev <= 0: quasi-static start (no time derivatives), two
        predictor-corrector passes starting from phi = chi = 0.
        """
        n = self.n
        if self.dep is None:
            raise RuntimeError("deposit() must run before solve()")
        if self.physics == NEWTONIAN:
            a = self.bg.a(self.tau)
            E = self.kappa() / (a * a) * self.dep[0]
            eb = self.bg.ebar(a)
            kt = lattice_symbols(n)
            k2 = kt[0] ** 2 + kt[1] ** 2 + kt[2] ** 2
            with np.errstate(divide="ignore", invalid="ignore"):
                pk = np.where(k2 > 0, fft3(E - eb) / (-np.where(k2 > 0, k2, 1.0)), 0.0)
            phi = ifft3(pk, n)
            self.phi_prev = self.phi
            self.phi = phi
            self.solved_once = True
            self.dep = None
            return
        kt = lattice_symbols(n)
        k2 = kt[0] ** 2 + kt[1] ** 2 + kt[2] ** 2
        if dtau_prev <= 0.0:
            z = np.zeros((n, n, n))
            phi1, chi1 = z, z
            for _ in range(2):
                phi, chi, B, sig_k = self._solve_once(phi1, chi1, 0.0, 0.0)
                phi1, chi1 = phi, chi
            self.phi_prev = phi
            self.phi = phi
            self.chi = chi
            self.dtau_last = 0.0
            if self.physics == FULL:
                # the start takes B from the momentum constraint with either route; the parabolic
                # route then integrates a^2 B from there
                self.B = B
                a = self.bg.a(self.tau)
                self.a2B_k = [a * a * bk for bk in self._B_k]
                self.h_k = [np.zeros_like(sig_k[0]) for _ in range(6)]
                self.pi_k = [np.zeros_like(sig_k[0]) for _ in range(6)]
        else:
            phidot = (self.phi - self.phi_prev) / self.dtau_last if self.dtau_last > 0 else 0.0
            parabolic = self.b_route == "parabolic"
            phi, chi, B, sig_k = self._solve_once(self.phi, self.chi, phidot, 1.0 / dtau_prev,
                                                  elliptic_b=not parabolic)
            if self.physics == FULL:
                src = tt_project(sig_k, kt)
                hc_half = self.bg.hconf(self.tau - 0.5 * dtau_prev)
                for s in range(6):
                    self.h_k[s], self.pi_k[s] = crank_nicolson_tensor(
                        self.h_k[s], self.pi_k[s], src[s], k2, dtau_prev, hc_half)
                if parabolic:
                    a_mid = self.bg.a(self.tau - 0.5 * dtau_prev)
                    self.a2B_k = b_parabolic_step(self.a2B_k, vector_source(sig_k, kt), kt, dtau_prev, a_mid)
                    a = self.bg.a(self.tau)
                    B = [ifft3(x / (a * a), n) for x in self.a2B_k]
                self.B = B
            self.phi_prev = self.phi
            self.phi = phi
            self.chi = chi
            self.dtau_last = dtau_prev
        self.last_sigma_k = sig_k
        self.solved_once = True
        self.dep = None

    def h_real(self):
        """Real-space tensor perturbation h_ij (6 components), zero before the first evolution."""
        return [ifft3(hk, self.n) for hk in self.h_k]

    # -- stage 3 ----------------------------------------------------------
    def gathered(self, pos=None):
        """CIC-interpolated fields at the particles (species 1, or the positions given): phi, chi,
        B (3), g_phi (3), g_chi (3), G_ij = d_i B_j (9)."""
        n = self.n
        fields = [self.phi, self.chi] + list(self.B)
        fields += grad(self.phi, n) + grad(self.chi, n)
        gB = [grad(self.B[j], n) for j in range(3)]
        fields += [gB[j][i] for i in range(3) for j in range(3)]
        return interpolate(fields, self.pos if pos is None else pos, n)

    def update(self, dtau: float, extra_gphi: np.ndarray | None = None):
        """Kick u^{n-1/2} -> u^{n+1/2} and drift x^n -> x^{n+1} (Eqs. 9-10 to first order in phi, psi, B).

        Kick, with a = a(tau_n), e = sqrt(a^2 + |u|^2) at u^{n-1/2}:
            du_i = dtau [ -((a^2 + 2|u|^2)/e) g^phi_i + e g^chi_i - u_j d_i B_j ]
        Drift, with a' = a(tau_n + dtau/2), e' = sqrt(a'^2 + |u|^2) at u^{n+1/2}:
            dx_i = dtau [ (u_i / e') (1 + (3 - |u|^2/e'^2) phi - chi) + B_i ]
        Newtonian limit (Sec. 3.2): du = -dtau a grad psi, dx = dtau u / a'.
        All fields are taken at x^n.  ``extra_gphi`` (3, N_p) is added to the
        gathered gradient of phi (the learned closure's correction).  The equations are per unit
        mass, so a second species takes the same update in the same fields.
        """
        a = self.bg.a(self.tau)
        ah = self.bg.a(self.tau + 0.5 * dtau)
        self.pos, self.u = self._kick_drift(self.pos, self.u, a, ah, dtau, extra_gphi)
        if self.pos2 is not None:
            self.pos2, self.u2 = self._kick_drift(self.pos2, self.u2, a, ah, dtau, None)
        self.tau += dtau

    def _kick_drift(self, pos, u_in, a, ah, dtau, extra_gphi):
        return kick_drift(self.gathered(pos), pos, u_in, a, ah, dtau, self.physics, extra_gphi)

    # -- whole step ---------------------------------------------------------
    def step(self, dtau: float, dtau_prev: float | None = None):
        """deposit -> solve -> kick/drift; dtau_prev defaults to the previous step's dtau (0 first)."""
        if dtau_prev is None:
            dtau_prev = self._last_step if self.solved_once else 0.0
        self.deposit()
        self.solve(dtau_prev)
        self.update(dtau)
        self._last_step = dtau

    _last_step: float = 0.0

    def particles_by_id(self):
        order = np.argsort(self.ids, kind="stable")
        return self.pos[order], self.u[order]

    def species2(self):
        """Positions and momenta of the second species (in their given order)."""
        return self.pos2, self.u2


def gathered_pointwise(phi, chi, B, pos: np.ndarray, n: int) -> np.ndarray:
    """The rows of OracleSim.gathered (phi, chi, B (3), g_phi (3), g_chi (3), G_ij = d_i B_j (9)) with the
    centred differences evaluated only at the vertices the particles need: the same quantities, for
    meshes whose full gradient arrays would not fit in host memory."""
    g = interpolate_with_gradients([phi, chi] + list(B), pos, n)
    rows = [g[0, 0], g[1, 0], g[2, 0], g[3, 0], g[4, 0]]
    rows += [g[0, 1], g[0, 2], g[0, 3], g[1, 1], g[1, 2], g[1, 3]]
    rows += [g[2 + j, 1 + i] for i in range(3) for j in range(3)]
    return np.stack(rows)


def kick_drift(g, pos, u_in, a, ah, dtau, physics, extra_gphi=None):
    """Kick and drift of particles from their gathered fields g (the rows of OracleSim.gathered); the
    equations of OracleSim.update.  Returns (wrapped positions, momenta)."""
    phi_p, chi_p = g[0], g[1]
    B_p = g[2:5]
    gphi = g[5:8].copy()
    gchi = g[8:11]
    G = g[11:20].reshape(3, 3, -1)  # G[i][j] = d_i B_j
    if extra_gphi is not None:
        gphi = gphi + extra_gphi
    u = u_in.T.copy()
    if physics == NEWTONIAN:
        u = u - dtau * a * gphi
        x = pos.T + dtau * u / ah
    else:
        u2 = np.sum(u * u, axis=0)
        e = np.sqrt(a * a + u2)
        force = -((a * a + 2.0 * u2) / e) * gphi + e * gchi
        if physics == FULL:
            force = force - np.einsum("j...,ij...->i...", u, G)
        u = u + dtau * force
        u2 = np.sum(u * u, axis=0)
        eh = np.sqrt(ah * ah + u2)
        vel = (u / eh) * (1.0 + (3.0 - u2 / (eh * eh)) * phi_p - chi_p)
        if physics == FULL:
            vel = vel + B_p
        x = pos.T + dtau * vel
    return wrap_positions(x.T.copy()), u.T.copy()
