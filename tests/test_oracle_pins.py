"""Pins of the FP64 oracle against facts fixed by the paper's equations and by mathematics.

None of these compare the oracle with itself: each checks a closed form, an
invariant, a brute-force evaluation or a special case that reduces to a
textbook result.
"""
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import pm
from synth import lattice_positions, plane_wave_particles

RNG = np.random.default_rng(12345)


def _rand_particles(n_p, seed=0, umax=0.3):
    r = np.random.default_rng(seed)
    return r.random((n_p, 3)), (r.random((n_p, 3)) - 0.5) * 2 * umax


# --------------------------------------------------------------------------
# P1-P3: deposit
# --------------------------------------------------------------------------

def test_p1_deposit_partition_of_unity():
    pos, u = _rand_particles(300, seed=1)
    a = 0.07
    dep = pm.deposit(pos, u, a, 8)
    q = pm.deposit_quantities(u, a)
    for c in range(10):
        tot = dep[c].sum()
        ref = q[c].sum()
        assert abs(tot - ref) <= 1e-13 * max(1.0, np.abs(q[c]).sum()), c
    # e = sqrt(a^2 + u^2) written out independently
    e = np.sqrt(a * a + (u ** 2).sum(1))
    assert np.allclose(dep[0].sum(), e.sum(), rtol=1e-14, atol=0)
    assert np.allclose(dep[4].sum(), (u[:, 0] ** 2 / e).sum(), rtol=1e-13, atol=0)


def test_p2_uniform_lattice_and_vertex_particle():
    n = 8
    pos = lattice_positions(n)
    a = 0.25
    dep = pm.deposit(pos, np.zeros_like(pos), a, n)
    assert np.all(dep[0] == a)  # exactly uniform
    assert np.all(dep[1:] == 0)
    # one particle exactly on vertex (3, 5, 6)
    p = np.array([[3 / n, 5 / n, 6 / n]])
    d = pm.deposit(p, np.zeros_like(p), 1.0, n)[0]
    assert d[6, 5, 3] == 1.0 and d.sum() == 1.0


def test_p3_bruteforce_loop():
    n = 6
    pos, u = _rand_particles(40, seed=3)
    a = 0.3
    dep = pm.deposit(pos, u, a, n)
    ref = np.zeros((10, n, n, n))
    for p in range(pos.shape[0]):
        e = math.sqrt(a * a + sum(u[p, d] ** 2 for d in range(3)))
        vals = [e, u[p, 0], u[p, 1], u[p, 2]] + [u[p, i] * u[p, j] / e for i, j in pm.SYM]
        s = [pos[p, d] * n for d in range(3)]
        b = [int(math.floor(s[d])) for d in range(3)]
        f = [s[d] - b[d] for d in range(3)]
        for cz in range(2):
            for cy in range(2):
                for cx in range(2):
                    w = (f[0] if cx else 1 - f[0]) * (f[1] if cy else 1 - f[1]) * (f[2] if cz else 1 - f[2])
                    for c in range(10):
                        ref[c, (b[2] + cz) % n, (b[1] + cy) % n, (b[0] + cx) % n] += w * vals[c]
    assert np.max(np.abs(dep - ref)) <= 1e-15 * np.max(np.abs(ref)) * 10


def test_p3_cic_interpolation_reproduces_trilinear_functions():
    """CIC interpolation is exact for any function that is trilinear inside a cell: a field
    f(x, y, z) = c0 + cx x + cy y + cz z + cxy x y + cxz x z + cyz y z + cxyz x y z sampled on the
    vertices returns f at every particle whose cell does not cross the periodic seam."""
    n = 8
    r = np.random.default_rng(3)
    c = r.standard_normal(8)
    v = np.arange(n) / n
    Z, Y, X = np.meshgrid(v, v, v, indexing="ij")

    def f(x, y, z):
        return (c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * x * z + c[6] * y * z
                + c[7] * x * y * z)

    pos = r.uniform(0.0, (n - 1) / n, (500, 3))  # cells 0 .. n-2: no corner wraps
    got = pm.interpolate([f(X, Y, Z)], pos, n)[0]
    want = f(pos[:, 0], pos[:, 1], pos[:, 2])
    assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))


# --------------------------------------------------------------------------
# P4: FFT against a brute-force DFT
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [4, 8, 16])
def test_p4_fft_bruteforce_parseval_roundtrip(n):
    f = np.random.default_rng(100 + n).standard_normal((n, n, n))
    fk = pm.fft3(f)
    idx = np.arange(n)
    # brute force: sum over all n^3 points for every (kz, ky, kx) of the half spectrum
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    pts = np.stack([zz.ravel(), yy.ravel(), xx.ravel()], 1)
    kz, ky, kx = np.meshgrid(idx, idx, np.arange(n // 2 + 1), indexing="ij")
    ks = np.stack([kz.ravel(), ky.ravel(), kx.ravel()], 1)
    phase = np.exp(-2j * np.pi * (ks @ pts.T) / n)
    ref = (phase @ f.ravel()).reshape(n, n, n // 2 + 1)
    assert np.max(np.abs(fk - ref)) < 1e-12 * np.max(np.abs(ref))
    # round trip and Parseval (full spectrum energy from the half spectrum)
    assert np.max(np.abs(pm.ifft3(fk, n) - f)) < 1e-14
    w = np.full(n // 2 + 1, 2.0)
    w[0] = w[-1] = 1.0
    e_k = (np.abs(fk) ** 2 * w).sum() / n ** 3
    assert abs(e_k - (f ** 2).sum()) < 1e-12 * (f ** 2).sum()


def test_p4_single_mode_lands_in_one_bin():
    """A real cosine of lattice mode m transforms to exactly the bins +m and -m of the full
    spectrum (in the half spectrum: one bin, or two when kx = 0 pairs them), each n^3 / 2."""
    n = 8
    idx = np.arange(n)
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    for m in [(1, 0, 0), (0, 3, 0), (2, 1, 3), (0, 0, 4)]:
        f = np.cos(2 * np.pi * (m[0] * x + m[1] * y + m[2] * z) / n)
        fk = pm.fft3(f)
        big = np.argwhere(np.abs(fk) > 1e-9 * n ** 3)
        want = {((m[2]) % n, (m[1]) % n, m[0])} if m[0] > 0 else {((m[2]) % n, (m[1]) % n, 0),
                                                                  ((-m[2]) % n, (-m[1]) % n, 0)}
        if m[0] == n // 2:
            want = {((m[2]) % n, (m[1]) % n, m[0]), ((-m[2]) % n, (-m[1]) % n, m[0])}
        assert {tuple(b) for b in big} == want, (m, big)
        val = n ** 3 / 2 if len(want) == 2 or m[0] not in (0, n // 2) else n ** 3
        for b in want:
            assert abs(fk[b] - val) < 1e-9 * n ** 3, (m, b, fk[b])


# --------------------------------------------------------------------------
# helpers to drive the solve with mesh sources
# --------------------------------------------------------------------------

def _sim_with_deposit(n, physics, dep, tau=30.0, box=320.0, n_p=None):
    n_p = n ** 3 if n_p is None else n_p
    pos = np.zeros((n_p, 3))
    s = pm.OracleSim(n=n, box_mpch=box, physics=physics, pos=pos, u=np.zeros_like(pos), tau=tau)
    s.dep = dep
    return s


def _plane(n, m):
    g = np.arange(n) / n
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    return np.cos(2 * np.pi * (m[0] * x + m[1] * y + m[2] * z))


def _kt(n, m):
    return np.array([2 * n * math.sin(math.pi * mi / n) for mi in m])


# --------------------------------------------------------------------------
# P5: phi for a plane-wave density
# --------------------------------------------------------------------------

@pytest.mark.parametrize("inv_dtau", [0.0, 1.0 / 0.7])
def test_p5_phi_plane_wave_closed_form(inv_dtau):
    n, m = 16, (1, 2, 3)
    s = _sim_with_deposit(n, pm.SCALAR, None)
    a, hc = s.bg.a(s.tau), s.bg.hconf(s.tau)
    eb = s.bg.ebar(a)
    A = 1e-3
    kap = s.bg.kappa(n, n ** 3) / a ** 2
    E = eb * (1 + A * _plane(n, m))
    dep = np.zeros((10, n, n, n))
    dep[0] = E / kap
    s.dep = dep
    z = np.zeros((n, n, n))
    phi, chi, _, _ = s._solve_once(z, z, 0.0, inv_dtau)
    kt2 = float((_kt(n, m) ** 2).sum())
    ref = eb * A * _plane(n, m) / (-kt2 - 3 * hc * inv_dtau - 6 * hc * hc - eb)
    # round-off scale is set by the source (E ~ ebar), not by its small modulation A
    assert np.max(np.abs(phi - ref)) < 1e-12 * np.max(np.abs(ref)) / A
    assert np.max(np.abs(chi)) == 0.0


def test_p5_newtonian_laplacian_real_space():
    n = 16
    s = _sim_with_deposit(n, pm.NEWTONIAN, None)
    a = s.bg.a(s.tau)
    rho = 1.0 + 0.3 * RNG.standard_normal((n, n, n))
    rho *= n ** 3 / rho.sum()  # mean one particle per cell
    s.dep = (rho * a)[None]
    s.solve(0.0)
    E = s.bg.kappa(n, n ** 3) / a * rho  # kappa a^-2 n00 with n00 = a rho
    src = E - s.bg.ebar(a)
    lap = pm.laplacian7(s.phi, n)
    assert np.max(np.abs(lap - src)) < 1e-11 * np.max(np.abs(src))


# --------------------------------------------------------------------------
# P6: chi
# --------------------------------------------------------------------------

def _solve_with_K(n, m, C, physics=pm.SCALAR):
    s = _sim_with_deposit(n, physics, None)
    a = s.bg.a(s.tau)
    kap = s.bg.kappa(n, n ** 3) / a ** 2
    dep = np.zeros((10, n, n, n))
    dep[0] = s.bg.ebar(a) / kap
    cosw = _plane(n, m)
    for idx, (i, j) in enumerate(pm.SYM):
        dep[4 + idx] = C[i, j] * cosw / kap
    s.dep = dep
    z = np.zeros((n, n, n))
    return s, s._solve_once(z, z, 0.0, 0.0)


def test_p6_chi_axis_wave_real_space_laplacian():
    n, m = 16, (3, 0, 0)
    C = np.array([[1.0, 0.2, -0.3], [0.2, -0.5, 0.1], [-0.3, 0.1, 0.7]]) * 1e-6
    _, (phi, chi, _, _) = _solve_with_K(n, m, C)
    sig = 4.0 * C * 1.0  # lagged phi = 0: Sigma = 4 K
    # k along x: chi satisfies (4/3) d_x^2 chi = Sigma_xx - tr(Sigma)/3 with the 3-point second difference
    lap = pm.laplacian7(chi, n)
    ref = 0.75 * (sig[0, 0] - np.trace(sig) / 3.0) * _plane(n, m)
    assert np.max(np.abs(lap - ref)) < 1e-10 * np.max(np.abs(ref))


def test_p6_chi_oblique_closed_form_and_isotropic_zero():
    n, m = 16, (1, 2, 2)
    C = np.array([[1.0, 0.4, -0.3], [0.4, -0.5, 0.25], [-0.3, 0.25, 0.2]]) * 1e-6
    _, (phi, chi, _, _) = _solve_with_K(n, m, C)
    kt = _kt(n, m)
    k2 = kt @ kt
    sig = 4.0 * C
    ref_amp = -(3.0 / (4.0 * k2 * k2)) * (kt @ sig @ kt - k2 * np.trace(sig) / 3.0)
    ref = ref_amp * _plane(n, m)
    assert np.max(np.abs(chi - ref)) < 1e-11 * np.max(np.abs(ref))
    _, (_, chi_iso, _, _) = _solve_with_K(n, m, np.eye(3) * 1e-6)
    assert np.max(np.abs(chi_iso)) < 1e-12 * np.max(np.abs(ref))


# --------------------------------------------------------------------------
# P7: B
# --------------------------------------------------------------------------

def _solve_with_J(n, m, V):
    s = _sim_with_deposit(n, pm.FULL, None)
    a = s.bg.a(s.tau)
    kap = s.bg.kappa(n, n ** 3) / a ** 2
    dep = np.zeros((10, n, n, n))
    dep[0] = s.bg.ebar(a) / kap
    for i in range(3):
        dep[1 + i] = V[i] * _plane(n, m) / kap
    s.dep = dep
    z = np.zeros((n, n, n))
    return s._solve_once(z, z, 0.0, 0.0)


def test_p7_b_closed_form_transverse_and_longitudinal():
    n, m = 16, (2, -1, 1)
    V = np.array([1.0, -2.0, 0.5]) * 1e-7
    _, _, B, _ = _solve_with_J(n, m, V)
    kt = _kt(n, m)
    k2 = kt @ kt
    ref = 4.0 / k2 * (V - kt * (kt @ V) / k2)
    for i in range(3):
        assert np.max(np.abs(B[i] - ref[i] * _plane(n, m))) < 1e-11 * np.max(np.abs(ref))
    # a longitudinal current sources no frame dragging
    _, _, B0, _ = _solve_with_J(n, m, kt / np.linalg.norm(kt) * 1e-7)
    assert max(np.max(np.abs(b)) for b in B0) < 1e-12 * np.max(np.abs(ref))
    # real-space check along an axis: -(1/4) lap B_y = S_y for k along x, V along y
    m2 = (2, 0, 0)
    _, _, B2, _ = _solve_with_J(n, m2, np.array([0.0, 1e-7, 0.0]))
    assert np.max(np.abs(-0.25 * pm.laplacian7(B2[1], n) - 1e-7 * _plane(n, m2))) < 1e-10 * 1e-7


# The other terms of the momentum source S_i = exp(psi + 3 phi) J_i - phidot d_i psi (Eq. 6 with the
# pure gradients dropped): the time-derivative term through an evolution solve whose lagged fields
# are single waves (product-to-sum gives B in closed form), the metric factor through uniform
# offsets of phi and chi (B is P7's closed form times exp(4 phi0 - chi0)).

def _plane_sin(n, m):
    g = np.arange(n) / n
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    return np.sin(2 * np.pi * (m[0] * x + m[1] * y + m[2] * z))


def _evolution_b(n, phi1, phi2, chi1, J, dtau_last, dtau):
    """B of one elliptic evolution solve of the oracle whose lagged fields and current are given
    (uniform energy density, no stresses)."""
    s = _sim_with_deposit(n, pm.FULL, None)
    a = s.bg.a(s.tau)
    kap = s.bg.kappa(n, n ** 3) / a ** 2
    dep = np.zeros((10, n, n, n))
    dep[0] = s.bg.ebar(a) / kap
    for i in range(3):
        dep[1 + i] = J[i] / kap
    s.dep = dep
    s.phi, s.phi_prev, s.chi = phi1, phi2, chi1
    s.dtau_last = dtau_last
    s.solved_once = True
    s.solve(dtau)
    return s.B


def _b_of_wave(V, m, n):
    """(4 / kt^2) (delta - kt kt / kt^2) V: B of a current (or momentum source) V sin/cos(k.x), P7."""
    kt = _kt(n, m)
    k2 = kt @ kt
    return 4.0 / k2 * (V - kt * (kt @ V) / k2)


def _phidot_term_error():
    """Relative max error of B against the closed form when S_i = -phidot d_i psi alone.

    phi_{n-1} = 0, phi_{n-2} = -dtau'' A cos(k1.x) -> phidot = A cos(k1.x);
    chi_{n-1} = -C cos(k2.x)                       -> psi = phi - chi = C cos(k2.x),
    centred difference d_i psi = -C s_i sin(k2.x) with s_i = n sin(2 pi m2_i / n), so
    S_i = A C s_i cos(k1.x) sin(k2.x) = (A C s_i / 2) [sin((k2 + k1).x) + sin((k2 - k1).x)],
    and each of the two waves q gets the transverse projector of P7 with its own kt(q)."""
    n = 16
    m1, m2 = np.array([1, 2, 0]), np.array([2, -1, 1])
    A, C, dtl = 3e-6, 2e-4, 0.5
    z = np.zeros((n, n, n))
    B = _evolution_b(n, z, -dtl * A * _plane(n, m1), -C * _plane(n, m2), [z, z, z], dtl, 0.4)
    sv = np.array([n * math.sin(2 * math.pi * mi / n) for mi in m2])
    ref = [np.zeros((n, n, n)) for _ in range(3)]
    for q in (m2 + m1, m2 - m1):
        bq = _b_of_wave(0.5 * A * C * sv, q, n)
        for i in range(3):
            ref[i] = ref[i] + bq[i] * _plane_sin(n, q)
    scale = max(np.max(np.abs(r)) for r in ref)
    return max(np.max(np.abs(B[i] - ref[i])) for i in range(3)) / scale


def _metric_factor_error():
    """Relative max error of B against P7's closed form times exp(psi0 + 3 phi0) = exp(4 phi0 - chi0)
    for uniform lagged phi0 (no time derivative) and chi0 and the current J = V cos(k.x)."""
    n, m = 16, (2, -1, 1)
    V = np.array([1.0, -2.0, 0.5]) * 1e-7
    phi0, chi0 = 3e-3, -2e-3
    one = np.ones((n, n, n))
    J = [V[i] * _plane(n, m) for i in range(3)]
    B = _evolution_b(n, phi0 * one, phi0 * one, chi0 * one, J, 0.5, 0.4)
    ref = _b_of_wave(V, m, n) * math.exp(4 * phi0 - chi0)
    return max(np.max(np.abs(B[i] - ref[i] * _plane(n, m))) for i in range(3)) / np.max(np.abs(ref))


def test_p7_momentum_source_time_derivative_term_two_waves():
    assert _phidot_term_error() < 1e-11


def test_p7_momentum_source_metric_factor_uniform_offsets():
    assert _metric_factor_error() < 1e-11


def test_p7_momentum_source_pins_catch_planted_mistakes(monkeypatch):
    """Each pin fails for a plausible mistake planted in the oracle's momentum source: the sign of the
    time-derivative term, psi in place of phi in the derivative, and the exponent of the metric factor
    (exp(psi + 2 phi), exp(phi - chi)... as written out below)."""
    good = pm.momentum_source

    def flipped(J, phi, chi, phidot, gphi, gchi):
        return [np.exp(phi - chi + 3 * phi) * J[i] + phidot * (gphi[i] - gchi[i]) for i in range(3)]

    def grad_phi_only(J, phi, chi, phidot, gphi, gchi):
        return [np.exp(phi - chi + 3 * phi) * J[i] - phidot * gphi[i] for i in range(3)]

    def exponent_2phi(J, phi, chi, phidot, gphi, gchi):
        return [np.exp(phi - chi + 2 * phi) * J[i] - phidot * (gphi[i] - gchi[i]) for i in range(3)]

    def exponent_plus_chi(J, phi, chi, phidot, gphi, gchi):
        return [np.exp(phi + chi + 3 * phi) * J[i] - phidot * (gphi[i] - gchi[i]) for i in range(3)]

    for bad, pin in ((flipped, _phidot_term_error), (grad_phi_only, _phidot_term_error),
                     (exponent_2phi, _metric_factor_error), (exponent_plus_chi, _metric_factor_error)):
        monkeypatch.setattr(pm, "momentum_source", bad)
        assert pin() > 1e-3, bad.__name__
    monkeypatch.setattr(pm, "momentum_source", good)
    assert _phidot_term_error() < 1e-11 and _metric_factor_error() < 1e-11


# --------------------------------------------------------------------------
# P8-P9: tensor sector and projectors
# --------------------------------------------------------------------------

def _rand_sym_spectra(n, seed):
    r = np.random.default_rng(seed)
    return [pm.fft3(r.standard_normal((n, n, n))) for _ in range(6)]


def test_p8_tt_projection_is_transverse_traceless_idempotent():
    n = 8
    kt = pm.lattice_symbols(n)
    sig = _rand_sym_spectra(n, 5)
    tt = pm.tt_project(sig, kt)
    tt2 = pm.tt_project(tt, kt)
    scale = max(np.max(np.abs(t)) for t in tt)
    for a_, b_ in zip(tt, tt2):
        assert np.max(np.abs(a_ - b_)) < 1e-12 * scale
    trace = tt[0] + tt[3] + tt[5]
    assert np.max(np.abs(trace)) < 1e-12 * scale
    for i in range(3):
        kh = sum(kt[j] * tt[pm.SYM_INDEX[(i, j)]] for j in range(3))
        assert np.max(np.abs(kh)) < 1e-9 * scale


def test_p8_crank_nicolson_energy_and_static_fixed_point():
    k2 = np.array([4.0, 100.0, 3e4])
    h = np.array([1.0, -0.5, 0.2]) + 0j
    pi = np.array([0.3, 2.0, -7.0]) + 0j
    e0 = k2 * np.abs(h) ** 2 + np.abs(pi) ** 2
    for _ in range(200):
        h, pi = pm.crank_nicolson_tensor(h, pi, 0.0, k2, 0.05, 0.0)
    e1 = k2 * np.abs(h) ** 2 + np.abs(pi) ** 2
    assert np.max(np.abs(e1 - e0) / e0) < 1e-12
    S = np.array([2.0, -1.0, 5.0]) + 0j
    hs, ps = pm.crank_nicolson_tensor(S / k2, 0 * S, S, k2, 0.3, 1.7)
    assert np.max(np.abs(hs - S / k2)) < 1e-15 and np.max(np.abs(ps)) < 1e-13


def test_p9_svt_decomposition_completes_identity():
    """Scalar (chi), vector and tensor parts add back to the trace-free source."""
    n = 8
    kt = pm.lattice_symbols(n)
    k2 = kt[0] ** 2 + kt[1] ** 2 + kt[2] ** 2
    sig = _rand_sym_spectra(n, 7)
    tr = (sig[0] + sig[3] + sig[5]) / 3.0
    tf = [s - (tr if i == j else 0.0) for s, (i, j) in zip(sig, pm.SYM)]
    chi = pm.chi_from_sigma(sig, kt, n)
    # the scalar part of Eq. 5 is 2 (-kt_i kt_j + delta_ij kt^2 / 3) chi
    scal = [2.0 * (-kt[i] * kt[j] + (k2 / 3.0 if i == j else 0.0)) * chi for i, j in pm.SYM]
    tt = pm.tt_project(sig, kt)
    vec = [t - s_ - h_ for t, s_, h_ in zip(tf, scal, tt)]
    mask = k2 > 0
    scale = max(np.max(np.abs(t[mask])) for t in tf)
    # the remainder is a pure vector mode: k_i k_j V_ij = 0, V_ii = 0 and Lambda^TT V = 0
    kk = sum((1.0 if i == j else 2.0) * kt[i] * kt[j] * v for v, (i, j) in zip(vec, pm.SYM))
    assert np.max(np.abs((kk / np.where(mask, k2, 1.0))[mask])) < 1e-10 * scale
    assert np.max(np.abs((vec[0] + vec[3] + vec[5])[mask])) < 1e-10 * scale
    assert max(np.max(np.abs(t[mask])) for t in pm.tt_project(vec, kt)) < 1e-10 * scale


# --------------------------------------------------------------------------
# P10: zero self-force and momentum conservation (Newtonian limit)
# --------------------------------------------------------------------------

def test_p10_zero_self_force_and_total_momentum():
    n = 16
    pos = np.array([[0.3141, 0.7182, 0.1618]])
    s = pm.OracleSim(n=n, box_mpch=320.0, physics=pm.NEWTONIAN, pos=pos, u=np.zeros_like(pos), tau=30.0)
    s.deposit()
    s.solve(0.0)
    g = s.gathered()[5:8, 0]
    gscale = np.max(np.abs(pm.grad(s.phi, n)[0]))
    assert np.max(np.abs(g)) < 1e-12 * gscale
    pos, _ = _rand_particles(500, seed=11)
    s = pm.OracleSim(n=n, box_mpch=320.0, physics=pm.NEWTONIAN, pos=pos, u=np.zeros_like(pos), tau=30.0)
    s.deposit()
    s.solve(0.0)
    g = s.gathered()[5:8]
    assert np.max(np.abs(g.sum(axis=1))) < 1e-11 * np.max(np.abs(g)) * pos.shape[0] ** 0.5


# --------------------------------------------------------------------------
# P11-P12: bulk flow, zero mode as exact roots of the constraint
# --------------------------------------------------------------------------

def test_p11_uniform_bulk_flow_drift():
    n = 8
    pos = lattice_positions(n)
    s = pm.OracleSim(n=n, box_mpch=320.0, physics=pm.FULL, pos=pos, u=np.zeros_like(pos), tau=30.0)
    a = s.bg.a(s.tau)
    uvec = np.array([3.0, -4.0, 12.0]) / 13.0 * 10.0 * a  # |u| = 10 a: relativistic
    s.u[:] = uvec
    dtau = 0.4
    s.deposit()
    s.solve(0.0)
    phibar = s.phi.mean()
    for f in [s.phi - phibar, s.chi] + list(s.B):
        assert np.max(np.abs(f)) < 1e-13 * max(1.0, abs(phibar))
    s.update(dtau)
    ah = s.bg.a(30.0 + 0.5 * dtau)
    u2 = uvec @ uvec
    eh = math.sqrt(ah * ah + u2)
    vel = uvec / eh * (1 + (3 - u2 / eh ** 2) * phibar)
    ref = pm.wrap_positions(pos + dtau * vel)
    d = s.pos - ref
    d -= np.round(d)
    # round-off of the (exactly zero) gradients is the only perturbation
    assert np.max(np.abs(d)) < 1e-13
    assert np.allclose(s.u, uvec, rtol=1e-13, atol=0)


def _uniform_sim(u_over_a):
    n = 4
    pos = lattice_positions(n)
    s = pm.OracleSim(n=n, box_mpch=320.0, physics=pm.SCALAR, pos=pos, u=np.zeros_like(pos), tau=30.0)
    a = s.bg.a(s.tau)
    s.u[:, 0] = u_over_a * a
    s.deposit()
    return s


def test_p12_zero_mode_quasistatic_root():
    """Iterating the lagged solve to its fixed point solves (3/2) H^2 exp(-4 phi) = E exp(phi) exactly."""
    s = _uniform_sim(0.3)
    a = s.bg.a(s.tau)
    E = s.bg.kappa(4, 64) / a ** 2 * s.dep[0].mean()
    hc = s.bg.hconf(s.tau)
    exact = math.log(1.5 * hc * hc / E) / 5.0
    z = np.zeros((4, 4, 4))
    phi, chi = z, z
    for _ in range(60):
        phi, chi, _, _ = s._solve_once(phi, chi, 0.0, 0.0)
    assert abs(phi.mean() - exact) < 1e-13 * abs(exact)
    assert np.max(np.abs(phi - phi.mean())) < 1e-15


def test_p12_zero_mode_time_derivative_root():
    """With an implicit time derivative, the fixed point solves (3/2)(H - phidot)^2 exp(-4 phi) = E exp(phi)."""
    s = _uniform_sim(0.2)
    a = s.bg.a(s.tau)
    E = s.bg.kappa(4, 64) / a ** 2 * s.dep[0].mean()
    hc = s.bg.hconf(s.tau)
    phi_prev, dt = -0.0021, 0.9

    def F(p):
        pd = (p - phi_prev) / dt
        return 1.5 * (hc - pd) ** 2 * math.exp(-4 * p) - E * math.exp(p)

    exact = brentq(F, -0.05, 0.05, xtol=1e-16)
    z = np.zeros((4, 4, 4))
    phi = z + phi_prev
    for _ in range(80):
        pd = (phi - phi_prev) / dt
        # the implicit part of the operator uses phi_prev; R takes the current iterate and its derivative
        E_, J, K, gphi, gchi = s._sources(phi, z, pd)
        eb = s.bg.ebar(a)
        R = pm.hamiltonian_remainder(E_, eb, hc, phi, z, pd, gphi)
        rhs = (E_ - eb) - 3 * hc / dt * phi_prev + R
        phi = rhs / (-3 * hc / dt - 6 * hc * hc - eb)
    assert abs(phi.mean() - exact) < 1e-12 * abs(exact)


def test_p12_zero_mode_time_derivative_root_with_slip():
    """The same with a homogeneous slip chi: the fixed point solves
    (3/2)(H - phidot)^2 exp(-2 (2 phi - chi)) = E exp(phi), i.e. Eq. 4 over exp(2 phi) with psi = phi - chi."""
    s = _uniform_sim(0.2)
    a = s.bg.a(s.tau)
    E = s.bg.kappa(4, 64) / a ** 2 * s.dep[0].mean()
    hc = s.bg.hconf(s.tau)
    eb = s.bg.ebar(a)
    phi_prev, dt = -0.0021, 0.9
    for chi0 in (0.004, -0.006):
        def F(p):
            pd = (p - phi_prev) / dt
            return 1.5 * (hc - pd) ** 2 * math.exp(-2 * (2 * p - chi0)) - E * math.exp(p)

        exact = brentq(F, -0.05, 0.05, xtol=1e-16)
        z = np.zeros((4, 4, 4))
        chi = z + chi0
        phi = z + phi_prev
        for _ in range(80):
            pd = (phi - phi_prev) / dt
            E_, J, K, gphi, gchi = s._sources(phi, chi, pd)
            R = pm.hamiltonian_remainder(E_, eb, hc, phi, chi, pd, gphi)
            rhs = (E_ - eb) - 3 * hc / dt * phi_prev - 3 * hc * hc * chi + R
            phi = rhs / (-3 * hc / dt - 6 * hc * hc - eb)
        assert abs(phi.mean() - exact) < 1e-12 * abs(exact), chi0
        # the slip moves the root by far more than the tolerance
        assert abs(exact - brentq(lambda p: 1.5 * (hc - (p - phi_prev) / dt) ** 2 * math.exp(-4 * p)
                                  - E * math.exp(p), -0.05, 0.05, xtol=1e-16)) > 1e-4


def test_p12_fixed_point_satisfies_full_constraint_pointwise():
    """A spatially varying fixed point satisfies Eq. 4 / exp(2 phi) in real space (7-point Laplacian)."""
    n = 8
    r = np.random.default_rng(21)
    pos = lattice_positions(n) + 0.3 / n * (r.random((n ** 3, 3)) - 0.5)
    u = 0.05 * (r.random((n ** 3, 3)) - 0.5)
    s = pm.OracleSim(n=n, box_mpch=4000.0, physics=pm.SCALAR, pos=pos, u=u, tau=3.0)
    s.deposit()
    a, hc = s.bg.a(s.tau), s.bg.hconf(s.tau)
    eb = s.bg.ebar(a)
    z = np.zeros((n, n, n))
    phi, chi = z, z
    for _ in range(60):
        phi, chi, _, _ = s._solve_once(phi, chi, 0.0, 0.0)
    E = s.bg.kappa(n, n ** 3) / a ** 2 * s.dep[0]
    g = pm.grad(phi, n)
    F = (pm.laplacian7(phi, n) - 0.5 * (g[0] ** 2 + g[1] ** 2 + g[2] ** 2)
         + 1.5 * hc * hc * np.exp(-2 * (2 * phi - chi)) - E * np.exp(phi))
    assert np.max(np.abs(F)) < 1e-10 * np.max(np.abs(E - eb))
    assert np.max(np.abs(phi)) > 1e-4  # non-trivial field


def test_p12_fixed_point_with_time_derivative_and_slip_pointwise():
    """Spatially varying fields with a time derivative and a varying slip: iterating the lagged
    equation (implicit operator, remainder R at the current iterate) to its fixed point satisfies
    Eq. 4 / exp(2 phi) pointwise, with phidot = (phi - phi_prev) / dtau and the real-space Laplacian."""
    n = 8
    r = np.random.default_rng(22)
    pos = lattice_positions(n) + 0.3 / n * (r.random((n ** 3, 3)) - 0.5)
    u = 0.05 * (r.random((n ** 3, 3)) - 0.5)
    s = pm.OracleSim(n=n, box_mpch=4000.0, physics=pm.SCALAR, pos=pos, u=u, tau=3.0)
    s.deposit()
    a, hc = s.bg.a(s.tau), s.bg.hconf(s.tau)
    eb = s.bg.ebar(a)
    x = (np.arange(n) + 0.0) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    phi_prev = -1e-3 + 4e-4 * np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    chi = 3e-4 * np.cos(2 * np.pi * Z) + 1e-4
    dt = 0.3
    E = s.kappa() / a ** 2 * s.dep[0]
    kt = pm.lattice_symbols(n)
    denom = -(kt[0] ** 2 + kt[1] ** 2 + kt[2] ** 2) - 3 * hc / dt - 6 * hc * hc - eb
    phi = phi_prev.copy()
    for _ in range(100):
        pd = (phi - phi_prev) / dt
        R = pm.hamiltonian_remainder(E, eb, hc, phi, chi, pd, pm.grad(phi, n))
        rhs = (E - eb) - 3 * hc / dt * phi_prev - 3 * hc * hc * chi + R
        phi = pm.ifft3(pm.fft3(rhs) / denom, n)
    pd = (phi - phi_prev) / dt
    g = pm.grad(phi, n)
    F = (pm.laplacian7(phi, n) - 0.5 * (g[0] ** 2 + g[1] ** 2 + g[2] ** 2)
         + 1.5 * (hc - pd) ** 2 * np.exp(-2 * (2 * phi - chi)) - E * np.exp(phi))
    assert np.max(np.abs(pd)) > 1e-4 * hc  # a real time derivative
    assert np.max(np.abs(F)) < 1e-10 * np.max(np.abs(E - eb))


# --------------------------------------------------------------------------
# P13-P14: linear plane wave; Zel'dovich growth
# --------------------------------------------------------------------------

def _project_wave(sim, q, k):
    pos, u = sim.particles_by_id()
    d = pos[:, 0] - q[:, 0]
    d -= np.round(d)
    s = np.sin(k * q[:, 0])
    return (d * s).sum() / (s * s).sum(), (u[:, 0] * s).sum() / (s * s).sum()


def _linear_recursion(bg, n, mode, U, P, tau, dtau, steps, physics):
    dx = 1.0 / n
    k = 2 * math.pi * mode
    kt2 = (2 * n * math.sin(math.pi * mode / n)) ** 2
    Phi_prev = None
    dtp = 0.0
    out = []
    for it in range(steps):
        a, hc = bg.a(tau), bg.hconf(tau)
        eb = bg.ebar(a)
        D = -(2 / dx) * math.sin(k * dx / 2) * U
        if physics == pm.NEWTONIAN:
            Phi = eb * D / (-kt2)
        elif Phi_prev is None:
            Phi = eb * D / (-kt2 - 6 * hc * hc - eb)
        else:
            Phi = (eb * D - 3 * hc / dtp * Phi_prev) / (-kt2 - 3 * hc / dtp - 6 * hc * hc - eb)
        P = P + dtau * a * Phi * math.sin(k * dx) * math.cos(k * dx / 2) / dx
        U = U + dtau * P / bg.a(tau + dtau / 2)
        tau += dtau
        Phi_prev, dtp = Phi, dtau
        out.append((U, P))
    return out


@pytest.mark.parametrize("physics", [pm.NEWTONIAN, pm.SCALAR])
def test_p13_linear_plane_wave_matches_scalar_recursion(physics):
    n, mode = 32, 2
    bg = pm.Background(320.0)
    tau0 = bg.tau(0.02)
    dtau = (bg.tau(0.05) - tau0) / 10
    eps = 1e-6 / n
    q = lattice_positions(n)
    P0 = 0.3 * eps * bg.a(tau0) * bg.hconf(tau0)
    pos, u = plane_wave_particles(n, n, eps, P0, mode=mode)
    sim = pm.OracleSim(n=n, box_mpch=320.0, physics=physics, pos=pos, u=u, tau=tau0)
    ref = _linear_recursion(bg, n, mode, eps, P0, tau0, dtau, 10, physics)
    k = 2 * math.pi * mode
    for it in range(10):
        sim.step(dtau)
        U, P = _project_wave(sim, q, k)
        assert abs(U - ref[it][0]) < 1e-5 * abs(ref[it][0]), (it, U, ref[it][0])
        assert abs(P - ref[it][1]) < 1e-5 * abs(ref[it][1]), (it, P, ref[it][1])


def _growth_run(steps, n=32, mode=1, physics=pm.NEWTONIAN):
    bg = pm.Background(320.0)
    tau0, tau1 = bg.tau(0.02), bg.tau(0.05)
    dtau = (tau1 - tau0) / steps
    gam = math.cos(math.pi * mode / n) ** 2
    s = (-1 + math.sqrt(1 + 24 * gam)) / 2
    U0 = 1e-6 / n
    th = tau0 - dtau / 2
    P0 = bg.a(th) * s * U0 * (th / tau0) ** s / th
    # only the x-profile matters: use a thin lattice in y, z (n_p = n still, mesh n)
    pos, u = plane_wave_particles(n, n, U0, P0, mode=mode)
    sim = pm.OracleSim(n=n, box_mpch=320.0, physics=physics, pos=pos, u=u, tau=tau0)
    q = lattice_positions(n)
    for _ in range(steps):
        sim.step(dtau)
    U, _ = _project_wave(sim, q, 2 * math.pi * mode)
    return U / U0, (tau1 / tau0) ** s


@pytest.mark.slow
def test_p14_zeldovich_growth_second_order_convergence():
    errs = []
    for steps in (10, 20, 40):
        g, exact = _growth_run(steps)
        errs.append(abs(g - exact))
    assert errs[0] < 5e-3 * 2.5
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.3 < r2 < 4.7, errs


def test_p14_relativistic_growth_approaches_newtonian_inside_the_horizon():
    """The relativistic scalar run of the same linear wave grows like the Newtonian one up to
    corrections of relative size ~3 H^2 / kt^2 (the Newtonian limit holds well inside the horizon):
    for modes 1, 2, 4 and 8 of the 320 Mpc/h box the growth ratio differs from 1 by less than
    3 H(tau_0)^2 / kt^2 and the difference shrinks with every doubling of k."""
    devs = []
    bg = pm.Background(320.0)
    h0 = bg.hconf(bg.tau(0.02))
    for mode in (1, 2, 4, 8):
        g_newt, _ = _growth_run(20, mode=mode)
        g_rel, _ = _growth_run(20, mode=mode, physics=pm.SCALAR)
        kt2 = (2 * 32 * math.sin(math.pi * mode / 32)) ** 2
        dev = abs(g_rel / g_newt - 1.0)
        assert dev < 3.0 * h0 * h0 / kt2, (mode, dev)
        devs.append(dev)
    assert all(b < a / 3 for a, b in zip(devs, devs[1:])), devs


# --------------------------------------------------------------------------
# P15: translation by whole cells
# --------------------------------------------------------------------------

def test_p15_translation_by_whole_cells():
    n = 16
    r = np.random.default_rng(8)
    pos = r.random((2000, 3))
    u = 0.01 * (r.random((2000, 3)) - 0.5)
    shift = np.array([3, 1, 5])
    s1 = pm.OracleSim(n=n, box_mpch=320.0, physics=pm.FULL, pos=pos, u=u, tau=30.0)
    s2 = pm.OracleSim(n=n, box_mpch=320.0, physics=pm.FULL, pos=pm.wrap_positions(pos + shift / n), u=u, tau=30.0)
    for s in (s1, s2):
        s.step(0.5)
        s.step(0.5)
    for f1, f2 in zip([s1.phi, s1.chi] + s1.B, [s2.phi, s2.chi] + s2.B):
        rolled = np.roll(f1, shift=(shift[2], shift[1], shift[0]), axis=(0, 1, 2))
        assert np.max(np.abs(rolled - f2)) < 1e-13 * np.max(np.abs(f1))
    d = s2.pos - pm.wrap_positions(s1.pos + shift / n)
    d -= np.round(d)
    assert np.max(np.abs(d)) < 1e-13


# --------------------------------------------------------------------------
# P18: B from the vector part of the trace-free space-space equation (parabolic route)
# --------------------------------------------------------------------------

def _sym_from(T):
    return [T[i, j] for i, j in pm.SYM]


def test_p18_vector_source_projects_the_spin1_part():
    kt = [np.array(v) for v in (0.7, -1.3, 0.4)]
    kv = np.array([float(v) for v in kt])
    kh = kv / np.linalg.norm(kv)
    e = np.cross(kh, [0.2, 0.9, -0.4])
    vec = np.outer(kh, e) + np.outer(e, kh)                      # spin-1
    t1 = np.cross(kh, [1.0, 0.0, 0.0]); t1 /= np.linalg.norm(t1)
    t2 = np.cross(kh, t1)
    tt = np.outer(t1, t1) - np.outer(t2, t2)                      # spin-2
    sc = np.outer(kh, kh) - np.eye(3) / 3                         # spin-0, trace-free
    w = pm.vector_source(_sym_from(vec + 3.0 * tt - 2.0 * sc), kt)
    assert np.allclose([float(x) for x in w], e, atol=1e-14)


def test_p18_parabolic_step_integrates_a2_exactly_to_second_order():
    """Constant vector source: a^2 B(tau) = -i w / |kt| * int a^2 dtau; EdS a^2 = (H0 tau / 2)^4."""
    bg = pm.Background(320.0)
    kt = [np.array(v) for v in (1.5, 0.0, 0.0)]
    w = [np.array(0.0), np.array(2.0e-6), np.array(0.0)]
    tau0, tau1 = bg.tau(0.02), bg.tau(0.1)
    h0 = bg.h0
    exact = -1j * 2.0e-6 / 1.5 * (h0 / 2) ** 4 * (tau1 ** 5 - tau0 ** 5) / 5
    errs = []
    for steps in (10, 20, 40):
        d = (tau1 - tau0) / steps
        state = [np.array(0j)] * 3
        for i in range(steps):
            t = tau0 + (i + 1) * d
            state = pm.b_parabolic_step(state, w, kt, d, bg.a(t - 0.5 * d))
        errs.append(abs(complex(state[1]) - exact) / abs(exact))
        assert abs(complex(state[0])) == 0.0 and abs(complex(state[2])) == 0.0
    assert errs[0] < 1e-2
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_p18_parabolic_and_elliptic_routes_agree():
    """The two B equations are equivalent through stress-energy conservation (Sec. 3.1, below Eq. 6):
    on a smooth Zel'dovich flow they agree to the deposit's discretisation (measured ~5 %)."""
    from synth import spectrum_power_law_m2, zeldovich_particles
    from synth.ics import eds_a_of_tau
    n, box, steps = 32, 320.0, 10
    bg = pm.Background(box)
    tau0 = bg.tau(0.02)
    dtau = (bg.tau(0.05) - tau0) / steps
    pos, u = zeldovich_particles(n, 1, spectrum_power_law_m2, box, 0.2, 0.02, 0.02, eds_a_of_tau(tau0 - 0.5 * dtau, box))
    sims = [pm.OracleSim(n=n, box_mpch=box, physics=pm.FULL, pos=pos, u=u, tau=tau0, b_route=r)
            for r in ("elliptic", "parabolic")]
    for _ in range(steps):
        for s in sims:
            s.step(dtau)
    num = math.sqrt(sum(np.sum((sims[1].B[j] - sims[0].B[j]) ** 2) for j in range(3)))
    den = math.sqrt(sum(np.sum(sims[0].B[j] ** 2) for j in range(3)))
    assert den > 0 and num / den < 0.1, num / den


# ---------------------------------------------------------------------------
# P19: a second particle species (the stress-energy sums run over all particles, each with its
# own mass, Sec. 3.1 below Eq. 10; the kick and drift are per unit mass and keep the momentum
# non-perturbative, so a hot species takes the same update)
# ---------------------------------------------------------------------------

def _two_species_fields(sim):
    return [sim.phi, sim.chi] + list(sim.B) + sim.h_real()


def test_p19_splitting_one_species_into_two_changes_nothing():
    """Half of the particles as species 2 with half of the mass (equal particle masses): the same run."""
    from synth import config_particles
    pos, u, tau0, dtau = config_particles("zeldovich_32_scalar_fp64", n=16)
    one = pm.OracleSim(n=16, box_mpch=160.0, physics=pm.FULL, pos=pos, u=u, tau=tau0)
    two = pm.OracleSim(n=16, box_mpch=160.0, physics=pm.FULL, pos=pos[0::2], u=u[0::2], tau=tau0,
                       pos2=pos[1::2], u2=u[1::2], mass_fraction2=0.5)
    assert abs(two.species_weight() - 1.0) < 1e-15 and abs(two.kappa() - one.kappa()) < 1e-15 * one.kappa()
    for _ in range(3):
        one.step(dtau)
        two.step(dtau)
    for f1, f2 in zip(_two_species_fields(one), _two_species_fields(two)):
        assert np.max(np.abs(f1 - f2)) <= 1e-12 * (np.max(np.abs(f1)) + 1e-300)
    assert np.max(np.abs(one.pos[0::2] - two.pos)) < 1e-14
    assert np.max(np.abs(one.pos[1::2] - two.pos2)) < 1e-14
    assert np.max(np.abs(one.u[1::2] - two.u2)) < 1e-14 * np.max(np.abs(one.u))


@pytest.mark.parametrize("f", [0.3, 1e-9])
def test_p19_copy_as_second_species_is_a_test_population(f):
    """Species 2 = an exact copy of species 1 carrying any fraction f of the mass: the mesh sees the
    same total (m_1 N (1 + m_2/m_1) is the whole mass either way), so the fields equal those of
    species 1 alone, and the copy follows the same trajectories."""
    from synth import config_particles
    pos, u, tau0, dtau = config_particles("zeldovich_32_scalar_fp64", n=16)
    one = pm.OracleSim(n=16, box_mpch=160.0, physics=pm.FULL, pos=pos, u=u, tau=tau0)
    two = pm.OracleSim(n=16, box_mpch=160.0, physics=pm.FULL, pos=pos, u=u, tau=tau0,
                       pos2=pos.copy(), u2=u.copy(), mass_fraction2=f)
    for _ in range(3):
        one.step(dtau)
        two.step(dtau)
    for f1, f2 in zip(_two_species_fields(one), _two_species_fields(two)):
        assert np.max(np.abs(f1 - f2)) <= 1e-12 * (np.max(np.abs(f1)) + 1e-300)
    assert np.max(np.abs(two.pos2 - two.pos)) == 0.0 and np.max(np.abs(two.u2 - two.u)) == 0.0
    assert np.max(np.abs(two.pos - one.pos)) < 1e-14


def test_p19_hot_species_raises_the_homogeneous_mode_by_its_kinetic_energy():
    """Species 1 at rest, species 2 with |u| = U in random directions, fraction f of the mass.  The mesh
    mean of kappa a^-2 n00 is (1 - f + f sqrt(1 + U^2/a^2)) ebar (CIC partition of unity), so the first
    quasi-static pass (phi = chi = 0 lagged, no remainder) gives the mean
    phi = f ebar (sqrt(1 + U^2/a^2) - 1) / (-6 H^2 - ebar)."""
    r = np.random.default_rng(19)
    n, box, f = 8, 80.0, 0.2
    bg = pm.Background(box)
    tau = bg.tau(0.05)
    a = bg.a(tau)
    U = 3.0 * a
    d = r.normal(size=(300, 3))
    u2 = U * d / np.linalg.norm(d, axis=1)[:, None]
    sim = pm.OracleSim(n=n, box_mpch=box, physics=pm.FULL, pos=lattice_positions(n), u=np.zeros((n ** 3, 3)),
                       tau=tau, pos2=r.random((300, 3)), u2=u2, mass_fraction2=f)
    sim.deposit()
    z = np.zeros((n, n, n))
    phi, _, _, _ = sim._solve_once(z, z, z, 0.0)
    eb, hc = bg.ebar(a), bg.hconf(tau)
    expect = f * eb * (math.sqrt(1.0 + (U / a) ** 2) - 1.0) / (-6.0 * hc * hc - eb)
    assert abs(phi.mean() - expect) < 1e-12 * abs(expect)
    # without the hot species' kinetic energy (U = 0) the mean vanishes
    sim0 = pm.OracleSim(n=n, box_mpch=box, physics=pm.FULL, pos=lattice_positions(n), u=np.zeros((n ** 3, 3)),
                        tau=tau, pos2=sim.pos2, u2=np.zeros_like(u2), mass_fraction2=f)
    sim0.deposit()
    phi0, _, _, _ = sim0._solve_once(z, z, z, 0.0)
    assert abs(phi0.mean()) < 1e-14 * abs(expect) / f


# --------------------------------------------------------------------------
# Transform count of one step against the per-field count of Sec. 4.1
# --------------------------------------------------------------------------

def _golden_fft_counts():
    rows = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "fft_counts_per_step.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if line:
                rows[line[0]] = (int(line[1]), int(line[2]))
    return rows


def _counted_step(monkeypatch, physics, b_route):
    """Second step of a small run (the first is the quasi-static start); returns the sequence of
    3D transforms it made, 'F' forward and 'B' backward."""
    pos, u = _rand_particles(200, seed=3, umax=0.01)
    s = pm.OracleSim(n=16, box_mpch=320.0, physics=physics, pos=pos, u=u, tau=30.0, b_route=b_route)
    s.step(0.3)
    calls = []
    fwd, inv = pm.fft3, pm.ifft3
    monkeypatch.setattr(pm, "fft3", lambda f: (calls.append("F"), fwd(f))[1])
    monkeypatch.setattr(pm, "ifft3", lambda fk, n: (calls.append("B"), inv(fk, n))[1])
    s.step(0.3)
    return "".join(calls)


def test_fft_count_of_a_parabolic_b_step_matches_sec_4_1(monkeypatch):
    g = _golden_fft_counts()
    seq = _counted_step(monkeypatch, pm.FULL, "parabolic")
    # phi: its source forward, phi back; chi: the six Sigma_ij forward, chi back; B: three back
    expect = ("F" * g["phi"][0] + "B" * g["phi"][1] + "F" * g["chi"][0] + "B" * g["chi"][1]
              + "F" * g["B"][0] + "B" * g["B"][1])
    assert seq == expect
    assert len(seq) == 12


def test_fft_counts_of_the_other_routes():
    """The same accounting for the other physics settings: B from the momentum constraint adds
    the three forward transforms of S_i (15 in all); scalar physics drops B (9); Newtonian
    gravity needs one transform each way (2)."""
    mp = pytest.MonkeyPatch()
    try:
        assert _counted_step(mp, pm.FULL, "elliptic") == "FB" + "F" * 6 + "B" + "F" * 3 + "B" * 3
    finally:
        mp.undo()
    for physics, want in ((pm.SCALAR, "FB" + "F" * 6 + "B"), (pm.NEWTONIAN, "FB")):
        mp = pytest.MonkeyPatch()
        try:
            assert _counted_step(mp, physics, "elliptic") == want
        finally:
            mp.undo()


# --------------------------------------------------------------------------
# P21: the exterior Schwarzschild metric in isotropic coordinates, an exact static vacuum
# solution of general relativity, pins the quadratic gradient terms of the scalar sources
# --------------------------------------------------------------------------

def _schwarzschild_isotropic(n_pts=400, seed=21, mass=1.0):
    """phi, chi = phi - psi and their derivatives at random points 2M <= r <= 40M.

    Isotropic form: g_tt = -((1 - M/2r) / (1 + M/2r))^2, g_ij = (1 + M/2r)^4 delta_ij; with the
    metric of Sec. 3.1 (g_00 = -a^2 e^{2 psi}, g_ij = a^2 e^{-2 phi} delta_ij at a = 1) that is
    e^{2 psi} = -g_tt and e^{-2 phi} = g_xx.  Derivatives are taken symbolically.
    """
    import sympy as sp
    X = sp.symbols("x y z", real=True)
    r = sp.sqrt(X[0] ** 2 + X[1] ** 2 + X[2] ** 2)
    q = mass / (2 * r)
    g_tt = -((1 - q) / (1 + q)) ** 2
    g_xx = (1 + q) ** 4
    psi = sp.log(-g_tt) / 2
    phi = -sp.log(g_xx) / 2
    chi = phi - psi
    f = lambda e: sp.lambdify(X, e, "numpy")
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n_pts, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pts = d * rng.uniform(2.0 * mass, 40.0 * mass, size=(n_pts, 1))
    ev = lambda e: np.broadcast_to(np.asarray(f(e)(*pts.T), dtype=float), (n_pts,)).copy()
    out = {"phi": ev(phi), "chi": ev(chi),
           "gphi": [ev(sp.diff(phi, v)) for v in X], "gchi": [ev(sp.diff(chi, v)) for v in X],
           "hchi": [[ev(sp.diff(chi, u, v)) for v in X] for u in X],
           "lap_phi": ev(sum(sp.diff(phi, v, 2) for v in X))}
    return out


def _trace_free(t):
    tr = (t[0] + t[3] + t[5]) / 3.0
    return [t[s] - (tr if i == j else 0.0) for s, (i, j) in enumerate(pm.SYM)]


def test_p21_schwarzschild_satisfies_the_trace_free_space_space_equation():
    """In vacuum (K = 0) the trace-free part of Eq. 5 reads TF[d_i d_j chi] = TF[Sigma_ij] / 2 with
    the oracle's Sigma; the exact metric satisfies it to rounding.  chi is second order in M/r, so
    the equation checks the d phi d phi term at O((M/r)^2), its balance with the phi-chi cross term
    at O((M/r)^3) and the d chi d chi term at O((M/r)^4)."""
    s = _schwarzschild_isotropic()
    zero = np.zeros_like(s["phi"])
    sig = pm.traceless_source([zero] * 6, s["phi"], s["chi"], s["gphi"], s["gchi"])
    sig_tf = _trace_free(sig)
    hess_tf = _trace_free([s["hchi"][i][j] for (i, j) in pm.SYM])
    scale = max(np.abs(x).max() for x in sig_tf)
    assert scale > 1e-4
    res = max(np.abs(2.0 * h - g).max() for h, g in zip(hess_tf, sig_tf))
    assert res <= 1e-12 * scale, res / scale
    # each quadratic term is needed: dropping any one of them leaves a residual far above rounding
    gp, gc = s["gphi"], s["gchi"]
    for drop in range(3):
        terms = [[gp[i] * gp[j], -(gp[i] * gc[j] + gc[i] * gp[j]), gc[i] * gc[j]] for (i, j) in pm.SYM]
        coef = [4.0, 4.0, 2.0]
        alt = _trace_free([sum(coef[t] * terms[s_][t] for t in range(3) if t != drop) for s_ in range(6)])
        bad = max(np.abs(2.0 * h - g).max() for h, g in zip(hess_tf, alt))
        assert bad > 1e-6 * scale, drop


def test_p21_schwarzschild_satisfies_the_hamiltonian_constraint():
    """Static vacuum with H = 0 and Ebar = 0: the lagged phi equation becomes Delta phi = R with
    R the oracle's non-linear remainder; for the exact metric (e^{-phi/2} = 1 + M/2r is harmonic)
    it holds to rounding."""
    s = _schwarzschild_isotropic()
    zero = np.zeros_like(s["phi"])
    R = pm.hamiltonian_remainder(zero, 0.0, 0.0, s["phi"], s["chi"], 0.0, s["gphi"])
    scale = np.abs(s["lap_phi"]).max()
    assert scale > 1e-4
    assert np.abs(s["lap_phi"] - R).max() <= 1e-12 * scale


def test_pointwise_gather_equals_the_gather_of_full_gradient_arrays():
    """The pointwise evaluation of the gathered values and centred-difference gradients (used where
    the full gradient arrays do not fit in host memory) equals the CIC interpolation of the full
    arrays of grad(f): the same sums, evaluated at the needed vertices only."""
    n = 16
    r = np.random.default_rng(3)
    pos, u = _rand_particles(300, 4, 0.01)
    sim = pm.OracleSim(n=n, box_mpch=160.0, physics=pm.FULL, pos=pos, u=u, tau=30.0)
    sim.phi, sim.chi = r.standard_normal((n, n, n)), r.standard_normal((n, n, n))
    sim.B = [r.standard_normal((n, n, n)) for _ in range(3)]
    full = sim.gathered()
    point = pm.gathered_pointwise(sim.phi, sim.chi, sim.B, sim.pos, n)
    assert full.shape == point.shape
    assert np.max(np.abs(full - point)) < 1e-12 * np.max(np.abs(full))
