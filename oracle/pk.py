"""Matter power spectrum estimator (TEST INFRASTRUCTURE; FP64).

The paper computes power spectra on the fly (Sec. 4.1) and judges accuracy by
power-spectrum ratios (Sec. 4.4).  This estimator: CIC number density on an
m^3 mesh, density contrast, FFT, division by the CIC window
prod_d sinc^2(k_d dx / 2), |delta_k|^2 L^3 / m^6 minus the Poisson shot noise
L^3 / N_p, averaged in shells of width k_f = 2 pi / L (bin = round(|k| / k_f)).
"""
from __future__ import annotations

import numpy as np

from .pm import deposit, fft3


def power_spectrum(pos: np.ndarray, m: int, box_mpch: float, subtract_shot_noise: bool = True):
    """Return (k [h/Mpc], P(k) [(Mpc/h)^3], modes per bin) for bins 1 .. m/2."""
    n_p = pos.shape[0]
    rho = deposit(pos, np.zeros_like(pos), 1.0, m, relativistic=False, ncomp=1)[0]
    delta = rho * (m ** 3 / n_p) - 1.0
    dk = fft3(delta)
    L = box_mpch
    kf = 2.0 * np.pi / L
    m_full = np.fft.fftfreq(m, d=1.0 / m)
    m_half = np.arange(m // 2 + 1, dtype=np.float64)
    mz = m_full[:, None, None]
    my = m_full[None, :, None]
    mx = m_half[None, None, :]

    def sinc(t):
        return np.sinc(t / np.pi)  # numpy sinc is sin(pi t)/(pi t)

    # k_d dx / 2 = pi m_d / m
    w = (sinc(np.pi * mx / m) * sinc(np.pi * my / m) * sinc(np.pi * mz / m)) ** 2
    p = (np.abs(dk / w) ** 2) * (L ** 3 / m ** 6)
    if subtract_shot_noise:
        p = p - L ** 3 / n_p
    kmag = kf * np.sqrt(mx * mx + my * my + mz * mz)
    # each half-spectrum entry with 0 < kx < m/2 stands for two modes (k and -k)
    weight = np.where((mx > 0) & (mx < m / 2), 2.0, 1.0) * np.ones_like(kmag)
    b = np.rint(kmag / kf).astype(np.int64)
    nb = m // 2 + 1
    sel = (b >= 1) & (b < nb)
    cnt = np.bincount(b[sel], weights=weight[sel], minlength=nb)
    psum = np.bincount(b[sel], weights=(weight * p)[sel], minlength=nb)
    ksum = np.bincount(b[sel], weights=(weight * kmag)[sel], minlength=nb)
    good = cnt > 0
    return ksum[good] / cnt[good], psum[good] / cnt[good], cnt[good]
