"""Training and evaluation driver of the learned force closure.

Everything numerical runs in the library's kernels (PM steps, the network's
forward and backward passes, Adam); this module only orders the calls and
forms the particle-level mean-squared-error gradient.

Training pairs: each seeded box is evolved with the 2x mesh; at a set of
snapshots both the 1x and the 2x mesh compute grad phi on the *same*
particles (quasi-static solves), and the target is their difference in units
of rms|grad phi| on the 1x mesh.  The loss is the particle MSE of the
network output interpolated to the particles.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L
from .pm import PMContext, tau_of_a


@dataclass
class Snapshot:
    pos: torch.Tensor      # [n][3] float64, identifier order
    u: torch.Tensor        # [n][3] momenta (float32)
    tau: float
    target: torch.Tensor   # [n][3] float32, (g_2x - g_1x) / rms_1x


def init_params(seed: int = 0) -> torch.Tensor:
    """He-style initialisation of the FP32 parameter vector (last layer small)."""
    r = np.random.default_rng(seed)
    out = []
    for li, (ci, co) in enumerate(((4, 16), (16, 16), (16, 3))):
        std = math.sqrt(2.0 / (ci * 27)) * (0.1 if li == 2 else 1.0)
        out.append(r.standard_normal(co * ci * 27) * std)
        out.append(np.zeros(co))
    return torch.tensor(np.concatenate(out), dtype=torch.float32)


def make_pairs(seeds, n_p: int, n1: int, box: float, a_snaps, steps: int, spectrum, rms_cells: float = 0.2,
               a0: float = 0.02, a1: float = 0.5, physics: str = "scalar", log=print):
    """Evolve each box on the 2x mesh and collect (particles, normalised force difference) snapshots."""
    from synth import zeldovich_particles
    from synth.ics import eds_a_of_tau

    n2 = 2 * n1
    tau0, tau1 = tau_of_a(box, a0), tau_of_a(box, a1)
    dtau = (tau1 - tau0) / steps
    snap_taus = sorted(tau_of_a(box, a) for a in a_snaps)
    c2 = PMContext(n2, n_p, box, physics=physics, precision="fp32")
    c2s = PMContext(n2, n_p, box, physics=physics, precision="fp32")
    c1 = PMContext(n1, n_p, box, physics=physics, precision="fp32", closure=True)
    out = []
    for seed in seeds:
        t0 = time.time()
        pos, u = zeldovich_particles(round(n_p ** (1 / 3)), seed, spectrum, box, rms_cells, 0.02, a0,
                                     eds_a_of_tau(tau0 - 0.5 * dtau, box))
        c2.init_particles(pos, u.astype(np.float32), tau0)
        k = 0
        for i in range(steps):
            c2.step(dtau)
            tau = c2.time()[0]
            while k < len(snap_taus) and tau >= snap_taus[k] - 1e-9 * tau:
                p, uu = c2.get_particles(device=True)
                g = []
                for ctx in (c1, c2s):
                    ctx.init_particles(p, uu, tau)
                    ctx.deposit()
                    ctx.solve_metric(0.0)
                    g.append(ctx.gather_grad_phi())
                c1.closure_set_params(torch.zeros(L.PM_CLOSURE_NPARAM))
                c1.closure_forward(False)
                rms = c1.closure_scale()
                out.append(Snapshot(pos=p, u=uu, tau=tau, target=((g[1] - g[0]) / rms).float().contiguous()))
                k += 1
        log(f"closure pairs: box seed {seed} done in {time.time() - t0:.1f} s ({len(out)} snapshots)")
    return out, c1


def train(ctx1: PMContext, snaps, params: torch.Tensor, iters: int, lr: float = 1e-3, log=print, log_every=100):
    """Adam on the particle MSE; returns (params, loss history)."""
    dev = ctx1.device
    p = params.to(dev).float().contiguous().clone()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    ctx1.closure_set_params(p)
    hist = []
    r = np.random.default_rng(1)
    for it in range(1, iters + 1):
        s = snaps[int(r.integers(len(snaps)))]
        ctx1.init_particles(s.pos, s.u, s.tau)
        ctx1.deposit()
        ctx1.solve_metric(0.0)
        ctx1.closure_forward(False)
        pred = ctx1.closure_gather()
        diff = pred - s.target
        loss = float((diff * diff).mean())
        g = ctx1.closure_backward(diff * (2.0 / diff.numel()))
        ctx1.closure_adam(p, m, v, g, it, lr)
        hist.append(loss)
        if log and (it % log_every == 0 or it == 1):
            log(f"closure train it {it}: loss {np.mean(hist[-log_every:]):.4e}")
    return p, hist


def evaluate(ctx1: PMContext, snaps, params: torch.Tensor):
    """(mean |target|^2, mean |pred - target|^2) over snapshots: plain 1x error vs error with the closure."""
    ctx1.closure_set_params(params)
    plain, corr = [], []
    for s in snaps:
        ctx1.init_particles(s.pos, s.u, s.tau)
        ctx1.deposit()
        ctx1.solve_metric(0.0)
        ctx1.closure_forward(False)
        pred = ctx1.closure_gather()
        plain.append(float((s.target * s.target).mean()))
        corr.append(float(((pred - s.target) ** 2).mean()))
    return float(np.mean(plain)), float(np.mean(corr))
