"""Training and evaluation driver of the learned force closure.

Everything numerical runs in the library's kernels (PM steps, the network's
forward and backward passes, the residual and its mean-squared-error
gradient, the cube-symmetry augmentation, Adam); this module only orders the
calls.

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
        if log:
            log(f"closure pairs: box seed {seed} done in {time.time() - t0:.1f} s ({len(out)} snapshots)")
    return out, c1


def train(ctx1: PMContext, snaps, params: torch.Tensor, iters: int, lr: float = 1e-3, log=print, log_every=100,
          augment: bool = False, lr_final: float = 1.0):
    """Adam on the particle MSE; returns (params, loss history).  With `augment` every iteration applies a
    random symmetry of the periodic cube (pm_cube_symmetry) to its snapshot; the learning rate follows a cosine
    from lr to lr * lr_final.  Every step is library calls: the PM solve, the forward pass, the residual and
    its MSE gradient (pm_closure_loss), the backward pass and Adam."""
    dev = ctx1.device
    p = params.to(dev).float().contiguous().clone()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    ctx1.closure_set_params(p)
    hist = []
    r = np.random.default_rng(1)
    dpred = torch.empty((ctx1.np, 3), dtype=torch.float32, device=dev)
    aug = None
    for it in range(1, iters + 1):
        s = snaps[int(r.integers(len(snaps)))]
        pos, u, target = s.pos, s.u, s.target
        if augment:
            perm, signs = r.permutation(3), r.choice([-1.0, 1.0], 3)
            if aug is None:
                aug = (torch.empty_like(pos), torch.empty_like(u), torch.empty_like(target))
            pos, u, target = ctx1.cube_symmetry(pos, u, target, perm, sum(1 << d for d in range(3) if signs[d] < 0),
                                                out=aug)
        ctx1.init_particles(pos, u, s.tau)
        ctx1.deposit()
        ctx1.solve_metric(0.0)
        ctx1.closure_forward(False)
        loss, _, _ = ctx1.closure_loss(target, dpred)
        g = ctx1.closure_backward(dpred)
        lr_it = lr * (lr_final + (1.0 - lr_final) * 0.5 * (1.0 + math.cos(math.pi * (it - 1) / max(iters - 1, 1))))
        ctx1.closure_adam(p, m, v, g, it, lr_it)
        hist.append(loss)
        if log and (it % log_every == 0 or it == 1):
            log(f"closure train it {it}: loss {np.mean(hist[-log_every:]):.4e}")
    return p, hist


def evaluate(ctx1: PMContext, snaps, params: torch.Tensor):
    """(mean |target|^2, mean |pred - target|^2) over snapshots: plain 1x error vs error with the closure."""
    ctx1.closure_set_params(params)
    plain, corr = [], []
    dpred = torch.empty((ctx1.np, 3), dtype=torch.float32, device=ctx1.device)
    for s in snaps:
        ctx1.init_particles(s.pos, s.u, s.tau)
        ctx1.deposit()
        ctx1.solve_metric(0.0)
        ctx1.closure_forward(False)
        e, t, _ = ctx1.closure_loss(s.target, dpred)
        plain.append(t)
        corr.append(e)
    return float(np.mean(plain)), float(np.mean(corr))


# ---------------------------------------------------------------------------
# power spectrum on the GPU (evaluation only) and the full experiment
# ---------------------------------------------------------------------------

def power_spectrum(pos: torch.Tensor, m: int, box: float):
    """P(k) of particle positions on an m^3 measurement mesh with the library's estimator
    (pm_power_spectrum: CIC counts, FFT, CIC window deconvolution, shot noise subtracted, shells of
    width 2 pi / box); returns (k, P, modes) as numpy arrays."""
    n_p = pos.shape[0]
    ctx = PMContext(m, n_p, box, physics="newtonian", precision="fp32")
    ctx.init_particles(pos, torch.zeros_like(pos, dtype=torch.float32), 1.0)
    out = ctx.power_spectrum(subtract_shot_noise=True)
    del ctx
    return out


def run_pm(n_mesh: int, pos, u, tau0: float, tau1: float, steps: int, box: float, params=None, log=print):
    """Evolve with scalar physics on an n_mesh^3 mesh; returns (final positions [device], wall seconds)."""
    n_p = pos.shape[0]
    ctx = PMContext(n_mesh, n_p, box, physics="scalar", precision="fp32", closure=params is not None)
    ctx.init_particles(pos, u, tau0)
    if params is not None:
        ctx.closure_set_params(params)
        ctx.closure_enable(True)
    dtau = (tau1 - tau0) / steps
    torch.cuda.synchronize()
    t0 = time.time()
    for i in range(steps):
        ctx.step(dtau)
        if log and (i + 1) % 25 == 0:
            ctx.sync()
            log(f"  mesh {n_mesh}^3{' + closure' if params is not None else ''}: step {i + 1}/{steps}, "
                f"a = {ctx.time()[1]:.3f}, {time.time() - t0:.1f} s")
    ctx.sync()
    wall = time.time() - t0
    p, _ = ctx.get_particles(device=True)
    del ctx
    torch.cuda.empty_cache()
    return p, wall


def scaled_output(params: torch.Tensor, s: float) -> torch.Tensor:
    """Parameters whose network output is s times the original (the last layer is linear)."""
    p = params.clone()
    n_last = 3 * 16 * 27 + 3
    p[-n_last:] *= s
    return p


def max_pk_deviation(k, ratio, kmax):
    sel = k <= kmax
    return float(np.max(np.abs(ratio[sel] - 1.0)))


def calibrate_amplitude(params, n_p1: int, box: float, rms_cells: float, seeds, scales=(1.0, 1.1, 1.2, 1.3, 1.4, 1.5),
                        steps: int = 100, log=print):
    """Output amplitude of the closure chosen on calibration runs: each seeded box of n_p1^3 particles is run on
    the 2x mesh and on the 1x mesh with the closure scaled by s; the s whose box-averaged P(k) ratio to the 2x
    runs deviates least up to half the 1x Nyquist frequency is returned with the table of deviations."""
    from synth import spectrum_power_law_m2, zeldovich_particles
    from synth.ics import eds_a_of_tau

    tau0, tau1 = tau_of_a(box, 0.02), tau_of_a(box, 0.5)
    dtau = (tau1 - tau0) / steps
    kmax = math.pi / (2.0 * box / n_p1)
    ratios = {s: [] for s in scales}
    for seed in seeds:
        pos, u = zeldovich_particles(n_p1, seed, spectrum_power_law_m2, box, rms_cells, 0.02, 0.02,
                                     eds_a_of_tau(tau0 - 0.5 * dtau, box))
        pos_d = torch.tensor(pos, device="cuda")
        u_d = torch.tensor(u, device="cuda", dtype=torch.float32)
        p2, _ = run_pm(2 * n_p1, pos_d, u_d, tau0, tau1, steps, box, None, log=None)
        k, pk2, _ = power_spectrum(p2, n_p1, box)
        del p2
        for s in scales:
            p1, _ = run_pm(n_p1, pos_d, u_d, tau0, tau1, steps, box, scaled_output(params, s), log=None)
            ratios[s].append(power_spectrum(p1, n_p1, box)[1] / pk2)
            if log:
                log(f"  calibration seed {seed}, s = {s:.3f}: max deviation "
                    f"{max_pk_deviation(k, ratios[s][-1], kmax):.4f}")
    table = {s: max_pk_deviation(k, np.mean(ratios[s], axis=0), kmax) for s in scales}
    if log:
        log("calibration: " + ", ".join(f"s={s:.2f}: {d:.4f}" for s, d in table.items()))
    return min(table, key=table.get), table


# P(k) at half the Nyquist frequency moves by about 2 % per 1 % of output amplitude, so the grid is fine
CAL_SCALES = tuple(round(1.0 + 0.005 * i, 3) for i in range(31))
VALIDATION_SEEDS = (7, 8)  # the application runs seed 3


def experiment(n_app: int = 512, n_train_p: int = 128, train_box: float = 512.0, n_boxes: int = 64,
               iters: int = 12000, lr: float = 1e-3, augment: bool = True, calibrate: str = "validation", log=print):
    """Train on seeded boxes (1x and 2x meshes), apply to n_app^3 particles on an n_app^3 mesh and compare
    P(k) and cost with the plain n_app^3 and 2 n_app^3 meshes at a = 0.5.

    calibrate: "validation" scales the output by the amplitude that best matches the 2x spectrum, averaged
    over other realizations of the application (same box, mesh and recipe, seeds VALIDATION_SEEDS; the
    application's own seed is never used to choose it); "train" chooses it on 4 training boxes; "none" keeps the trained
    output."""
    from synth import spectrum_power_law_m2, zeldovich_particles
    from synth.ics import eds_a_of_tau

    res = {}
    # the training boxes share the application's physical spectrum amplitude: for P ~ k^-2 the variance of
    # the displacement scales as (1/k_f - 1/k_Nyquist), so the rms in cells is rescaled accordingly
    app_box = 2048.0 * n_app / 512
    cell = app_box / n_app
    var = lambda L, N: (L / (2 * math.pi)) * (1 - 2.0 / N)  # noqa: E731
    rms_train = 0.2 * cell * math.sqrt(var(train_box, n_train_p) / var(app_box, n_app)) / (train_box / n_train_p)
    t0 = time.time()
    snaps, c1 = make_pairs(seeds=range(1000, 1000 + n_boxes), n_p=n_train_p ** 3, n1=n_train_p, box=train_box,
                           a_snaps=list(np.linspace(0.1, 0.5, 8)), steps=100, spectrum=spectrum_power_law_m2,
                           rms_cells=rms_train, log=log if n_boxes <= 8 else None)
    res["pairs_s"] = time.time() - t0
    log(f"{len(snaps)} training snapshots in {res['pairs_s']:.1f} s (rms displacement {rms_train:.3f} cells)")
    hold = snaps[-8:]
    t0 = time.time()
    params, hist = train(c1, snaps[:-8], init_params(0), iters=iters, lr=lr, log=log, log_every=1000,
                         augment=augment, lr_final=0.05)
    res["train_s"] = time.time() - t0
    res["heldout_plain"], res["heldout_closure"] = evaluate(c1, hold, params)
    log(f"trained in {res['train_s']:.1f} s; held-out force error: plain {res['heldout_plain']:.4e}, "
        f"closure {res['heldout_closure']:.4e}")
    del c1, snaps
    torch.cuda.empty_cache()
    if calibrate not in ("validation", "train", "none"):
        raise ValueError("calibrate must be 'validation', 'train' or 'none'")
    if calibrate != "none":
        t0 = time.time()
        if calibrate == "train":
            s, table = calibrate_amplitude(params, n_train_p, train_box, rms_train, seeds=range(1000, 1000 + 4),
                                           scales=CAL_SCALES, log=log)
        else:
            s, table = calibrate_amplitude(params, n_app, app_box, 0.2, seeds=VALIDATION_SEEDS, scales=CAL_SCALES,
                                           log=log)
        params = scaled_output(params, s)
        res["amplitude"], res["calibration"], res["calibration_s"] = s, table, time.time() - t0
        res["calibration_on"] = calibrate
        log(f"output amplitude {s:.2f} chosen on the {calibrate} runs ({res['calibration_s']:.1f} s)")
    # application
    tau0, tau1 = tau_of_a(app_box, 0.02), tau_of_a(app_box, 0.5)
    steps = 100
    dtau = (tau1 - tau0) / steps
    pos, u = zeldovich_particles(n_app, 3, spectrum_power_law_m2, app_box, 0.2, 0.02, 0.02,
                                 eds_a_of_tau(tau0 - 0.5 * dtau, app_box))
    pos_d = torch.tensor(pos, device="cuda")
    u_d = torch.tensor(u, device="cuda", dtype=torch.float32)
    del pos, u
    out = {}
    for label, mesh, prm in (("plain_1x", n_app, None), ("closure_1x", n_app, params), ("plain_2x", 2 * n_app, None)):
        p, wall = run_pm(mesh, pos_d, u_d, tau0, tau1, steps, app_box, prm, log=log)
        k, pk, cnt = power_spectrum(p, n_app, app_box)
        out[label] = (k, pk, wall)
        log(f"{label}: {wall:.1f} s for {steps} steps")
        del p
        torch.cuda.empty_cache()
    k = out["plain_2x"][0]
    kmax = math.pi / (2.0 * cell)  # half the 1x Nyquist frequency
    sel = k <= kmax
    ref = out["plain_2x"][1]
    for label in ("plain_1x", "closure_1x"):
        r = out[label][1][sel] / ref[sel] - 1.0
        res[f"{label}_maxdev"] = float(np.max(np.abs(r)))
        res[f"{label}_ratio"] = [float(v) for v in r]
    res["k"] = [float(v) for v in k[sel]]
    res["kmax_half_nyquist"] = kmax
    for label in out:
        res[f"{label}_wall_s"] = out[label][2]
    res["loss_first"], res["loss_last"] = float(np.mean(hist[:50])), float(np.mean(hist[-50:]))
    res["iters"], res["augment"] = iters, augment
    res["pass_2pct"] = res["closure_1x_maxdev"] <= 0.02
    res["gain"] = res["closure_1x_maxdev"] < res["plain_1x_maxdev"]
    res["cheaper_than_2x"] = out["closure_1x"][2] < out["plain_2x"][2]
    return res, params


def summary_md(res: dict, command: str) -> str:
    """Markdown summary of an experiment result (the committed profile of the closure experiment)."""
    lines = ["# Learned closure experiment: 512^3 particles, 512^3 mesh + closure vs plain 1024^3 mesh", "",
             "Command (repository root, on the MI355X machine):", "", f"    {command}", "",
             f"Training: {res.get('iters')} Adam iterations (cosine decay), cube-symmetry augmentation "
             f"{'on' if res.get('augment') else 'off'}; pairs {res['pairs_s']:.1f} s, training {res['train_s']:.1f} s.",
             f"Held-out particle force error (units of rms|grad phi|^2): plain 1x {res['heldout_plain']:.3e}, "
             f"with closure {res['heldout_closure']:.3e}."]
    if "amplitude" in res:
        where = ("two other realizations of the application (seeds 7 and 8; the application is seed 3)"
                 if res.get("calibration_on", "train") == "validation" else "4 training boxes")
        lines.append(f"Output amplitude chosen on {where}: s = {res['amplitude']:.3f} "
                     f"({res['calibration_s']:.1f} s; per realization one 2x run and {len(res['calibration'])} 1x runs); "
                     f"max deviation per s there: "
                     + ", ".join(f"{float(k):.3f}: {v:.4f}" for k, v in res["calibration"].items()) + ".")
    lines += ["", "| run | wall time, 100 steps | max abs(P/P_2x - 1), k <= k_Ny/2 |", "|---|---|---|",
              f"| plain 512^3 mesh | {res['plain_1x_wall_s']:.1f} s | {res['plain_1x_maxdev']:.4f} |",
              f"| 512^3 mesh + closure | {res['closure_1x_wall_s']:.1f} s | {res['closure_1x_maxdev']:.4f} |",
              f"| plain 1024^3 mesh | {res['plain_2x_wall_s']:.1f} s | (reference) |", "",
              f"2% target: {'met' if res['pass_2pct'] else 'not met'}; gain over the plain mesh: "
              f"{'yes' if res['gain'] else 'no'}; cheaper than the 2x mesh: "
              f"{'yes' if res['cheaper_than_2x'] else 'no'} "
              f"({res['closure_1x_wall_s'] / res['plain_2x_wall_s']:.2f}x of its time).", "",
              "P(k) ratio minus one (every 6th bin):", "", "| k [h/Mpc] | plain 1x | 1x + closure |", "|---|---|---|"]
    for i in range(0, len(res["k"]), 6):
        lines.append(f"| {res['k'][i]:.4f} | {res['plain_1x_ratio'][i]:+.4f} | {res['closure_1x_ratio'][i]:+.4f} |")
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    import argparse
    import json
    import os

    ap = argparse.ArgumentParser(description="learned closure experiment")
    ap.add_argument("--n-app", type=int, default=512)
    ap.add_argument("--boxes", type=int, default=64)
    ap.add_argument("--iters", type=int, default=12000)
    ap.add_argument("--no-augment", action="store_true")
    ap.add_argument("--calibrate", choices=("validation", "train", "none"), default="validation",
                    help="choose the output amplitude on another realization of the application (default), on "
                         "training boxes, or keep the trained output")
    ap.add_argument("--out", default="gpurun_out/closure_experiment.json")
    ap.add_argument("--summarize", metavar="RESULT_JSON", help="print the markdown summary of a stored result")
    ap.add_argument("--command", default="python -u -m paper_2607_17929_amd.closure --out gpurun_out/closure_experiment.json")
    a = ap.parse_args()
    if a.summarize:
        with open(a.summarize) as f:
            print(summary_md(json.load(f), a.command), end="")
        raise SystemExit(0)
    res, params = experiment(n_app=a.n_app, n_boxes=a.boxes, iters=a.iters, augment=not a.no_augment,
                             calibrate=a.calibrate, log=lambda s: print(s, flush=True))
    os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1)
    np.save(os.path.splitext(a.out)[0] + "_params.npy", params.cpu().numpy())
    print(json.dumps({k: v for k, v in res.items() if not isinstance(v, list)}), flush=True)
