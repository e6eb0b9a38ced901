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
               a0: float = 0.02, a1: float = 0.5, physics: str = "scalar", log=print, closure_params=None, c1=None):
    """Evolve each box and collect (particles, normalised force difference) snapshots.

    Without closure_params the boxes are evolved on the 2x mesh; with them, on the 1x mesh with the closure
    switched on (on-policy data: the particle states the corrected 1x run actually visits, each labelled with
    the 2x - 1x force difference on those same particles).  c1 reuses a training context."""
    from synth import zeldovich_particles
    from synth.ics import eds_a_of_tau

    n2 = 2 * n1
    tau0, tau1 = tau_of_a(box, a0), tau_of_a(box, a1)
    dtau = (tau1 - tau0) / steps
    snap_taus = sorted(tau_of_a(box, a) for a in a_snaps)
    if closure_params is None:
        ce = PMContext(n2, n_p, box, physics=physics, precision="fp32")
    else:
        ce = PMContext(n1, n_p, box, physics=physics, precision="fp32", closure=True)
        ce.closure_set_params(closure_params)
        ce.closure_enable(True)
    c2s = PMContext(n2, n_p, box, physics=physics, precision="fp32")
    if c1 is None:
        c1 = PMContext(n1, n_p, box, physics=physics, precision="fp32", closure=True)
    out = []
    for seed in seeds:
        t0 = time.time()
        pos, u = zeldovich_particles(round(n_p ** (1 / 3)), seed, spectrum, box, rms_cells, 0.02, a0,
                                     eds_a_of_tau(tau0 - 0.5 * dtau, box))
        ce.init_particles(pos, u.astype(np.float32), tau0)
        k = 0
        for i in range(steps):
            ce.step(dtau)
            tau = ce.time()[0]
            while k < len(snap_taus) and tau >= snap_taus[k] - 1e-9 * tau:
                p, uu = ce.get_particles(device=True)
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
# realizations of the application configuration the closure is judged on: seed 3 is the application run,
# seeds 7 and 8 are two more realizations of the same configuration; none is used for training or tuning
EVAL_SEEDS = (3, 7, 8)


def _app_setup(n_app: int):
    app_box = 2048.0 * n_app / 512
    tau0, tau1 = tau_of_a(app_box, 0.02), tau_of_a(app_box, 0.5)
    return app_box, tau0, tau1, 100


_APP_ICS = {}


def _app_particles(n_app: int, seed: int, rms: float = 0.2):
    """Initial particles of one realization (n_app^3 particles, box 4 n_app Mpc/h, rms displacement `rms` cells at
    a = 0.02; 0.2 is the application configuration), kept on the device."""
    from synth import spectrum_power_law_m2, zeldovich_particles
    from synth.ics import eds_a_of_tau
    if (n_app, seed, rms) not in _APP_ICS:
        app_box, tau0, tau1, steps = _app_setup(n_app)
        dtau = (tau1 - tau0) / steps
        pos, u = zeldovich_particles(n_app, seed, spectrum_power_law_m2, app_box, rms, 0.02, 0.02,
                                     eds_a_of_tau(tau0 - 0.5 * dtau, app_box))
        _APP_ICS[(n_app, seed, rms)] = (torch.tensor(pos, device="cuda"),
                                        torch.tensor(u, device="cuda", dtype=torch.float32))
    return _APP_ICS[(n_app, seed, rms)]


def reference_runs(n_app: int, seeds, log=print, rms: float = 0.2):
    """Per realization: P(k) of the plain 2x-mesh run (the reference) and of the plain 1x run, with wall times."""
    app_box, tau0, tau1, steps = _app_setup(n_app)
    kmax = math.pi / (2.0 * app_box / n_app)  # half the 1x Nyquist frequency
    out = {}
    for seed in seeds:
        pos_d, u_d = _app_particles(n_app, seed, rms)
        p2, w2 = run_pm(2 * n_app, pos_d, u_d, tau0, tau1, steps, app_box, None, log=None)
        k, pk2, _ = power_spectrum(p2, n_app, app_box)
        del p2
        p1, w1 = run_pm(n_app, pos_d, u_d, tau0, tau1, steps, app_box, None, log=None)
        pk1 = power_spectrum(p1, n_app, app_box)[1]
        del p1
        torch.cuda.empty_cache()
        sel = k <= kmax
        out[seed] = {"k": k, "pk2": pk2, "sel": sel, "plain_2x_wall_s": w2, "plain_1x_wall_s": w1, "rms": rms,
                     "plain_1x_ratio": pk1[sel] / pk2[sel] - 1.0}
        out[seed]["plain_1x_maxdev"] = float(np.max(np.abs(out[seed]["plain_1x_ratio"])))
        if log:
            log(f"reference seed {seed}: 2x run {w2:.1f} s, plain 1x run {w1:.1f} s, plain 1x max deviation "
                f"{out[seed]['plain_1x_maxdev']:.4f}")
    return out


def closure_runs(params, n_app: int, refs, log=print):
    """Per realization: the 1x run with the closure, its P(k) ratio to the 2x run (k up to half the 1x Nyquist
    frequency), its maximum deviation and its wall time."""
    app_box, tau0, tau1, steps = _app_setup(n_app)
    out = {}
    for seed, ref in refs.items():
        pos_d, u_d = _app_particles(n_app, seed, ref["rms"])
        p, wall = run_pm(n_app, pos_d, u_d, tau0, tau1, steps, app_box, params, log=None)
        pk = power_spectrum(p, n_app, app_box)[1]
        del p
        torch.cuda.empty_cache()
        ratio = pk[ref["sel"]] / ref["pk2"][ref["sel"]] - 1.0
        out[seed] = {"maxdev": float(np.max(np.abs(ratio))), "wall_s": wall, "ratio": [float(v) for v in ratio]}
        if log:
            log(f"  closure on seed {seed}: max deviation {out[seed]['maxdev']:.4f} ({wall:.1f} s)")
    return out


def experiment(n_app: int = 512, n_train_p: int = 128, train_box: float = 512.0, n_boxes: int = 64,
               iters: int = 12000, lr: float = 1e-3, augment: bool = True, phases: int = 2, phase_boxes: int = 32,
               phase_iters: int = 6000, calibrate: str = "none", train_rms: float | None = None,
               eval_seeds=None, probe=(), log=print):
    """Train on seeded boxes (1x and 2x meshes), apply to n_app^3 particles on an n_app^3 mesh and compare P(k)
    and cost with the plain n_app^3 and 2 n_app^3 meshes at a = 0.5, on the realizations EVAL_SEEDS.

    Phase 0 trains on snapshots of 2x-mesh runs.  Each further phase (on-policy data) evolves phase_boxes new
    training boxes on the 1x mesh with the current closure, labels their snapshots with the 2x - 1x force
    difference on the same particles, adds them to the training set and continues training for phase_iters
    iterations.  The closure's output is used as trained (calibrate "none"), or scaled by the amplitude whose
    P(k) ratio matches best on 4 training boxes (calibrate "train"); no 2x run of the application
    configuration is ever used to choose anything.

    train_rms: rms displacement of the training boxes at a = 0.02 in cells; None gives them the application's
    physical spectrum amplitude (for P ~ k^-2 about half the application's displacement in cells).
    probe: (n_app, rms) cases on which the final network is also evaluated (seeds 3, 7, 8, 9, 10; boxes of
    4 n_app Mpc/h, i.e. the same 4 Mpc/h cell), to show how its error depends on box size and amplitude."""
    from synth import spectrum_power_law_m2

    if calibrate not in ("train", "none"):
        raise ValueError("calibrate must be 'train' or 'none'")
    seeds_eval = tuple(eval_seeds) if eval_seeds else EVAL_SEEDS
    res = {"eval_seeds": list(seeds_eval), "iters": iters, "augment": augment, "calibrate": calibrate}
    # the training boxes share the application's physical spectrum amplitude: for P ~ k^-2 the variance of
    # the displacement scales as (1/k_f - 1/k_Nyquist), so the rms in cells is rescaled accordingly
    app_box = 2048.0 * n_app / 512
    cell = app_box / n_app
    var = lambda L, N: (L / (2 * math.pi)) * (1 - 2.0 / N)  # noqa: E731
    rms_train = 0.2 * cell * math.sqrt(var(train_box, n_train_p) / var(app_box, n_app)) / (train_box / n_train_p)
    if train_rms is not None:
        rms_train = train_rms
    res["train_rms_cells"] = rms_train
    a_snaps = list(np.linspace(0.1, 0.5, 8))
    kw = dict(n_p=n_train_p ** 3, n1=n_train_p, box=train_box, a_snaps=a_snaps, steps=100,
              spectrum=spectrum_power_law_m2, rms_cells=rms_train)
    t0 = time.time()
    refs = reference_runs(n_app, seeds_eval, log=log)
    res["reference_s"] = time.time() - t0
    res["k"] = [float(v) for v in refs[seeds_eval[0]]["k"][refs[seeds_eval[0]]["sel"]]]
    res["kmax_half_nyquist"] = math.pi / (2.0 * cell)
    res["ref"] = {str(sd): {"plain_1x_maxdev": r["plain_1x_maxdev"], "plain_1x_wall_s": r["plain_1x_wall_s"],
                            "plain_2x_wall_s": r["plain_2x_wall_s"],
                            "plain_1x_ratio": [float(v) for v in r["plain_1x_ratio"]]} for sd, r in refs.items()}
    t0 = time.time()
    snaps, c1 = make_pairs(seeds=range(1000, 1000 + n_boxes), log=None, **kw)
    hold = snaps[-8:]
    train_set = snaps[:-8]
    res["phases"] = []
    params = init_params(0)
    cost = time.time() - t0
    for rnd in range(phases + 1):
        t0 = time.time()
        if rnd > 0:
            seeds = range(2000 + 1000 * rnd, 2000 + 1000 * rnd + phase_boxes)
            new = make_pairs(seeds=seeds, log=None, closure_params=params, c1=c1, **kw)[0]
            hold_new, new = new[-8:], new[:-8]
            hold = hold + hold_new
            train_set = train_set + new
        pairs_s = time.time() - t0 + (cost if rnd == 0 else 0.0)
        t0 = time.time()
        params, hist = train(c1, train_set, params, iters=iters if rnd == 0 else phase_iters,
                             lr=lr, log=None, augment=augment, lr_final=0.05)
        train_s = time.time() - t0
        plain, corr = evaluate(c1, hold, params)
        r = {"phase": rnd, "snapshots": len(train_set), "pairs_s": pairs_s, "train_s": train_s,
             "heldout_plain": plain, "heldout_closure": corr, "loss_first": float(np.mean(hist[:50])),
             "loss_last": float(np.mean(hist[-50:]))}
        log(f"phase {rnd}: {len(train_set)} snapshots, pairs {pairs_s:.1f} s, training {train_s:.1f} s; held-out "
            f"force error plain {plain:.4e}, closure {corr:.4e}")
        r["eval"] = {str(sd): v for sd, v in closure_runs(params, n_app, refs, log=log).items()}
        r["maxdev"] = max(v["maxdev"] for v in r["eval"].values())
        res["phases"].append(r)
    if calibrate == "train":
        t0 = time.time()
        sc, table = calibrate_amplitude(params, n_train_p, train_box, rms_train, seeds=range(1000, 1000 + 4),
                                        scales=CAL_SCALES, log=log)
        params = scaled_output(params, sc)
        res["amplitude"], res["calibration"], res["calibration_s"] = sc, table, time.time() - t0
        res["calibrated_eval"] = {str(sd): v for sd, v in closure_runs(params, n_app, refs, log=log).items()}
        log(f"output amplitude {sc:.3f} chosen on training boxes ({res['calibration_s']:.1f} s)")
    res["probe"] = []
    for n_p, rms in probe:
        t0 = time.time()
        pr = reference_runs(n_p, (3, 7, 8, 9, 10), log=None, rms=rms)
        ev = closure_runs(params, n_p, pr, log=None)
        res["probe"].append({"n_app": n_p, "box": 4.0 * n_p, "rms_cells": rms,
                             "plain_1x_maxdev": [pr[sd]["plain_1x_maxdev"] for sd in pr],
                             "closure_maxdev": [ev[sd]["maxdev"] for sd in ev]})
        log(f"probe {n_p}^3 (box {4 * n_p} Mpc/h, rms {rms:.4f} cells): closure max deviation "
            + ", ".join(f"{ev[sd]['maxdev']:.4f}" for sd in ev) + f" ({time.time() - t0:.1f} s)")
    final = res["phases"][-1] if calibrate == "none" else {"eval": res["calibrated_eval"]}
    ev = final["eval"]
    res["final_maxdev"] = {sd: v["maxdev"] for sd, v in ev.items()}
    res["pass_2pct_all"] = all(v["maxdev"] <= 0.02 for v in ev.values())
    res["gain_all"] = all(ev[str(sd)]["maxdev"] < refs[sd]["plain_1x_maxdev"] for sd in seeds_eval)
    res["closure_wall_s"] = float(np.mean([v["wall_s"] for v in ev.values()]))
    res["plain_2x_wall_s"] = float(np.mean([refs[sd]["plain_2x_wall_s"] for sd in seeds_eval]))
    res["plain_1x_wall_s"] = float(np.mean([refs[sd]["plain_1x_wall_s"] for sd in seeds_eval]))
    res["training_cost_s"] = sum(r["pairs_s"] + r["train_s"] for r in res["phases"]) + res.get("calibration_s", 0.0)
    return res, params


def summary_md(res: dict, command: str) -> str:
    """Markdown summary of an experiment result (the committed profile of the closure experiment)."""
    seeds = [str(s) for s in res["eval_seeds"]]
    lines = ["# Learned closure experiment: 512^3 particles, 512^3 mesh + closure vs plain 1024^3 mesh", "",
             "Command (repository root, on the MI355X machine):", "", f"    {command}", "",
             f"Three realizations of the application configuration (seeds {', '.join(seeds)}; seed {seeds[0]} is the "
             "application run), none used for training or for choosing anything.  Phase 0 trains on snapshots of "
             "2x-mesh runs of 512 Mpc/h training boxes; each later phase adds snapshots of training boxes evolved on "
             "the 1x mesh with the current closure (on-policy data), labelled with the 2x - 1x force on the same "
             f"particles, and trains on.  Cube-symmetry augmentation {'on' if res.get('augment') else 'off'}; "
             f"training boxes at rms displacement {res.get('train_rms_cells', 0.0994):.4f} cells at a = 0.02 "
             "(the application: 0.2 cells in a 2048 Mpc/h box).", ""]
    if "amplitude" in res:
        lines.append(f"Output amplitude chosen on 4 training boxes: s = {res['amplitude']:.3f} "
                     f"({res['calibration_s']:.1f} s).")
    else:
        lines.append("Output used as trained (s = 1): no amplitude tuning.")
    lines += ["", "| phase | training snapshots | pairs + training | held-out force error, plain -> closure | "
              + " | ".join(f"max dev. seed {s}" for s in seeds) + " |",
              "|---|---|---|---|" + "---|" * len(seeds)]
    for r in res["phases"]:
        lines.append(f"| {r['phase']} | {r['snapshots']} | {r['pairs_s'] + r['train_s']:.1f} s | "
                     f"{r['heldout_plain']:.3e} -> {r['heldout_closure']:.3e} | "
                     + " | ".join(f"{r['eval'][s]['maxdev']:.4f}" for s in seeds) + " |")
    if "calibrated_eval" in res:
        lines.append(f"| s = {res['amplitude']:.3f} | | | | "
                     + " | ".join(f"{res['calibrated_eval'][s]['maxdev']:.4f}" for s in seeds) + " |")
    lines += ["", "| run | wall time, 100 steps (mean) | max abs(P/P_2x - 1), k <= k_Ny/2, per realization |",
              "|---|---|---|",
              f"| plain 512^3 mesh | {res['plain_1x_wall_s']:.1f} s | "
              + ", ".join(f"{res['ref'][s]['plain_1x_maxdev']:.4f}" for s in seeds) + " |",
              f"| 512^3 mesh + closure | {res['closure_wall_s']:.1f} s | "
              + ", ".join(f"{res['final_maxdev'][s]:.4f}" for s in seeds) + " |",
              f"| plain 1024^3 mesh | {res['plain_2x_wall_s']:.1f} s | (reference) |", "",
              f"2% target on every realization: {'met' if res['pass_2pct_all'] else 'not met'}; gain over the plain "
              f"mesh on every realization: {'yes' if res['gain_all'] else 'no'}.  Closure run "
              f"{res['closure_wall_s'] / res['plain_2x_wall_s']:.2f}x the 2x run's time; one-off training cost "
              f"{res['training_cost_s']:.1f} s (pairs, training{', calibration' if 'amplitude' in res else ''}).", "",
              ]
    if res.get("probe"):
        lines += ["The final network on other boxes with the same 4 Mpc/h cell (seeds 3, 7, 8, 9, 10; s = 1):", "",
                  "| particles = mesh | box | rms displacement at a = 0.02 | plain 1x max dev. | closure max dev. |",
                  "|---|---|---|---|---|"]
        for pr in res["probe"]:
            lines.append(f"| {pr['n_app']}^3 | {pr['box']:.0f} Mpc/h | {pr['rms_cells']:.4f} cells | "
                         + ", ".join(f"{v:.3f}" for v in pr["plain_1x_maxdev"]) + " | "
                         + ", ".join(f"{v:.4f}" for v in pr["closure_maxdev"]) + " |")
        lines.append("")
    lines += [f"P(k) ratio minus one, seed {seeds[0]} (every 6th bin):", "",
              "| k [h/Mpc] | plain 1x | 1x + closure |", "|---|---|---|"]
    final = res["phases"][-1]["eval"][seeds[0]] if "calibrated_eval" not in res else res["calibrated_eval"][seeds[0]]
    for i in range(0, len(res["k"]), 6):
        lines.append(f"| {res['k'][i]:.4f} | {res['ref'][seeds[0]]['plain_1x_ratio'][i]:+.4f} | "
                     f"{final['ratio'][i]:+.4f} |")
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    import argparse
    import json
    import os

    ap = argparse.ArgumentParser(description="learned closure experiment")
    ap.add_argument("--n-app", type=int, default=512)
    ap.add_argument("--boxes", type=int, default=64)
    ap.add_argument("--iters", type=int, default=12000)
    ap.add_argument("--phases", type=int, default=2, help="on-policy phases after the first training")
    ap.add_argument("--phase-boxes", type=int, default=32)
    ap.add_argument("--phase-iters", type=int, default=6000)
    ap.add_argument("--no-augment", action="store_true")
    ap.add_argument("--train-rms", type=float, default=None,
                    help="rms displacement of the training boxes at a = 0.02 in cells (default: the application's "
                         "physical amplitude)")
    ap.add_argument("--eval-seeds", default=None, help="comma-separated realizations to evaluate on")
    ap.add_argument("--probe", default="128:0.0994,128:0.2,256:0.1411,256:0.2",
                    help="n_app:rms cases the final network is also evaluated on ('' for none)")
    ap.add_argument("--calibrate", choices=("train", "none"), default="none",
                    help="keep the trained output (default) or scale it by the amplitude chosen on training boxes")
    ap.add_argument("--out", default="closure_experiment.json")
    ap.add_argument("--summarize", metavar="RESULT_JSON", help="print the markdown summary of a stored result")
    ap.add_argument("--command", default="python -u -m paper_2607_17929_amd.closure",
                    help="the command line recorded in the summary")
    a = ap.parse_args()
    if a.summarize:
        with open(a.summarize) as f:
            print(summary_md(json.load(f), a.command), end="")
        raise SystemExit(0)
    res, params = experiment(n_app=a.n_app, n_boxes=a.boxes, iters=a.iters, augment=not a.no_augment,
                             phases=a.phases, phase_boxes=a.phase_boxes, phase_iters=a.phase_iters,
                             calibrate=a.calibrate, train_rms=a.train_rms,
                             eval_seeds=[int(v) for v in a.eval_seeds.split(",")] if a.eval_seeds else None,
                             probe=[(int(c.split(":")[0]), float(c.split(":")[1])) for c in a.probe.split(",") if c],
                             log=lambda s: print(s, flush=True))
    os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1)
    np.save(os.path.splitext(a.out)[0] + "_params.npy", params.cpu().numpy())
    print(json.dumps({k: v for k, v in res.items() if not isinstance(v, (list, dict))}), flush=True)
