#!/usr/bin/env python
"""Particle updates per second of one relativistic PM step at 512^3 on one MI355X.

Workload (clustered mixed-precision run): 512^3 particles on a 512^3 mesh in a
2048 Mpc/h box; Zel'dovich initial conditions from a seeded Gaussian field with
P(k) ~ k^-2 cut at the Nyquist wavenumber (rms displacement 0.2 cells at
a = 0.02), evolved by the FP64 GPU path in 100 uniform-tau steps to a = 0.5 so
that the particles are clustered.  From that snapshot the FP32 path (FP32
fields, FFTs, deposit and momenta; FP64 positions and homogeneous mode) and the
FP64 path are each timed over K steps of dtau = 0.01 tau with full
scalar + vector + tensor physics.  One step = deposit + metric solve (15 FFTs
and the Fourier-space solves) + gather/kick/drift + re-sort.

Prints one JSON line.  `value` is the FP32 path's particle updates per second
(B from the momentum constraint); `fp32_parabolic_b` is the same step with B
integrated from the vector part of the space-space equation (12 FFTs per step,
the paper's own benchmark configuration) and `fp64` the all-FP64 path.
`copy_ceiling` is the library's own copy kernel measured in the same run (the runtime's device copy
beside it);
`closure_vs_2x_mesh` repeats the committed closure experiment's figures.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stage_bytes(n: int, n_p: int, rs: int) -> dict:
    """Algorithmic bytes of one launch of each stage's kernel (each unique input read and output written once)."""
    F = n ** 3 * rs                      # one real field
    S = n * n * (n // 2 + 1) * 2 * rs    # one half spectrum
    P = 24 + 3 * rs                      # position + momentum of one particle
    return {
        "deposit": n_p * P + 10 * F,
        "fft_x_fwd": 13 * F + 10 * S,
        "fft_y_fwd": 2 * 10 * S,
        "kspace": 10 * S + 5 * S + 8 * S,  # sources in, solutions out, tensor state in and out
        "fft_y_inv": 2 * 5 * S,
        "fft_x_inv": 5 * S + 7 * F,  # 5 spectra in, 5 fields out; phi_{n-1} in and the increment out
        "kick_drift": n_p * (2 * P + 4) + 5 * F,                  # state in and out, rank out, 5 fields in
        "sort": 16 * n ** 3 + n_p * (4 + 2 * (P + 4)),           # counts/offsets; rank, state and id in and out
    }


LAUNCHES: dict = {}  # stages that run as several launches of one kernel (none)


def measured_traffic(n: int, stage: str):
    """HBM bytes per launch of an FP32 stage from the committed counter summary, or None when there is
    none for this mesh or the stage's kernel sources have changed since it was measured."""
    from paper_2607_17929_amd import profsum
    t = profsum.load_traffic(os.path.join(ROOT, "profiles", f"pm_step_{n}_clustered_traffic.md"))
    if not t or t.get("n") != n:
        return None
    e = t["stages"].get(f"fp32:{stage}")
    if not e or e["source_sha256"] != profsum.source_hash(stage):
        return None
    return e["traffic_bytes_per_launch"]


def closure_result():
    """The learned closure's figures from the committed experiment summary (the experiment trains a network
    and runs 100-step simulations of several realizations, too long for the bench; its command is in the
    summary): the largest P(k) deviation over the realizations at s = 1, and the cost against the 2x run."""
    import re
    path = os.path.join(ROOT, "profiles", "closure_experiment_512.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    row = lambda name: re.search(r"\| " + name + r" \| ([0-9.]+) s \| ([0-9., ]+|\(reference\)) \|", text)  # noqa: E731
    plain, corr, ref = row(r"plain 512\^3 mesh"), row(r"512\^3 mesh \+ closure"), row(r"plain 1024\^3 mesh")
    if not (plain and corr and ref):
        return None
    devs = [float(v) for v in corr.group(2).split(",")]
    return {"max_pk_deviation_to_half_nyquist": max(devs), "per_realization": devs,
            "plain_1x_deviation": max(float(v) for v in plain.group(2).split(",")),
            "cost_vs_2x": round(float(corr.group(1)) / float(ref.group(1)), 3), "amplitude_gain": 1.0,
            "target": 0.02, "source": "profiles/closure_experiment_512.md (not measured by this run)"}


def run_gpu(args):
    import numpy as np
    import torch

    from paper_2607_17929_amd import PMContext, tau_of_a
    from paper_2607_17929_amd.pm import copy_probe
    from synth import spectrum_power_law_m2, zeldovich_particles
    from synth.ics import eds_a_of_tau

    n = args.n
    box = 2048.0 * n / 512
    n_p = n ** 3
    a0, a1 = 0.02, 0.5
    tau0, tau1 = tau_of_a(box, a0), tau_of_a(box, a1)
    dtau_ev = (tau1 - tau0) / args.evolve_steps
    t0 = time.time()
    pos, u = zeldovich_particles(n, 3, spectrum_power_law_m2, box, 0.2, 0.02, a0,
                                 eds_a_of_tau(tau0 - 0.5 * dtau_ev, box))
    log(f"initial conditions {n}^3 built in {time.time() - t0:.1f} s")

    ctx64 = PMContext(n, n_p, box, physics="full", precision="fp64", timings=True)
    ctx64.init_particles(pos, u, tau0)
    del pos, u
    t0 = time.time()
    for i in range(args.evolve_steps):
        ctx64.step(dtau_ev)
        if (i + 1) % 20 == 0:
            ctx64.sync()
            log(f"fp64 evolution step {i + 1}/{args.evolve_steps}, a = {ctx64.time()[1]:.4f}")
    ctx64.sync()
    tau_s, a_s, _ = ctx64.time()
    log(f"clustered snapshot at a = {a_s:.4f} after {time.time() - t0:.1f} s")
    ctx64.timings()

    def timed(ctx, label):
        dtau = 0.01 * ctx.time()[0]
        for _ in range(args.warmup):
            ctx.step(dtau)
        ctx.sync()
        ctx.timings()  # reset the stage counters
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(args.steps):
            ctx.step(dtau)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        st = ctx.timings()
        ctx.sync()
        log(f"{label}: {ms:.3f} ms/step, {n_p / ms * 1e3:.3e} particle updates/s")
        return ms, st

    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib * 2 ** 20 // 4
        src = torch.ones(nb, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {nb * 4} bytes read, {nb * 4} bytes written")
        del src, dst
        torch.cuda.empty_cache()

    # achievable streaming ceiling on this device: the library's own copy kernel (16-byte accesses,
    # eight loads in flight per thread) on 2 GiB, beside the runtime's device-to-device copy
    copy_gbs = copy_probe(2 ** 31, 5) / 1e9
    log(f"copy ceiling (own copy kernel): {copy_gbs:.0f} GB/s read + write on 2 GiB")
    nb = 2 ** 31 // 4
    src = torch.ones(nb, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    rt_gbs = 2 * nb * 4 / (c0.elapsed_time(c1) / 5 * 1e-3) / 1e9
    log(f"runtime device copy: {rt_gbs:.0f} GB/s")
    del src, dst
    torch.cuda.empty_cache()

    # FP32 path from the same snapshot
    pos_d, u_d = ctx64.get_particles(device=True)
    ctx32 = PMContext(n, n_p, box, physics="full", precision="fp32", timings=True)
    ctx32.init_particles(pos_d, u_d.to(torch.float32), tau_s)
    del pos_d, u_d
    torch.cuda.synchronize()
    ms32, st32 = timed(ctx32, "fp32")
    res = {"ms32": ms32, "st32": st32, "n": n, "n_p": n_p, "box": box, "a_snap": a_s,
           "ws32": ctx32.ws_bytes, "ws64": ctx64.ws_bytes, "copy_gbs": copy_gbs, "rt_copy_gbs": rt_gbs}
    del ctx32
    torch.cuda.empty_cache()
    if not args.no_deterministic:
        # the same step with PM_FLAG_DETERMINISTIC (particles of each cell put in identifier order)
        pos_d, u_d = ctx64.get_particles(device=True)
        ctxd = PMContext(n, n_p, box, physics="full", precision="fp32", timings=True, deterministic=True)
        ctxd.init_particles(pos_d, u_d.to(torch.float32), tau_s)
        del pos_d, u_d
        torch.cuda.synchronize()
        res["msd"], res["std"] = timed(ctxd, "fp32, deterministic")
        del ctxd
        torch.cuda.empty_cache()
    if not args.no_parabolic:
        # the same step with B from the vector part of the space-space equation (12 FFTs per step)
        pos_d, u_d = ctx64.get_particles(device=True)
        ctxp = PMContext(n, n_p, box, physics="full", precision="fp32", timings=True, b_route="parabolic")
        ctxp.init_particles(pos_d, u_d.to(torch.float32), tau_s)
        del pos_d, u_d
        torch.cuda.synchronize()
        res["msp"], res["stp"] = timed(ctxp, "fp32, parabolic B")
        del ctxp
        torch.cuda.empty_cache()
    if not args.no_fp64:
        ms64, st64 = timed(ctx64, "fp64")
        res.update(ms64=ms64, st64=st64)
    if not args.no_closure_cost:
        # the closure's cost against the 2x mesh, measured here on the same particles (scalar physics, FP32,
        # as in the closure experiment): a step on the n^3 mesh with the closure on (its cost does not depend
        # on the trained values, so the initial parameters serve) and a plain step on the (2n)^3 mesh
        from paper_2607_17929_amd import closure as cl
        pos_d, u_d = ctx64.get_particles(device=True)
        u_d = u_d.to(torch.float32)
        ctxc = PMContext(n, n_p, box, physics="scalar", precision="fp32", closure=True, timings=True)
        ctxc.init_particles(pos_d, u_d, tau_s)
        ctxc.closure_set_params(cl.init_params(0))
        ctxc.closure_enable(True)
        res["ms_closure"], _ = timed(ctxc, "fp32 scalar + closure")
        del ctxc
        torch.cuda.empty_cache()
        ctx2 = PMContext(2 * n, n_p, box, physics="scalar", precision="fp32", timings=True)
        ctx2.init_particles(pos_d, u_d, tau_s)
        del pos_d, u_d
        res["ms_2x"], _ = timed(ctx2, f"fp32 scalar, {2 * n}^3 mesh")
        del ctx2
        torch.cuda.empty_cache()
    return res


def cpu_baseline(n: int):
    """The FP64 oracle timed on the host: one full-physics step (after the quasi-static first step) at n^3."""
    import numpy as np

    from oracle import pm as opm
    from synth import spectrum_power_law_m2, zeldovich_particles
    from synth.ics import eds_a_of_tau, eds_tau_of_a

    box = 2048.0 * n / 512
    tau0 = eds_tau_of_a(0.5, box)
    dtau = 0.01 * tau0
    pos, u = zeldovich_particles(n, 3, spectrum_power_law_m2, box, 0.2, 0.02, 0.5,
                                 eds_a_of_tau(tau0 - 0.5 * dtau, box))
    sim = opm.OracleSim(n=n, box_mpch=box, physics="full", pos=pos, u=u, tau=tau0)
    sim.step(dtau)
    t0 = time.time()
    sim.step(dtau)
    dt = time.time() - t0
    cores = opm._WORKERS
    return {"value": n ** 3 / dt, "unit": "particle updates/s", "cores": cores, "kind": "oracle",
            "sample": (f"one FP64 oracle step (deposit + solve + kick/drift, full physics) of {n}^3 particles on a "
                       f"{n}^3 mesh with the same cell size, spectrum and a = 0.5 Zel'dovich start, {dt:.1f} s; "
                       f"numpy/scipy, FFTs on {cores} threads (the host's CPU share for this GPU), deposit and gather "
                       f"single-threaded")}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--evolve-steps", type=int, default=100)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-parabolic", action="store_true", help="skip the parabolic-B FP32 leg")
    ap.add_argument("--no-deterministic", action="store_true", help="skip the deterministic FP32 leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-closure-cost", action="store_true", help="skip timing the closure against the 2x mesh")
    ap.add_argument("--cpu-n", type=int, default=256)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB before timing (a known-size dispatch that "
                         "calibrates hardware byte counters in a profiler run)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path "
              "(the PM step is measured on a single MI355X); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    r = run_gpu(args)
    n, n_p = r["n"], r["n_p"]
    st = r["st32"]
    per_launch = {}
    for k, (ms, calls) in st.items():
        if calls:
            per_launch[k] = ms / calls / LAUNCHES.get(k, 1)
    totals = {k: ms for k, (ms, calls) in st.items()}
    dom = max(totals, key=totals.get)
    nbytes = stage_bytes(n, n_p, 4)
    achieved = nbytes[dom] / (per_launch[dom] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(n, dom),
            "frac_of_copy": round(achieved / r["copy_gbs"], 4),
            "algorithmic_bytes_per_launch": nbytes[dom], "ms_per_launch": round(per_launch[dom], 4)}
    stages = {k: {"ms_per_launch": round(per_launch.get(k, 0.0), 4),
                  "GBs": round(nbytes[k] / (per_launch[k] * 1e-3) / 1e9, 1) if k in per_launch else None}
              for k in st}
    out = {
        "metric": "particle updates/s per PM step at 512^3 (FP32 vs FP64); closure vs 2x mesh",
        "value": n_p / r["ms32"] * 1e3,
        "unit": "particle updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms32"], 4),
        "higher_is_better": True,
        "scaling": None,  # one GPU: no scaling claim
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"clustered mixed-precision run: {n}^3 particles on a {n}^3 mesh, box "
                                f"{r['box']:.0f} Mpc/h, k^-2 Zel'dovich start at a=0.02 evolved by the FP64 GPU path "
                                f"to a={r['a_snap']:.3f}, full scalar+vector+tensor physics, dtau = 0.01 tau"),
                   "n_mesh": n, "n_particles": n_p, "physics": "full",
                   "precision": "FP32 fields/FFT/deposit/momenta, FP64 positions and zero mode"},
        "stages_fp32": stages,
        "roofline": roof,
        "copy_ceiling": {"GBs": round(r["copy_gbs"], 1),
                         "kind": "library copy kernel (pm_copy_probe): 2 GiB, 16-byte accesses, read + write",
                         "frac_of_peak": round(r["copy_gbs"] / HBM_PEAK_GBS, 4),
                         "runtime_copy_GBs": round(r["rt_copy_gbs"], 1)},
        "workspace_GB": {"fp32": round(r["ws32"] / 1e9, 2), "fp64": round(r["ws64"] / 1e9, 2)},
    }
    if "msp" in r:
        out["fp32_parabolic_b"] = {
            "value": n_p / r["msp"] * 1e3, "ms_per_step": round(r["msp"], 4),
            "stages": {k: round(ms / calls / LAUNCHES.get(k, 1), 4) for k, (ms, calls) in r["stp"].items() if calls}}
    if "msd" in r:
        out["fp32_deterministic"] = {
            "value": n_p / r["msd"] * 1e3, "ms_per_step": round(r["msd"], 4),
            "cost_vs_fp32": round(r["msd"] / r["ms32"], 4),
            "stages": {k: round(ms / calls / LAUNCHES.get(k, 1), 4) for k, (ms, calls) in r["std"].items() if calls}}
    if "ms64" in r:
        out["fp64"] = {"value": n_p / r["ms64"] * 1e3, "ms_per_step": round(r["ms64"], 4),
                       "stages": {k: round(ms / calls / LAUNCHES.get(k, 1), 4) for k, (ms, calls) in r["st64"].items()
                                  if calls}}
    cl = closure_result() or {}
    if "ms_closure" in r:
        cl.update({"cost_vs_2x_measured": round(r["ms_closure"] / r["ms_2x"], 4),
                   "closure_ms_per_step": round(r["ms_closure"], 4), "plain_2x_ms_per_step": round(r["ms_2x"], 4),
                   "cost_measured": f"this run: FP32 scalar-physics steps on the {n}^3 mesh with the closure and on "
                                    f"the {2 * n}^3 mesh, same particles"})
    if cl:
        out["closure_vs_2x_mesh"] = cl
    if not args.no_cpu_baseline:
        log(f"timing the CPU oracle at {args.cpu_n}^3")
        out["cpu_baseline"] = cpu_baseline(args.cpu_n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
