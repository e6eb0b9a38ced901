"""Summaries of rocprofv3 output for the PM step (offline tooling, no GPU needed).

    python -m paper_2607_17929_amd.profsum trace  <kernel_trace.csv> --command "..."
    python -m paper_2607_17929_amd.profsum traffic <fetch counter csv> <write counter csv> \
        --probe-bytes B --steps K --command "..."

`trace` turns a `--kernel-trace` CSV into a table of per-kernel durations.
`counters` averages other `--pmc` counters per dispatch of each stage's kernels.
`traffic` turns two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs into HBM bytes
per launch of each stage's kernels.  Both counters are reported in KiB per
dispatch; each is scaled by what the same counter reads for the runtime's
plain device-to-device copy of a known size (the bench's copy probe), which
absorbs the counters' request-size accounting on this GPU.  The table carries
the SHA-256 of the kernel sources it was measured with, so that a reader (the
bench) can tell when a kernel has changed since.  `traffic` and `counters` take
the last launches of each stage's kernels, so the profiled run must end with the
legs they describe: the bench is profiled without its closure-cost legs
(`--no-closure-cost`), which run some of the same kernels on other meshes.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")

# stage -> (kernel-name pattern, launches of that kernel per step); {T} is float or double
STAGE_KERNELS = {
    "deposit": [(r"deposit_kernel<{T}, 10", 1)],
    "fft_x_fwd": [(r"fft_x_r2c_kernel<{T}", 1)],
    "fft_y_fwd": [(r"fft_cols_kernel<{T}, \d+, \d+, \d+, false>", 1)],
    "kspace": [(r"kspace_kernel<{T}", 1)],
    "fft_y_inv": [(r"fft_cols_kernel<{T}, \d+, \d+, \d+, true>", 1)],
    "fft_x_inv": [(r"fft_x_c2r_kernel<{T}", 1)],
    "kick_drift": [(r"kick_drift_kernel<{T}", 1)],
    "sort": [(r"scan_reduce_kernel", 1), (r"scan_blocks_kernel", 1), (r"scan_apply_kernel", 1),
             (r"scatter_kernel<{T}", 1)],
}
# stages whose kernels run as separate launches (the bench reports per-launch figures for them)
LAUNCHES: dict = {}
# source files each stage's kernels are built from
STAGE_SOURCES = {
    "deposit": ["particles.hip"], "kick_drift": ["particles.hip"], "sort": ["particles.hip"],
    "fft_x_fwd": ["fft.hip"], "fft_y_fwd": ["fft.hip", "fft_lds.h"], "fft_y_inv": ["fft.hip", "fft_lds.h"],
    "fft_x_inv": ["fft.hip"], "kspace": ["solve.hip", "fft_lds.h"],
}
COMMON_SOURCES = ["common.h", "kernels.h"]


def source_hash(stage: str, csrc: str = CSRC) -> str:
    h = hashlib.sha256()
    for f in STAGE_SOURCES[stage] + COMMON_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _rows(path: str):
    with open(path, newline="") as fh:
        yield from csv.DictReader(fh)


def trace_table(path: str, command: str) -> str:
    agg = defaultdict(list)
    for r in _rows(path):
        agg[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    lines = ["| Kernel | Calls | Avg (us) | Min (us) | Max (us) | Total (ms) |", "|---|---|---|---|---|---|"]
    for name, d in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        short = re.sub(r"\(.*", "", name).replace("void ", "")[:90]
        lines.append(f"| `{short}` | {len(d)} | {sum(d) / len(d):.1f} | {min(d):.1f} | {max(d):.1f} | "
                     f"{sum(d) * 1e-3:.2f} |")
    return f"Command:\n\n    {command}\n\n" + "\n".join(lines) + "\n"


def _per_dispatch(path: str, counter: str):
    out = []  # (dispatch id, kernel name, value KiB)
    for r in _rows(path):
        if r["Counter_Name"] == counter:
            out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    out.sort()
    return out


def traffic(fetch_csv: str, write_csv: str, probe_bytes: int, steps: int, n: int) -> dict:
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(write_csv, "WRITE_SIZE")
    kib = probe_bytes / 1024.0

    def probe(rows, other_rows=None):
        # the runtime's copy kernel whose write counter matches the probe size (to 1 %)
        cands = [d for d, k, v in (other_rows or rows) if "copyBuffer" in k and abs(v - kib) < 0.01 * kib]
        if not cands:
            raise SystemExit("copy probe dispatch not found")
        d = cands[-1]
        return d, {dd: v for dd, k, v in rows}[d]

    d_w, w_probe = probe(write)
    # the same dispatch in the FETCH run: the copy right before the timed FP32 run (same position)
    d_f = d_w
    f_probe = {dd: v for dd, k, v in fetch}.get(d_f)
    if f_probe is None or "copyBuffer" not in {dd: k for dd, k, v in fetch}[d_f]:
        raise SystemExit("copy probe dispatch differs between the two runs")
    read_scale, write_scale = kib / f_probe, kib / w_probe
    result = {"n": n, "probe_bytes": probe_bytes, "fetch_probe_kib": f_probe, "write_probe_kib": w_probe,
              "read_scale": read_scale, "write_scale": write_scale, "stages": {}}
    for prec, T in (("fp32", "float"), ("fp64", "double")):
        for stage, kernels in STAGE_KERNELS.items():
            rd = wr = 0.0
            detail = []
            ok = True
            for pat, per_step in kernels:
                rx = re.compile(pat.replace("{T}", T))
                fv = [v for d, k, v in fetch if rx.search(k)]
                wv = [v for d, k, v in write if rx.search(k)]
                take = steps * per_step
                if len(fv) < take or len(wv) < take:
                    ok = False
                    break
                f_avg = sum(fv[-take:]) / take
                w_avg = sum(wv[-take:]) / take
                detail.append({"pattern": pat.replace("{T}", T), "dispatches": take, "fetch_kib": round(f_avg, 1),
                               "write_kib": round(w_avg, 1)})
                rd += f_avg * 1024 * read_scale * per_step
                wr += w_avg * 1024 * write_scale * per_step
            if not ok:
                continue
            nl = LAUNCHES.get(stage, 1)
            result["stages"][f"{prec}:{stage}"] = {
                "read_bytes_per_launch": round(rd / nl), "write_bytes_per_launch": round(wr / nl),
                "traffic_bytes_per_launch": round((rd + wr) / nl), "kernels": detail,
                "source_sha256": source_hash(stage)}
    return result


def traffic_md(res: dict, command_fetch: str, command_write: str) -> str:
    n = res["n"]
    lines = [f"# HBM traffic per launch: PM step, {n}^3 clustered workload", "",
             "Commands (from the repository root on the MI355X machine):", "",
             f"    {command_fetch}", f"    {command_write}", "",
             f"Calibration: the copy probe moves {res['probe_bytes']} bytes; FETCH_SIZE reads "
             f"{res['fetch_probe_kib']:.1f} KiB and WRITE_SIZE {res['write_probe_kib']:.1f} KiB for it, so read "
             f"counts are scaled by {res['read_scale']:.4f} and write counts by {res['write_scale']:.4f}.", "",
             "| Stage | Read GB / launch | Write GB / launch | Traffic GB / launch |", "|---|---|---|---|"]
    for k, v in res["stages"].items():
        lines.append(f"| {k} | {v['read_bytes_per_launch'] / 1e9:.3f} | {v['write_bytes_per_launch'] / 1e9:.3f} | "
                     f"{v['traffic_bytes_per_launch'] / 1e9:.3f} |")
    lines += ["", "Machine-readable (read by bench.py, which reports a stage's traffic only while the SHA-256 of",
              "its kernel sources still matches):", "", "```json", json.dumps(res, indent=1), "```", ""]
    return "\n".join(lines)


def load_traffic(md_path: str) -> dict | None:
    """The JSON block of a traffic summary, or None."""
    try:
        with open(md_path) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    return json.loads(m.group(1)) if m else None


def counters(csvs, steps: int, prec: str = "float") -> dict:
    """Average per dispatch of every counter in the `--pmc` CSVs for the last `steps` dispatches of each stage's
    kernels (the first pattern of the stage), {stage: {counter: value}}."""
    out = {}
    for stage, kernels in STAGE_KERNELS.items():
        rx = re.compile(kernels[-1][0].replace("{T}", prec))
        vals = {}
        for path in csvs:
            per = defaultdict(list)
            for r in _rows(path):
                if rx.search(r["Kernel_Name"]):
                    per[r["Counter_Name"]].append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
            for c, v in per.items():
                v.sort()
                tail = [x for _, x in v[-steps:]]
                vals[c] = sum(tail) / len(tail)
        if vals:
            out[stage] = vals
    return out


def counters_md(res: dict, n_particles: int, commands) -> str:
    """Table of the counters per stage with the derived ratios that separate latency from issue limits."""
    names = sorted({c for v in res.values() for c in v})
    lines = ["Commands (from the repository root on the MI355X machine):", ""] + [f"    {c}" for c in commands] + [""]
    lines += ["| Stage | " + " | ".join(names) + " |", "|---|" + "---|" * len(names)]
    for st, v in res.items():
        lines.append(f"| {st} | " + " | ".join(f"{v[c]:.4g}" if c in v else "" for c in names) + " |")
    lines += ["", "| Stage | waves waiting on a dependency (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES) | VALU instructions per "
              "particle | LDS bank-conflict cycles / LDS active cycles | L2 hit rate |", "|---|---|---|---|---|"]
    for st, v in res.items():
        def ratio(a, b):
            return f"{v[a] / v[b]:.2f}" if a in v and b in v and v[b] else ""
        valu = f"{v['SQ_INSTS_VALU'] * 64 / n_particles:.0f}" if "SQ_INSTS_VALU" in v else ""
        hit = (f"{v['TCC_HIT_sum'] / (v['TCC_HIT_sum'] + v['TCC_MISS_sum']):.2f}"
               if "TCC_HIT_sum" in v and "TCC_MISS_sum" in v else "")
        lines.append(f"| {st} | {ratio('SQ_WAIT_INST_ANY', 'SQ_WAVE_CYCLES')} | {valu} | "
                     f"{ratio('SQ_LDS_BANK_CONFLICT', 'SQ_LDS_IDX_ACTIVE')} | {hit} |")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("counters")
    k.add_argument("csv", nargs="+")
    k.add_argument("--steps", type=int, required=True)
    k.add_argument("--particles", type=int, required=True)
    k.add_argument("--command", action="append", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("--command", required=True)
    f = sub.add_parser("traffic")
    f.add_argument("fetch_csv")
    f.add_argument("write_csv")
    f.add_argument("--probe-bytes", type=int, required=True)
    f.add_argument("--steps", type=int, required=True)
    f.add_argument("--n", type=int, default=512)
    f.add_argument("--command-fetch", required=True)
    f.add_argument("--command-write", required=True)
    a = ap.parse_args()
    if a.cmd == "counters":
        print(counters_md(counters(a.csv, a.steps), a.particles, a.command), end="")
    elif a.cmd == "trace":
        print(trace_table(a.csv, a.command), end="")
    else:
        res = traffic(a.fetch_csv, a.write_csv, a.probe_bytes, a.steps, a.n)
        print(traffic_md(res, a.command_fetch, a.command_write), end="")


if __name__ == "__main__":
    main()
