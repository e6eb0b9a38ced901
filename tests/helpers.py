"""Shared helpers of the GPU parity tests (run on both sides with identical seeded inputs)."""
from __future__ import annotations

import numpy as np

from oracle import pm as opm

FIELD_NAMES_FULL = ["phi", "chi", "bx", "by", "bz"]
H_NAMES = ["hxx", "hxy", "hxz", "hyy", "hyz", "hzz"]


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def rel_linf(a, b) -> float:
    """max |a - b| / max |b|: a single wrong vertex, or a wrong plane of modes with little power, that
    the relative L2 norm over the whole mesh would average away."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mb = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / mb) if mb > 0 else float(np.max(np.abs(a - b)))


# bars of the field comparisons: relative L2 over the mesh (the stated tolerance of each path) and the
# largest pointwise difference relative to the field's largest magnitude (ten times the L2 bar)
FIELD_L2 = {"fp64": 1e-10, "fp32": 1e-5}
FIELD_LINF = {"fp64": 1e-9, "fp32": 1e-4}


def field_errors(got: dict, ref: dict) -> dict:
    """{name: (relative L2, relative max-norm)} of each field in got against ref."""
    return {k: (rel_l2(got[k], ref[k]), rel_linf(got[k], ref[k])) for k in got}


def assert_fields(errs: dict, precision: str, scale: float = 1.0) -> None:
    for k, (l2, linf) in errs.items():
        assert l2 < scale * FIELD_L2[precision], (k, "rel-L2", l2)
        assert linf < scale * FIELD_LINF[precision], (k, "rel-max", linf)


def periodic_max_dx(p1, p2, n) -> float:
    """max over particles and axes of the minimum-image |p1 - p2| in units of the mesh spacing."""
    d = np.asarray(p1, dtype=np.float64) - np.asarray(p2, dtype=np.float64)
    d -= np.round(d)
    return float(np.max(np.abs(d)) * n)


def oracle_fields(sim: opm.OracleSim, physics: str):
    out = {"phi": sim.phi}
    if physics != "newtonian":
        out["chi"] = sim.chi
    if physics == "full":
        out["bx"], out["by"], out["bz"] = sim.B
        for name, h in zip(H_NAMES, sim.h_real()):
            out[name] = h
    return out


def gpu_fields(ctx, physics: str):
    names = ["phi"] + (["chi"] if physics != "newtonian" else []) + (["bx", "by", "bz"] + H_NAMES if physics == "full" else [])
    return {k: ctx.get_field(k).astype(np.float64) for k in names}
