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
