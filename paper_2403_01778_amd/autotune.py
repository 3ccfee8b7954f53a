"""Autotuner of the TTVc sweep's level-1 tiling.

For one tensor (its storage dtype and dims) it times whole sweeps under each
candidate tiling with HIP events (hoscf_profile_sweep), registers the fastest
with the library (hoscf_tune_set), and can save or load the resulting table
as JSON so that a later process starts from the tuned tilings.  A tiling is
(workgroups the grid is sized for, smallest p-range, lanes per row, aligned
q-chunks, rows per lane group, waves per workgroup); 0 keeps a field's rule.
"""
from __future__ import annotations

import json
from typing import Dict, Iterable, List, Optional, Sequence

import torch

from . import hoscf

# rows per lane group of each storage format (its half is the other option)
_MB = {hoscf.F64: 16, hoscf.F32: 16, hoscf.BF16: 8, hoscf.FP8E4M3: 4}


def candidates(dtype: int) -> List[tuple]:
    mb = _MB[dtype]
    return [(0, 1, lr, 1, m, nw) for lr in (16, 32, 64) for m in (mb, mb // 2) for nw in (4, 8)]


def autotune(T: torch.Tensor, x: torch.Tensor, reps: int = 10, scale: float = 1.0,
             cands: Optional[Iterable[Sequence[int]]] = None, register: bool = True) -> Dict:
    """Times each candidate (whole sweep, ms) and returns the table record
    {dtype, dims, tiling, ms, default_ms, timings}; registers the winner
    unless register is False."""
    desc = hoscf.describe(T, scale)
    dtype = int(desc.dtype)
    dims = [int(d) for d in T.shape]
    hoscf.tune_set(dtype, dims, None)
    default_ms = hoscf.profile_sweep(T, x, reps=reps, scale=scale)[0]
    timings = []
    for t in (cands if cands is not None else candidates(dtype)):
        ms = hoscf.profile_sweep(T, x, reps=reps, scale=scale, tiling=tuple(t))[0]
        timings.append((list(t), ms))
    best_t, best_ms = min(timings, key=lambda r: r[1])
    rec = {"dtype": dtype, "dims": dims, "tiling": best_t, "ms": best_ms, "default_ms": default_ms,
           "timings": timings}
    if register and best_ms < default_ms:
        hoscf.tune_set(dtype, dims, best_t)
    return rec


def save(records: Iterable[Dict], path: str) -> None:
    with open(path, "w") as f:
        json.dump([{k: r[k] for k in ("dtype", "dims", "tiling", "ms", "default_ms")} for r in records], f, indent=1)


def load(path: str) -> List[Dict]:
    """Registers every record of a saved table whose tiling beat the rule."""
    with open(path) as f:
        recs = json.load(f)
    for r in recs:
        if r["ms"] < r["default_ms"]:
            hoscf.tune_set(int(r["dtype"]), r["dims"], r["tiling"])
    return recs
