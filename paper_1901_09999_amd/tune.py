"""Launch-shape choice for batched matching.

The fused apply kernel of a batch visits the 64 x 64 tiles of every pair;
its grid (one workgroup per tile, or a grid-stride loop over a fixed number
of workgroups) and the order of the pairs in the tile list (as given,
smallest first, largest first) are chosen by timing each candidate on the
batch itself.  Results are cached as JSON, keyed by the device and the shape
of the batch, so a later plan of the same shape skips the search.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import psfm

DEFAULT_GRIDS = (0, 256, 512, 1024, 2048)
DEFAULT_ORDERS = (0, 1, 2)


def cache_path() -> str:
    return os.environ.get("PSFM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "psfm", "tune.json"))


def batch_key(ctx: psfm.Context, pairs: Sequence[dict]) -> str:
    dev = torch.cuda.get_device_properties(ctx.device)
    shape = [(int(q["I1"].shape[1]), int(q["I1"].shape[0]), int(q["S"]),
              int(q["stamps"].shape[0])) for q in pairs]
    h = hashlib.sha256(json.dumps([dev.name, ctx.cfg.h, ctx.cfg.r, ctx.cfg.P, shape]).encode())
    return h.hexdigest()[:24]


def _load() -> Dict[str, dict]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, rec: dict):
    data = _load()
    data[key] = rec
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1)
    os.replace(tmp, path)


def _time_runs(b: psfm.Batch, reps: int) -> float:
    b.run()                                   # warm
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(b.stream):
            e0.record()
        b.run()
        with torch.cuda.stream(b.stream):
            e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def choose(ctx: psfm.Context, pairs: Sequence[dict], c_out: int = 10,
           grids: Sequence[int] = DEFAULT_GRIDS, orders: Sequence[int] = DEFAULT_ORDERS,
           reps: int = 2, use_cache: bool = True, log=None) -> Tuple[int, int, List[dict]]:
    """Returns (apply_grid, order, table of timings in ms)."""
    key = batch_key(ctx, pairs)
    if use_cache:
        rec = _load().get(key)
        if rec:
            return rec["apply_grid"], rec["order"], rec["table"]
    table = []
    for order in orders:
        b = psfm.Batch(ctx, pairs, c_out=c_out, order=order)
        for g in grids:
            b.set_apply_grid(g)
            ms = _time_runs(b, reps)
            table.append(dict(apply_grid=g, order=order, ms=round(ms, 4)))
            if log:
                log(f"tune: order {order} apply_grid {g}: {ms:.3f} ms")
        b.close()
        del b
        torch.cuda.empty_cache()
    best = min(table, key=lambda t: t["ms"])
    _store(key, dict(apply_grid=best["apply_grid"], order=best["order"], table=table,
                     when=time.strftime("%Y-%m-%dT%H:%M:%S")))
    return best["apply_grid"], best["order"], table
