"""Launch-shape choice for batched matching.

The fit's band height and three launch parameters are chosen by timing
each candidate on the batch itself:
  * the stamp fit's band height (stamp rows per workgroup, 7, 9 or 11: the
    kernels are built for all three), timed on the fit stage alone;
  * the fused apply kernel's grid (one workgroup per 64 x 64 tile, or a
    grid-stride loop over a fixed number of workgroups) and the order of the
    pairs in its tile list (as given, smallest first, largest first), timed
    on the whole batch;
  * the split of the batch into plans by spatial order, run side by side as
    the branches of one graph (one plan; the highest order alone; the two
    highest each alone; every order alone), timed on the whole batch with
    the chosen apply parameters: pairs of different unknown counts finish
    their solves at different times, so one plan's tile pass can fill the
    device while another still solves.
The searches are separate because the band height changes only the fit
and the apply parameters only the tile pass.  Results are cached as JSON,
keyed by the device and the shape of the batch, so a later plan of the same
shape skips the search.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import os
import time
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import psfm

DEFAULT_GRIDS = (0, 256, 512, 1024, 2048)
DEFAULT_ORDERS = (0, 1, 2)
DEFAULT_BAND_ROWS = (7, 9, 11)


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


def _time_stage(b: psfm.Batch, stage: int, reps: int) -> float:
    b.run()                                   # warm (and every stage's inputs in place)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(b.stream):
            e0.record()
            b.run_stage(stage)
            e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def order_groups(pairs: Sequence[dict]) -> List[List[List[int]]]:
    """Candidate splits of the pairs by spatial order (see split_by_order):
    none, the highest order alone, the two highest each alone, every order
    alone."""
    orders = sorted({int(q["S"]) for q in pairs}, reverse=True)
    cands: List[List[List[int]]] = [[]]
    if len(orders) >= 2:
        cands.append([[orders[0]]])
    if len(orders) >= 3:
        cands.append([[orders[0]], [orders[1]]])
    if len(orders) >= 4:
        cands.append([[o] for o in orders[:-1]])
    return cands


def _time_group(ctx: psfm.Context, pairs: Sequence[dict], groups, c_out: int, grid: int,
                order: int, reps: int) -> float:
    idx = psfm.split_by_order(pairs, groups)
    subs = [psfm.Batch(ctx, [pairs[k] for k in ix], c_out=c_out, apply_grid=grid, order=order)
            for ix in idx]
    grp = psfm.BatchGroup(subs)
    grp.launch()                              # warm
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(grp.stream):
            e0.record()
        grp.launch()
        with torch.cuda.stream(grp.stream):
            e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    grp.close()
    for b in subs:
        b.close()
    del grp, subs
    torch.cuda.empty_cache()
    return best


def context_for(ctx: psfm.Context, fit_band_rows: int) -> psfm.Context:
    """ctx itself, or a context of the same configuration with the given fit band height."""
    if ctx.cfg.fit_band_rows == fit_band_rows:
        return ctx
    return psfm.Context(dataclasses.replace(ctx.cfg, fit_band_rows=fit_band_rows), ctx.device)


def choose(ctx: psfm.Context, pairs: Sequence[dict], c_out: int = 10,
           grids: Sequence[int] = DEFAULT_GRIDS, orders: Sequence[int] = DEFAULT_ORDERS,
           band_rows: Sequence[int] = DEFAULT_BAND_ROWS, reps: int = 2, use_cache: bool = True,
           log=None) -> dict:
    """Returns dict(apply_grid, order, fit_band_rows, groups, table of timings
    in ms); groups: the spatial orders of each side-by-side plan but the
    last (split_by_order), [] for one plan."""
    key = batch_key(ctx, pairs)
    if use_cache:
        rec = _load().get(key)
        if rec and "fit_band_rows" in rec and "groups" in rec:
            return rec
    table = []
    fit_ms = {}
    for br in band_rows:
        try:
            c = context_for(ctx, br)
        except psfm.PsfmError:                # that band's LDS does not fit this basis
            continue
        b = psfm.Batch(c, pairs, c_out=c_out)
        ms = _time_stage(b, 0, reps)
        fit_ms[br] = ms
        table.append(dict(fit_band_rows=br, stage="fit", ms=round(ms, 4)))
        if log:
            log(f"tune: fit band rows {br}: {ms:.3f} ms")
        b.close()
        del b
        if c is not ctx:
            c.close()
        torch.cuda.empty_cache()
    best_br = min(fit_ms, key=fit_ms.get) if fit_ms else ctx.cfg.fit_band_rows
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
    best = min((t for t in table if "apply_grid" in t), key=lambda t: t["ms"])
    c = context_for(ctx, best_br)
    group_ms = []
    for groups in order_groups(pairs):
        ms = _time_group(c, pairs, groups, c_out, best["apply_grid"], best["order"], reps)
        group_ms.append((ms, groups))
        table.append(dict(groups=groups, ms=round(ms, 4)))
        if log:
            log(f"tune: plans split by spatial order {groups or 'none'}: {ms:.3f} ms")
    if c is not ctx:
        c.close()
    best_groups = min(group_ms, key=lambda t: t[0])[1] if group_ms else []
    rec = dict(apply_grid=best["apply_grid"], order=best["order"], fit_band_rows=best_br,
               groups=best_groups, table=table, when=time.strftime("%Y-%m-%dT%H:%M:%S"))
    _store(key, rec)
    return rec
