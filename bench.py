"""Throughput of the PSF-matching hot path on one MI355X.

One step = one whole pass of the path over synthetic input already resident
in HBM.

Default workload (batch64): one batch of 64 independent image pairs of uneven
size (1024 to 6000 px a side, 734 Mpx in all; per pair its own PSFs, spatial
order 0-3, 50-400 stamps of 41 x 41, 10% mask, 5% variable sources, 21 x 21
kernel with the 49-term ISIS basis) through psfm_batch_* as one captured HIP
graph: stamp fits -> solves with rejection -> pseudo-matrices -> fused
image + variance convolution and difference over every output tile.  Also
reports the p50 / p99 completion latency of the pairs, the stage split, the
tuner's table, the learned prior's leg on the same pairs, the plain vs
16-bit comparison on the detector-chip pair and the paper's other modes
(two kernels with the penalty, normalisation and quality, homogenisation
for stacking, binning and addition) on 2048^2 images.

--workload pair2048 / chip4846: one pair,
    psfm_fit_stamps -> psfm_solve (with rejection) -> psfm_match_pair.
--workload cells200k: the learned prior's training throughput.

Prints one JSON line.  `value` is pixels matched per second (Mpix/s).
`roofline` is for the kernel with the largest share of the step (for the
batch: k_match_tiles_b, the fused convolution / difference pass), timed
with HIP events on the stream it runs on.  `cpu_baseline` is the FP64 oracle
on the host's cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VALU_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak (packed)
FP64_PEAK_TFLOPS = 78.6           # MI355X published FP64 vector and matrix peak
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
METRIC = "Mpix/s PSF-matched subtraction (fit+convolve), plain vs mixed/learned @χ² tol"


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch64")
    ap.add_argument("--no-extra", action="store_true",
                    help="batch: skip the learned-prior leg and the 16-bit comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--retune", action="store_true", help="ignore cached batch launch shapes")
    ap.add_argument("--no-tune", action="store_true",
                    help="batch: skip the launch-shape search (one workgroup per tile, smallest "
                         "pair first; for profiling runs)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp16", "bf16"],
                    help="arithmetic of the stamp fit for the reported value")
    ap.add_argument("--refine", type=int, default=None, help="refinement steps of 16-bit modes")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip timing the other fit arithmetic beside the reported one")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (calibrates HBM counters)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="bound on the oracle's timed sample")
    return ap.parse_args()


def source_sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(record, kernel_src):
    """HBM bytes per launch of a kernel from its committed rocprofv3 counter
    summary (profiles/<record>), if that was taken on the current source."""
    path = os.path.join(PROFILES, record)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha") != source_sha(kernel_src):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(wl, pair, budget_s):
    import oracle as O
    O.build()
    cfg = O.Config.from_workload(wl)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    os.environ.setdefault("OMP_NUM_THREADS", str(threads))
    runs, t_total, res = 0, 0.0, None
    while runs < 1 or (t_total < budget_s and runs < 20):
        t0 = time.perf_counter()
        res = O.match_pair(cfg, pair, c_out=wl.cov_half)
        t_total += time.perf_counter() - t0
        runs += 1
    per = t_total / runs
    return dict(value=round(wl.pixels / 1e6 / per, 3), unit="Mpix/s", cores=threads,
                kind="oracle",
                sample=f"whole path (fit, solve, convolve, variance, subtract) on the same "
                       f"{wl.width}x{wl.height} pair, {runs} run(s), {per:.3f} s each, FP64, "
                       f"OpenMP over stamps and patches"), res


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))


def oracle_batch_baseline(wls, dps, px, st, budget_s):
    """The FP64 oracle on the smallest pairs of the batch: all host threads
    until ~budget_s, and one thread on the smallest pair.  Returns
    (cpu_baseline dict, parity dict)."""
    import oracle as O
    O.build()
    threads = host_threads()
    order_px = np.argsort(px)
    O.set_threads(threads)
    done_px, spent, used, rel = 0.0, 0.0, [], []
    for k in order_px:
        if spent > 0 and spent + spent / max(len(used), 1) > budget_s:
            break
        hp = dps[k].host()
        t1 = time.perf_counter()
        ref = O.match_pair(O.Config.from_workload(wls[k]), hp, c_out=10)
        spent += time.perf_counter() - t1
        done_px += px[k]
        used.append(int(k))
        rs = ref["stats"]
        if rs["info"] == 0 and st[k]["info"] == 0:
            rel.append((abs(st[k]["kernel_sum_centre"] / rs["kernel_sum_centre"] - 1),
                        abs(st[k]["chi2_dof"] / rs["chi2_dof"] - 1)))
    k0 = int(order_px[0])
    O.set_threads(1)
    hp = dps[k0].host()
    t1 = time.perf_counter()
    O.match_pair(O.Config.from_workload(wls[k0]), hp, c_out=10)
    one = time.perf_counter() - t1
    O.set_threads(threads)
    base = dict(value=round(done_px / 1e6 / spent, 3), unit="Mpix/s", cores=threads, kind="oracle",
                cpu=cpu_model(),
                sample=f"whole path on the {len(used)} smallest pair(s) of the batch "
                       f"({done_px / 1e6:.1f} Mpx, {spent:.1f} s), FP64, OpenMP over stamps and "
                       f"patches on {threads} threads; rate = their pixels / their time",
                one_thread=dict(value=round(px[k0] / 1e6 / one, 3), unit="Mpix/s", cores=1,
                                sample=f"the smallest pair ({px[k0] / 1e6:.2f} Mpx) once, "
                                       f"{one:.1f} s"))
    par = None
    if rel:
        par = {"pairs": used, "kernel_sum_rel_max": max(r[0] for r in rel),
               "chi2_dof_rel_max": max(r[1] for r in rel)}
    return base, par


def bench_batch(args, torch, psfm, synth):
    from paper_1901_09999_amd import tune
    spec = synth.BATCHES[args.workload]
    t0 = time.perf_counter()
    wls, dps = synth.make_batch_device(args.workload,
                                       log=lambda s: log(f"{s} ({time.perf_counter() - t0:.1f} s)"))
    px = np.array([wl.pixels for wl in wls], dtype=np.float64)
    total_px = float(px.sum())
    ctx = psfm.Context(psfm.Config(h=spec.kernel_half, r=spec.stamp_half, S=0))
    pairs = [dict(I1=d.I1, V1=d.V1, M1=d.M1, I2=d.I2, V2=d.V2, M2=d.M2,
                  stamps=torch.from_numpy(d.stamps.astype(np.int32)).cuda(),
                  S=d.workload.spatial_order) for d in dps]
    if args.no_tune:
        grid, order, band, groups, table = 0, 1, 0, [], []
    else:
        tu = tune.choose(ctx, pairs, c_out=10, log=log, use_cache=not args.retune)
        grid, order, band, table = tu["apply_grid"], tu["order"], tu["fit_band_rows"], tu["table"]
        groups = tu.get("groups", [])
        ctx = tune.context_for(ctx, band)
    plans = psfm.split_by_order(pairs, groups)
    log(f"tuned: apply_grid {grid}, order {order}, fit band rows {band}, "
        f"plans by spatial order {[sorted({int(pairs[k]['S']) for k in ix}) for ix in plans]}")
    b = psfm.Batch(ctx, pairs, c_out=10, apply_grid=grid, order=order)
    b.run()
    torch.cuda.synchronize()
    # stage times (eager, events on the batch stream)
    NS = 4
    stage = np.zeros(NS)
    reps = 3
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(NS + 1)]
        with torch.cuda.stream(b.stream):
            ev[0].record()
            for sidx in range(NS):
                b.run_stage(sidx)
                ev[sidx + 1].record()
        ev[NS].synchronize()
        stage += [ev[i].elapsed_time(ev[i + 1]) for i in range(NS)]
    stage /= reps
    # the dominant kernel alone: k_match_tiles_b is stage 3 (one launch over
    # the tiles of every pair), timed with HIP events on the batch stream over
    # as many launches as steps
    kreps = max(args.steps, 5)
    k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(b.stream):
        k0.record()
        for _ in range(kreps):
            b.run_stage(3)
        k1.record()
    k1.synchronize()
    tiles_us = k0.elapsed_time(k1) * 1e3 / kreps
    # the timed step: one graph; with a split by spatial order, one plan per
    # group as the graph's parallel branches
    if len(plans) > 1:
        b.close()
        del b
        torch.cuda.empty_cache()
        subs = [psfm.Batch(ctx, [pairs[k] for k in ix], c_out=10, apply_grid=grid, order=order)
                for ix in plans]
        runner = psfm.BatchGroup(subs)
    else:
        subs = [b]
        b.capture()
        runner = b
    for _ in range(args.warmup):
        runner.launch()
    torch.cuda.synchronize()
    lat, per = [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(runner.stream):
            e0.record()
        runner.launch()
        with torch.cuda.stream(runner.stream):
            e1.record()
        e1.synchronize()
        per.append(e0.elapsed_time(e1))
        lat.append(np.concatenate([sb.latencies_s() for sb in subs]) * 1e3)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = 1e3 * wall / args.steps
    lat = np.concatenate(lat)
    st = [None] * len(wls)
    for ix, sb in zip(plans, subs):
        for j, k in enumerate(ix):
            st[k] = sb.stats(j)
    T = (2 * spec.kernel_half + 1) ** 2
    flops = 4.0 * T * total_px                 # I' and V' (2T flop per pixel each)
    achieved = flops / (tiles_us * 1e-6) / 1e12
    traffic = measured_traffic("match_tiles_b_batch64_traffic.json",
                               os.path.join(ROOT, "paper_1901_09999_amd", "csrc", "convolve.hip"))
    out = {
        "metric": METRIC,
        "value": round(total_px / 1e6 / (ms_per_step * 1e-3), 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {len(wls)} independent pairs, "
                               f"{total_px / 1e6:.0f} Mpx in all, sides U{{{spec.size_lo}..{spec.size_hi}}}, "
                               f"spatial order U{{0..{spec.S_max}}}, stamps U{{{spec.stamps_lo}.."
                               f"{spec.stamps_hi}}}, 21^2 kernel, 49-term ISIS basis, "
                               f"{int(spec.variable_frac * 100)}% variable sources, one HIP graph, "
                               f"FP32 fit",
                   "pairs": len(wls), "total_pixels": int(total_px),
                   "apply_grid": grid, "tile_order": order, "fit_band_rows": band,
                   "plans_by_spatial_order": [sorted({int(pairs[k]["S"]) for k in ix}) for ix in plans],
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3),
                       "max": round(float(lat.max()), 3)},
        "graph_ms_per_step": round(float(np.median(per)), 4),
        "stages_ms": {k: round(float(v), 4) for k, v in
                      zip(["fit", "solve", "patch_kernels_pseudo_matrices", "match_tiles"], stage)},
        "fit": {"solved": int(sum(s["info"] == 0 for s in st)),
                "rejected_stamps": int(sum(s["n_rejected"] for s in st)),
                "solutions": int(sum(s["n_iter"] for s in st)),
                "chi2_dof_median": float(np.median([s["chi2_dof"] for s in st if s["info"] == 0]))},
        "roofline": dict(kernel="k_match_tiles_b<10> (fused I', V', D, masks and per-tile C_D sums "
                                "over the tiles of all pairs)",
                         bound="alu", achieved=round(achieved, 2), peak=FP32_VALU_PEAK_TFLOPS,
                         unit="TFLOP/s", frac=round(achieved / FP32_VALU_PEAK_TFLOPS, 4),
                         traffic=traffic, avg_launch_us=round(tiles_us, 2),
                         algorithmic_flops_per_launch=flops,
                         algorithmic_bytes_per_launch=27.0 * total_px,
                         share_of_step=round(tiles_us * 1e-3 / ms_per_step, 3)),
        "tuning": table,
    }
    if not args.no_extra:
        try:
            out["learned"] = learned_batch_leg(args, torch, psfm, synth, ctx, pairs, wls, st)
        except Exception as e:          # the headline stands without the extra leg
            out["learned"] = {"error": repr(e)}
        try:
            out["compare_precision"] = precision_leg(args, torch, psfm, synth)
        except Exception as e:
            out["compare_precision"] = {"error": repr(e)}
        try:
            out["modes"] = modes_leg(args, torch, psfm, synth)
        except Exception as e:
            out["modes"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        base, par = oracle_batch_baseline(wls, dps, px, st, args.cpu_seconds)
        out["cpu_baseline"] = base
        if par:
            out["parity_vs_oracle"] = par
    print(json.dumps(out), flush=True)


def learned_batch_leg(args, torch, psfm, synth, ctx_b, pairs, wls, st_plain):
    """The learned prior on the batch's pairs: the network is trained on the
    GPU (200k method-solved stamp pairs), then every pair runs the
    single-pair path twice -- fit -> solve -> match, and fit -> predict ->
    solve with the prior -> match -- each timed with HIP events (one warm-up
    run first).  Both legs are sequential single-pair calls, so their Mpix/s
    compare with each other, not with the captured batch."""
    from paper_1901_09999_amd import cnn
    t0 = time.perf_counter()
    net, rep = cnn.fit_prior(n=200_000, seed=11, epochs=8, n_val=10_000)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    ctxs = {}
    acc = dict(px=0.0, plain_ms=0.0, prior_ms=0.0, plain_solve_ms=0.0, prior_solve_ms=0.0,
               predict_ms=0.0, sol_plain=0, sol_prior=0, excluded=0, fallbacks=0, trusted=0,
               stamps=0)
    dchi, dks = [], []
    for k, q in enumerate(pairs):
        S = int(q["S"])
        if S not in ctxs:
            ctxs[S] = psfm.Context(psfm.Config(h=ctx_b.cfg.h, r=ctx_b.cfg.r, S=S))
        ctx = ctxs[S]
        H, W = q["I1"].shape
        n = int(q["stamps"].shape[0])
        bufs = ctx.alloc_pair(W, H, n, 10)

        def leg(use_prior, ev):
            f = ctx.fit_stamps(q["I1"], q["M1"], q["I2"], q["V2"], q["M2"], q["stamps"], out=bufs["fit"])
            ev[0].record()
            pred = None
            if use_prior:
                pred = cnn.predict_local(ctx, net, q["I1"], q["M1"], q["I2"], q["M2"], q["stamps"])
            ev[1].record()
            s = ctx.solve(W, H, q["stamps"], f, flags=f["flags"], out=bufs["sol"], flags_inplace=True,
                          prior=pred)
            ev[2].record()
            ctx.match(s["coeffs"], q["I1"], q["V1"], q["M1"], q["I2"], q["V2"], q["M2"], c_out=10,
                      stats=s["stats"], out=bufs["sub"], cov_conv=bufs["cov"])
            ev[3].record()
            return s

        res = {}
        for use_prior in (False, True):
            for rep_i in range(2):                  # warm-up, then the timed run
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
                ev[4].record()
                s = leg(use_prior, ev[:4])
                ev[3].synchronize()
            st = psfm.read_stats(s["stats"])
            res[use_prior] = dict(total=ev[4].elapsed_time(ev[3]), predict=ev[0].elapsed_time(ev[1]),
                                  solve=ev[1].elapsed_time(ev[2]), st=st)
        a, b = res[False], res[True]
        acc["px"] += W * H
        acc["plain_ms"] += a["total"]
        acc["prior_ms"] += b["total"]
        acc["plain_solve_ms"] += a["solve"]
        acc["prior_solve_ms"] += b["solve"]
        acc["predict_ms"] += b["predict"]
        acc["sol_plain"] += a["st"]["n_iter"]
        acc["sol_prior"] += b["st"]["n_iter"]
        acc["excluded"] += b["st"]["n_prior"]
        acc["fallbacks"] += b["st"]["prior_fallback"]
        acc["trusted"] += b["st"]["n_trusted"]
        acc["stamps"] += n
        if a["st"]["info"] == 0 and b["st"]["info"] == 0:
            dchi.append(b["st"]["chi2_dof"] / a["st"]["chi2_dof"] - 1)
            dks.append(abs(b["st"]["kernel_sum_centre"] / a["st"]["kernel_sum_centre"] - 1))
        del bufs
    for c in ctxs.values():
        c.close()
    return dict(
        train=dict(seconds=round(t_train, 1), stamps=rep["n_train"], epochs=rep["epochs"],
                   train_stamps_per_s=rep["train_samples_per_s"],
                   within_1p05=round(rep["within_1p05"], 3),
                   kernel_sum_err_median=round(rep["kernel_sum_err_median"], 4)),
        pairs=len(pairs),
        plain_sequential_mpix_s=round(acc["px"] / 1e3 / acc["plain_ms"], 1),
        learned_sequential_mpix_s=round(acc["px"] / 1e3 / acc["prior_ms"], 1),
        solve_ms=dict(plain=round(acc["plain_solve_ms"], 3), prior=round(acc["prior_solve_ms"], 3),
                      predict=round(acc["predict_ms"], 3)),
        solutions=dict(plain=acc["sol_plain"], prior=acc["sol_prior"]),
        stamps=acc["stamps"], predictions_kept_by_1p05_rule=acc["trusted"],
        excluded_by_prior=acc["excluded"], fallbacks=acc["fallbacks"],
        chi2_dof_change_median=float(np.median(dchi)) if dchi else None,
        chi2_dof_change_max=float(np.max(dchi)) if dchi else None,
        pairs_with_lower_chi2_dof=int(sum(x < 0 for x in dchi)),
        kernel_sum_change_max=float(np.max(dks)) if dks else None)


def modes_leg(args, torch, psfm, synth, W=2048, H=2048, reps=3):
    """The paper's other modes, each on 2048^2 synthetic images resident in
    HBM, timed with HIP events over `reps` calls after one warm-up:
    both images matched to a common PSF (psfm_fit_dual -> psfm_solve_dual ->
    psfm_dual_subtract, penalty 0.02) beside the single kernel on the same
    orthogonally elongated pair; the normalisation and quality mode (fit,
    unweighted b0/d0 sums, held solve, quality record, match); PSF
    homogenisation of three inputs (envelope, fake target, three matchings,
    outlier rejection, trace-back, stack); binning and image addition
    (HBM-bound: achieved GB/s of their algorithmic bytes)."""
    dev = "cuda"
    rng = np.random.default_rng(5)
    n_src = 3000
    xs = rng.uniform(0, W, n_src)
    ys = rng.uniform(0, H, n_src)
    fl = np.exp(rng.uniform(np.log(1e3), np.log(1e5), n_src))

    def image(psf, theta, seed):
        m = synth._render_torch(torch, W, H, xs, ys, fl, psf, theta, dev).reshape(H, W).double() + 100.0
        g = torch.Generator(device=dev)
        g.manual_seed(seed)
        var = m.abs() + 1.0
        img = m + var.sqrt() * torch.randn((H, W), generator=g, device=dev, dtype=torch.float64)
        return img.float().contiguous(), var.float().contiguous()

    Z = torch.zeros((H, W), dtype=torch.uint8, device=dev)
    R = 30
    st = [(int(xs[i]), int(ys[i])) for i in np.argsort(-fl)
          if R <= xs[i] < W - R and R <= ys[i] < H - R][:200]
    stamps = torch.tensor(st, dtype=torch.int32, device=dev)

    def timed(fn):
        out = fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            out = fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps, out

    res = {}
    # (1) two kernels vs one on orthogonally elongated PSFs
    I1, V1 = image(synth.PsfField(1.8, 1.8, 0.45), 0.0, 1)
    I2, V2 = image(synth.PsfField(1.8, 1.8, 0.45), np.pi / 2, 2)
    ctx = psfm.Context(psfm.Config(S=1))

    def dual():
        f = ctx.fit_dual(I1, Z, I2, V2, Z, stamps)
        s = ctx.solve_dual(W, H, stamps, f, 0.02)
        ctx.dual_subtract(s["coeffs"], I1, V1, Z, I2, V2, Z)
        return s

    def single():
        f = ctx.fit_stamps(I1, Z, I2, V2, Z, stamps)
        s = ctx.solve(W, H, stamps, f)
        ctx.match(s["coeffs"], I1, V1, Z, I2, V2, Z, stats=s["stats"])
        return s

    ms_d, sd = timed(dual)
    ms_s, ss = timed(single)
    a, b = psfm.read_stats(sd["stats"]), psfm.read_stats(ss["stats"])
    res["two_kernels"] = dict(mpix_s=round(W * H / 1e3 / ms_d, 1), ms=round(ms_d, 3),
                              unknowns=ctx.N2, chi2_dof=a["chi2_dof"],
                              single_kernel=dict(mpix_s=round(W * H / 1e3 / ms_s, 1), ms=round(ms_s, 3),
                                                 unknowns=ctx.N, chi2_dof=b["chi2_dof"]))
    # (2) the paper's normalisation and quality mode on a plain pair
    J1, U1 = image(synth.PsfField(1.4, 1.4, 0.0), 0.0, 3)
    J2, U2 = image(synth.PsfField(2.0, 2.2, 0.2), 0.3, 4)

    def paper_mode():
        f = ctx.fit_stamps(J1, Z, J2, U2, Z, stamps)
        nrm = ctx.fit_norm(J1, J2, stamps, f["flags"])
        s = ctx.solve_norm(W, H, stamps, f, nrm)
        q = ctx.quality(s["coeffs"], J1, J2, U2, stamps, s["flags"], soft=0.1)[0]
        ctx.match(s["coeffs"], J1, U1, Z, J2, U2, Z, stats=s["stats"])
        return s, q

    ms_p, (sp, qp) = timed(paper_mode)
    qd = psfm.read_quality(qp)
    res["normalisation_quality_mode"] = dict(mpix_s=round(W * H / 1e3 / ms_p, 1), ms=round(ms_p, 3),
                                             chi2_dof=psfm.read_stats(sp["stats"])["chi2_dof"],
                                             cut_flags=int(qd.get("cut_flags", -1)))
    # (3) homogenisation of three inputs to their envelope, outliers, stack
    psfs = [(synth.PsfField(1.5, 1.5, 0.2), 0.2), (synth.PsfField(1.8, 1.8, 0.1), 1.1),
            (synth.PsfField(1.3, 1.3, 0.3), 2.0)]
    ins = [image(p_, th, 10 + k) for k, (p_, th) in enumerate(psfs)]
    params = []
    for p_, th in psfs:
        sa, sb = p_.params(np.array([W / 2.0]), np.array([H - 1.0]), W, H)
        params.append((float(sa[0]), float(sb[0]), th))
    params_d = torch.tensor(params, dtype=torch.float64, device=dev)
    src_d = torch.tensor(np.stack([xs, ys, fl], axis=1), dtype=torch.float64, device=dev)
    hctx = psfm.Context(psfm.Config(S=1, max_iter=2))

    def homogenise():
        sig, _ = psfm.envelope_psf(params_d, 15)
        target = psfm.render_target(src_d, float(sig[0]), W, H)
        conv, var, co = [], [], []
        for img, v in ins:
            f = hctx.fit_stamps(img, Z, target, v, Z, stamps)
            s = hctx.solve(W, H, stamps, f)
            conv.append(hctx.convolve_image(s["coeffs"], img, Z)[0])
            var.append(hctx.propagate_variance(s["coeffs"], v, Z)[0])
            co.append(s["coeffs"])
        Ic, Vc = torch.stack(conv), torch.stack(var)
        Mc = torch.zeros((3, H, W), dtype=torch.uint8, device=dev)
        outl = psfm.stack_reject(Ic, Vc, Mc, 5.0)
        for k in range(3):
            psfm.trace_mask(hctx, co[k], outl[k], 0.8)
        return psfm.stack_combine(Ic, Vc, Mc)

    ms_h, _ = timed(homogenise)
    res["homogenisation"] = dict(inputs=3, mpix_s=round(3 * W * H / 1e3 / ms_h, 1), ms=round(ms_h, 3))
    # (4) binning and addition (HBM-bound)
    B4 = 4096
    gb = torch.Generator(device=dev)
    gb.manual_seed(7)
    Ib = torch.randn((B4, B4), generator=gb, device=dev).float()
    Vb = torch.rand((B4, B4), generator=gb, device=dev).float() + 1.0
    Mb = torch.zeros((B4, B4), dtype=torch.uint8, device=dev)
    ms_b, _ = timed(lambda: psfm.bin_image(Ib, Vb, Mb, 2, c_out=4))
    ms_a, _ = timed(lambda: psfm.add_images(0.7, Ib, Vb, Mb, None, 1.3, Ib, Vb, Mb, None, 3))
    px = B4 * B4
    bin_bytes = 9 * px + 9 * px / 4              # I, V, M read; binned planes written
    add_bytes = 18 * px + 9 * px                 # two inputs read, S, V_S, M_S written
    res["noise_ops"] = dict(
        image=f"{B4}x{B4}",
        bin2=dict(ms=round(ms_b, 4), gb_s=round(bin_bytes / ms_b / 1e6, 1),
                  hbm_frac=round(bin_bytes / ms_b / 1e6 / HBM_PEAK_GBS, 3)),
        add=dict(ms=round(ms_a, 4), gb_s=round(add_bytes / ms_a / 1e6, 1),
                 hbm_frac=round(add_bytes / ms_a / 1e6 / HBM_PEAK_GBS, 3)))
    ctx.close()
    hctx.close()
    torch.cuda.empty_cache()
    return res


def precision_leg(args, torch, psfm, synth, name="chip4846", steps=5, warmup=2):
    """Plain FP32 vs the 16-bit stamp fits (one refinement step each) on the
    detector-chip pair, each against the FP64 oracle."""
    wl = synth.WORKLOADS[name]
    pair = synth.make_pair(wl, synth.workload_seed(synth.SEED_INDEX[name]))
    d = psfm.to_device(pair)
    res = {}
    for mode in ("fp32", "fp16", "bf16"):
        r = run_pair_mode(torch, psfm, wl, d, mode, 1, steps, warmup, conv_reps=0)
        res[mode] = dict(value=round(wl.pixels / 1e6 / (r["ms_per_step"] * 1e-3), 2),
                         ms_per_step=round(r["ms_per_step"], 4), refine=r["refine"],
                         stages_ms={k: round(float(v), 4) for k, v in
                                    zip(["fit", "solve", "apply"], r["stage"])},
                         kernel_sum_centre=r["stats"]["kernel_sum_centre"],
                         chi2_dof=r["stats"]["chi2_dof"], n_iter=r["stats"]["n_iter"])
    if not args.no_cpu_baseline:
        import oracle as O
        O.build()
        O.set_threads(host_threads())
        ref = O.match_pair(O.Config.from_workload(wl), pair, c_out=wl.cov_half)["stats"]
        for r in res.values():
            r["kernel_sum_rel"] = abs(r["kernel_sum_centre"] / ref["kernel_sum_centre"] - 1)
            r["chi2_dof_rel"] = abs(r["chi2_dof"] / ref["chi2_dof"] - 1)
    del d
    torch.cuda.empty_cache()
    return dict(workload=f"{name}: {wl.width}x{wl.height}, {wl.n_unknowns} unknowns, "
                         f"{wl.n_stamps} stamps of {2 * wl.stamp_half + 1}^2", modes=res)


# multiply-adds per stamp of one training step of the stamp-pair CNN (forward,
# data gradients of layers 2..6 and fc, weight gradients of every layer)
CNN_FWD_MAC = 41 * 41 * 32 * 2 * 9 + 21 * 21 * 32 * 32 * 9 + 11 * 11 * 32 * 32 * 9 + 6 * 6 * 32 * 32 * 9 \
    + 1152 * 128 + 128 * 49
CNN_TRAIN_FLOP = 2 * (2 * CNN_FWD_MAC + (CNN_FWD_MAC - 41 * 41 * 32 * 2 * 9))


def bench_cells(args, torch, psfm, synth):
    from paper_1901_09999_amd import cnn
    B = 256
    n_data = 25_000
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    data = cnn.make_dataset(n_data, seed=synth.workload_seed(synth.SEED_INDEX["cells200k"]))
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    z = cnn.standardize(data)
    n = z["x"].shape[0]
    net = cnn.Net(seed=1)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    g = torch.Generator(device="cpu")
    g.manual_seed(0)
    batches = [torch.randint(0, n, (B,), generator=g).cuda() for _ in range(8)]

    def step(k):
        idx = batches[k % len(batches)]
        net.loss_grad(z["x"][idx], z["target"][idx], loss, z["weight"][idx])
        net.adam(1e-3)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(args.steps):
        step(k)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    rate = B / (ms * 1e-3)
    achieved = CNN_TRAIN_FLOP * B / (ms * 1e-3) / 1e12

    # the prior in use (after a few untimed epochs, so that the predictions
    # mean something): plain solve and solve with the predicted kernels on one pair
    cnn.train(net, z, epochs=4, batch=B)
    wl = synth.scaled(synth.WORKLOADS["pair2048"], "prior", 1024, 1024, n_stamps=150, spatial_order=2,
                      variable_frac=0.10)
    pair = synth.make_pair(wl, synth.workload_seed(synth.SEED_INDEX["cells200k"], 1))
    d = psfm.to_device(pair)
    ctx = psfm.Context(psfm.Config.from_workload(wl))
    fit = ctx.fit_stamps(d["I1"], d["M1"], d["I2"], d["V2"], d["M2"], d["stamps"])
    net.fold_output(z["mu"], z["sd"])

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    t_plain = timed(lambda: ctx.solve(wl.width, wl.height, d["stamps"], fit))
    t_pred = timed(lambda: cnn.predict_local(ctx, net, d["I1"], d["M1"], d["I2"], d["M2"], d["stamps"]))
    pred = cnn.predict_local(ctx, net, d["I1"], d["M1"], d["I2"], d["M2"], d["stamps"])
    t_prior = timed(lambda: ctx.solve(wl.width, wl.height, d["stamps"], fit, prior=pred))
    sp = psfm.read_stats(ctx.solve(wl.width, wl.height, d["stamps"], fit)["stats"])
    sq = psfm.read_stats(ctx.solve(wl.width, wl.height, d["stamps"], fit, prior=pred)["stats"])

    out = {
        "metric": "CNN training throughput (learned prior)",
        "value": round(rate, 1),
        "unit": "stamps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16 storage, f32 accumulate",
        "data": "synthetic",
        "config": {"workload": f"cells200k: single-star 64x64 cells with neighbours, 41x41 stamp pairs, "
                               f"batch {B}; dataset of {n} stamps from {n_data} cells"},
        "roofline": dict(kernel="whole training step (forward, backward, Adam; the weight-gradient "
                                "kernels hold most of it)", bound="alu",
                         achieved=round(achieved, 3), peak=FP32_VALU_PEAK_TFLOPS, unit="TFLOP/s",
                         frac=round(achieved / FP32_VALU_PEAK_TFLOPS, 4), traffic=None,
                         algorithmic_flops_per_stamp=CNN_TRAIN_FLOP),
        "dataset": {"stamps_per_s": round(n_data / t_data, 1), "seconds": round(t_data, 3)},
        "prior": {"solve_ms": round(t_plain, 3), "predict_ms": round(t_pred, 3),
                  "solve_prior_ms": round(t_prior, 3), "stamps": int(pair.stamps.shape[0]),
                  "solutions_plain": int(sp["n_iter"]), "solutions_prior": int(sq["n_iter"]),
                  "prior_excluded": int(sq["n_prior"]), "restored": int(sq["n_restored"]),
                  "chi2_dof_plain": round(float(sp["chi2_dof"]), 5),
                  "chi2_dof_prior": round(float(sq["chi2_dof"]), 5)},
    }
    if not args.no_cpu_baseline:
        from oracle import cnn_oracle as CO
        xs = z["x"][batches[0][:8]].float().cpu().numpy().astype(np.float64)
        ts = z["target"][batches[0][:8]].cpu().numpy().astype(np.float64)
        wt = z["weight"][batches[0][:8]].cpu().numpy().astype(np.float64)
        theta = CO.init_params(1)
        m, v = np.zeros_like(theta), np.zeros_like(theta)
        done, c0, w0 = 0, time.process_time(), time.perf_counter()
        while done == 0 or (time.perf_counter() - w0 < args.cpu_seconds and done < 400):
            _, gr = CO.loss_and_grad(theta, xs, ts, wt)
            theta, m, v = CO.adam_step(theta, m, v, gr, done + 1, lr=1e-3)
            done += xs.shape[0]
        wall, cpu = time.perf_counter() - w0, time.process_time() - c0
        out["cpu_baseline"] = dict(value=round(done / wall, 2), unit="stamps/s",
                                   cores=max(1, int(round(cpu / wall))), kind="oracle",
                                   sample=f"FP64 NumPy loss, gradient and Adam step on batches of "
                                          f"{xs.shape[0]} stamps, {done} stamps in {wall:.1f} s")
    print(json.dumps(out), flush=True)


PRECS = {"fp32": 0, "bf16": 1, "fp16": 2}


def run_pair_mode(torch, psfm, wl, d, prec_name, refine, steps, warmup, conv_reps=20):
    """fit -> solve -> match on one resident pair in one stamp-fit arithmetic:
    wall ms per step, GPU ms per step, the stage split and the stats."""
    W, H, n = wl.width, wl.height, int(d["stamps"].shape[0])
    prec = PRECS[prec_name]
    ctx = psfm.Context(psfm.Config.from_workload(wl, precision=prec, refine=refine))
    bufs = ctx.alloc_pair(W, H, n, wl.cov_half)

    def step(ev=None):
        f = ctx.fit_stamps(d["I1"], d["M1"], d["I2"], d["V2"], d["M2"], d["stamps"], out=bufs["fit"])
        if ev: ev[0].record()
        # the fit rewrites every stamp's flags, so the solve marks its
        # rejections in them (no copy)
        s = ctx.solve(W, H, d["stamps"], f, flags=f["flags"], out=bufs["sol"], flags_inplace=True)
        if ev: ev[1].record()
        # convolutions of I1 and V1 and the difference in one pass over the
        # tiles (the convolved planes are not stored: the difference is the product)
        ctx.match(s["coeffs"], d["I1"], d["V1"], d["M1"], d["I2"], d["V2"], d["M2"],
                  c_out=wl.cov_half, stats=s["stats"], out=bufs["sub"], cov_conv=bufs["cov"])
        if ev: ev[2].record()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # the timed steps carry no events of their own (a timing event between
    # stages idles the GPU for a few microseconds)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for k in range(steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = float(start.elapsed_time(stop)) / steps
    # stage split: the same number of steps again, with an event after each stage
    NS = 3      # stages: fit, solve, apply (convolutions, pseudo-matrices, difference)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(NS)] for _ in range(steps)]
    start.record()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    stage = np.zeros(NS)
    for k in range(steps):
        prev = start if k == 0 else evs[k - 1][NS - 1]
        marks = [prev] + evs[k]
        stage += [marks[i].elapsed_time(marks[i + 1]) for i in range(NS)]
    stage /= steps
    stats = psfm.read_stats(bufs["sol"]["stats"])
    conv_ms = None
    if conv_reps:
        # the image convolution alone (its own launches, HIP events), for its roofline
        s = bufs["sol"]
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        for _ in range(conv_reps):
            ctx.convolve_image(s["coeffs"], d["I1"], d["M1"], out=bufs["conv"], out_mask=bufs["conv_mask"])
        c1.record()
        torch.cuda.synchronize()
        conv_ms = c0.elapsed_time(c1) / conv_reps
    ctx.close()
    return dict(ms_per_step=1e3 * wall / steps, stage=stage, gpu_ms=gpu_ms, stats=stats,
                refine=refine, conv_ms=conv_ms)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "psfm runs on one GPU; --gpus must be 1 "
                                   "(sharding over several GPUs is not implemented)"}))
        sys.exit(2)
    import torch
    from paper_1901_09999_amd import psfm, synth

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a HIP device")
    if args.copy_mb > 0:
        src = torch.empty(args.copy_mb << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)             # one plain elementwise kernel: read N, write N
        torch.cuda.synchronize()
        log(f"calibration copy: {args.copy_mb} MiB read + {args.copy_mb} MiB written")
        del src, dst
    if args.workload in synth.BATCHES:
        return bench_batch(args, torch, psfm, synth)
    if args.workload in synth.STAMP_SETS:
        return bench_cells(args, torch, psfm, synth)
    wl = synth.WORKLOADS[args.workload]
    seed_index = synth.SEED_INDEX[args.workload]
    pair = synth.make_pair(wl, synth.workload_seed(seed_index))
    d = psfm.to_device(pair)
    W, H, n = wl.width, wl.height, pair.stamps.shape[0]
    def run_mode(name, steps, warmup):
        refine = args.refine if args.refine is not None else 1
        return run_pair_mode(torch, psfm, wl, d, name, refine, steps, warmup)

    main_run = run_mode(args.precision, args.steps, args.warmup)
    other = None
    if not args.no_compare:
        other_name = "fp16" if args.precision == "fp32" else "fp32"
        other = (other_name, run_mode(other_name, args.steps, args.warmup))
    ms_per_step, stage, gpu_ms, stats = (main_run["ms_per_step"], main_run["stage"],
                                         main_run["gpu_ms"], main_run["stats"])

    # rooflines: the FP64 Cholesky (one per solution, latency-bound) and the
    # image convolution (one launch per step, FP32 VALU-bound)
    conv_us = main_run["conv_ms"] * 1e3
    T = (2 * wl.kernel_half + 1) ** 2
    flops = 2.0 * T * W * H
    achieved = flops / (conv_us * 1e-6) / 1e12
    traffic = measured_traffic("conv_tile_pair2048_traffic.json" if wl.name == "pair2048" else "-",
                               os.path.join(ROOT, "paper_1901_09999_amd", "csrc", "convolve.hip"))
    roof_conv = dict(kernel="k_conv_tile<h, 0> (image convolution)", bound="alu",
                     achieved=round(achieved, 2), peak=FP32_VALU_PEAK_TFLOPS, unit="TFLOP/s",
                     frac=round(achieved / FP32_VALU_PEAK_TFLOPS, 4), traffic=traffic,
                     avg_launch_us=round(conv_us, 2), algorithmic_flops_per_launch=flops,
                     launches_per_step=0,
                     note="timed in launches of its own; the step forms the image and variance "
                          "planes and the difference in one fused tile kernel (k_match_tile)")
    Nu = wl.n_unknowns
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    A = torch.randn((Nu, Nu), generator=g, dtype=torch.float64, device="cuda")
    Mspd = (A @ A.T + Nu * torch.eye(Nu, dtype=torch.float64, device="cuda")).contiguous()
    bvec = torch.ones(Nu, dtype=torch.float64, device="cuda")
    xw, infow = torch.empty_like(bvec), torch.zeros(1, dtype=torch.int32, device="cuda")
    cws = torch.empty(int(psfm.lib().psfm_cholesky_workspace_bytes(Nu)), dtype=torch.uint8, device="cuda")
    for _ in range(3):
        psfm.cholesky_solve(Mspd, bvec, xw, infow, cws)
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        psfm.cholesky_solve(Mspd, bvec, xw, infow, cws)
    e1.record()
    torch.cuda.synchronize()
    chol_us = e0.elapsed_time(e1) * 1e3 / reps
    chol_flops = Nu ** 3 / 3.0 + 2.0 * Nu ** 2
    chol_per_step = stats["n_iter"]
    roof_chol = dict(kernel=f"k_cholesky<true> (FP64 equilibrated Cholesky + substitutions, N={Nu})",
                     bound="mfma", achieved=round(chol_flops / (chol_us * 1e-6) / 1e12, 4),
                     peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                     frac=round(chol_flops / (chol_us * 1e-6) / 1e12 / FP64_PEAK_TFLOPS, 6),
                     traffic=measured_traffic(f"cholesky_n{Nu}_traffic.json",
                                              os.path.join(ROOT, "paper_1901_09999_amd", "csrc", "solve.hip")),
                     avg_launch_us=round(chol_us, 2),
                     algorithmic_flops_per_launch=chol_flops, launches_per_step=chol_per_step)
    share_chol = chol_per_step * chol_us / (gpu_ms * 1e3)
    share_conv = conv_us / (gpu_ms * 1e3)
    roof, roof_other = (roof_chol, roof_conv) if share_chol >= share_conv else (roof_conv, roof_chol)
    roof["share_of_step"] = round(max(share_chol, share_conv), 3)
    roof_other["share_of_step"] = round(min(share_chol, share_conv), 3)

    out = {
        "metric": METRIC,
        "value": round(W * H / 1e6 / (ms_per_step * 1e-3), 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else f"{args.precision} gram, f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {W}x{H} FP32 pair, {wl.n_sources} sources, "
                               f"{int(wl.mask_frac * 100)}% mask, {2 * wl.kernel_half + 1}^2 kernel, "
                               f"{wl.n_basis}-term ISIS basis x spatial order {wl.spatial_order} "
                               f"({wl.n_unknowns} unknowns), {n} stamps of {2 * wl.stamp_half + 1}^2, "
                               f"{args.precision} stamp fit",
                   "width": W, "height": H, "n_stamps": n, "unknowns": wl.n_unknowns,
                   "parallelism": "single GPU"},
        "stages_ms": {k: round(float(v), 4) for k, v in
                      zip(["fit", "solve", "apply"], stage)},
        "gpu_ms_per_step": round(gpu_ms, 4),
        "fit": {"chi2_dof": stats["chi2_dof"], "kernel_sum_centre": stats["kernel_sum_centre"],
                "n_used": stats["n_used"], "n_iter": stats["n_iter"]},
        "roofline": roof,
        "roofline_other": roof_other,
    }
    if other is not None:
        o = other[1]
        out["compare"] = {"precision": other[0], "refine": o["refine"],
                          "value": round(W * H / 1e6 / (o["ms_per_step"] * 1e-3), 2),
                          "ms_per_step": round(o["ms_per_step"], 4),
                          "stages_ms": {k: round(float(v), 4) for k, v in
                                        zip(["fit", "solve", "apply"],
                                            o["stage"])},
                          "fit": {"chi2_dof": o["stats"]["chi2_dof"],
                                  "kernel_sum_centre": o["stats"]["kernel_sum_centre"],
                                  "n_used": o["stats"]["n_used"]}}
    if not args.no_cpu_baseline:
        base, res = cpu_baseline(wl, pair, args.cpu_seconds)
        out["cpu_baseline"] = base
        ref = res["stats"]
        out["parity_vs_oracle"] = {
            "kernel_sum_rel": abs(stats["kernel_sum_centre"] / ref["kernel_sum_centre"] - 1),
            "chi2_dof_rel": abs(stats["chi2_dof"] / ref["chi2_dof"] - 1)}
        if other is not None:
            os_ = other[1]["stats"]
            out["compare"]["parity_vs_oracle"] = {
                "kernel_sum_rel": abs(os_["kernel_sum_centre"] / ref["kernel_sum_centre"] - 1),
                "chi2_dof_rel": abs(os_["chi2_dof"] / ref["chi2_dof"] - 1)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
