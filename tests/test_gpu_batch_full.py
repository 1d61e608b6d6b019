"""The batch at its full size, in the launch configuration the benchmark
times: the 64 pairs of the batch64 workload (sides U{1024..6000}, 50 to 400
stamps, spatial orders 0 to 3, 734 Mpx in all), the tuner's fit band height,
apply grid and pair order, one captured HIP graph, replayed.

The oracle cannot run 734 Mpx in seconds, so the checks sample:
  * whole path on sampled pairs (the largest, the one with most stamps and
    the largest of each spatial order): the oracle fits all their stamps and
    solves; the batch's kernel sum (1e-4 relative) and chi2/dof (1%) and the
    stamps' validity bits (exact) against it;
  * the batch against single-pair calls on the largest pair (same device
    code per pair, so coefficients, flags and the difference planes are
    equal bit for bit: a property at any size);
  * the benchmark's schedule (the batch split by spatial order into plans
    that run as the branches of one graph) against the one-plan batch on
    every pair, bit for bit;
  * the tile kernels against the oracle on the largest pair from the
    oracle's coefficients: sampled rectangles (the four corners, which hold
    the ragged right and bottom tails, a patch corner, the brightest source
    and random interior spots) of the convolved image (2e-5 of the largest
    convolved value), its variance (1e-5 relative) and mask (exact), and of
    the difference image (2e-5 of that scale plus one rounding of I2) with
    its variance and mask.
"""
import numpy as np
import pytest

import oracle as O
from paper_1901_09999_amd import synth

from gpu_common import hip

pytestmark = pytest.mark.gpu

VALIDITY = 1 | 4          # PSFM_STAMP_INVALID | PSFM_STAMP_NONFINITE: decided by the fit alone


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def full():
    """(workloads, device pairs, pair dicts, the replayed batch, the tuning);
    the batch's device memory is released after the module."""
    torch, psfm = hip()
    from paper_1901_09999_amd import tune

    print("generating the batch64 pairs", flush=True)
    wls, dps = synth.make_batch_device("batch64")
    spec = synth.BATCHES["batch64"]
    ctx = psfm.Context(psfm.Config(h=spec.kernel_half, r=spec.stamp_half, S=0))
    pairs = [dict(I1=d.I1, V1=d.V1, M1=d.M1, I2=d.I2, V2=d.V2, M2=d.M2,
                  stamps=torch.from_numpy(d.stamps.astype(np.int32)).cuda(), S=d.workload.spatial_order)
             for d in dps]
    print("tuning", flush=True)
    tu = tune.choose(ctx, pairs, c_out=10)
    ctx = tune.context_for(ctx, tu["fit_band_rows"])
    b = psfm.Batch(ctx, pairs, c_out=10, apply_grid=tu["apply_grid"], order=tu["order"])
    b.capture()
    for _ in range(2):
        b.launch()
    torch.cuda.synchronize()
    print(f"batch of {len(wls)} pairs run: grid {tu['apply_grid']}, order {tu['order']}, "
          f"fit band rows {tu['fit_band_rows']}", flush=True)
    yield wls, dps, pairs, b, tu
    b.close()
    _ORACLE.clear()
    del b, pairs, dps
    torch.cuda.empty_cache()


_ORACLE = {}


def _oracle_solve(full, k):
    if k in _ORACLE:
        return _ORACLE[k]
    wls, dps = full[0], full[1]
    wl, hp = wls[k], dps[k].host()
    cfg = O.Config.from_workload(wl)
    fit = O.fit_stamps(cfg, hp.I1, hp.M1, hp.I2, hp.V2, hp.M2, hp.stamps)
    ret, a, chi2, flags, st = O.solve(cfg, wl.width, wl.height, hp.stamps, fit)
    _ORACLE[k] = (cfg, hp, ret, a, flags, st)
    return _ORACLE[k]


def _sampled_pairs(wls):
    px = [wl.width * wl.height for wl in wls]
    pick = {int(np.argmax(px)), int(np.argmax([wl.n_stamps for wl in wls]))}
    for S in range(4):
        ks = [k for k, wl in enumerate(wls) if wl.spatial_order == S]
        if ks:
            pick.add(max(ks, key=lambda k: px[k]))
    return sorted(pick)


def test_full_batch_whole_path_on_sampled_pairs(full):
    torch, psfm = hip()
    wls, dps, pairs, b, tu = full
    for k in _sampled_pairs(wls):
        wl = wls[k]
        print(f"pair {k}: {wl.width}x{wl.height}, S={wl.spatial_order}, {len(dps[k].stamps)} stamps",
              flush=True)
        cfg, hp, ret, a, flags, rs = _oracle_solve(full, k)
        st = b.stats(k)
        assert ret == 0 and st["info"] == 0
        ks = abs(st["kernel_sum_centre"] / rs["kernel_sum_centre"] - 1)
        cd = abs(st["chi2_dof"] / rs["chi2_dof"] - 1)
        print(f"  kernel sum {ks:.2e}, chi2/dof {cd:.2e}, used {st['n_used']} ({rs['n_used']})", flush=True)
        assert ks < 1e-4 and cd < 1e-2
        fl = _np(b.out[k]["flags"])[:len(flags)]
        assert np.array_equal(fl & VALIDITY, flags & VALIDITY)


def _largest(wls):
    return int(np.argmax([wl.width * wl.height for wl in wls]))


def test_full_batch_equals_single_pair_calls_on_the_largest_pair(full):
    torch, psfm = hip()
    wls, dps, pairs, b, tu = full
    k = _largest(wls)
    wl, q = wls[k], pairs[k]
    ctx = psfm.Context(psfm.Config(h=wl.kernel_half, r=wl.stamp_half, S=wl.spatial_order,
                                   fit_band_rows=tu["fit_band_rows"]))
    r = ctx.match_pair(q["I1"], q["V1"], q["M1"], q["I2"], q["V2"], q["M2"], q["stamps"], c_out=10)
    torch.cuda.synchronize()
    o = b.out[k]
    n = q["stamps"].shape[0]
    assert np.array_equal(_np(o["coeffs"]), _np(r["sol"]["coeffs"]))
    assert np.array_equal(_np(o["flags"])[:n], _np(r["sol"]["flags"])[:n])
    for key in ("diff", "diff_var", "diff_mask"):
        assert np.array_equal(_np(o[key]), _np(r[key])), key


def _rects(wl, I1, rng, side=40):
    W, H = wl.width, wl.height
    P = wl.patch
    rects = [(0, 0), (W - side, 0), (0, H - side), (W - side, H - side),
             ((W // 2) // P * P - side // 2, (H // 2) // P * P - side // 2)]
    finite = np.where(np.isfinite(I1), I1, -np.inf)
    yb, xb = np.unravel_index(np.argmax(finite), I1.shape)
    rects.append((int(np.clip(xb - side // 2, 0, W - side)), int(np.clip(yb - side // 2, 0, H - side))))
    for _ in range(4):
        rects.append((int(rng.integers(0, W - side)), int(rng.integers(0, H - side))))
    return [(x, y, x + side, y + side) for x, y in rects]


def test_full_size_tiles_against_oracle_rectangles(full):
    torch, psfm = hip()
    wls, dps, pairs, b, tu = full
    k = _largest(wls)
    wl, q = wls[k], pairs[k]
    cfg, hp, ret, a, _, _ = _oracle_solve(full, k)
    assert ret == 0
    ctx = psfm.Context(psfm.Config(h=wl.kernel_half, r=wl.stamp_half, S=wl.spatial_order))
    conv = torch.empty_like(q["I1"])
    cm = torch.empty_like(q["M1"])
    var = torch.empty_like(q["V1"])
    r = ctx.match(torch.from_numpy(a).cuda(), q["I1"], q["V1"], q["M1"], q["I2"], q["V2"], q["M2"],
                  c_out=10, conv=conv, conv_mask=cm, conv_var=var)
    torch.cuda.synchronize()
    c_g, cm_g, v_g = _np(conv), _np(cm), _np(var)
    D_g, VD_g, MD_g = _np(r["diff"]), _np(r["diff_var"]), _np(r["diff_mask"])
    rects = _rects(wl, hp.I1, np.random.default_rng(k))
    refs = [O.convolve_region(cfg, a, hp.I1, hp.V1, hp.M1, rc) for rc in rects]
    scale = max(float(np.max(np.abs(ref[0]))) for ref in refs)
    print(f"pair {k} ({wl.width}x{wl.height}): {len(rects)} rectangles, scale {scale:.3g}", flush=True)
    for (x0, y0, x1, y1), (c_r, m_r, v_r) in zip(rects, refs):
        sl = (slice(y0, y1), slice(x0, x1))
        assert np.array_equal(cm_g[sl], m_r), (x0, y0)
        ok = m_r == 0
        assert np.max(np.abs(c_g[sl][ok] - c_r[ok]), initial=0.0) < 2e-5 * scale, (x0, y0)
        assert np.max(np.abs(v_g[sl][ok] - v_r[ok]) / np.abs(v_r[ok]), initial=0.0) < 1e-5, (x0, y0)
        I2, V2, M2 = hp.I2[sl], hp.V2[sl], hp.M2[sl]
        cc = np.zeros((21, 21))
        cc[10, 10] = 1.0
        D_r, VD_r, MD_r, _ = O.subtract(cfg, a, I2, V2, M2, c_r, v_r, m_r, cc)
        assert np.array_equal(MD_g[sl], MD_r), (x0, y0)
        okd = MD_r == 0
        tol = 2e-5 * scale + 1e-6 * np.abs(I2[okd])
        assert np.all(np.abs(D_g[sl][okd] - D_r[okd]) <= tol), (x0, y0)
        assert np.max(np.abs(VD_g[sl][okd] - VD_r[okd]) / np.abs(VD_r[okd]), initial=0.0) < 1e-5


def test_full_batch_split_schedule_equals_one_plan(full):
    """The schedule the benchmark times: the batch split by spatial order
    (the tuner's choice, else orders 3 and 2 each alone) into plans that run
    as the parallel branches of one graph.  Every pair's coefficients, stamp
    flags and difference planes equal the one-plan batch's bit for bit."""
    torch, psfm = hip()
    wls, dps, pairs, b, tu = full
    groups = tu.get("groups") or [[3], [2]]
    plans = psfm.split_by_order(pairs, groups)
    assert sorted(k for ix in plans for k in ix) == list(range(len(pairs)))
    ctx = b.ctx
    subs = [psfm.Batch(ctx, [pairs[k] for k in ix], c_out=10, apply_grid=tu["apply_grid"],
                       order=tu["order"]) for ix in plans]
    grp = psfm.BatchGroup(subs)
    for _ in range(2):
        grp.launch()
    torch.cuda.synchronize()
    print(f"{len(plans)} plans: {[len(ix) for ix in plans]} pairs", flush=True)
    for ix, sb in zip(plans, subs):
        for j, k in enumerate(ix):
            o, r = sb.out[j], b.out[k]
            n = pairs[k]["stamps"].shape[0]
            assert torch.equal(o["coeffs"], r["coeffs"]), k
            assert torch.equal(o["flags"][:n], r["flags"][:n]), k
            for f in ("diff", "diff_var", "diff_mask", "cov_diff"):
                assert torch.equal(o[f], r[f]), (k, f)
    grp.close()
    for sb in subs:
        sb.close()
    del grp, subs
    torch.cuda.empty_cache()
