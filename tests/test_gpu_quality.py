"""The paper's normalisation and quality mode on the GPU (Sections 3.2, 3.3,
3.6, 3.7) against the FP64 oracle, through the C interface.

Tolerances: the normalisation sums are FP64 sums of FP64 products of the
same FP32 inputs in another order (1e-10 relative); b0 and d0 come from
them (1e-9); the held solve starts from the FP32-MFMA stamp Grams, so the
whole-path targets apply (kernel sum 1e-4 relative -- here b0 itself --,
chi2/dof 1%); stamp decisions (rejections, replacements) are compared
exactly; the quality record's deviations are FP64 pixel sums of an FP64
model (1e-9), moments and the deconvolution fraction 1e-10, cut bits exact.
"""
import numpy as np
import pytest

import oracle as O
from paper_1901_09999_amd import synth

from gpu_common import hip

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _pair(W=1024, H=1024, n=150, S=1, seed=61, var=0.08):
    wl = synth.scaled(synth.WORKLOADS["pair2048"], f"q{W}x{H}", W, H, n_stamps=n, spatial_order=S,
                      variable_frac=var)
    return wl, synth.make_pair(wl, seed)


def _groups(n, n_res):
    """The last n_res stamps are reserves of the groups of the first ones
    (group of stamp k = k for the primaries)."""
    group = np.arange(n, dtype=np.int32)
    prim = n - n_res
    group[prim:] = np.arange(n_res, dtype=np.int32) % prim
    return group


def test_fit_norm_matches_oracle():
    torch, psfm = hip()
    wl, pair = _pair()
    ctx = psfm.Context(psfm.Config.from_workload(wl))
    d = psfm.to_device(pair)
    fit = ctx.fit_stamps(d["I1"], d["M1"], d["I2"], d["V2"], d["M2"], d["stamps"])
    fl = fit["flags"].clone()
    fl[-10:] = torch.where(fl[-10:] == 0, torch.full_like(fl[-10:], psfm.STAMP_RESERVE), fl[-10:])
    norm = _np(ctx.fit_norm(d["I1"], d["I2"], d["stamps"], fl))
    ref = O.fit_norm(O.Config.from_workload(wl), pair.I1, pair.I2, pair.stamps, _np(fl))
    assert np.array_equal(norm == 0, ref == 0)
    ok = ref[:, 0] > 0
    assert ok.sum() > 100 and (ok[-10:]).sum() > 0          # reserves keep their sums
    err = np.abs(norm[ok] - ref[ok]) / np.maximum(np.abs(ref[ok]), 1.0)
    print(f"normalisation sums: max relative error {err.max():.2e}")
    assert err.max() < 1e-10


@pytest.mark.parametrize("with_groups", [False, True])
def test_solve_norm_matches_oracle(with_groups):
    torch, psfm = hip()
    wl, pair = _pair()
    cfg = O.Config.from_workload(wl)
    ctx = psfm.Context(psfm.Config.from_workload(wl))
    d = psfm.to_device(pair)
    n = pair.stamps.shape[0]
    fit = ctx.fit_stamps(d["I1"], d["M1"], d["I2"], d["V2"], d["M2"], d["stamps"])
    ofit = O.fit_stamps(cfg, pair.I1, pair.M1, pair.I2, pair.V2, pair.M2, pair.stamps)
    assert np.array_equal(_np(fit["flags"]), ofit["flags"])
    flags = ofit["flags"].copy()
    group = None
    if with_groups:
        group = _groups(n, 40)
        flags[n - 40:] = np.where(flags[n - 40:] == 0, O.STAMP_RESERVE, flags[n - 40:])
    fl_d = torch.from_numpy(flags).cuda()
    norm = ctx.fit_norm(d["I1"], d["I2"], d["stamps"], fl_d)
    onorm = O.fit_norm(cfg, pair.I1, pair.I2, pair.stamps, flags)
    sol = ctx.solve_norm(wl.width, wl.height, d["stamps"], fit, norm, flags=fl_d,
                         group=None if group is None else torch.from_numpy(group).cuda())
    st = psfm.read_stats(sol["stats"])
    ret, a, chi2, ofl, ost, nrep = O.solve_norm(cfg, wl.width, wl.height, pair.stamps, ofit, onorm,
                                                flags=flags, group=group)
    assert ret == 0 and st["info"] == 0
    g = _np(sol["coeffs"])
    print(f"groups={with_groups}: b0 {g[0]:.6f} (oracle {a[0]:.6f}), d0 {g[-1]:.4f} ({a[-1]:.4f}); "
          f"used {st['n_used']} ({ost['n_used']}), rejected {st['n_rejected']} ({ost['n_rejected']}), "
          f"replaced {st['n_replaced']} ({nrep}); chi2/dof {st['chi2_dof']:.5f} ({ost['chi2_dof']:.5f})")
    assert abs(g[0] / a[0] - 1) < 1e-9 and abs(g[-1] - a[-1]) < 1e-6 * max(1.0, abs(a[-1]))
    assert np.all(g[1:cfg.n_spatial] == 0.0)
    assert abs(st["kernel_sum_centre"] / ost["kernel_sum_centre"] - 1) < 1e-4
    assert abs(st["chi2_dof"] / ost["chi2_dof"] - 1) < 1e-2
    assert np.array_equal(_np(sol["flags"]), ofl)
    assert st["n_replaced"] == nrep and st["n_rejected"] == ost["n_rejected"]
    assert st["dof"] == ost["dof"]
    if with_groups:
        assert nrep > 0


def test_quality_matches_oracle():
    torch, psfm = hip()
    wl, pair = _pair(S=2, seed=63)
    cfg = O.Config.from_workload(wl)
    ref = O.match_pair(cfg, pair, c_out=wl.cov_half)
    ctx = psfm.Context(psfm.Config.from_workload(wl))
    d = psfm.to_device(pair)
    a = torch.from_numpy(ref["coeffs"]).cuda()
    fl = torch.from_numpy(ref["flags"]).cuda()
    for soft in (0.0, 0.05):
        q, dev = ctx.quality(a, d["I1"], d["I2"], d["V2"], d["stamps"], fl, soft=soft)
        qg = psfm.read_quality(q)
        qo, devo = O.quality(cfg, ref["coeffs"], pair.I1, pair.I2, pair.V2, pair.stamps, ref["flags"],
                             soft=soft)
        dg = _np(dev)
        print(f"soft {soft}: {qg}")
        assert np.array_equal(dg == 0, devo == 0)
        assert np.max(np.abs(dg - devo) / np.maximum(devo, 1e-30)) < 1e-9
        for k in ("dev_mean", "dev_rms"):
            assert abs(qg[k] - qo[k]) < 1e-9 * max(1.0, abs(qo[k])), k
        for k in ("kernel_sum", "mom_x", "mom_y", "mom_xx", "mom_yy", "deconv_max"):
            assert abs(qg[k] - qo[k]) < 1e-10 * max(1.0, abs(qo[k])), k
        assert qg["n_used"] == qo["n_used"] and qg["cut_flags"] == qo["cut_flags"]
    # soft = 0: the pixel pass equals the solve's own chi2 / npix
    q, dev = ctx.quality(a, d["I1"], d["I2"], d["V2"], d["stamps"], fl, soft=0.0)
    used = ref["flags"] == 0
    c2 = ref["chi2"][used] / ref["fit"]["npix"][used]
    assert np.max(np.abs(_np(dev)[used] / c2 - 1)) < 1e-8
