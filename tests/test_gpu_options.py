"""Configuration options of the C interface against the FP64 oracle:
the fit weights 1 / (V1 + V2) (weight_mode), the solve in the
orthonormalised basis (ortho_basis), PSFM_SYNC's returned device status, the
two fit band heights (fit_band_rows) and the tuner that picks among them.

Tolerances are those of the default options (the same arithmetic runs):
stamp sums within 2e-5 of their Cauchy-Schwarz scale, e_s 1e-5 relative; a
solve from identical sums keeps every stamp decision, kernel sum and chi2/dof
within 1e-9 relative and coefficients within 1e-5 of max|a|; the whole path
within 1e-4 (kernel sum) and 1% (chi2/dof).
"""
import numpy as np
import pytest

import oracle as O
from paper_1901_09999_amd import synth

from gpu_common import hip, norm_err_M, oracle_run, pair_for

pytestmark = pytest.mark.gpu

SEED = synth.workload_seed(0)


def _np(t):
    return t.detach().cpu().numpy()


def _sums_close(fit, ref):
    assert np.array_equal(_np(fit["flags"]), ref["flags"])
    assert np.array_equal(_np(fit["npix"]), ref["npix"])
    err = norm_err_M(_np(fit["M"]), ref["M"])
    assert err < 2e-5, err
    Md = np.sqrt(np.einsum("sii->si", ref["M"]))
    den = Md * np.sqrt(np.maximum(ref["e"], 1e-300))[:, None]
    den[den == 0] = 1
    assert np.max(np.abs(_np(fit["b"]) - ref["b"]) / den) < 2e-5
    ok = ref["e"] > 0
    assert np.max(np.abs(_np(fit["e"])[ok] - ref["e"][ok]) / ref["e"][ok]) < 1e-5
    return err


def test_weight_mode_v1v2_fit_and_whole_path():
    torch, psfm = hip()
    wl, pair = pair_for("pair512", SEED)
    cfg = O.Config.from_workload(wl)
    ctx = psfm.Context(psfm.Config.from_workload(wl, weight_mode=psfm.WEIGHT_V1V2))
    d = psfm.to_device(pair)
    fit = ctx.fit_stamps(d["I1"], d["M1"], d["I2"], d["V2"], d["M2"], d["stamps"], V1=d["V1"])
    ref = O.fit_stamps(cfg, pair.I1, pair.M1, pair.I2, pair.V2, pair.M2, pair.stamps, V1=pair.V1)
    err = _sums_close(fit, ref)
    print(f"weights 1/(V1+V2): Gram normalised error {err:.2e}")
    # the whole path (fit -> solve) against the oracle's solve of its own sums
    sol = ctx.solve(wl.width, wl.height, d["stamps"], fit)
    st = psfm.read_stats(sol["stats"])
    ret, a, _, _, rs = O.solve(cfg, wl.width, wl.height, pair.stamps, ref)
    assert ret == 0 and st["info"] == 0
    assert abs(st["kernel_sum_centre"] / rs["kernel_sum_centre"] - 1) < 1e-4
    assert abs(st["chi2_dof"] / rs["chi2_dof"] - 1) < 1e-2
    # a different answer from the 1 / V2 weights
    r0 = oracle_run("pair512", SEED)["stats"]
    assert abs(rs["chi2_dof"] / r0["chi2_dof"] - 1) > 1e-3
    with pytest.raises(psfm.PsfmError):
        ctx.fit_stamps(d["I1"], d["M1"], d["I2"], d["V2"], d["M2"], d["stamps"])   # V1 missing


def test_weight_mode_v1v2_batch_matches_single_pair():
    torch, psfm = hip()
    wl, pair = pair_for("pair512", SEED)
    cfg = psfm.Config.from_workload(wl, weight_mode=psfm.WEIGHT_V1V2)
    ctx = psfm.Context(cfg)
    d = psfm.to_device(pair)
    single = ctx.match_pair(d["I1"], d["V1"], d["M1"], d["I2"], d["V2"], d["M2"], d["stamps"], c_out=10)
    b = psfm.Batch(ctx, [dict(d, S=wl.spatial_order)], c_out=10)
    b.run()
    torch.cuda.synchronize()
    assert np.array_equal(_np(b.out[0]["coeffs"]), _np(single["sol"]["coeffs"]))
    assert np.array_equal(_np(b.out[0]["diff"]), _np(single["diff"]))
    assert np.array_equal(_np(b.out[0]["diff_mask"]), _np(single["diff_mask"]))


@pytest.mark.parametrize("S", [0, 2])
def test_ortho_basis_solve_parity_same_sums(S):
    """The solve in the orthonormalised basis answers the same least-squares
    problem: from the oracle's sums it keeps every decision of the oracle's
    solve, and its kernel sum, chi2/dof and coefficients match."""
    torch, psfm = hip()
    wl, pair = pair_for("pair512", SEED, 512, 512, n_stamps=120, spatial_order=S)
    cfg = O.Config.from_workload(wl)
    ref_fit = O.fit_stamps(cfg, pair.I1, pair.M1, pair.I2, pair.V2, pair.M2, pair.stamps)
    ret, a_ref, chi2_ref, fl_ref, st_ref = O.solve(cfg, wl.width, wl.height, pair.stamps, ref_fit)
    assert ret == 0
    ctx = psfm.Context(psfm.Config.from_workload(wl, ortho_basis=1))
    d = psfm.to_device(pair)
    fit = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in ref_fit.items()}
    sol = ctx.solve(wl.width, wl.height, d["stamps"], fit)
    st = psfm.read_stats(sol["stats"])
    assert st["info"] == 0 and st["n_iter"] == st_ref["n_iter"] and st["n_used"] == st_ref["n_used"]
    assert np.array_equal(_np(sol["flags"]), fl_ref)
    assert abs(st["kernel_sum_centre"] / st_ref["kernel_sum_centre"] - 1) < 1e-9
    assert abs(st["chi2_dof"] / st_ref["chi2_dof"] - 1) < 1e-9
    a = _np(sol["coeffs"])
    print(f"S={S}: max |a - a_ref| / max|a_ref| = {np.max(np.abs(a - a_ref)) / np.max(np.abs(a_ref)):.2e}")
    assert np.max(np.abs(a - a_ref)) < 1e-5 * np.max(np.abs(a_ref))
    assert np.allclose(_np(sol["chi2"]), chi2_ref, rtol=1e-8, atol=1e-6)


def test_ortho_basis_unsupported_forms():
    torch, psfm = hip()
    wl, pair = pair_for("pair512", SEED)
    ctx = psfm.Context(psfm.Config.from_workload(wl, ortho_basis=1))
    d = psfm.to_device(pair)
    with pytest.raises(psfm.PsfmError, match="-7"):
        psfm.Batch(ctx, [dict(d, S=wl.spatial_order)], c_out=10)
    c16 = psfm.Context(psfm.Config.from_workload(wl, ortho_basis=1, precision=psfm.PREC_FP16))
    fit = c16.fit_stamps(d["I1"], d["M1"], d["I2"], d["V2"], d["M2"], d["stamps"])
    with pytest.raises(psfm.PsfmError, match="-7"):
        c16.solve(wl.width, wl.height, d["stamps"], fit)


def test_sync_returns_device_status():
    torch, psfm = hip()
    wl, pair = pair_for("pair512", SEED)
    ctx = psfm.Context(psfm.Config.from_workload(wl, flags=psfm.SYNC))
    d = psfm.to_device(pair)
    fit = ctx.fit_stamps(d["I1"], d["M1"], d["I2"], d["V2"], d["M2"], d["stamps"])
    sol = ctx.solve(wl.width, wl.height, d["stamps"], fit)          # PSFM_OK
    assert psfm.read_stats(sol["stats"])["info"] == 0
    # every stamp excluded by the caller: too few stamps (-3)
    excl = torch.full_like(fit["flags"], 8)
    with pytest.raises(psfm.PsfmError, match=r"\(-3\)"):
        ctx.solve(wl.width, wl.height, d["stamps"], fit, flags=excl)
    # zero sums on usable stamps: the first pivot is not positive (-4)
    zero = {k: torch.zeros_like(v) for k, v in fit.items() if v is not None}
    zero["npix"] = fit["npix"].clone()
    with pytest.raises(psfm.PsfmError, match=r"\(-4\)"):
        ctx.solve(wl.width, wl.height, d["stamps"], zero)
    # without the flag the same calls return PSFM_OK and report in stats
    ctx0 = psfm.Context(psfm.Config.from_workload(wl))
    sol = ctx0.solve(wl.width, wl.height, d["stamps"], zero)
    assert psfm.read_stats(sol["stats"])["info"] == 1


@pytest.mark.parametrize("rows", [7, 9, 11])
def test_fit_band_rows_parity(rows):
    torch, psfm = hip()
    wl, pair = pair_for("pair512", SEED)
    ref = oracle_run("pair512", SEED)["fit"]
    ctx = psfm.Context(psfm.Config.from_workload(wl, fit_band_rows=rows))
    d = psfm.to_device(pair)
    fit = ctx.fit_stamps(d["I1"], d["M1"], d["I2"], d["V2"], d["M2"], d["stamps"])
    err = _sums_close(fit, ref)
    print(f"band of {rows} rows: Gram normalised error {err:.2e}")


def test_tuner_choices(tmp_path, monkeypatch):
    """The tuner times both fit band heights and the apply candidates, keeps
    the fastest of each, caches the record, and a batch planned with its
    choice matches the oracle at the whole-path targets."""
    torch, psfm = hip()
    from paper_1901_09999_amd import tune

    monkeypatch.setenv("PSFM_TUNE_CACHE", str(tmp_path / "tune.json"))
    pairs_h = []
    for k, (W, H, S, n) in enumerate([(300, 260, 0, 30), (520, 384, 2, 40)]):
        wl = synth.scaled(synth.WORKLOADS["pair2048"], f"tune{k}", W, H, n_stamps=n, spatial_order=S,
                          n_sources=300, mask_frac=0.04)
        pairs_h.append((wl, synth.make_pair(wl, 9100 + k)))
    ctx = psfm.Context(psfm.Config.from_workload(pairs_h[0][0], S=0))
    dev = [dict(psfm.to_device(p), S=wl.spatial_order) for wl, p in pairs_h]
    rec = tune.choose(ctx, dev, c_out=10, grids=(0, 256), orders=(0, 1), reps=1, use_cache=False)
    assert rec["fit_band_rows"] in (7, 9, 11) and rec["apply_grid"] in (0, 256) and rec["order"] in (0, 1)
    fits = [t for t in rec["table"] if t.get("stage") == "fit"]
    assert sorted(t["fit_band_rows"] for t in fits) == [7, 9, 11]
    best = min(fits, key=lambda t: t["ms"])
    assert best["fit_band_rows"] == rec["fit_band_rows"]
    assert tune.choose(ctx, dev, c_out=10, use_cache=True)["when"] == rec["when"]     # cached
    c2 = tune.context_for(ctx, rec["fit_band_rows"])
    b = psfm.Batch(c2, dev, c_out=10, apply_grid=rec["apply_grid"], order=rec["order"])
    b.run()
    torch.cuda.synchronize()
    for k, (wl, p) in enumerate(pairs_h):
        ref = O.match_pair(O.Config.from_workload(wl), p, c_out=10)["stats"]
        st = b.stats(k)
        assert st["info"] == 0
        assert abs(st["kernel_sum_centre"] / ref["kernel_sum_centre"] - 1) < 1e-4
        assert abs(st["chi2_dof"] / ref["chi2_dof"] - 1) < 1e-2
