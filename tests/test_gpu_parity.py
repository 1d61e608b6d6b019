"""Parity of the HIP path (called through the C interface) with the FP64 oracle.

Tolerances follow from the arithmetic of the HIP kernels:
  * per-stamp Gram (FP32 separable basis convolution of the FP32 weighted
    block, its products summed on FP64 MFMA over <= 11 rows of a stamp per
    band, bands added in FP64): every entry within 2e-5 of sqrt(M_ii M_jj)
    (Cauchy-Schwarz scale of the entry; the FP32 design's rounding sets it),
    e_s within 1e-5 relative;
  * solve from identical stamp sums (both FP64): kernel sum and chi2/dof
    within 1e-9 relative; coefficients within 1e-5 of max|a| (the equations
    have condition numbers near 1e8, so raw coefficients are only pinned to
    ~1e-8 relative by FP64);
  * whole path: kernel sum within 1e-4 relative and chi2/dof within 1% (the
    targets of the build);
  * image convolution: FP32 taps and FP32 accumulation of (2h+1)^2 products,
    |error| <= (2h+1)^2 * 2^-24 * sum|K||I|, well inside 2e-5 of max|I'|;
    variance likewise within 1e-5 relative; masks bit-exact;
  * covariance pseudo-matrix (FP64): 1e-12 absolute;
  * difference image from identical inputs: one FP32 rounding, 1e-6 of |I2|.
"""
import numpy as np
import pytest

import oracle as O
from paper_1901_09999_amd import synth

from gpu_common import hip, norm_err_M, oracle_run, pair_for

pytestmark = pytest.mark.gpu

SEEDS = {"pair512": synth.workload_seed(0), "pair2048": synth.workload_seed(1)}


def _ctx(wl, **kw):
    torch, psfm = hip()
    return psfm.Context(psfm.Config.from_workload(wl, **kw))


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name", ["pair512", "pair2048"])
def test_fit_stamps_parity(name):
    torch, psfm = hip()
    wl, pair = pair_for(name, SEEDS[name])
    ref = oracle_run(name, SEEDS[name])["fit"]
    ctx = _ctx(wl)
    d = psfm.to_device(pair)
    fit = ctx.fit_stamps(d["I1"], d["M1"], d["I2"], d["V2"], d["M2"], d["stamps"])
    torch.cuda.synchronize()
    assert np.array_equal(_np(fit["flags"]), ref["flags"])
    assert np.array_equal(_np(fit["npix"]), ref["npix"])
    err = norm_err_M(_np(fit["M"]), ref["M"])
    print(f"{name}: Gram normalised error {err:.3e}")
    assert err < 2e-5
    e = _np(fit["e"])
    ok = ref["e"] > 0
    assert np.max(np.abs(e[ok] - ref["e"][ok]) / ref["e"][ok]) < 1e-5
    # b against the same Cauchy-Schwarz scale
    Md = np.sqrt(np.einsum("sii->si", ref["M"]))
    den = Md * np.sqrt(np.maximum(ref["e"], 1e-300))[:, None]
    den[den == 0] = 1
    assert np.max(np.abs(_np(fit["b"]) - ref["b"]) / den) < 2e-5


@pytest.mark.parametrize("degrees", [(6, 4, 2), (6, 6, 2), (4, 2, 2), (9, 2)])
def test_fit_stamps_basis_sizes(degrees):
    """Every part of the fit's Gram: bases of 49, 62 (the largest: 64 Gram
    columns), 27 and 61 terms (the rows beyond 47 are summed outside the
    MFMA blocks, by one to four lane slots each)."""
    torch, psfm = hip()
    wl, pair = pair_for("pair512", SEEDS["pair512"], 384, 320, n_stamps=30)
    sig = (0.7, 1.5, 3.0)[:len(degrees)]
    cfg = O.Config.from_workload(wl, sigmas=sig, degrees=degrees)
    ctx = _ctx(wl, sigmas=sig, degrees=degrees)
    assert ctx.nb == cfg.n_basis
    d = psfm.to_device(pair)
    fit = ctx.fit_stamps(d["I1"], d["M1"], d["I2"], d["V2"], d["M2"], d["stamps"])
    ref = O.fit_stamps(cfg, pair.I1, pair.M1, pair.I2, pair.V2, pair.M2, pair.stamps)
    assert np.array_equal(_np(fit["flags"]), ref["flags"])
    err = norm_err_M(_np(fit["M"]), ref["M"])
    print(f"degrees {degrees} ({ctx.nb} terms): Gram normalised error {err:.3e}")
    assert err < 2e-5
    Md = np.sqrt(np.einsum("sii->si", ref["M"]))
    den = Md * np.sqrt(np.maximum(ref["e"], 1e-300))[:, None]
    den[den == 0] = 1
    assert np.max(np.abs(_np(fit["b"]) - ref["b"]) / den) < 2e-5
    ok = ref["e"] > 0
    assert np.max(np.abs(_np(fit["e"])[ok] - ref["e"][ok]) / ref["e"][ok]) < 1e-5


@pytest.mark.parametrize("name", ["pair512", "pair2048"])
def test_solve_parity_same_sums(name):
    torch, psfm = hip()
    wl, pair = pair_for(name, SEEDS[name])
    run = oracle_run(name, SEEDS[name])
    ctx = _ctx(wl)
    d = psfm.to_device(pair)
    fit = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in run["fit"].items()}
    sol = ctx.solve(wl.width, wl.height, d["stamps"], fit)
    torch.cuda.synchronize()
    st = psfm.read_stats(sol["stats"])
    ref = run["stats"]
    assert st["info"] == 0 and st["n_iter"] == ref["n_iter"] and st["n_used"] == ref["n_used"]
    assert np.array_equal(_np(sol["flags"]), run["flags"])
    assert abs(st["kernel_sum_centre"] / ref["kernel_sum_centre"] - 1) < 1e-9
    assert abs(st["chi2_dof"] / ref["chi2_dof"] - 1) < 1e-9
    a = _np(sol["coeffs"])
    assert np.max(np.abs(a - run["coeffs"])) < 1e-5 * np.max(np.abs(run["coeffs"]))
    chi2 = _np(sol["chi2"])
    assert np.allclose(chi2, run["chi2"], rtol=1e-8, atol=1e-6)


@pytest.mark.parametrize("name", ["pair512", "pair2048"])
def test_whole_path_parity(name):
    torch, psfm = hip()
    wl, pair = pair_for(name, SEEDS[name])
    run = oracle_run(name, SEEDS[name])
    ctx = _ctx(wl)
    d = psfm.to_device(pair)
    out = ctx.match_pair(d["I1"], d["V1"], d["M1"], d["I2"], d["V2"], d["M2"], d["stamps"],
                         c_out=wl.cov_half)
    torch.cuda.synchronize()
    st = psfm.read_stats(out["sol"]["stats"])
    ref = run["stats"]
    ks = abs(st["kernel_sum_centre"] / ref["kernel_sum_centre"] - 1)
    cd = abs(st["chi2_dof"] / ref["chi2_dof"] - 1)
    print(f"{name}: kernel-sum rel err {ks:.2e}, chi2/dof rel err {cd:.2e}, gpu {st}")
    assert st["info"] == 0
    assert ks < 1e-4
    assert cd < 1e-2
    # rejection decisions: equal, or the stamps that differ sit at the threshold
    gf, rf = _np(out["sol"]["flags"]), run["flags"]
    diff = np.nonzero(gf != rf)[0]
    if diff.size:
        q = run["chi2"] / np.maximum(run["fit"]["npix"], 1)
        used = (rf == 0)
        thr = q[used].mean() + 3.0 * q[used].std()
        assert np.all(np.abs(q[diff] / thr - 1) < 1e-3), (diff, q[diff], thr)
    # The difference image agrees to a small fraction of its noise: the FP32
    # stamp sums move the solution only along directions the data barely
    # constrain (condition numbers ~1e8), which by construction change the
    # model by much less than the noise.
    D, Dr = _np(out["diff"]), run["diff"]
    clean = (run["diff_mask"] == 0) & (_np(out["diff_mask"]) == 0)
    z = (D[clean] - Dr[clean]) / np.sqrt(run["diff_var"][clean])
    print(f"{name}: difference image max |dD|/sigma {np.max(np.abs(z)):.2e}, rms {np.sqrt(np.mean(z * z)):.2e}")
    assert np.max(np.abs(z)) < 5e-2 and np.sqrt(np.mean(z * z)) < 5e-3
    # Masks: bit-exact for identical coefficients (test_convolution_parity);
    # here the two kernels come from different stamp sums, so a patch whose
    # BAD radius sits at the 0.2 threshold may move pixels between CONV_BAD
    # and CONV_POOR -- nothing else may differ.
    mg, mr = _np(out["diff_mask"]), run["diff_mask"]
    dm = mg != mr
    swap = {O.MASK_CONV_BAD, O.MASK_CONV_POOR}
    assert np.all((mg[dm].astype(int) & ~6) == (mr[dm].astype(int) & ~6))
    assert np.all(np.isin(mg[dm] & 6, list(swap)) & np.isin(mr[dm] & 6, list(swap)))
    assert dm.mean() < 5e-3


@pytest.mark.parametrize("name", ["pair512", "pair2048"])
def test_convolution_parity(name):
    torch, psfm = hip()
    wl, pair = pair_for(name, SEEDS[name])
    run = oracle_run(name, SEEDS[name])
    ctx = _ctx(wl)
    d = psfm.to_device(pair)
    a = torch.from_numpy(run["coeffs"]).cuda()
    conv, cm = ctx.convolve_image(a, d["I1"], d["M1"])
    var, cov = ctx.propagate_variance(a, d["V1"], d["M1"], c_out=wl.cov_half)
    torch.cuda.synchronize()
    c, v = _np(conv), _np(var)
    err = np.max(np.abs(c - run["conv"])) / np.max(np.abs(run["conv"]))
    print(f"{name}: conv max err / max {err:.2e}")
    assert err < 2e-5
    assert np.array_equal(_np(cm), run["conv_mask"])
    rel = np.max(np.abs(v - run["var"]) / np.maximum(np.abs(run["var"]), 1e-30))
    assert rel < 1e-5
    assert np.max(np.abs(_np(cov) - run["cov"])) < 1e-12


def test_variance_with_correlated_input():
    torch, psfm = hip()
    wl, pair = pair_for("pair512", SEEDS["pair512"])
    run = oracle_run("pair512", SEEDS["pair512"])
    cfg = O.Config.from_workload(wl)
    q = np.array([[0.05, 0.2, 0.0], [0.1, 1.0, 0.3], [0.0, 0.2, 0.1]])
    cin = np.zeros((3, 3))
    for dy in range(-1, 2):
        for dx in range(-1, 2):
            cin[dy + 1, dx + 1] = sum(q[y, x] * q[y + dy, x + dx]
                                      for y in range(3) for x in range(3)
                                      if 0 <= y + dy < 3 and 0 <= x + dx < 3)
    cin /= cin[1, 1]
    var_r, cov_r, disc_r = O.propagate_variance(cfg, run["coeffs"], pair.V1, pair.M1, cov_in=cin,
                                                c_in=1, c_out=12)
    ctx = _ctx(wl)
    d = psfm.to_device(pair)
    stats = torch.zeros(psfm.STATS_BYTES, dtype=torch.uint8, device="cuda")
    var, cov = ctx.propagate_variance(torch.from_numpy(run["coeffs"]).cuda(), d["V1"], d["M1"],
                                      cov_in=torch.from_numpy(cin).cuda(), c_out=12, stats=stats)
    torch.cuda.synchronize()
    assert np.max(np.abs(_np(var) - var_r) / np.abs(var_r)) < 1e-5
    assert np.max(np.abs(_np(cov) - cov_r)) < 1e-12
    assert abs(psfm.read_stats(stats)["cov_discarded_frac"] - disc_r) < 1e-12


def test_subtract_parity():
    torch, psfm = hip()
    wl, pair = pair_for("pair2048", SEEDS["pair2048"])
    run = oracle_run("pair2048", SEEDS["pair2048"])
    ctx = _ctx(wl)
    d = psfm.to_device(pair)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    cov2 = np.zeros((5, 5))
    cov2[2, 2] = 1.0
    cov2[2, 3] = cov2[2, 1] = 0.25
    sub = ctx.subtract(t(run["coeffs"]), d["I2"], d["V2"], d["M2"], t(run["conv"]), t(run["var"]),
                       t(run["conv_mask"]), t(run["cov"]), cov2=t(cov2))
    torch.cuda.synchronize()
    D, VD, MD, CD = O.subtract(O.Config.from_workload(wl), run["coeffs"], pair.I2, pair.V2, pair.M2,
                               run["conv"], run["var"], run["conv_mask"], run["cov"], cov2=cov2)
    assert np.max(np.abs(_np(sub["diff"]) - D) / np.maximum(np.abs(np.nan_to_num(pair.I2)), 1)) < 1e-6
    assert np.array_equal(_np(sub["diff_var"]), VD)
    assert np.array_equal(_np(sub["diff_mask"]), MD)
    assert np.max(np.abs(_np(sub["cov_diff"]) - CD)) < 1e-12


@pytest.mark.parametrize("W,H,P,h,r,S", [(300, 217, 64, 5, 12, 1), (161, 190, 50, 3, 6, 2),
                                         (97, 75, 16, 7, 9, 0), (256, 129, 128, 12, 24, 3)])
def test_ragged_shapes(W, H, P, h, r, S):
    """Image sizes that leave ragged tiles and patches, patch sides above and
    below the 64-pixel tile, several kernel and stamp sizes, masks, and stamps
    whose footprint leaves the image."""
    torch, psfm = hip()
    base = synth.WORKLOADS["pair2048"]
    wl = synth.scaled(base, f"rag{W}x{H}", W, H, n_sources=max(40, W * H // 600), n_stamps=30,
                      kernel_half=h, stamp_half=r, spatial_order=S, patch=P)
    pair = synth.make_pair(wl, 4242 + W)
    rng = np.random.default_rng(W)
    extra = rng.integers(0, [W, H], (6, 2)).astype(np.int32)      # may be invalid
    stamps = np.concatenate([pair.stamps, extra, [[1, 1], [W - 2, H - 2]]]).astype(np.int32)
    cfg = O.Config.from_workload(wl, min_stamps=1)
    fit_r = O.fit_stamps(cfg, pair.I1, pair.M1, pair.I2, pair.V2, pair.M2, stamps)
    ctx = _ctx(wl, min_stamps=1)
    d = psfm.to_device(pair)
    st_t = torch.from_numpy(stamps).cuda()
    fit = ctx.fit_stamps(d["I1"], d["M1"], d["I2"], d["V2"], d["M2"], st_t)
    torch.cuda.synchronize()
    assert np.array_equal(_np(fit["flags"]), fit_r["flags"])
    assert (fit_r["flags"] != 0).sum() >= 2
    assert norm_err_M(_np(fit["M"]), fit_r["M"]) < 2e-5
    a = np.zeros(cfg.n_unknowns)
    a[0 * cfg.n_spatial] = 1.1
    a[1 * cfg.n_spatial] = 0.05
    if S > 0:
        a[1] = 0.2
    a[-1] = 3.0
    conv_r, cm_r = O.convolve_image(cfg, a, pair.I1, pair.M1)
    var_r, cov_r, _ = O.propagate_variance(cfg, a, pair.V1, pair.M1, c_out=2 * h)
    at = torch.from_numpy(a).cuda()
    conv, cm = ctx.convolve_image(at, d["I1"], d["M1"])
    var, cov = ctx.propagate_variance(at, d["V1"], d["M1"], c_out=2 * h)
    torch.cuda.synchronize()
    assert np.max(np.abs(_np(conv) - conv_r)) < 2e-5 * np.max(np.abs(conv_r))
    assert np.array_equal(_np(cm), cm_r)
    assert np.max(np.abs(_np(var) - var_r) / np.maximum(np.abs(var_r), 1e-30)) < 1e-5
    assert np.max(np.abs(_np(cov) - cov_r)) < 1e-12
    # the difference on the oracle's convolved planes (widths that are not a
    # multiple of 4 take the one-pixel-per-thread subtraction)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    sub = ctx.subtract(at, d["I2"], d["V2"], d["M2"], t(conv_r), t(var_r), t(cm_r), t(cov_r))
    torch.cuda.synchronize()
    D, VD, MD, CD = O.subtract(cfg, a, pair.I2, pair.V2, pair.M2, conv_r, var_r, cm_r, cov_r)
    assert np.max(np.abs(_np(sub["diff"]) - D) / np.maximum(np.abs(np.nan_to_num(pair.I2)), 1)) < 1e-6
    assert np.array_equal(_np(sub["diff_var"]), VD)
    assert np.array_equal(_np(sub["diff_mask"]), MD)
    assert np.max(np.abs(_np(sub["cov_diff"]) - CD)) < 1e-12


def test_too_few_stamps_and_empty():
    torch, psfm = hip()
    wl, pair = pair_for("pair512", SEEDS["pair512"])
    ctx = _ctx(wl)
    d = psfm.to_device(pair)
    M1 = d["M1"].clone()
    M1[:, :] = 1                                            # every stamp masked
    fit = ctx.fit_stamps(d["I1"], M1, d["I2"], d["V2"], d["M2"], d["stamps"])
    sol = ctx.solve(wl.width, wl.height, d["stamps"], fit)
    torch.cuda.synchronize()
    st = psfm.read_stats(sol["stats"])
    assert st["info"] == psfm_too_few()
    assert np.all(_np(sol["coeffs"]) == 0)
    assert np.all(_np(fit["flags"]) == O.STAMP_INVALID)
    # zero stamps: nothing is launched by the fit; the solve reports too few
    empty = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    fit0 = ctx.fit_stamps(d["I1"], d["M1"], d["I2"], d["V2"], d["M2"], empty)
    sol0 = ctx.solve(wl.width, wl.height, empty, fit0)
    torch.cuda.synchronize()
    assert psfm.read_stats(sol0["stats"])["info"] == psfm_too_few()


def psfm_too_few():
    return -3


def test_tiny_image_all_border():
    """An image smaller than the kernel: every output pixel sees the outside."""
    torch, psfm = hip()
    W = H = 15
    cfg = O.Config(h=10, S=0)
    rng = np.random.default_rng(1)
    I = rng.normal(100, 5, (H, W)).astype(np.float32)
    V = np.full((H, W), 100, np.float32)
    Mk = np.zeros((H, W), np.uint8)
    a = np.zeros(cfg.n_unknowns)
    a[0] = 1.0
    conv_r, cm_r = O.convolve_image(cfg, a, I, Mk)
    ctx = psfm.Context(psfm.Config(h=10))
    t = lambda x: torch.from_numpy(x).cuda()
    conv, cm = ctx.convolve_image(t(a), t(I), t(Mk))
    torch.cuda.synchronize()
    assert np.array_equal(_np(cm), cm_r) and (cm_r != 0).all()
    assert np.max(np.abs(_np(conv) - conv_r)) < 1e-4


def test_noiseless_inspan_recovery_gpu():
    """A kernel in the basis span is recovered by the HIP path from a
    noiseless pair made with the oracle's realised kernel (property at any
    size): kernel sum, background and the difference image."""
    torch, psfm = hip()
    from scipy import signal
    cfg = O.Config(S=0, max_iter=1)
    W = H = 256
    rng = np.random.default_rng(5)
    I1 = np.full((H, W), 100.0)
    yy, xx = np.mgrid[0:H, 0:W]
    for _ in range(40):
        x0, y0 = rng.uniform(30, W - 30, 2)
        f = np.exp(rng.uniform(np.log(2e3), np.log(5e4)))
        I1 += f / (2 * np.pi * 2.25) * np.exp(-((xx - x0) ** 2 + (yy - y0) ** 2) / 4.5)
    # the reference keeps its photon noise (a noiseless reference makes the
    # basis convolutions nearly degenerate, condition ~1e11, beyond FP32 data);
    # the target is the exact convolution of that noisy reference
    I1 = (I1 + rng.standard_normal((H, W)) * np.sqrt(I1)).astype(np.float32)
    a_true = np.zeros(cfg.n_unknowns)
    a_true[0] = 1.25
    a_true[15] = 0.4
    a_true[2] = 0.03
    a_true[-1] = 5.0
    K = O.kernel_at(cfg, a_true, 0, 0, W, H)
    I2 = (signal.convolve2d(I1.astype(np.float64), K, mode="same") + 5.0).astype(np.float32)
    V2 = (np.abs(I2) + 1).astype(np.float32)
    Z = np.zeros((H, W), np.uint8)
    stamps = np.array([(x, y) for y in range(40, 220, 45) for x in range(40, 220, 45)], np.int32)
    ctx = psfm.Context(psfm.Config(S=0, max_iter=1))
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    out = ctx.match_pair(t(I1), t(V2), t(Z), t(I2), t(V2), t(Z), t(stamps))
    torch.cuda.synchronize()
    st = psfm.read_stats(out["sol"]["stats"])
    assert abs(st["kernel_sum_centre"] / 1.25 - 1) < 1e-5
    assert abs(_np(out["sol"]["coeffs"])[-1] - 5.0) < 1e-2
    clean = _np(out["diff_mask"]) == 0
    assert np.max(np.abs(_np(out["diff"])[clean])) < 2e-4 * np.abs(I2).max()


def test_cholesky_solve_matches_oracle():
    """psfm_cholesky_solve on the assembled 295 x 295 normal matrix of the
    2048^2 pair: the same solution as the oracle's equilibrated Cholesky
    (FP64 both; residual and kernel sum to 1e-9), and the same failing pivot
    for a matrix made indefinite."""
    torch, psfm = hip()
    wl, pair = pair_for("pair2048", SEEDS["pair2048"])
    ref = oracle_run("pair2048", SEEDS["pair2048"])
    cfg = O.Config.from_workload(wl)
    used = (ref["fit"]["flags"] == 0).astype(np.uint8)
    M, b = O.assemble(cfg, wl.width, wl.height, pair.stamps, ref["fit"]["M"], ref["fit"]["b"], used)
    xo, info_o = O.cholesky_solve(M, b)
    x, info = psfm.cholesky_solve(torch.from_numpy(M).cuda(), torch.from_numpy(b).cuda())
    torch.cuda.synchronize()
    x = _np(x)
    assert int(_np(info)[0]) == 0 and info_o == 0
    assert np.linalg.norm(M @ x - b) <= 1e-9 * np.linalg.norm(b)
    g = O.spatial(cfg, 0.5 * (wl.width - 1), 0.5 * (wl.height - 1), wl.width, wl.height)
    ns = len(g)
    assert abs((x[:ns] @ g) / (xo[:ns] @ g) - 1) < 1e-9
    M2 = M.copy()
    M2[100, 100] = -1.0
    _, info_o2 = O.cholesky_solve(M2, b)
    _, info2 = psfm.cholesky_solve(torch.from_numpy(M2).cuda(), torch.from_numpy(b).cuda())
    torch.cuda.synchronize()
    assert int(_np(info2)[0]) == info_o2 == 101


@pytest.mark.parametrize("W,H,P,h,c_in", [(2048, 2048, 64, 10, 0), (300, 217, 64, 5, 1),
                                          (161, 190, 50, 3, 2)])
def test_convolve_pair_equals_separate_calls(W, H, P, h, c_in):
    """psfm_convolve_pair (one patch realisation per tile for both planes) is
    bit-identical to psfm_convolve_image + psfm_propagate_variance, with an
    uncorrelated or a correlated input, on full and ragged tilings."""
    torch, psfm = hip()
    base = synth.WORKLOADS["pair2048"]
    wl = base if W == 2048 else synth.scaled(base, f"cp{W}x{H}", W, H, n_sources=max(40, W * H // 600),
                                             n_stamps=20, kernel_half=h, patch=P)
    pair = synth.make_pair(wl, 31 + W)
    cfg = O.Config.from_workload(wl)
    ctx = _ctx(wl)
    d = psfm.to_device(pair)
    rng = np.random.default_rng(W)
    a = np.zeros(cfg.n_unknowns)
    a[0] = 1.0
    a[: cfg.n_unknowns - 1] += 0.02 * rng.standard_normal(cfg.n_unknowns - 1)
    a[-1] = 2.0
    at = torch.from_numpy(a).cuda()
    cin = None
    if c_in:
        q = rng.uniform(0.0, 1.0, (2 * c_in + 1, 2 * c_in + 1))
        cin_np = np.array([[np.sum(q[max(0, -dy):q.shape[0] - max(0, dy), max(0, -dx):q.shape[1] - max(0, dx)] *
                                   q[max(0, dy):q.shape[0] - max(0, -dy), max(0, dx):q.shape[1] - max(0, -dx)])
                            for dx in range(-c_in, c_in + 1)] for dy in range(-c_in, c_in + 1)])
        cin = torch.from_numpy(cin_np / cin_np[c_in, c_in]).cuda()
    print(f"{W}x{H} P={P} h={h} c_in={c_in}", flush=True)
    s1 = torch.zeros(psfm.STATS_BYTES, dtype=torch.uint8, device="cuda")
    s2 = torch.zeros(psfm.STATS_BYTES, dtype=torch.uint8, device="cuda")
    conv, cm = ctx.convolve_image(at, d["I1"], d["M1"])
    var, cov = ctx.propagate_variance(at, d["V1"], d["M1"], cov_in=cin, c_out=12, stats=s1)
    conv2, cm2, var2, cov2 = ctx.convolve_pair(at, d["I1"], d["V1"], d["M1"], cov_in=cin, c_out=12,
                                               stats=s2)
    torch.cuda.synchronize()
    assert np.array_equal(_np(conv2), _np(conv))
    assert np.array_equal(_np(cm2), _np(cm))
    assert np.array_equal(_np(var2), _np(var))
    assert np.array_equal(_np(cov2), _np(cov))
    assert psfm.read_stats(s2)["cov_discarded_frac"] == psfm.read_stats(s1)["cov_discarded_frac"]


@pytest.mark.gpu
@pytest.mark.parametrize("W,H,P,h,c_in", [(2048, 2048, 64, 10, 0), (300, 217, 64, 5, 1),
                                          (161, 190, 50, 3, 2)])
def test_match_pair_equals_separate_calls(W, H, P, h, c_in):
    """psfm_match_pair (convolutions and difference in one pass over the
    tiles) gives psfm_convolve_pair + psfm_subtract's difference image
    bit for bit, with or without the convolved planes written, with
    uncorrelated or correlated inputs, on full and ragged tilings; C_D's
    variance means are summed per tile, so it agrees to rounding."""
    torch, psfm = hip()
    base = synth.WORKLOADS["pair2048"]
    wl = base if W == 2048 else synth.scaled(base, f"mp{W}x{H}", W, H, n_sources=max(40, W * H // 600),
                                             n_stamps=20, kernel_half=h, patch=P)
    pair = synth.make_pair(wl, 57 + W)
    cfg = O.Config.from_workload(wl)
    ctx = _ctx(wl)
    d = psfm.to_device(pair)
    rng = np.random.default_rng(W + 1)
    a = np.zeros(cfg.n_unknowns)
    a[0] = 1.0
    a[: cfg.n_unknowns - 1] += 0.02 * rng.standard_normal(cfg.n_unknowns - 1)
    a[-1] = 2.0
    at = torch.from_numpy(a).cuda()
    cin = c2 = None
    if c_in:
        def corr(c):
            q = rng.uniform(0.0, 1.0, (2 * c + 1, 2 * c + 1))
            m = np.array([[np.sum(q[max(0, -dy):q.shape[0] - max(0, dy), max(0, -dx):q.shape[1] - max(0, dx)] *
                                  q[max(0, dy):q.shape[0] - max(0, -dy), max(0, dx):q.shape[1] - max(0, -dx)])
                           for dx in range(-c, c + 1)] for dy in range(-c, c + 1)])
            return torch.from_numpy(m / m[c, c]).cuda()
        cin, c2 = corr(c_in), corr(c_in + 1)
    print(f"{W}x{H} P={P} h={h} c_in={c_in}", flush=True)
    conv, cm, var, cov = ctx.convolve_pair(at, d["I1"], d["V1"], d["M1"], cov_in=cin, c_out=12)
    ref = ctx.subtract(at, d["I2"], d["V2"], d["M2"], conv, var, cm, cov, cov2=c2)
    conv_f = torch.full_like(conv, -1.0)
    cm_f = torch.full_like(cm, 7)
    var_f = torch.full_like(var, -1.0)
    full = ctx.match(at, d["I1"], d["V1"], d["M1"], d["I2"], d["V2"], d["M2"], cov1=cin, cov2=c2,
                     c_out=12, conv=conv_f, conv_mask=cm_f, conv_var=var_f)
    bare = ctx.match(at, d["I1"], d["V1"], d["M1"], d["I2"], d["V2"], d["M2"], cov1=cin, cov2=c2,
                     c_out=12)
    torch.cuda.synchronize()
    assert np.array_equal(_np(conv_f), _np(conv))
    assert np.array_equal(_np(cm_f), _np(cm))
    assert np.array_equal(_np(var_f), _np(var))
    for r in (full, bare):
        assert np.array_equal(_np(r["cov"]), _np(cov))
        for k in ("diff", "diff_var", "diff_mask"):
            assert np.array_equal(_np(r[k]), _np(ref[k])), k
        cd, cd_ref = _np(r["cov_diff"]), _np(ref["cov_diff"])
        assert cd.shape == cd_ref.shape
        assert np.max(np.abs(cd - cd_ref)) <= 1e-12 * np.max(np.abs(cd_ref))

