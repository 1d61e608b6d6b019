"""Pins of the oracle's normalisation and quality mode (Sections 3.2, 3.3,
3.6, 3.7) against what the paper and the mathematics fix: exact totals,
recovery of an injected kernel, a constrained least-squares problem solved
by numpy on the stacked design, hand-built rejection and replacement cases,
and the moments and enclosed fractions of Gaussian kernels."""
import math

import numpy as np
import pytest
from scipy import signal

import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def conv_same(img, K):
    return signal.convolve2d(img, K, mode="same", boundary="fill", fillvalue=0.0)


def gauss_img(W, H, x0, y0, s, flux=1.0):
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    return flux / (2 * math.pi * s * s) * np.exp(-((x - x0) ** 2 + (y - y0) ** 2) / (2 * s * s))


def term_index(cfg, j, p, q):
    i = 0
    for jj, D in enumerate(cfg.degrees):
        for d in range(D + 1):
            for pp in range(d, -1, -1):
                if (jj, pp, d - pp) == (j, p, q):
                    return i
                i += 1
    raise KeyError


def test_norm_solve_recovers_exact_totals(orc):
    """T2 = b0 T1 + d0 npix holds exactly for every stamp: the stamp-total fit
    returns b0 and d0; unused stamps do not count; equal totals everywhere
    (no lever arm between b0 and d0) are singular."""
    rng = np.random.default_rng(3)
    n = 40
    t1 = rng.uniform(1e3, 5e5, n)
    npix = np.full(n, 1681.0)
    t2 = 1.3 * t1 + 7.5 * npix
    norm = np.stack([npix, t1, t2, np.zeros(n), np.zeros(n)], axis=1)
    used = np.ones(n, np.uint8)
    ret, b0, d0 = O.norm_solve(norm, used)
    assert ret == 0 and abs(b0 - 1.3) < 1e-12 and abs(d0 - 7.5) < 1e-8
    norm_bad = norm.copy()
    norm_bad[5, 2] *= 3.0                     # a variable source, left out of the fit
    used[5] = 0
    ret, b0, d0 = O.norm_solve(norm_bad, used)
    assert ret == 0 and abs(b0 - 1.3) < 1e-12
    flat = norm.copy()
    flat[:, 1] = 1e4
    assert O.norm_solve(flat, np.ones(n, np.uint8))[0] == 1


def _isolated_pair(a_true, cfg, W=260, H=260, seed=4):
    """Isolated stars on a grid of stamp centres (no flux crosses a stamp
    edge), image 2 = K (x) image 1 + background, noiseless."""
    rng = np.random.default_rng(seed)
    grid = [(x, y) for y in range(40, H - 30, 45) for x in range(40, W - 30, 45)]
    I1 = np.full((H, W), 0.0)
    for (x, y) in grid:
        I1 += gauss_img(W, H, x + rng.uniform(-0.5, 0.5), y + rng.uniform(-0.5, 0.5), 1.5,
                        math.exp(rng.uniform(math.log(2e3), math.log(5e4))))
    I1 += 100.0
    K = O.kernel_at(cfg, a_true, 0, 0, W, H)
    I2 = conv_same(I1, K)
    # the constant sky convolves to K.sum() * 100 away from the edges; add d0
    I2 = I2 + a_true[-1]
    return I1.astype(np.float32), I2.astype(np.float32), np.array(grid, np.int32)


def test_separate_normalisation_recovers_flux_ratio(orc):
    """Noiseless isolated stars, kernel of sum 1.3 (zero-sum terms add no
    flux) and background difference 7.5: the unweighted stamp totals give
    b0 = 1.3 and d0 = 7.5, and the held solve recovers the injected kernel."""
    cfg = O.Config(S=0, max_iter=1)
    a_true = np.zeros(cfg.n_unknowns)
    a_true[0] = 1.3
    a_true[term_index(cfg, 1, 0, 0)] = 0.5
    a_true[term_index(cfg, 0, 2, 0)] = 0.04
    a_true[term_index(cfg, 1, 1, 0)] = 0.03
    a_true[-1] = 7.5
    I1, I2, stamps = _isolated_pair(a_true, cfg)
    H, W = I1.shape
    V2 = (np.abs(I2) + 1.0).astype(np.float32)
    Z = np.zeros((H, W), np.uint8)
    fit = O.fit_stamps(cfg, I1, Z, I2, V2, Z, stamps)
    assert (fit["flags"] == 0).all()
    norm = O.fit_norm(cfg, I1, I2, stamps, fit["flags"])
    assert np.all(norm[:, 0] == (2 * cfg.r + 1) ** 2)
    ret, b0, d0 = O.norm_solve(norm, np.ones(len(stamps), np.uint8))
    assert ret == 0 and abs(b0 - 1.3) < 1e-6 and abs(d0 - 7.5) < 1e-3
    ret, a, chi2, fl, st, nrep = O.solve_norm(cfg, W, H, stamps, fit, norm)
    assert ret == 0 and st["n_used"] == len(stamps) and nrep == 0
    assert a[0] == b0 and a[-1] == d0 and st["kernel_sum_centre"] == b0
    Kt = O.kernel_at(cfg, a_true, 0, 0, W, H)
    Kg = O.kernel_at(cfg, a, 0, 0, W, H)
    assert np.abs(Kg - Kt).max() < 1e-4 * np.abs(Kt).max()


def test_held_solve_is_constrained_least_squares(orc):
    """Tiny problem with S = 1: the solution with b0, d0 held equals numpy's
    least squares on the stacked weighted design whose held columns (term 0
    at every spatial term, the background) are moved to the right-hand side
    with their values (b0 and d0 from numpy sums of the stamp totals)."""
    cfg = O.Config(sigmas=(0.8, 1.5), degrees=(2, 1), h=2, r=3, S=1, max_iter=1)
    W, H = 44, 40
    rng = np.random.default_rng(12)
    I1 = rng.normal(300, 60, (H, W)).astype(np.float32)
    I2 = (1.2 * I1 + rng.normal(5, 20, (H, W))).astype(np.float32)
    V2 = rng.uniform(50, 150, (H, W)).astype(np.float32)
    Z = np.zeros((H, W), np.uint8)
    stamps = np.array([[8, 8], [30, 9], [13, 28], [34, 30], [22, 19], [27, 12], [9, 31]], np.int32)
    fit = O.fit_stamps(cfg, I1, Z, I2, V2, Z, stamps)
    norm = O.fit_norm(cfg, I1, I2, stamps, fit["flags"])
    kb = O.basis(cfg)
    Ai = [conv_same(I1.astype(np.float64), kb[i]) for i in range(cfg.n_basis)]
    r, ns = cfg.r, cfg.n_spatial
    T1 = np.array([Ai[0][y - r:y + r + 1, x - r:x + r + 1].sum() for x, y in stamps])
    T2 = np.array([I2[y - r:y + r + 1, x - r:x + r + 1].astype(np.float64).sum() for x, y in stamps])
    npx = float((2 * r + 1) ** 2)
    assert np.allclose(norm[:, 1], T1, rtol=1e-12) and np.allclose(norm[:, 2], T2, rtol=1e-12)
    G = np.stack([T1, np.full(len(stamps), npx)], axis=1)
    b0, d0 = np.linalg.lstsq(G, T2, rcond=None)[0]
    ret, a, chi2, fl, st, nrep = O.solve_norm(cfg, W, H, stamps, fit, norm)
    assert ret == 0 and abs(a[0] - b0) < 1e-10 * abs(b0) and abs(a[-1] - d0) < 1e-8 * max(1, abs(d0))
    rows, rhs = [], []
    for xc, yc in stamps:
        sl = (slice(yc - r, yc + r + 1), slice(xc - r, xc + r + 1))
        xt, yt = (2 * xc - (W - 1)) / (W - 1), (2 * yc - (H - 1)) / (H - 1)
        g = [1.0, xt, yt]
        cols = [g[t] * Ai[i][sl].ravel() for i in range(1, cfg.n_basis) for t in range(ns)]
        sw = 1.0 / np.sqrt(V2[sl].astype(np.float64).ravel())
        rows.append(sw[:, None] * np.stack(cols, axis=1))
        held = b0 * Ai[0][sl].ravel() + d0
        rhs.append(sw * (I2[sl].astype(np.float64).ravel() - held))
    ls = np.linalg.lstsq(np.vstack(rows), np.concatenate(rhs), rcond=None)[0]
    free = a[ns:-1]
    assert np.allclose(free, ls, rtol=1e-7, atol=1e-9)
    assert np.all(a[1:ns] == 0.0)                  # the normalisation is spatially constant
    assert st["dof"] == len(stamps) * npx - (len(free) + 2)


def test_rejected_stamp_is_replaced_from_its_group(orc):
    """Section 3.3: a rejected stamp is replaced by a reserve of its own
    subregion (group); reserves of other groups stay out; a group without a
    reserve loses its stamp.  Per-stamp sums are hand-built (b_s = 0, M_s = I)
    so the clip statistic is set by e_s; totals give b0 = 1, d0 = 0."""
    cfg = O.Config(sigmas=(0.8, 1.5), degrees=(2, 1), h=2, r=2, S=0, max_iter=3, min_stamps=3)
    L = cfg.n_basis + 1
    q = [1.0] * 30 + [40.0, 45.0] + [1.0, 1.0, 1.0]      # stamps 30, 31 outliers; 32-34 reserves
    n = len(q)
    npix = 100
    fit = dict(M=np.repeat(np.eye(L)[None], n, axis=0), b=np.zeros((n, L)),
               e=np.asarray(q) * npix, npix=np.full(n, npix, np.int32), flags=np.zeros(n, np.int32))
    group = np.array(list(range(30)) + [40, 41] + [40, 40, 50], np.int32)
    flags = np.zeros(n, np.int32)
    flags[32:] = O.STAMP_RESERVE
    t1 = np.linspace(1e3, 1e4, n)
    norm = np.stack([np.full(n, npix, float), t1, t1, np.zeros(n), np.zeros(n)], axis=1)
    stamps = np.array([[10 + s, 10] for s in range(n)], np.int32)
    ret, a, chi2, fl, st, nrep = O.solve_norm(cfg, 100, 100, stamps, fit, norm, flags=flags, group=group)
    assert ret == 0 and abs(a[0] - 1.0) < 1e-12 and abs(a[-1]) < 1e-6
    assert fl[30] & O.STAMP_REJECTED and fl[31] & O.STAMP_REJECTED
    assert fl[32] == 0 and fl[33] == O.STAMP_RESERVE and fl[34] == O.STAMP_RESERVE
    assert nrep == 1 and st["n_used"] == 31 and st["n_rejected"] == 2
    # without groups nothing is replaced
    ret, a, chi2, fl, st, nrep = O.solve_norm(cfg, 100, 100, stamps, fit, norm, flags=flags)
    assert nrep == 0 and st["n_used"] == 30


def test_quality_deviation_without_softening_is_chi2(orc):
    """With no softening the stamp deviation of the pixel pass (kernel
    realised at the stamp centre) equals chi2_s / npix_s from the stamp sums
    (the stamp-centre model both use), for a spatially varying solution."""
    cfg = O.Config(sigmas=(0.8, 1.5, 2.5), degrees=(2, 2, 0), h=4, r=5, S=2)
    W, H = 90, 80
    rng = np.random.default_rng(21)
    I1 = rng.normal(400, 80, (H, W)).astype(np.float32)
    I2 = rng.normal(420, 80, (H, W)).astype(np.float32)
    V2 = rng.uniform(60, 160, (H, W)).astype(np.float32)
    Z = np.zeros((H, W), np.uint8)
    stamps = np.array([[15, 15], [70, 12], [40, 40], [20, 62], [66, 60]], np.int32)
    fit = O.fit_stamps(cfg, I1, Z, I2, V2, Z, stamps)
    a = rng.normal(0, 0.1, cfg.n_unknowns)
    a[0] = 1.05
    a[-1] = 3.0
    flags = np.zeros(len(stamps), np.int32)
    flags[3] = O.STAMP_REJECTED
    q, dev = O.quality(cfg, a, I1, I2, V2, stamps, flags, soft=0.0)
    L = cfg.n_basis + 1
    for s, (x, y) in enumerate(stamps):
        if flags[s]:
            assert dev[s] == 0.0
            continue
        c2 = O.stamp_chi2(cfg, a, W, H, x, y, fit["M"][s], fit["b"][s], fit["e"][s])
        assert abs(dev[s] - c2 / fit["npix"][s]) < 1e-9 * dev[s]
    used = dev[flags == 0]
    assert q["n_used"] == 4 and abs(q["dev_mean"] - (used.mean() - 1)) < 1e-12
    assert abs(q["dev_rms"] - used.std()) < 1e-12
    # softening only lowers the deviation (fluxes are positive here); brute
    # force with scipy's convolution of the kernel realised at each centre
    q2, dev2 = O.quality(cfg, a, I1, I2, V2, stamps, flags, soft=0.5)
    assert np.all(dev2[flags == 0] < dev[flags == 0])
    r = cfg.r
    for s, (x, y) in enumerate(stamps):
        if flags[s]:
            continue
        K = O.kernel_at(cfg, a, x, y, W, H)
        m = conv_same(I1.astype(np.float64), K)[y - r:y + r + 1, x - r:x + r + 1] + a[-1]
        res = I2[y - r:y + r + 1, x - r:x + r + 1].astype(np.float64) - m
        ref = np.mean(res ** 2 / (V2[y - r:y + r + 1, x - r:x + r + 1] + 0.5 * np.abs(m)))
        assert abs(dev2[s] - ref) < 1e-10 * ref


def test_quality_of_gaussian_and_deconvolving_kernels(orc):
    """Kernel moments and enclosed fractions at the image centre.  A unit-sum
    Gaussian of sigma 1.5: first moments 0, second moments sigma^2 (to
    e^(-2 pi^2 sigma^2)), enclosed fraction rising to exactly 1, so no cut.
    A difference of Gaussians 1.5 G(1.5) - 0.5 G(3): its enclosed fraction
    overshoots -- the continuous form 1.5 (1 - e^(-rho^2 / 4.5)) -
    0.5 (1 - e^(-rho^2 / 18)) peaks at 1.164 near rho = 3.9 -- and the
    deconvolution cut is raised; a shifted kernel (odd term) raises the
    first-moment cut; a noiseless in-span pair has zero deviations."""
    cfg = O.Config(S=0)
    W = H = 200
    g15 = term_index(cfg, 1, 0, 0)
    g30 = term_index(cfg, 2, 0, 0)
    a = np.zeros(cfg.n_unknowns)
    a[0] = 1.0
    a[g15] = 1.0
    I = np.full((H, W), 100.0, np.float32)
    V = np.full((H, W), 100.0, np.float32)
    stamps = np.array([[50, 50], [150, 50], [50, 150], [150, 150]], np.int32)
    fl = np.zeros(4, np.int32)
    K = O.kernel_at(cfg, a, 0, 0, W, H)
    I2 = conv_same(I.astype(np.float64), K).astype(np.float32)
    q, dev = O.quality(cfg, a, I, I2, V, stamps, fl)
    assert abs(q["kernel_sum"] - 1.0) < 1e-14
    assert abs(q["mom_x"]) < 1e-14 and abs(q["mom_y"]) < 1e-14
    assert abs(q["mom_xx"] - 2.25) < 1e-9 and abs(q["mom_yy"] - 2.25) < 1e-9
    assert abs(q["deconv_max"] - 1.0) < 1e-12
    assert np.all(dev < 1e-10) and abs(q["dev_mean"] + 1.0) < 1e-10
    assert q["cut_flags"] == 0
    b = np.zeros(cfg.n_unknowns)
    b[0] = 1.0
    b[g15] = 1.5
    b[g30] = -0.5
    qd, _ = O.quality(cfg, b, I, I2, V, stamps, fl)
    assert abs(qd["kernel_sum"] - 1.0) < 1e-14
    assert abs(qd["deconv_max"] - 1.164) < 0.03
    assert qd["cut_flags"] & O.CUT_DECONV
    c = a.copy()
    c[term_index(cfg, 1, 1, 0)] = 2.0                 # u-odd term: shifts the kernel along +x
    qs, _ = O.quality(cfg, c, I, I2, V, stamps, fl)
    assert qs["mom_x"] > 0.5 and abs(qs["mom_y"]) < 1e-12
    assert qs["cut_flags"] & O.CUT_MOMENT1
    qf, _ = O.quality(cfg, a, I, I2, V, stamps, np.array([0, 0, 2, 2], np.int32))
    assert qf["n_used"] == 2 and qf["cut_flags"] & O.CUT_FEW_STAMPS


def test_deconvolution_fraction_uses_circular_radius(orc):
    """The enclosed sum is taken within a radius (a circle), not a box: a
    kernel with centre 0.5, the four edge neighbours 0.2 each and the four
    corner neighbours -0.075 each (sum 1) encloses 1.3 within radius 1 (the
    corners lie at sqrt 2), while a box of half-width 1 would already hold
    the corners (1.0)."""
    # one Gaussian times all monomials of degree <= 8 spans every 5 x 5
    # pattern (u^p v^q with p, q <= 4 among them): the target is reproduced
    cfg = O.Config(sigmas=(1.0,), degrees=(8,), h=2, S=0)
    kb = O.basis(cfg).reshape(cfg.n_basis, -1)
    T = np.zeros((5, 5))
    T[2, 2] = 0.5
    T[1, 2] = T[3, 2] = T[2, 1] = T[2, 3] = 0.2
    T[1, 1] = T[1, 3] = T[3, 1] = T[3, 3] = -0.075
    coef, *_ = np.linalg.lstsq(kb.T, T.ravel(), rcond=None)
    K = (coef @ kb).reshape(5, 5)
    assert np.abs(K - T).max() < 1e-10
    a = np.zeros(cfg.n_unknowns)
    a[:cfg.n_basis] = coef
    v, u = np.mgrid[-2:3, -2:3]
    enc = [K[u * u + v * v <= rho * rho].sum() / K.sum() for rho in range(0, 4)]
    I = np.full((60, 60), 10.0, np.float32)
    q, _ = O.quality(cfg, a, I, I, I, np.array([[30, 30]], np.int32), np.zeros(1, np.int32))
    assert abs(q["deconv_max"] - max(enc)) < 1e-12
    box1 = K[1:4, 1:4].sum() / K.sum()
    circ1 = enc[1]
    assert circ1 - box1 > 0.1 and abs(q["deconv_max"] - circ1) < 1e-12
