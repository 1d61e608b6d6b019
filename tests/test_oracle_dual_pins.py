"""Pins of the oracle's two-kernel form (Section 2, Eqs. 1-4, penalty of
Eq. 9): the penalised solution equals the ridge least-squares solution of the
explicit design matrix built here from convolutions of both images; the
penalty weight of an odd Gaussian term against its closed form; growing the
penalty shrinks the penalised norm and raises the data chi2; on images whose
PSFs are elongated along orthogonal axes the two-kernel form matches where
the single kernel (which would have to deconvolve) cannot; K2 has unit sum;
the difference image, its variance and mask against direct convolutions."""
import math

import numpy as np
import pytest
from scipy import signal

import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def conv_same(img, K):
    return signal.convolve2d(img, K, mode="same", boundary="fill", fillvalue=0.0)


def render(W, H, xs, ys, fl, sx, sy):
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.zeros((H, W))
    for x0, y0, f in zip(xs, ys, fl):
        img += f / (2 * math.pi * sx * sy) * np.exp(-0.5 * (((x - x0) / sx) ** 2 + ((y - y0) / sy) ** 2))
    return img


def spatial_terms(S, x, y, W, H):
    xt = (2.0 * x - (W - 1)) / (W - 1)
    yt = (2.0 * y - (H - 1)) / (H - 1)
    return np.array([xt ** l * yt ** (d - l) for d in range(S + 1) for l in range(d, -1, -1)])


def _pair(W, H, n_src, seed, s1=(1.2, 2.2), s2=(2.2, 1.2), noise=1.0, bg=(20.0, 35.0)):
    rng = np.random.default_rng(seed)
    xs = rng.uniform(8, W - 8, n_src)
    ys = rng.uniform(8, H - 8, n_src)
    fl = np.exp(rng.uniform(math.log(300), math.log(3e4), n_src))
    I1 = render(W, H, xs, ys, fl, *s1) + bg[0]
    I2 = render(W, H, xs, ys, fl, *s2) + bg[1]
    V1 = np.abs(I1) + noise ** 2
    V2 = np.abs(I2) + noise ** 2
    I1 = I1 + np.sqrt(V1) * rng.standard_normal((H, W))
    I2 = I2 + np.sqrt(V2) * rng.standard_normal((H, W))
    return (I1.astype(np.float32), V1.astype(np.float32), I2.astype(np.float32), V2.astype(np.float32),
            xs, ys)


def _stamps(xs, ys, W, H, R, n):
    keep = [(int(round(x)), int(round(y))) for x, y in zip(xs, ys)
            if R <= round(x) < W - R and R <= round(y) < H - R]
    return np.array(keep[:n], dtype=np.int32)


@pytest.mark.parametrize("with_v1", [False, True])
def test_penalised_solution_is_ridge_least_squares(orc, with_v1):
    """One solution (no rejection) of the oracle equals the minimiser of
    sum w (A a - I2)^2 + sum P_j a_j^2 with A built here: for every stamp
    pixel, the columns g_s(stamp) k_i (x) I1, g_s(stamp) k_i (x) I2 (i >= 1)
    and 1, and P_j = Phi Q_i on the b-terms i >= 1 and all c-terms; w is
    1 / V2, or 1 / (V1 + V2) when V1 is given."""
    cfg = O.Config(sigmas=(0.8, 1.6), degrees=(2, 1), h=4, r=5, S=1, max_iter=1)
    W = H = 90
    I1, V1, I2, V2, xs, ys = _pair(W, H, 40, 3)
    Z = np.zeros((H, W), np.uint8)
    st = _stamps(xs, ys, W, H, cfg.r + cfg.h, 14)
    kb = O.basis(cfg)
    nb, ns = cfg.n_basis, cfg.n_spatial
    fit = O.fit_dual(cfg, I1, Z, I2, V2, Z, st, V1=V1 if with_v1 else None)
    assert np.all(fit["flags"] == 0)
    phi = 0.05
    ret, a, chi2, fl, stats = O.solve_dual(cfg, W, H, st, fit, phi)
    assert ret == 0
    c1 = [conv_same(I1.astype(np.float64), kb[i]) for i in range(nb)]
    c2 = [conv_same(I2.astype(np.float64), kb[i]) for i in range(nb)]
    rows, ws, ds = [], [], []
    for (xc, yc) in st:
        g = spatial_terms(cfg.S, xc, yc, W, H)
        for y in range(yc - cfg.r, yc + cfg.r + 1):
            for x in range(xc - cfg.r, xc + cfg.r + 1):
                row = [g[s] * c1[i][y, x] for i in range(nb) for s in range(ns)]
                row += [g[s] * c2[i][y, x] for i in range(1, nb) for s in range(ns)]
                row.append(1.0)
                rows.append(row)
                ws.append(1.0 / (float(V2[y, x]) + (float(V1[y, x]) if with_v1 else 0.0)))
                ds.append(float(I2[y, x]))
    A = np.array(rows)
    w = np.array(ws)
    d = np.array(ds)
    M = A.T @ (w[:, None] * A)
    v = A.T @ (w * d)
    Q = np.array([((np.add.outer(np.arange(-cfg.h, cfg.h + 1) ** 2,
                                 np.arange(-cfg.h, cfg.h + 1) ** 2)) ** 2 * kb[i] ** 2).sum()
                  for i in range(nb)])
    pen = np.zeros(A.shape[1])
    for i in range(1, nb):
        pen[i * ns:(i + 1) * ns] = Q[i]
        pen[(nb + i - 1) * ns:(nb + i) * ns] = Q[i]
    Phi = phi * np.diag(M)[pen > 0].sum() / pen[pen > 0].sum()
    expect = np.linalg.solve(M + np.diag(Phi * pen), v)
    assert np.allclose(a, expect, rtol=1e-6, atol=1e-9 * np.abs(expect).max())
    # the data chi2 of the solution
    r = A @ a - d
    assert abs(stats["chi2"] / (w * r * r).sum() - 1) < 1e-8
    assert stats["dof"] == len(d) - A.shape[1]


def test_penalty_weight_closed_form(orc):
    """Q of the odd term u g / sum|u g| (one Gaussian, s = 2): the numerator
    sum (u^2 + v^2)^2 u^2 g^2 equals its integral 3 pi s^8 (sampling error
    ~exp(-pi^2 s^2)); the normaliser is a product of 1-D sums."""
    s, h = 2.0, 14
    cfg = O.Config(sigmas=(s,), degrees=(1,), h=h, r=4)
    Q = O.penalty_q(cfg)
    t = np.arange(-h, h + 1, dtype=np.float64)
    A = (np.abs(t) * np.exp(-t * t / (2 * s * s))).sum() * np.exp(-t * t / (2 * s * s)).sum()
    expect = 3 * math.pi * s ** 8 / A ** 2
    assert abs(Q[1] / expect - 1) < 1e-9 and abs(Q[2] / expect - 1) < 1e-9


def test_penalty_shrinks_the_kernels(orc):
    """Ridge behaviour: larger phi, smaller penalised norm sum Q a^2 and
    larger data chi2 (strictly, over three decades)."""
    cfg = O.Config(sigmas=(0.8, 1.6), degrees=(2, 1), h=4, r=5, S=0, max_iter=1)
    W = H = 90
    I1, V1, I2, V2, xs, ys = _pair(W, H, 40, 4)
    Z = np.zeros((H, W), np.uint8)
    st = _stamps(xs, ys, W, H, cfg.r + cfg.h, 14)
    fit = O.fit_dual(cfg, I1, Z, I2, V2, Z, st)
    Q = O.penalty_q(cfg)
    nb = cfg.n_basis
    norms, chis = [], []
    for phi in (0.001, 0.01, 0.1, 1.0):
        ret, a, chi2, fl, stats = O.solve_dual(cfg, W, H, st, fit, phi)
        assert ret == 0
        qa = sum(Q[i] * a[i] ** 2 for i in range(1, nb)) + sum(Q[i] * a[nb + i - 1] ** 2 for i in range(1, nb))
        norms.append(qa)
        chis.append(stats["chi2"])
    assert all(x > y for x, y in zip(norms, norms[1:]))
    assert all(x < y for x, y in zip(chis, chis[1:]))


def test_orthogonal_elongation_needs_two_kernels(orc):
    """I1 narrow in x and wide in y, I2 the other way round: one kernel on
    I1 would have to deconvolve along y and leaves chi2/dof far above 1; the
    two-kernel form goes far below it (its residual is a difference of two
    smoothed images, measured against V2).  K2 has unit sum; K1 keeps the
    flux (the images share their sources)."""
    cfg = O.Config(h=8, r=10, S=0, max_iter=1)
    W = H = 200
    I1, V1, I2, V2, xs, ys = _pair(W, H, 120, 5)
    Z = np.zeros((H, W), np.uint8)
    st = _stamps(xs, ys, W, H, cfg.r + cfg.h, 60)
    fit1 = O.fit_stamps(cfg, I1, Z, I2, V2, Z, st)
    ret1, a1, _, _, s1 = O.solve(cfg, W, H, st, fit1)
    fit2 = O.fit_dual(cfg, I1, Z, I2, V2, Z, st)
    ret2, a2, _, _, s2 = O.solve_dual(cfg, W, H, st, fit2, 0.01)
    assert ret1 == 0 and ret2 == 0
    print(f"single chi2/dof {s1['chi2_dof']:.3f}, two kernels {s2['chi2_dof']:.3f}")
    assert s2["chi2_dof"] < 1.3 and s1["chi2_dof"] > 2.0 * s2["chi2_dof"]
    K1, K2 = O.dual_kernels(cfg, a2, W / 2, H / 2, W, H)
    assert abs(K2.sum() - 1.0) < 1e-12
    assert abs(K1.sum() - 1.0) < 0.02


def test_dual_apply_against_direct_convolutions(orc):
    """D = K2 (x) I2 - K1 (x) I1 - d0 and V_D = K1^2 (x) V1 + K2^2 (x) V2 in
    one patch's interior, from the patch kernels convolved here; the unit sum
    of K2 and its centre term delta; a masked I1 pixel gives CONV_BAD within
    K1's BAD radius and CONV_POOR out to h."""
    cfg = O.Config(sigmas=(0.8, 1.6), degrees=(2, 1), h=4, r=5, S=1, P=40)
    W, H = 120, 80
    rng = np.random.default_rng(9)
    I1 = rng.normal(50, 5, (H, W)).astype(np.float32)
    I2 = rng.normal(60, 5, (H, W)).astype(np.float32)
    V1 = rng.uniform(20, 30, (H, W)).astype(np.float32)
    V2 = rng.uniform(20, 30, (H, W)).astype(np.float32)
    M1 = np.zeros((H, W), np.uint8)
    M2 = np.zeros((H, W), np.uint8)
    M1[20, 60] = 1
    M2[60, 20] = 1
    N2 = O.dual_unknowns(cfg)
    a = rng.normal(0, 0.05, N2)
    a[0] = 1.0
    a[-1] = 3.0
    D, VD, MD = O.dual_apply(cfg, a, I1, V1, M1, I2, V2, M2)
    kb = O.basis(cfg)
    nb, ns = cfg.n_basis, cfg.n_spatial
    # patch (1, 0): x in [40, 80), y in [0, 40)
    xc, yc = 0.5 * (40 + 80 - 1), 0.5 * (0 + 40 - 1)
    K1, K2 = O.dual_kernels(cfg, a, xc, yc, W, H)
    g = spatial_terms(cfg.S, xc, yc, W, H)
    b_loc = [a[i * ns:(i + 1) * ns] @ g for i in range(nb)]
    c_loc = [a[(nb + i - 1) * ns:(nb + i) * ns] @ g for i in range(1, nb)]
    assert np.allclose(K1, sum(b_loc[i] * kb[i] for i in range(nb)), rtol=0, atol=1e-14)
    delta = np.zeros_like(K2)
    delta[cfg.h, cfg.h] = 1.0
    assert np.allclose(K2, delta - sum(c_loc[i - 1] * kb[i] for i in range(1, nb)), rtol=0, atol=1e-14)
    assert abs(K2.sum() - 1) < 1e-13
    I1m = np.where(M1 == 0, I1, 0).astype(np.float64)
    V1m = np.where(M1 == 0, V1, 0).astype(np.float64)
    expD = conv_same(I2.astype(np.float64), K2) - conv_same(I1m, K1) - a[-1]
    expV = conv_same(V1m, K1 ** 2) + conv_same(V2.astype(np.float64), K2 ** 2)
    sl = (slice(5, 35), slice(45, 75))
    assert np.allclose(D[sl], expD[sl], rtol=2e-6, atol=1e-4)
    assert np.allclose(VD[sl], expV[sl], rtol=2e-6, atol=0)
    rb = O.bad_radius(K1, cfg.h, cfg.bad_frac)
    # a masked I2 pixel in patch (0, 1): its mask follows K2 there
    _, K2b = O.dual_kernels(cfg, a, 0.5 * (0 + 40 - 1), 0.5 * (40 + 80 - 1), W, H)
    rb2 = O.bad_radius(K2b, cfg.h, cfg.bad_frac)
    for (py, px), r_bad in [((20, 60), rb), ((60, 20), rb2)]:
        for dy in range(-cfg.h - 1, cfg.h + 2):
            for dx in range(-cfg.h - 1, cfg.h + 2):
                dd = max(abs(dx), abs(dy))
                m = MD[py + dy, px + dx]
                if dd <= r_bad:
                    assert m == O.MASK_CONV_BAD
                elif dd <= cfg.h:
                    assert m == O.MASK_CONV_POOR
                else:
                    assert m == 0


def test_dual_stamp_validity(orc):
    """A masked I2 pixel in a stamp's convolution footprint (outside the
    stamp itself) invalidates that stamp in the two-kernel form (I2 is
    convolved there) but not in the single form; a non-finite I2 pixel
    there flags NONFINITE."""
    cfg = O.Config(sigmas=(0.8, 1.6), degrees=(2, 1), h=4, r=5, S=0)
    W = H = 90
    I1, V1, I2, V2, xs, ys = _pair(W, H, 40, 6)
    st = np.array([[30, 30], [60, 60], [30, 62]], dtype=np.int32)
    Z = np.zeros((H, W), np.uint8)
    M2 = Z.copy()
    M2[30, 30 + cfg.r + 2] = 1                   # in the footprint ring of stamp 0
    I2b = I2.copy()
    I2b[60 - cfg.r - 3, 60] = np.nan             # in the ring of stamp 1
    fd = O.fit_dual(cfg, I1, Z, I2b, V2, M2, st)
    fs = O.fit_stamps(cfg, I1, Z, I2b, V2, M2, st)
    assert fd["flags"].tolist() == [O.STAMP_INVALID, O.STAMP_NONFINITE, 0]
    assert fs["flags"].tolist() == [0, 0, 0]
    assert np.all(fd["M"][:2] == 0) and fd["npix"].tolist() == [0, 0, (2 * cfg.r + 1) ** 2]
