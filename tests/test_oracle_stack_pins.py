"""Pins of the oracle's PSF homogenisation for stacking (Section 5.1, with
the combination of Section 5.2): the envelope of Gaussian PSFs, the moments
of the fake target, the end-to-end homogenisation of two inputs with
different elliptical PSFs to the envelope, median-based outlier flags, the
trace-back of outliers through the matched filter, and the noise of the
weighted stack (Section 4.4 statistic)."""
import math

import numpy as np
import pytest
from scipy import signal

import oracle as O
from paper_1901_09999_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def conv_same(img, K):
    return signal.convolve2d(img, K, mode="same", boundary="fill", fillvalue=0.0)


def test_envelope_of_gaussians(orc):
    """Circular versions (major-axis width, peak 1) of Gaussian PSFs: the
    widest one is the pointwise maximum everywhere, so the envelope is that
    Gaussian and the fit returns its width."""
    params = [(1.5, 1.2, 0.3), (2.1, 1.7, 1.0), (1.8, 1.8, 0.0)]
    s, env = O.envelope_psf(params, 12)
    assert abs(s - 2.1) < 1e-8
    v, u = np.mgrid[-12:13, -12:13]
    assert np.allclose(env, np.exp(-(u * u + v * v) / (2 * 2.1 ** 2)), rtol=0, atol=1e-15)
    assert env[12, 12] == 1.0


def test_fake_target_moments(orc):
    """A sampled unit-flux Gaussian's flux, centroid and variance are exact
    to ~exp(-2 pi^2 sigma^2) (Poisson summation): sources away from the
    edges keep their fluxes and positions, the spread is sigma^2."""
    W, H, sig = 120, 100, 2.3
    src = np.array([[40.3, 30.7, 1000.0], [85.9, 70.2, 250.0]])
    img = O.render_target(src, sig, W, H).astype(np.float64)
    y, x = np.mgrid[0:H, 0:W]
    for (x0, y0, f), box in zip(src, [(slice(10, 52), slice(18, 63)), (slice(50, 92), slice(60, 112))]):
        sub, xs, ys = img[box], x[box], y[box]
        assert abs(sub.sum() / f - 1) < 1e-6
        cx, cy = (xs * sub).sum() / sub.sum(), (ys * sub).sum() / sub.sum()
        assert abs(cx - x0) < 1e-6 and abs(cy - y0) < 1e-6
        assert abs(((xs - cx) ** 2 * sub).sum() / sub.sum() - sig ** 2) < 1e-5


def _star_moments(img, xs, ys, r=9):
    out = []
    H, W = img.shape
    for x0, y0 in zip(xs, ys):
        xi, yi = int(round(x0)), int(round(y0))
        if xi < r or yi < r or xi >= W - r or yi >= H - r:
            continue
        sub = img[yi - r:yi + r + 1, xi - r:xi + r + 1].astype(np.float64)
        sub = sub - np.median(img)
        v, u = np.mgrid[-r:r + 1, -r:r + 1]
        f = sub.sum()
        cx, cy = (u * sub).sum() / f, (v * sub).sum() / f
        out.append((((u - cx) ** 2 * sub).sum() / f, ((v - cy) ** 2 * sub).sum() / f,
                    ((u - cx) * (v - cy) * sub).sum() / f))
    return np.array(out)


def test_homogenisation_brings_inputs_to_the_envelope(orc):
    """Two noiseless inputs with different elliptical PSFs, matched (c = 0)
    to the fake target of their envelope: every isolated star of each
    convolved input has the envelope's second moments (sigma_env^2 on both
    axes, no cross term) to 3%, where the inputs differed by up to 60%."""
    W = H = 320
    rng = np.random.default_rng(7)
    n = 36
    gx, gy = np.meshgrid(np.arange(30, W - 20, 45), np.arange(30, H - 20, 45))
    xs = gx.ravel()[:n] + rng.uniform(-0.5, 0.5, n)
    ys = gy.ravel()[:n] + rng.uniform(-0.5, 0.5, n)
    fl = np.exp(rng.uniform(math.log(5e3), math.log(5e4), n))
    psfs = [(synth.PsfField(1.6, 1.6, 0.25), 0.4), (synth.PsfField(1.3, 1.3, 0.15), 1.2)]
    inputs = [synth._render(W, H, xs, ys, fl, psf, th) + 100.0 for psf, th in psfs]
    # each input's ellipticity grows along y: its envelope entry is the widest
    # (last-row) PSF
    params = []
    for psf, th in psfs:
        sa, sb = psf.params(np.array([W / 2.0]), np.array([H - 1.0]), W, H)
        params.append((float(sa[0]), float(sb[0]), th))
    s_env, _ = O.envelope_psf(params, 15)
    target = O.render_target(np.stack([xs, ys, fl], axis=1), s_env, W, H)
    cfg = O.Config(S=1, max_iter=1)
    stamps = np.stack([np.round(xs), np.round(ys)], axis=1).astype(np.int32)
    Z = np.zeros((H, W), np.uint8)
    m0 = [_star_moments(im, xs, ys) for im in inputs]
    assert abs(m0[0][:, 0].mean() / m0[1][:, 1].mean() - 1) > 0.2          # inputs differ
    for img in inputs:
        I1 = img.astype(np.float32)
        V = (np.abs(img) + 1.0).astype(np.float32)
        fit = O.fit_stamps(cfg, I1, Z, target, V, Z, stamps)
        ret, a, chi2, fl2, st = O.solve(cfg, W, H, stamps, fit)
        assert ret == 0
        conv, cm = O.convolve_image(cfg, a, I1, Z)
        mom = _star_moments(conv, xs, ys)
        assert len(mom) > 20
        assert np.all(np.abs(mom[:, 0] / s_env ** 2 - 1) < 0.03)
        assert np.all(np.abs(mom[:, 1] / s_env ** 2 - 1) < 0.03)
        assert np.all(np.abs(mom[:, 2]) < 0.03 * s_env ** 2)


def test_stack_reject_median(orc):
    """Outliers against the median of the unmasked inputs (numpy's median):
    a planted cosmic ray is flagged in its input only; masked inputs neither
    vote nor get flagged; below 3 unmasked inputs nothing is flagged."""
    rng = np.random.default_rng(3)
    n, H, W = 5, 20, 24
    V = np.full((n, H, W), 4.0, np.float32)
    I = (50 + 2.0 * rng.standard_normal((n, H, W))).astype(np.float32)
    M = np.zeros((n, H, W), np.uint8)
    I[2, 7, 9] += 500.0
    M[0, 7, 9] = 1
    M[:3, 15, 3] = 1                                     # only 2 unmasked here
    I[:, 12, 12] = [0.0, 4.0, 6.0, 15.5, 50.0]           # even count: median 5, not 6
    M[4, 12, 12] = 1
    out = O.stack_reject(I, V, M, 5.0)
    assert out[2, 7, 9] == 1 and out[:, 7, 9].sum() == 1 and out[0, 7, 9] == 0
    assert out[:, 15, 3].sum() == 0
    assert out[3, 12, 12] == 1 and out[:, 12, 12].sum() == 1
    for (y, x) in [(3, 4), (7, 9), (11, 20)]:
        ok = M[:, y, x] == 0
        med = np.median(I[ok, y, x].astype(np.float64))
        expect = ok & (np.abs(I[:, y, x] - med) > 5.0 * 2.0)
        assert np.array_equal(out[:, y, x] == 1, expect)


def test_trace_mask_through_the_matched_filter(orc):
    """One outlier pixel p on the convolved image: the original pixels whose
    kernel weight at p is at least frac of sum |K| are marked (brute force
    on a constant kernel).  A cosmic ray convolved with the kernel and
    flagged where bright is traced back to its own pixel."""
    cfg = O.Config(S=0, P=64)
    W = H = 64
    a = np.zeros(cfg.n_unknowns)
    a[0] = 1.0
    a[28] = 1.0                                          # unit-sum Gaussian, sigma 1.5
    a[29] = 0.2                                          # an odd term: asymmetric kernel
    K = O.kernel_at(cfg, a, 0, 0, W, H)
    h = cfg.h
    outl = np.zeros((H, W), np.uint8)
    p = (30, 33)                                         # (y, x)
    outl[p] = 1
    frac = 0.02
    bad = O.trace_mask(cfg, a, outl, frac)
    tot = np.abs(K).sum()
    expect = np.zeros((H, W), bool)
    for v in range(-h, h + 1):
        for u in range(-h, h + 1):
            if abs(K[v + h, u + h]) >= frac * tot:
                expect[p[0] - v, p[1] - u] = True        # x + u = p
    assert np.array_equal(bad == 1, expect) and expect.sum() > 1
    img = np.zeros((H, W))
    img[20, 40] = 1000.0
    conv = conv_same(img, K)
    flagged = (conv > 10.0).astype(np.uint8)             # the bright part of its footprint
    bad2 = O.trace_mask(cfg, a, flagged, 0.8)
    assert bad2[20, 40] == 1 and bad2.sum() <= 4


def test_weighted_stack_noise_statistic(orc):
    """Three independent correlated-noise inputs of different variance and
    correlation, with masks: the inverse-variance stack, its variance map and
    pseudo-matrix give the Section 4.4 statistic unit std (3%); weights are
    the inverse mean variances; a pixel masked everywhere is masked."""
    rng = np.random.default_rng(5)
    n, H, W = 3, 512, 512
    gs = [np.array([[0.0, 0.3, 0.0], [0.2, 1.0, 0.4], [0.0, 0.1, 0.0]]),
          np.array([[0.2, 0.2, 0.2], [0.2, 1.0, 0.2], [0.2, 0.2, 0.2]]),
          np.array([[0.0, 0.0, 0.0], [0.5, 1.0, 0.5], [0.0, 0.0, 0.0]])]
    sig = [3.0, 1.5, 2.0]
    I = np.stack([conv_same(rng.standard_normal((H, W)) * s, g) for s, g in zip(sig, gs)]).astype(np.float32)
    V = np.stack([np.full((H, W), s * s * (g ** 2).sum()) for s, g in zip(sig, gs)]).astype(np.float32)
    M = np.zeros((n, H, W), np.uint8)
    M[0, 100:110, :] = 1
    M[:, 5, 5] = 1

    def pseudo(g):
        c = signal.correlate2d(g, g, mode="full")
        return c / c[2, 2]
    covs = np.stack([pseudo(g) for g in gs])
    S, VS, MS, CS, w = O.stack_combine(I, V, M, covs)
    assert np.allclose(w, [1.0 / V[k][M[k] == 0].astype(np.float64).mean() for k in range(n)],
                       rtol=1e-12)
    assert MS[5, 5] == 1 and S[5, 5] == 0 and MS.sum() == 1
    y, x = 50, 60
    expect = (w * I[:, y, x]).sum() / w.sum()
    assert abs(S[y, x] - expect) < 1e-5 * abs(expect) + 1e-6
    hm = 6
    g = np.exp(-np.add.outer(np.arange(-hm, hm + 1) ** 2, np.arange(-hm, hm + 1) ** 2) / 8.0)
    g /= g.sum()
    mm = signal.correlate2d(g, g, mode="full")
    Cp = np.zeros((4 * hm + 1, 4 * hm + 1))
    Cp[2 * hm - 2:2 * hm + 3, 2 * hm - 2:2 * hm + 3] = CS
    F = signal.fftconvolve(S.astype(np.float64), g, mode="same")
    sl = (slice(130, H - 30), slice(30, W - 30))          # away from the masked rows
    z = F[sl] / np.sqrt(VS[sl] * (mm * Cp).sum())
    assert abs(z.std() - 1.0) < 0.03
