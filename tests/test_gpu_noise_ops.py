"""Noise-model operations beyond convolution on the GPU (Section 4.3)
against the FP64 oracle, through the C interface.

Binned image sums are FP64 sums of the same FP32 inputs in the oracle's
order (bit-exact); the binned variance carries the covariance factor, formed
from the pseudo-matrix in another order (1e-12 relative before the FP32
rounding, so within one FP32 ulp); pseudo-matrices 1e-12; the weighted sum
of images and its variance are the oracle's FP64 expressions rounded once
to FP32 (bit-exact for coefficients +-1; otherwise the device may fuse a
product into an FP64 FMA, one FP32 ulp), its pseudo-matrix 1e-12 (variance
means summed per workgroup).
"""
import numpy as np
import pytest
from scipy import signal

import oracle as O

from gpu_common import hip

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _pseudo(g):
    c = signal.correlate2d(g, g, mode="full")
    k = c.shape[0] // 2
    return c / c[k, k]


def _planes(W, H, seed, mask=True):
    rng = np.random.default_rng(seed)
    I = rng.normal(100, 10, (H, W)).astype(np.float32)
    V = rng.uniform(50, 150, (H, W)).astype(np.float32)
    M = np.zeros((H, W), np.uint8)
    if mask:
        M[rng.integers(0, H, 40), rng.integers(0, W, 40)] = 1
        M[:, 17:21] = 2
    return I, V, M


@pytest.mark.parametrize("W,H,B,corr", [(1003, 777, 2, True), (640, 480, 3, False), (512, 515, 8, True)])
def test_binning_matches_oracle(W, H, B, corr):
    torch, psfm = hip()
    I, V, M = _planes(W, H, B)
    g = np.array([[0.0, 0.4, 0.1], [0.3, 1.0, 0.5], [0.1, 0.2, 0.0]])
    cin = _pseudo(g) if corr else None
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Ib, Vb, Mb, cov, disc = psfm.bin_image(t(I), t(V), t(M), B, cov_in=None if cin is None else t(cin),
                                           c_out=3)
    rI, rV, rM, rC, rd = O.bin_image(I, V, M, B, cov_in=cin, c_out=3)
    assert np.array_equal(_np(Ib), rI) and np.array_equal(_np(Mb), rM)
    vg = _np(Vb)
    assert np.array_equal(vg == 0, rV == 0)
    assert np.max(np.abs(vg - rV) / np.where(rV > 0, rV, 1.0)) < 2.4e-7
    assert np.max(np.abs(_np(cov) - rC)) < 1e-12
    assert abs(float(_np(disc)[0]) - rd) < 1e-12


def test_resample_cov_matches_oracle():
    torch, psfm = hip()
    g = np.array([[0.1, 0.4, 0.1], [0.3, 1.0, 0.5], [0.1, 0.2, 0.3]])
    c = _pseudo(signal.convolve2d(g, g))
    ct = torch.from_numpy(c).cuda()
    for scale, c_out in [(1.0, 4), (1.37, 3), (0.55, 7), (2.5, 2)]:
        got = _np(psfm.resample_cov(ct, scale, c_out))
        ref = O.resample_cov(c, scale, c_out)
        assert np.max(np.abs(got - ref)) < 1e-12, scale


@pytest.mark.parametrize("alpha,beta", [(1.0, -1.0), (0.7, 1.3)])
def test_add_images_matches_oracle(alpha, beta):
    torch, psfm = hip()
    W, H = 1500, 1201
    Ia, Va, Ma = _planes(W, H, 5)
    Ib, Vb, Mb = _planes(W, H, 6)
    ga = np.array([[0.0, 0.3, 0.0], [0.2, 1.0, 0.4], [0.0, 0.1, 0.0]])
    Ca, Cb = _pseudo(ga), None
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    r = psfm.add_images(alpha, t(Ia), t(Va), t(Ma), t(Ca), beta, t(Ib), t(Vb), t(Mb), None, 3)
    S, VS, MS, CS = O.add_images(alpha, Ia, Va, Ma, Ca, beta, Ib, Vb, Mb, Cb, 3)
    sg, vg = _np(r["S"]), _np(r["VS"])
    assert np.max(np.abs(sg - S) / np.maximum(np.abs(S), 1e-30)) <= 1.2e-7
    assert np.max(np.abs(vg - VS) / np.maximum(VS, 1e-30)) <= 1.2e-7
    if abs(alpha) == 1.0 and abs(beta) == 1.0:
        assert np.array_equal(sg, S) and np.array_equal(vg, VS)
    assert np.array_equal(_np(r["MS"]), MS)
    assert np.max(np.abs(_np(r["cov"]) - CS)) < 1e-12
