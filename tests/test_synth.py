"""The input generators (no method arithmetic): the device renderer, run here
on the CPU through torch, follows the same recipe as the numpy one."""
import math

import numpy as np
import pytest

from paper_1901_09999_amd import synth


def test_batch_workloads_follow_the_spec():
    spec = synth.BATCHES["batch64"]
    wls = [synth.batch_pair_workload(spec, k) for k in range(spec.n_pairs)]
    assert len(wls) == 64
    for wl in wls:
        assert spec.size_lo <= wl.width <= spec.size_hi and spec.size_lo <= wl.height <= spec.size_hi
        assert spec.stamps_lo <= wl.n_stamps <= spec.stamps_hi and 0 <= wl.spatial_order <= 3
        assert wl.ref_psf.sigma_lo <= wl.sci_psf.sigma_lo        # the narrower image is convolved
        assert 1.0 <= wl.ref_psf.sigma_lo and wl.sci_psf.sigma_lo <= 3.0
        assert wl.kernel_half == 10 and wl.stamp_half == 20 and wl.variable_frac == 0.05
    px = sum(wl.pixels for wl in wls)
    assert 5e8 < px < 1.1e9          # E[px] = 64 x 3512^2 ~ 7.9e8
    assert len({wl.spatial_order for wl in wls}) == 4


def test_device_generator_on_cpu():
    torch = pytest.importorskip("torch")
    wl = synth.scaled(synth.WORKLOADS["pair2048"], "gen", 400, 330, n_sources=300, n_stamps=30,
                      variable_frac=0.05)
    p = synth.make_pair_device(wl, 1234, device="cpu")
    M1, M2 = p.M1.numpy(), p.M2.numpy()
    assert M1.mean() >= wl.mask_frac and M2.mean() >= wl.mask_frac
    for I, V, M in ((p.I1, p.V1, M1), (p.I2, p.V2, M2)):
        I, V = I.numpy(), V.numpy()
        assert np.all(np.isnan(I[M != 0])) and np.all(np.isnan(V[M != 0]))
        assert np.all(np.isfinite(I[M == 0])) and np.all(V[M == 0] >= wl.sky * 0.999)
    # stamps: the device footprint test picks what the summed-area one picks
    ref = synth.select_stamps(p.xs, p.ys, p.fluxes, M1, M2, wl.n_stamps, wl.stamp_half,
                              wl.kernel_half)
    assert p.stamps.shape[0] > 5 and np.array_equal(p.stamps, ref)
    # the rendered flux of an isolated unmasked source matches its catalogue flux
    V1 = p.V1.numpy()
    k = int(np.argmax(p.fluxes))
    x, y = int(p.xs[k]), int(p.ys[k])
    R = 12
    if R <= x < wl.width - R and R <= y < wl.height - R and not M1[y - R:y + R, x - R:x + R].any():
        box = V1[y - R:y + R, x - R:x + R] - wl.sky
        assert box.sum() == pytest.approx(p.fluxes[k], rel=0.05)
