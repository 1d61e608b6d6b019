"""Pins of the FP64 CNN oracle: brute-force convolution sums, a delta kernel,
output sizes, central finite differences of the loss, and Adam's first step."""
import numpy as np
import pytest

from oracle import cnn_oracle as C


def test_shapes_and_parameter_count():
    assert C.SIDES == [41, 41, 21, 11, 6]
    assert C.FLAT == 1152
    # conv1 2*32*9+32, conv2..4 32*32*9+32, fc1 1152*128+128, fc2 128*49+49
    assert C.n_params() == 608 + 3 * 9248 + 147584 + 6321 == 182257


def test_conv_matches_brute_force_sums():
    rng = np.random.default_rng(0)
    for s in (1, 2):
        x = rng.standard_normal((2, 3, 7, 7))
        w = rng.standard_normal((4, 3, 3, 3))
        b = rng.standard_normal(4)
        y = C.conv_forward(x, w, b, s)
        Ho = (7 + 2 - 3) // s + 1
        assert y.shape == (2, 4, Ho, Ho)
        for bb in range(2):
            for o in range(4):
                for i in range(Ho):
                    for j in range(Ho):
                        acc = b[o]
                        for c in range(3):
                            for u in range(3):
                                for v in range(3):
                                    p, q = s * i + u - 1, s * j + v - 1
                                    if 0 <= p < 7 and 0 <= q < 7:
                                        acc += w[o, c, u, v] * x[bb, c, p, q]
                        assert abs(y[bb, o, i, j] - acc) < 1e-12


def test_delta_kernel_is_identity():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 2, 9, 9))
    w = np.zeros((2, 2, 3, 3))
    w[0, 0, 1, 1] = 1.0
    w[1, 1, 1, 1] = 1.0
    assert np.array_equal(C.conv_forward(x, w, np.zeros(2), 1), x)
    # stride 2 keeps every other pixel
    assert np.array_equal(C.conv_forward(x, w, np.zeros(2), 2), x[:, :, ::2, ::2])


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    theta = C.init_params(3) + 0.01 * rng.standard_normal(C.n_params())
    x = rng.standard_normal((2, 2, 41, 41))
    t = rng.standard_normal((2, 49))
    loss, g = C.loss_and_grad(theta, x, t)
    assert np.isfinite(loss)
    # probe parameters in every tensor
    offs, o = [], 0
    for name, shp in C.layer_shapes():
        n = int(np.prod(shp))
        offs += list(rng.choice(np.arange(o, o + n), size=min(6, n), replace=False))
        o += n
    h = 1e-6
    for k in offs:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (C.loss_and_grad(tp, x, t)[0] - C.loss_and_grad(tm, x, t)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g[k]), 1e-3), (k, fd, g[k])


def test_weighted_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    theta = C.init_params(5) + 0.01 * rng.standard_normal(C.n_params())
    x = rng.standard_normal((2, 2, 41, 41))
    t = rng.standard_normal((2, 49))
    A = rng.standard_normal((2, 49, 49))
    Wt = A @ A.transpose(0, 2, 1) / 49.0                       # symmetric positive definite
    loss, g = C.loss_and_grad(theta, x, t, Wt)
    out = C.forward(theta, x)
    r = out - t
    assert abs(loss - sum(r[b] @ Wt[b] @ r[b] for b in range(2)) / r.size) < 1e-12 * abs(loss)
    # identity weights give the plain loss and gradient
    l0, g0 = C.loss_and_grad(theta, x, t)
    l1, g1 = C.loss_and_grad(theta, x, t, np.broadcast_to(np.eye(49), (2, 49, 49)))
    assert abs(l0 - l1) < 1e-14 * abs(l0) and np.allclose(g0, g1, rtol=1e-12, atol=0)
    h = 1e-6
    for k in rng.choice(C.n_params(), size=12, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (C.loss_and_grad(tp, x, t, Wt)[0] - C.loss_and_grad(tm, x, t, Wt)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g[k]), 1e-3), (k, fd, g[k])


def test_adam_first_step_is_lr_times_sign():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 4.0])
    new, m, v = C.adam_step(theta, np.zeros(3), np.zeros(3), g, 1, lr=0.01, eps=0.0)
    assert np.allclose(new, theta - 0.01 * np.sign(g), rtol=0, atol=1e-15)
