"""The learned prior on the GPU: the FP16 network kernels against the FP64
CNN oracle, the per-stamp solve and the orthonormal-basis map against the
FP64 method oracle, training, and what the prior gains in the solve.

Tolerances: the kernels keep weights and activations in FP16 (unit roundoff
2^-11) with FP32 accumulation, and the oracle runs on the same FP16-rounded
weights and inputs in FP64.  Each layer's output is rounded once, so the
network output is held to 2e-2 of its scale and every parameter tensor's
gradient to 3e-2 relative L2 error (with cosine similarity > 0.999); the
Adam step is FP32 arithmetic on identical inputs (1e-5 relative).
"""
import numpy as np
import pytest

import oracle as O
from oracle import cnn_oracle as CO
from paper_1901_09999_amd import synth

from gpu_common import hip

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _net_and_batch(B=8, seed=5):
    torch, psfm = hip()
    from paper_1901_09999_amd import cnn
    rng = np.random.default_rng(seed)
    theta = CO.init_params(seed).astype(np.float32)
    theta += (0.01 * rng.standard_normal(theta.size)).astype(np.float32)   # non-zero biases
    net = cnn.Net(params=theta)
    x = rng.standard_normal((B, 2, 41, 41)).astype(np.float16)
    t = (0.3 * rng.standard_normal((B, 49))).astype(np.float32)
    theta16 = theta.astype(np.float16).astype(np.float64)
    return torch, cnn, net, x, t, theta16


def test_forward_matches_oracle():
    torch, cnn, net, x, t, theta16 = _net_and_batch()
    out = _np(net.forward(torch.from_numpy(x).cuda()))
    ref = CO.forward(theta16, x.astype(np.float64))
    err = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
    print(f"forward max error / scale {err:.2e}")
    assert err < 2e-2


def test_forward_ragged_batch_and_unaligned_weights():
    """37 samples: two full 16-sample tiles of the first fully connected
    layer and a ragged one; then the same weights one element past a 16-byte
    boundary, which takes the layer's one-wave-per-output kernel instead."""
    torch, cnn, net, x, t, theta16 = _net_and_batch(B=37, seed=11)
    xd = torch.from_numpy(x).cuda()
    ref = CO.forward(theta16, x.astype(np.float64))
    out = _np(net.forward(xd))
    err = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
    print(f"aligned: forward max error / scale {err:.2e}")
    assert err < 2e-2
    buf = torch.empty(net.w16.numel() + 1, dtype=torch.float16, device=net.w16.device)
    buf[1:].copy_(net.w16)
    net.w16 = buf[1:]
    assert net.w16.data_ptr() % 16 != 0
    out_u = _np(net.forward(xd))
    err_u = np.max(np.abs(out_u - ref)) / np.max(np.abs(ref))
    print(f"unaligned: forward max error / scale {err_u:.2e}")
    assert err_u < 2e-2
    assert np.max(np.abs(out_u - out)) <= 5e-3 * np.max(np.abs(ref))


@pytest.mark.parametrize("B", [8, 37])
def test_gradient_matches_oracle(B):
    """B = 37: the weight-gradient kernels' sample quarters are uneven (10,
    10, 10, 7) and the first fully connected layer's last tile is ragged."""
    torch, cnn, net, x, t, theta16 = _net_and_batch(B=B)
    loss, grad = net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = _np(grad).astype(np.float64)
    l_ref, g_ref = CO.loss_and_grad(theta16, x.astype(np.float64), t.astype(np.float64))
    assert abs(float(loss[0]) / l_ref - 1) < 2e-2
    o = 0
    for name, shp in CO.layer_shapes():
        n = int(np.prod(shp))
        a, b = g[o:o + n], g_ref[o:o + n]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        cos = a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30)
        print(f"{name}: rel {rel:.2e} cos {cos:.6f}")
        assert rel < 3e-2 and cos > 0.999, name
        o += n


def test_weighted_gradient_matches_oracle():
    """The chi2-weighted loss every training step uses: r^T W_b r with SPD
    per-sample weights, loss and per-tensor gradients against the oracle's
    weighted form (same tolerances as the plain loss)."""
    torch, cnn, net, x, t, theta16 = _net_and_batch(B=8, seed=11)
    rng = np.random.default_rng(12)
    Q = rng.standard_normal((8, 49, 49))
    Wt = np.einsum("bij,bkj->bik", Q, Q) / 49.0 + 0.05 * np.eye(49)[None]
    Wt *= np.exp(rng.uniform(-2, 2, 8))[:, None, None]          # per-stamp scales differ
    W32 = Wt.astype(np.float32)
    loss, grad = net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(),
                               weight=torch.from_numpy(W32).cuda())
    g = _np(grad).astype(np.float64)
    l_ref, g_ref = CO.loss_and_grad(theta16, x.astype(np.float64), t.astype(np.float64),
                                    W32.astype(np.float64))
    print(f"weighted loss {float(loss[0]):.6e} oracle {l_ref:.6e}")
    assert abs(float(loss[0]) / l_ref - 1) < 2e-2
    o = 0
    for name, shp in CO.layer_shapes():
        n = int(np.prod(shp))
        a, b = g[o:o + n], g_ref[o:o + n]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        cos = a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30)
        print(f"{name}: rel {rel:.2e} cos {cos:.6f}")
        assert rel < 3e-2 and cos > 0.999, name
        o += n


def test_loss_weights_are_the_chi2_excess():
    """psfm_cnn_loss_weights from the oracle's per-stamp sums: for kernel
    coefficient offsets a (orthonormal form c = R a, mapped by the library),
    c^T W c equals the chi2/dof excess of that kernel with the background
    re-fitted, min over d of [a; d]^T M_s [a; d] / npix, computed from the
    oracle's stamp matrix (FP64) -- a statement independent of the factor R
    the library picked.  Flagged stamps get zero weights."""
    torch, psfm = hip()
    from paper_1901_09999_amd import cnn
    spec = synth.STAMP_SETS["cells200k"]
    planes, stamps, par = synth.make_stamp_cells(spec, 24, 321)
    cfg = O.Config(S=0, min_stamps=1)
    host = {k: _np(v) for k, v in planes.items()}
    fit = O.fit_stamps(cfg, host["I1"], host["M1"], host["I2"], host["V2"], host["M2"], stamps)
    fl = fit["flags"].copy()
    fl[3] = 1                                                   # one stamp flagged on input
    ctx = psfm.Context(psfm.Config(h=10, r=20, S=0, min_stamps=1))
    dfit = dict(M=torch.from_numpy(fit["M"]).cuda(), npix=torch.from_numpy(fit["npix"]).cuda(),
                flags=torch.from_numpy(fl).cuda())
    Wg = _np(cnn.loss_weights(ctx, dfit)).astype(np.float64)
    assert np.all(Wg[3] == 0)
    rng = np.random.default_rng(5)
    n = stamps.shape[0]
    a = np.zeros((n, 50))
    a[:, :49] = 0.01 * rng.standard_normal((n, 49))
    c = _np(cnn.to_ortho(ctx, torch.from_numpy(a).cuda())).astype(np.float64)
    for s in range(n):
        if fl[s]:
            continue
        M = fit["M"][s]
        u = a[s, :49]
        q = lambda d: np.concatenate([u, [d]]) @ M @ np.concatenate([u, [d]])
        d_opt = -(M[49, :49] @ u) / M[49, 49]                # minimiser of the quadratic in d
        assert q(d_opt) <= min(q(d_opt + 1e-3), q(d_opt - 1e-3))
        excess = q(d_opt) / fit["npix"][s]
        got = c[s] @ Wg[s] @ c[s]
        assert abs(got / excess - 1) < 2e-4, (s, got, excess)
        assert np.allclose(Wg[s], Wg[s].T, rtol=0, atol=1e-6 * np.abs(Wg[s]).max())


def test_adam_matches_oracle():
    torch, cnn, net, x, t, theta16 = _net_and_batch()
    rng = np.random.default_rng(9)
    g = (1e-2 * rng.standard_normal(net.w32.numel())).astype(np.float32)
    w0 = _np(net.w32).astype(np.float64)
    m, v = np.zeros_like(w0), np.zeros_like(w0)
    for step in range(1, 4):
        net.grad.copy_(torch.from_numpy(g * step))
        net.adam(1e-3)
        w0, m, v = CO.adam_step(w0, m, v, (g * step).astype(np.float64), step, 1e-3)
    w = _np(net.w32)
    assert np.max(np.abs(w - w0)) <= 1e-5 * np.max(np.abs(w0))
    assert np.array_equal(_np(net.w16), net.w32.cpu().numpy().astype(np.float16))


def test_stamp_inputs_definition():
    torch, psfm = hip()
    from paper_1901_09999_amd import cnn
    wl = synth.scaled(synth.WORKLOADS["pair2048"], "inp", 200, 150, n_sources=60, n_stamps=6)
    p = synth.make_pair(wl, 31)
    d = psfm.to_device(p)
    st = np.array([[100, 75], [10, 12], [190, 140]], np.int32)    # inside, corner, edge
    x = _np(cnn.stamp_inputs(d["I1"], d["M1"], d["I2"], d["M2"], torch.from_numpy(st).cuda()))
    for k, (xc, yc) in enumerate(st):
        win = []
        for I, M in ((p.I1, p.M1), (p.I2, p.M2)):
            w = np.zeros((41, 41)); ok = np.zeros((41, 41), bool)
            for dy in range(-20, 21):
                for dx in range(-20, 21):
                    gx, gy = xc + dx, yc + dy
                    if 0 <= gx < wl.width and 0 <= gy < wl.height and M[gy, gx] == 0:
                        w[dy + 20, dx + 20] = I[gy, gx]; ok[dy + 20, dx + 20] = True
            border = np.zeros((41, 41), bool)
            border[0, :] = border[-1, :] = border[:, 0] = border[:, -1] = True
            bv = w[border & ok]
            sky = bv.mean() if bv.size else 0.0
            sig = bv.std() if bv.size > 1 else 0.0
            win.append((w, ok, sky, sig))
        (w1, ok1, s1, sg1), (w2, ok2, s2, _) = win
        f = ((w1 - s1) * ok1).sum()
        den = max(f, 3.0 * sg1 * np.sqrt(ok1.sum()))
        for c, (w, ok, s, _) in enumerate(win):
            ref = np.where(ok, (w - s) * 100.0 / den, 0.0) if den > 0 else np.zeros((41, 41))
            ref = np.clip(ref, -60000.0, 60000.0)
            assert np.max(np.abs(x[k, c] - ref)) <= 2e-3 * max(np.max(np.abs(ref)), 1.0), (k, c)


def test_per_stamp_solve_and_ortho_map_against_oracle():
    torch, psfm = hip()
    from paper_1901_09999_amd import cnn
    spec = synth.STAMP_SETS["cells200k"]
    planes, stamps, par = synth.make_stamp_cells(spec, 64, 123)
    ctx = psfm.Context(psfm.Config(h=10, r=20, S=0, min_stamps=1))
    st = torch.from_numpy(stamps).cuda()
    fit = ctx.fit_stamps(planes["I1"], planes["M1"], planes["I2"], planes["V2"], planes["M2"], st)
    local, chi2 = ctx.solve_stamps(fit)
    local, chi2 = _np(local), _np(chi2)
    Ms, bs, es = _np(fit["M"]), _np(fit["b"]), _np(fit["e"])
    cfg = O.Config(S=0, min_stamps=1)
    for s in range(64):
        a, info = O.cholesky_solve(Ms[s], bs[s])
        assert info == 0
        c_ref = es[s] - 2 * a @ bs[s] + a @ Ms[s] @ a
        assert abs(chi2[s] / c_ref - 1) < 1e-8
        assert abs(local[s, 0] / a[0] - 1) < 1e-6          # kernel sum = a_0
    # orthonormal map: |R a| = |sum_i a_i k_i| (oracle basis taps), and back
    kb = O.basis(cfg).reshape(49, -1)
    orth = _np(cnn.to_ortho(ctx, torch.from_numpy(local).cuda())).astype(np.float64)
    K = local[:, :49] @ kb
    assert np.allclose(np.linalg.norm(orth, axis=1), np.linalg.norm(K, axis=1), rtol=1e-5)
    back = _np(cnn.to_local(ctx, torch.from_numpy(orth.astype(np.float32)).cuda()))
    Kb = back[:, :49] @ kb
    assert np.max(np.abs(Kb - K)) < 1e-5 * np.max(np.abs(K))


def test_training_reduces_validation_loss():
    torch, psfm = hip()
    from paper_1901_09999_amd import cnn
    data = cnn.make_dataset(12288, 2024, chunk=12288)
    n = data["x"].shape[0]
    tr, val = slice(0, n - 1024), slice(n - 1024, n)
    view = cnn.standardize(data, n - 1024)
    net = cnn.Net(seed=1)
    xv, zv, wv = view["x"][val], view["target"][val], view["weight"][val]
    before = cnn.evaluate(net, xv, zv, 512, wv)
    hist = cnn.train(net, {k: view[k][tr] for k in ("x", "target", "weight")}, epochs=6,
                     batch=128, lr=1e-3)
    after = cnn.evaluate(net, xv, zv, 512, wv)
    mean0 = cnn.evaluate_constant(torch.zeros(49, device=zv.device), zv, wv)
    print(f"weighted validation loss {before:.4e} -> {after:.4e} (mean predictor {mean0:.4e}); "
          f"{hist['steps']} steps in {hist['seconds']:.2f} s")
    assert after < 0.5 * before and after < 0.5 * mean0
    # folded output = orthonormal coefficients; predicted kernel sums against the method's
    net.fold_output(view["mu"], view["sd"])
    ctx = psfm.Context(psfm.Config(h=10, r=20, S=0, min_stamps=1))
    pred = _np(cnn.to_local(ctx, net.forward(data["x"][val])))
    ks = np.abs(pred[:, 0] / _np(data["local"][val])[:, 0] - 1)
    print(f"median kernel-sum error of the predictions {np.median(ks):.3e}")
    assert np.median(ks) < 0.1


def test_standardize_fold_and_excess_against_numpy():
    """psfm_cnn_standardize (column statistics over a prefix of the rows,
    z-scores and the weights carried into z coordinates), psfm_cnn_excess
    (r^T W r per sample, also for a constant predictor) and
    psfm_cnn_fold_output (the folded network returns sd * out + mu) against
    FP64 numpy on random SPD weights.  FP32 data with FP64 sums: 1e-5
    relative; the folded output layer, rounded to FP16 again: 1e-2 of the output
    scale."""
    torch, psfm = hip()
    from paper_1901_09999_amd import cnn
    rng = np.random.default_rng(3)
    n, n_stats = 300, 250
    T = (rng.normal(0, 1, (n, 49)) * rng.uniform(0.1, 5, 49) + rng.normal(0, 3, 49)).astype(np.float32)
    A = rng.normal(size=(n, 49, 49))
    W = (A @ A.transpose(0, 2, 1) / 49).astype(np.float32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    v = cnn.standardize(dict(x=None, target=t(T), weight=t(W)), n_stats)
    T64, W64 = T.astype(np.float64), W.astype(np.float64)
    mu, sd = T64[:n_stats].mean(0), T64[:n_stats].std(0, ddof=1)
    assert np.allclose(_np(v["mu"]), mu, rtol=1e-5, atol=1e-6)
    assert np.allclose(_np(v["sd"]), sd, rtol=1e-5)
    z = (T64 - mu) / sd
    assert np.max(np.abs(_np(v["target"]) - z)) < 1e-5 * np.max(np.abs(z))
    Wz = W64 * sd[None, :, None] * sd[None, None, :]
    Wz /= (np.einsum("sii->s", Wz) / 49)[:, None, None]
    assert np.max(np.abs(_np(v["weight"]) - Wz)) < 1e-5 * np.max(np.abs(Wz))
    P = rng.normal(size=(n, 49)).astype(np.float32)
    r = P.astype(np.float64) - T64
    ref = np.einsum("bi,bij,bj->b", r, W64, r)
    assert np.allclose(_np(cnn.quad_excess(t(P), t(T), t(W))), ref, rtol=1e-5)
    c = P[0]
    rc = c.astype(np.float64)[None, :] - T64
    refc = np.einsum("bi,bij,bj->b", rc, W64, rc)
    assert np.allclose(_np(cnn.quad_excess(t(c), t(T), t(W))), refc, rtol=1e-5)
    assert abs(cnn.evaluate_constant(t(c), t(T), t(W)) / (refc.sum() / T.size) - 1) < 1e-5
    # the folded network
    net = cnn.Net(seed=2)
    x = t(rng.standard_normal((16, 2, 41, 41)).astype(np.float16))
    out0 = _np(net.forward(x)).astype(np.float64)
    net.fold_output(v["mu"], v["sd"])
    out1 = _np(net.forward(x)).astype(np.float64)
    expect = out0 * _np(v["sd"]) + _np(v["mu"])
    assert np.max(np.abs(out1 - expect)) < 1e-2 * np.max(np.abs(expect))
