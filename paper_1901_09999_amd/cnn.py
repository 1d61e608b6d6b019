"""Learned prior of the kernel fit (binding and training driver).

A small CNN predicts each stamp's kernel from the stamp pair; it is trained
on single-star stamp pairs whose targets are the kernels the method itself
solves for each stamp (psfm_fit_stamps + psfm_solve_stamps).  In use, its
predictions feed psfm_solve_prior: a warm start and a rejection prior, with
the full least-squares solve as the fallback and the final word.

This module only marshals: the network's forward, loss gradient and Adam
steps run in the library's FP16 kernels (psfm_cnn_*).
"""
from __future__ import annotations

import ctypes as C
import math
import time
from typing import Callable, Dict, Optional

import numpy as np
import torch

from . import psfm, synth
from .psfm import _check, _ptr, _stream, lib

OUT = 49
SIDE = 41


def param_count() -> int:
    return int(lib().psfm_cnn_param_count())


def layer_shapes():
    shapes, cin = [], 2
    for k in range(4):
        shapes += [(f"conv{k + 1}.w", (32, cin, 3, 3)), (f"conv{k + 1}.b", (32,))]
        cin = 32
    return shapes + [("fc1.w", (128, 1152)), ("fc1.b", (128,)), ("fc2.w", (OUT, 128)),
                     ("fc2.b", (OUT,))]


def he_init(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in layer_shapes():
        if name.endswith(".b"):
            parts.append(np.zeros(int(np.prod(shp))))
        else:
            parts.append(rng.standard_normal(int(np.prod(shp))) * math.sqrt(2.0 / np.prod(shp[1:])))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == param_count()
    return theta


class Net:
    """Parameters (FP32 master, FP16 working copy), Adam moments and the
    library workspace for one batch size."""

    def __init__(self, device=None, seed: int = 0, params: Optional[np.ndarray] = None):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        theta = he_init(seed) if params is None else np.asarray(params, np.float32)
        self.w32 = torch.from_numpy(theta.copy()).to(self.device)
        self.w16 = self.w32.to(torch.float16)
        self.m = torch.zeros_like(self.w32)
        self.v = torch.zeros_like(self.w32)
        self.grad = torch.zeros_like(self.w32)
        self.step = 0
        self._ws: Dict[int, torch.Tensor] = {}

    def workspace(self, batch: int) -> torch.Tensor:
        ws = self._ws.get(batch)
        if ws is None:
            self._ws = {batch: torch.empty(int(lib().psfm_cnn_workspace_bytes(batch)), dtype=torch.uint8,
                                           device=self.device)}
            ws = self._ws[batch]
        return ws

    def forward(self, x16: torch.Tensor) -> torch.Tensor:
        B = x16.shape[0]
        out = torch.empty((B, OUT), dtype=torch.float32, device=self.device)
        ws = self.workspace(B)
        _check(lib().psfm_cnn_forward(_ptr(self.w16), _ptr(x16), B, _ptr(out), _ptr(ws), ws.numel(),
                                      _stream()), "psfm_cnn_forward")
        return out

    def loss_grad(self, x16: torch.Tensor, target: torch.Tensor, loss: Optional[torch.Tensor] = None,
                  weight: Optional[torch.Tensor] = None):
        B = x16.shape[0]
        loss = torch.zeros(1, dtype=torch.float32, device=self.device) if loss is None else loss
        ws = self.workspace(B)
        _check(lib().psfm_cnn_loss_grad(_ptr(self.w16), _ptr(x16), _ptr(target), _ptr(weight), B,
                                        _ptr(self.grad), _ptr(loss), _ptr(ws), ws.numel(), _stream()),
               "psfm_cnn_loss_grad")
        return loss, self.grad

    def adam(self, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        _check(lib().psfm_cnn_adam(_ptr(self.w32), _ptr(self.w16), _ptr(self.m), _ptr(self.v),
                                   _ptr(self.grad), self.w32.numel(), self.step, lr, b1, b2, eps,
                                   _stream()), "psfm_cnn_adam")

    def fold_output(self, mu: torch.Tensor, sd: torch.Tensor):
        """psfm_cnn_fold_output: make the network output sd * z + mu directly
        (z its current output)."""
        _check(lib().psfm_cnn_fold_output(_ptr(self.w32), _ptr(self.w16), _ptr(mu.contiguous()),
                                          _ptr(sd.contiguous()), _stream()), "psfm_cnn_fold_output")

    def state(self) -> dict:
        return dict(w32=self.w32.cpu().numpy(), m=self.m.cpu().numpy(), v=self.v.cpu().numpy(),
                    step=np.int64(self.step))

    def save(self, path: str):
        np.savez(path, **self.state())

    @classmethod
    def load(cls, path: str, device=None) -> "Net":
        with np.load(path) as f:
            net = cls(device=device, params=f["w32"])
            net.m.copy_(torch.from_numpy(f["m"]))
            net.v.copy_(torch.from_numpy(f["v"]))
            net.step = int(f["step"])
        return net


def stamp_inputs(I1, M1, I2, M2, stamps) -> torch.Tensor:
    """Network inputs (n x 2 x 41 x 41 FP16) of the stamps of one pair."""
    H, W = I1.shape
    n = stamps.shape[0]
    x = torch.empty((n, 2, SIDE, SIDE), dtype=torch.float16, device=I1.device)
    _check(lib().psfm_cnn_stamp_inputs(_ptr(I1), _ptr(M1), _ptr(I2), _ptr(M2), W, H, W, _ptr(stamps),
                                       n, _ptr(x), None, _stream()), "psfm_cnn_stamp_inputs")
    return x


def to_ortho(ctx: psfm.Context, local: torch.Tensor) -> torch.Tensor:
    n = local.shape[0]
    c = torch.empty((n, OUT), dtype=torch.float32, device=local.device)
    _check(lib().psfm_cnn_targets(ctx.handle, _ptr(local), n, _ptr(c), _stream()), "psfm_cnn_targets")
    return c


def loss_weights(ctx: psfm.Context, fit: dict) -> torch.Tensor:
    n = fit["M"].shape[0]
    W = torch.empty((n, OUT, OUT), dtype=torch.float32, device=fit["M"].device)
    _check(lib().psfm_cnn_loss_weights(ctx.handle, _ptr(fit["M"]), _ptr(fit["npix"]), _ptr(fit["flags"]),
                                       n, _ptr(W), _stream()), "psfm_cnn_loss_weights")
    return W


def to_local(ctx: psfm.Context, ortho: torch.Tensor) -> torch.Tensor:
    n = ortho.shape[0]
    a = torch.empty((n, ctx.L), dtype=torch.float64, device=ortho.device)
    _check(lib().psfm_cnn_local_coeffs(ctx.handle, _ptr(ortho), n, _ptr(a), _stream()),
           "psfm_cnn_local_coeffs")
    return a


def make_dataset(n: int, seed: int, spec: synth.StampSetSpec = synth.STAMP_SETS["cells200k"],
                 chunk: int = 25_000, log: Optional[Callable[[str], None]] = None) -> dict:
    """Inputs, method-solved targets and loss weights for n single-star stamp
    pairs: the fit of each cell's stamp (psfm_fit_stamps), its own
    least-squares kernel (psfm_solve_stamps) in orthonormal-basis
    coefficients, and the stamp's loss weight (psfm_cnn_loss_weights), under
    which the loss is the chi2/dof excess of the predicted kernel.  Along the
    poorly constrained kernel directions the solved coefficients are mostly
    noise; the weight gives those directions the little importance the data
    gives them."""
    ctx = psfm.Context(psfm.Config(h=10, r=20, S=0, min_stamps=1))
    xs, ts, locs, chis, params, ws_ = [], [], [], [], [], []
    for k0 in range(0, n, chunk):
        m = min(chunk, n - k0)
        planes, stamps, par = synth.make_stamp_cells(spec, m, seed + k0)
        st = torch.from_numpy(stamps).to(planes["I1"].device)
        fit = ctx.fit_stamps(planes["I1"], planes["M1"], planes["I2"], planes["V2"], planes["M2"], st)
        local, chi2 = ctx.solve_stamps(fit)
        ws_.append(loss_weights(ctx, fit))
        xs.append(stamp_inputs(planes["I1"], planes["M1"], planes["I2"], planes["M2"], st))
        ts.append(to_ortho(ctx, local))
        locs.append(local)
        chis.append(chi2)
        params.append(par)
        del planes, fit
        if log:
            torch.cuda.synchronize()
            log(f"dataset: {k0 + m}/{n} stamps")
    ok = torch.cat(chis) >= 0
    return dict(x=torch.cat(xs)[ok], target=torch.cat(ts)[ok], local=torch.cat(locs)[ok],
                chi2=torch.cat(chis)[ok], weight=torch.cat(ws_)[ok],
                params={k: np.concatenate([p[k] for p in params])[ok.cpu().numpy()] for k in params[0]})


def standardize(data: dict, n_stats: Optional[int] = None) -> dict:
    """Training view of a dataset (psfm_cnn_standardize): targets
    z = (c - mu) / sd per component (mu, sd over the first ``n_stats`` rows,
    all by default), and the chi2/dof-excess weights carried into z
    coordinates, W_z = diag(sd) W diag(sd), each divided by its mean
    eigenvalue (trace / 49) so that every stamp counts alike while its well
    constrained kernel directions dominate its term."""
    T, W = data["target"].contiguous(), data["weight"].contiguous()
    n = T.shape[0]
    n_stats = n if n_stats is None else n_stats
    mu = torch.empty(OUT, dtype=torch.float32, device=T.device)
    sd = torch.empty_like(mu)
    z = torch.empty_like(T)
    Wz = torch.empty_like(W)
    _check(lib().psfm_cnn_standardize(_ptr(T), _ptr(W), n, n_stats, _ptr(mu), _ptr(sd), _ptr(z), _ptr(Wz),
                                      _stream()), "psfm_cnn_standardize")
    return dict(x=data["x"], target=z, weight=Wz, mu=mu, sd=sd)


def quad_excess(pred, target, weight) -> torch.Tensor:
    """psfm_cnn_excess: r^T W r per sample, r = pred - target; ``pred`` is
    n x 49 or one row of 49 shared by every sample."""
    target, weight, pred = target.contiguous(), weight.contiguous(), pred.contiguous()
    n = target.shape[0]
    exc = torch.empty(n, dtype=torch.float32, device=target.device)
    _check(lib().psfm_cnn_excess(_ptr(pred), 0 if pred.dim() == 1 else OUT, _ptr(target), _ptr(weight),
                                 n, _ptr(exc), _stream()), "psfm_cnn_excess")
    return exc


def evaluate_constant(c: torch.Tensor, target, weight) -> float:
    """The weighted loss of predicting the constant c for every sample."""
    exc = quad_excess(c.to(torch.float32), target, weight).cpu().numpy()
    return float(np.sum(exc, dtype=np.float64)) / target.numel()


def excess(net: Net, x, target, weight, batch: int = 1024) -> np.ndarray:
    """Per-stamp chi2/dof excess r^T W r of the network's predicted kernels
    (r the orthonormal-coefficient error, W the stamp's loss weight)."""
    out = [quad_excess(net.forward(x[s:s + batch]), target[s:s + batch], weight[s:s + batch])
           for s in range(0, x.shape[0], batch)]
    return torch.cat(out).cpu().numpy()


def train(net: Net, data: dict, epochs: int = 3, batch: int = 256, lr: float = 1e-3,
          val_frac: float = 0.05, seed: int = 0, log: Optional[Callable[[str], None]] = None) -> dict:
    """Adam on the (weighted) mean squared error of the targets in ``data``
    (x, target and, if present, weight); returns the per-epoch train and
    validation losses and the time spent."""
    n = data["x"].shape[0]
    n_val = max(1, int(n * val_frac))
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    perm = torch.randperm(n, generator=g).to(data["x"].device)
    val, tr = perm[:n_val], perm[n_val:]
    hist = dict(train=[], val=[], seconds=0.0, steps=0)
    loss_buf = torch.zeros(1, dtype=torch.float32, device=net.device)
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = tr[torch.randperm(tr.numel(), generator=g).to(tr.device)]
        tot, cnt = torch.zeros((), device=net.device), 0
        for s in range(0, order.numel() - batch + 1, batch):
            idx = order[s:s + batch]
            wt = data["weight"][idx] if "weight" in data else None
            net.loss_grad(data["x"][idx], data["target"][idx], loss_buf, wt)
            net.adam(lr)
            tot += loss_buf[0]
            cnt += 1
        hist["train"].append(float(tot) / max(cnt, 1))
        hist["val"].append(evaluate(net, data["x"][val], data["target"][val], batch,
                                    data["weight"][val] if "weight" in data else None))
        hist["steps"] += cnt
        if log:
            log(f"epoch {ep + 1}: train {hist['train'][-1]:.4e} val {hist['val'][-1]:.4e}")
    torch.cuda.synchronize()
    hist["seconds"] = time.perf_counter() - t0
    hist["val_index"] = val
    return hist


def evaluate(net: Net, x, target, batch: int = 1024, weight=None) -> float:
    """The training loss (weighted if ``weight`` is given) on held-out samples."""
    tot, cnt = 0.0, 0
    loss = torch.zeros(1, dtype=torch.float32, device=net.device)
    for s in range(0, x.shape[0], batch):
        xb, tb = x[s:s + batch], target[s:s + batch]
        net.loss_grad(xb, tb, loss, None if weight is None else weight[s:s + batch])
        tot += float(loss[0]) * tb.numel()
        cnt += tb.numel()
    return tot / max(cnt, 1)


def fit_prior(n: int = 200_000, seed: int = 4, epochs: int = 6, batch: int = 256, lr: float = 1e-3,
              n_val: int = 10_000, log: Optional[Callable[[str], None]] = None):
    """Dataset, training and evaluation of the learned prior.  Returns the
    network (outputs orthonormal-basis coefficients) and a report."""
    t0 = time.perf_counter()
    data = make_dataset(n, seed, log=log)
    t_data = time.perf_counter() - t0
    m = data["x"].shape[0]
    tr_rows, val_rows = slice(0, m - n_val), slice(m - n_val, m)
    view = standardize(data, m - n_val)
    net = Net(seed=seed)
    train_view = {k: view[k][tr_rows] for k in ("x", "target", "weight")}
    hist = train(net, train_view, epochs=epochs, batch=batch, lr=lr, val_frac=0.02, seed=seed, log=log)
    net.fold_output(view["mu"], view["sd"])
    xv, tv, wv = data["x"][val_rows], data["target"][val_rows], data["weight"][val_rows]
    exc = excess(net, xv, tv, wv)
    exc_mean = quad_excess(view["mu"], tv, wv).cpu().numpy()
    ctx = psfm.Context(psfm.Config(h=10, r=20, S=0, min_stamps=1))
    pred = to_local(ctx, net.forward(xv)).cpu().numpy()
    ks = np.abs(pred[:, 0] / data["local"][val_rows][:, 0].cpu().numpy() - 1)
    snr = data["params"]["snr"][m - n_val:]
    steps = hist["steps"]
    flops = 3.0 * 13.2e6 * steps * batch          # forward + backward ~ 3 forwards
    report = dict(n_train=m - n_val, n_val=n_val, epochs=epochs, batch=batch, lr=lr,
                  dataset_seconds=round(t_data, 2), train_seconds=round(hist["seconds"], 2),
                  train_samples_per_s=round(steps * batch / max(hist["seconds"], 1e-9), 1),
                  train_tflops=round(flops / max(hist["seconds"], 1e-9) / 1e12, 3),
                  loss_train=hist["train"], loss_val=hist["val"],
                  excess_median=float(np.median(exc)), excess_mean=float(np.mean(exc)),
                  excess_mean_of_mean_predictor=float(np.mean(exc_mean)),
                  within_1p05=float(np.mean(exc < 0.05)),
                  kernel_sum_err_median=float(np.median(ks)),
                  kernel_sum_err_median_snr150=float(np.median(ks[snr > 150])))
    return net, report


def predict_local(ctx: psfm.Context, net: Net, I1, M1, I2, M2, stamps) -> torch.Tensor:
    """Per-stamp predicted local kernel coefficients (n x L float64) for
    psfm_solve_prior."""
    if stamps.shape[0] == 0:
        return torch.zeros((0, ctx.L), dtype=torch.float64, device=I1.device)
    return to_local(ctx, net.forward(stamp_inputs(I1, M1, I2, M2, stamps)))
