"""FP64 NumPy oracle of the stamp-pair CNN (test infrastructure only).

Only tests/, the smoke entry point and the benchmark's CPU baseline use this
module; the product path never imports it.

The network predicts a kernel's basis coefficients from a 2-channel stamp
pair (the reference stamp and the target stamp, 41 x 41 each):

    conv1  3x3, 2 -> 32 channels, stride 1, zero padding 1, ReLU   41 -> 41
    conv2  3x3, 32 -> 32, stride 2, padding 1, ReLU                41 -> 21
    conv3  3x3, 32 -> 32, stride 2, padding 1, ReLU                21 -> 11
    conv4  3x3, 32 -> 32, stride 2, padding 1, ReLU                11 -> 6
    fc1    1152 -> 128, ReLU          (flattened channel-major: c, y, x)
    fc2    128 -> 49                  (no activation)

Loss: mean over the batch and the 49 outputs of (out - target)^2, or with a
per-sample symmetric weight W_b (49 x 49): sum_b r_b^T W_b r_b / (B * 49),
r_b = out_b - target_b (the plain loss is W_b = identity).

A convolution here is the cross-correlation used by neural networks:
    y[b, o, i, j] = bias[o] + sum_{c, u, v} w[o, c, u, v] x[b, c, s i + u - 1, s j + v - 1]
with out-of-range inputs read as zero.  The backward pass is the chain rule
applied to these definitions, written as explicit sums (no library
autograd), so a reader can check each gradient against the formula above.

Parameter vector layout (shared with the C interface, which documents the
same order): for each of conv1..conv4, fc1, fc2 the weight (row-major in the
index order used above) followed by the bias.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

IN_SIDE = 41
IN_CH = 2
CH = 32
HIDDEN = 128
OUT = 49
STRIDES = (1, 2, 2, 2)


def conv_out(n: int, s: int) -> int:
    return (n + 2 - 3) // s + 1


SIDES = [IN_SIDE]
for _s in STRIDES:
    SIDES.append(conv_out(SIDES[-1], _s))
FLAT = CH * SIDES[-1] * SIDES[-1]          # 32 * 6 * 6 = 1152


def layer_shapes() -> List[Tuple[str, Tuple[int, ...]]]:
    shapes = []
    cin = IN_CH
    for k in range(4):
        shapes.append((f"conv{k + 1}.w", (CH, cin, 3, 3)))
        shapes.append((f"conv{k + 1}.b", (CH,)))
        cin = CH
    shapes += [("fc1.w", (HIDDEN, FLAT)), ("fc1.b", (HIDDEN,)),
               ("fc2.w", (OUT, HIDDEN)), ("fc2.b", (OUT,))]
    return shapes


def n_params() -> int:
    return int(sum(np.prod(s) for _, s in layer_shapes()))


def unpack(theta: np.ndarray) -> Dict[str, np.ndarray]:
    out, o = {}, 0
    for name, shp in layer_shapes():
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    return out


def pack(parts: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([parts[name].reshape(-1) for name, _ in layer_shapes()])


def init_params(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    parts = {}
    for name, shp in layer_shapes():
        if name.endswith(".b"):
            parts[name] = np.zeros(shp)
        else:
            fan_in = int(np.prod(shp[1:]))
            parts[name] = rng.standard_normal(shp) * np.sqrt(2.0 / fan_in)
    return pack(parts)


def _pad(x):
    return np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))


def conv_forward(x, w, b, s):
    """y[b,o,i,j] = bias[o] + sum_{c,u,v} w[o,c,u,v] x[b,c,s i+u-1, s j+v-1]."""
    B, C, H, _ = x.shape
    Ho = conv_out(H, s)
    xp = _pad(x)
    y = np.zeros((B, w.shape[0], Ho, Ho))
    for u in range(3):
        for v in range(3):
            patch = xp[:, :, u:u + s * (Ho - 1) + 1:s, v:v + s * (Ho - 1) + 1:s]   # [B,C,Ho,Ho]
            y += np.einsum("oc,bcij->boij", w[:, :, u, v], patch)
    return y + b[None, :, None, None]


def conv_backward(x, w, s, dy):
    """Gradients of sum(dy * y) for y = conv_forward(x, w, b, s):
       dw[o,c,u,v] = sum_{b,i,j} dy[b,o,i,j] x[b,c,s i+u-1, s j+v-1]
       db[o]       = sum_{b,i,j} dy[b,o,i,j]
       dx[b,c,p,q] = sum over (o,u,v,i,j) with s i+u-1 = p, s j+v-1 = q of w[o,c,u,v] dy[b,o,i,j]."""
    B, C, H, _ = x.shape
    Ho = dy.shape[2]
    xp = _pad(x)
    dw = np.zeros_like(w)
    dxp = np.zeros_like(xp)
    for u in range(3):
        for v in range(3):
            sl = (slice(None), slice(None), slice(u, u + s * (Ho - 1) + 1, s),
                  slice(v, v + s * (Ho - 1) + 1, s))
            dw[:, :, u, v] = np.einsum("boij,bcij->oc", dy, xp[sl])
            dxp[sl] += np.einsum("oc,boij->bcij", w[:, :, u, v], dy)
    db = dy.sum(axis=(0, 2, 3))
    return dw, db, dxp[:, :, 1:H + 1, 1:H + 1]


def forward(theta: np.ndarray, x: np.ndarray, keep: bool = False):
    """x: [B, 2, 41, 41].  Returns out [B, 49] (and the activations)."""
    p = unpack(theta)
    acts = [x]
    h = x
    for k, s in enumerate(STRIDES):
        h = np.maximum(conv_forward(h, p[f"conv{k + 1}.w"], p[f"conv{k + 1}.b"], s), 0.0)
        acts.append(h)
    f = h.reshape(h.shape[0], -1)
    z = np.maximum(f @ p["fc1.w"].T + p["fc1.b"], 0.0)
    out = z @ p["fc2.w"].T + p["fc2.b"]
    if keep:
        return out, dict(acts=acts, flat=f, hidden=z)
    return out


def loss_and_grad(theta: np.ndarray, x: np.ndarray, target: np.ndarray, weight=None):
    """(Weighted) mean squared error over batch and outputs, and its gradient
    in theta.  weight: [B, 49, 49] symmetric, or None for the identity."""
    p = unpack(theta)
    out, a = forward(theta, x, keep=True)
    B = x.shape[0]
    r = out - target
    if weight is None:
        loss = float(np.mean(r * r))
        dout = 2.0 * r / r.size
    else:
        u = np.einsum("bij,bj->bi", weight, r)
        loss = float(np.sum(r * u) / r.size)
        dout = 2.0 * u / r.size
    g = {}
    g["fc2.w"] = dout.T @ a["hidden"]
    g["fc2.b"] = dout.sum(0)
    dz = (dout @ p["fc2.w"]) * (a["hidden"] > 0)
    g["fc1.w"] = dz.T @ a["flat"]
    g["fc1.b"] = dz.sum(0)
    dh = (dz @ p["fc1.w"]).reshape(a["acts"][-1].shape) * (a["acts"][-1] > 0)
    for k in range(3, -1, -1):
        dw, db, dx = conv_backward(a["acts"][k], p[f"conv{k + 1}.w"], STRIDES[k], dh)
        g[f"conv{k + 1}.w"] = dw
        g[f"conv{k + 1}.b"] = db
        if k > 0:
            dh = dx * (a["acts"][k] > 0)
    return loss, pack(g)


def adam_step(theta, m, v, grad, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba): bias-corrected first and second moments."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
