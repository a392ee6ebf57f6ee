"""Reference of the per-level variant-selector network -- TEST INFRASTRUCTURE ONLY.

The network (not in the paper; its shape is the selector's contract):
12 features -> 64 -> 64 -> 4 logits, ReLU between layers.  Weights are kept as
fp32 master copies and used rounded to bfloat16 (round to nearest even); each
layer's input activations are rounded to bfloat16; products are accumulated in
fp32 starting from the bias, in ascending input index.  The loss is mean
softmax cross-entropy over the batch; training uses Adam.

Flat parameter layout (5,252 fp32 values):
  W1[64][12] @0, b1[64] @768, W2[64][64] @832, b2[64] @4928,
  W3[4][64] @4992, b3[4] @5248   (weights are [out][in], row-major)

Two accumulation modes:
  acc="fp32"  the arithmetic the network is specified with: a bf16*bf16
              product is exact in fp32, and the running sum is rounded to fp32
              after every addition, in ascending input order.
  acc="fp64"  the same expression evaluated in float64 (used to pin the fp32
              mode within its rounding bound and, with rounding switched off,
              to pin the backward pass by central finite differences).
The backward pass treats every bf16 rounding as the identity
(straight-through), evaluated at the rounded values the forward used.
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 12, 64, 4
OFF_W1, OFF_B1 = 0, 768
OFF_W2, OFF_B2 = 832, 4928
OFF_W3, OFF_B3 = 4992, 5248
NPARAM = 5252


def bf16_round(x) -> np.ndarray:
    """fp32 -> nearest bfloat16 (ties to even), returned as fp32 values.
    NaN stays NaN; overflow rounds to +-inf as the IEEE rule gives."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    nan = np.isnan(x)
    out = r.view(np.float32).copy()
    out[nan] = np.float32(np.nan)
    return out


def unpack(params):
    p = np.asarray(params)
    return (p[OFF_W1:OFF_B1].reshape(NH, NIN), p[OFF_B1:OFF_W2],
            p[OFF_W2:OFF_B2].reshape(NH, NH), p[OFF_B2:OFF_W3],
            p[OFF_W3:OFF_B3].reshape(NOUT, NH), p[OFF_B3:NPARAM])


def _layer(h, W, b, acc):
    """z[r, j] = b[j] + sum_k h[r, k] * W[j, k] in the given accumulation."""
    if acc == "fp64":
        return np.asarray(h, np.float64) @ np.asarray(W, np.float64).T + np.asarray(b, np.float64)
    h = np.asarray(h, np.float32)
    W = np.asarray(W, np.float32)
    z = np.broadcast_to(np.asarray(b, np.float32), (h.shape[0], W.shape[0])).copy()
    for k in range(W.shape[1]):
        prod = (h[:, k:k + 1].astype(np.float64) * W[None, :, k].astype(np.float64)).astype(np.float32)
        z = (z.astype(np.float64) + prod.astype(np.float64)).astype(np.float32)
    return z


def forward(params, x, acc: str = "fp32", rounding: bool = True):
    """Returns (logits, cache).  x: [B,12] normalised features."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    rnd = bf16_round if rounding else (lambda a: np.asarray(a, np.float64 if acc == "fp64" else np.float32))
    W1r, W2r, W3r = rnd(W1), rnd(W2), rnd(W3)
    h0 = rnd(x)
    z1 = _layer(h0, W1r, b1, acc)
    h1 = rnd(np.maximum(z1, 0))
    z2 = _layer(h1, W2r, b2, acc)
    h2 = rnd(np.maximum(z2, 0))
    logits = _layer(h2, W3r, b3, acc)
    cache = dict(h0=h0, z1=z1, h1=h1, z2=z2, h2=h2, W1r=W1r, W2r=W2r, W3r=W3r)
    return logits, cache


def softmax(logits):
    l = np.asarray(logits, np.float64)
    e = np.exp(l - l.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def loss(logits, labels) -> float:
    p = softmax(logits)
    B = p.shape[0]
    return float(-np.log(p[np.arange(B), np.asarray(labels)]).mean())


def backward(params, x, labels, acc: str = "fp64", rounding: bool = True):
    """Gradient of the mean cross-entropy w.r.t. the flat parameters (fp64)."""
    logits, c = forward(params, x, acc=acc, rounding=rounding)
    B = logits.shape[0]
    p = softmax(logits)
    g = p.copy()
    g[np.arange(B), np.asarray(labels)] -= 1.0
    g /= B
    f = lambda a: np.asarray(a, np.float64)
    dW3 = g.T @ f(c["h2"])
    db3 = g.sum(0)
    dh2 = g @ f(c["W3r"])
    dz2 = dh2 * (f(c["z2"]) > 0)
    dW2 = dz2.T @ f(c["h1"])
    db2 = dz2.sum(0)
    dh1 = dz2 @ f(c["W2r"])
    dz1 = dh1 * (f(c["z1"]) > 0)
    dW1 = dz1.T @ f(c["h0"])
    db1 = dz1.sum(0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])


def adam(params, grad, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015, with bias correction) in fp64.
    Returns new (params, m, v)."""
    params = np.asarray(params, np.float64)
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def predict(params, x, acc: str = "fp32"):
    """Argmax class per row (ties to the lowest index) and the max softmax."""
    logits, _ = forward(params, x, acc=acc)
    p = softmax(logits)
    return np.argmax(logits, axis=1), p.max(axis=1)


def init_params(seed: int) -> np.ndarray:
    """He-style uniform initialisation, deterministic in ``seed``."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM, dtype=np.float32)
    for off, fan_in, nout in ((OFF_W1, NIN, NH), (OFF_W2, NH, NH), (OFF_W3, NH, NOUT)):
        lim = np.sqrt(6.0 / fan_in)
        p[off:off + nout * fan_in] = rng.uniform(-lim, lim, nout * fan_in).astype(np.float32)
    return p
