"""FP64 reference of the control-proposal network (test infrastructure only).

A 4 -> 128 -> 128 -> 3 perceptron with exact (erf) GELU activations maps a
node state, scaled to [-1, 1] per axis, to (cos u, sin u, throttle logit).
The loss of a sample with target (cos u*, sin u*, thr*) is
    thr* * ((c - cos u*)^2 + (s - sin u*)^2) + BCE(logit, thr*)
averaged over the batch; training uses Adam.  Forward and backward are
written out by hand so finite differences can pin them.

bf16=True rounds the operands of the two products of the 128 x 128 layer
(forward: h1 and W2; backward: delta2, h1 and W2) to bfloat16 with
round-to-nearest-even, as the device's matrix-core products do; everything
else stays in FP64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

HIDDEN = 128
SHAPES = [("W1", (HIDDEN, 4)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
          ("W3", (3, HIDDEN)), ("b3", (3,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(theta):
    out, o = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + size], dtype=np.float64).reshape(shape)
        o += size
    return out


def flatten(params):
    return np.concatenate([np.asarray(params[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def from_init(init):
    """Flat parameters from inputs.mlp_init's [(W, b), ...] list."""
    (W1, b1), (W2, b2), (W3, b3) = init
    return flatten(dict(W1=W1, b1=b1, W2=W2, b2=b2, W3=W3, b3=b3))


def bf16(a):
    """Round float values to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, x, bf16_ops=False):
    p = unflatten(theta)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = gelu(z1)
    if bf16_ops:
        z2 = bf16(h1) @ bf16(p["W2"]).T + p["b2"]
    else:
        z2 = h1 @ p["W2"].T + p["b2"]
    h2 = gelu(z2)
    y = h2 @ p["W3"].T + p["b3"]
    return y, dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2)


def bce(logit, t):
    return np.maximum(logit, 0.0) - logit * t + np.log1p(np.exp(-np.abs(logit)))


def loss(y, target):
    c, s, lg = y[:, 0], y[:, 1], y[:, 2]
    tc, ts, tt = target[:, 0], target[:, 1], target[:, 2]
    per = tt * ((c - tc) ** 2 + (s - ts) ** 2) + bce(lg, tt)
    return float(per.mean())


def loss_grad(theta, x, target, bf16_ops=False):
    """Mean loss and its gradient with respect to the flat parameters."""
    p = unflatten(theta)
    target = np.asarray(target, dtype=np.float64)
    y, c = forward(theta, x, bf16_ops)
    B = y.shape[0]
    L = loss(y, target)
    tt = target[:, 2]
    dy = np.empty_like(y)
    dy[:, 0] = 2.0 * tt * (y[:, 0] - target[:, 0]) / B
    dy[:, 1] = 2.0 * tt * (y[:, 1] - target[:, 1]) / B
    dy[:, 2] = (1.0 / (1.0 + np.exp(-y[:, 2])) - tt) / B
    g = {}
    g["W3"] = dy.T @ c["h2"]
    g["b3"] = dy.sum(axis=0)
    d2 = (dy @ p["W3"]) * gelu_grad(c["z2"])
    if bf16_ops:
        g["W2"] = bf16(d2).T @ bf16(c["h1"])
        dh1 = bf16(d2) @ bf16(p["W2"])
    else:
        g["W2"] = d2.T @ c["h1"]
        dh1 = d2 @ p["W2"]
    g["b2"] = d2.sum(axis=0)
    d1 = dh1 * gelu_grad(c["z1"])
    g["W1"] = d1.T @ c["x"]
    g["b1"] = d1.sum(axis=0)
    return L, flatten(g)


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step t >= 1), returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def normalise(states, lo, hi):
    """Scale states (n x 4) to [-1, 1] per axis of the box [lo, hi]."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return 2.0 * (np.asarray(states, dtype=np.float64) - lo) / (hi - lo) - 1.0
