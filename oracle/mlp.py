"""FP64 reference of the learned corrector's network (TEST INFRASTRUCTURE).

A 12 -> 64 -> 64 -> 5 multilayer perceptron with tanh hidden layers and a
linear output, trained with mean squared error on normalised targets and Adam.
Plain numpy in float64: forward, backward by the chain rule, and one Adam
update, written out so that a reader can check each line. Used only to check
the GPU's BF16-MFMA kernels (same weights, same inputs).

Weight layout (shared with the GPU through the flat vector returned by
`flatten`): W1 (12 x 64), b1 (64), W2 (64 x 64), b2 (64), W3 (64 x 5), b3 (5);
a layer computes h_out = act(h_in @ W + b) with W stored row-major
(input index major).
"""
from __future__ import annotations

import numpy as np

SIZES = [(12, 64), (64, 64), (64, 5)]


def n_params() -> int:
    return sum(i * o + o for i, o in SIZES)


def init(seed: int = 0):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for i, o in SIZES:
        lim = 1.0 / np.sqrt(i)
        params.append(rng.uniform(-lim, lim, size=(i, o)))
        params.append(np.zeros(o))
    return params


def flatten(params) -> np.ndarray:
    return np.concatenate([p.ravel() for p in params])


def unflatten(v: np.ndarray):
    out, k = [], 0
    for i, o in SIZES:
        out.append(v[k:k + i * o].reshape(i, o)); k += i * o
        out.append(v[k:k + o].copy()); k += o
    return out


def forward(params, X):
    W1, b1, W2, b2, W3, b3 = params
    a1 = X @ W1 + b1
    h1 = np.tanh(a1)
    a2 = h1 @ W2 + b2
    h2 = np.tanh(a2)
    y = h2 @ W3 + b3
    return y, (X, h1, h2)


def loss(params, X, Y):
    """Mean over samples of the squared error summed over the 5 outputs, / 2."""
    y, _ = forward(params, X)
    d = y - Y
    return 0.5 * np.sum(d * d) / X.shape[0]


def grad(params, X, Y):
    """Gradient of `loss` with respect to every parameter (chain rule)."""
    W1, b1, W2, b2, W3, b3 = params
    y, (X_, h1, h2) = forward(params, X)
    n = X.shape[0]
    dy = (y - Y) / n                      # dL/dy
    gW3 = h2.T @ dy
    gb3 = dy.sum(axis=0)
    dh2 = dy @ W3.T
    da2 = dh2 * (1.0 - h2 * h2)           # tanh'
    gW2 = h1.T @ da2
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2.T
    da1 = dh1 * (1.0 - h1 * h1)
    gW1 = X_.T @ da1
    gb1 = da1.sum(axis=0)
    return [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba): returns new params, m, v."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1 - b1) * g
        vv = b2 * vv + (1 - b2) * g * g
        mh = mm / (1 - b1 ** t)
        vh = vv / (1 - b2 ** t)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v


def to_bf16(a: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (ties to even), as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
