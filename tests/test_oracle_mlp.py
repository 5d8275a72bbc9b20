"""Pins of the FP64 reference network: backpropagation against central finite
differences, the Adam update against its closed form on a quadratic, and the
bfloat16 rounding against its definition."""
import numpy as np
import pytest

from oracle import mlp


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    params = mlp.init(3)
    params = [p + 0.1 * rng.normal(size=p.shape) for p in params]   # non-zero biases
    X = rng.normal(size=(37, 12))
    Y = rng.normal(size=(37, 5))
    g = mlp.flatten(mlp.grad(params, X, Y))
    v = mlp.flatten(params)
    idx = rng.choice(v.size, 60, replace=False)
    for i in idx:
        e = 1e-6
        vp, vm = v.copy(), v.copy()
        vp[i] += e; vm[i] -= e
        fd = (mlp.loss(mlp.unflatten(vp), X, Y) - mlp.loss(mlp.unflatten(vm), X, Y)) / (2 * e)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_loss_decreases_with_adam():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(256, 12))
    Wt = rng.normal(size=(12, 5)) * 0.3
    Y = np.tanh(X @ Wt)
    params = mlp.init(0)
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    l0 = mlp.loss(params, X, Y)
    for t in range(1, 201):
        params, m, v = mlp.adam_step(params, mlp.grad(params, X, Y), m, v, t, 3e-3)
    assert mlp.loss(params, X, Y) < 0.2 * l0


def test_adam_first_step_closed_form():
    # the first Adam step moves every parameter by lr * sign(g) (bias-corrected m/sqrt(v) = g/|g|)
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -1e-3, 2.0])]
    out, _, _ = mlp.adam_step(p, g, [np.zeros(3)], [np.zeros(3)], 1, 0.01, eps=0.0)
    assert np.allclose(out[0], p[0] - 0.01 * np.sign(g[0]), rtol=1e-12)


def test_bf16_rounding():
    # bfloat16 keeps 8 significand bits: 1 + 2^-8 rounds to even (1.0), 1 + 3*2^-8 to 1 + 2^-6
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.14159265])
    r = mlp.to_bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -6 and r[3] == -2.5
    assert abs(r[4] - 3.14159265) <= 2 ** -7 * 2
    assert np.all(mlp.to_bf16(r) == r)
