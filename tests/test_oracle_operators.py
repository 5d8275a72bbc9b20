"""Pins of the corrected SPH operators in the oracle.

* First-order consistency of the corrected gradient (Eqs. sph1stDerivative and
  sphCorrectionMatrix): a linear field is differentiated exactly on any
  particle configuration.
* The corrected Laplacian on the periodic lattice is a convolution, so plane
  waves are its eigenfunctions; the eigenvalue tends to -|k|^2 as the wave is
  resolved by more particles (continuum limit).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_exact_for_linear_field(seed):
    L = 24
    p = wl.Params(L=float(L))
    x, y = wl.jittered_lattice(L, 1.0, 0.35, seed=seed)
    g = np.array([0.37, -1.21])
    f = g[0] * x + g[1] * y
    _, _, grad, _ = oracle.operators(p, x, y, f)
    R = 3 * p.h
    inner = (x > R + 0.5) & (x < L - R - 0.5) & (y > R + 0.5) & (y < L - R - 0.5)
    assert inner.sum() > 50
    err = np.abs(grad[inner] - g[None, :]).max()
    assert err < 1e-12


def test_laplacian_quadratic_interior():
    # f = (x^2 + y^2)/2 has Laplacian 2; on a lattice interior the discrete
    # operator is exact for quadratics up to the kernel's second-moment error.
    L = 32
    p = wl.Params(L=float(L))
    x, y = wl.lattice(L)
    f = 0.5 * ((x - 16) ** 2 + (y - 16) ** 2)
    _, _, _, lap = oracle.operators(p, x, y, f)
    R = 3 * p.h
    inner = (x > R + 1) & (x < L - R - 1) & (y > R + 1) & (y < L - R - 1)
    assert np.all(np.abs(lap[inner] - 2.0) < 5e-3)


@pytest.mark.parametrize("L,m,ratio_min", [(64, 1, 0.997), (64, 4, 0.96), (256, 1, 0.9998), (512, 1, 0.99996)])
def test_laplacian_plane_wave_eigen(L, m, ratio_min):
    p = wl.Params(L=float(L))
    x, y = wl.lattice(L)
    k = 2 * math.pi * m / L
    f = np.cos(k * x)
    _, _, _, lap = oracle.operators(p, x, y, f)
    lam = np.dot(lap, f) / np.dot(f, f)
    assert np.abs(lap - lam * f).max() < 1e-9 * np.abs(lap).max()   # eigenfunction
    ratio = lam / (-k * k)
    assert ratio_min < ratio <= 1.0 + 1e-9
    if (L, m) == (64, 1):
        # lattice symbol -0.0096193344248 against the exact -(2pi/64)^2
        assert lam == pytest.approx(-0.0096193344248, rel=1e-9)


def test_gradient_plane_wave_on_lattice():
    L = 64
    p = wl.Params(L=float(L))
    x, y = wl.lattice(L)
    k = 2 * math.pi / L
    f = np.sin(k * y)
    _, _, grad, _ = oracle.operators(p, x, y, f)
    assert np.abs(grad[:, 0]).max() < 1e-14
    exact = k * np.cos(k * y)
    assert np.abs(grad[:, 1] - exact).max() < 1e-2 * k   # O((k h)^2) truncation
