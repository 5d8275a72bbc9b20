"""Pins of the Wendland C2 kernel variant in the oracle (support 2h).

Sources of truth: the continuum normalisation int W d^2r = 1, the closed form
W(0) = 7/(4 pi h^2), C2 smoothness at the support edge and at r = 0 (finite
differences), the 20 lattice sites inside 2h = 2.6 dx, an independent numpy
neighbour search, first-order consistency of the corrected gradient, the
lattice Laplacian's plane-wave symbol tending to -k^2, momentum conservation of
the conservative form and the closed-form relaxation of a uniform nematic."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads as wl
from test_oracle_neighbors import numpy_brute, rows

WC2 = 1


@pytest.mark.parametrize("h", [1.3, 4.0 / 3.0, 0.7])
def test_normalised(h):
    tot = integrate.quad(lambda r: oracle.W(h, r, WC2) * 2 * math.pi * r, 0, 2 * h, epsabs=1e-14, epsrel=1e-13)[0]
    assert abs(tot - 1.0) < 1e-12


@pytest.mark.parametrize("h", [1.3, 0.7])
def test_values_and_smoothness(h):
    assert oracle.kappa(WC2) == 2.0 and oracle.kappa(0) == 3.0
    assert oracle.W(h, 0.0, WC2) == pytest.approx(7.0 / (4.0 * math.pi * h * h), rel=1e-15)
    assert oracle.W(h, 2 * h, WC2) == 0.0 and oracle.W(h, 2.2 * h, WC2) == 0.0
    assert oracle.dWdr(h, 2 * h, WC2) == 0.0
    for r in [0.01 * h, 0.4 * h, h, 1.5 * h, 1.99 * h]:
        e = 1e-6 * h
        fd = (oracle.W(h, r + e, WC2) - oracle.W(h, r - e, WC2)) / (2 * e)
        assert oracle.dWdr(h, r, WC2) == pytest.approx(fd, rel=1e-7, abs=1e-12)
    # C2 at both ends: the slope vanishes at r = 0 and at 2h, and so does the
    # curvature at 2h (dW/dr ~ (2h - r)^3)
    assert abs(oracle.dWdr(h, 1e-7 * h, WC2)) < 1e-6 * oracle.W(h, 0.0, WC2) / h
    e = 1e-3 * h
    curv_edge = (oracle.dWdr(h, 2 * h - e, WC2) - oracle.dWdr(h, 2 * h - 2 * e, WC2)) / e
    assert abs(curv_edge) < 1e-4 * oracle.W(h, 0.0, WC2) / h ** 2


@pytest.mark.parametrize("hdx", [1.3, 4.0 / 3.0])
def test_twenty_lattice_neighbours(hdx):
    p = wl.Params(L=16.0, h=hdx, kernel=WC2)
    x, y = wl.lattice(16)
    rp, _ = oracle.neighbors(p, x, y, 0)
    assert np.all(np.diff(rp) == 20)


@pytest.mark.parametrize("kind,L", [("lattice", 8), ("jitter", 12), ("uniform", 10)])
def test_neighbours_match_numpy(kind, L):
    p = wl.Params(L=float(L), kernel=WC2)
    if kind == "lattice":
        x, y = wl.lattice(L)
    elif kind == "jitter":
        x, y = wl.jittered_lattice(L, 1.0, 0.3, seed=L)
    else:
        x, y = wl.uniform_positions(L * L, float(L), seed=L)
    ref, _ = numpy_brute(x, y, float(L), 2 * p.h)
    for mode in (0, 1):
        rp, col = oracle.neighbors(p, x, y, mode)
        assert rows(rp, col) == ref


def test_lattice_volume_and_correction():
    """Lattice sums of a normalised radial kernel tend to the continuum
    moments (sum W -> 1, alpha -> I) as h/dx grows; the cubic symmetry of
    the lattice keeps alpha isotropic. At h = 1.3 dx the 20-site Wendland
    stencil is 1% and 4% off."""
    dev = []
    for h in (1.3, 1.6, 2.0, 3.0):
        p = wl.Params(L=24.0, h=h, kernel=WC2)
        x, y = wl.lattice(24)
        V, B, _, _ = oracle.operators(p, x, y)
        assert np.ptp(V) < 1e-14
        alpha = np.linalg.inv(B[0])
        assert abs(alpha[0, 1]) < 1e-15 and alpha[0, 0] == pytest.approx(alpha[1, 1], rel=1e-14)
        dev.append((abs(1.0 / V[0] - 1.0), abs(alpha[0, 0] - 1.0)))
    assert dev[0][0] < 2e-2 and dev[0][1] < 5e-2
    assert all(a[0] > b[0] and a[1] > b[1] for a, b in zip(dev, dev[1:]))
    assert dev[-1][0] < 3e-4 and dev[-1][1] < 5e-4


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_exact_for_linear_field(seed):
    L = 24
    p = wl.Params(L=float(L), kernel=WC2)
    x, y = wl.jittered_lattice(L, 1.0, 0.35, seed=seed)
    g = np.array([0.37, -1.21])
    _, _, grad, _ = oracle.operators(p, x, y, g[0] * x + g[1] * y)
    R = 2 * p.h
    inner = (x > R + 0.5) & (x < L - R - 0.5) & (y > R + 0.5) & (y < L - R - 0.5)
    assert inner.sum() > 100
    assert np.abs(grad[inner] - g[None, :]).max() < 1e-12


def test_laplacian_plane_wave_symbol_converges():
    ratios = []
    for L in (64, 256):
        p = wl.Params(L=float(L), kernel=WC2)
        x, y = wl.lattice(L)
        k = 2 * math.pi / L
        f = np.cos(k * x)
        _, _, _, lap = oracle.operators(p, x, y, f)
        lam = np.dot(lap, f) / np.dot(f, f)
        assert np.abs(lap - lam * f).max() < 1e-9 * np.abs(lap).max()
        ratios.append(lam / (-k * k))
    assert 0.99 < ratios[0] <= 1.0 + 1e-9 and ratios[0] < ratios[1] <= 1.0 + 1e-9
    assert (1 - ratios[0]) / (1 - ratios[1]) == pytest.approx(16.0, rel=0.05)   # second order in k h


def test_momentum_conserved_conservative_form():
    L = 16
    p = wl.Params(L=float(L), form=1, zeta=0.05, kernel=WC2)
    x, y = wl.jittered_lattice(L, 1.0, 0.2, seed=4)
    rng = np.random.default_rng(4)
    th = rng.uniform(0, math.pi, x.size)
    n = x.size
    st = oracle.State(dict(x=x, y=y, ux=1e-3 * rng.normal(size=n), uy=1e-3 * rng.normal(size=n),
                           qxx=np.cos(2 * th), qxy=np.sin(2 * th), rho=1 + 1e-4 * rng.normal(size=n),
                           ax=np.zeros(n), ay=np.zeros(n)))
    d0 = oracle.diagnostics(p, st)
    oracle.step(p, st, 5)
    d1 = oracle.diagnostics(p, st)
    assert abs(d1["px"] - d0["px"]) < 1e-13 and abs(d1["py"] - d0["py"]) < 1e-13


def test_uniform_nematic_relaxes_by_the_closed_form():
    """A uniform aligned nematic at rest: no gradients, so q follows
    dq/dt = -2 Gamma C q^3 whatever the kernel (exact Euler recurrence)."""
    L = 16
    p = wl.Params(L=float(L), A=0.0, C=0.5, zeta=0.02, kernel=WC2)
    x, y = wl.lattice(L)
    n = x.size
    st = oracle.State(dict(x=x, y=y, ux=np.zeros(n), uy=np.zeros(n), qxx=np.ones(n), qxy=np.zeros(n),
                           rho=np.ones(n), ax=np.zeros(n), ay=np.zeros(n)))
    q = 1.0
    for _ in range(20):
        oracle.step(p, st, 1)
        q = q - p.dt * 2 * p.Gamma * p.C * q ** 3
    f = st.fields()
    assert np.abs(f["qxx"] - q).max() < 1e-14 and np.abs(f["ux"]).max() == 0.0
