"""Pins of the grid diagnostics (spectrum, defect counter) on analytic fields."""
import math

import numpy as np
import pytest

import oracle
from oracle import diag
import workloads as wl


def test_spectrum_single_mode_and_parseval():
    M = 64
    j, i = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    y = (j + 0.5) * (64.0 / M)
    for m in (1, 3, 7):
        ux = 0.2 * np.sin(2 * math.pi * m * y / 64.0)
        uy = np.zeros_like(ux)
        E = diag.spectrum_from_grid(ux, uy)
        assert E.sum() == pytest.approx(0.5 * np.mean(ux ** 2 + uy ** 2), rel=1e-12)
        assert E[m] == pytest.approx(E.sum(), rel=1e-12)


def test_spectrum_slope_recovered():
    M = 256
    rng = np.random.default_rng(0)
    k = np.fft.fftfreq(M) * M
    KX, KY = np.meshgrid(k, k, indexing="xy")
    kk = np.sqrt(KX ** 2 + KY ** 2)
    kk[0, 0] = 1.0
    # |u_hat|^2 ~ k^{-s-1} so that the shell sum scales as k^{-s}
    s = 4.0
    amp = kk ** (-(s + 1) / 2)
    amp[0, 0] = 0
    ph = np.exp(2j * math.pi * rng.uniform(size=(M, M)))
    u = np.real(np.fft.ifft2(amp * ph))
    v = np.real(np.fft.ifft2(amp * np.exp(2j * math.pi * rng.uniform(size=(M, M)))))
    E = diag.spectrum_from_grid(u, v)
    assert diag.slope(E, 8, 64) == pytest.approx(-s, abs=0.15)


def defect_field(M, centers):
    j, i = np.meshgrid(np.arange(M) + 0.5, np.arange(M) + 0.5, indexing="ij")
    th = np.zeros((M, M))
    for (cx, cy, q) in centers:
        th += q * np.arctan2(j - cy, i - cx)
    return np.cos(2 * th), np.sin(2 * th)


@pytest.mark.parametrize("centers,plus,minus", [
    ([(20.3, 30.7, 0.5)], 1, 0),
    ([(20.3, 30.7, -0.5)], 0, 1),
    ([(20.3, 30.7, 0.5), (40.1, 25.2, -0.5)], 1, 1),
    ([(12.2, 12.9, 0.5), (50.6, 12.1, 0.5), (30.4, 45.3, -0.5), (30.9, 20.6, -0.5)], 2, 2),
])
def test_defects_analytic(centers, plus, minus):
    # defects well inside the box; the winding field of a +-1/2 sum is smooth elsewhere
    qxx, qxy = defect_field(64, centers)
    p, m, w = diag.defects_from_grid(qxx, qxy)
    interior = np.zeros((64, 64), bool)
    interior[4:60, 4:60] = True
    pp = int(np.count_nonzero((w > math.pi / 2) & interior))
    mm = int(np.count_nonzero((w < -math.pi / 2) & interior))
    assert (pp, mm) == (plus, minus)
    # each defect sits in the plaquette that contains its centre
    for (cx, cy, q) in centers:
        ci, cj = int(np.floor(cx - 0.5)), int(np.floor(cy - 0.5))
        assert abs(w[cj, ci] - math.copysign(math.pi, q)) < 1e-9


def test_defects_through_deposit():
    # particles on the lattice carry the analytic director field; after the
    # Shepard deposit the counter still finds the single +1/2 / -1/2 pair
    L = 64
    p = wl.Params(L=float(L))
    x, y = wl.lattice(L)
    th = 0.5 * np.arctan2(y - 30.2, x - 20.7) - 0.5 * np.arctan2(y - 33.9, x - 44.3)
    pl, mi = diag.defects(p, x, y, np.cos(2 * th), np.sin(2 * th), 64)
    assert (pl, mi) == (1, 1)


def test_deposit_reproduces_constant_and_linear():
    L = 32
    p = wl.Params(L=float(L))
    x, y = wl.jittered_lattice(L, 1.0, 0.3, 3)
    g = oracle.deposit(p, x, y, [np.full(x.size, 2.5)], 32)
    assert np.abs(g - 2.5).max() < 1e-14


def _grid(M, L):
    j, i = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    return (i + 0.5) * (L / M), (j + 0.5) * (L / M)   # x varies along columns, y along rows


@pytest.mark.parametrize("m", [1, 2, 5])
def test_vorticity_correlation_single_mode(m):
    """uy = U sin(k x): omega = U k cos(k x), whose normalised autocorrelation is
    cos(k r) along x (zero at L/4m) and 1 along y."""
    M, L, U = 64, 64.0, 0.3
    x, y = _grid(M, L)
    k = 2 * math.pi * m / L
    ux, uy = np.zeros((M, M)), U * np.sin(k * x)
    w = diag.vorticity_from_grid(ux, uy, L)
    assert np.abs(w - U * k * np.cos(k * x)).max() < 1e-12 * U * k
    cx, cy, lx, ly = diag.vorticity_correlation_from_grid(ux, uy, L)
    n = np.arange(M // 2 + 1)
    assert np.abs(cx - np.cos(2 * math.pi * m * n / M)).max() < 1e-12
    assert np.abs(cy - 1.0).max() < 1e-12
    # zero of cos between grid shifts n0 and n0+1, linearly interpolated
    c = np.cos(2 * math.pi * m * n / M)
    n0 = int(np.argmax(c <= 0)) - 1
    lx_lin = (n0 + c[n0] / (c[n0] - c[n0 + 1])) * (L / M)
    assert lx == pytest.approx(lx_lin, rel=1e-9)
    if (M % (4 * m)) == 0:
        assert lx == pytest.approx(L / (4 * m), rel=1e-9)
    assert ly == -1.0
    A = diag.autocorrelation(w)
    assert A[0, 0] == pytest.approx(0.5 * (U * k) ** 2, rel=1e-12)


def test_vorticity_of_two_dimensional_field():
    """A field varying in both directions against its analytic curl."""
    M, L = 32, 32.0
    x, y = _grid(M, L)
    a, b = 2 * math.pi / L, 2 * math.pi * 3 / L
    ux = np.sin(b * y) * np.cos(a * x)
    uy = 0.5 * np.cos(2 * a * x) * np.sin(a * y)
    w_exact = -a * np.sin(2 * a * x) * np.sin(a * y) * 1.0 - b * np.cos(b * y) * np.cos(a * x)
    assert np.abs(diag.vorticity_from_grid(ux, uy, L) - w_exact).max() < 1e-12


def test_autocorrelation_equals_direct_sum():
    """Wiener-Khinchin route against the direct periodic sum over all shifts."""
    rng = np.random.default_rng(5)
    M = 12
    f = rng.normal(size=(M, M))
    A = diag.autocorrelation(f)
    D = np.zeros((M, M))
    for ry in range(M):
        for rx in range(M):
            D[ry, rx] = np.mean(np.roll(np.roll(f, -ry, axis=0), -rx, axis=1) * f)
    assert np.abs(A - D).max() < 1e-12


def test_vorticity_correlation_axes_swap_under_transposition():
    """Reflecting the field across the diagonal (x <-> y) swaps C_x and C_y."""
    rng = np.random.default_rng(6)
    M, L = 32, 32.0
    ux, uy = rng.normal(size=(M, M)), rng.normal(size=(M, M))
    cx, cy, lx, ly = diag.vorticity_correlation_from_grid(ux, uy, L)
    tx, ty, mx, my = diag.vorticity_correlation_from_grid(uy.T.copy(), ux.T.copy(), L)
    assert np.abs(tx - cy).max() < 1e-12 and np.abs(ty - cx).max() < 1e-12
    assert (mx, my) == pytest.approx((ly, lx), abs=1e-12)
