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
