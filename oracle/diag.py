"""Grid diagnostics of the oracle (TEST INFRASTRUCTURE): kinetic-energy spectrum
and +-1/2 defect counts (paper Sec. 5: Eq. kineticenergy and the energy
spectrum figure; the defect maps of Fig. nematicdirector).

Readings (the paper gives no formulas for either):
* spectrum: Shepard-interpolate u onto an M x M grid, take the 2D FFT,
  E(n) = 1/2 sum_{shell n} |u_hat|^2 / M^4 with shell n = floor(|k| L/2pi + 1/2),
  so that sum_n E(n) = 1/2 <|u|^2> over the grid (Parseval). The slope is the
  least-squares fit of ln E against ln n over n in [k_lo, k_hi].
* defects: director angle theta = atan2(Qxy, Qxx)/2 on the grid; around each
  unit plaquette add the four edge differences of theta, each wrapped into
  (-pi/2, pi/2]; a total of +pi is a +1/2 defect, -pi a -1/2 defect.
* vorticity correlation (Eq. corr): the paper fixes C(r) = <f(r) f(0)> / f(0)^2
  with f the vorticity and r along the horizontal centre line; in a periodic
  box every point can serve as the origin, so the average runs over all grid
  points: C(r) = <omega(x + r) omega(x)>_x / <omega^2>_x, reported along x (the
  paper's direction) and along y. omega = d uy/dx - d ux/dy on the grid is taken
  spectrally, omega_hat = i (kx uy_hat - ky ux_hat) with k = 2 pi n / L, the
  Nyquist wavenumber n = -M/2 set to zero. The length scale is the first zero
  crossing of C, linearly interpolated between grid separations.
The FFT is numpy's (a library primitive); everything else is written out.
"""
from __future__ import annotations

import math

import numpy as np


def spectrum_from_grid(ux: np.ndarray, uy: np.ndarray, nbins: int | None = None):
    M = ux.shape[0]
    fx = np.fft.fft2(ux)
    fy = np.fft.fft2(uy)
    e = 0.5 * (np.abs(fx) ** 2 + np.abs(fy) ** 2) / float(M) ** 4
    k = np.fft.fftfreq(M) * M                 # integer wavenumbers
    KX, KY = np.meshgrid(k, k, indexing="xy")
    shell = np.floor(np.sqrt(KX ** 2 + KY ** 2) + 0.5).astype(np.int64)
    nb = nbins if nbins is not None else int(shell.max()) + 1
    E = np.zeros(nb)
    for s in range(nb):
        E[s] = e[shell == s].sum()
    return E


def slope(E: np.ndarray, k_lo: int, k_hi: int) -> float:
    n = np.arange(E.size)
    sel = (n >= k_lo) & (n <= k_hi) & (E > 0)
    lx, ly = np.log(n[sel].astype(np.float64)), np.log(E[sel])
    A = np.vstack([lx, np.ones_like(lx)]).T
    coef, *_ = np.linalg.lstsq(A, ly, rcond=None)
    return float(coef[0])


def _wrap_half_pi(d: np.ndarray) -> np.ndarray:
    """Wrap angle differences into (-pi/2, pi/2]."""
    w = d - math.pi * np.floor(d / math.pi + 0.5)
    w = np.where(w <= -math.pi / 2, w + math.pi, w)
    return w


def defects_from_grid(qxx: np.ndarray, qxy: np.ndarray):
    th = 0.5 * np.arctan2(qxy, qxx)
    a = th
    b = np.roll(th, -1, axis=1)               # (i+1, j)
    c = np.roll(b, -1, axis=0)                # (i+1, j+1)
    d = np.roll(th, -1, axis=0)               # (i, j+1)
    w = _wrap_half_pi(b - a) + _wrap_half_pi(c - b) + _wrap_half_pi(d - c) + _wrap_half_pi(a - d)
    plus = int(np.count_nonzero(w > 0.5 * math.pi))
    minus = int(np.count_nonzero(w < -0.5 * math.pi))
    return plus, minus, w


def spectrum(params, x, y, ux, uy, M: int, k_lo: int | None = None, k_hi: int | None = None):
    from . import deposit
    g = deposit(params, x, y, [ux, uy], M)
    E = spectrum_from_grid(g[0], g[1])
    lo = 4 if k_lo is None else k_lo
    hi = M // 8 if k_hi is None else k_hi
    return E, slope(E, lo, hi)


def defects(params, x, y, qxx, qxy, M: int):
    from . import deposit
    g = deposit(params, x, y, [qxx, qxy], M)
    p, m, _ = defects_from_grid(g[0], g[1])
    return p, m


def vorticity_from_grid(ux: np.ndarray, uy: np.ndarray, L: float) -> np.ndarray:
    """omega = d uy/dx - d ux/dy of grid fields (rows = y, columns = x)."""
    M = ux.shape[0]
    n = np.fft.fftfreq(M) * M
    n[M // 2] = 0.0                             # the Nyquist wavenumber has no derivative
    k = 2.0 * math.pi * n / L
    KX, KY = np.meshgrid(k, k, indexing="xy")   # KX varies along columns (x)
    w_hat = 1j * (KX * np.fft.fft2(uy) - KY * np.fft.fft2(ux))
    return np.real(np.fft.ifft2(w_hat))


def autocorrelation(f: np.ndarray) -> np.ndarray:
    """A[ry, rx] = mean over grid points x of f(x + r) f(x) (periodic), from the
    power spectrum (Wiener-Khinchin)."""
    M = f.shape[0]
    F = np.fft.fft2(f)
    return np.real(np.fft.ifft2(np.abs(F) ** 2)) / float(M * M)


def first_zero(c: np.ndarray, dl: float) -> float:
    for n in range(1, c.size):
        if c[n] <= 0.0:
            return (n - 1 + c[n - 1] / (c[n - 1] - c[n])) * dl
    return -1.0


def vorticity_correlation_from_grid(ux: np.ndarray, uy: np.ndarray, L: float):
    """(C_x, C_y, l_x, l_y) for separations n L/M, n = 0..M/2."""
    M = ux.shape[0]
    A = autocorrelation(vorticity_from_grid(ux, uy, L))
    H = M // 2
    cx = A[0, :H + 1] / A[0, 0]
    cy = A[:H + 1, 0] / A[0, 0]
    dl = L / M
    return cx, cy, first_zero(cx, dl), first_zero(cy, dl)


def vorticity_correlation(params, x, y, ux, uy, M: int):
    from . import deposit
    g = deposit(params, x, y, [ux, uy], M)
    return vorticity_correlation_from_grid(g[0], g[1], params.L)
