"""Oracle for the Lagrangian diagnostics of Sec. 5: pathlines of tagged
particles and the mixing of colour-marked regions (test infrastructure only:
imported by tests, never by the library).

Readings (the paper shows pathlines and mixing as pictures and gives no
formula for either):
* pathline: the unwrapped position of a particle, i.e. its position in the
  periodic box plus L times the number of times it crossed each boundary;
  from positions sampled often enough that no particle moves L/2 between two
  samples, each step adds the minimum-image displacement. Its length is the
  sum of |dr| over the samples.
* colours: the four quadrants of the box at the start (x >= L/2 and y >= L/2
  select the colour bits).
* mixing index: 1 - I with I Danckwerts' intensity of segregation on a B x B
  partition of the box,
      I = sum_b sum_c N_b (phi_cb - phi_c)^2 / sum_c N phi_c (1 - phi_c),
  phi_cb = N_cb / N_b the colour fractions in bin b and phi_c = N_c / N those of
  the box. I = 1 while every bin holds one colour and 0 when every bin holds
  the box's mixture.
"""
from __future__ import annotations

import math

import numpy as np


def min_image(d: np.ndarray, L: float) -> np.ndarray:
    return d - L * np.round(d / L)


def unwrap(prev: np.ndarray, wrapped: np.ndarray, L: float) -> np.ndarray:
    """Next unwrapped position from the previous one and the new wrapped one."""
    return prev + min_image(wrapped - prev, L)


def pathline_length(xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """Arc length of each pathline; xs, ys have shape (samples, particles)."""
    return np.sqrt(np.diff(xs, axis=0) ** 2 + np.diff(ys, axis=0) ** 2).sum(axis=0)


def quadrant_colour(x: np.ndarray, y: np.ndarray, L: float) -> np.ndarray:
    return ((x >= 0.5 * L).astype(np.uint8) + 2 * (y >= 0.5 * L).astype(np.uint8)).astype(np.uint8)


def colour_counts(x, y, colour, ncol: int, B: int, L: float) -> np.ndarray:
    """counts[by, bx, c]: particles of colour c in bin (bx, by), bx = floor(x B / L)
    of the position wrapped into [0, L)."""
    counts = np.zeros((B, B, ncol), dtype=np.int64)
    for xi, yi, c in zip(np.asarray(x, float), np.asarray(y, float), np.asarray(colour)):
        xw = xi - L * math.floor(xi / L)
        if xw >= L:
            xw -= L
        yw = yi - L * math.floor(yi / L)
        if yw >= L:
            yw -= L
        bx = min(max(int(math.floor(xw * B / L)), 0), B - 1)
        by = min(max(int(math.floor(yw * B / L)), 0), B - 1)
        counts[by, bx, int(c)] += 1
    return counts


def mixing_index(counts: np.ndarray) -> float:
    """1 - I from a histogram counts[..., c] (bins x colours)."""
    h = counts.reshape(-1, counts.shape[-1]).astype(np.float64)
    N = h.sum()
    phi = h.sum(axis=0) / N
    den = (N * phi * (1.0 - phi)).sum()
    if den <= 0.0:
        return float("nan")
    num = 0.0
    for row in h:
        Nb = row.sum()
        if Nb > 0:
            num += (Nb * (row / Nb - phi) ** 2).sum()
    return 1.0 - num / den
