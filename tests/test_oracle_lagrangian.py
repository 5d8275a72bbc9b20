"""Pins of the Lagrangian-diagnostics oracle: mixing index limits and an
independent form of its definition, colour histograms against a brute-force
count, and pathlines of a uniformly translating box against u t."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import lagrangian as lg


def test_segregated_quadrants_have_index_zero():
    L, B = 16, 4
    x, y = wl.lattice(L)
    col = lg.quadrant_colour(x, y, float(L))
    assert np.bincount(col).tolist() == [64, 64, 64, 64]
    assert lg.mixing_index(lg.colour_counts(x, y, col, 4, B, float(L))) == pytest.approx(0.0, abs=1e-15)


def test_interleaved_colours_have_index_one():
    L, B = 16, 4
    x, y = wl.lattice(L)
    i, j = np.floor(x).astype(int), np.floor(y).astype(int)
    col = ((i % 2) + 2 * (j % 2)).astype(np.uint8)
    c = lg.colour_counts(x, y, col, 4, B, float(L))
    assert (c == 4).all()
    assert lg.mixing_index(c) == pytest.approx(1.0, abs=1e-15)


def test_index_matches_variance_form_and_ignores_labels():
    """I = (sum_b N_b sum_c phi_cb^2 - N sum_c phi_c^2) / (N (1 - sum_c phi_c^2)),
    the same quantity expanded; relabelling the colours changes nothing."""
    rng = np.random.default_rng(3)
    counts = rng.integers(0, 9, size=(5, 5, 3))
    h = counts.reshape(-1, 3).astype(float)
    N, Nb = h.sum(), h.sum(axis=1)
    phi = h.sum(axis=0) / N
    keep = Nb > 0
    I = ((h[keep] ** 2 / Nb[keep, None]).sum() - N * (phi ** 2).sum()) / (N * (1 - (phi ** 2).sum()))
    assert lg.mixing_index(counts) == pytest.approx(1.0 - I, abs=1e-13)
    assert lg.mixing_index(counts[..., [2, 0, 1]]) == pytest.approx(1.0 - I, abs=1e-13)


def test_random_colouring_segregation_is_bins_over_particles():
    """Independent random colours: E[I] = B^2 / N (multinomial variance per bin)."""
    L, B = 64, 8
    x, y = wl.lattice(L)
    rng = np.random.default_rng(9)
    col = rng.integers(0, 4, size=x.size).astype(np.uint8)
    I = 1.0 - lg.mixing_index(lg.colour_counts(x, y, col, 4, B, float(L)))
    assert I == pytest.approx(B * B / x.size, rel=0.35)


def test_colour_counts_against_direct_binning():
    rng = np.random.default_rng(4)
    L, B = 10.0, 5
    x = rng.uniform(-L, 2 * L, 500)
    y = rng.uniform(-L, 2 * L, 500)
    col = rng.integers(0, 3, 500)
    c = lg.colour_counts(x, y, col, 3, B, L)
    for by in range(B):
        for bx in range(B):
            for k in range(3):
                xw, yw = np.mod(x, L), np.mod(y, L)
                sel = (xw >= bx * L / B) & (xw < (bx + 1) * L / B) & (yw >= by * L / B) & (yw < (by + 1) * L / B)
                assert c[by, bx, k] == int((sel & (col == k)).sum())
    assert c.sum() == 500


def test_uniform_translation_pathlines():
    """A uniformly moving box stays uniform (every difference sum vanishes), so
    each particle travels u t through several periodic crossings."""
    L = 16
    x, y = wl.lattice(L)
    n = x.size
    u = (0.7, -0.4)
    p = wl.Params(L=float(L), dt=0.05)
    st = oracle.State(dict(x=x, y=y, ux=np.full(n, u[0]), uy=np.full(n, u[1]), qxx=np.ones(n), qxy=np.zeros(n),
                           rho=np.ones(n), ax=np.zeros(n), ay=np.zeros(n)))
    xs, ys = [x.copy()], [y.copy()]
    for _ in range(600):
        oracle.step(p, st, 1)
        f = st.fields()
        xs.append(lg.unwrap(xs[-1], f["x"], L))
        ys.append(lg.unwrap(ys[-1], f["y"], L))
    t = 600 * p.dt
    assert np.abs(xs[-1] - (x + u[0] * t)).max() < 1e-10
    assert np.abs(ys[-1] - (y + u[1] * t)).max() < 1e-10
    assert u[0] * t > L                       # crossed the box in x
    ln = lg.pathline_length(np.array(xs), np.array(ys))
    assert np.abs(ln - math.hypot(*u) * t).max() < 1e-9
