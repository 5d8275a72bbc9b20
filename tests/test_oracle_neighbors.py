"""Neighbour search pins: the oracle's cell list and brute force against an
independent O(N^2) numpy minimum-image search on tiny periodic boxes, and the
FP32 cell-relative predicate against FP64 on inputs with no pair near 3h."""
import numpy as np
import pytest

import oracle
import workloads as wl


def numpy_brute(x, y, L, R):
    dx = x[:, None] - x[None, :]
    dy = y[:, None] - y[None, :]
    dx -= L * np.round(dx / L)
    dy -= L * np.round(dy / L)
    r2 = dx * dx + dy * dy
    ok = (r2 > 0) & (r2 < R * R)
    return [set(np.nonzero(ok[i])[0].tolist()) for i in range(x.size)], r2


def rows(rp, col):
    return [set(col[rp[i]:rp[i + 1]].tolist()) for i in range(rp.size - 1)]


CASES = []
for L in (8, 12, 16):
    CASES.append(("lattice", L))
    CASES.append(("jitter", L))
    CASES.append(("uniform", L))


@pytest.mark.parametrize("kind,L", CASES)
def test_cell_and_brute_match_numpy(kind, L):
    p = wl.Params(L=float(L))
    if kind == "lattice":
        x, y = wl.lattice(L)
    elif kind == "jitter":
        x, y = wl.jittered_lattice(L, 1.0, 0.3, seed=L)
    else:
        x, y = wl.uniform_positions(L * L, float(L), seed=L)
    ref, _ = numpy_brute(x, y, float(L), 3 * p.h)
    for mode in (0, 1):
        rp, col = oracle.neighbors(p, x, y, mode)
        assert rows(rp, col) == ref
        for i in range(x.size):                         # rows are sorted ascending
            r = col[rp[i]:rp[i + 1]]
            assert np.all(np.diff(r) > 0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fp32_predicate_agrees_away_from_boundary(seed):
    L = 16
    p = wl.Params(L=float(L))
    x, y = wl.uniform_positions(L * L, float(L), seed=seed)
    ref, r2 = numpy_brute(x, y, float(L), 3 * p.h)
    nc = int(np.floor(L / (3 * p.h + p.skin)))
    rp, col = oracle.neighbors(p, x, y, 2, nc)
    got = rows(rp, col)
    R2 = (3 * p.h) ** 2
    margin = np.abs(r2 - R2) < 1e-4
    for i in range(x.size):
        near = set(np.nonzero(margin[i])[0].tolist())
        assert got[i] - near == ref[i] - near


def test_fp32_predicate_on_lattice_is_exact():
    L = 16
    p = wl.Params(L=float(L))
    x, y = wl.lattice(L)
    nc = int(np.floor(L / (3 * p.h + p.skin)))
    rp, col = oracle.neighbors(p, x, y, 2, nc)
    ref, _ = numpy_brute(x, y, float(L), 3 * p.h)
    assert rows(rp, col) == ref


@pytest.mark.parametrize("kernel,L,seed", [(0, 24, 1), (0, 40, 2), (1, 24, 3)])
def test_step_list_in_fp32_equals_the_brute_force_rule(kernel, L, seed):
    """search = 2: the list the step builds (cell list, each pair decided by
    the FP32 rule on its own cell-relative offsets) equals the brute-force
    application of the same rule over all pairs in adjacent cells (mode 2),
    on jittered and uniform positions, for both kernels."""
    p = wl.Params(L=float(L), kernel=kernel)
    nc = int(np.floor(L / (oracle.kappa(kernel) * p.h + p.skin)))
    for x, y in (wl.jittered_lattice(L, 1.0, 0.4, seed), wl.uniform_positions(L * L, float(L), seed)):
        a = oracle.neighbors(p, x, y, 2, nc)
        b = oracle.neighbors(p, x, y, 3, nc)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_fp32_decision_changes_nothing_away_from_the_support_edge():
    """On the lattice no pair lies near 3h (the nearest lattice distances are
    sqrt(13) = 3.61 and 4), so a step that decides pairs in FP32 (search 2)
    equals the FP64-decided step (search 0) bit for bit over five steps."""
    cfg = wl.config("C1")
    s0 = wl.state_for(cfg, 0)
    a, b = oracle.State(s0), oracle.State(s0)
    oracle.step(cfg["params"], a, 5, search=0)
    oracle.step(cfg["params"], b, 5, search=2)
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
