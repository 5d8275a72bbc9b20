"""GPU Lagrangian diagnostics against the oracle: unwrapped pathlines through
periodic crossings and rebinning, colour histograms and the mixing index."""
import math
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import lagrangian as lg

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import random_state  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_08919_amd as P
    P.lib()
    yield


def _uniform(L, u, shift=0.0):
    x, y = wl.lattice(L)
    n = x.size
    return dict(x=x + shift, y=y - shift, ux=np.full(n, u[0]), uy=np.full(n, u[1]), qxx=np.ones(n),
                qxy=np.zeros(n), rho=np.ones(n), ax=np.zeros(n), ay=np.zeros(n))


def test_uniform_translation_through_several_crossings():
    import paper_2108_08919_amd as P
    L = 16
    u = (0.75, -0.375)          # u, dt and the lattice are binary fractions:
    p = wl.Params(L=float(L), dt=0.0625)   # FP32 storage of u adds no error
    st = _uniform(L, u)
    n = st["x"].size
    sim = P.Sim([p], [n])
    sim.set_state(0, st)
    ids = np.arange(n)
    x0, y0 = sim.track(ids)
    assert np.abs(x0 - st["x"]).max() < 1e-12 and np.abs(y0 - st["y"]).max() < 1e-12
    done = 0
    for chunk in (300, 300, 400):
        sim.step(chunk)
        done += chunk
        x, y = sim.track(ids)
        t = done * p.dt
        print(done, np.abs(x - (st["x"] + u[0] * t)).max(), flush=True)
        assert np.abs(x - (st["x"] + u[0] * t)).max() < 1e-9 * L
        assert np.abs(y - (st["y"] + u[1] * t)).max() < 1e-9 * L
    assert u[0] * done * p.dt > 2 * L            # two crossings in x, one in -y
    # the wrapped state is unchanged by tracking
    g = sim.get_state(0)
    assert g["x"].min() >= 0 and g["x"].max() < L
    sim.close()


def test_state_set_from_unwrapped_coordinates_reads_back():
    import paper_2108_08919_amd as P
    L = 16
    p = wl.Params(L=float(L))
    st = _uniform(L, (0.0, 0.0), shift=-37.0)      # every particle a few images away
    n = st["x"].size
    sim = P.Sim([p], [n])
    sim.set_state(0, st)
    x, y = sim.track(np.arange(n))
    assert np.abs(x - st["x"]).max() < 1e-12 and np.abs(y - st["y"]).max() < 1e-12
    sub = np.array([5, 0, n - 1, 5], dtype=np.int32)
    xs, ys = sim.track(sub)
    assert np.array_equal(xs, x[sub]) and np.array_equal(ys, y[sub])
    with pytest.raises(P.NemError):
        sim.track(np.array([n]))
    with pytest.raises(P.NemError):
        sim.track(np.array([-1]))
    sim.close()


def test_tracking_survives_snapshot_restore():
    """The autotuner runs trial steps from a snapshot and restores it: the image
    counters come back with the rest of the state."""
    import paper_2108_08919_amd as P
    L = 32
    u = (0.625, 0.4375)
    p = wl.Params(L=float(L), dt=0.0625)
    st = _uniform(L, u)
    n = st["x"].size
    sim = P.Sim([p], [n])
    sim.set_state(0, st)
    sim.step(700)
    sim.autotune(40)
    sim.step(500)
    x, y = sim.track(np.arange(n))
    t = 1200 * p.dt
    assert np.abs(x - (st["x"] + u[0] * t)).max() < 1e-9 * L
    assert np.abs(y - (st["y"] + u[1] * t)).max() < 1e-9 * L
    sim.close()


def test_pathlines_match_oracle_with_rebinning():
    """A drifting random state: particles change cells and cross the periodic
    boundary; GPU pathlines against the oracle's unwrapped per step."""
    import paper_2108_08919_amd as P
    L = 32
    p = wl.Params(L=float(L), zeta=0.03, K=0.04, dt=5e-3)
    s0 = random_state(L, 21, amp_u=2e-3)
    s0["ux"] = s0["ux"] + 1.5
    s0["uy"] = s0["uy"] - 1.0
    n = s0["x"].size
    st = oracle.State(s0)
    sim = P.Sim([p], [n])
    sim.set_state(0, s0)
    ox, oy = s0["x"].copy(), s0["y"].copy()
    crossed = 0
    for k in range(1, 61):
        oracle.step(p, st, 1)
        f = st.fields()
        nx, ny = lg.unwrap(ox, f["x"], L), lg.unwrap(oy, f["y"], L)
        crossed += int(((np.floor(nx / L) != np.floor(ox / L)) | (np.floor(ny / L) != np.floor(oy / L))).sum())
        ox, oy = nx, ny
        if k % 20 == 0:
            sim.step(20)
            gx, gy = sim.track(np.arange(n))
            err = max(np.abs(gx - ox).max(), np.abs(gy - oy).max())
            print(k, "crossings so far", crossed, "max err", err, flush=True)
            # FP32 u and APD cutoff flips leave errors of 1e-8..1e-6; a wrong
            # image or cell shift would be L or a cell side
            assert err < 1e-5
    assert crossed > 10
    sim.close()


def test_mixing_counts_and_index():
    import paper_2108_08919_amd as P
    L, B = 32, 8
    p = wl.Params(L=float(L), zeta=0.03, K=0.04)
    s0 = random_state(L, 22, amp_u=3e-3, jitter=0.2)
    n = s0["x"].size
    col = lg.quadrant_colour(np.mod(s0["x"], L), np.mod(s0["y"], L), float(L))
    sim = P.Sim([p], [n])
    sim.set_state(0, s0)
    idx0, c0 = sim.mixing(col, 4, B)
    o0 = lg.colour_counts(s0["x"], s0["y"], col, 4, B, float(L))
    assert np.array_equal(c0, o0)
    assert idx0 == pytest.approx(lg.mixing_index(o0), abs=1e-13)
    sim.step(30)
    g = sim.get_state(0)
    idx, c = sim.mixing(col, 4, B)
    assert np.array_equal(c, lg.colour_counts(g["x"], g["y"], col, 4, B, float(L)))
    assert idx == pytest.approx(lg.mixing_index(c), abs=1e-13)
    st = oracle.State(s0)
    oracle.step(p, st, 30)
    f = st.fields()
    oc = lg.colour_counts(f["x"], f["y"], col, 4, B, float(L))
    assert np.abs(c - oc).sum() <= 2
    # the colours are a function of the id, so the histogram of the ids does not
    # depend on the sorted order: a second call gives the same counts
    idx2, c2 = sim.mixing(col, 4, B)
    assert np.array_equal(c2, c) and idx2 == idx
    with pytest.raises(P.NemError):
        sim.mixing(np.full(n, 4, dtype=np.uint8), 4, B)
    sim.close()


def test_pathlines_and_mixing_grow_with_activity():
    """Sec. 5: pathlines lengthen and the quadrants mix faster as |zeta| grows,
    for extensile and contractile activity."""
    from paper_2108_08919_amd import lagrangian, sweep
    reps = sweep.build_replicas([0.1, 0.4], [0.02], 1, 64, "both")
    print("replicas", len(reps), flush=True)
    rows = {r["zeta"]: r for r in lagrangian.table(lagrangian.run(reps, 10000, 2500, n_tag=64))}
    print({z: (r["path_length"], r["mixing"]) for z, r in rows.items()}, flush=True)
    for sg in (1.0, -1.0):
        lo, hi = rows[0.1 * sg], rows[0.4 * sg]
        assert hi["path_length"] > 2.5 * lo["path_length"] > 0
        assert hi["net_displacement"] <= hi["path_length"]
        assert hi["mixing"] > lo["mixing"] + 0.01
