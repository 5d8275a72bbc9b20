"""Batched replicas: uneven boxes over a (zeta, K) sweep in one launch per pass,
with hipGraph replay of step chunks, persistent pass kernels and the
autotuner; each replica must equal its solo run, and the 32 replicas of the
batched workload (sides drawn from U{128..384}) must each match the oracle."""
import os
import sys

import numpy as np
import pytest

import workloads as wl

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import check_increments, field_errors, gpu_run, random_state, run_oracle  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_08919_amd as P
    P.lib()
    yield


def sweep(nrep=6, seed=0):
    rng = np.random.default_rng(seed)
    reps = []
    for r in range(nrep):
        side = int(rng.integers(24, 49))
        p = wl.Params(L=float(side), zeta=[0.005, 0.01, 0.02, 0.04][r % 4], K=[0.01, 0.02, 0.04, 0.08][(r // 2) % 4])
        reps.append((p, random_state(side, 100 + r, amp_u=2e-3)))
    return reps


@pytest.mark.parametrize("opts", [{}, {"graph": 4}, {"graph": 3, "persist": 7}, {"persist": 64, "tile": 8, "lpp": 2}])
def test_batch_equals_solo(opts):
    import paper_2108_08919_amd as P
    keymap = {"graph": P.NEM_OPT_GRAPH, "persist": P.NEM_OPT_PERSIST, "tile": P.NEM_OPT_TILE, "lpp": P.NEM_OPT_LPP}
    reps = sweep()
    sim = P.Sim([p for p, _ in reps], [s["x"].size for _, s in reps])
    for k, v in opts.items():
        sim.set_option(keymap[k], v)
    for r, (_, s) in enumerate(reps):
        sim.set_state(r, s)
    sim.step(10)
    sim.check()
    solo_opts = {keymap[k]: v for k, v in opts.items() if k in ("tile", "lpp")}
    for r, (p, s) in enumerate(reps):
        g = sim.get_state(r)
        h, hs = gpu_run(p, s, 10, solo_opts)
        for k in g:
            assert np.array_equal(g[k], h[k]), (r, k)
        hs.close()
    sim.close()


def test_autotune_keeps_state():
    import paper_2108_08919_amd as P
    reps = sweep(4, 1)
    sim = P.Sim([p for p, _ in reps], [s["x"].size for _, s in reps])
    for r, (_, s) in enumerate(reps):
        sim.set_state(r, s)
    sim.step(2)
    before = [sim.get_state(r) for r in range(len(reps))]
    t, l, ms = sim.autotune(3)
    assert t in (4, 8) and l in (1, 2, 4) and ms > 0
    assert sim.get_option(P.NEM_OPT_PERSIST) in (0, 512, 1024, 2048)
    assert (sim.get_option(P.NEM_OPT_TILE), sim.get_option(P.NEM_OPT_LPP)) == (t, l)
    after = [sim.get_state(r) for r in range(len(reps))]
    for a, b in zip(before, after):
        for k in a:
            assert np.array_equal(a[k], b[k]), k
    sim.step(3)
    sim.check()
    sim.close()


def test_ensemble_draw_against_oracle():
    """The batched workload itself: 32 replicas with sides drawn from
    U{128..384} (seeded), zeta x K sweep x 2 seeds, isotropic starts, advanced
    10 steps in one launch per pass with a persistent grid and graph replay;
    every replica against its own oracle run, to the fields' and increments'
    bars of the single-box tests."""
    import paper_2108_08919_amd as P
    reps = wl.ensemble(0)
    sides = [r["n_side"] for r in reps]
    assert len(reps) == 32 and min(sides) >= 128 and max(sides) <= 384
    states = [wl.state_for(r) for r in reps]
    sim = P.Sim([r["params"] for r in reps], [s["x"].size for s in states])
    sim.set_option(P.NEM_OPT_PERSIST, 1024)
    sim.set_option(P.NEM_OPT_GRAPH, 5)
    for i, s in enumerate(states):
        sim.set_state(i, s)
    sim.step(10)
    sim.check()
    worst = {}
    for i, (r, s0) in enumerate(zip(reps, states)):
        print("replica", i, "side", r["n_side"], "zeta", r["params"].zeta, "K", r["params"].K, flush=True)
        o, _ = run_oracle(r["params"], s0, 10)
        e = field_errors(sim.get_state(i), o, s0, r["params"].L, 10)
        for k in ("u", "Q", "rho", "pos"):
            assert e[k] <= 1e-5, (i, k, e[k])
        check_increments(e)
        for k, v in e.items():
            worst[k] = max(worst.get(k, 0.0), v)
    print({k: f"{v:.3e}" for k, v in worst.items()}, flush=True)
    sim.close()


def test_every_graph_replay_equals_eager_steps():
    """A captured graph of 5 steps replayed four times, with the program's own
    eager work between the replays (FP64 reductions, a grid deposit and defect
    count with its counter clearing, state reads) and a synchronisation after
    each: every replay's state equals that of the same batch stepped eagerly,
    bit for bit."""
    import paper_2108_08919_amd as P
    reps = sweep(4, 5)
    sims = []
    for graph in (0, 5):
        sim = P.Sim([p for p, _ in reps], [s["x"].size for _, s in reps])
        if graph:
            sim.set_option(P.NEM_OPT_GRAPH, graph)
        for r, (_, s) in enumerate(reps):
            sim.set_state(r, s)
        sims.append(sim)
    eager, graphed = sims
    for k in range(4):
        for sim in sims:
            sim.step(5)
            sim.check()
        for r in range(len(reps)):
            a, b = eager.get_state(r), graphed.get_state(r)
            for f in a:
                assert np.array_equal(a[f], b[f]), (k, r, f)
        # eager work on the graphed simulation's stream between replays
        graphed.diagnostics(0)
        graphed.defects(1, 32)
        graphed.check()
    for sim in sims:
        sim.close()


def test_persistent_grid_equals_dispatch():
    """The same batch with one workgroup per tile and with persistent grids of
    several sizes: identical results (the work list is walked in the same
    per-tile order either way)."""
    import paper_2108_08919_amd as P
    reps = sweep(5, 2)
    out = []
    for g in (0, 300, 1024):
        sim = P.Sim([p for p, _ in reps], [s["x"].size for _, s in reps])
        sim.set_option(P.NEM_OPT_PERSIST, g)
        assert sim.get_option(P.NEM_OPT_PERSIST) == g
        for r, (_, s) in enumerate(reps):
            sim.set_state(r, s)
        sim.step(8)
        sim.check()
        out.append([sim.get_state(r) for r in range(len(reps))])
        sim.close()
    for other in out[1:]:
        for a, b in zip(out[0], other):
            for k in a:
                assert np.array_equal(a[k], b[k]), k
