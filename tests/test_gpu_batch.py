"""Batched replicas: uneven boxes over a (zeta, K) sweep in one launch per pass,
with hipGraph replay of step chunks, persistent pass kernels and the
autotuner; each replica must equal its solo run."""
import os
import sys

import numpy as np
import pytest

import workloads as wl

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import gpu_run, random_state  # noqa: E402

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
    after = [sim.get_state(r) for r in range(len(reps))]
    for a, b in zip(before, after):
        for k in a:
            assert np.array_equal(a[k], b[k]), k
    sim.step(3)
    sim.check()
    sim.close()
