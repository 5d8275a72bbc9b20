"""Checkpoints: a simulation loaded from nem_save_raw's bytes continues bit
for bit as the saved one does, across Verlet rebuilds and rebins, with the
saved launch options; mismatched or damaged checkpoints are refused and leave
the simulation unchanged; the portable .npz field record reads back."""
import os
import sys

import numpy as np
import pytest

import workloads as wl

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import random_state  # noqa: E402

pytestmark = pytest.mark.gpu

FIELDS = ("x", "y", "ux", "uy", "qxx", "qxy", "rho", "ax", "ay")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_08919_amd as P
    P.lib()
    yield


def _replicas():
    """Two boxes of different size; the first drifts fast enough to rebuild its
    Verlet list every two steps and to rebin (a drift of 0.029 per step against
    a rebuild distance of 0.044 and cells of side 4; c0 dt / h = 0.23), the
    second is the plain random state."""
    pa = wl.Params(L=32.0, zeta=0.02, dt=0.01)
    pb = wl.Params(L=24.0, zeta=-0.03, K=0.04, dt=0.01)
    sa = random_state(32, 6, amp_u=0.05)
    sa["ux"] = sa["ux"] + 2.5
    sa["uy"] = sa["uy"] - 1.5
    sb = random_state(24, 3, amp_u=2e-3)
    return [pa, pb], [sa, sb]


def _sim(params, states, tile=4, lpp=1):
    import paper_2108_08919_amd as P
    sim = P.Sim(params, [s["x"].size for s in states])
    sim.set_option(P.NEM_OPT_TILE, tile)
    sim.set_option(P.NEM_OPT_LPP, lpp)
    for r, s in enumerate(states):
        sim.set_state(r, s)
    return sim


def test_checkpoint_resumes_bit_for_bit(tmp_path):
    import paper_2108_08919_amd as P
    params, states = _replicas()
    a = _sim(params, states, tile=8, lpp=2)
    a.step(7)
    a.check()
    path = str(tmp_path / "run.nemraw")
    a.checkpoint(path)
    a.step(25)
    a.check()
    ref = [a.get_state(r) for r in range(2)]
    a.close()
    # a fresh simulation with default options picks up the saved ones
    b = P.Sim(params, [s["x"].size for s in states])
    b.restore(path)
    assert b.get_option(P.NEM_OPT_TILE) == 8 and b.get_option(P.NEM_OPT_LPP) == 2
    b.step(25)
    b.check()
    for r in range(2):
        g = b.get_state(r)
        for k in FIELDS:
            assert np.array_equal(g[k], ref[r][k]), (r, k)
    # the drifting box moved 0.8 along x over the 32 steps: cells changed and the list was rebuilt
    dx = np.mod(ref[0]["x"] - states[0]["x"] + 16.0, 32.0) - 16.0
    assert dx.mean() > 0.7
    b.close()


def test_mismatched_or_damaged_checkpoints_are_refused():
    import paper_2108_08919_amd as P
    params, states = _replicas()
    a = _sim(params, states)
    a.step(3)
    buf = a.save_raw()
    before = a.get_state(1)
    # another parameter, another size, another replica count
    for other_params, other_states in (([params[0], params[1].replace(zeta=0.03)], states),
                                       ([params[0], wl.Params(L=28.0)], [states[0], random_state(28, 1)]),
                                       ([params[0]], [states[0]])):
        c = _sim(other_params, other_states)
        with pytest.raises(P.NemError) as e:
            c.load_raw(buf)
        assert e.value.code == P.NEM_E_INVAL
        c.close()
    with pytest.raises(P.NemError) as e:
        a.load_raw(buf[: buf.size // 2])
    assert e.value.code == P.NEM_E_NOMEM
    bad = buf.copy()
    bad[:8] = np.frombuffer(b"NOTRAW00", dtype=np.uint8)
    with pytest.raises(P.NemError) as e:
        a.load_raw(bad)
    assert e.value.code == P.NEM_E_INVAL
    after = a.get_state(1)
    for k in FIELDS:
        assert np.array_equal(before[k], after[k]), k
    # and it loads into itself: the state saved three steps in
    a.step(2)
    a.load_raw(buf)
    for k in FIELDS:
        assert np.array_equal(a.get_state(1)[k], before[k]), k
    a.close()


def test_fields_record_reads_back(tmp_path):
    params, states = _replicas()
    a = _sim(params, states)
    a.step(2)
    path = str(tmp_path / "fields.npz")
    a.save_fields(path)
    rec = np.load(path)
    for r in range(2):
        g = a.get_state(r)
        for k in FIELDS:
            assert np.array_equal(rec[f"{k}_{r}"], g[k]), (r, k)
    a.close()
