"""Entry points that the physics tests reach only indirectly: the per-pass
timers, the read-back of every launch option, and the learned corrector's
weight read-back, output masking and evaluation statistics."""
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


def _sim():
    import paper_2108_08919_amd as P
    sim = P.Sim([wl.Params(L=32.0, zeta=0.02, dt=0.01)], [32 * 32])
    sim.set_state(0, random_state(32, 4, amp_u=0.02))
    return sim


def test_pass_times_count_every_launch_group_and_change_nothing():
    import paper_2108_08919_amd as P
    a, b = _sim(), _sim()
    b.set_option(P.NEM_OPT_TIMING, 1)
    assert b.get_option(P.NEM_OPT_TIMING) == 1
    b.pass_times(reset=True)
    b.step(12)
    ms, cnt = b.pass_times()
    assert cnt.tolist() == [12] * P.NEM_NPASS
    assert np.all(ms > 0.0) and np.all(np.isfinite(ms))
    # reading without reset keeps the totals; reset clears them
    ms2, cnt2 = b.pass_times(reset=True)
    assert np.array_equal(ms, ms2) and np.array_equal(cnt, cnt2)
    ms3, cnt3 = b.pass_times()
    assert cnt3.tolist() == [0] * P.NEM_NPASS and np.all(ms3 == 0.0)
    # graph replay is set aside while timing is on: the steps still run (and count) eagerly
    b.set_option(P.NEM_OPT_GRAPH, 4)
    b.step(8)
    _, cnt4 = b.pass_times(reset=True)
    assert cnt4.tolist() == [8] * P.NEM_NPASS
    # timing off: nothing more is recorded
    b.set_option(P.NEM_OPT_TIMING, 0)
    b.set_option(P.NEM_OPT_GRAPH, 0)
    b.step(5)
    _, cnt5 = b.pass_times()
    assert cnt5.tolist() == [0] * P.NEM_NPASS
    b.check()
    # the events only observe: the timed simulation equals the untimed one bit for bit
    a.step(25)
    a.check()
    ga, gb = a.get_state(0), b.get_state(0)
    for k in FIELDS:
        assert np.array_equal(ga[k], gb[k]), k
    a.close()
    b.close()


def test_every_option_reads_back_and_bad_values_leave_it_unchanged():
    import paper_2108_08919_amd as P
    sim = _sim()
    good = {P.NEM_OPT_TILE: (4, 8), P.NEM_OPT_LPP: (1, 2, 4), P.NEM_OPT_COMP: (0, 1, 2),
            P.NEM_OPT_TIMING: (0, 1), P.NEM_OPT_GRAPH: (0, 1, 7, 4096), P.NEM_OPT_PERSIST: (0, 512, 1 << 20)}
    bad = {P.NEM_OPT_TILE: (0, 2, 6, 16), P.NEM_OPT_LPP: (0, 3, 8), P.NEM_OPT_COMP: (-1, 3),
           P.NEM_OPT_GRAPH: (-1, 4097), P.NEM_OPT_PERSIST: (-1, (1 << 20) + 1)}
    for key, values in good.items():
        for v in values:
            sim.set_option(key, v)
            assert sim.get_option(key) == v, (key, v)
        keep = values[-1]
        for v in bad.get(key, ()):
            with pytest.raises(P.NemError) as e:
                sim.set_option(key, v)
            assert e.value.code == P.NEM_E_INVAL
            assert sim.get_option(key) == keep, (key, v)
    for key in (0, 7, 99):
        with pytest.raises(P.NemError):
            sim.get_option(key)
        with pytest.raises(P.NemError):
            sim.set_option(key, 1)
    # and the simulation still steps under the last values set
    sim.set_option(P.NEM_OPT_PERSIST, 0)
    sim.set_option(P.NEM_OPT_GRAPH, 0)
    sim.step(3)
    sim.check()
    sim.close()


def _weights(nparams, seed, scale=0.3):
    return np.random.default_rng(seed).normal(0.0, scale, nparams).astype(np.float32)


def _inputs(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    X = torch.from_numpy(rng.normal(0.0, 1.0, (n, 12)).astype(np.float32)).cuda()
    T = torch.from_numpy(rng.normal(0.5, 2.0, (n, 5)).astype(np.float32)).cuda()
    return X, T


def test_network_weights_and_normalisation_read_back():
    import paper_2108_08919_amd as P
    m = P.Mlp()
    assert m.nparams == 12 * 64 + 64 + 64 * 64 + 64 + 64 * 5 + 5
    assert np.all(m.get_weights() == 0.0)
    nm0 = m.get_norm()
    assert np.all(nm0[[*range(12), *range(24, 29)]] == 0.0) and np.all(nm0[[*range(12, 24), *range(29, 34)]] == 1.0)
    w = _weights(m.nparams, 1)
    m.set_weights(w)
    assert np.array_equal(m.get_weights(), w)
    nm = np.random.default_rng(2).uniform(0.5, 2.0, 34).astype(np.float32)
    m.set_norm(nm)
    assert np.array_equal(m.get_norm(), nm)
    m.close()


def test_masked_outputs_are_exactly_zero_and_the_rest_unchanged():
    import paper_2108_08919_amd as P
    m = P.Mlp()
    w = _weights(m.nparams, 3)
    m.set_weights(w)
    nm = np.concatenate([np.zeros(12), np.ones(12), [0.1, -0.2, 0.3, -0.4, 0.5], [2.0, 1.5, 1.0, 0.5, 0.25]])
    m.set_norm(nm.astype(np.float32))
    X, _ = _inputs(1000, 4)
    y0 = m.forward(X).cpu().numpy()
    m.mask_outputs([1, 3])
    y1 = m.forward(X).cpu().numpy()
    assert np.all(y1[:, [1, 3]] == 0.0)
    assert np.array_equal(y1[:, [0, 2, 4]], y0[:, [0, 2, 4]])
    # the last layer's columns and biases of the masked outputs are zero, every other weight is kept
    off_w3 = 12 * 64 + 64 + 64 * 64 + 64
    wm = m.get_weights()
    keep = np.ones(m.nparams, dtype=bool)
    for o in (1, 3):
        keep[off_w3 + np.arange(64) * 5 + o] = False
        keep[off_w3 + 64 * 5 + o] = False
    assert np.all(wm[~keep] == 0.0) and np.array_equal(wm[keep], w[keep])
    nmm = m.get_norm()
    assert nmm[25] == 0.0 and nmm[27] == 0.0 and np.array_equal(nmm[[24, 26, 28]], nm[[24, 26, 28]].astype(np.float32))
    m.mask_outputs(range(5))
    assert np.all(m.forward(X).cpu().numpy() == 0.0)
    _, mx = m.evaluate(X)
    assert mx == 0.0
    m.close()


def test_evaluation_statistics_equal_their_definition():
    """rel_mse[o] = mean (t - y)^2 / var t over the samples, max_norm = the
    largest Euclidean norm of (y - mean_T) / std_T, y the network's output."""
    import paper_2108_08919_amd as P
    m = P.Mlp()
    m.set_weights(_weights(m.nparams, 5))
    tm = np.array([0.1, -0.2, 0.3, -0.4, 0.5])
    ts = np.array([2.0, 1.5, 1.0, 0.5, 0.25])
    m.set_norm(np.concatenate([np.zeros(12), np.ones(12), tm, ts]).astype(np.float32))
    for n in (1, 257, 5003):
        X, T = _inputs(n, 6 + n)
        rel, mx = m.evaluate(X, T)
        y = m.forward(X).cpu().numpy().astype(np.float64)
        t = T.cpu().numpy().astype(np.float64)
        norm = np.sqrt((((y - tm.astype(np.float32)) / ts.astype(np.float32)) ** 2).sum(axis=1)).max()
        assert mx == pytest.approx(norm, rel=1e-5), n
        rel_none, mx_none = m.evaluate(X)
        assert rel_none is None and mx_none == mx
        if n == 1:
            assert all(np.isnan(r) for r in rel)  # one sample has no variance
            continue
        want = ((t - y) ** 2).mean(axis=0) / t.var(axis=0)
        np.testing.assert_allclose(rel, want, rtol=1e-10)
        # a perfect prediction scores zero
        rel0, _ = m.evaluate(X, m.forward(X))
        assert np.all(np.array(rel0) == 0.0)
    m.close()
