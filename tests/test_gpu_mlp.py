"""The learned corrector on the GPU: BF16-MFMA forward and backward kernels
against the FP64 reference network on the same (BF16-rounded) weights and
inputs, training, sample generation from the solver, and the learned macro
step with its fallback."""
import os
import sys

import numpy as np
import pytest

from oracle import mlp as ref
import workloads as wl

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import field_errors, gpu_run, random_state  # noqa: E402

pytestmark = pytest.mark.gpu

IDENT = np.concatenate([np.zeros(12), np.ones(12), np.zeros(5), np.ones(5)]).astype(np.float32)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_08919_amd as P
    P.lib()
    yield


def cosine(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


def setup(n, seed):
    import torch
    import paper_2108_08919_amd as P
    rng = np.random.default_rng(seed)
    params = [p + 0.05 * rng.normal(size=p.shape) for p in ref.init(seed)]
    w32 = ref.flatten(params).astype(np.float32)
    X = rng.normal(size=(n, 12)).astype(np.float32)
    T = rng.normal(size=(n, 5)).astype(np.float32)
    m = P.Mlp()
    m.set_weights(w32)
    m.set_norm(IDENT)
    Xt = torch.from_numpy(X).cuda()
    Tt = torch.from_numpy(T).cuda()
    # reference on the values the GPU sees: BF16 weights and inputs
    pb = [ref.to_bf16(p) for p in ref.unflatten(w32.astype(np.float64))]
    for k in (1, 3, 5):                  # biases stay FP32 on the GPU
        pb[k] = ref.unflatten(w32.astype(np.float64))[k]
    return m, Xt, Tt, pb, ref.to_bf16(X.astype(np.float64)), T.astype(np.float64)


@pytest.mark.parametrize("n", [32, 1000, 4133])
def test_forward_matches_reference(n):
    m, Xt, Tt, pb, Xb, T = setup(n, 1)
    Y = m.forward(Xt).cpu().numpy().astype(np.float64)
    y_ref, _ = ref.forward(pb, Xb)
    rel = np.linalg.norm(Y - y_ref) / np.linalg.norm(y_ref)
    print("forward rel", rel, "cos", cosine(Y.ravel(), y_ref.ravel()), flush=True)
    assert cosine(Y.ravel(), y_ref.ravel()) >= 0.999
    assert rel <= 2e-2
    m.close()


@pytest.mark.parametrize("n", [64, 2050])
def test_gradient_matches_reference(n):
    m, Xt, Tt, pb, Xb, T = setup(n, 2)
    g, loss = m.grad(Xt, Tt)
    g_ref = ref.flatten(ref.grad(pb, Xb, T))
    l_ref = ref.loss(pb, Xb, T)
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print("grad rel", rel, "cos", cosine(g, g_ref), "loss", loss, l_ref, flush=True)
    assert cosine(g.astype(np.float64), g_ref) >= 0.999
    assert rel <= 2e-2
    assert loss == pytest.approx(l_ref, rel=2e-2)
    # every block of the flat vector is non-trivially matched
    off = 0
    for a, b in [(12, 64), (64, 64), (64, 5)]:
        for size in (a * b, b):
            blk = slice(off, off + size)
            assert cosine(g[blk].astype(np.float64), g_ref[blk]) >= 0.99
            off += size
    m.close()


def test_training_reduces_loss():
    import torch
    import paper_2108_08919_amd as P
    rng = np.random.default_rng(3)
    n = 8192
    X = rng.normal(size=(n, 12)).astype(np.float32)
    Wt = rng.normal(size=(12, 5)) * 0.4
    T = (np.tanh(X @ Wt) * 3.0 + 1.0).astype(np.float32)
    m = P.Mlp()
    m.set_weights(ref.flatten(ref.init(0)).astype(np.float32))
    Xt, Tt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    m.fit_norm(Xt, Tt)
    nm = m.get_norm()
    assert np.allclose(nm[:12], X.mean(0), atol=1e-4) and np.allclose(nm[12:24], X.std(0), rtol=1e-4)
    _, l0 = m.grad(Xt, Tt)
    m.train(Xt, Tt, epochs=30, batch=512, lr=3e-3)
    _, l1 = m.grad(Xt, Tt)
    print("loss", l0, "->", l1, flush=True)
    assert l1 < 0.1 * l0
    Y = m.forward(Xt).cpu().numpy()
    assert np.linalg.norm(Y - T) / np.linalg.norm(T - T.mean(0)) < 0.3
    m.close()


def test_samples_leave_state_unchanged():
    L = 32
    p = wl.Params(L=float(L), zeta=0.03, K=0.04)
    s0 = random_state(L, 21, amp_u=3e-3)
    g0, sim = gpu_run(p, s0, 3)
    X, T = sim.samples(4)
    g1 = sim.get_state(0)
    for k in g0:
        assert np.array_equal(g0[k], g1[k]), k
    X, T = X.cpu().numpy(), T.cpu().numpy()
    assert X.shape == (L * L, 12) and T.shape == (L * L, 5)
    assert np.all(np.isfinite(X)) and np.all(np.isfinite(T))
    assert np.allclose(X[:, 0], g0["qxx"], atol=1e-6) and np.allclose(X[:, 1], g0["qxy"], atol=1e-6)
    assert np.all(X[:, 9] == np.float32(p.zeta))
    assert np.allclose(T[:, 2], -T[:, 0], atol=1e-7)
    # inputs 10-11: the coarse step's change of acceleration, a^{n+1/2} - a^{n-1/2}
    # (here against a coarse step from the re-ingested state, whose prediction
    # rounds differently in FP32: agreement to a few ulps of a)
    c, sc = gpu_run(p.replace(dt=4 * p.dt), g0, 1)
    da = np.stack([c["ax"] - g0["ax"], c["ay"] - g0["ay"]], 1)
    assert np.abs(X[:, 10:12] - da).max() < 1e-3 * np.abs(da).max()
    # targets are the small difference between fine and coarse stepping
    assert np.abs(T[:, :2]).max() < 1e-2 * np.abs(X[:, :2]).max()
    # rows: the same samples for a chosen subset
    rows = np.array([5, 17, 400, L * L - 1])
    Xr, Tr = sim.samples_rows(rows, 4)
    assert np.array_equal(Xr.cpu().numpy(), X[rows]) and np.array_equal(Tr.cpu().numpy(), T[rows])
    sim.close(); sc.close()


def test_learned_step_zero_network_is_coarse_stepping():
    import paper_2108_08919_amd as P
    L = 32
    p = wl.Params(L=float(L), zeta=0.03, K=0.04)
    s0 = random_state(L, 22, amp_u=3e-3)
    sim = P.Sim([p], [L * L])
    sim.set_state(0, s0)
    m = P.Mlp()
    m.set_weights(np.zeros(m.nparams, dtype=np.float32))
    m.set_norm(IDENT)
    nfb, mx = sim.step_learned(m, 5, 4, 1.0)
    sim.check()
    g = sim.get_state(0)
    c, sc = gpu_run(p.replace(dt=4 * p.dt), s0, 5)
    e = field_errors(g, c, s0, L)
    print(e, flush=True)
    assert nfb == 0 and mx == 0.0
    assert e["u"] < 1e-5 and e["Q"] < 1e-6 and e["rho"] < 1e-9 and e["pos_abs_max"] < 1e-7
    sim.close(); sc.close(); m.close()


def test_learned_step_fallback_is_fine_stepping():
    import paper_2108_08919_amd as P
    L = 32
    p = wl.Params(L=float(L), zeta=0.03, K=0.04)
    s0 = random_state(L, 23, amp_u=3e-3)
    sim = P.Sim([p], [L * L])
    sim.set_state(0, s0)
    m = P.Mlp()
    m.set_weights(ref.flatten(ref.init(5)).astype(np.float32))
    m.set_norm(IDENT)
    nfb, mx = sim.step_learned(m, 3, 4, 1e-30)
    sim.check()
    assert nfb == 3
    g = sim.get_state(0)
    f, sf = gpu_run(p, s0, 12)
    e = field_errors(g, f, s0, L)
    print(e, flush=True)
    assert e["u"] < 1e-5 and e["Q"] < 1e-6 and e["pos_abs_max"] < 1e-7
    sim.close(); sf.close(); m.close()


def _train_small(mult, epochs=12):
    from paper_2108_08919_amd import learned
    X, T = learned.training_set(side=64, replicas=8, times=(0.1, 0.2, 0.3), per_replica=4096, seed=0, mult=mult)
    m, loss = learned.fit(X, T, epochs=epochs, batch=1024, lr=3e-3)
    Xh, Th = learned.training_set(side=64, replicas=4, times=(0.15, 0.25), per_replica=None, seed=1, mult=mult)
    return m, loss, Xh, Th


@pytest.mark.parametrize("mult", [4, 16])
def test_trained_network_predicts_q_and_u_corrections(mult):
    """A network trained by the library's kernels on solver samples (boxes
    advanced by uncorrected macro steps) predicts the (mult fine steps) -
    (one mult*dt step) difference on held-out boxes of other seeds and
    activity/elasticity draws: the Q part from the local fields, the velocity
    part from the step's change of acceleration (the lagged predictor's
    error). Components without held-out skill would be switched off and
    return exactly zero."""
    from paper_2108_08919_amd import learned
    m, loss, Xh, Th = _train_small(mult)
    rel = learned.held_out_errors(m, Xh, Th)
    print("mult", mult, "held-out relative MSE", [round(v, 4) for v in rel], "loss", loss, flush=True)
    assert max(rel[:3]) < 0.1
    assert max(rel[3:]) < 0.5
    masked = learned.mask_unskilled(m, [r if o != 4 else 1.5 for o, r in enumerate(rel)])
    assert masked == [4]
    Y = m.forward(Xh).cpu().numpy()
    assert np.all(Y[:, 4] == 0.0)
    rel2 = learned.held_out_errors(m, Xh, Th)
    for o in range(4):
        assert rel2[o] == pytest.approx(rel[o], rel=1e-6)
    assert rel2[4] >= 1.0 - 1e-9   # a zero correction cannot beat the target's mean
    m.close()


def test_fallback_threshold_trips_out_of_distribution():
    """tau = 1.5 x the largest correction norm on held-out boxes: learned macro
    steps on a box of the training distribution never fall back; on a box with
    an activity ten times the training range the corrections go beyond tau and
    those macro steps are replayed as fine steps (the tanh layers bound how far
    the outputs can go, so not every macro step needs to trip)."""
    import paper_2108_08919_amd as P
    from paper_2108_08919_amd import learned
    m, loss, Xh, Th = _train_small(4)
    learned.mask_unskilled(m, learned.held_out_errors(m, Xh, Th))
    tau = learned.fallback_threshold(m, Xh)
    L = 64
    s0 = wl.initial_state(L, 1.0, 1.0, seed=77, kind="isotropic")
    for zeta, expect_fallback in ((0.02, False), (0.4, True)):
        p = wl.Params(L=float(L), zeta=zeta, K=0.04)
        sim = P.Sim([p], [L * L])
        sim.set_state(0, s0)
        sim.step(100)                      # develop a flow first
        mid = sim.get_state(0)
        nfb, mx = sim.step_learned(m, 3, 4, tau)
        sim.check()
        print("zeta", zeta, "tau", tau, "largest norm", mx, "fallbacks", nfb, flush=True)
        if expect_fallback:
            assert nfb >= 1 and mx > tau
        else:
            assert nfb == 0 and mx <= tau
        sim.close()
    m.close()


@pytest.mark.parametrize("mult", [16, 64])
def test_large_multipliers_zero_net_fallback_and_gain(mult):
    """At 16 and 64 x dt: a network of zeros gives plain mult*dt stepping, a
    forced fallback gives mult plain dt steps, and a trained network applied
    over macro steps on held-out boxes leaves smaller Q and u errors against
    the fine run than plain mult*dt stepping."""
    import paper_2108_08919_amd as P
    from paper_2108_08919_amd import learned
    L = 48
    p = wl.Params(L=float(L), zeta=0.03, K=0.04)
    s0 = random_state(L, 31, amp_u=3e-3)
    # zero network: coarse stepping
    sim = P.Sim([p], [L * L])
    sim.set_state(0, s0)
    z = learned.zero_network()
    nfb, mx = sim.step_learned(z, 2, mult, 1.0)
    g = sim.get_state(0)
    c, sc = gpu_run(p.replace(dt=mult * p.dt), s0, 2)
    e = field_errors(g, c, s0, L)
    print("zero net", mult, e, flush=True)
    assert nfb == 0 and e["u"] < 1e-5 and e["Q"] < 1e-6 and e["pos_abs_max"] < 1e-7
    sim.close(); sc.close()
    # forced fallback (a network that always corrects, tau below any norm): fine stepping
    sim = P.Sim([p], [L * L])
    sim.set_state(0, s0)
    rnd = P.Mlp()
    rnd.set_weights(ref.flatten(ref.init(5)).astype(np.float32))
    rnd.set_norm(IDENT)
    nfb, _ = sim.step_learned(rnd, 1, mult, 1e-30)
    g = sim.get_state(0)
    f, sf = gpu_run(p, s0, mult)
    e = field_errors(g, f, s0, L)
    print("fallback", mult, e, flush=True)
    assert nfb == 1 and e["u"] < 1e-5 and e["Q"] < 1e-6 and e["pos_abs_max"] < 1e-7
    sim.close(); sf.close(); rnd.close()
    # trained network against plain coarse stepping on held-out boxes
    m, loss, Xh, Th = _train_small(mult)
    rel = learned.held_out_errors(m, Xh, Th)
    learned.mask_unskilled(m, rel)
    tau = learned.fallback_threshold(m, Xh)
    print("mult", mult, "held-out relative MSE", [round(v, 4) for v in rel], "tau", tau, flush=True)
    n_macro = max(2, 96 // mult)
    gains = {"q": [], "u": []}
    for seed in (40, 41):
        q = wl.Params(L=64.0, zeta=0.02, K=0.03)
        st = wl.initial_state(64, 1.0, 1.0, seed=seed, kind="isotropic")
        # the start: uncorrected macro steps to t ~ 0.2, as a learned run gets there
        pre = P.Sim([q], [64 * 64]); pre.set_state(0, st); pre.step_learned(z, max(1, 200 // mult), mult)
        mid = pre.get_state(0); pre.close()
        fine, sfi = gpu_run(q, mid, n_macro * mult)
        co, sco = gpu_run(q.replace(dt=mult * q.dt), mid, n_macro)
        ls = P.Sim([q], [64 * 64]); ls.set_state(0, mid)
        nfb, _ = ls.step_learned(m, n_macro, mult, tau)
        ls.check()
        le = ls.get_state(0); ls.close(); sco.close(); sfi.close()
        dq = lambda a: np.concatenate([a["qxx"] - fine["qxx"], a["qxy"] - fine["qxy"]])
        du = lambda a: np.concatenate([a["ux"] - fine["ux"], a["uy"] - fine["uy"]])
        gains["q"].append(np.linalg.norm(dq(co)) / np.linalg.norm(dq(le)))
        gains["u"].append(np.linalg.norm(du(co)) / np.linalg.norm(du(le)))
        print("seed", seed, "fallbacks", nfb, "Q error coarse/learned", gains["q"][-1],
              "u error coarse/learned", gains["u"][-1], flush=True)
        assert nfb == 0
    assert min(gains["q"]) > 1.5 and min(gains["u"]) > 1.2
    m.close(); z.close()
