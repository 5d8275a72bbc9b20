"""GPU parity of the quasi-2D variant (3x3 order tensor, printed I/3) against
the FP64 oracle: fields over 10 steps, uniform relaxation, diagnostics,
deposit, state I/O of Qyy and the rules around the variant."""
import math
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as wl

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import check_increments, field_errors, rel_l2, run_oracle  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_08919_amd as P
    P.lib()
    yield


def _state(L, seed, amp_u=2e-3):
    x, y = wl.jittered_lattice(L, 1.0, 0.2, seed)
    n = x.size
    rng = np.random.default_rng(seed + 11)
    qxx, qxy, qyy, qzz = wl.order_tensor3(rng.uniform(0, math.pi, n), rng.uniform(0.6, 1.0, n))
    ux, uy = wl.smooth_velocity(x, y, float(L), amp_u, seed)
    return dict(x=x, y=y, ux=ux, uy=uy, qxx=qxx, qxy=qxy, qyy=qyy, qzz=qzz,
                rho=1.0 + 1e-4 * rng.normal(size=n), ax=np.zeros(n), ay=np.zeros(n))


def _gpu(p, s0, nsteps, opts=None):
    import paper_2108_08919_amd as P
    sim = P.Sim([p], [s0["x"].size])
    for k, v in (opts or {}).items():
        sim.set_option(k, v)
    sim.set_state(0, s0)
    if nsteps:
        sim.step(nsteps)
    sim.check()
    return sim.get_state(0), sim


@pytest.mark.parametrize("seed,tile,kernel", [(0, 4, 0), (1, 8, 0), (2, 8, 1)])
def test_ten_steps_match_oracle(seed, tile, kernel):
    import paper_2108_08919_amd as P
    L = 40
    p = wl.Params(L=float(L), zeta=0.03, K=0.04, B=0.3, q3d=1, kernel=kernel)
    s0 = _state(L, seed)
    print("quasi-2D 10 steps", seed, tile, kernel, flush=True)
    o, _ = run_oracle(p, s0, 10)
    g, sim = _gpu(p, s0, 10, {P.NEM_OPT_TILE: tile})
    e = field_errors(g, o, s0, L, 10)
    e["Qyy"] = rel_l2(g["qyy"], o["qyy"])
    e["dQyy"] = rel_l2(g["qyy"] - s0["qyy"], o["qyy"] - s0["qyy"])
    e["trace"] = float(np.abs(g["qxx"] + g["qyy"] + g["qzz"]).max())
    print({k: f"{v:.3e}" for k, v in e.items()}, flush=True)
    for k in ("u", "Q", "Qyy", "rho", "pos"):
        assert e[k] <= 1e-5, (k, e[k])
    check_increments(e)
    # Qyy's increment, in units of the FP32 resolution of Qyy per step
    res = np.abs((g["qyy"] - s0["qyy"]) - (o["qyy"] - s0["qyy"])).max() / (10 * 2.0 ** -24 * np.abs(o["qyy"]).max())
    assert res <= 4.0, res
    assert np.abs(o["qxx"] + o["qyy"] + o["qzz"]).max() < 1e-13   # oracle keeps Qzz on its own
    sim.close()


def test_uniform_uniaxial_relaxation():
    L, S0, theta = 16, 1.5, 0.4
    A, B, C = -1.0, 0.5, 1.0
    p = wl.Params(L=float(L), A=A, B=B, C=C, zeta=0.02, q3d=1)
    x, y = wl.lattice(L)
    n = x.size
    qxx, qxy, qyy, qzz = wl.order_tensor3(np.full(n, theta), 2.0 * S0 / 3.0)
    s0 = dict(x=x, y=y, ux=np.zeros(n), uy=np.zeros(n), qxx=qxx, qxy=qxy, qyy=qyy, qzz=qzz,
              rho=np.ones(n), ax=np.zeros(n), ay=np.zeros(n))
    g, sim = _gpu(p, s0, 50)
    S = S0
    for _ in range(50):
        S = S + p.dt * p.Gamma * (-A * S + B * S * S / 3.0 - 2.0 * C * S ** 3 / 3.0)
    c, s = math.cos(theta), math.sin(theta)
    assert np.abs(g["qxx"] - S * (c * c - 1 / 3)).max() < 2e-6
    assert np.abs(g["qxy"] - S * c * s).max() < 2e-6
    assert np.abs(g["qyy"] - S * (s * s - 1 / 3)).max() < 2e-6
    assert np.all(g["ux"] == 0.0)
    d = sim.diagnostics(0)
    assert d["qmax"] == pytest.approx(S * math.sqrt(2.0 / 3.0), rel=1e-5)
    sim.close()


def test_diagnostics_and_deposit():
    L = 32
    p = wl.Params(L=float(L), zeta=0.03, K=0.05, B=0.2, q3d=1)
    s0 = _state(L, 4)
    o, ost = run_oracle(p, s0, 5)
    g, sim = _gpu(p, s0, 5)
    dg, do = sim.diagnostics(0), oracle.diagnostics(p, ost)
    assert dg["F"] == pytest.approx(do["F"], rel=1e-5)
    assert dg["F_grad"] == pytest.approx(do["F_grad"], rel=1e-5)
    assert dg["ke"] == pytest.approx(do["ke"], rel=1e-5)
    G = sim.deposit(0, 32)
    O = oracle.deposit(p, g["x"], g["y"], [g["ux"], g["uy"], 0.5 * (g["qxx"] - g["qyy"]), g["qxy"]], 32)
    for f in range(4):
        assert np.abs(G[f] - O[f]).max() <= 1e-5 * np.abs(O[f]).max(), f
    sim.close()


def test_qyy_io_and_snapshot_restore():
    import paper_2108_08919_amd as P
    L = 32
    p = wl.Params(L=float(L), zeta=0.03, q3d=1)
    s0 = _state(L, 5)
    g, sim = _gpu(p, s0, 0)
    assert np.abs(g["qyy"] - s0["qyy"]).max() < 1e-7           # FP32 storage
    sim.step(5)
    sim.autotune(2)                                             # trial steps from a snapshot, restored
    sim.step(5)
    g = sim.get_state(0)
    o, _ = run_oracle(p, s0, 10)
    assert rel_l2(g["qyy"], o["qyy"]) < 1e-5
    sim.close()


def test_variant_rules():
    import paper_2108_08919_amd as P
    L = 32
    s0 = _state(L, 6)
    g, sim = _gpu(wl.Params(L=float(L)), s0, 0)                 # d = 2 simulation
    with pytest.raises(P.NemError):
        sim.set_qyy(0, s0["qyy"])
    sim.close()
    with pytest.raises(P.NemError):
        P.Sim([wl.Params(L=float(L), q3d=1, form=1)], [s0["x"].size])
