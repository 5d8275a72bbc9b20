"""GPU parity of the Wendland C2 kernel variant (support 2h) against the FP64
oracle: bit-exact neighbour sets, 10-step fields in every launch variant and
both momentum forms, the Shepard deposit, and the replica rules."""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as wl

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import check_increments, field_errors, gpu_run, random_state, run_oracle  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_08919_amd as P
    P.lib()
    yield


def _rows(rp, col):
    return [tuple(col[rp[i]:rp[i + 1]].tolist()) for i in range(rp.size - 1)]


def _check(e):
    print({k: f"{v:.3e}" for k, v in e.items()}, flush=True)
    for k in ("u", "Q", "rho", "pos"):
        assert e[k] <= TOL, (k, e[k])
    check_increments(e)


# L = 20: Wendland cells (side >= 2h + skin) hold 8.2 lattice particles, within
# the LDS staging capacity of 10 per cell (a 16^2 lattice would put 10.2 in each)
@pytest.mark.parametrize("kind,L,seed", [("lattice", 20, 0), ("jitter", 24, 1), ("uniform", 24, 3)])
def test_neighbors_bit_exact(kind, L, seed):
    import paper_2108_08919_amd as P
    p = wl.Params(L=float(L), kernel=1)
    if kind == "lattice":
        x, y = wl.lattice(L)
    elif kind == "jitter":
        x, y = wl.jittered_lattice(L, 1.0, 0.4, seed)
    else:
        x, y = wl.uniform_positions(L * L, float(L), seed)
    n = x.size
    z = np.zeros(n)
    print("neighbors", kind, L, seed, flush=True)
    sim = P.Sim([p], [n])
    sim.set_state(0, dict(x=x, y=y, ux=z, uy=z, qxx=np.ones(n), qxy=z, rho=np.ones(n), ax=z, ay=z))
    rp, col = sim.neighbors(0)
    sim.check()
    nc = int(np.floor(L / (2 * p.h + p.skin)))
    orp, ocol = oracle.neighbors(p, x, y, 2, nc)
    assert _rows(rp, col) == _rows(orp, ocol)
    if kind == "lattice":
        assert np.all(np.diff(rp) == 20)
    sim.close()


@pytest.mark.parametrize("seed,opts", [(0, {}), (1, {"tile": 8}), (2, {"lpp": 2}), (3, {"comp": 2}),
                                       (4, {"tile": 8, "lpp": 4})])
def test_random_state_ten_steps(seed, opts):
    import paper_2108_08919_amd as P
    keymap = {"comp": P.NEM_OPT_COMP, "tile": P.NEM_OPT_TILE, "lpp": P.NEM_OPT_LPP}
    L = 40
    p = wl.Params(L=float(L), zeta=0.03, K=0.04, kernel=1)
    s0 = random_state(L, seed, amp_u=2e-3)
    print("wendland 10 steps", seed, opts, flush=True)
    o, _ = run_oracle(p, s0, 10)
    g, sim = gpu_run(p, s0, 10, {keymap[k]: v for k, v in opts.items()})
    _check(field_errors(g, o, s0, L, 10))
    sim.close()


def test_full_size_ten_steps_tile8():
    """The 2048 x 2048 box with the Wendland kernel (cells of side 2.70, 7.3
    particles each) in the launch configuration that `bench.py --kernel
    wendland --tile 8` times, 10 steps against the oracle."""
    import paper_2108_08919_amd as P
    cfg = wl.config("C4")
    p = cfg["params"].replace(kernel=1)
    s0 = wl.state_for(cfg, 0)
    s0["ux"], s0["uy"] = wl.smooth_velocity(s0["x"], s0["y"], p.L, 1e-3, 7)
    print("oracle 10 steps at 4.2M particles, Wendland", flush=True)
    o, _ = run_oracle(p, s0, 10)
    g, sim = gpu_run(p, s0, 10, {P.NEM_OPT_TILE: 8})
    _check(field_errors(g, o, s0, p.L, 10))
    sim.close()


@pytest.mark.parametrize("form,elastic", [(1, 0), (0, 1)])
def test_forms(form, elastic):
    L = 32
    p = wl.Params(L=float(L), zeta=0.05, form=form, elastic=elastic, K=0.05, kernel=1)
    s0 = random_state(L, 5, amp_u=2e-3)
    print("wendland form", form, "elastic", elastic, flush=True)
    o, _ = run_oracle(p, s0, 10)
    g, sim = gpu_run(p, s0, 10)
    _check(field_errors(g, o, s0, L, 10))
    sim.close()


def test_c1_lattice_and_diagnostics():
    cfg = wl.config("C1")
    p = cfg["params"].replace(kernel=1)
    s0 = wl.state_for(cfg, 0)
    o, ost = run_oracle(p, s0, 10)
    g, sim = gpu_run(p, s0, 10)
    _check(field_errors(g, o, s0, p.L, 10))
    dg, do = sim.diagnostics(0), oracle.diagnostics(p, ost)
    assert dg["ke"] == pytest.approx(do["ke"], rel=1e-5)
    assert dg["F"] == pytest.approx(do["F"], rel=1e-5)
    G = sim.deposit(0, 64)
    O = oracle.deposit(p, g["x"], g["y"], [g["ux"], g["uy"], g["qxx"], g["qxy"]], 64)
    for f in range(4):
        assert np.abs(G[f] - O[f]).max() <= 1e-5 * np.abs(O[f]).max(), f
    sim.close()
