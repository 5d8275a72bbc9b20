"""GPU diagnostics against the oracle: FP64 reductions (momentum, kinetic
energy, free energy), Shepard deposit, kinetic-energy spectrum and +-1/2
defect counts."""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import diag
import workloads as wl

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import gpu_run, random_state, run_oracle  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_08919_amd as P
    P.lib()
    yield


def test_reductions_match_oracle():
    L = 32
    p = wl.Params(L=float(L), zeta=0.03, K=0.05)
    s0 = random_state(L, 11, amp_u=3e-3)
    o, ost = run_oracle(p, s0, 5)
    g, sim = gpu_run(p, s0, 5)
    dg = sim.diagnostics(0)
    do = oracle.diagnostics(p, ost)
    print({k: (dg.get(k), do.get(k)) for k in ("px", "py", "ke", "F", "F_grad", "umax")}, flush=True)
    m = p.rho0 * p.dx ** 2
    scale = m * np.hypot(o["ux"], o["uy"]).sum()
    assert abs(dg["px"] - do["px"]) <= 1e-6 * scale and abs(dg["py"] - do["py"]) <= 1e-6 * scale
    assert dg["ke"] == pytest.approx(do["ke"], rel=1e-5)
    assert dg["umax"] == pytest.approx(do["umax"], rel=1e-5)
    assert dg["F"] == pytest.approx(do["F"], rel=1e-5)
    assert dg["F_grad"] == pytest.approx(do["F_grad"], rel=1e-5)
    assert dg["qmax"] == pytest.approx(math.sqrt(2.0) * np.hypot(o["qxx"], o["qxy"]).max(), rel=1e-6)
    sim.close()


def test_free_energy_monotone_gpu():
    L = 32
    p = wl.Params(L=float(L), zeta=0.0, K=0.05)
    st = wl.initial_state(L, 1.0, 1.0, seed=5, kind="isotropic")
    import paper_2108_08919_amd as P
    sim = P.Sim([p], [L * L])
    sim.set_state(0, st)
    F = [sim.diagnostics(0)["F"]]
    for _ in range(20):
        sim.step(1)
        F.append(sim.diagnostics(0)["F"])
    F = np.array(F)
    assert np.all(F[1:] <= F[:-1] * (1 + 1e-6))
    assert F[-1] < F[0]
    sim.close()


def test_deposit_matches_oracle():
    L = 32
    p = wl.Params(L=float(L), zeta=0.03)
    s0 = random_state(L, 12, amp_u=3e-3)
    g, sim = gpu_run(p, s0, 3)
    G = sim.deposit(0, 32)
    O = oracle.deposit(p, g["x"], g["y"], [g["ux"], g["uy"], g["qxx"], g["qxy"]], 32)
    for f in range(4):
        err = np.abs(G[f] - O[f]).max() / np.abs(O[f]).max()
        assert err < 1e-5, (f, err)
    sim.close()


def test_spectrum_matches_oracle():
    L = 64
    p = wl.Params(L=float(L), zeta=0.03)
    s0 = random_state(L, 13, amp_u=3e-3)
    g, sim = gpu_run(p, s0, 2)
    E, sl = sim.spectrum(0, 64)
    # FFT and shell sums: GPU against numpy on the GPU's own deposit grid
    G = sim.deposit(0, 64)
    Eg = diag.spectrum_from_grid(G[0], G[1], nbins=E.size)
    assert np.allclose(E, Eg, rtol=1e-9, atol=1e-14 * Eg.sum())
    assert E.sum() == pytest.approx(0.5 * np.mean(G[0] ** 2 + G[1] ** 2), rel=1e-9)
    # whole pipeline against the FP64 oracle deposit of the same particles
    Eo, slo = diag.spectrum(p, g["x"], g["y"], g["ux"], g["uy"], 64)
    big = Eo[:E.size] > 1e-6 * Eo.max()
    assert np.allclose(E[big], Eo[:E.size][big], rtol=1e-4)
    assert sl == pytest.approx(slo, abs=1e-4)
    sim.close()


def test_single_mode_spectrum():
    L = 64
    p = wl.Params(L=float(L), zeta=0.0, K=0.0, eta=0.0, apd=0)
    x, y = wl.lattice(L)
    n = x.size
    z = np.zeros(n)
    m = 3
    ux = 1e-3 * np.sin(2 * math.pi * m * y / L)
    st = dict(x=x, y=y, ux=ux, uy=z, qxx=np.ones(n), qxy=z, rho=np.ones(n), ax=z, ay=z)
    import paper_2108_08919_amd as P
    sim = P.Sim([p], [n])
    sim.set_state(0, st)
    E, _ = sim.spectrum(0, 64)
    assert E[m] > 0.999 * E.sum()
    sim.close()


def test_defects_match_oracle_on_gpu_grid():
    L = 64
    p = wl.Params(L=float(L), zeta=0.03)
    s0 = wl.initial_state(L, 1.0, 1.0, seed=3, kind="isotropic")
    g, sim = gpu_run(p, s0, 2)
    n_plus, n_minus = sim.defects(0, 64)
    G = sim.deposit(0, 64)
    op, om, _ = diag.defects_from_grid(G[2], G[3])
    assert (n_plus, n_minus) == (op, om)
    assert n_plus == n_minus            # zero total charge on a torus
    sim.close()


def test_defects_analytic_pair():
    L = 64
    p = wl.Params(L=float(L))
    x, y = wl.lattice(L)
    th = 0.5 * np.arctan2(y - 30.2, x - 20.7) - 0.5 * np.arctan2(y - 33.9, x - 44.3)
    n = x.size
    z = np.zeros(n)
    st = dict(x=x, y=y, ux=z, uy=z, qxx=np.cos(2 * th), qxy=np.sin(2 * th), rho=np.ones(n), ax=z, ay=z)
    import paper_2108_08919_amd as P
    sim = P.Sim([p], [n])
    sim.set_state(0, st)
    assert sim.defects(0, 64) == (1, 1)
    sim.close()
