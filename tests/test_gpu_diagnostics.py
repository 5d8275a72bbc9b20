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


def _smooth_velocity(L, x, y, seed, nmax=4, amp=1e-3):
    """Sum of random Fourier modes with |n| <= nmax: a field with a finite
    vorticity correlation length."""
    rng = np.random.default_rng(seed)
    ux = np.zeros_like(x)
    uy = np.zeros_like(x)
    for nx in range(-nmax, nmax + 1):
        for ny in range(0, nmax + 1):
            if (nx, ny) == (0, 0):
                continue
            ph = 2 * math.pi * (nx * x + ny * y) / L
            a, b, c, d = rng.normal(size=4)
            ux += a * np.cos(ph) + b * np.sin(ph)
            uy += c * np.cos(ph) + d * np.sin(ph)
    s = amp / np.sqrt(np.mean(ux ** 2 + uy ** 2))
    return ux * s, uy * s


def test_vorticity_correlation_matches_oracle():
    L = 64
    p = wl.Params(L=float(L), zeta=0.03)
    x, y = wl.lattice(L)
    n = x.size
    rng = np.random.default_rng(14)
    x = (x + 0.05 * rng.uniform(-1, 1, n)) % L
    y = (y + 0.05 * rng.uniform(-1, 1, n)) % L
    ux, uy = _smooth_velocity(L, x, y, 15)
    th = rng.uniform(0, math.pi, n)
    z = np.zeros(n)
    st = dict(x=x, y=y, ux=ux, uy=uy, qxx=np.cos(2 * th), qxy=np.sin(2 * th), rho=np.ones(n), ax=z, ay=z)
    import paper_2108_08919_amd as P
    sim = P.Sim([p], [n])
    sim.set_state(0, st)
    sim.step(2)
    g = sim.get_state(0)
    for M in (32, 64):
        cx, cy, lx, ly = sim.vorticity_correlation(0, M)
        assert cx.size == M // 2 + 1 and cx[0] == 1.0 and cy[0] == 1.0
        # FFTs and axes: GPU against numpy on the GPU's own deposit grid
        G = sim.deposit(0, M)
        ex, ey, mx, my = diag.vorticity_correlation_from_grid(G[0], G[1], float(L))
        assert np.abs(cx - ex).max() < 1e-9 and np.abs(cy - ey).max() < 1e-9
        assert (lx, ly) == pytest.approx((mx, my), abs=1e-7)
        # whole pipeline against the FP64 oracle deposit of the same particles
        ox, oy, olx, oly = diag.vorticity_correlation(p, g["x"], g["y"], g["ux"], g["uy"], M)
        print(M, lx, olx, ly, oly, np.abs(cx - ox).max(), np.abs(cy - oy).max(), flush=True)
        assert np.abs(cx - ox).max() < 1e-5 and np.abs(cy - oy).max() < 1e-5
        assert lx > 0 and ly > 0
        assert (lx, ly) == pytest.approx((olx, oly), rel=1e-4)
    sim.close()


def test_vorticity_correlation_single_mode():
    L = 64
    p = wl.Params(L=float(L), zeta=0.0, K=0.0, eta=0.0, apd=0)
    x, y = wl.lattice(L)
    n = x.size
    z = np.zeros(n)
    m = 2
    uy = 1e-3 * np.sin(2 * math.pi * m * x / L)
    st = dict(x=x, y=y, ux=z, uy=uy, qxx=np.ones(n), qxy=z, rho=np.ones(n), ax=z, ay=z)
    import paper_2108_08919_amd as P
    sim = P.Sim([p], [n])
    sim.set_state(0, st)
    cx, cy, lx, ly = sim.vorticity_correlation(0, 64)
    k = np.arange(33)
    assert np.abs(cx - np.cos(2 * math.pi * m * k / 64)).max() < 1e-6
    assert np.abs(cy - 1.0).max() < 1e-6
    assert lx == pytest.approx(L / (4 * m), rel=1e-6)
    assert ly == -1.0
    # a field with no vorticity has no normalised correlation
    st["uy"] = z
    sim.set_state(0, st)
    cx, cy, lx, ly = sim.vorticity_correlation(0, 64)
    assert np.isnan(cx).all() and np.isnan(lx)
    assert sim.vrms(0) == 0.0
    sim.close()
