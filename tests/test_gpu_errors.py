"""Error paths of the GPU library that the kernels detect themselves: an
over-full cell (more particles than a cell's staging capacity of 48) is
reported as NEM_E_OVERFLOW by the step that meets it, and the error is sticky.
The kernels cap their loops at the capacity, so every access stays in bounds."""
import os
import sys

import numpy as np
import pytest

import workloads as wl

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


def test_overfull_cell_reports_overflow():
    import paper_2108_08919_amd as P
    L = 32                                   # 8 x 8 cells of side 4 (3h + skin = 4.0)
    p = wl.Params(L=float(L), zeta=0.0, K=0.02)
    s0 = random_state(L, 5, amp_u=0.0)
    rng = np.random.default_rng(11)
    idx = rng.choice(L * L, 60, replace=False)
    s0["x"][idx] = rng.uniform(8.2, 11.8, 60)   # 60 particles inside the cell [8, 12)^2
    s0["y"][idx] = rng.uniform(8.2, 11.8, 60)
    sim = P.Sim([p], [L * L])
    sim.set_state(0, s0)
    sim.step(1)
    with pytest.raises(P.NemError) as e:
        sim.check()
    assert e.value.code == P.NEM_E_OVERFLOW
    sim.step(1)                              # sticky: still reported
    with pytest.raises(P.NemError) as e:
        sim.check()
    assert e.value.code == P.NEM_E_OVERFLOW
    sim.close()


def test_regular_state_after_overflow_in_another_simulation():
    """An overflow in one simulation does not leak into a fresh one."""
    import paper_2108_08919_amd as P
    L = 32
    p = wl.Params(L=float(L), zeta=0.01, K=0.02)
    sim = P.Sim([p], [L * L])
    sim.set_state(0, random_state(L, 6))
    sim.step(3)
    sim.check()
    sim.close()


def test_isolated_particles_report_singular_and_match_oracle():
    """Degenerate case of Eq. sphCorrectionMatrix: particles with no neighbour
    within 3h have alpha = 0. Both sides fall back to B = I; the GPU raises the
    sticky NEM_E_SINGULAR, and the fields (u carried unchanged, Q relaxing by
    its bulk term only) still match the oracle."""
    import ctypes as C
    import oracle
    import paper_2108_08919_amd as P
    from gpu_common import field_errors, run_oracle
    L = 32
    g = (np.arange(4) * 8.0 + 4.0)
    X, Y = np.meshgrid(g, g, indexing="xy")
    x, y = X.ravel().copy(), Y.ravel().copy()          # 16 particles 8 apart: no pair within 3h
    n = x.size
    rng = np.random.default_rng(3)
    th = rng.uniform(0, np.pi, n)
    s0 = dict(x=x, y=y, ux=1e-3 * rng.normal(size=n), uy=1e-3 * rng.normal(size=n), qxx=np.cos(2 * th),
              qxy=np.sin(2 * th), rho=np.ones(n), ax=np.zeros(n), ay=np.zeros(n))
    p = wl.Params(L=float(L), zeta=0.02)
    sim = P.Sim([p], [n])
    sim.set_state(0, s0)
    sim.step(3)
    assert sim.sync() == P.NEM_E_SINGULAR
    out = {k: np.zeros(n) for k in ("x", "y", "ux", "uy", "qxx", "qxy", "rho", "ax", "ay")}
    rc = P.lib().nem_get_state(C.c_void_p(sim.h), 0, *[out[k].ctypes.data_as(C.POINTER(C.c_double))
                                                     for k in ("x", "y", "ux", "uy", "qxx", "qxy", "rho", "ax", "ay")])
    assert rc == P.NEM_E_SINGULAR                         # sticky, the state is still returned
    o, _ = run_oracle(p, s0, 3)
    e = field_errors(out, o, s0, L)
    print({k: f"{v:.3e}" for k, v in e.items()}, flush=True)
    for k in ("u", "Q", "rho", "pos"):
        assert e[k] <= 1e-6, (k, e[k])
    assert np.allclose(out["ux"], s0["ux"], rtol=0, atol=1e-9)   # no force without neighbours
    sim.close()


def test_duplicated_particle_matches_oracle():
    """A duplicated particle: one particle replaced by an exact copy of its
    neighbour (position, velocity, Q, density), leaving a hole. The neighbour
    predicate 0 < r^2 < R^2 keeps the pair out of every sum (no division by
    r = 0), so both copies see the same neighbours in the same order, move
    identically and stay exactly coincident; the fields match the oracle over
    ten steps with no error status. (A pair that separates from coincidence is
    another matter: its direction is below the FP32 offsets' resolution, and
    the APD sum of r_ij / r^3 grows without limit as r -> 0, as Eq. APD is
    printed; no test runs that regime.)"""
    import paper_2108_08919_amd as P
    from gpu_common import check_increments, field_errors, gpu_run, run_oracle
    L = 24
    p = wl.Params(L=float(L), zeta=0.02)
    s0 = random_state(L, 9, amp_u=2e-3)
    i, j = 10 * L + 10, 10 * L + 11
    for k in ("x", "y", "ux", "uy", "qxx", "qxy", "rho"):
        s0[k][i] = s0[k][j]
    o, _ = run_oracle(p, s0, 10)
    g, sim = gpu_run(p, s0, 10)
    assert sim.sync() == P.NEM_OK
    e = field_errors(g, o, s0, L, 10)
    print({k: f"{v:.3e}" for k, v in e.items()}, flush=True)
    for k in ("u", "Q", "rho", "pos"):
        assert e[k] <= 1e-5, (k, e[k])
    check_increments(e)
    for k in ("x", "y", "ux", "uy", "qxx", "qxy", "rho"):
        assert g[k][i] == g[k][j] and o[k][i] == o[k][j], k
    sim.close()
