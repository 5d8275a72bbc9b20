"""Algebraic pins of the nematic terms in the oracle (Eqs. corotation,
molecularfield/molecularfielddis, sphEos) read with d = 2."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl


def Qof(theta, q=1.0):
    c, s = math.cos(2 * theta), math.sin(2 * theta)
    return q * np.array([[c, s], [s, -c]])


@pytest.mark.parametrize("theta", [0.0, 0.3, 1.1, 2.7])
@pytest.mark.parametrize("lam", [0.0, 0.7, -1.0])
def test_rigid_rotation_rotates_director(theta, lam):
    # u = omega (-y, x): G = omega [[0,-1],[1,0]] (G_ab = du_a/dx_b). A director
    # carried by a rigid rotation turns at d(theta)/dt = omega for any lambda.
    w = 0.37
    G = w * np.array([[0.0, -1.0], [1.0, 0.0]])
    S = oracle.corotation(lam, Qof(theta), G)
    dQ = (Qof(theta + 1e-6) - Qof(theta - 1e-6)) / 2e-6
    assert np.allclose(S, w * dQ, atol=1e-9)


@pytest.mark.parametrize("seed", range(5))
def test_corotation_trace_and_symmetry(seed):
    rng = np.random.default_rng(seed)
    lam = rng.uniform(-1, 1)
    a, b = rng.normal(size=2)
    Q = np.array([[a, b], [b, -a]])
    G = rng.normal(size=(2, 2))
    S = oracle.corotation(lam, Q, G)
    assert abs(S[0, 1] - S[1, 0]) < 1e-14
    # in d = 2: tr S = lam tr G exactly (Q symmetric traceless, D = Q + I/2)
    assert np.trace(S) == pytest.approx(lam * np.trace(G), abs=1e-13)


def test_corotation_isotropic_state_gives_lambda_E():
    E = np.array([[0.3, 0.1], [0.1, -0.3]])
    S = oracle.corotation(0.7, np.zeros((2, 2)), E)
    assert np.allclose(S, 0.7 * E, atol=1e-15)


@pytest.mark.parametrize("seed", range(3))
def test_molecular_field_2d(seed):
    rng = np.random.default_rng(seed)
    p = wl.Params(A=rng.normal(), B=rng.normal(), C=rng.uniform(0.1, 1), K=0.05)
    a, b = rng.normal(size=2)
    Q = np.array([[a, b], [b, -a]])
    lap = rng.normal(size=(2, 2)); lap = 0.5 * (lap + lap.T); lap -= 0.5 * np.trace(lap) * np.eye(2)
    H = oracle.molecular_field(p, Q, lap)
    q2 = a * a + b * b
    # 2D: Q^2 = (a^2+b^2) I so the B term vanishes; tr Q^2 = 2 q2
    expect = -(p.A + 2 * p.C * q2) * Q + p.K * lap
    assert np.allclose(H, expect, atol=1e-14)
    assert abs(np.trace(H)) < 1e-14


def test_eos():
    rho0, c0, g = 1.0, 0.3, 7.0
    assert oracle.eos(rho0, rho0, c0, g) == 0.0
    for x in [1e-7, -3e-5, 2e-3, 0.05]:
        binom = sum(math.comb(7, k) * x ** k for k in range(1, 8))   # (1+x)^7 - 1
        assert oracle.eos(rho0 * (1 + x), rho0, c0, g) == pytest.approx(rho0 * c0 * c0 / g * binom, rel=1e-9)


def test_paper_scales():
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
    t = gold["table2"]
    lq = math.sqrt(t["K"] / t["zeta"])
    vq = lq * t["zeta"] / t["Gamma"]
    Re = t["rho"] * vq * lq / t["mu"]
    assert Re == pytest.approx(gold["scales"]["Re_approx"], rel=1e-12)
