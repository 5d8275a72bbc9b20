"""Pins of the quasi-2D variant in the oracle: a 3x3 order tensor in an in-plane
flow with the printed I/3 (Eqs. corotation, molecularfielddis).

Sources of truth: the uniaxial closed form of the molecular field
(Q = S (n n - I/3) gives Q^2 - tr(Q^2) I/3 = (S/3) Q and tr Q^2 = 2 S^2/3),
rigid rotation of the director, the trace identity tr S = (2 lambda/3) div u
that the I/3 implies (the d = 2 form gives lambda div u instead), the scalar
relaxation of a uniform uniaxial nematic at rest, and tracelessness."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl


def Q3(theta, S=1.0, phi=None):
    n = np.array([math.cos(theta), math.sin(theta), 0.0]) if phi is None else \
        np.array([math.sin(phi) * math.cos(theta), math.sin(phi) * math.sin(theta), math.cos(phi)])
    return S * (np.outer(n, n) - np.eye(3) / 3.0)


@pytest.mark.parametrize("theta,phi,S", [(0.3, None, 1.0), (1.2, 0.7, 0.6), (2.5, 2.0, -0.4)])
@pytest.mark.parametrize("A,B,C", [(0.0, 0.0, 0.5), (1.0, 0.3, 0.0), (-0.5, 0.8, 0.2)])
def test_molecular_field_uniaxial_closed_form(theta, phi, S, A, B, C):
    p = wl.Params(A=A, B=B, C=C, K=0.0)
    Q = Q3(theta, S, phi)
    H = oracle.molecular_field3(p, Q, np.zeros((3, 3)))
    assert np.allclose(H, (-A + B * S / 3.0 - C * 2.0 * S * S / 3.0) * Q, atol=1e-14)
    p = p.replace(K=0.7)
    L = np.arange(9.0).reshape(3, 3)
    assert np.allclose(oracle.molecular_field3(p, Q, L) - H, 0.7 * L, atol=1e-14)


@pytest.mark.parametrize("theta", [0.0, 0.4, 2.2])
@pytest.mark.parametrize("lam", [0.0, 0.7, -1.0])
def test_rigid_rotation_rotates_director(theta, lam):
    w = 0.37
    G = w * np.array([[0.0, -1.0], [1.0, 0.0]])
    S = oracle.corotation3(lam, Q3(theta, 0.8), G)
    dQ = (Q3(theta + 1e-6, 0.8) - Q3(theta - 1e-6, 0.8)) / 2e-6
    assert np.allclose(S, w * dQ, atol=1e-9)
    assert abs(S[2, 2]) < 1e-15


@pytest.mark.parametrize("seed", range(4))
def test_trace_of_corotation_is_two_thirds_lambda_div_u(seed):
    rng = np.random.default_rng(seed)
    lam = rng.uniform(-1, 1)
    M = rng.normal(size=(3, 3))
    M[0, 2] = M[2, 0] = M[1, 2] = M[2, 1] = 0.0
    Q = 0.5 * (M + M.T)
    Q -= np.trace(Q) / 3.0 * np.eye(3)
    G = rng.normal(size=(2, 2))
    S = oracle.corotation3(lam, Q, G)
    assert np.allclose(S, S.T, atol=1e-14)
    assert np.trace(S) == pytest.approx(2.0 * lam / 3.0 * np.trace(G), abs=1e-13)


def _uniform_state(L, theta, S0):
    x, y = wl.lattice(L)
    n = x.size
    qxx, qxy, qyy, qzz = wl.order_tensor3(np.full(n, theta), 2.0 * S0 / 3.0)
    return dict(x=x, y=y, ux=np.zeros(n), uy=np.zeros(n), qxx=qxx, qxy=qxy, qyy=qyy, qzz=qzz,
                rho=np.ones(n), ax=np.zeros(n), ay=np.zeros(n))


@pytest.mark.parametrize("A,B,C", [(0.0, 0.0, 0.5), (-1.0, 0.5, 1.0)])
def test_uniform_uniaxial_relaxation(A, B, C):
    """At rest and uniform, Q = S (n n - I/3) stays uniaxial and S follows the
    explicit Euler recurrence of dS/dt = Gamma (-A S + B S^2/3 - 2 C S^3/3)."""
    L, S0, theta = 16, 1.5, 0.4
    p = wl.Params(L=float(L), A=A, B=B, C=C, zeta=0.02, q3d=1)
    s = oracle.State(_uniform_state(L, theta, S0))
    S = S0
    for _ in range(50):
        S = S + p.dt * p.Gamma * (-A * S + B * S * S / 3.0 - 2.0 * C * S ** 3 / 3.0)
    oracle.step(p, s, 50)
    f = s.fields()
    ref = Q3(theta, S)
    assert np.abs(f["qxx"] - ref[0, 0]).max() < 1e-14 and np.abs(f["qxy"] - ref[0, 1]).max() < 1e-14
    assert np.abs(f["qyy"] - ref[1, 1]).max() < 1e-14 and np.abs(f["qzz"] - ref[2, 2]).max() < 1e-14
    assert np.all(f["ux"] == 0.0) and np.all(f["uy"] == 0.0)


def test_traceless_and_symmetric_under_flow():
    L = 24
    p = wl.Params(L=float(L), zeta=0.05, K=0.04, q3d=1)
    x, y = wl.jittered_lattice(L, 1.0, 0.2, seed=3)
    n = x.size
    rng = np.random.default_rng(3)
    qxx, qxy, qyy, qzz = wl.order_tensor3(rng.uniform(0, math.pi, n), 1.0)
    ux, uy = wl.smooth_velocity(x, y, float(L), 2e-3, 3)
    s = oracle.State(dict(x=x, y=y, ux=ux, uy=uy, qxx=qxx, qxy=qxy, qyy=qyy, qzz=qzz,
                          rho=1 + 1e-4 * rng.normal(size=n), ax=np.zeros(n), ay=np.zeros(n)))
    oracle.step(p, s, 10)
    f = s.fields()
    assert np.abs(f["qxx"] + f["qyy"] + f["qzz"]).max() < 1e-14
    assert np.abs(f["qxy"] - f["qyx"]).max() < 1e-15
    assert oracle.diagnostics(p, s)["trq_max"] < 1e-14
    assert np.abs(f["qzz"] - (-0.5)).max() > 1e-6          # Qzz evolves with the flow


def test_free_energy_monotone_at_zero_activity():
    L = 24
    p = wl.Params(L=float(L), zeta=0.0, K=0.05, q3d=1)
    x, y = wl.lattice(L)
    n = x.size
    qxx, qxy, qyy, qzz = wl.order_tensor3(np.random.default_rng(5).uniform(0, math.pi, n), 1.0)
    s = oracle.State(dict(x=x, y=y, ux=np.zeros(n), uy=np.zeros(n), qxx=qxx, qxy=qxy, qyy=qyy, qzz=qzz,
                          rho=np.ones(n), ax=np.zeros(n), ay=np.zeros(n)))
    F = [oracle.diagnostics(p, s)["F"]]
    for _ in range(20):
        oracle.step(p, s, 1)
        F.append(oracle.diagnostics(p, s)["F"])
    F = np.array(F)
    assert np.all(F[1:] <= F[:-1] * (1 + 1e-14)) and F[-1] < F[0]


def test_rejects_unsupported_combinations():
    x, y = wl.lattice(16)
    n = x.size
    st = dict(x=x, y=y, ux=np.zeros(n), uy=np.zeros(n), qxx=np.ones(n), qxy=np.zeros(n), rho=np.ones(n),
              ax=np.zeros(n), ay=np.zeros(n))
    with pytest.raises(RuntimeError):
        oracle.step(wl.Params(L=16.0, q3d=1), oracle.State(st), 1)          # no Qzz given
    st["qzz"] = np.zeros(n)
    with pytest.raises(RuntimeError):
        oracle.step(wl.Params(L=16.0, q3d=1, form=1), oracle.State(st), 1)
