"""Pins of the two correctors of Sec. 3.1 in the oracle.

A shear wave u_x = A sin(k y) on the lattice is an eigenfunction of the
discrete viscous operator, divergence-free (the density stays exactly rho0, so
the pressure vanishes) and, at zeta = 0, decoupled from Q: the velocity obeys
du/dt = lambda u with the operator's eigenvalue lambda. So
* each corrector must reproduce its own scalar recurrence exactly (with
  lambda read off the first acceleration), which pins the update formulas;
* against the exact solution u = exp(lambda t), x - x0 = (exp(lambda t) - 1)/lambda
  the kick-drift-kick reading (lagged predictor a^{n-1/2}) converges at first
  order and the midpoint reading (u^n + a dt, r^n + u^{n+1/2} dt) at second
  order in dt, for velocity and position alike."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl

L, M_MODE, AMP = 32, 8, 1e-6


def _run(integ, dt, steps):
    x, y = wl.lattice(L)
    n = x.size
    k = 2 * math.pi * M_MODE / L
    p = wl.Params(L=float(L), zeta=0.0, K=0.0, apd=0, dt=dt, integrator=integ)
    st = oracle.State(dict(x=x, y=y, ux=AMP * np.sin(k * y), uy=np.zeros(n), qxx=np.ones(n), qxy=np.zeros(n),
                           rho=np.ones(n), ax=np.zeros(n), ay=np.zeros(n)))
    oracle.step(p, st, steps)
    f = st.fields()
    i = int(np.argmax(np.sin(k * y)))
    s = AMP * math.sin(k * y[i])
    return f["ux"][i] / s, (f["x"][i] - x[i]) / s, f["ax"][i] / s, f


def _lambda():
    return _run(0, 0.05, 1)[2]


@pytest.mark.parametrize("integ", [0, 1])
def test_corrector_follows_its_recurrence(integ):
    lam, dt, N = _lambda(), 0.05, 20
    u, ap = 1.0, 0.0
    for _ in range(N):
        uh = u + 0.5 * dt * ap          # predictor with the last acceleration
        a = lam * uh
        u = uh + 0.5 * dt * a if integ == 0 else u + dt * a
        ap = a
    r, _, _, f = _run(integ, dt, N)
    assert r == pytest.approx(u, rel=1e-10)
    assert np.abs(f["rho"] - 1.0).max() == 0.0 and np.abs(f["uy"]).max() < 1e-8 * AMP


def test_convergence_orders():
    lam, T = _lambda(), 1.0
    assert -2.0 < lam < -1.0           # about -nu k^2 for k = pi/2
    exact_u, exact_x = math.exp(lam * T), (math.exp(lam * T) - 1.0) / lam
    for integ, order in ((0, 1), (1, 2)):
        eu, ex = [], []
        for dt in (0.05, 0.025, 0.0125):
            u, xd, _, _ = _run(integ, dt, int(round(T / dt)))
            eu.append(abs(u - exact_u))
            ex.append(abs(xd - exact_x))
        for e in (eu, ex):
            for a, b in zip(e, e[1:]):
                assert a / b == pytest.approx(2.0 ** order, rel=0.08), (integ, e)
