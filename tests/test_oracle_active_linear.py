"""Pin of the active / flow-alignment coupling in the oracle against the linear
theory of the isotropic state (Sec. 2: Eqs. nematodynamic, corotation,
activestress and the momentum balance; 2x2 Q with D = Q + I/2).

Around Q = 0, u = 0 the co-rotation term is S = lambda E to first order (the
vorticity terms cancel against D = I/2 and the Q:grad u term is second order),
so a single shear mode Qxy = q(t) sin(kx) with the flow it drives,
u_y = v(t) cos(kx), obeys two linear equations:
    dq/dt = -Gamma K k^2 q - (lambda k / 2) v     (E_xy = -(k/2) v sin kx)
    dv/dt = -(zeta k / rho0) q - (eta k^2 / rho0) v  (the active force -zeta div Q)
The flow is transverse (div u = 0), so pressure and density stay out of it.
The product of the two couplings is lambda zeta k^2 / (2 rho0): when lambda
zeta > 0 the flow feeds the order that drives it, when lambda zeta < 0 it
damps it. With the paper's lambda = 0.7 this makes extensile activity
(zeta > 0) sustain larger flows than contractile activity of the same
magnitude; the map (lambda, zeta) -> (-lambda, -zeta) leaves q unchanged and
flips v. The oracle, run from rest with a small Qxy mode, must follow the
closed-form solution exp(M t) of this 2x2 system, converging with k h."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
import workloads as wl

EPS, DT, T = 1e-4, 0.05, 20.0


def _run(L, zeta, lam):
    """Projections of Qxy on sin(kx) and of u_y on cos(kx) at t = T, in units
    of the initial amplitude; and the closed-form values."""
    x, y = wl.lattice(L)
    n = x.size
    k = 2 * math.pi / L
    st = oracle.State(dict(x=x, y=y, ux=np.zeros(n), uy=np.zeros(n), qxx=np.zeros(n), qxy=EPS * np.sin(k * x),
                           rho=np.ones(n), ax=np.zeros(n), ay=np.zeros(n)))
    p = wl.Params(L=float(L), zeta=zeta, lam=lam, apd=0, dt=DT)
    oracle.step(p, st, int(round(T / DT)))
    f = st.fields()
    q = 2 * np.mean(f["qxy"] * np.sin(k * x)) / EPS
    v = 2 * np.mean(f["uy"] * np.cos(k * x)) / EPS
    M = np.array([[-p.Gamma * p.K * k * k, -lam * k / 2],
                  [-zeta * k / p.rho0, -p.eta * k * k / p.rho0]])
    qe, ve = expm(M * T) @ np.array([1.0, 0.0])
    return q, v, qe, ve


def _errors(L, zeta, lam):
    q, v, qe, ve = _run(L, zeta, lam)
    # the change of q is the coupled part; compare it, not q itself
    return abs((q - 1.0) / (qe - 1.0) - 1.0), abs(v / ve - 1.0), q, v, qe


@pytest.mark.parametrize("zeta", [0.2, -0.2])
def test_single_mode_follows_linear_theory(zeta):
    e64q, e64v, q, v, qe = _errors(64, zeta, 0.7)
    print(f"zeta {zeta}: q {q:.6f} (closed form {qe:.6f}), v {v:.6f}; errors {e64q:.2e} {e64v:.2e}")
    assert e64q < 0.01 and e64v < 0.003
    if zeta > 0:
        # the discretisation error shrinks as k h does (second order plus the
        # corrector's first order in dt)
        e32q, _, _, _, _ = _errors(32, zeta, 0.7)
        assert e32q > 2.0 * e64q


def test_growth_is_ordered_by_sign_of_lambda_zeta():
    qe, ve, _, _ = _run(64, 0.2, 0.7)       # extensile, lambda > 0
    qc, vc, _, _ = _run(64, -0.2, 0.7)      # contractile, lambda > 0
    qm, vm, _, _ = _run(64, -0.2, -0.7)     # contractile, lambda < 0
    assert qe > 1.1 and qc < 0.9            # fed against damped
    assert abs(ve) > abs(vc)
    assert qm == pytest.approx(qe, rel=1e-9) and vm == pytest.approx(-ve, rel=1e-9)
