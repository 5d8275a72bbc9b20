"""Invariants of the oracle's full time step (CPU only).

* total momentum is conserved to rounding by the conservative pair forces;
* Q stays symmetric and traceless;
* a uniform aligned nematic at rest stays at rest, uniform and aligned, with its
  magnitude following the scalar explicit-Euler recurrence of dq/dt =
  -Gamma (A + 2 C q^2) q (exact closed form of the ODE within O(dt));
* at zeta = 0 on the lattice the free energy decays monotonically;
* the density filter leaves a uniform density unchanged;
* the APD displacement vanishes on a perfect lattice.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl


def random_state(L, seed, amp_u=1e-3, jitter=0.2):
    x, y = wl.jittered_lattice(L, 1.0, jitter, seed)
    ux, uy = wl.smooth_velocity(x, y, float(L), amp_u, seed)
    th = wl.director_angles(x.size, seed, "isotropic")
    qxx, qxy = wl.order_tensor(th)
    rng = np.random.default_rng(seed + 7)
    return dict(x=x, y=y, ux=ux, uy=uy, qxx=qxx, qxy=qxy,
                rho=1.0 + 1e-4 * rng.normal(size=x.size), ax=np.zeros_like(x), ay=np.zeros_like(x))


@pytest.mark.parametrize("elastic", [0, 1])
def test_momentum_conserved_conservative_form(elastic):
    L = 20
    p = wl.Params(L=float(L), form=1, elastic=elastic, zeta=0.05)
    s = oracle.State(random_state(L, 3))
    m = p.rho0 * p.dx ** 2
    P0 = np.array([m * s.ux.sum(), m * s.uy.sum()])
    scale = m * np.hypot(s.ux, s.uy).sum()
    for _ in range(5):
        oracle.step(p, s, 1)
        P = np.array([m * s.ux.sum(), m * s.uy.sum()])
        assert np.abs(P - P0).max() <= 1e-13 * scale
    assert np.abs(s.ux).max() > 0


def test_q_symmetric_traceless():
    L = 20
    p = wl.Params(L=float(L), zeta=0.05)
    s = oracle.State(random_state(L, 4))
    oracle.step(p, s, 10)
    d = oracle.diagnostics(p, s)
    assert d["trq_max"] <= 1e-14 and d["asym_max"] <= 1e-14


@pytest.mark.parametrize("A,C", [(0.0, 0.5), (1.0, 0.0), (-1.0, 0.5), (0.3, 0.2)])
def test_uniform_aligned_nematic_at_rest(A, C):
    cfg = wl.config("C1")
    p = cfg["params"].replace(A=A, C=C)
    st = wl.state_for(cfg)
    st["qxx"] = np.ones_like(st["qxx"]); st["qxy"] = np.zeros_like(st["qxy"])
    s = oracle.State(st)
    x0, y0 = s.x.copy(), s.y.copy()
    nsteps = 100
    oracle.step(p, s, nsteps)
    assert np.all(s.ux == 0) and np.all(s.uy == 0)
    assert np.all(s.x == x0) and np.all(s.y == y0)
    assert np.all(s.rho == p.rho0)
    q = s.q[:, 0]
    assert np.ptp(q) == 0.0 and np.all(s.q[:, 1] == 0) and np.all(s.q[:, 2] == 0)
    qn = 1.0
    for _ in range(nsteps):                  # explicit Euler of dq/dt = -Gamma (A + 2 C q^2) q
        qn = qn * (1.0 - p.dt * p.Gamma * (A + 2 * C * qn * qn))
    assert q[0] == pytest.approx(qn, rel=1e-14)
    t = nsteps * p.dt
    if A == 0.0:
        exact = 1.0 / math.sqrt(1.0 + 4 * p.Gamma * C * t)
    else:
        e = math.exp(-2 * p.Gamma * A * t)
        exact = math.sqrt(A * e / (A + 2 * C * (1 - e)))
    assert abs(q[0] - exact) < 2 * p.dt * p.Gamma * (abs(A) + 2 * C) * t + 1e-12
    if A == -1.0 and C == 0.5:
        assert q[0] == 1.0                   # q = 1 is an exact fixed point
    if (A, C) == (0.0, 0.5):
        assert q[0] == pytest.approx(0.967626039103667, rel=1e-13)


def test_free_energy_monotone_at_zero_activity():
    L = 32
    p = wl.Params(L=float(L), zeta=0.0, K=0.05)
    st = wl.initial_state(L, 1.0, 1.0, seed=5, kind="isotropic")
    s = oracle.State(st)
    F = [oracle.diagnostics(p, s)["F"]]
    for _ in range(30):
        oracle.step(p, s, 1)
        assert np.all(s.ux == 0)
        F.append(oracle.diagnostics(p, s)["F"])
    F = np.array(F)
    assert np.all(F[1:] <= F[:-1] * (1 + 1e-14))
    assert F[-1] < F[0]


def test_density_filter_uniform():
    L = 16
    p = wl.Params(L=float(L))
    st = wl.initial_state(L, 1.0, 1.0, seed=1, kind="isotropic")
    st["rho"] = np.full(L * L, 1.0 + 3e-6)
    s = oracle.State(st)
    f = oracle.step_fields(p, s)
    # u = 0 so k = 0 and rho^{n+1/2} is uniform; the filter must return it
    assert np.abs(f["rho_hat"] - (1.0 + 3e-6)).max() < 1e-15


def test_apd_zero_on_lattice():
    L = 16
    p = wl.Params(L=float(L))
    x, y = wl.lattice(L)
    ux, uy = wl.smooth_velocity(x, y, float(L), 1e-3, 2)
    # place r^n so that the projected configuration r^{n+1/2} is the lattice
    x0 = np.mod(x - 0.5 * ux * p.dt, L); y0 = np.mod(y - 0.5 * uy * p.dt, L)
    st = dict(x=x0, y=y0, ux=ux, uy=uy, qxx=np.ones(L * L), qxy=np.zeros(L * L),
              rho=np.ones(L * L), ax=np.zeros(L * L), ay=np.zeros(L * L))
    f = oracle.step_fields(p, oracle.State(st))
    # scale of an uncancelled displacement: r0^2 u_v dt sum 1/r^2
    assert np.abs(f["dr_apd"]).max() < 1e-12 * (9.0 * 1e-3 * p.dt * 10.0)


def test_forms_agree_at_rest():
    cfg = wl.config("C1")
    st = wl.state_for(cfg)
    s0 = oracle.State(st); s1 = oracle.State(st)
    oracle.step(cfg["params"], s0, 3)
    oracle.step(cfg["params"].replace(form=1), s1, 1)
    # first step: u = 0 so form only changes the active term's discretisation;
    # both produce the same sign pattern of the first acceleration
    assert np.corrcoef(s0.ax, s1.ax)[0, 1] > 0.9


def _first_active_acceleration(L, zeta, A=0.1):
    x, y = wl.lattice(L)
    n = x.size
    k = 2 * math.pi / L
    st = dict(x=x, y=y, ux=np.zeros(n), uy=np.zeros(n), qxx=A * np.cos(k * x), qxy=np.zeros(n),
              rho=np.ones(n), ax=np.zeros(n), ay=np.zeros(n))
    s1 = oracle.State(st)
    oracle.step(wl.Params(L=float(L), zeta=zeta, K=0.02, apd=0), s1, 1)
    return s1.ax, s1.ay, zeta * A * k * np.sin(k * x), abs(zeta) * A * k


@pytest.mark.parametrize("zeta", [0.02, -0.02])
def test_active_force_is_minus_zeta_div_q(zeta):
    """From rest with uniform density the only force of the first step is the
    active one, -(zeta/rho) div Q (Eq. activestress in the momentum balance).
    Q = (A cos kx, 0) gives a_x = zeta A k sin(kx), a_y = 0: extensile
    (zeta > 0) and contractile (zeta < 0) activity push in opposite directions,
    the force is linear in zeta, and the SPH sum converges to the continuum
    value at second order in k h."""
    err = []
    for L in (32, 64):
        ax, ay, exact, scale = _first_active_acceleration(L, zeta)
        assert np.abs(ay).max() < 1e-12 * scale
        err.append(np.abs(ax - exact).max() / scale)
    assert err[1] < 5e-3
    assert 3.8 < err[0] / err[1] < 4.2
    ax2, _, _, scale = _first_active_acceleration(64, 2 * zeta)
    assert np.abs(ax2 - 2 * ax).max() < 1e-13 * scale
