"""Pins of the individual rate terms of the oracle's step (paper Sec. 3 and 3.1),
each against a closed form or a continuum limit that the term reaches at its
known order, on the periodic square lattice (dx = 1, h = 1.3 dx unless stated).

* Pressure force (Eq. sphMomentum, first term, with Eq. sphEos and
  c0 = 10 max|u|): a uniform drift U fixes c0 = 10 U without entering any
  gradient; on the density wave rho0 (1 + eps cos kx) the acceleration tends
  to -dp/dx / rho = c0^2 eps k sin kx, with error falling as (kh)^2.
* Continuity (Eq. sphContinuity): u = (U sin kx, 0) gives the rate
  k -> -rho U k cos kx at second order.
* Viscous term (Eq. sphMomentum, second term, factor 8 eta): a shear wave
  u_x = A sin ky is an eigenfunction. Its eigenvalue equals the closed-form
  lattice symbol 8 nu V b sum_s W'(s) s_x^2 (1 - cos k s_y) / s^3 (b = 1/alpha,
  Eq. sphCorrectionMatrix), whose long-wave limit c(h/dx) (-nu k^2) tends to
  -nu k^2 as the kernel spans more particles: c = 0.940 at h = 1.3 dx (the
  lattice's fourth moment of W' is not the integral's), 0.9993 at h = 4 dx.
* Density filter (Eq. densityCorrection, beta = 1, self term included):
  the lattice symbol V (W(0) + sum_s W(s) cos k s_x) multiplies a density
  wave exactly, and 1 - symbol -> k^2 mu2 / 2 (mu2 = int x^2 W) as k -> 0;
  leaving out the self term would give 1.22 times that.
* APD (Eq. APD): one particle displaced by d along x on the lattice, moving
  with U along y while every other particle rests, is pushed by
  r0^2 U (1 - W(0) V) dt (-d/2) sum_s s^-3 to first order in d
  (linear response of sum_j r_ij / r^3 about the lattice site).
* lambda stress (Eq. elasticstress): the literal matrix products reduce in
  2D (Cayley-Hamilton) to lam (2 (Q:H) Q - H); for Q = (A cos kx, 0) at
  rest the stress divergence adds -lam (A_L + K k^2) A k sin kx / rho to
  the x acceleration, at second order.

Sign, factor and self-term mistakes in any of these terms change the
leading coefficient, so each fails its pin.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle
import workloads as wl

H = 1.3
LS = (64, 128, 256)


def w_quintic(r, h):
    """Quintic spline of Eq. quintic (2D normalisation 7 / (478 pi h^2))."""
    q = np.asarray(r, dtype=np.float64) / h
    t = lambda m: np.clip(m - q, 0.0, None)
    return 7.0 / (478.0 * math.pi * h * h) * (t(3) ** 5 - 6 * t(2) ** 5 + 15 * t(1) ** 5)


def dw_quintic(r, h):
    q = np.asarray(r, dtype=np.float64) / h
    t = lambda m: np.clip(m - q, 0.0, None)
    return -5.0 * 7.0 / (478.0 * math.pi * h ** 3) * (t(3) ** 4 - 6 * t(2) ** 4 + 15 * t(1) ** 4)


def lattice_offsets(R):
    """Lattice vectors s != 0 with |s| < R."""
    m = int(math.ceil(R)) + 1
    i = np.arange(-m, m + 1, dtype=np.float64)
    X, Y = np.meshgrid(i, i)
    X, Y = X.ravel(), Y.ravel()
    r = np.hypot(X, Y)
    sel = (r > 0) & (r < R)
    return X[sel], Y[sel], r[sel]


def rest_state(L):
    x, y = wl.lattice(L)
    n = x.size
    z = np.zeros(n)
    return dict(x=x, y=y, ux=z.copy(), uy=z.copy(), qxx=np.ones(n), qxy=z.copy(), rho=np.ones(n),
                ax=z.copy(), ay=z.copy())


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def second_order(errs):
    for a, b in zip(errs, errs[1:]):
        assert a / b == pytest.approx(4.0, rel=0.05), errs


@pytest.mark.parametrize("rho0", [1.0, 2.0])
def test_pressure_force_continuum_limit(rho0):
    U, eps = 0.01, 1e-6
    c0 = 10.0 * U
    errs = []
    for L in LS:
        s = rest_state(L)
        k = 2 * math.pi / L
        s["ux"] = np.full(L * L, U)
        s["rho"] = rho0 * (1.0 + eps * np.cos(k * s["x"]))
        f = oracle.step_fields(wl.Params(L=float(L), zeta=0.0, K=0.0, rho0=rho0), oracle.State(s))
        assert f["k"].max() == 0.0 and f["k"].min() == 0.0   # uniform drift: no compression
        expect = c0 * c0 * eps * k * np.sin(k * s["x"])
        errs.append(rel_max(f["a"][:, 0], expect))
        assert np.abs(f["a"][:, 1]).max() < 1e-12 * np.abs(expect).max()
    assert errs[0] < 1e-2
    second_order(errs)


@pytest.mark.parametrize("rho0", [1.0, 2.0])
def test_continuity_rate_continuum_limit(rho0):
    U = 1e-3
    errs = []
    for L in LS:
        s = rest_state(L)
        k = 2 * math.pi / L
        s["ux"] = U * np.sin(k * s["x"])
        s["rho"] = np.full(L * L, rho0)
        f = oracle.step_fields(wl.Params(L=float(L), zeta=0.0, K=0.0, rho0=rho0), oracle.State(s))
        errs.append(rel_max(f["k"], -rho0 * U * k * np.cos(k * s["x"])))
    assert errs[0] < 5e-3
    second_order(errs)


@pytest.mark.parametrize("h,L,rho0", [(1.3, 64, 1.0), (1.3, 128, 2.0), (2.0, 128, 1.0), (2.6, 128, 1.0),
                                       (4.0, 256, 1.0)])
def test_viscous_shear_wave_eigenvalue(h, L, rho0):
    A = 1e-6
    s = rest_state(L)
    k = 2 * math.pi / L
    s["ux"] = A * np.sin(k * s["y"])
    s["rho"] = np.full(L * L, rho0)
    p = wl.Params(L=float(L), h=h, zeta=0.0, K=0.0, apd=0, rho0=rho0)
    f = oracle.step_fields(p, oracle.State(s))
    lam = np.dot(f["a"][:, 0], s["ux"]) / np.dot(s["ux"], s["ux"])
    assert np.abs(f["a"][:, 0] - lam * s["ux"]).max() < 1e-10 * np.abs(f["a"][:, 0]).max()
    sx, sy, r = lattice_offsets(3 * h)
    dW = dw_quintic(r, h)
    V = 1.0 / (w_quintic(0.0, h) + w_quintic(r, h).sum())
    b = 1.0 / (-V * (dW * sx * sx / r).sum())          # alpha = (1/b) I on the lattice
    nu = p.eta / p.rho0
    symbol = 8.0 * nu * V * b * (dW * sx * sx * (1.0 - np.cos(k * sy)) / r ** 3).sum()
    assert lam == pytest.approx(symbol, rel=1e-11)
    c = -4.0 * V * b * (dW * sx * sx * sy * sy / r ** 3).sum()   # long-wave limit / (-nu k^2)
    assert lam / (-nu * k * k) == pytest.approx(c, rel=2.5 * (k * h) ** 2)
    # the limit approaches the continuum value 1 as h/dx grows
    assert {1.3: 0.93, 2.0: 0.985, 2.6: 0.995, 4.0: 0.999}[h] < c < 1.0


def test_density_filter_lattice_symbol():
    eps = 1e-6
    W0 = w_quintic(0.0, H)
    sx, _, r = lattice_offsets(3 * H)
    Ws = w_quintic(r, H)
    V = 1.0 / (W0 + Ws.sum())
    mu2 = 0.5 * quad(lambda q: 2 * math.pi * q ** 3 * w_quintic(q, H), 0.0, 3 * H)[0]   # int x^2 W d^2r
    ratios = []
    for L in LS:
        s = rest_state(L)
        k = 2 * math.pi / L
        s["rho"] = 1.0 + eps * np.cos(k * s["x"])
        f = oracle.step_fields(wl.Params(L=float(L), zeta=0.0, K=0.0), oracle.State(s))
        symbol = V * (W0 + (Ws * np.cos(k * sx)).sum())
        assert np.abs(f["rho_hat"] - (1.0 + eps * symbol * np.cos(k * s["x"]))).max() < 1e-9 * eps
        ratios.append((1.0 - symbol) / (0.5 * k * k * mu2))
    assert abs(ratios[-1] - 1.0) < 2e-3
    assert abs(ratios[0] - 1.0) > abs(ratios[-1] - 1.0)


@pytest.mark.parametrize("d", [2e-3, 1e-3, 5e-4])
def test_apd_single_displaced_particle(d):
    L, U = 16, 1e-3
    s = rest_state(L)
    i = 8 * L + 8
    s["x"][i] += d
    s["uy"][i] = U
    p = wl.Params(L=float(L), zeta=0.0, K=0.0)
    f = oracle.step_fields(p, oracle.State(s))
    _, _, r = lattice_offsets(3 * H)
    V = 1.0 / (w_quintic(0.0, H) + w_quintic(r, H).sum())
    r0 = r.mean()
    expect = r0 ** 2 * U * (1.0 - w_quintic(0.0, H) * V) * p.dt * (-0.5 * d * (r ** -3.0).sum())
    got = f["dr_apd"][i, 0]
    assert got == pytest.approx(expect, rel=5.0 * d * d)
    # particles outside the moving particle's support have u_v = 0 and stay put
    far = np.hypot(s["x"] - s["x"][i], s["y"] - s["y"][i]) > 3 * H + 0.01
    assert far.sum() > 100 and np.abs(f["dr_apd"][far]).max() == 0.0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_elastic_stress_reduces_in_two_dimensions(seed):
    rng = np.random.default_rng(seed)
    a, b, c, e = rng.normal(size=4)
    Q = np.array([[a, b], [b, -a]])
    Hm = np.array([[c, e], [e, -c]])
    lam = 0.7
    Pi = oracle.elastic_stress(lam, Q, Hm)
    assert np.abs(Pi - lam * (2.0 * np.sum(Q * Hm) * Q - Hm)).max() < 1e-14 * (1 + np.abs(Pi).max())


@pytest.mark.parametrize("AL,K,rho0", [(0.05, 0.0, 1.0), (0.0, 1.0, 1.0), (0.05, 0.0, 2.0)])
def test_elastic_stress_divergence_continuum_limit(AL, K, rho0):
    A = 1e-4
    errs = []
    for L in LS:
        s = rest_state(L)
        k = 2 * math.pi / L
        s["qxx"] = A * np.cos(k * s["x"])
        s["rho"] = np.full(L * L, rho0)
        p = wl.Params(L=float(L), zeta=0.0, K=K, A=AL, C=0.0, elastic=1, rho0=rho0)
        f1 = oracle.step_fields(p, oracle.State(s))
        f0 = oracle.step_fields(p.replace(elastic=0), oracle.State(s))
        d = f1["a"][:, 0] - f0["a"][:, 0]
        errs.append(rel_max(d, -p.lam * (AL + K * k * k) * A * k * np.sin(k * s["x"]) / rho0))
        assert np.abs(f1["a"][:, 1] - f0["a"][:, 1]).max() < 1e-12 * np.abs(d).max()
    assert errs[0] < 1e-2
    second_order(errs)
