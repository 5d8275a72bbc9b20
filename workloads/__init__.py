"""Seeded synthetic inputs for the SPH active-nematic solver.

This module produces *data only*: particle positions on a square lattice, seeded
director angles, initial fields, and the parameter sets of the standard
workloads. It holds none of the method's arithmetic, so both the FP64 CPU oracle
(test infrastructure) and the HIP library can take their inputs from here
without sharing any code with each other.

Initial condition (paper Sec. 5, text after Table 2): zero velocity and a
slightly perturbed (or fully random) director field; particles start on a
square lattice of spacing dx. The 2D order tensor for a director angle theta and
magnitude q (Sec. 2, definition of Q with d = 2) is
q * [[cos 2theta, sin 2theta], [sin 2theta, -cos 2theta]].
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Params:
    """Physical and numerical parameters of one box (one replica).

    Paper symbols: Table 2 (Gamma, lambda, A, B, C, K, mu, rho, zeta), Eq. quintic
    (h, support 3h; the Wendland C2 variant has support 2h), Eq. sphEos (gamma = 7, c0 = 10 max|u|), Eq. densityCorrection
    (beta = 1). dx is the lattice spacing, L the periodic box side.
    """

    L: float = 64.0
    dx: float = 1.0
    h: float = 1.3
    rho0: float = 1.0
    eta: float = 1.0
    Gamma: float = 0.34
    lam: float = 0.7
    A: float = 0.0
    B: float = 0.0
    C: float = 0.5
    K: float = 0.02
    zeta: float = 0.01
    dt: float = 1e-3
    gamma_eos: float = 7.0
    beta: float = 1.0
    c0_factor: float = 10.0
    skin: float = 0.1
    form: int = 0      # 0: corrected (B-contracted) momentum, 1: conservative pair forces
    elastic: int = 0   # 0: reduced stress (Eq. mainstress), 1: plus lambda terms of Eq. elasticstress
    apd: int = 1       # artificial particle displacement on/off
    kernel: int = 0    # smoothing kernel: 0 quintic spline (support 3h), 1 Wendland C2 (support 2h)
    integrator: int = 0  # corrector: 0 kick-drift-kick, 1 midpoint (u^n + a dt)
    q3d: int = 0       # 0: 2x2 Q (d = 2); 1: quasi-2D 3x3 Q with the printed I/3

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


def lattice(n_side: int, dx: float = 1.0):
    """Square lattice of n_side x n_side particles at ((i+1/2)dx, (j+1/2)dx).

    Particle id = j * n_side + i (x index fastest)."""
    i = np.arange(n_side, dtype=np.float64)
    X, Y = np.meshgrid((i + 0.5) * dx, (i + 0.5) * dx, indexing="xy")
    return X.ravel().copy(), Y.ravel().copy()


def director_angles(n: int, seed: int, kind: str) -> np.ndarray:
    """Seeded director angles: 'small' = U(-0.1, 0.1) about x, 'isotropic' = U[0, pi)."""
    rng = np.random.default_rng(seed)
    if kind == "small":
        return rng.uniform(-0.1, 0.1, size=n)
    if kind == "isotropic":
        return rng.uniform(0.0, math.pi, size=n)
    if kind == "aligned":
        return np.zeros(n)
    raise ValueError(kind)


def order_tensor(theta: np.ndarray, q0: float = 1.0):
    """(Qxx, Qxy) of the 2D order tensor for director angle theta, magnitude q0."""
    return q0 * np.cos(2.0 * theta), q0 * np.sin(2.0 * theta)


def order_tensor3(theta: np.ndarray, q0: float = 1.0):
    """(Qxx, Qxy, Qyy, Qzz) of the 3x3 order tensor Q = (3/2) q0 (n n - I/3) for
    an in-plane director at angle theta (the d = 3 form of the paper's Q)."""
    c, s = np.cos(theta), np.sin(theta)
    return (1.5 * q0 * (c * c - 1.0 / 3.0), 1.5 * q0 * c * s, 1.5 * q0 * (s * s - 1.0 / 3.0),
            -0.5 * q0 * np.ones_like(theta))


def initial_state(n_side: int, dx: float, rho0: float, seed: int, kind: str, q0: float = 1.0) -> Dict[str, np.ndarray]:
    """Lattice positions, u = 0, rho = rho0, Q from seeded angles, a = 0 (id order)."""
    x, y = lattice(n_side, dx)
    n = x.size
    th = director_angles(n, seed, kind)
    qxx, qxy = order_tensor(th, q0)
    z = np.zeros(n)
    return dict(x=x, y=y, ux=z.copy(), uy=z.copy(), qxx=qxx, qxy=qxy,
                rho=np.full(n, rho0), ax=z.copy(), ay=z.copy())


def jittered_lattice(n_side: int, dx: float, amp: float, seed: int):
    """Lattice positions displaced by U(-amp, amp) per coordinate, wrapped into [0, L)."""
    rng = np.random.default_rng(seed)
    x, y = lattice(n_side, dx)
    L = n_side * dx
    x = np.mod(x + rng.uniform(-amp, amp, x.size), L)
    y = np.mod(y + rng.uniform(-amp, amp, y.size), L)
    return x, y


def uniform_positions(n: int, L: float, seed: int):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, L, n), rng.uniform(0.0, L, n)


def smooth_velocity(x, y, L, amp, seed):
    """A seeded smooth periodic velocity field (a few low Fourier modes)."""
    rng = np.random.default_rng(seed)
    ux = np.zeros_like(x)
    uy = np.zeros_like(y)
    for _ in range(4):
        kx, ky = rng.integers(-3, 4, size=2)
        ph = rng.uniform(0, 2 * math.pi, size=2)
        a = rng.normal(size=2) * amp
        arg = 2 * math.pi * (kx * x + ky * y) / L
        ux += a[0] * np.sin(arg + ph[0])
        uy += a[1] * np.sin(arg + ph[1])
    return ux, uy


# ---------------------------------------------------------------------------
# Standard workloads. Sizes and physics: lattice dx = 1, h = 1.3 dx, quintic
# kernel, rho0 = 1, eta = 1, Gamma = 0.34, lambda = 0.7, A = 0, C = 0.5.
# ---------------------------------------------------------------------------

def config(name: str) -> Dict:
    base = Params()
    if name == "C1":   # FP64-CPU-sized box: 64 x 64 lattice, director +-0.1 rad about x
        return dict(name=name, n_side=64, params=base.replace(L=64.0, zeta=0.01, K=0.02),
                    kind="small", steps=100)
    if name == "C2":   # single run at scale: 512 x 512, isotropic start
        return dict(name=name, n_side=512, params=base.replace(L=512.0, zeta=0.02, K=0.02),
                    kind="isotropic", steps=10000, diag_every=500)
    if name == "C4":   # large box: 2048 x 2048 = 4,194,304 particles
        return dict(name=name, n_side=2048, params=base.replace(L=2048.0, zeta=0.02, K=0.02),
                    kind="isotropic", steps=2000)
    if name == "C5eval":  # learned-corrector evaluation box 1024 x 1024
        return dict(name=name, n_side=1024, params=base.replace(L=1024.0, zeta=0.02, K=0.02),
                    kind="isotropic", steps=2000)
    raise ValueError(name)


def ensemble(seed: int = 0) -> List[Dict]:
    """32 replicas of uneven size: side ~ U{128..384} (seeded), zeta x K sweep x 2 seeds."""
    rng = np.random.default_rng(seed)
    zetas = [0.005, 0.01, 0.02, 0.04]
    Ks = [0.01, 0.02, 0.04, 0.08]
    reps = []
    r = 0
    for z in zetas:
        for k in Ks:
            for s in range(2):
                side = int(rng.integers(128, 385))
                reps.append(dict(name=f"R{r}", n_side=side,
                                 params=Params().replace(L=float(side), zeta=z, K=k),
                                 kind="isotropic", seed=1000 + r, steps=5000))
                r += 1
    return reps


def state_for(cfg: Dict, seed: int = 0) -> Dict[str, np.ndarray]:
    p: Params = cfg["params"]
    return initial_state(cfg["n_side"], p.dx, p.rho0, cfg.get("seed", seed), cfg["kind"])
