"""Pins of the oracle's SPH kernel, volumes and correction tensor (CPU only).

Sources of truth are not the oracle itself: the continuum normalisation
int W d^2r = 1 that a_d is chosen for (Eq. quintic), the polynomial's value at
b = 0, finite differences, the paper's "about 45 neighbours within 3h" for
h = 4/3 dx, and continuum moment identities of a normalised radial kernel.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads as wl

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


@pytest.mark.parametrize("h", [1.3, 4.0 / 3.0, 0.7])
def test_kernel_normalised(h):
    # int_0^{3h} W(r) 2 pi r dr = 1 (the role of a_d in Eq. quintic)
    pieces = [(0, h), (h, 2 * h), (2 * h, 3 * h)]
    tot = sum(integrate.quad(lambda r: oracle.W(h, r) * 2 * math.pi * r, a, b, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
              for a, b in pieces)
    assert abs(tot - 1.0) < 1e-12


@pytest.mark.parametrize("h", [1.3, 4.0 / 3.0])
def test_kernel_values(h):
    k = GOLD["kernel"]
    ad = k["a_d_2d_numerator"] / (k["a_d_2d_denominator_over_pi_h2"] * math.pi * h * h)
    # b = 0: 3^5 - 6 2^5 + 15 = 66
    assert oracle.W(h, 0.0) == pytest.approx(66 * ad, rel=1e-15)
    R = k["kappa"] * h
    assert oracle.W(h, R) == 0.0 and oracle.W(h, R * 1.0001) == 0.0
    assert oracle.dWdr(h, R) == 0.0
    # continuity at the break points b = 1, 2 and derivative by central differences
    for r in [0.3 * h, 0.999 * h, h, 1.5 * h, 2 * h, 2.5 * h, 2.99 * h]:
        e = 1e-6 * h
        fd = (oracle.W(h, r + e) - oracle.W(h, r - e)) / (2 * e)
        assert oracle.dWdr(h, r) == pytest.approx(fd, rel=1e-7, abs=1e-12)
    assert oracle.dWdr(h, 1e-9) == pytest.approx(0.0, abs=1e-9)


@pytest.mark.parametrize("hdx", [4.0 / 3.0, 1.3])
def test_lattice_neighbour_count(hdx):
    # Paper: with h = 4/3 dx there are about 45 neighbours within 3h.
    p = wl.Params(L=16.0, h=hdx)
    x, y = wl.lattice(16)
    rp, col = oracle.neighbors(p, x, y, 0)
    counts = np.diff(rp)
    assert np.all(counts == 44)         # 45 lattice sites including the particle itself
    assert counts[0] + 1 == GOLD["kernel"]["neighbours_approx"]


@pytest.mark.parametrize("hdx", [4.0 / 3.0, 1.3])
def test_lattice_volume_and_correction(hdx):
    p = wl.Params(L=16.0, h=hdx)
    x, y = wl.lattice(16)
    V, B, _, _ = oracle.operators(p, x, y)
    # a normalised kernel sums to ~1 on a unit lattice: V ~ dx^2
    assert np.all(np.abs(V - 1.0) < 1e-4)
    assert np.ptp(V) < 1e-14
    # correction tensor: alpha^{sl} = -sum V W'(r) r^s r^l / r ~ delta^{sl}
    # (second-moment identity of a normalised radial kernel); cubic symmetry
    # of the lattice makes it exactly isotropic.
    alpha = np.linalg.inv(B[0])
    assert abs(alpha[0, 1]) < 1e-15 and abs(alpha[1, 0]) < 1e-15
    assert alpha[0, 0] == pytest.approx(alpha[1, 1], rel=1e-14)
    assert abs(alpha[0, 0] - 1.0) < 2e-3


def test_lattice_sums_reference_values():
    # FP64 lattice sums for dx = 1, h = 1.3 (regression values of this oracle);
    # they follow from the pins above and fix the digits.
    p = wl.Params(L=16.0, h=1.3)
    x, y = wl.lattice(16)
    V, B, _, _ = oracle.operators(p, x, y)
    assert 1.0 / V[0] == pytest.approx(0.99995481865735, abs=1e-13)
    assert np.linalg.inv(B[0])[0, 0] == pytest.approx(1.00065312239676, abs=1e-13)
