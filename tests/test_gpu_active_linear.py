"""Extensile against contractile activity in the linear regime of the isotropic
state, on batched replicas: four 64x64 boxes from one weakly ordered random
start (q0 = 0.01, director angles seeded), zeta = +-0.02 and lambda = +-0.7,
dt = 0.01, 2,000 steps.

Linear theory of the isotropic state (Sec. 2, D = Q + I/2) couples each Q
shear mode to the flow it drives with the product lambda zeta k^2 / (2 rho0):
the flow feeds the order when lambda zeta > 0 and damps it when lambda zeta <
0, and the map (lambda, zeta) -> (-lambda, -zeta) flips u and keeps Q. So the
velocity scale must be larger for lambda zeta > 0 whatever the sign of lambda,
and equal for the mirrored pairs. The GPU's V_rms samples are checked against
the FP64 oracle for lambda = 0.7 (both signs of zeta)."""
import math

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

SIDE, Q0, DT, STEPS, EVERY = 64, 0.01, 0.01, 2000, 500
CASES = ((0.02, 0.7), (-0.02, 0.7), (0.02, -0.7), (-0.02, -0.7))


def _params(zeta, lam):
    return wl.Params(L=float(SIDE), zeta=zeta, lam=lam, dt=DT)


def _start():
    return wl.initial_state(SIDE, 1.0, 1.0, 1000, "isotropic", q0=Q0)


def _oracle_series(zeta, lam):
    import oracle
    st = oracle.State(_start())
    out = []
    for _ in range(STEPS // EVERY):
        oracle.step(_params(zeta, lam), st, EVERY)
        out.append(math.sqrt(2.0 * oracle.diagnostics(_params(zeta, lam), st)["ke"]))
    return np.array(out)


def test_velocity_scale_ordered_by_sign_of_lambda_zeta():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_08919_amd as P
    sim = P.Sim([_params(z, l) for z, l in CASES], [SIDE * SIDE] * len(CASES))
    s0 = _start()
    for r in range(len(CASES)):
        sim.set_state(r, s0)
    gpu = np.zeros((len(CASES), STEPS // EVERY))
    for s in range(STEPS // EVERY):
        sim.step(EVERY)
        sim.check()
        for r in range(len(CASES)):
            gpu[r, s] = sim.vrms(r)
    sim.close()
    for (z, l), v in zip(CASES, gpu):
        print(f"zeta {z:+.2f} lambda {l:+.1f}: V_rms", " ".join(f"{x:.6e}" for x in v), flush=True)
    for r in (0, 1):
        orc = _oracle_series(*CASES[r])
        rel = np.abs(gpu[r] - orc) / orc
        print(f"case {CASES[r]}: oracle", " ".join(f"{x:.6e}" for x in orc), f"largest rel. deviation {rel.max():.2e}",
              flush=True)
        assert rel.max() < 1e-5
    ext_pos, con_pos, ext_neg, con_neg = gpu[:, -1]
    print(f"lambda zeta > 0 over < 0: {ext_pos / con_pos:.4f} (lambda > 0), {con_neg / ext_neg:.4f} (lambda < 0)")
    assert ext_pos > 1.05 * con_pos             # lambda > 0: extensile above contractile
    assert con_neg > 1.05 * ext_neg             # lambda < 0: contractile above extensile
    np.testing.assert_allclose(gpu[3], gpu[0], rtol=1e-3)   # mirrored pairs
    np.testing.assert_allclose(gpu[2], gpu[1], rtol=1e-3)
