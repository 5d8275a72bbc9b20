"""Long-run statistics of the single run at scale (512 x 512 lattice box,
262,144 particles, zeta = K = 0.02, isotropic start): the GPU runs the full
10,000 steps with the kinetic energy, the defect density and the spectrum
slope sampled every 500 steps; the FP64 oracle runs a shortened horizon of
2,000 steps (about 4 minutes on 16 host cores) and the samples they share must
agree within 2%. Runs only when NEM_LONG_TESTS=1 (it takes minutes)."""
import json
import os
import sys
import time

import numpy as np
import pytest

import oracle
from oracle import diag
import workloads as wl

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("NEM_LONG_TESTS") != "1", reason="set NEM_LONG_TESTS=1 to run")]


def _say(*a):
    print(*a, flush=True)


def test_c2_statistics_against_oracle_horizon():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_08919_amd as P
    cfg = wl.config("C2")
    p, side = cfg["params"], cfg["n_side"]
    s0 = wl.state_for(cfg, 0)
    every, n_gpu, n_orc = 500, cfg["steps"], 2000
    sim = P.Sim([p], [side * side])
    sim.set_state(0, s0)
    series = []
    t0 = time.perf_counter()
    for k in range(every, n_gpu + 1, every):
        sim.step(every)
        sim.check()
        pl, mi = sim.defects(0, side)
        _, slope = sim.spectrum(0, side)
        series.append(dict(step=k, ke=sim.diagnostics(0)["ke"], defects=(pl + mi) / side ** 2, slope=slope))
        _say("gpu", json.dumps(series[-1]))
    _say(f"gpu: {n_gpu} steps in {time.perf_counter() - t0:.1f} s")
    sim.close()
    st = oracle.State(s0)
    orc = []
    t0 = time.perf_counter()
    for k in range(every, n_orc + 1, every):
        oracle.step(p, st, every)
        f = st.fields()
        op, om = diag.defects(p, f["x"], f["y"], f["qxx"], f["qxy"], side)
        _, so = diag.spectrum(p, f["x"], f["y"], f["ux"], f["uy"], side)
        orc.append(dict(step=k, ke=oracle.diagnostics(p, st)["ke"], defects=(op + om) / side ** 2, slope=so))
        _say("oracle", json.dumps(orc[-1]), f"{time.perf_counter() - t0:.0f} s on {oracle.num_threads()} threads")
    g = series[:len(orc)]
    for key in ("ke", "defects", "slope"):
        mg, mo = np.mean([s[key] for s in g]), np.mean([s[key] for s in orc])
        _say(key, "gpu", mg, "oracle", mo, "rel", abs(mg - mo) / abs(mo))
        assert mg == pytest.approx(mo, rel=0.02), key
