"""Long-run statistics against the FP64 oracle's stored series of the same run
(tests/golden/make_c2_statistics.py writes them; only the oracle runs there):
  * the single run at scale, the 512 x 512 lattice box (262,144 particles),
    10,000 steps sampled every 500 (c2_512box_oracle_statistics.json);
  * the benchmark's 2048 x 2048 lattice box (4,194,304 particles), 2,000 steps
    sampled every 250 (c4_2048box_oracle_statistics.json);
  * the 512 x 512 box with the Wendland C2 kernel, 5,000 steps sampled every
    500 (c2_512box_wendland_oracle_statistics.json);
  * the 512 x 512 box with contractile activity (zeta = -0.02), 5,000 steps
    sampled every 500 (c2_512box_contractile_oracle_statistics.json);
  * the 512 x 512 box with the midpoint corrector, 2,500 steps sampled every
    500 (c2_512box_midpoint_oracle_statistics.json);
  * the 512 x 512 box with the conservative pair forces (form 1), 2,500 steps
    sampled every 500 (c2_512box_form1_oracle_statistics.json).
All start isotropic (seed 0) with zeta = K = 0.02 unless stated, dt = 1e-3.
The GPU runs the same steps and records the kinetic energy, the defect density
and the spectrum slope at the same samples; the means over the run must agree
within 2%, and the samples are reported one by one."""
import json
import os
import time

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(*a):
    print(*a, flush=True)


def _against_series(config, name, make=None, **change):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_08919_amd as P
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not written yet (python tests/golden/make_c2_statistics.py --config {make or config})")
    with open(path) as fh:
        ref = json.load(fh)
    cfg = wl.config(config)
    p, side = cfg["params"].replace(**change), cfg["n_side"]
    w = ref["workload"]
    assert (w["n_side"], w["L"], w["zeta"], w["K"], w["dt"], w["seed"]) == (side, p.L, p.zeta, p.K, p.dt, 0)
    assert w.get("kernel", 0) == p.kernel and w.get("integrator", 0) == p.integrator
    assert w.get("form", 0) == p.form
    every, n_steps = w["every"], w["steps"]
    sim = P.Sim([p], [side * side])
    sim.set_state(0, wl.state_for(cfg, 0))
    series = []
    t0 = time.perf_counter()
    for k in range(every, n_steps + 1, every):
        sim.step(every)
        sim.check()
        pl, mi = sim.defects(0, side)
        _, slope = sim.spectrum(0, side)
        series.append(dict(step=k, ke=sim.diagnostics(0)["ke"], defects=(pl + mi) / side ** 2, slope=slope))
    _say(f"gpu: {n_steps} steps of {side * side} particles in {time.perf_counter() - t0:.1f} s with the samples")
    orc = ref["series"]
    assert [s["step"] for s in orc] == [s["step"] for s in series]
    for key in ("ke", "defects", "slope"):
        g = np.array([s[key] for s in series])
        o = np.array([s[key] for s in orc])
        worst = float(np.max(np.abs(g - o) / np.abs(o)))
        mg, mo = g.mean(), o.mean()
        _say(f"{key}: gpu mean {mg:.9g}, oracle mean {mo:.9g}, rel {abs(mg - mo) / abs(mo):.2e}; "
             f"largest sample deviation {worst:.2e}")
        assert mg == pytest.approx(mo, rel=0.02), key
    for s, o in zip(series, orc):
        _say("step", s["step"], "ke", s["ke"], o["ke"], "defects", s["defects"], o["defects"],
             "slope", s["slope"], o["slope"])
    sim.close()


def test_c2_statistics_against_oracle_series():
    _against_series("C2", "c2_512box_oracle_statistics.json")


def test_c4_statistics_against_oracle_series():
    _against_series("C4", "c4_2048box_oracle_statistics.json")


def test_c2_wendland_statistics_against_oracle_series():
    _against_series("C2", "c2_512box_wendland_oracle_statistics.json", make="C2W", kernel=1)


def test_c2_contractile_statistics_against_oracle_series():
    _against_series("C2", "c2_512box_contractile_oracle_statistics.json", make="C2C", zeta=-0.02)


def test_c2_midpoint_statistics_against_oracle_series():
    _against_series("C2", "c2_512box_midpoint_oracle_statistics.json", make="C2M", integrator=1)


def test_c2_form1_statistics_against_oracle_series():
    _against_series("C2", "c2_512box_form1_oracle_statistics.json", make="C2F", form=1)
