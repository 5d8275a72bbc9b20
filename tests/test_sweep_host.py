"""Host logic of the activity / elastic-constant sweep (no GPU)."""
import math

import workloads as wl
from paper_2108_08919_amd import sweep


def test_positive_sweep_is_the_ensemble_workload():
    reps = sweep.build_replicas([0.005, 0.01, 0.02, 0.04], [0.01, 0.02, 0.04, 0.08], 2, None, "pos")
    ens = wl.ensemble(0)
    assert len(reps) == len(ens) == 32
    for a, b in zip(reps, ens):
        assert a["n_side"] == b["n_side"] and a["params"] == b["params"] and a["seed"] == b["seed"]


def test_contractile_mirrors_share_the_initial_state():
    reps = sweep.build_replicas([0.01, 0.02], [0.02, 0.04], 2, 64, "both")
    assert len(reps) == 16
    for a, b in zip(reps[0::2], reps[1::2]):
        assert b["params"].zeta == -a["params"].zeta and a["params"].K == b["params"].K
        assert a["seed"] == b["seed"] and a["n_side"] == b["n_side"] == 64
    assert len({r["seed"] for r in reps}) == 8


def test_table_averages_over_seeds():
    rec = [dict(zeta=0.01, K=0.02, vrms=1.0, l=2.0, defect_density=0.1),
           dict(zeta=0.01, K=0.02, vrms=3.0, l=float("nan"), defect_density=0.3),
           dict(zeta=-0.01, K=0.02, vrms=5.0, l=4.0, defect_density=0.5),
           dict(wall_s=1.0, particle_steps=10.0)]
    rows = sweep.table(rec)
    assert [(r["zeta"], r["n"]) for r in rows] == [(-0.01, 1), (0.01, 2)]
    assert rows[1]["vrms"] == 2.0 and rows[1]["l"] == 2.0 and math.isclose(rows[1]["defect_density"], 0.2)


def test_grid_side_is_a_power_of_two_covering_the_box():
    assert [sweep._pow2_at_least(v) for v in (5.0, 64.0, 65.0, 128.0, 384.0)] == [8, 64, 128, 128, 512]


def test_lagrangian_quadrant_colours_match_the_oracle_reading():
    import numpy as np
    from oracle import lagrangian as lg
    from paper_2108_08919_amd import lagrangian
    rng = np.random.default_rng(2)
    L = 40.0
    x, y = rng.uniform(-L, 2 * L, 1000), rng.uniform(-L, 2 * L, 1000)
    assert np.array_equal(lagrangian.quadrant_colour(x, y, L), lg.quadrant_colour(np.mod(x, L), np.mod(y, L), L))
