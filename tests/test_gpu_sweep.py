"""Trend-level checks of the activity / elastic-constant sweep on batched
replicas against the qualitative statements of Sec. 5: the velocity scale
grows with |zeta| for extensile and contractile activity alike, and a larger
elastic constant K leaves fewer defects."""
import numpy as np
import pytest

from paper_2108_08919_amd import sweep

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_08919_amd as P
    P.lib()
    yield


def test_vrms_grows_with_activity_of_both_signs():
    reps = sweep.build_replicas([0.01, 0.02, 0.04], [0.02], 1, 96, "both")
    print("replicas", len(reps), flush=True)
    rec = sweep.run(reps, 2000, 500, 1000, graph=10, autotune=False)
    rows = {r["zeta"]: r for r in sweep.table(rec)}
    print({z: r["vrms"] for z, r in rows.items()}, flush=True)
    for sg in (1.0, -1.0):
        v = [rows[sg * z]["vrms"] for z in (0.01, 0.02, 0.04)]
        assert 0 < v[0] < v[1] < v[2]
        # weak activity: the flow is the linear response of the Stokes problem
        assert 1.8 < v[1] / v[0] < 2.2 and 1.8 < v[2] / v[1] < 2.2
    for z in (0.01, 0.02, 0.04):
        assert rows[-z]["vrms"] == pytest.approx(rows[z]["vrms"], rel=0.2)
        assert np.isfinite(rows[z]["l"]) and rows[z]["l"] > 0


def test_defect_density_falls_with_elastic_constant():
    reps = sweep.build_replicas([0.02], [0.01, 0.04, 0.08], 1, 128, "pos")
    print("replicas", len(reps), flush=True)
    rec = sweep.run(reps, 20000, 5000, 10000, graph=10, autotune=False)
    rows = {r["K"]: r for r in sweep.table(rec)}
    d = [rows[k]["defect_density"] for k in (0.01, 0.04, 0.08)]
    print(d, flush=True)
    assert d[0] > 1.05 * d[1] and d[1] > 1.05 * d[2] > 0


def test_vortex_size_grows_with_elastic_constant():
    """Sec. 5: larger K gives larger vortices (the active length sqrt(K/zeta)).
    Same initial state for every K, so only K differs."""
    import workloads as wl
    reps = [dict(name=f"K{k}", n_side=128, params=wl.Params(L=128.0, zeta=0.02, K=k), kind="isotropic", seed=1000)
            for k in (0.01, 0.04, 0.16)]
    rec = sweep.run(reps, 5000, 500, 2500, graph=10, autotune=False)
    ls = [r["l"] for r in rec[:-1]]
    print("l_omega", ls, flush=True)
    assert ls[0] < ls[1] < ls[2]
