"""Write the FP64 oracle's long-run statistics of the single run at scale.

Workload: the 512 x 512 lattice box (262,144 particles, L = 512, zeta = K = 0.02,
dt = 1e-3, isotropic director start, seed 0), 10,000 steps. Every 500 steps the
oracle records the kinetic energy (Eq. kineticenergy as a particle average),
the defect density ((n+ + n-)/L^2 from the director winding on the 512 x 512
deposit grid) and the slope of the kinetic-energy spectrum over shells 4..64
(paper Sec. 5: energy spectrum and defect maps).

Only the oracle runs here (test infrastructure: oracle/ and the seeded inputs of
workloads/); the GPU suite compares its own run of the same workload against
the stored series. It takes about an hour on 8 host cores:

    python tests/golden/make_c2_statistics.py [--steps 10000] [--every 500]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import diag  # noqa: E402
import workloads as wl  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--out", default=os.path.join(HERE, "c2_512box_oracle_statistics.json"))
    a = ap.parse_args()
    cfg = wl.config("C2")
    p, side = cfg["params"], cfg["n_side"]
    st = oracle.State(wl.state_for(cfg, 0))
    series = []
    t0 = time.perf_counter()
    for k in range(a.every, a.steps + 1, a.every):
        oracle.step(p, st, a.every)
        f = st.fields()
        npl, nmi = diag.defects(p, f["x"], f["y"], f["qxx"], f["qxy"], side)
        _, slope = diag.spectrum(p, f["x"], f["y"], f["ux"], f["uy"], side)
        series.append(dict(step=k, ke=oracle.diagnostics(p, st)["ke"], n_plus=int(npl), n_minus=int(nmi),
                           defects=(npl + nmi) / side ** 2, slope=slope))
        print(json.dumps(series[-1]), f"{time.perf_counter() - t0:.0f} s", flush=True)
    out = dict(
        _source=("FP64 oracle (oracle/orc.c, oracle/diag.py) on the 512 x 512 lattice box, written by "
                 "tests/golden/make_c2_statistics.py; no value comes from the GPU path"),
        workload=dict(n_side=side, L=p.L, zeta=p.zeta, K=p.K, dt=p.dt, seed=0, kind=cfg["kind"],
                      steps=a.steps, every=a.every, spectrum_shells=[4, side // 8]),
        threads=oracle.num_threads(), seconds=time.perf_counter() - t0, series=series)
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()
