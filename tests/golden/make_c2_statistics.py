"""Write the FP64 oracle's long-run statistics of a single box.

Workloads (isotropic director start, seed 0, zeta = K = 0.02 unless stated, dt = 1e-3):
  C2: the 512 x 512 lattice box (262,144 particles), 10,000 steps, a sample
      every 500 (about an hour on 8 host cores);
  C4: the 2048 x 2048 lattice box (4,194,304 particles), 2,000 steps, a sample
      every 250 (about four and a half hours on 8 host cores);
  C2W: the C2 box with the Wendland C2 kernel (support 2h, 20 lattice
      neighbours), 5,000 steps, a sample every 500;
  C2C: the C2 box with contractile activity, zeta = -0.02, 5,000 steps, a
      sample every 500;
  C2M: the C2 box with the midpoint corrector, 2,500 steps, a sample every
      500;
  C2F: the C2 box with the conservative pair forces (form 1), 2,500 steps, a
      sample every 500.
Each sample records the kinetic energy (Eq. kineticenergy as a particle
average), the defect density ((n+ + n-)/L^2 from the director winding on the
side x side deposit grid) and the slope of the kinetic-energy spectrum over
shells 4..side/8 (paper Sec. 5: energy spectrum and defect maps).

Only the oracle runs here (test infrastructure: oracle/ and the seeded inputs of
workloads/); the GPU suite compares its own run of the same workload against
the stored series:

    python tests/golden/make_c2_statistics.py [--config C2|C4|C2W|C2C|C2M|C2F] [--steps N] [--every K]
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
    ap.add_argument("--config", choices=("C2", "C4", "C2W", "C2C", "C2M", "C2F"), default="C2")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--every", type=int, default=None)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    # config -> (base workload, parameter changes, steps, sample interval, file)
    base, change, steps, every, name = {
        "C2": ("C2", {}, 10000, 500, "c2_512box_oracle_statistics.json"),
        "C4": ("C4", {}, 2000, 250, "c4_2048box_oracle_statistics.json"),
        "C2W": ("C2", {"kernel": 1}, 5000, 500, "c2_512box_wendland_oracle_statistics.json"),
        "C2C": ("C2", {"zeta": -0.02}, 5000, 500, "c2_512box_contractile_oracle_statistics.json"),
        "C2M": ("C2", {"integrator": 1}, 2500, 500, "c2_512box_midpoint_oracle_statistics.json"),
        "C2F": ("C2", {"form": 1}, 2500, 500, "c2_512box_form1_oracle_statistics.json")}[a.config]
    defaults = (steps, every, name)
    a.steps = a.steps or defaults[0]
    a.every = a.every or defaults[1]
    a.out = a.out or os.path.join(HERE, defaults[2])
    cfg = wl.config(base)
    p, side = cfg["params"].replace(**change), cfg["n_side"]
    kernel = p.kernel
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
        _source=(f"FP64 oracle (oracle/orc.c, oracle/diag.py) on the {side} x {side} lattice box, written by "
                 "tests/golden/make_c2_statistics.py; no value comes from the GPU path"),
        workload=dict(n_side=side, L=p.L, zeta=p.zeta, K=p.K, dt=p.dt, seed=0, kind=cfg["kind"], kernel=kernel,
                      integrator=p.integrator, form=p.form,
                      steps=a.steps, every=a.every, spectrum_shells=[4, side // 8]),
        threads=oracle.num_threads(), seconds=time.perf_counter() - t0, series=series)
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()
