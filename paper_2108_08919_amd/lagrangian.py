"""Lagrangian diagnostics over an activity / elastic-constant sweep: pathlines
of tagged particles and the mixing of the four quadrants of the box.

Sec. 5 of the paper follows single particles through the run (their
pathlines grow longer with |zeta|) and colours the four quadrants of the box to
watch them mix (faster at higher activity, slower at higher K). Here every
(zeta, K, seed) is one replica of a batched simulation (the replicas of the
activity sweep); each replica tags `n_tag` particles and colours every particle
by the quadrant of its initial position. Every `every` steps the library
returns the unwrapped positions of the tagged particles (periodic image
counters carried with each particle, so no sampling rate is needed for
unwrapping) and the colour histogram on a B x B partition with its mixing
index (1 - Danckwerts' intensity of segregation).

Reported per replica: mean pathline length (sum of |dr| between samples),
mean net displacement |r(T) - r(0)|, and the mixing index at the end.

    python -m paper_2108_08919_amd.lagrangian --side 128 --steps 50000 --every 1000
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from typing import Dict, List

import numpy as np

from .sweep import build_replicas


def quadrant_colour(x: np.ndarray, y: np.ndarray, L: float) -> np.ndarray:
    xw, yw = np.mod(x, L), np.mod(y, L)
    return ((xw >= 0.5 * L).astype(np.uint8) + 2 * (yw >= 0.5 * L).astype(np.uint8)).astype(np.uint8)


def run(reps: List[Dict], steps: int, every: int, n_tag: int = 64, bins: int = 0, graph: int = 10,
        keep_paths: int = 5, log=sys.stdout) -> List[Dict]:
    import workloads as wl
    import paper_2108_08919_amd as P
    params = [r["params"] for r in reps]
    ns = [r["n_side"] ** 2 for r in reps]
    sim = P.Sim(params, ns)
    try:
        colours, tags, B = [], [], []
        for i, r in enumerate(reps):
            st = wl.state_for(r)
            sim.set_state(i, st)
            L = r["params"].L
            colours.append(quadrant_colour(st["x"], st["y"], L))
            rng = np.random.default_rng(r["seed"])
            tags.append(np.sort(rng.choice(ns[i], size=min(n_tag, ns[i]), replace=False)).astype(np.int32))
            b = bins or max(2, int(round(L / 4)))
            B.append(b + (b & 1))   # even, so that the quadrants start segregated
        if graph:
            sim.set_option(P.NEM_OPT_GRAPH, graph)
        paths = [[sim.track(tags[i], i)] for i in range(len(reps))]
        mix = [[sim.mixing(colours[i], 4, B[i], i)[0]] for i in range(len(reps))]
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            n = min(every, steps - done)
            sim.step(n)
            done += n
            sim.check()
            for i in range(len(reps)):
                paths[i].append(sim.track(tags[i], i))
                mix[i].append(sim.mixing(colours[i], 4, B[i], i)[0])
            print(f"[lagrangian] step {done}/{steps}  {time.perf_counter() - t0:.1f} s  "
                  f"mixing {min(m[-1] for m in mix):.4f}..{max(m[-1] for m in mix):.4f}", file=log, flush=True)
        out = []
        for i, r in enumerate(reps):
            xs = np.array([p[0] for p in paths[i]])
            ys = np.array([p[1] for p in paths[i]])
            length = np.sqrt(np.diff(xs, axis=0) ** 2 + np.diff(ys, axis=0) ** 2).sum(axis=0)
            net = np.hypot(xs[-1] - xs[0], ys[-1] - ys[0])
            p = r["params"]
            out.append(dict(replica=i, side=r["n_side"], zeta=p.zeta, K=p.K, seed=r["seed"], bins=B[i],
                            path_length=float(length.mean()), net_displacement=float(net.mean()),
                            mixing=float(mix[i][-1]), mixing_series=[float(v) for v in mix[i]],
                            paths=[[xs[:, k].tolist(), ys[:, k].tolist()] for k in range(min(keep_paths, xs.shape[1]))]))
        return out
    finally:
        sim.close()


def table(records: List[Dict]) -> List[Dict]:
    rows: Dict = {}
    for r in records:
        rows.setdefault((r["zeta"], r["K"]), []).append(r)
    return [dict(zeta=z, K=k, n=len(rs), path_length=float(np.mean([r["path_length"] for r in rs])),
                 net_displacement=float(np.mean([r["net_displacement"] for r in rs])),
                 mixing=float(np.mean([r["mixing"] for r in rs])))
            for (z, k), rs in sorted(rows.items())]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--zeta", type=float, nargs="+", default=[0.005, 0.01, 0.02, 0.04])
    ap.add_argument("--K", type=float, nargs="+", default=[0.01, 0.02, 0.04, 0.08])
    ap.add_argument("--seeds", type=int, default=1)
    ap.add_argument("--side", type=int, default=128)
    ap.add_argument("--signs", choices=("pos", "neg", "both"), default="both")
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--tags", type=int, default=64, help="tagged particles per replica")
    ap.add_argument("--bins", type=int, default=0, help="mixing bins per side (0: L/4)")
    ap.add_argument("--json", default="", help="write the records (with 5 pathlines each) to this file")
    a = ap.parse_args(argv)
    reps = build_replicas(a.zeta, a.K, a.seeds, a.side or None, a.signs)
    print(f"[lagrangian] {len(reps)} replicas, {sum(r['n_side'] ** 2 for r in reps)} particles, "
          f"{a.steps} steps, sampled every {a.every}", flush=True)
    rec = run(reps, a.steps, a.every, a.tags, a.bins)
    print(f"{'zeta':>8} {'K':>6} {'path length':>12} {'net disp':>10} {'mixing':>9}")
    for r in table(rec):
        print(f"{r['zeta']:8.3f} {r['K']:6.3f} {r['path_length']:12.4e} {r['net_displacement']:10.4e} "
              f"{r['mixing']:9.5f}")
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rec, f)


if __name__ == "__main__":
    main()
