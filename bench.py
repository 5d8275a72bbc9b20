"""Throughput benchmark of the SPH active-nematic step on one MI355X.

Workload: the 2048 x 2048 lattice box (4,194,304 particles, L = 2048, quintic
kernel with h = 1.3 dx, zeta = 0.02, K = 0.02, dt = 1e-3, isotropic director
start, seeded), FP32 pair arithmetic with compensated sums and compensated
positions. One step = rebin check + the four pair passes (volume; gradients,
molecular field, co-rotation and Q update; density filter and EoS; pressure,
corrector, APD and next predictor), all on the GPU with the state resident.

Prints one JSON line. `value` is the median over --reps repetitions (default
5) of particle-steps per second over exactly --steps timed steps, each
repetition bracketed by stream synchronisation. The first repetition of the
timed region also records HIP events on the library's own stream around every
launch: the per-kernel durations come from it (its own rate is reported as
value_with_events). For context the line also carries the median with hipGraph
replay of 10-step chunks, and the FP64 oracle timed on the host: all cores over
whole steps of the same box, and one core over one step of a 1024 x 1024 box of
the same physics; the metric's learned part (learned_4x: the corrector trained
and evaluated against plain dt and plain 4 dt at the 2% budget, after the
timed region; --no-learned skips it); and the platform (device, architecture,
HIP version, clock levels).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SPH particle-steps/s at 4.2M particles, % HBM peak; learned-4×dt vs plain at ε"

# Algorithmic work per accepted pair (FMA = 2 FLOP; no candidate rejection,
# no compensation terms) and per particle (epilogue), per pass. Pass A is the
# Verlet-list walk on most steps and the candidate search on rebuild steps;
# its time below covers both launches.
FLOP_PER_PAIR = {"pass_a_volume": 26, "pass_b_rates": 87, "pass_c_eos": 27, "pass_d_update": 45}
FLOP_PER_PARTICLE = {"pass_a_volume": 2, "pass_b_rates": 120, "pass_c_eos": 30, "pass_d_update": 60}
# Compulsory HBM bytes per particle per pass (own fields read + written once, FP32).
BYTES_PER_PARTICLE = {"pass_a_volume": 12, "pass_b_rates": 72, "pass_c_eos": 24, "pass_d_update": 100}
NEIGHBOURS = 44          # accepted pairs per particle on the h = 1.3 dx lattice (45 sites incl. self)
HBM_PEAK = 8.0e12        # B/s, MI355X
FP32_PEAK = 157.3e12     # FLOP/s, MI355X vector FP32 (packed FMA)

# HBM bytes per launch measured with two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) on the default
# configuration (2048^2 box, tile 4, 1 lane/particle, compensation 1), each scaled by what the same
# counter reads for a 1 GiB device-to-device copy in the same run (fetch x 2.0, write x 1.0). They hold
# for the kernel sources with this fingerprint only; otherwise `traffic` is reported as null.
MEASURED_TRAFFIC = {
    "fingerprint": "a9898c4ea0aea4c4",
    "config": (2048, 4, 1, 1),
    # per launch that does work (pass A: the Verlet walk of a step without rebuild)
    "bytes": {"pass_a_volume": 463.07e6, "pass_b_rates": 749.19e6, "pass_c_eos": 597.96e6,
              "pass_d_update": 901.70e6},
}


def kernel_fingerprint():
    """sha1 of the pair-pass sources with comments, trailing blanks and empty
    lines removed, so that an edit of a comment keeps the measurement."""
    import hashlib
    import re
    h = hashlib.sha1()
    for f in ("nem_passes.hip", "nem_pair.h", "nem_dev.h"):
        with open(os.path.join(ROOT, "paper_2108_08919_amd", "csrc", f), encoding="utf-8") as fh:
            src = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        lines = (re.sub(r"//.*", "", line).rstrip() for line in src.split("\n"))
        h.update("\n".join(line for line in lines if line).encode())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--reps", type=int, default=5, help="timed repetitions of --steps steps (median reported)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--side", type=int, default=2048, help="lattice side (default: the 4.2M-particle box)")
    ap.add_argument("--tile", type=int, default=4)
    ap.add_argument("--lpp", type=int, default=1)
    ap.add_argument("--comp", type=int, default=1)
    ap.add_argument("--kernel", choices=("quintic", "wendland"), default="quintic",
                    help="smoothing kernel: the paper's quintic spline (default) or the Wendland C2 variant")
    ap.add_argument("--autotune", action="store_true", help="pick tile and lanes per particle by timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-4x dt part of the metric (train on 256^2 boxes, evaluate on 1024^2)")
    ap.add_argument("--workload", choices=("box", "ensemble", "diagnostics"), default="box",
                    help="box: the 4.2M-particle box (default); ensemble: 32 uneven replicas in one launch; "
                         "diagnostics: time each grid and Lagrangian diagnostic on the box")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB device to device once "
                         "(a kernel of known traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "multi-GPU sharding is a design note, not an implemented path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as wl
    import paper_2108_08919_amd as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "ensemble":
        return ensemble(args)
    if args.workload == "diagnostics":
        return diagnostics(args)
    cfg = wl.config("C4")
    p = cfg["params"]
    if args.side != 2048:
        cfg = dict(cfg, n_side=args.side)
        p = p.replace(L=float(args.side))
        cfg["params"] = p
    if args.kernel == "wendland":
        p = p.replace(kernel=1)
        cfg["params"] = p
    n = cfg["n_side"] ** 2
    s0 = wl.state_for(cfg, 0)

    sim = P.Sim([p], [n])
    sim.set_option(P.NEM_OPT_TILE, args.tile)
    sim.set_option(P.NEM_OPT_LPP, args.lpp)
    sim.set_option(P.NEM_OPT_COMP, args.comp)
    sim.set_state(0, s0)
    sim.step(args.warmup)
    sim.check()
    if args.autotune:
        args.tile, args.lpp, _ = sim.autotune(3)
        sim.step(2)
        sim.check()

    def timed_reps(reps):
        out = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(args.steps)
            rc = sim.sync()
            torch.cuda.synchronize()
            out.append(time.perf_counter() - t0)
            if rc != 0:
                raise SystemExit(f"device error {rc}: {P.strerror(rc)}")
        return out

    # the timed region: the first repetition with per-launch HIP events on the
    # library's stream (the kernel durations), the others without (eager launches)
    sim.set_option(P.NEM_OPT_TIMING, 1)
    sim.pass_times(reset=True)
    rep_s = timed_reps(1)
    ms_pass, cnt = sim.pass_times(reset=True)
    sim.set_option(P.NEM_OPT_TIMING, 0)
    rep_s += timed_reps(args.reps - 1)
    elapsed = float(np.median(rep_s))
    value = n * args.steps / elapsed
    events_value = n * args.steps / rep_s[0]
    avg = {name: (ms_pass[i] / cnt[i] if cnt[i] else None) for i, name in enumerate(P.PASS_NAMES)}
    # context: graph replay of 10-step chunks
    sim.set_option(P.NEM_OPT_GRAPH, 10)
    sim.step(10)
    sim.check()
    graph_value = n * args.steps / float(np.median(timed_reps(args.reps)))
    sim.set_option(P.NEM_OPT_GRAPH, 0)

    # dominant kernel: the longest average launch
    dom = max((k for k in FLOP_PER_PAIR if avg.get(k)), key=lambda k: avg[k])
    bytes_step = sum(BYTES_PER_PARTICLE.values())
    roofline = None
    flops_step = None
    if args.kernel == "quintic":
        # the per-pair FLOP counts are those of the quintic kernel evaluation
        flops_launch = n * (NEIGHBOURS * FLOP_PER_PAIR[dom] + FLOP_PER_PARTICLE[dom])
        achieved = flops_launch / (avg[dom] * 1e-3)
        flops_step = sum(NEIGHBOURS * FLOP_PER_PAIR[k] + FLOP_PER_PARTICLE[k] for k in FLOP_PER_PAIR)

    traffic = None
    hbm_counters = None
    if (args.kernel == "quintic" and kernel_fingerprint() == MEASURED_TRAFFIC["fingerprint"]
            and (cfg["n_side"], args.tile, args.lpp, args.comp) == MEASURED_TRAFFIC["config"]):
        tb = MEASURED_TRAFFIC["bytes"]
        traffic = tb[dom]
        # bytes per launch from the recorded counter runs of the same kernel sources,
        # over the pass times of this run
        hbm_counters = {"GB/s": sum(tb.values()) / (sum(avg[k] for k in tb) * 1e-3) / 1e9,
                        "frac": sum(tb.values()) / (sum(avg[k] for k in tb) * 1e-3) / HBM_PEAK,
                        "bytes_per_step": sum(tb.values()),
                        "source": "profiles/step_2048box_hbm_counters.md (rocprofv3 FETCH_SIZE and WRITE_SIZE "
                                  "of the same kernel sources, copy-calibrated)"}

    if args.kernel == "quintic":
        roofline = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": FP32_PEAK / 1e12,
                    "unit": "TFLOP/s", "frac": achieved / FP32_PEAK, "traffic": traffic,
                    "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"}

    plat = platform()   # right after the GPU work, while the clocks are at their working level
    sim.close()
    learned4 = None
    if args.kernel == "quintic" and args.side == 2048 and not args.no_learned:
        learned4 = learned_part()
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        # a bounded sample: whole steps of the same box until about 10 s of CPU work
        st = oracle.State(s0)
        c0 = time.perf_counter()
        done = 0
        while done < 20 and (done == 0 or time.perf_counter() - c0 < 10.0):
            oracle.step(p, st, 1)
            done += 1
        c1 = time.perf_counter()
        cpu = {"value": n * done / (c1 - c0), "unit": "particle-steps/s", "cores": oracle.num_threads(),
               "kind": "oracle", "sample": f"{done} steps of the same {cfg['n_side']}x{cfg['n_side']} box "
                                           f"from its initial state ({c1 - c0:.1f} s, FP64 C + OpenMP)"}
        cpu.update(oracle_one_core(p))

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg['n_side']}x{cfg['n_side']} lattice box, {n} particles, L={p.L:g}, "
                               f"h=1.3dx {args.kernel}, zeta={p.zeta}, K={p.K}, dt={p.dt}, isotropic start (seed 0)",
                   "particles": n, "tile": args.tile, "lanes_per_particle": args.lpp,
                   "compensation": args.comp},
        "roofline": roofline,
        "repetitions": args.reps,
        "ms_per_step_reps": [1e3 * t / args.steps for t in rep_s],
        "value_with_events": events_value,
        "graph_value": graph_value,
        "hbm_counters": hbm_counters,
        "hbm_frac_algorithmic": value * bytes_step / HBM_PEAK,
        "valu_frac_algorithmic": value * flops_step / FP32_PEAK if flops_step else None,
        "bytes_per_particle_step": bytes_step,
        "flop_per_particle_step": flops_step,
        "kernel_ms": avg,
        "cpu_baseline": cpu,
        "learned_4x": learned4,
        "platform": plat,
    }
    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = 2 * src.numel() * 4
    print(json.dumps(out), flush=True)


def learned_part():
    """The metric's second part, learned 4x dt against plain stepping at the
    error budget: the corrector trained on 256x256 boxes (1M samples) and
    evaluated on the 1024x1024 box, 4 seeds, t in [0, 2], against plain dt =
    1e-3 and plain 4 dt without the network (the full record is what
    `python -m paper_2108_08919_amd.learned --mult 4` prints)."""
    from paper_2108_08919_amd import learned
    r = learned.run(mult=4)
    L, Cc = r["learned"], r["plain_coarse"]
    return {"workload": "1024x1024 box (1,048,576 particles), zeta = K = 0.02, 4 seeds, t in [0, 2]; "
                        "dt = 1e-3 (plain) against 4e-3 (plain coarse, learned); trained on 256x256 boxes",
            "speedup_learned_vs_plain": r["speedup_learned_vs_plain"],
            "speedup_coarse_vs_plain": r["speedup_coarse_vs_plain"],
            "eps_ke": L["eps_ke"], "eps_defects": L["eps_defects"],
            "eps_ke_coarse": Cc["eps_ke"], "eps_defects_coarse": Cc["eps_defects"],
            "within_2pct": bool(L["eps_ke"] <= 0.02 and L["eps_defects"] <= 0.02),
            "q_field_err": L["q_field_err"], "q_field_err_coarse": Cc["q_field_err"],
            "u_field_err": L["u_field_err"], "u_field_err_coarse": Cc["u_field_err"],
            "fallbacks": r["fallbacks"], "held_out_rel_mse": r["held_out_rel_mse"]}


def platform():
    """The device, its architecture and compute units, the HIP version torch
    was built with, and what rocm-smi reports: the product name and the current
    clock levels (taken right after the timed work; None where a query is not
    available)."""
    import subprocess
    import torch
    pr = torch.cuda.get_device_properties(0)
    out = {"device": pr.name, "arch": getattr(pr, "gcnArchName", None), "compute_units": pr.multi_processor_count,
           "memory_gib": round(pr.total_memory / 2 ** 30, 1), "hip": torch.version.hip, "clocks": None}
    def smi(flag, key):
        try:
            r = subprocess.run(["rocm-smi", flag], capture_output=True, text=True, timeout=20)
        except (OSError, subprocess.SubprocessError):
            return None
        lines = [ln.split(":", 1)[-1].strip() for ln in r.stdout.splitlines()
                 if "GPU[0]" in ln and key in ln.lower()]
        return lines or None
    out["clocks"] = smi("--showclocks", "clock level")
    prod = [" ".join(v.split()) for v in (smi("--showproductname", "card") or [])]
    out["product"] = [v for v in prod if not v.upper().endswith("N/A")] or None
    return out


def oracle_one_core(p):
    """The oracle on one host core (a child process with OMP_NUM_THREADS=1,
    which touches no GPU): one step of a 1024 x 1024 box of the same physics
    (same density, kernel and parameters, so the same work per particle-step
    as the 2048 x 2048 box)."""
    import subprocess
    code = ("import sys, time, json; sys.path.insert(0, %r); import oracle, workloads as wl; "
            "p = wl.Params(L=1024.0, zeta=%r, K=%r, dt=%r); "
            "st = oracle.State(wl.initial_state(1024, 1.0, 1.0, 0, 'isotropic')); "
            "t0 = time.perf_counter(); oracle.step(p, st, 1); t = time.perf_counter() - t0; "
            "print(json.dumps([oracle.num_threads(), t]))") % (ROOT, p.zeta, p.K, p.dt)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    if r.returncode != 0:
        return {"value_1core": None, "sample_1core": f"failed: {r.stderr[-300:]}"}
    threads, t = json.loads(r.stdout.strip().splitlines()[-1])
    return {"value_1core": 1024 * 1024 / t, "cores_1core": threads,
            "sample_1core": f"1 step of a 1024x1024 box of the same physics on {threads} core ({t:.1f} s)"}


def diagnostics(args):
    """Wall time per call of each diagnostic on the 2048 x 2048 box after a few
    steps (the calls synchronise and return host arrays, so wall time is the
    cost a caller sees): FP64 reductions, Shepard deposit, spectrum, defects and
    vorticity correlation on the M x M grid (M = 2048), pathlines of 4096 tagged
    particles and the quadrant mixing histogram (512 x 512 bins)."""
    import numpy as np
    import torch
    import workloads as wl
    import paper_2108_08919_amd as P
    cfg = wl.config("C4")
    p = cfg["params"]
    n = cfg["n_side"] ** 2
    s0 = wl.state_for(cfg, 0)
    ux, uy = wl.smooth_velocity(s0["x"], s0["y"], p.L, 1e-3, 7)
    s0["ux"], s0["uy"] = ux, uy
    sim = P.Sim([p], [n])
    sim.set_state(0, s0)
    sim.step(10)
    sim.check()
    M = cfg["n_side"]
    ids = np.arange(0, n, n // 4096, dtype=np.int32)
    colour = ((s0["x"] >= p.L / 2).astype(np.uint8) + 2 * (s0["y"] >= p.L / 2).astype(np.uint8)).astype(np.uint8)
    calls = {
        "reductions": lambda: sim.diagnostics(0),
        "deposit": lambda: sim.deposit(0, M),
        "spectrum": lambda: sim.spectrum(0, M),
        "defects": lambda: sim.defects(0, M),
        "vorticity_correlation": lambda: sim.vorticity_correlation(0, M),
        "track_4096": lambda: sim.track(ids),
        "mixing_512": lambda: sim.mixing(colour, 4, 512),
    }
    out = {}
    for name, f in calls.items():
        f()                                   # first call allocates the grid buffers
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            f()
        t1 = time.perf_counter()
        out[name] = 1e3 * (t1 - t0) / 5
        print(f"[diagnostics] {name}: {out[name]:.3f} ms", file=sys.stderr, flush=True)
    sim.close()
    print(json.dumps({"metric": "diagnostic wall time per call", "unit": "ms", "higher_is_better": False,
                      "config": {"workload": f"{M}x{M} lattice box, {n} particles, grid {M}x{M}"},
                      "ms": out}), flush=True)


def ensemble(args):
    """32 replicas, sides drawn from U{128..384} (seeded), zeta x K sweep x 2
    seeds, advanced together: one launch per pass over the tiles of all
    replicas, launch shape (tile, lanes per particle, persistent grid) picked
    by the autotuner, steps replayed from a captured graph of 10 steps. The
    median of --reps repetitions; the same with a persistent grid forced off
    and on for comparison."""
    import numpy as np
    import torch
    import workloads as wl
    import paper_2108_08919_amd as P
    reps = wl.ensemble(0)
    params = [r["params"] for r in reps]
    ns = [r["n_side"] ** 2 for r in reps]
    sim = P.Sim(params, ns)
    for i, r in enumerate(reps):
        sim.set_state(i, wl.state_for(r))
    sim.step(2)
    tile, lpp, _ = sim.autotune(3)
    persist = sim.get_option(P.NEM_OPT_PERSIST)
    sim.set_option(P.NEM_OPT_GRAPH, 10)
    sim.step(args.warmup)
    sim.check()
    N = sum(ns)

    def median_value():
        out = []
        for _ in range(args.reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(args.steps)
            rc = sim.sync()
            torch.cuda.synchronize()
            out.append(time.perf_counter() - t0)
            if rc != 0:
                raise SystemExit(f"device error {rc}: {P.strerror(rc)}")
        return N * args.steps / float(np.median(out)), out

    value, rep_s = median_value()
    plat = platform()
    by_grid = {}
    for g in (0, 1024):
        sim.set_option(P.NEM_OPT_PERSIST, g)
        sim.set_option(P.NEM_OPT_GRAPH, 10)
        sim.step(10)
        by_grid[str(g)] = median_value()[0]
    out = {"metric": "SPH particle-steps/s, batched ensemble", "value": value, "unit": "particle-steps/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "repetitions": args.reps,
           "ms_per_step": 1e3 * float(np.median(rep_s)) / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{len(reps)} replicas, sides U{{128..384}}, {N} particles, zeta x K sweep",
                      "particles": N, "tile": tile, "lanes_per_particle": lpp, "persistent_grid": persist,
                      "graph_steps": 10},
           "value_by_persistent_grid": by_grid,
           "platform": plat,
           "hbm_frac_algorithmic": value * sum(BYTES_PER_PARTICLE.values()) / HBM_PEAK}
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
