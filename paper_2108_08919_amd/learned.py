"""Learned corrector: training data from the solver, training, evaluation.

Every numerical step runs in the library (nem_samples_rows, nem_mlp_fit_norm,
nem_mlp_train, nem_mlp_eval, nem_mlp_mask_outputs, nem_step_learned,
nem_diagnostics, nem_defects); this module only schedules the calls, draws the
seeded parameters and sample rows, and collects the results (torch supplies
device memory).

Workloads:
* training: 16 replicas of a 256 x 256 lattice box with (zeta, K) drawn from
  U[0.005, 0.04] x U[0.01, 0.08] (seeded), isotropic director start, advanced
  by macro steps of mult*dt without corrections (a network of zeros), the way a
  learned run advances; at six times t in {0.02, 0.1, 0.25, 0.75, 1.25, 1.75}
  (the first two in the transient that follows the start from rest) every
  replica contributes the inputs and the (mult steps of dt) - (one step of
  mult*dt) targets of a seeded subset of 10,923 of its particles:
  6 x 16 x 10,923 = 1,048,608 samples. Coarse trajectories matter for the
  velocity inputs: the change of acceleration over a step spans the previous
  macro step, as it does in a learned run;
* held out: 4 more replicas from other seeds, same recipe, every particle;
  the network's mean squared error per output relative to the output's
  variance (1 = no better than no correction), and the largest correction norm
  it predicts on these states;
* evaluation: the 1024 x 1024 box at zeta = K = 0.02 over t in [0, 2] from four
  seeded isotropic starts: plain steps of dt = 1e-3 (reference), plain steps of
  mult dt, and learned macro steps of mult dt; the errors are those of the
  ensemble- and time-averaged kinetic energy and defect density over t in
  [1, 2], and the relative L2 errors of the final fields against the plain-dt
  run from the same start (Q relative to its change over the run, u relative to
  its size).

Output components with no skill on the held-out boxes (relative MSE not below
1) are switched off before the evaluation. The fallback threshold tau is then
TAU_MARGIN times the largest correction norm the network predicts on the
held-out boxes: a macro step whose corrections go beyond anything the network
produced on states of its training distribution is replayed as mult fine steps.

Run: python -m paper_2108_08919_amd.learned [--mult 4]  (prints one JSON line)
"""
from __future__ import annotations

import json
import math
import sys
import time

import numpy as np

TAU_MARGIN = 1.5


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _sim(params, n):
    from . import Sim
    return Sim(params, n)


def zero_network():
    """A network of zeros with identity normalisation: learned macro steps with
    it are plain steps of mult*dt."""
    from . import Mlp
    m = Mlp()
    m.set_weights(np.zeros(m.nparams, dtype=np.float32))
    m.set_norm(np.concatenate([np.zeros(12), np.ones(12), np.zeros(5), np.ones(5)]).astype(np.float32))
    return m


TRAIN_TIMES = (0.02, 0.1, 0.25, 0.75, 1.25, 1.75)


def training_set(side=256, replicas=16, times=TRAIN_TIMES, per_replica=10923, mult=4, seed=0, dt=1e-3):
    """(X, T) on the device: seeded replicas advanced by uncorrected macro steps
    of mult*dt; per_replica=None takes every particle."""
    import torch
    import workloads as wl
    rng = np.random.default_rng(seed)
    params, states = [], []
    for r in range(replicas):
        zeta = float(rng.uniform(0.005, 0.04))
        K = float(rng.uniform(0.01, 0.08))
        params.append(wl.Params(L=float(side), zeta=zeta, K=K, dt=dt))
        states.append(wl.initial_state(side, 1.0, 1.0, seed=2000 + 100 * seed + r, kind="isotropic"))
    n = side * side
    take = n if per_replica is None else per_replica
    sim = _sim(params, [n] * replicas)
    for r in range(replicas):
        sim.set_state(r, states[r])
    z = zero_network()
    rows_per_time = replicas * take
    X = torch.empty((len(times) * rows_per_time, 12), dtype=torch.float32, device=sim.device)
    T = torch.empty((len(times) * rows_per_time, 5), dtype=torch.float32, device=sim.device)
    t = 0.0
    for i, tk in enumerate(times):
        k = int(round((tk - t) / (mult * dt)))
        sim.step_learned(z, k, mult)
        t += k * mult * dt
        rows = np.concatenate([(np.arange(n) if per_replica is None else np.sort(rng.choice(n, take, replace=False)))
                               + r * n for r in range(replicas)])
        sl = slice(i * rows_per_time, (i + 1) * rows_per_time)
        sim.samples_rows(rows, mult, X[sl], T[sl])
    sim.check()
    sim.close()
    z.close()
    return X, T


def init_weights(seed=0):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases (flat FP32 vector)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in ((12, 64), (64, 64), (64, 5)):
        lim = 1.0 / math.sqrt(i)
        parts.append(rng.uniform(-lim, lim, size=i * o))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def fit(X, T, epochs=20, batch=4096, lr=2e-3, seed=0):
    """Train a network on (X, T); returns (mlp, final batch loss)."""
    from . import Mlp
    m = Mlp()
    m.set_weights(init_weights(seed))
    m.fit_norm(X, T)
    loss = m.train(X, T, epochs=epochs, batch=batch, lr=lr)
    return m, loss


def held_out_errors(m, X, T):
    """Per-output mean squared error of the network on (X, T) relative to the
    variance of T (1 = no better than predicting the mean, 0 = exact)."""
    return m.evaluate(X, T)[0]


def mask_unskilled(m, rel, threshold=1.0):
    """Switch off the output components whose held-out relative MSE is not
    below `threshold` (no better than no correction); returns their indices."""
    masked = [o for o, r in enumerate(rel) if not r < threshold]
    if masked:
        m.mask_outputs(masked)
    return masked


def fallback_threshold(m, X):
    """tau = TAU_MARGIN x the largest correction norm the (masked) network
    predicts on the held-out inputs X."""
    return TAU_MARGIN * m.evaluate(X)[1]


def _observe(sim, side):
    d = sim.diagnostics(0)
    p, mi = sim.defects(0, side)
    return d["ke"], (p + mi) / float(side * side)


def evaluate(m, tau, side=1024, seeds=(0, 1, 2, 3), t_end=2.0, t_avg=(1.0, 2.0), dt=1e-3, mult=4, every=0.1):
    """Plain dt, plain mult*dt and learned mult*dt from the same seeded starts.
    All three observe at the same times: the start of the averaging window and
    every `every` after it, both rounded to whole macro steps of mult*dt. The
    speedups are timed separately, each method over the whole horizon in one
    call (the interleaved timings of the observed runs are reported too)."""
    import torch
    import workloads as wl
    p = wl.Params(L=float(side), zeta=0.02, K=0.02, dt=dt)
    n = side * side
    res = {"plain": [], "plain_coarse": [], "learned": []}
    times = {"plain": 0.0, "plain_coarse": 0.0, "learned": 0.0}
    # field errors at the end of the run against the plain-dt fields of the same
    # start: Q relative to its change over the run, u relative to its size
    ferr = {"plain_coarse": {"q": [], "u": []}, "learned": {"q": [], "u": []}}
    fallbacks = 0
    k_first = max(1, int(round(t_avg[0] / (mult * dt))))        # macro steps to the window
    k_every = max(1, int(round(every / (mult * dt))))           # macro steps between observations
    n_obs = int(round((t_avg[1] - t_avg[0]) / (k_every * mult * dt))) + 1
    spans = [k_first] + [k_every] * (n_obs - 1)
    for s in seeds:
        st = wl.initial_state(side, 1.0, 1.0, seed=3000 + s, kind="isotropic")
        ref = None
        for mode in ("plain", "plain_coarse", "learned"):
            q = p if mode != "plain_coarse" else p.replace(dt=mult * dt)
            sim = _sim([q], [n])
            sim.set_state(0, st)
            obs = []
            for k in spans:
                torch.cuda.synchronize()
                c0 = time.perf_counter()
                if mode == "plain":
                    sim.step(k * mult)
                    sim.sync()
                elif mode == "plain_coarse":
                    sim.step(k)
                    sim.sync()
                else:
                    nfb, _ = sim.step_learned(m, k, mult, tau)
                    fallbacks += nfb
                torch.cuda.synchronize()
                times[mode] += time.perf_counter() - c0
                obs.append(_observe(sim, side))
            sim.check()
            f = sim.get_state(0)
            sim.close()
            res[mode].append(obs)
            q = np.concatenate([f["qxx"], f["qxy"]])
            u = np.concatenate([f["ux"], f["uy"]])
            if mode == "plain":
                ref = (q, u, q - np.concatenate([st["qxx"], st["qxy"]]))
            else:
                ferr[mode]["q"].append(float(np.linalg.norm(q - ref[0]) / np.linalg.norm(ref[2])))
                ferr[mode]["u"].append(float(np.linalg.norm(u - ref[1]) / np.linalg.norm(ref[1])))
            _log(f"evaluated seed {s} {mode}: {times[mode]:.2f} s cumulative")
    out = {"window": [k_first * mult * dt, (k_first + k_every * (n_obs - 1)) * mult * dt], "observations": n_obs}
    ref = np.array(res["plain"])           # seeds x times x (ke, defects)
    for mode in res:
        a = np.array(res[mode])
        ke, de = a[..., 0].mean(), a[..., 1].mean()
        out[mode] = {"ke": float(ke), "defect_density": float(de), "seconds": times[mode]}
        out[mode]["eps_ke"] = float(abs(ke - ref[..., 0].mean()) / ref[..., 0].mean())
        out[mode]["eps_defects"] = float(abs(de - ref[..., 1].mean()) / ref[..., 1].mean())
        if mode in ferr:
            out[mode]["q_field_err"] = float(np.mean(ferr[mode]["q"]))
            out[mode]["u_field_err"] = float(np.mean(ferr[mode]["u"]))
    # Speed: each method over the whole horizon from seed 0's start, as one
    # call with one synchronisation (the runs above synchronise at every
    # observation; at large multipliers a span is a few macro steps and that
    # overhead is a sizeable share of it), after one untimed macro step; the
    # median of three runs.
    k_total = sum(spans)
    st0 = wl.initial_state(side, 1.0, 1.0, seed=3000 + seeds[0], kind="isotropic")
    wall = {}
    fallbacks_timed = 0
    for mode in ("plain", "plain_coarse", "learned"):
        q = p if mode != "plain_coarse" else p.replace(dt=mult * dt)
        sim = _sim([q], [n])

        def run(k):
            if mode == "plain":
                sim.step(k * mult)
                sim.sync()
                return 0
            if mode == "plain_coarse":
                sim.step(k)
                sim.sync()
                return 0
            return sim.step_learned(m, k, mult, tau)[0]

        sim.set_state(0, st0)
        run(1)
        reps = []
        for _ in range(3):                       # median of three
            sim.set_state(0, st0)
            torch.cuda.synchronize()
            c0 = time.perf_counter()
            nfb = run(k_total)
            torch.cuda.synchronize()
            reps.append(time.perf_counter() - c0)
            if mode == "learned":
                fallbacks_timed += nfb
        wall[mode] = sorted(reps)[1]
        sim.check()
        sim.close()
        _log(f"timed {mode} over {k_total} macro steps: " + " ".join(f"{t:.4f}" for t in reps) + " s")
    out["seconds_uninterrupted"] = wall
    out["speedup_learned_vs_plain"] = wall["plain"] / wall["learned"] if wall["learned"] > 0 else None
    out["speedup_coarse_vs_plain"] = wall["plain"] / wall["plain_coarse"] if wall["plain_coarse"] > 0 else None
    out["speedup_learned_vs_plain_interleaved"] = times["plain"] / times["learned"] if times["learned"] > 0 else None
    out["speedup_coarse_vs_plain_interleaved"] = (times["plain"] / times["plain_coarse"]
                                                  if times["plain_coarse"] > 0 else None)
    out["fallbacks"] = fallbacks
    out["fallbacks_timed"] = fallbacks_timed
    out["tau"] = tau
    return out


def run(mult=4, epochs=20, side=1024, seeds=4):
    """Build the training set, train, mask, set the fallback threshold and
    evaluate against plain stepping; returns the record main() prints."""
    t0 = time.perf_counter()
    X, T = training_set(mult=mult)
    t1 = time.perf_counter()
    _log(f"training set: {X.shape[0]} samples in {t1 - t0:.1f} s")
    m, loss = fit(X, T, epochs=epochs)
    t2 = time.perf_counter()
    _log(f"trained: loss {loss:.4g}, {t2 - t1:.1f} s")
    # held-out boxes: other seeds, same recipe, every particle
    Xh, Th = training_set(replicas=4, mult=mult, seed=1, per_replica=None)
    rel = held_out_errors(m, Xh, Th)
    _log(f"held-out relative MSE per output (dQxx, dQxy, dQyy, dux, duy): {[round(v, 4) for v in rel]}")
    masked = mask_unskilled(m, rel)
    rel_masked = held_out_errors(m, Xh, Th)
    tau = fallback_threshold(m, Xh)
    _log(f"masked outputs {masked}; held-out relative MSE after masking {[round(v, 4) for v in rel_masked]}; "
         f"tau {tau:.4g}")
    ev = evaluate(m, tau, side=side, seeds=tuple(range(seeds)), mult=mult)
    t3 = time.perf_counter()
    return {"samples": int(X.shape[0]), "mult": mult, "train_loss": loss,
            "held_out_rel_mse": rel, "masked_outputs": masked, "held_out_rel_mse_masked": rel_masked,
            "t_samples_s": t1 - t0, "t_train_s": t2 - t1, "t_eval_s": t3 - t2, **ev}


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--side", type=int, default=1024)
    ap.add_argument("--seeds", type=int, default=4)
    ap.add_argument("--mult", type=int, default=4)
    args = ap.parse_args()
    print(json.dumps(run(mult=args.mult, epochs=args.epochs, side=args.side, seeds=args.seeds)), flush=True)


if __name__ == "__main__":
    main()
