"""Learned corrector: training data from the solver, training, evaluation.

Every numerical step runs in the library (nem_samples, nem_mlp_fit_norm,
nem_mlp_train, nem_step_learned, nem_diagnostics, nem_defects); this module
only schedules the calls and collects the results.

Workloads:
* training: 16 replicas of a 256 x 256 lattice box with (zeta, K) drawn from
  U[0.005, 0.04] x U[0.01, 0.08] (seeded), isotropic director start; at four
  times t in {0.25, 0.75, 1.25, 1.75} every replica contributes the inputs and
  the (4 dt fine) - (one 4 dt step) targets of a seeded subset of 16,384 of its
  particles: 4 x 16 x 16,384 = 1,048,576 samples;
* held out: 4 more replicas from other seeds, same recipe; the network's mean
  squared error per output relative to the output's variance (1 = no better
  than no correction);
* evaluation: the 1024 x 1024 box at zeta = K = 0.02 over t in [0, 2] from four
  seeded isotropic starts: plain steps of dt = 1e-3 (reference), plain steps of
  4 dt, and learned macro steps of 4 dt; the errors are those of the ensemble-
  and time-averaged kinetic energy and defect density over t in [1, 2], and
  the relative L2 errors of the final fields against the plain-dt run from the
  same start (Q relative to its change over the run, u relative to its size).

The fallback threshold tau is the 99.9th percentile of the training
corrections' norm in the network's normalised output units; a macro step whose
largest predicted correction norm exceeds it is replayed as 4 fine steps.
Output components with no skill on the held-out boxes (relative MSE not below
1) are switched off before the evaluation, so they contribute no correction.

Run: python -m paper_2108_08919_amd.learned  (prints one JSON line)
"""
from __future__ import annotations

import json
import math
import sys
import time

import numpy as np


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _sim(params, n):
    from . import Sim
    return Sim(params, n)


def training_set(side=256, replicas=16, times=(0.25, 0.75, 1.25, 1.75), per_replica=16384, mult=4, seed=0,
                 dt=1e-3):
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
    sim = _sim(params, [n] * replicas)
    for r in range(replicas):
        sim.set_state(r, states[r])
    Xs, Ts = [], []
    t = 0.0
    for tk in times:
        k = int(round((tk - t) / dt))
        sim.step(k)
        t = tk
        X, T = sim.samples(mult)
        pick = []
        for r in range(replicas):
            sel = rng.choice(n, per_replica, replace=False)
            pick.append(torch.from_numpy(np.sort(sel) + r * n))
        idx = torch.cat(pick).to(X.device)
        Xs.append(X[idx])
        Ts.append(T[idx])
    sim.check()
    sim.close()
    return torch.cat(Xs).contiguous(), torch.cat(Ts).contiguous()


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
    """Train a network on (X, T); returns (mlp, final batch loss, tau) where tau
    is the 99.9th percentile of the norm of the training corrections T in the
    network's normalised output units (the fallback threshold)."""
    import torch
    from . import Mlp
    m = Mlp()
    m.set_weights(init_weights(seed))
    m.fit_norm(X, T)
    loss = m.train(X, T, epochs=epochs, batch=batch, lr=lr)
    nm = torch.from_numpy(m.get_norm()).to(X.device)
    z = (T - nm[24:29]) / nm[29:34]
    tau = float(torch.quantile(z.norm(dim=1)[:: max(1, X.shape[0] // 200000)], 0.999).item())
    return m, loss, tau


def mask_unskilled(m, rel, threshold=1.0):
    """Switch off the output components whose held-out relative MSE is not
    below `threshold` (no better than no correction): their last-layer weights,
    bias and output mean are set to zero, so the network returns exactly zero
    for them. Returns the masked component indices."""
    w = m.get_weights()
    nm = m.get_norm()
    off_w3 = 12 * 64 + 64 + 64 * 64 + 64          # W3 (64 x 5, input-major), then b3 (5)
    off_b3 = off_w3 + 64 * 5
    masked = [o for o, r in enumerate(rel) if not r < threshold]
    for o in masked:
        w[off_w3 + o: off_b3: 5] = 0.0
        w[off_b3 + o] = 0.0
        nm[24 + o] = 0.0
    m.set_weights(w)
    m.set_norm(nm)
    return masked


def held_out_errors(m, X, T):
    """Per-output mean squared error of the network on (X, T) relative to the
    variance of T (1 = no better than predicting the mean, 0 = exact)."""
    Y = m.forward(X).double()
    Td = T.double()
    return (((Td - Y) ** 2).mean(0) / Td.var(0, unbiased=False)).tolist()


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


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--side", type=int, default=1024)
    ap.add_argument("--seeds", type=int, default=4)
    ap.add_argument("--mult", type=int, default=4)
    args = ap.parse_args()
    t0 = time.perf_counter()
    X, T = training_set(mult=args.mult)
    t1 = time.perf_counter()
    _log(f"training set: {X.shape[0]} samples in {t1 - t0:.1f} s")
    m, loss, tau = fit(X, T, epochs=args.epochs)
    t2 = time.perf_counter()
    _log(f"trained: loss {loss:.4g}, tau {tau:.3g}, {t2 - t1:.1f} s")
    # held-out samples: other seeds, same recipe
    Xh, Th = training_set(replicas=4, mult=args.mult, seed=1)
    rel = held_out_errors(m, Xh, Th)
    _log(f"held-out relative MSE per output (dQxx, dQxy, dQyy, dux, duy): {[round(v, 4) for v in rel]}")
    masked = mask_unskilled(m, rel)
    rel_masked = held_out_errors(m, Xh, Th)
    _log(f"masked outputs {masked}; held-out relative MSE after masking {[round(v, 4) for v in rel_masked]}")
    ev = evaluate(m, tau, side=args.side, seeds=tuple(range(args.seeds)), mult=args.mult)
    t3 = time.perf_counter()
    print(json.dumps({"samples": int(X.shape[0]), "mult": args.mult, "train_loss": loss,
                      "held_out_rel_mse": rel, "masked_outputs": masked, "held_out_rel_mse_masked": rel_masked,
                      "t_samples_s": t1 - t0,
                      "t_train_s": t2 - t1, "t_eval_s": t3 - t2, **ev}), flush=True)


if __name__ == "__main__":
    main()
