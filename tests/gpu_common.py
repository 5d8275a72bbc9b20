"""Helpers shared by the GPU parity tests: run the oracle and the HIP library
on the same seeded inputs and compare fields."""
import numpy as np

import oracle
import workloads as wl


def minimg(d, L):
    return d - L * np.round(d / L)


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def field_errors(g, o, s0, L, nsteps=None):
    """Per-field relative L2 errors of GPU fields g against oracle fields o
    (both dicts in id order). Position errors are measured on displacements
    from the start state s0 and on the absolute positions. With nsteps, the
    increment errors of increment_errors() are included as well."""
    e = {}
    if nsteps:
        e.update(increment_errors(g, o, s0, L, nsteps))
    dgx, dgy = minimg(g["x"] - s0["x"], L), minimg(g["y"] - s0["y"], L)
    dox, doy = minimg(o["x"] - s0["x"], L), minimg(o["y"] - s0["y"], L)
    ex, ey = minimg(g["x"] - o["x"], L), minimg(g["y"] - o["y"], L)
    e["pos_abs_max"] = float(max(np.abs(ex).max(), np.abs(ey).max()))
    e["pos"] = float(np.sqrt((ex ** 2 + ey ** 2).sum() / (o["x"] ** 2 + o["y"] ** 2).sum()))
    dn = np.sqrt((dox ** 2 + doy ** 2).sum())
    e["disp"] = float(np.sqrt(((dgx - dox) ** 2 + (dgy - doy) ** 2).sum()) / dn) if dn > 0 else float(
        np.abs(ex).max())
    e["u"] = rel_l2(np.concatenate([g["ux"], g["uy"]]), np.concatenate([o["ux"], o["uy"]]))
    e["Q"] = rel_l2(np.concatenate([g["qxx"], g["qxy"]]), np.concatenate([o["qxx"], o["qxy"]]))
    e["dQ"] = rel_l2(np.concatenate([g["qxx"] - s0["qxx"], g["qxy"] - s0["qxy"]]),
                     np.concatenate([o["qxx"] - s0["qxx"], o["qxy"] - s0["qxy"]]))
    e["rho"] = rel_l2(g["rho"], o["rho"])
    e["drho"] = rel_l2(g["rho"] - s0["rho"], o["rho"] - s0["rho"])
    e["a"] = rel_l2(np.concatenate([g["ax"], g["ay"]]), np.concatenate([o["ax"], o["ay"]]))
    return e


EPS32 = 2.0 ** -24   # unit roundoff of FP32 storage


def increment_errors(g, o, s0, L, nsteps):
    """Errors of the increments over a run, per field f in r, u, Q, rho (GPU g
    and oracle o against the common start s0, all in id order):
      d{f}_l2   ||df_g - df_o||_2 / ||df_o||_2 with df = f - f0 (minimum image
                for r), the relative L2 error of what the steps changed;
      d{f}_max  max_i |df_g - df_o|_i / max_i |df_o|_i, the largest element
                error relative to the largest increment;
      d{f}_res  max_i |df_g - df_o|_i / (nsteps * 2^-24 * max|f|), the same error
                in units of the FP32 resolution of the stored field per step
                (f: u and Q as stored; rho as rho - rho0, its stored form)."""
    def pair(a, b):
        return np.concatenate(a), np.concatenate(b)
    fields = {
        "r": pair([minimg(g["x"] - s0["x"], L), minimg(g["y"] - s0["y"], L)],
                  [minimg(o["x"] - s0["x"], L), minimg(o["y"] - s0["y"], L)]),
        "u": pair([g["ux"] - s0["ux"], g["uy"] - s0["uy"]], [o["ux"] - s0["ux"], o["uy"] - s0["uy"]]),
        "Q": pair([g["qxx"] - s0["qxx"], g["qxy"] - s0["qxy"]], [o["qxx"] - s0["qxx"], o["qxy"] - s0["qxy"]]),
        "rho": (g["rho"] - s0["rho"], o["rho"] - s0["rho"]),
    }
    scale = {
        "r": None,
        "u": max(np.abs(o["ux"]).max(), np.abs(o["uy"]).max()),
        "Q": max(np.abs(o["qxx"]).max(), np.abs(o["qxy"]).max()),
        "rho": np.abs(o["rho"] - 1.0).max(),
    }
    e = {}
    for f, (dg, do) in fields.items():
        err = np.abs(dg - do)
        e[f"d{f}_l2"] = float(np.linalg.norm(dg - do) / max(np.linalg.norm(do), 1e-300))
        e[f"d{f}_max"] = float(err.max() / max(np.abs(do).max(), 1e-300))
        if scale[f] is not None:
            e[f"d{f}_res"] = float(err.max() / (nsteps * EPS32 * max(scale[f], 1e-300)))
    return e


# Bars on the increments of an n-step run (the DESIGN parity section derives them):
# * u and Q are stored in FP32, so every step rounds them once: an element of
#   the increment can be off by about n * 2^-24 * max|f| before any arithmetic
#   error; held to RES_BAR times that;
# * rho is stored as rho - rho0 and its increment comes from the continuity
#   rate's FP32 pair sums: relative L2 and largest-element error <= DRHO_BAR;
# * positions are compensated (hi + lo) FP32 offsets: displacement errors
#   relative to the displacements <= DR_BAR.
RES_BAR = 4.0
DRHO_BAR = 3e-5
DR_BAR = 1e-5


def check_increments(e):
    for k, bar in (("du_res", RES_BAR), ("dQ_res", RES_BAR), ("drho_l2", DRHO_BAR), ("drho_max", DRHO_BAR),
                   ("dr_l2", DR_BAR), ("dr_max", DR_BAR)):
        assert e[k] <= bar, (k, e[k], bar)


def run_oracle(params, s0, nsteps, search=2):
    """The oracle over nsteps steps. search = 2: each pair's neighbour decision
    in FP32 on cell-relative offsets, the library's rule (an integer decision
    that floating point takes is taken in the same precision on both sides);
    every other operation stays FP64."""
    st = oracle.State(s0)
    if nsteps:
        oracle.step(params, st, nsteps, search=search)
    f = st.fields()
    return f, st


def random_state(L, seed, amp_u=1e-3, jitter=0.2, drho=1e-4):
    x, y = wl.jittered_lattice(L, 1.0, jitter, seed)
    ux, uy = wl.smooth_velocity(x, y, float(L), amp_u, seed)
    th = wl.director_angles(x.size, seed, "isotropic")
    qxx, qxy = wl.order_tensor(th)
    rng = np.random.default_rng(seed + 7)
    return dict(x=x, y=y, ux=ux, uy=uy, qxx=qxx, qxy=qxy, rho=1.0 + drho * rng.normal(size=x.size),
                ax=np.zeros_like(x), ay=np.zeros_like(x))


def gpu_run(params, s0, nsteps, opts=None):
    import paper_2108_08919_amd as P
    sim = P.Sim([params], [s0["x"].size])
    for k, v in (opts or {}).items():
        sim.set_option(k, v)
    sim.set_state(0, s0)
    if nsteps:
        sim.step(nsteps)
    sim.check()
    g = sim.get_state(0)
    return g, sim
