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


def field_errors(g, o, s0, L):
    """Per-field relative L2 errors of GPU fields g against oracle fields o
    (both dicts in id order). Position errors are measured on displacements
    from the start state s0 and on the absolute positions."""
    e = {}
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


def run_oracle(params, s0, nsteps, search=0):
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
