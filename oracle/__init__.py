"""FP64 CPU oracle of the SPH active-nematic step (TEST INFRASTRUCTURE).

Only tests/, the smoke check and bench.py's cpu_baseline leg may import this
package. It is a plain double-precision implementation of the paper's
Sec. 3-3.1 written for checking, not for speed, and shares no code with the
HIP library. The C part lives in orc.c; this module is ctypes marshalling plus
the grid diagnostics in diag.py.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class OrcParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("L", "dx", "h", "rho0", "eta", "Gamma", "lam", "A", "B", "C", "K", "zeta",
                 "dt", "gamma_eos", "beta", "c0_factor", "skin")] + \
               [(k, C.c_int32) for k in ("form", "elastic", "apd", "search", "kernel", "integrator", "q3d")]


class OrcState(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.POINTER(C.c_double)) for k in
                                     ("x", "y", "ux", "uy", "q", "rho", "ax", "ay", "qzz")]


class OrcDiag(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("px", "py", "ke", "F", "F_grad", "umax", "trq_max",
                                          "asym_max", "c0_last")]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liborc.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.orc_W.restype = C.c_double; L.orc_W.argtypes = [C.c_int32, C.c_double, C.c_double]
        L.orc_dWdr.restype = C.c_double; L.orc_dWdr.argtypes = [C.c_int32, C.c_double, C.c_double]
        L.orc_kappa.restype = C.c_double; L.orc_kappa.argtypes = [C.c_int32]
        L.orc_eos.restype = C.c_double; L.orc_eos.argtypes = [C.c_double] * 4
        L.orc_neighbors.restype = C.c_int64
        L.orc_neighbors.argtypes = [C.POINTER(OrcParams), C.c_int64, dp, dp, C.c_int32, C.c_int32,
                                    C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.c_int64]
        L.orc_neighbors_offsets.restype = C.c_int64
        L.orc_neighbors_offsets.argtypes = [C.POINTER(OrcParams), C.c_int64, C.c_int32, C.POINTER(C.c_int32),
                                            C.POINTER(C.c_float), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                            C.c_int64]
        L.orc_operators.restype = C.c_int
        L.orc_operators.argtypes = [C.POINTER(OrcParams), C.c_int64, dp, dp, dp, dp, dp, dp, dp]
        L.orc_corotation.restype = None; L.orc_corotation.argtypes = [C.c_double, dp, dp, dp]
        L.orc_corotation3.restype = None; L.orc_corotation3.argtypes = [C.c_double, dp, dp, dp]
        L.orc_molecular_field3.restype = None
        L.orc_molecular_field3.argtypes = [C.POINTER(OrcParams), dp, dp, dp]
        L.orc_molecular_field.restype = None
        L.orc_molecular_field.argtypes = [C.POINTER(OrcParams), dp, dp, dp]
        L.orc_elastic_stress.restype = None
        L.orc_elastic_stress.argtypes = [C.c_double, dp, dp, dp]
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [C.POINTER(OrcParams), C.POINTER(OrcState), C.c_int64, C.POINTER(OrcDiag)]
        L.orc_diagnostics.restype = C.c_int
        L.orc_diagnostics.argtypes = [C.POINTER(OrcParams), C.POINTER(OrcState), C.POINTER(OrcDiag)]
        L.orc_step_fields.restype = C.c_int
        L.orc_step_fields.argtypes = [C.POINTER(OrcParams), C.POINTER(OrcState)] + [dp] * 7
        L.orc_deposit.restype = C.c_int
        L.orc_deposit.argtypes = [C.POINTER(OrcParams), C.c_int64, dp, dp, C.c_int32,
                                  C.POINTER(dp), C.c_int32, dp]
        L.orc_num_threads.restype = C.c_int
        _LIB = L
    return _LIB


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(p, search: int = 0) -> OrcParams:
    """From a workloads.Params (or any object with the same attribute names)."""
    return OrcParams(L=p.L, dx=p.dx, h=p.h, rho0=p.rho0, eta=p.eta, Gamma=p.Gamma, lam=p.lam,
                     A=p.A, B=p.B, C=p.C, K=p.K, zeta=p.zeta, dt=p.dt, gamma_eos=p.gamma_eos,
                     beta=p.beta, c0_factor=p.c0_factor, skin=p.skin, form=p.form,
                     elastic=p.elastic, apd=p.apd, search=search, kernel=getattr(p, "kernel", 0),
                     integrator=getattr(p, "integrator", 0), q3d=getattr(p, "q3d", 0))


def W(h: float, r: float, kernel: int = 0) -> float:
    return lib().orc_W(kernel, h, r)


def dWdr(h: float, r: float, kernel: int = 0) -> float:
    return lib().orc_dWdr(kernel, h, r)


def kappa(kernel: int = 0) -> float:
    return lib().orc_kappa(kernel)


def eos(rho, rho0, c0, gamma_eos):
    return lib().orc_eos(rho, rho0, c0, gamma_eos)


def num_threads() -> int:
    return lib().orc_num_threads()


class State:
    """Oracle state in particle-id order; Q kept with four components."""

    def __init__(self, fields: Dict[str, np.ndarray]):
        n = fields["x"].size
        self.n = n
        f = lambda k: np.ascontiguousarray(fields[k], dtype=np.float64).copy()
        self.x, self.y, self.ux, self.uy = f("x"), f("y"), f("ux"), f("uy")
        self.rho, self.ax, self.ay = f("rho"), f("ax"), f("ay")
        self.q = np.zeros((n, 4))
        self.q[:, 0] = fields["qxx"]; self.q[:, 1] = fields["qxy"]
        self.q[:, 2] = fields["qxy"]; self.q[:, 3] = -np.asarray(fields["qxx"])
        if "qyx" in fields:
            self.q[:, 2] = fields["qyx"]
        if "qyy" in fields:
            self.q[:, 3] = fields["qyy"]
        # quasi-2D 3x3 Q: Qzz kept as its own component (None for the d = 2 reading)
        self.qzz = f("qzz") if "qzz" in fields else None

    def c(self) -> OrcState:
        return OrcState(n=self.n, x=_dp(self.x), y=_dp(self.y), ux=_dp(self.ux), uy=_dp(self.uy),
                        q=_dp(self.q), rho=_dp(self.rho), ax=_dp(self.ax), ay=_dp(self.ay), qzz=_dp(self.qzz))

    def fields(self) -> Dict[str, np.ndarray]:
        out = dict(x=self.x.copy(), y=self.y.copy(), ux=self.ux.copy(), uy=self.uy.copy(),
                   qxx=self.q[:, 0].copy(), qxy=self.q[:, 1].copy(), qyx=self.q[:, 2].copy(),
                   qyy=self.q[:, 3].copy(), rho=self.rho.copy(), ax=self.ax.copy(), ay=self.ay.copy())
        if self.qzz is not None:
            out["qzz"] = self.qzz.copy()
        return out


def step(params, state: State, nsteps: int, search: int = 0) -> OrcDiag:
    cp = make_params(params, search)
    st = state.c()
    info = OrcDiag()
    rc = lib().orc_step(C.byref(cp), C.byref(st), nsteps, C.byref(info))
    if rc != 0:
        raise RuntimeError(f"orc_step failed: {rc}")
    return info


def diagnostics(params, state: State, search: int = 0) -> Dict[str, float]:
    cp = make_params(params, search)
    st = state.c()
    d = OrcDiag()
    rc = lib().orc_diagnostics(C.byref(cp), C.byref(st), C.byref(d))
    if rc != 0:
        raise RuntimeError(f"orc_diagnostics failed: {rc}")
    return {k: getattr(d, k) for k, _ in OrcDiag._fields_}


def step_fields(params, state: State, search: int = 0) -> Dict[str, np.ndarray]:
    n = state.n
    out = dict(V=np.zeros(n), k=np.zeros(n), rho_hat=np.zeros(n), p=np.zeros(n),
               m=np.zeros((n, 4)), a=np.zeros((n, 2)), dr_apd=np.zeros((n, 2)))
    cp = make_params(params, search)
    st = state.c()
    rc = lib().orc_step_fields(C.byref(cp), C.byref(st), _dp(out["V"]), _dp(out["k"]),
                               _dp(out["rho_hat"]), _dp(out["p"]), _dp(out["m"]), _dp(out["a"]),
                               _dp(out["dr_apd"]))
    if rc < 0:
        raise RuntimeError(f"orc_step_fields failed: {rc}")
    return out


def neighbors(params, x, y, mode: int = 0, nc: int = 0):
    """CSR (row_ptr, col) by particle index, rows ascending."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = x.size
    cap = max(64 * n, 16)
    while True:
        rp = np.zeros(n + 1, dtype=np.int64)
        col = np.zeros(cap, dtype=np.int32)
        cp = make_params(params)
        nnz = lib().orc_neighbors(C.byref(cp), n, _dp(x), _dp(y), mode, nc,
                                  rp.ctypes.data_as(C.POINTER(C.c_int64)),
                                  col.ctypes.data_as(C.POINTER(C.c_int32)), cap)
        if nnz == -2:
            cap *= 4
            continue
        if nnz < 0:
            raise RuntimeError(f"orc_neighbors failed: {nnz}")
        return rp, col[:nnz].copy()


def neighbors_offsets(params, nc: int, cell_xy, off_xy):
    """CSR of the FP32 predicate on given cell coordinates (n, 2) and FP32
    cell-relative offsets (n, 2)."""
    cxy = np.ascontiguousarray(cell_xy, dtype=np.int32)
    oxy = np.ascontiguousarray(off_xy, dtype=np.float32)
    n = cxy.shape[0]
    cap = max(64 * n, 16)
    while True:
        rp = np.zeros(n + 1, dtype=np.int64)
        col = np.zeros(cap, dtype=np.int32)
        cp = make_params(params)
        nnz = lib().orc_neighbors_offsets(C.byref(cp), n, nc, cxy.ctypes.data_as(C.POINTER(C.c_int32)),
                                          oxy.ctypes.data_as(C.POINTER(C.c_float)),
                                          rp.ctypes.data_as(C.POINTER(C.c_int64)),
                                          col.ctypes.data_as(C.POINTER(C.c_int32)), cap)
        if nnz == -2:
            cap *= 4
            continue
        if nnz < 0:
            raise RuntimeError(f"orc_neighbors_offsets failed: {nnz}")
        return rp, col[:nnz].copy()


def operators(params, x, y, f=None, search: int = 0):
    """V, B (n,2,2), corrected gradient (n,2) and Laplacian (n) of scalar f."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = x.size
    V = np.zeros(n); B = np.zeros((n, 4)); g = np.zeros((n, 2)); lap = np.zeros(n)
    fa = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
    cp = make_params(params, search)
    rc = lib().orc_operators(C.byref(cp), n, _dp(x), _dp(y), _dp(fa), _dp(V), _dp(B), _dp(g), _dp(lap))
    if rc != 0:
        raise RuntimeError(f"orc_operators failed: {rc}")
    return V, B.reshape(n, 2, 2), g, lap


def corotation(lam: float, Q, G):
    Q = np.ascontiguousarray(np.asarray(Q, dtype=np.float64).reshape(4))
    G = np.ascontiguousarray(np.asarray(G, dtype=np.float64).reshape(4))
    S = np.zeros(4)
    lib().orc_corotation(lam, _dp(Q), _dp(G), _dp(S))
    return S.reshape(2, 2)


def corotation3(lam: float, Q, G):
    """Quasi-2D co-rotation (3x3 Q, I/3) for an in-plane 2x2 velocity gradient G."""
    Q = np.ascontiguousarray(np.asarray(Q, dtype=np.float64).reshape(9))
    G = np.ascontiguousarray(np.asarray(G, dtype=np.float64).reshape(4))
    S = np.zeros(9)
    lib().orc_corotation3(lam, _dp(Q), _dp(G), _dp(S))
    return S.reshape(3, 3)


def molecular_field3(params, Q, lapQ):
    Q = np.ascontiguousarray(np.asarray(Q, dtype=np.float64).reshape(9))
    lq = np.ascontiguousarray(np.asarray(lapQ, dtype=np.float64).reshape(9))
    H = np.zeros(9)
    cp = make_params(params)
    lib().orc_molecular_field3(C.byref(cp), _dp(Q), _dp(lq), _dp(H))
    return H.reshape(3, 3)


def molecular_field(params, Q, lapQ):
    Q = np.ascontiguousarray(np.asarray(Q, dtype=np.float64).reshape(4))
    lq = np.ascontiguousarray(np.asarray(lapQ, dtype=np.float64).reshape(4))
    H = np.zeros(4)
    cp = make_params(params)
    lib().orc_molecular_field(C.byref(cp), _dp(Q), _dp(lq), _dp(H))
    return H.reshape(2, 2)


def elastic_stress(lam: float, Q, H):
    """lambda part of the elastic stress (2x2) for Q and H (2x2 each)."""
    Q = np.ascontiguousarray(np.asarray(Q, dtype=np.float64).reshape(4))
    H = np.ascontiguousarray(np.asarray(H, dtype=np.float64).reshape(4))
    Pi = np.zeros(4)
    lib().orc_elastic_stress(lam, _dp(Q), _dp(H), _dp(Pi))
    return Pi.reshape(2, 2)


def deposit(params, x, y, fields, M: int):
    """Shepard interpolation of a list of fields onto an M x M grid (out[f, j, i])."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    fs = [np.ascontiguousarray(f, dtype=np.float64) for f in fields]
    arr = (C.POINTER(C.c_double) * len(fs))(*[_dp(f) for f in fs])
    out = np.zeros((len(fs), M, M))
    cp = make_params(params)
    rc = lib().orc_deposit(C.byref(cp), x.size, _dp(x), _dp(y), len(fs), arr, M, _dp(out))
    if rc != 0:
        raise RuntimeError(f"orc_deposit failed: {rc}")
    return out
