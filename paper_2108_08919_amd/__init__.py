"""Python binding of the MI355X SPH active-nematic library (libnematic_sph.so).

Argument marshalling only: every step of the method runs in the HIP kernels of
libnematic_sph.so, whose C ABI is include/nematic_sph.h. PyTorch provides the
device arena (a uint8 tensor) and the stream. The functions keep the C names
(nem_create, nem_step, ...); `Sim` wraps them for convenience.

Importing torch before the library matters: torch's HIP runtime then serves
both, so torch streams and allocations are valid handles for the library.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnematic_sph.so")

NEM_OK = 0
NEM_E_INVAL = -1
NEM_E_NOMEM = -2
NEM_E_HIP = -3
NEM_E_NUMERIC = -4
NEM_E_OVERFLOW = -5
NEM_E_SINGULAR = -6
NEM_E_STATE = -7
NEM_E_RANGE = -8

NEM_OPT_TILE = 1
NEM_OPT_LPP = 2
NEM_OPT_COMP = 3
NEM_OPT_TIMING = 4
NEM_OPT_GRAPH = 5
NEM_OPT_PERSIST = 6
NEM_NPASS = 5
PASS_NAMES = ("rebin", "pass_a_volume", "pass_b_rates", "pass_c_eos", "pass_d_update")

EXPORTED = ("nem_version", "nem_arena_bytes", "nem_create", "nem_set_state", "nem_get_state", "nem_step",
            "nem_sync", "nem_neighbors", "nem_diagnostics", "nem_deposit", "nem_spectrum", "nem_defects",
            "nem_set_option", "nem_pass_times", "nem_strerror", "nem_last_error", "nem_destroy",
            "nem_mlp_nparams", "nem_mlp_create", "nem_mlp_set_weights", "nem_mlp_get_weights", "nem_mlp_set_norm",
            "nem_mlp_get_norm", "nem_mlp_fit_norm", "nem_mlp_forward", "nem_mlp_grad", "nem_mlp_train",
            "nem_mlp_destroy", "nem_samples", "nem_step_learned", "nem_autotune", "nem_vorticity_correlation",
            "nem_track", "nem_mixing", "nem_set_qyy", "nem_get_qyy", "nem_neighbor_list",
            "nem_defects_noalloc", "nem_get_option", "nem_mlp_eval", "nem_mlp_mask_outputs", "nem_samples_rows",
            "nem_raw_bytes", "nem_save_raw", "nem_load_raw")


class NemParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("L", "dx", "h", "rho0", "eta", "Gamma", "lam", "A", "B", "C", "K",
                                          "zeta", "dt", "gamma_eos", "beta", "c0_factor", "skin")] + \
               [(k, C.c_int32) for k in ("form", "elastic", "apd", "kernel", "integrator", "q3d")]


class NemDiag(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("px", "py", "ke", "F", "F_grad", "umax", "c0", "qmax")]


class NemError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        self.code = code
        super().__init__(f"{what} failed: {code} ({strerror(code)}) {detail}".strip())


_lib = None


def lib(path: Optional[str] = None):
    """Load libnematic_sph.so (never builds; raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    try:
        import torch  # noqa: F401  (load torch's HIP runtime first, see module docstring)
    except Exception:
        pass
    L = C.CDLL(p)
    dp = C.POINTER(C.c_double)
    vp = C.c_void_p
    L.nem_version.restype = C.c_int
    L.nem_arena_bytes.restype = C.c_int
    L.nem_arena_bytes.argtypes = [C.POINTER(NemParams), C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_uint64)]
    L.nem_create.restype = C.c_int
    L.nem_create.argtypes = [C.POINTER(NemParams), C.POINTER(C.c_int64), C.c_int32, vp, C.c_uint64, vp,
                             C.POINTER(vp)]
    L.nem_set_state.restype = C.c_int
    L.nem_set_state.argtypes = [vp, C.c_int32] + [dp] * 9
    L.nem_get_state.restype = C.c_int
    L.nem_get_state.argtypes = [vp, C.c_int32] + [dp] * 9
    L.nem_step.restype = C.c_int
    L.nem_step.argtypes = [vp, C.c_int64]
    L.nem_sync.restype = C.c_int
    L.nem_sync.argtypes = [vp]
    L.nem_raw_bytes.restype = C.c_int
    L.nem_raw_bytes.argtypes = [vp, C.POINTER(C.c_uint64)]
    L.nem_save_raw.restype = C.c_int
    L.nem_save_raw.argtypes = [vp, vp, C.c_uint64]
    L.nem_load_raw.restype = C.c_int
    L.nem_load_raw.argtypes = [vp, vp, C.c_uint64]
    L.nem_neighbors.restype = C.c_int
    L.nem_neighbors.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.c_int64,
                                C.POINTER(C.c_int64)]
    L.nem_neighbor_list.restype = C.c_int
    L.nem_neighbor_list.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                    C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_float)]
    L.nem_diagnostics.restype = C.c_int
    L.nem_diagnostics.argtypes = [vp, C.c_int32, C.POINTER(NemDiag)]
    L.nem_deposit.restype = C.c_int
    L.nem_deposit.argtypes = [vp, C.c_int32, C.c_int32, dp]
    L.nem_spectrum.restype = C.c_int
    L.nem_spectrum.argtypes = [vp, C.c_int32, C.c_int32, dp, C.c_int32, C.c_int32, C.c_int32, dp]
    L.nem_defects.restype = C.c_int
    L.nem_defects.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.nem_defects_noalloc.restype = C.c_int
    L.nem_defects_noalloc.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.nem_vorticity_correlation.restype = C.c_int
    L.nem_vorticity_correlation.argtypes = [vp, C.c_int32, C.c_int32, dp, dp, dp, dp]
    L.nem_set_qyy.restype = C.c_int
    L.nem_set_qyy.argtypes = [vp, C.c_int32, dp]
    L.nem_get_qyy.restype = C.c_int
    L.nem_get_qyy.argtypes = [vp, C.c_int32, dp]
    L.nem_track.restype = C.c_int
    L.nem_track.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.c_int32, dp, dp]
    L.nem_mixing.restype = C.c_int
    L.nem_mixing.argtypes = [vp, C.c_int32, C.POINTER(C.c_uint8), C.c_int32, C.c_int32, C.POINTER(C.c_int64), dp]
    L.nem_set_option.restype = C.c_int
    L.nem_set_option.argtypes = [vp, C.c_int32, C.c_int64]
    L.nem_get_option.restype = C.c_int
    L.nem_get_option.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64)]
    L.nem_pass_times.restype = C.c_int
    L.nem_pass_times.argtypes = [vp, dp, C.POINTER(C.c_int64), C.c_int32]
    fp = C.POINTER(C.c_float)
    L.nem_mlp_nparams.restype = C.c_int
    L.nem_mlp_create.restype = C.c_int
    L.nem_mlp_create.argtypes = [vp, C.POINTER(vp)]
    for name in ("nem_mlp_set_weights", "nem_mlp_get_weights", "nem_mlp_set_norm", "nem_mlp_get_norm"):
        getattr(L, name).restype = C.c_int
        getattr(L, name).argtypes = [vp, fp]
    L.nem_mlp_fit_norm.restype = C.c_int
    L.nem_mlp_fit_norm.argtypes = [vp, vp, vp, C.c_int64]
    L.nem_mlp_forward.restype = C.c_int
    L.nem_mlp_forward.argtypes = [vp, vp, C.c_int64, vp]
    L.nem_mlp_grad.restype = C.c_int
    L.nem_mlp_grad.argtypes = [vp, vp, vp, C.c_int64, fp, dp]
    L.nem_mlp_train.restype = C.c_int
    L.nem_mlp_train.argtypes = [vp, vp, vp, C.c_int64, C.c_int32, C.c_int32, C.c_double, dp]
    L.nem_mlp_destroy.restype = None
    L.nem_mlp_destroy.argtypes = [vp]
    L.nem_samples.restype = C.c_int
    L.nem_samples.argtypes = [vp, C.c_int32, vp, vp]
    L.nem_samples_rows.restype = C.c_int
    L.nem_samples_rows.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), C.c_int64, vp, vp]
    L.nem_mlp_eval.restype = C.c_int
    L.nem_mlp_eval.argtypes = [vp, vp, vp, C.c_int64, dp, dp]
    L.nem_mlp_mask_outputs.restype = C.c_int
    L.nem_mlp_mask_outputs.argtypes = [vp, C.POINTER(C.c_int32)]
    L.nem_step_learned.restype = C.c_int
    L.nem_step_learned.argtypes = [vp, vp, C.c_int64, C.c_int32, C.c_double, C.POINTER(C.c_int64), dp]
    L.nem_autotune.restype = C.c_int
    L.nem_autotune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), dp]
    L.nem_strerror.restype = C.c_char_p
    L.nem_strerror.argtypes = [C.c_int]
    L.nem_last_error.restype = C.c_char_p
    L.nem_last_error.argtypes = [vp]
    L.nem_destroy.restype = None
    L.nem_destroy.argtypes = [vp]
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return lib().nem_strerror(code).decode()
    except ImportError:
        return "library not loaded"


def make_params(p) -> NemParams:
    """From workloads.Params (or any object with the same attribute names)."""
    return NemParams(L=p.L, dx=p.dx, h=p.h, rho0=p.rho0, eta=p.eta, Gamma=p.Gamma, lam=p.lam, A=p.A, B=p.B,
                     C=p.C, K=p.K, zeta=p.zeta, dt=p.dt, gamma_eos=p.gamma_eos, beta=p.beta,
                     c0_factor=p.c0_factor, skin=p.skin, form=p.form, elastic=p.elastic, apd=p.apd, kernel=p.kernel,
                     integrator=p.integrator, q3d=getattr(p, "q3d", 0))


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ---------------------------------------------------------------- C names

def nem_version() -> int:
    return lib().nem_version()


def nem_arena_bytes(params: Sequence, n: Sequence[int]) -> int:
    R = len(params)
    arr = (NemParams * R)(*[make_params(p) for p in params])
    nn = (C.c_int64 * R)(*[int(v) for v in n])
    out = C.c_uint64(0)
    rc = lib().nem_arena_bytes(arr, nn, R, C.byref(out))
    if rc:
        raise NemError(rc, "nem_arena_bytes")
    return int(out.value)


def nem_create(params: Sequence, n: Sequence[int], arena_ptr: int, arena_bytes: int, stream: int) -> int:
    R = len(params)
    arr = (NemParams * R)(*[make_params(p) for p in params])
    nn = (C.c_int64 * R)(*[int(v) for v in n])
    h = C.c_void_p(0)
    rc = lib().nem_create(arr, nn, R, C.c_void_p(arena_ptr or None), arena_bytes, C.c_void_p(stream or None),
                          C.byref(h))
    if rc:
        raise NemError(rc, "nem_create")
    return h.value


def _check(h, rc, what):
    if rc:
        detail = lib().nem_last_error(C.c_void_p(h)).decode() if h else ""
        raise NemError(rc, what, detail)


def nem_set_state(h, r, x, y, ux, uy, qxx, qxy, rho, ax=None, ay=None):
    arrs = [np.ascontiguousarray(v, dtype=np.float64) if v is not None else None
            for v in (x, y, ux, uy, qxx, qxy, rho, ax, ay)]
    _check(h, lib().nem_set_state(C.c_void_p(h), r, *[_dp(a) for a in arrs]), "nem_set_state")


def nem_get_state(h, r, n) -> Dict[str, np.ndarray]:
    out = {k: np.zeros(n) for k in ("x", "y", "ux", "uy", "qxx", "qxy", "rho", "ax", "ay")}
    _check(h, lib().nem_get_state(C.c_void_p(h), r, *[_dp(out[k]) for k in
                                                     ("x", "y", "ux", "uy", "qxx", "qxy", "rho", "ax", "ay")]),
           "nem_get_state")
    return out


def nem_step(h, nsteps: int):
    _check(h, lib().nem_step(C.c_void_p(h), int(nsteps)), "nem_step")


def nem_sync(h) -> int:
    return lib().nem_sync(C.c_void_p(h))


def nem_neighbors(h, r, n):
    rp = np.zeros(n + 1, dtype=np.int64)
    nnz = C.c_int64(0)
    cap = 64 * n
    while True:
        col = np.zeros(max(cap, 1), dtype=np.int32)
        rc = lib().nem_neighbors(C.c_void_p(h), r, rp.ctypes.data_as(C.POINTER(C.c_int64)),
                                 col.ctypes.data_as(C.POINTER(C.c_int32)), cap, C.byref(nnz))
        if rc == NEM_E_NOMEM and nnz.value > cap:
            cap = int(nnz.value)
            continue
        _check(h, rc, "nem_neighbors")
        return rp, col[:nnz.value].copy()


def nem_neighbor_list(h, r, n, which=0, offsets=False):
    """CSR (row_ptr, col) of the pairs the passes walk (which 0) or of the
    Verlet list (which 1); with offsets, also (cell_xy (n, 2) int32,
    off_xy (n, 2) float32), the predicate's inputs."""
    rp = np.zeros(n + 1, dtype=np.int64)
    nnz = C.c_int64(0)
    cap = 64 * n
    cxy = np.zeros((n, 2), dtype=np.int32) if offsets else None
    oxy = np.zeros((n, 2), dtype=np.float32) if offsets else None
    while True:
        col = np.zeros(max(cap, 1), dtype=np.int32)
        rc = lib().nem_neighbor_list(C.c_void_p(h), r, which, rp.ctypes.data_as(C.POINTER(C.c_int64)),
                                     col.ctypes.data_as(C.POINTER(C.c_int32)), cap, C.byref(nnz),
                                     None if cxy is None else cxy.ctypes.data_as(C.POINTER(C.c_int32)),
                                     None if oxy is None else oxy.ctypes.data_as(C.POINTER(C.c_float)))
        if rc == NEM_E_NOMEM and nnz.value > cap:
            cap = int(nnz.value)
            continue
        _check(h, rc, "nem_neighbor_list")
        out = (rp, col[:nnz.value].copy())
        return out + (cxy, oxy) if offsets else out


def nem_diagnostics(h, r) -> Dict[str, float]:
    d = NemDiag()
    _check(h, lib().nem_diagnostics(C.c_void_p(h), r, C.byref(d)), "nem_diagnostics")
    return {k: getattr(d, k) for k, _ in NemDiag._fields_}


def nem_deposit(h, r, M):
    out = np.zeros((4, M, M))
    _check(h, lib().nem_deposit(C.c_void_p(h), r, M, _dp(out)), "nem_deposit")
    return out


def nem_spectrum(h, r, M, k_lo: int = 0, k_hi: int = 0):
    nb = int(np.floor(np.sqrt(2.0) * (M // 2) + 0.5)) + 1
    E = np.zeros(nb)
    sl = C.c_double(0.0)
    _check(h, lib().nem_spectrum(C.c_void_p(h), r, M, _dp(E), nb, k_lo, k_hi, C.byref(sl)), "nem_spectrum")
    return E, sl.value


def nem_defects(h, r, M):
    a, b = C.c_int64(0), C.c_int64(0)
    _check(h, lib().nem_defects(C.c_void_p(h), r, M, C.byref(a), C.byref(b)), "nem_defects")
    return a.value, b.value


def nem_defects_noalloc(h, r, M):
    a, b = C.c_int64(0), C.c_int64(0)
    _check(h, lib().nem_defects_noalloc(C.c_void_p(h), r, M, C.byref(a), C.byref(b)), "nem_defects_noalloc")
    return a.value, b.value


def nem_vorticity_correlation(h, r, M):
    cx = np.zeros(M // 2 + 1)
    cy = np.zeros(M // 2 + 1)
    lx, ly = C.c_double(0), C.c_double(0)
    _check(h, lib().nem_vorticity_correlation(C.c_void_p(h), r, M, _dp(cx), _dp(cy), C.byref(lx), C.byref(ly)),
           "nem_vorticity_correlation")
    return cx, cy, lx.value, ly.value


def nem_track(h, r, ids):
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    x = np.zeros(ids.size)
    y = np.zeros(ids.size)
    _check(h, lib().nem_track(C.c_void_p(h), r, ids.ctypes.data_as(C.POINTER(C.c_int32)), ids.size, _dp(x), _dp(y)),
           "nem_track")
    return x, y


def nem_mixing(h, r, colour, ncol, B):
    colour = np.ascontiguousarray(colour, dtype=np.uint8)
    counts = np.zeros(B * B * ncol, dtype=np.int64)
    idx = C.c_double(0)
    _check(h, lib().nem_mixing(C.c_void_p(h), r, colour.ctypes.data_as(C.POINTER(C.c_uint8)), ncol, B,
                               counts.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(idx)), "nem_mixing")
    return idx.value, counts.reshape(B, B, ncol)


def nem_set_option(h, key: int, value: int):
    _check(h, lib().nem_set_option(C.c_void_p(h), key, int(value)), "nem_set_option")


def nem_save_raw(h) -> np.ndarray:
    nb = C.c_uint64(0)
    _check(h, lib().nem_raw_bytes(C.c_void_p(h), C.byref(nb)), "nem_raw_bytes")
    buf = np.empty(nb.value, dtype=np.uint8)
    _check(h, lib().nem_save_raw(C.c_void_p(h), buf.ctypes.data_as(C.c_void_p), nb.value), "nem_save_raw")
    return buf


def nem_load_raw(h, buf):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(h, lib().nem_load_raw(C.c_void_p(h), buf.ctypes.data_as(C.c_void_p), buf.size), "nem_load_raw")


def nem_get_option(h, key: int) -> int:
    v = C.c_int64(0)
    _check(h, lib().nem_get_option(C.c_void_p(h), key, C.byref(v)), "nem_get_option")
    return v.value


def nem_pass_times(h, reset: bool = False):
    ms = np.zeros(NEM_NPASS)
    cnt = np.zeros(NEM_NPASS, dtype=np.int64)
    _check(h, lib().nem_pass_times(C.c_void_p(h), _dp(ms), cnt.ctypes.data_as(C.POINTER(C.c_int64)),
                                   1 if reset else 0), "nem_pass_times")
    return ms, cnt


def nem_destroy(h):
    if h:
        lib().nem_destroy(C.c_void_p(h))


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _mcheck(rc, what):
    if rc:
        raise NemError(rc, what)


class Mlp:
    """The learned corrector's network (BF16 MFMA kernels, FP32 master weights).
    Device arrays are torch float32 tensors on the GPU."""

    NI, NO = 12, 5

    def __init__(self, stream=None):
        import torch
        lib()
        st = stream if stream is not None else torch.cuda.current_stream()
        self.stream = st
        h = C.c_void_p(0)
        _mcheck(lib().nem_mlp_create(C.c_void_p(st.cuda_stream or None), C.byref(h)), "nem_mlp_create")
        self.h = h.value
        self.nparams = lib().nem_mlp_nparams()

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.size == self.nparams
        _mcheck(lib().nem_mlp_set_weights(C.c_void_p(self.h), _fp(w)), "nem_mlp_set_weights")

    def get_weights(self):
        w = np.zeros(self.nparams, dtype=np.float32)
        _mcheck(lib().nem_mlp_get_weights(C.c_void_p(self.h), _fp(w)), "nem_mlp_get_weights")
        return w

    def set_norm(self, norm):
        nm = np.ascontiguousarray(norm, dtype=np.float32)
        assert nm.size == 34
        _mcheck(lib().nem_mlp_set_norm(C.c_void_p(self.h), _fp(nm)), "nem_mlp_set_norm")

    def get_norm(self):
        nm = np.zeros(34, dtype=np.float32)
        _mcheck(lib().nem_mlp_get_norm(C.c_void_p(self.h), _fp(nm)), "nem_mlp_get_norm")
        return nm

    def fit_norm(self, X, T):
        _mcheck(lib().nem_mlp_fit_norm(C.c_void_p(self.h), C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                       X.shape[0]), "nem_mlp_fit_norm")

    def forward(self, X):
        import torch
        Y = torch.empty((X.shape[0], self.NO), dtype=torch.float32, device=X.device)
        _mcheck(lib().nem_mlp_forward(C.c_void_p(self.h), C.c_void_p(X.data_ptr()), X.shape[0],
                                      C.c_void_p(Y.data_ptr())), "nem_mlp_forward")
        return Y

    def grad(self, X, T):
        g = np.zeros(self.nparams, dtype=np.float32)
        loss = C.c_double(0)
        _mcheck(lib().nem_mlp_grad(C.c_void_p(self.h), C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                   X.shape[0], _fp(g), C.byref(loss)), "nem_mlp_grad")
        return g, loss.value

    def train(self, X, T, epochs: int, batch: int, lr: float) -> float:
        loss = C.c_double(0)
        _mcheck(lib().nem_mlp_train(C.c_void_p(self.h), C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                    X.shape[0], epochs, batch, lr, C.byref(loss)), "nem_mlp_train")
        return loss.value

    def evaluate(self, X, T=None):
        """(per-output relative MSE against T or None, largest predicted
        correction norm in normalised units) on the device inputs X."""
        rel = np.zeros(self.NO) if T is not None else None
        mx = C.c_double(0)
        _mcheck(lib().nem_mlp_eval(C.c_void_p(self.h), C.c_void_p(X.data_ptr()),
                                   C.c_void_p(T.data_ptr()) if T is not None else None, X.shape[0],
                                   _dp(rel) if rel is not None else None, C.byref(mx)), "nem_mlp_eval")
        return (rel.tolist() if rel is not None else None), mx.value

    def mask_outputs(self, outputs):
        """Switch off the given output components (they return exactly zero)."""
        off = (C.c_int32 * self.NO)(*[1 if o in set(outputs) else 0 for o in range(self.NO)])
        _mcheck(lib().nem_mlp_mask_outputs(C.c_void_p(self.h), off), "nem_mlp_mask_outputs")

    def close(self):
        if getattr(self, "h", None):
            lib().nem_mlp_destroy(C.c_void_p(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- wrapper

class Sim:
    """R periodic boxes advanced together. The device arena is a torch uint8
    tensor on `device`; work goes to torch's current stream on that device."""

    def __init__(self, params: Sequence, n: Sequence[int], device: str = "cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the nematic SPH library runs only on the GPU")
        lib()
        self.params = list(params)
        self.n = [int(v) for v in n]
        self.R = len(self.params)
        self.device = torch.device(device)
        nbytes = nem_arena_bytes(self.params, self.n)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = nem_create(self.params, self.n, self.arena.data_ptr(), nbytes, self.stream.cuda_stream)

    def set_state(self, r: int, f: Dict[str, np.ndarray]):
        nem_set_state(self.h, r, f["x"], f["y"], f["ux"], f["uy"], f["qxx"], f["qxy"], f["rho"],
                      f.get("ax"), f.get("ay"))
        if getattr(self.params[r], "q3d", 0) and "qyy" in f:
            self.set_qyy(r, f["qyy"])

    def get_state(self, r: int = 0) -> Dict[str, np.ndarray]:
        out = nem_get_state(self.h, r, self.n[r])
        if getattr(self.params[r], "q3d", 0):
            out["qyy"] = self.get_qyy(r)
            out["qzz"] = -out["qxx"] - out["qyy"]
        return out

    def set_qyy(self, r: int, qyy):
        """Qyy of the quasi-2D variant (after set_state)."""
        a = np.ascontiguousarray(qyy, dtype=np.float64)
        if a.size != self.n[r]:
            raise ValueError("one value per particle")
        _check(self.h, lib().nem_set_qyy(C.c_void_p(self.h), r, _dp(a)), "nem_set_qyy")

    def get_qyy(self, r: int = 0):
        a = np.zeros(self.n[r])
        _check(self.h, lib().nem_get_qyy(C.c_void_p(self.h), r, _dp(a)), "nem_get_qyy")
        return a

    def step(self, nsteps: int):
        nem_step(self.h, nsteps)

    def sync(self) -> int:
        return nem_sync(self.h)

    def check(self):
        rc = self.sync()
        _check(self.h, rc, "nem_sync")

    def neighbors(self, r: int = 0):
        return nem_neighbors(self.h, r, self.n[r])

    def neighbor_list(self, r: int = 0, which: int = 0, offsets: bool = False):
        return nem_neighbor_list(self.h, r, self.n[r], which, offsets)

    def diagnostics(self, r: int = 0):
        return nem_diagnostics(self.h, r)

    def deposit(self, r: int = 0, M: int = 0):
        return nem_deposit(self.h, r, M or int(self.params[r].L))

    def spectrum(self, r: int = 0, M: int = 0, k_lo: int = 0, k_hi: int = 0):
        return nem_spectrum(self.h, r, M or int(self.params[r].L), k_lo, k_hi)

    def defects(self, r: int = 0, M: int = 0):
        return nem_defects(self.h, r, M or int(self.params[r].L))

    def defects_noalloc(self, r: int = 0, M: int = 0):
        """nem_defects on the library's static scratch (no allocation; M <= 512)."""
        return nem_defects_noalloc(self.h, r, M or int(self.params[r].L))

    def vorticity_correlation(self, r: int = 0, M: int = 0):
        """(C_x, C_y, l_x, l_y): vorticity autocorrelation along x and y on the
        M x M deposit grid and their first zero crossings (length units)."""
        return nem_vorticity_correlation(self.h, r, M or int(self.params[r].L))

    def track(self, ids, r: int = 0):
        """Unwrapped positions (x, y) of the particles `ids` at the integer time level."""
        return nem_track(self.h, r, ids)

    def mixing(self, colour, ncol: int, B: int, r: int = 0):
        """(mixing index, counts[by, bx, colour]) of the colouring `colour` (by id) on B x B bins."""
        if len(colour) != self.n[r]:
            raise ValueError("one colour per particle")
        return nem_mixing(self.h, r, colour, ncol, B)

    def vrms(self, r: int = 0):
        """Root mean square speed over the particles, sqrt(2 KE) with
        KE = sum |u|^2 / (2N) at the integer time level."""
        return float(np.sqrt(2.0 * nem_diagnostics(self.h, r)["ke"]))

    def samples(self, mult: int = 4):
        """Training inputs X (ntot x 12) and targets T (ntot x 5) at the current state."""
        import torch
        N = sum(self.n)
        X = torch.empty((N, 12), dtype=torch.float32, device=self.device)
        T = torch.empty((N, 5), dtype=torch.float32, device=self.device)
        _check(self.h, lib().nem_samples(C.c_void_p(self.h), mult, C.c_void_p(X.data_ptr()),
                                         C.c_void_p(T.data_ptr())), "nem_samples")
        return X, T

    def samples_rows(self, rows, mult: int = 4, X=None, T=None):
        """Training inputs and targets of the particles `rows` (indices into all
        replicas' particles, part_base + id) only, into X and T when given
        (contiguous device tensors of len(rows) x 12 and x 5)."""
        import torch
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        if X is None:
            X = torch.empty((rows.size, 12), dtype=torch.float32, device=self.device)
        if T is None:
            T = torch.empty((rows.size, 5), dtype=torch.float32, device=self.device)
        assert X.is_contiguous() and T.is_contiguous() and X.shape == (rows.size, 12) and T.shape == (rows.size, 5)
        _check(self.h, lib().nem_samples_rows(C.c_void_p(self.h), mult, rows.ctypes.data_as(C.POINTER(C.c_int64)),
                                              rows.size, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr())),
               "nem_samples_rows")
        return X, T

    def step_learned(self, mlp: "Mlp", n_macro: int, mult: int = 4, tau: float = 1e30):
        nfb = C.c_int64(0)
        mx = C.c_double(0)
        _check(self.h, lib().nem_step_learned(C.c_void_p(self.h), C.c_void_p(mlp.h), n_macro, mult, tau,
                                              C.byref(nfb), C.byref(mx)), "nem_step_learned")
        return nfb.value, mx.value

    def autotune(self, steps: int = 5):
        """Pick the fastest (tile, lanes per particle) on the current state; returns (tile, lpp, ms/step)."""
        t, l = C.c_int32(0), C.c_int32(0)
        ms = C.c_double(0)
        _check(self.h, lib().nem_autotune(C.c_void_p(self.h), steps, C.byref(t), C.byref(l), C.byref(ms)),
               "nem_autotune")
        return t.value, l.value, ms.value

    def set_option(self, key: int, value: int):
        nem_set_option(self.h, key, value)

    def save_raw(self) -> np.ndarray:
        """Bitwise checkpoint of every replica (bytes as a uint8 array)."""
        return nem_save_raw(self.h)

    def load_raw(self, buf):
        """Continue from a checkpoint of a simulation with the same replicas."""
        nem_load_raw(self.h, buf)

    def checkpoint(self, path: str):
        """Write the bitwise checkpoint to a file."""
        self.save_raw().tofile(path)

    def restore(self, path: str):
        """Load a checkpoint file written by checkpoint()."""
        self.load_raw(np.fromfile(path, dtype=np.uint8))

    def save_fields(self, path: str):
        """Every replica's fields at the integer time level (FP64, particle-id
        order) in one .npz archive, keys '<field>_<replica>': a portable record
        that set_state can start from (not bitwise: see checkpoint)."""
        out = {}
        for r in range(len(self.n)):
            for k, v in self.get_state(r).items():
                out[f"{k}_{r}"] = v
        np.savez(path, **out)

    def get_option(self, key: int) -> int:
        return nem_get_option(self.h, key)

    def pass_times(self, reset: bool = False):
        return nem_pass_times(self.h, reset)

    def close(self):
        if getattr(self, "h", None):
            nem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
