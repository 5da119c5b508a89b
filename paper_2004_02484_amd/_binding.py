"""ctypes binding of libnmpc.so: argument marshalling only."""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libnmpc.so")

NMPC_OK = 0
NMPC_E_ARG = 1
NMPC_E_NOCONV = 2
NMPC_E_NONFINITE = 3
NMPC_E_DEVICE = 4
NMPC_E_OOM = 5
NMPC_E_UNSUPPORTED = 6
NMPC_FP64 = 0
NMPC_FP32_SWEEP = 1
NMPC_UPPER_JACOBI = 0
NMPC_UPPER_FGS = 1
NMPC_UPPER_BGS = 2
NMPC_UPPER_SGS = 3
NMPC_PATH_AUTO = 0
NMPC_PATH_FUSED = 1
NMPC_PATH_STREAM = 2
NMPC_RES_SCALED = 0
NMPC_RES_PAPER = 1
NMPC_MODEL_HEAT = 0
NMPC_MODEL_PLATE = 1
NMPC_MODEL_WAVE = 2
NMPC_BC_DIRICHLET = 0
NMPC_BC_NEUMANN = 1

_dp = ctypes.POINTER(ctypes.c_double)


class nmpc_problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nsx", ctypes.c_int32), ("nsy", ctypes.c_int32),
                ("horizon", ctypes.c_int32), ("lx", ctypes.c_int32), ("ly", ctypes.c_int32),
                ("gx", _dp), ("gy", _dp),
                ("h", ctypes.c_double), ("k0", ctypes.c_double), ("k1", ctypes.c_double),
                ("q", ctypes.c_double), ("r", ctypes.c_double), ("gamma", ctypes.c_double),
                ("tau", ctypes.c_double), ("u_lo", ctypes.c_double), ("u_hi", ctypes.c_double),
                ("b_kind", ctypes.c_int32), ("B", _dp)]


NMPC_B_DENSE = 0
NMPC_B_KRON = 1


class nmpc_options(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("n_sweep", ctypes.c_int32), ("n_schur", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("xref_per_stage", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("warm_sweeps", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("upper", ctypes.c_int32), ("path", ctypes.c_int32),
                ("omega", ctypes.c_double), ("fp32_finish", ctypes.c_int32),
                ("residual", ctypes.c_int32), ("warm_sweeps_lambda", ctypes.c_int32)]


class nmpc_model_problem(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("boundary", ctypes.c_int32),
                ("nsx", ctypes.c_int32), ("nsy", ctypes.c_int32), ("horizon", ctypes.c_int32),
                ("n_inputs", ctypes.c_int32), ("act", ctypes.POINTER(ctypes.c_int32)),
                ("B", _dp), ("h", ctypes.c_double), ("q", ctypes.c_double),
                ("qv", ctypes.c_double), ("r", ctypes.c_double), ("gamma", ctypes.c_double),
                ("tau", ctypes.c_double), ("u_lo", ctypes.c_double), ("u_hi", ctypes.c_double),
                ("u_cold", ctypes.c_double), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("rad", ctypes.c_double), ("t_amb", ctypes.c_double),
                ("k0", ctypes.c_double), ("k1", ctypes.c_double), ("damp", ctypes.c_double)]


class nmpc_info(ctypes.Structure):
    _fields_ = [("r_scaled", ctypes.c_double), ("r_paper", ctypes.c_double),
                ("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("fp32_iters", ctypes.c_int32), ("start_used", ctypes.c_int32),
                ("err_vs_fp64", ctypes.c_double)]

    def as_dict(self):
        return {"r_scaled": self.r_scaled, "r_paper": self.r_paper, "iters": self.iters,
                "status": self.status, "fp32_iters": self.fp32_iters,
                "start_used": self.start_used, "err_vs_fp64": self.err_vs_fp64}


# nmpc_info as a numpy record: batched calls return one structured array (the
# library writes into it directly; infos[b]["iters"], infos["iters"]), which
# costs nothing per instance, unlike a list of dicts.
INFO_DTYPE = np.dtype([(name, np.float64 if ct is ctypes.c_double else np.int32)
                       for name, ct in nmpc_info._fields_], align=True)
assert INFO_DTYPE.itemsize == ctypes.sizeof(nmpc_info)


def _info_array(count: int):
    a = np.zeros(count, dtype=INFO_DTYPE)
    return a, a.ctypes.data_as(ctypes.POINTER(nmpc_info))


class NmpcError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {nmpc_strerror(code)} ({code}) {nmpc_last_error()}")


_lib = None


def library_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with "
                          "`python -m paper_2004_02484_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(_LIB_PATH)
    vp = ctypes.c_void_p
    lib.nmpc_default_options.argtypes = [ctypes.POINTER(nmpc_options)]
    lib.nmpc_default_options.restype = None
    lib.nmpc_create.argtypes = [ctypes.POINTER(nmpc_problem), ctypes.POINTER(nmpc_options),
                                ctypes.c_int32, ctypes.POINTER(vp)]
    lib.nmpc_create.restype = ctypes.c_int
    lib.nmpc_set_options.argtypes = [vp, ctypes.POINTER(nmpc_options)]
    lib.nmpc_set_options.restype = ctypes.c_int
    lib.nmpc_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(nmpc_info)]
    lib.nmpc_solve.restype = ctypes.c_int
    lib.nmpc_solve_batch.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp,
                                     ctypes.POINTER(nmpc_info), vp]
    lib.nmpc_solve_batch.restype = ctypes.c_int
    lib.nmpc_residual_batch.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.nmpc_residual_batch.restype = ctypes.c_int
    lib.nmpc_destroy.argtypes = [vp]
    lib.nmpc_destroy.restype = None
    lib.nmpc_strerror.argtypes = [ctypes.c_int]
    lib.nmpc_strerror.restype = ctypes.c_char_p
    lib.nmpc_last_error.argtypes = []
    lib.nmpc_last_error.restype = ctypes.c_char_p
    lib.nmpc_kernel_config.argtypes = [vp, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]
    lib.nmpc_kernel_config.restype = ctypes.c_int
    lib.nmpc_timing_enable.argtypes = [vp, ctypes.c_int32]
    lib.nmpc_timing_enable.restype = ctypes.c_int
    lib.nmpc_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int64)]
    lib.nmpc_timing_read.restype = ctypes.c_int
    lib.nmpc_timing_read_eval.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.nmpc_timing_read_eval.restype = ctypes.c_int
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.nmpc_shift_batch.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp]
    lib.nmpc_shift_batch.restype = ctypes.c_int
    lib.nmpc_plant_step_batch.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_int32,
                                          ctypes.c_double, vp, vp]
    lib.nmpc_plant_step_batch.restype = ctypes.c_int
    lib.nmpc_autotune.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_int32, vp, i32p]
    lib.nmpc_autotune.restype = ctypes.c_int
    lib.nmpc_ragged_create.argtypes = [ctypes.POINTER(nmpc_problem), ctypes.c_int32,
                                       ctypes.POINTER(nmpc_options), ctypes.c_int32,
                                       ctypes.POINTER(vp)]
    lib.nmpc_ragged_create.restype = ctypes.c_int
    lib.nmpc_ragged_solve.argtypes = [vp, ctypes.c_int32, i32p, vp, vp, vp, vp, vp, vp, vp, vp,
                                      ctypes.POINTER(nmpc_info), vp]
    lib.nmpc_ragged_solve.restype = ctypes.c_int
    lib.nmpc_ragged_autotune.argtypes = [vp, ctypes.c_int32, i32p, vp, vp, ctypes.c_int32, vp,
                                         i32p]
    lib.nmpc_ragged_autotune.restype = ctypes.c_int
    lib.nmpc_ragged_config.argtypes = [vp, ctypes.c_int32, i32p, i32p]
    lib.nmpc_ragged_config.restype = ctypes.c_int
    lib.nmpc_ragged_timing_enable.argtypes = [vp, ctypes.c_int32]
    lib.nmpc_ragged_timing_enable.restype = ctypes.c_int
    lib.nmpc_ragged_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int64)]
    lib.nmpc_ragged_timing_read.restype = ctypes.c_int
    lib.nmpc_ragged_timing_read_eval.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.nmpc_ragged_timing_read_eval.restype = ctypes.c_int
    lib.nmpc_ragged_destroy.argtypes = [vp]
    lib.nmpc_ragged_destroy.restype = None
    lib.nmpc_model_create.argtypes = [ctypes.POINTER(nmpc_model_problem),
                                      ctypes.POINTER(nmpc_options), ctypes.c_int32,
                                      ctypes.POINTER(vp)]
    lib.nmpc_model_create.restype = ctypes.c_int
    lib.nmpc_model_set_options.argtypes = [vp, ctypes.POINTER(nmpc_options)]
    lib.nmpc_model_set_options.restype = ctypes.c_int
    lib.nmpc_model_solve_batch.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp,
                                           ctypes.POINTER(nmpc_info), vp]
    lib.nmpc_model_solve_batch.restype = ctypes.c_int
    lib.nmpc_model_residual_batch.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp,
                                              vp]
    lib.nmpc_model_residual_batch.restype = ctypes.c_int
    lib.nmpc_model_timing_enable.argtypes = [vp, ctypes.c_int32]
    lib.nmpc_model_timing_enable.restype = ctypes.c_int
    lib.nmpc_model_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_int64)]
    lib.nmpc_model_timing_read.restype = ctypes.c_int
    lib.nmpc_model_destroy.argtypes = [vp]
    lib.nmpc_model_destroy.restype = None
    _lib = lib
    return lib


# ------------------------------------------------------------- C-named calls

def nmpc_strerror(code: int) -> str:
    return _load().nmpc_strerror(int(code)).decode()


def nmpc_last_error() -> str:
    return _load().nmpc_last_error().decode()


def nmpc_default_options(**overrides) -> nmpc_options:
    o = nmpc_options()
    _load().nmpc_default_options(ctypes.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


class _Problem:
    """nmpc_problem plus the host arrays it points at (kept alive here)."""

    def __init__(self, p):
        self.gx = np.ascontiguousarray(p.gx, dtype=np.float64)
        self.gy = np.ascontiguousarray(p.gy, dtype=np.float64)
        dense = getattr(p, "B", None)
        self.B = None if dense is None else np.ascontiguousarray(dense, dtype=np.float64)
        self.s = nmpc_problem(int(p.dim), int(p.nsx), int(p.nsy), int(p.N), int(p.lx), int(p.ly),
                              self.gx.ctypes.data_as(_dp), self.gy.ctypes.data_as(_dp),
                              float(p.h), float(p.k0), float(p.k1), float(p.q), float(p.r),
                              float(p.gamma), float(getattr(p, "tau", 0.0)),
                              float(getattr(p, "u_lo", 0.0)), float(getattr(p, "u_hi", 0.0)),
                              NMPC_B_KRON if self.B is None else NMPC_B_DENSE,
                              None if self.B is None else self.B.ctypes.data_as(_dp))


def nmpc_create(problem, options: nmpc_options, max_batch: int = 1) -> ctypes.c_void_p:
    """problem: any object with dim, nsx, nsy, N, lx, ly, gx, gy, h, k0, k1, q, r, gamma."""
    pr = _Problem(problem)
    hd = ctypes.c_void_p()
    rc = _load().nmpc_create(ctypes.byref(pr.s), ctypes.byref(options), int(max_batch),
                             ctypes.byref(hd))
    if rc != NMPC_OK:
        raise NmpcError(rc, "nmpc_create")
    return hd


def nmpc_set_options(hd, options: nmpc_options) -> None:
    rc = _load().nmpc_set_options(hd, ctypes.byref(options))
    if rc != NMPC_OK:
        raise NmpcError(rc, "nmpc_set_options")


def nmpc_destroy(hd) -> None:
    if hd:
        _load().nmpc_destroy(hd)


def _host(a, size, name):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != size:
        raise ValueError(f"{name}: expected {size} values, got {a.size}")
    return a


def nmpc_solve(hd, x0, xref, warm=None, *, n: int, m: int, N: int, xref_stages: bool = False):
    """Host-buffer solve. Returns (status, X [N,n], U [N,m], LAM [N,n], info dict)."""
    x0 = _host(x0, n, "x0")
    xref = _host(xref, n * (N if xref_stages else 1), "xref")
    X = np.empty((N, n)); U = np.empty((N, m)); L = np.empty((N, n))
    ws = [None, None, None]
    if warm is not None:
        ws = [None if warm[0] is None else _host(warm[0], N * n, "warm x"),
              None if warm[1] is None else _host(warm[1], N * m, "warm u"),
              None if warm[2] is None else _host(warm[2], N * n, "warm lam")]
    info = nmpc_info()
    ptr = lambda a: None if a is None else a.ctypes.data
    rc = _load().nmpc_solve(hd, x0.ctypes.data, xref.ctypes.data, ptr(ws[0]), ptr(ws[1]),
                            ptr(ws[2]), X.ctypes.data, U.ctypes.data, L.ctypes.data,
                            ctypes.byref(info))
    if rc not in (NMPC_OK, NMPC_E_NOCONV, NMPC_E_NONFINITE):
        raise NmpcError(rc, "nmpc_solve")
    return rc, X, U, L, info.as_dict()


def _dev(t, shape, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise ValueError(f"{name}: need a contiguous float64 device tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)} != {tuple(shape)}")
    return t.data_ptr()


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def nmpc_solve_batch(hd, x0, xref, warm=None, out=None, *, n: int, m: int, N: int,
                     xref_stages: bool = False):
    """Device-tensor solve of count = x0.shape[0] instances on torch's current
    stream. Returns (status, X, U, LAM, infos): infos is a numpy structured
    array of nmpc_info records (INFO_DTYPE)."""
    import torch
    B = x0.shape[0]
    xs = (B, N, n) if xref_stages else (B, n)
    px0 = _dev(x0, (B, n), "x0")
    pxr = _dev(xref, xs, "xref")
    if out is None:
        out = (torch.empty((B, N, n), dtype=torch.float64, device=x0.device),
               torch.empty((B, N, m), dtype=torch.float64, device=x0.device),
               torch.empty((B, N, n), dtype=torch.float64, device=x0.device))
    po = [_dev(out[0], (B, N, n), "out x"), _dev(out[1], (B, N, m), "out u"),
          _dev(out[2], (B, N, n), "out lam")]
    pw = [None, None, None]
    if warm is not None:
        pw = [None if warm[0] is None else _dev(warm[0], (B, N, n), "warm x"),
              None if warm[1] is None else _dev(warm[1], (B, N, m), "warm u"),
              None if warm[2] is None else _dev(warm[2], (B, N, n), "warm lam")]
    infos, pinfo = _info_array(B)
    rc = _load().nmpc_solve_batch(hd, B, px0, pxr, pw[0], pw[1], pw[2], po[0], po[1], po[2],
                                  pinfo, _stream())
    if rc not in (NMPC_OK, NMPC_E_NOCONV, NMPC_E_NONFINITE):
        raise NmpcError(rc, "nmpc_solve_batch")
    return rc, out[0], out[1], out[2], infos


def nmpc_residual_batch(hd, x0, xref, X, U, LAM, *, n: int, m: int, N: int,
                        xref_stages: bool = False):
    """(r_scaled [B], r_paper [B]) numpy arrays for device trajectories."""
    B = x0.shape[0]
    xs = (B, N, n) if xref_stages else (B, n)
    rs = np.zeros(B); rp = np.zeros(B)
    rc = _load().nmpc_residual_batch(hd, B, _dev(x0, (B, n), "x0"), _dev(xref, xs, "xref"),
                                     _dev(X, (B, N, n), "x"), _dev(U, (B, N, m), "u"),
                                     _dev(LAM, (B, N, n), "lam"), rs.ctypes.data,
                                     rp.ctypes.data, _stream())
    if rc != NMPC_OK:
        raise NmpcError(rc, "nmpc_residual_batch")
    return rs, rp


def nmpc_kernel_config(hd):
    r = ctypes.c_int32(); w = ctypes.c_int32(); g = ctypes.c_int32()
    rc = _load().nmpc_kernel_config(hd, ctypes.byref(r), ctypes.byref(w), ctypes.byref(g))
    if rc != NMPC_OK:
        raise NmpcError(rc, "nmpc_kernel_config")
    return {"rows_per_lane": r.value, "waves": w.value, "workgroups": g.value}


def nmpc_timing_enable(hd, enable: bool = True) -> None:
    rc = _load().nmpc_timing_enable(hd, 1 if enable else 0)
    if rc != NMPC_OK:
        raise NmpcError(rc, "nmpc_timing_enable")


def nmpc_timing_read(hd):
    ms = ctypes.c_double(); la = ctypes.c_int64(); un = ctypes.c_int64()
    ev = ctypes.c_int64()
    rc = _load().nmpc_timing_read(hd, ctypes.byref(ms), ctypes.byref(la), ctypes.byref(un))
    if rc == NMPC_OK:
        rc = _load().nmpc_timing_read_eval(hd, ctypes.byref(ev))
    if rc != NMPC_OK:
        raise NmpcError(rc, "nmpc_timing_read")
    return {"kernel_ms": ms.value, "launches": la.value, "units": un.value,
            "eval_units": ev.value}


def nmpc_shift_batch(hd, X, U, LAM, out=None, *, n: int, m: int, N: int, **_):
    """Shifted start (s_i <- s_{i+1}, last stage repeated) of device trajectories."""
    import torch
    B = X.shape[0]
    if out is None:
        out = (torch.empty_like(X), torch.empty_like(U), torch.empty_like(LAM))
    rc = _load().nmpc_shift_batch(hd, B, _dev(X, (B, N, n), "x"), _dev(U, (B, N, m), "u"),
                                  _dev(LAM, (B, N, n), "lam"), _dev(out[0], (B, N, n), "out x"),
                                  _dev(out[1], (B, N, m), "out u"),
                                  _dev(out[2], (B, N, n), "out lam"), _stream())
    if rc != NMPC_OK:
        raise NmpcError(rc, "nmpc_shift_batch")
    return out


def nmpc_plant_step_batch(hd, x, U, dt: float, out=None, *, n: int, m: int, N: int, **_):
    """x+ = x + dt f(u_1, x) for device x [B, n] and trajectories U [B, N, m]."""
    import torch
    B = x.shape[0]
    if out is None:
        out = torch.empty_like(x)
    rc = _load().nmpc_plant_step_batch(hd, B, _dev(x, (B, n), "x"), _dev(U, (B, N, m), "u"),
                                       N * m, float(dt), _dev(out, (B, n), "out"), _stream())
    if rc != NMPC_OK:
        raise NmpcError(rc, "nmpc_plant_step_batch")
    return out


def nmpc_autotune(hd, x0, xref, iters: int = 8, *, n: int, m: int, N: int,
                  xref_stages: bool = False) -> int:
    """Time the tile heights on this batch; returns the chosen tile_rows."""
    B = x0.shape[0]
    if xref_stages:
        raise ValueError("nmpc_autotune takes one xref per instance")
    tr = ctypes.c_int32()
    rc = _load().nmpc_autotune(hd, B, _dev(x0, (B, n), "x0"), _dev(xref, (B, n), "xref"),
                               int(iters), _stream(), ctypes.byref(tr))
    if rc != NMPC_OK:
        raise NmpcError(rc, "nmpc_autotune")
    return tr.value


def nmpc_ragged_create(classes, options: nmpc_options, max_instances: int):
    """classes: problem objects as for nmpc_create. Returns (handle, keep-alive)."""
    prs = [_Problem(c) for c in classes]
    arr = (nmpc_problem * len(prs))(*[p.s for p in prs])
    hd = ctypes.c_void_p()
    rc = _load().nmpc_ragged_create(arr, len(prs), ctypes.byref(options), int(max_instances),
                                    ctypes.byref(hd))
    if rc != NMPC_OK:
        raise NmpcError(rc, "nmpc_ragged_create")
    return hd, prs


def _cls_array(cls):
    c = np.ascontiguousarray(cls, dtype=np.int32)
    return c, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def nmpc_ragged_solve(hd, cls, x0, xref, warm, out, sizes):
    """Packed device tensors (1-D float64): x0, xref, out = (x, u, lam), warm
    None or (x, u, lam). sizes = (sum n_b, sum N_b n_b, sum N_b m)."""
    nx, nS, nU = sizes
    c, cp = _cls_array(cls)
    px0 = _dev(x0, (nx,), "x0")
    pxr = _dev(xref, (nx,), "xref")
    po = [_dev(out[0], (nS,), "out x"), _dev(out[1], (nU,), "out u"),
          _dev(out[2], (nS,), "out lam")]
    pw = [None, None, None]
    if warm is not None:
        pw = [_dev(warm[0], (nS,), "warm x"), _dev(warm[1], (nU,), "warm u"),
              _dev(warm[2], (nS,), "warm lam")]
    infos, pinfo = _info_array(len(c))
    rc = _load().nmpc_ragged_solve(hd, len(c), cp, px0, pxr, pw[0], pw[1], pw[2], po[0], po[1],
                                   po[2], pinfo, _stream())
    if rc not in (NMPC_OK, NMPC_E_NOCONV, NMPC_E_NONFINITE):
        raise NmpcError(rc, "nmpc_ragged_solve")
    return rc, infos


def nmpc_ragged_autotune(hd, cls, x0, xref, nx: int, iters: int = 8) -> int:
    c, cp = _cls_array(cls)
    w = ctypes.c_int32()
    rc = _load().nmpc_ragged_autotune(hd, len(c), cp, _dev(x0, (nx,), "x0"),
                                      _dev(xref, (nx,), "xref"), int(iters), _stream(),
                                      ctypes.byref(w))
    if rc != NMPC_OK:
        raise NmpcError(rc, "nmpc_ragged_autotune")
    return w.value


def nmpc_ragged_config(hd, cls) -> int:
    c, cp = _cls_array(cls)
    w = ctypes.c_int32()
    rc = _load().nmpc_ragged_config(hd, len(c), cp, ctypes.byref(w))
    if rc != NMPC_OK:
        raise NmpcError(rc, "nmpc_ragged_config")
    return w.value


def nmpc_ragged_timing_enable(hd, enable: bool = True) -> None:
    rc = _load().nmpc_ragged_timing_enable(hd, 1 if enable else 0)
    if rc != NMPC_OK:
        raise NmpcError(rc, "nmpc_ragged_timing_enable")


def nmpc_ragged_timing_read(hd):
    ms = ctypes.c_double(); la = ctypes.c_int64(); un = ctypes.c_int64()
    ev = ctypes.c_int64()
    rc = _load().nmpc_ragged_timing_read(hd, ctypes.byref(ms), ctypes.byref(la), ctypes.byref(un))
    if rc == NMPC_OK:
        rc = _load().nmpc_ragged_timing_read_eval(hd, ctypes.byref(ev))
    if rc != NMPC_OK:
        raise NmpcError(rc, "nmpc_ragged_timing_read")
    return {"kernel_ms": ms.value, "launches": la.value, "units": un.value,
            "eval_units": ev.value}


def nmpc_ragged_destroy(hd) -> None:
    if hd:
        _load().nmpc_ragged_destroy(hd)


# ------------------------------------------------------------- convenience

class Solver:
    """Owns one handle; methods forward to the C-named calls above."""

    def __init__(self, problem, *, max_batch: int = 1, **options):
        _load()
        self.problem = problem
        self.n = int(problem.nsx) * int(problem.nsy)
        self.m = int(problem.lx) * int(problem.ly)
        self.N = int(problem.N)
        self.options = nmpc_default_options(**options)
        self.max_batch = max_batch
        self.hd = nmpc_create(problem, self.options, max_batch)

    def set_options(self, **kw):
        for k, v in kw.items():
            setattr(self.options, k, v)
        nmpc_set_options(self.hd, self.options)

    @property
    def _dims(self):
        return dict(n=self.n, m=self.m, N=self.N, xref_stages=bool(self.options.xref_per_stage))

    def solve(self, x0, xref, warm: Optional[Sequence] = None):
        return nmpc_solve(self.hd, x0, xref, warm, **self._dims)

    def solve_batch(self, x0, xref, warm=None, out=None):
        return nmpc_solve_batch(self.hd, x0, xref, warm, out, **self._dims)

    def residual_batch(self, x0, xref, X, U, LAM):
        return nmpc_residual_batch(self.hd, x0, xref, X, U, LAM, **self._dims)

    def shift_batch(self, X, U, LAM, out=None):
        return nmpc_shift_batch(self.hd, X, U, LAM, out, **self._dims)

    def plant_step_batch(self, x, U, dt: float, out=None):
        return nmpc_plant_step_batch(self.hd, x, U, dt, out, **self._dims)

    def autotune(self, x0, xref, iters: int = 8) -> int:
        tr = nmpc_autotune(self.hd, x0, xref, iters, **self._dims)
        self.options.tile_rows = tr
        return tr

    def kernel_config(self):
        return nmpc_kernel_config(self.hd)

    def timing_enable(self, enable: bool = True):
        nmpc_timing_enable(self.hd, enable)

    def timing_read(self):
        return nmpc_timing_read(self.hd)

    def close(self):
        if getattr(self, "hd", None):
            nmpc_destroy(self.hd)
            self.hd = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RaggedSolver:
    """Instances of several problem classes in one launch per iteration.

    solve() takes per-instance lists (class index, x0, xref as device tensors
    or host arrays), packs them into the library's instance-order layout and
    returns per-instance (X [N,n], U [N,m], LAM [N,n]) device views."""

    def __init__(self, classes, *, max_instances: int, **options):
        _load()
        self.classes = list(classes)
        self.options = nmpc_default_options(**options)
        self.max_instances = max_instances
        self.hd, self._keep = nmpc_ragged_create(self.classes, self.options, max_instances)

    def _sizes(self, cls):
        n = [int(self.classes[c].nsx) * int(self.classes[c].nsy) for c in cls]
        N = [int(self.classes[c].N) for c in cls]
        m = [int(self.classes[c].lx) * int(self.classes[c].ly) for c in cls]
        return n, N, m

    def pack(self, cls, arrays):
        """Concatenate per-instance device tensors (any shape) into one 1-D tensor."""
        import torch
        return torch.cat([a.reshape(-1) for a in arrays]).contiguous()

    def solve(self, cls, x0, xref, warm=None):
        """cls: class per instance; x0, xref: packed 1-D device tensors or lists
        of per-instance device tensors; warm: None or packed (x, u, lam)."""
        import torch
        cls = [int(c) for c in cls]
        n, N, m = self._sizes(cls)
        if isinstance(x0, (list, tuple)):
            x0 = self.pack(cls, x0)
        if isinstance(xref, (list, tuple)):
            xref = self.pack(cls, xref)
        nx = sum(n)
        nS = sum(a * b for a, b in zip(n, N))
        nU = sum(a * b for a, b in zip(m, N))
        dev = x0.device
        out = (torch.empty(nS, dtype=torch.float64, device=dev),
               torch.empty(nU, dtype=torch.float64, device=dev),
               torch.empty(nS, dtype=torch.float64, device=dev))
        rc, infos = nmpc_ragged_solve(self.hd, cls, x0, xref, warm, out, (nx, nS, nU))
        res, so, uo = [], 0, 0
        for b in range(len(cls)):
            k, ku = N[b] * n[b], N[b] * m[b]
            res.append((out[0][so:so + k].view(N[b], n[b]), out[1][uo:uo + ku].view(N[b], m[b]),
                        out[2][so:so + k].view(N[b], n[b])))
            so += k
            uo += ku
        return rc, res, infos, out

    def autotune(self, cls, x0, xref, iters: int = 8) -> int:
        cls = [int(c) for c in cls]
        if isinstance(x0, (list, tuple)):
            x0 = self.pack(cls, x0)
        if isinstance(xref, (list, tuple)):
            xref = self.pack(cls, xref)
        return nmpc_ragged_autotune(self.hd, cls, x0, xref, x0.numel(), iters)

    def config(self, cls) -> int:
        return nmpc_ragged_config(self.hd, [int(c) for c in cls])

    def timing_enable(self, enable: bool = True):
        nmpc_ragged_timing_enable(self.hd, enable)

    def timing_read(self):
        return nmpc_ragged_timing_read(self.hd)

    def close(self):
        if getattr(self, "hd", None):
            nmpc_ragged_destroy(self.hd)
            self.hd = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- model engine

_MODELS = {"heat": NMPC_MODEL_HEAT, "plate": NMPC_MODEL_PLATE, "wave": NMPC_MODEL_WAVE}
_BCS = {"dirichlet": NMPC_BC_DIRICHLET, "neumann": NMPC_BC_NEUMANN}


class _ModelProblem:
    """nmpc_model_problem plus the host arrays it points at (kept alive here)."""

    def __init__(self, p):
        self.act = None if p.act is None else np.ascontiguousarray(p.act, dtype=np.int32)
        self.B = None if p.B is None else np.ascontiguousarray(p.B, dtype=np.float64)
        m = len(self.act) if self.act is not None else self.B.shape[1]
        self.s = nmpc_model_problem(
            _MODELS[p.model], _BCS[p.boundary], int(p.nsx), int(p.nsy), int(p.N), int(m),
            None if self.act is None else self.act.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            None if self.B is None else self.B.ctypes.data_as(_dp),
            float(p.h), float(p.q), float(p.qv), float(p.r), float(p.gamma), float(p.tau),
            float(p.u_lo), float(p.u_hi), float(p.u_cold), float(p.alpha), float(p.beta),
            float(p.rad), float(p.t_amb), float(p.k0), float(p.k1), float(p.damp))
        self.m = m


def nmpc_model_create(problem, options: nmpc_options, max_batch: int = 1):
    pr = _ModelProblem(problem)
    hd = ctypes.c_void_p()
    rc = _load().nmpc_model_create(ctypes.byref(pr.s), ctypes.byref(options), int(max_batch),
                                   ctypes.byref(hd))
    if rc != NMPC_OK:
        raise NmpcError(rc, "nmpc_model_create")
    return hd, pr.m


class ModelSolver:
    """Model engine handle (plate, wave, dense-B heat); device tensors in and
    out on torch's current stream. x0 [B][nx], xref [B][nodes]; returns
    (status, X [B][N][nx], U [B][N][m], LAM [B][N][nx], infos: a numpy structured array of
    nmpc_info records)."""

    def __init__(self, problem, *, max_batch: int = 1, **options):
        _load()
        self.problem = problem
        self.nodes = int(problem.nsx) * int(problem.nsy)
        self.nx = 2 * self.nodes if problem.model == "wave" else self.nodes
        self.N = int(problem.N)
        self.options = nmpc_default_options(**options)
        self.max_batch = max_batch
        self.hd, self.m = nmpc_model_create(problem, self.options, max_batch)

    def set_options(self, **kw):
        for k, v in kw.items():
            setattr(self.options, k, v)
        rc = _load().nmpc_model_set_options(self.hd, ctypes.byref(self.options))
        if rc != NMPC_OK:
            raise NmpcError(rc, "nmpc_model_set_options")

    def solve_batch(self, x0, xref, warm=None, out=None):
        import torch
        B, N, nx, m = x0.shape[0], self.N, self.nx, self.m
        px0 = _dev(x0, (B, nx), "x0")
        pxr = _dev(xref, (B, self.nodes), "xref")
        if out is None:
            out = (torch.empty((B, N, nx), dtype=torch.float64, device=x0.device),
                   torch.empty((B, N, m), dtype=torch.float64, device=x0.device),
                   torch.empty((B, N, nx), dtype=torch.float64, device=x0.device))
        po = [_dev(out[0], (B, N, nx), "out x"), _dev(out[1], (B, N, m), "out u"),
              _dev(out[2], (B, N, nx), "out lam")]
        pw = [None, None, None]
        if warm is not None:
            pw = [_dev(warm[0], (B, N, nx), "warm x"), _dev(warm[1], (B, N, m), "warm u"),
                  _dev(warm[2], (B, N, nx), "warm lam")]
        infos, pinfo = _info_array(B)
        rc = _load().nmpc_model_solve_batch(self.hd, B, px0, pxr, pw[0], pw[1], pw[2], po[0],
                                            po[1], po[2], pinfo, _stream())
        if rc not in (NMPC_OK, NMPC_E_NOCONV, NMPC_E_NONFINITE):
            raise NmpcError(rc, "nmpc_model_solve_batch")
        return rc, out[0], out[1], out[2], infos

    def residual_batch(self, x0, xref, X, U, LAM):
        B, N, nx, m = x0.shape[0], self.N, self.nx, self.m
        rs = np.zeros(B); rp = np.zeros(B)
        rc = _load().nmpc_model_residual_batch(
            self.hd, B, _dev(x0, (B, nx), "x0"), _dev(xref, (B, self.nodes), "xref"),
            _dev(X, (B, N, nx), "x"), _dev(U, (B, N, m), "u"), _dev(LAM, (B, N, nx), "lam"),
            rs.ctypes.data, rp.ctypes.data, _stream())
        if rc != NMPC_OK:
            raise NmpcError(rc, "nmpc_model_residual_batch")
        return rs, rp

    def timing_enable(self, enable: bool = True):
        rc = _load().nmpc_model_timing_enable(self.hd, 1 if enable else 0)
        if rc != NMPC_OK:
            raise NmpcError(rc, "nmpc_model_timing_enable")

    def timing_read(self):
        ms = ctypes.c_double(); la = ctypes.c_int64(); un = ctypes.c_int64()
        rc = _load().nmpc_model_timing_read(self.hd, ctypes.byref(ms), ctypes.byref(la),
                                            ctypes.byref(un))
        if rc != NMPC_OK:
            raise NmpcError(rc, "nmpc_model_timing_read")
        return {"kernel_ms": ms.value, "launches": la.value, "units": un.value}

    def close(self):
        if getattr(self, "hd", None):
            _load().nmpc_model_destroy(self.hd)
            self.hd = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
