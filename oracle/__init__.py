"""CPU oracle of the double-layer Jacobi NMPC solver (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package. The product library never does, and this package imports
nothing from the product: the two share only the seeded instance generator
``nmpc_inputs``.

* ``dlj_ref.c`` (loaded here through ctypes) -- plain FP64 loops of the method
  (KKT function, point-Jacobi lower layer, stage-parallel Jacobi upper layer
  and the Gauss-Seidel upper layers FGS / BGS / SGS).
* ``dense.py`` -- dense numpy forms for tiny instances: KKT Jacobian, Newton,
  Lagrangian, LQ condensed optimum and direct NLP minimization.

Pins (tests marked ``not gpu``) tie both to what the paper and mathematics fix;
see ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from nmpc_inputs import Problem

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dlj_ref.c")
_LIB = os.path.join(_HERE, "libdlj_ref.so")
_LIB_NATIVE = os.path.join(_HERE, "libdlj_ref_native.so")


def build(force: bool = True, native: bool = False) -> str:
    """Compile dlj_ref.c into libdlj_ref.so (gcc, FP64, OpenMP over stages).
    native: a copy tuned for the CPU it is built on (-march=native), for timing
    the oracle on the machine that runs it (built there, never shipped)."""
    lib = _LIB_NATIVE if native else _LIB
    if force or not os.path.exists(lib):
        tmp = lib + ".tmp"
        flags = ["-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99"]
        if native:
            flags.append("-march=native")
        subprocess.check_call(["gcc", *flags, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, lib)
    return lib


_use_native = False


def use_native() -> None:
    """Build the host-tuned copy here and load it for every later call (must be
    called before the first call into the oracle)."""
    global _use_native
    if _use_native:
        return
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    build(force=True, native=True)
    _use_native = True


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's parallel loops."""
    _load().ref_set_threads(int(n))


class _RefProblem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nsx", ctypes.c_int), ("nsy", ctypes.c_int),
                ("N", ctypes.c_int), ("m", ctypes.c_int),
                ("B", ctypes.POINTER(ctypes.c_double)),
                ("h", ctypes.c_double), ("k0", ctypes.c_double), ("k1", ctypes.c_double),
                ("q", ctypes.c_double), ("r", ctypes.c_double), ("gamma", ctypes.c_double),
                ("tau", ctypes.c_double), ("u_lo", ctypes.c_double), ("u_hi", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _LIB_NATIVE if _use_native else _LIB
        if not os.path.exists(path):
            build(force=False, native=_use_native)
        lib = ctypes.CDLL(path)
        lib.ref_set_threads.argtypes = [ctypes.c_int]
        lib.ref_set_threads.restype = None
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_RefProblem)
        lib.ref_kkt.argtypes = [pp, dp, dp, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp]
        lib.ref_kkt.restype = None
        lib.ref_norms.argtypes = [pp, dp, dp, dp, dp, dp]
        lib.ref_norms.restype = None
        lib.ref_alpha_max.argtypes = [pp, dp, dp]
        lib.ref_alpha_max.restype = ctypes.c_double
        lib.ref_stage_solve.argtypes = [pp, dp, dp, dp, dp, dp, dp, ctypes.c_int, ctypes.c_int,
                                        dp, dp, dp]
        lib.ref_stage_solve.restype = None
        lib.ref_iterate.argtypes = [pp, dp, dp, ctypes.c_int, dp, dp, dp, dp, dp, dp,
                                    ctypes.c_int, ctypes.c_int, dp, dp]
        lib.ref_iterate.restype = None
        lib.ref_solve.argtypes = [pp, dp, dp, ctypes.c_int, dp, dp, dp, ctypes.c_double,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_int), dp, dp, dp]
        lib.ref_solve.restype = ctypes.c_int
        lib.ref_gs_sweep.argtypes = [pp, dp, dp, ctypes.c_int, dp, dp, dp, dp, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_double]
        lib.ref_gs_sweep.restype = None
        lib.ref_solve_gs.argtypes = [pp, dp, dp, ctypes.c_int, dp, dp, dp, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int), dp, dp, dp, ctypes.c_double]
        lib.ref_solve_gs.restype = ctypes.c_int
        _lib = lib
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _Ctx:
    """Keeps the dense B alive for the lifetime of a ctypes problem struct."""

    def __init__(self, P: Problem):
        self.B = np.ascontiguousarray(P.dense_B(), dtype=np.float64)
        self.s = _RefProblem(P.dim, P.nsx, P.nsy, P.N, P.m, _d(self.B),
                             P.h, P.k0, P.k1, P.q, P.r, P.gamma, P.tau, P.u_lo, P.u_hi)
        self.P = P

    @property
    def ptr(self):
        return ctypes.byref(self.s)


def _c(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _xref(P, xref):
    xref = _c(xref)
    stride = P.n if xref.ndim == 2 and xref.shape[0] == P.N else 0
    return xref, stride


def cold_start(P: Problem, x0):
    """S^0 with x_i = x0, u_i = 0, lambda_i = 0."""
    return (np.tile(np.asarray(x0, float), (P.N, 1)), np.zeros((P.N, P.m)),
            np.zeros((P.N, P.n)))


def feasible_inputs(P: Problem, U):
    """With an input box (tau > 0) the method starts from a strictly feasible
    S^0 (Sec. 4.2); the paper gives no rule for a start outside the box. The
    reading taken: clip the start's inputs to [u_lo + d, u_hi - d] with d half
    a percent of the box width (NaN stays NaN). Without a box U is returned
    unchanged."""
    U = np.array(U, dtype=np.float64)
    if P.tau > 0.0:
        d = 0.005 * (P.u_hi - P.u_lo)
        lo, hi = P.u_lo + d, P.u_hi - d
        U = np.where(U < lo, lo, np.where(U > hi, hi, U))
    return U


def kkt(P: Problem, x0, xref, X, U, LAM, UT=None):
    lib = _load()
    C = _Ctx(P)
    xr, st = _xref(P, xref)
    KX = np.zeros((P.N, P.n)); KU = np.zeros((P.N, P.m)); KL = np.zeros((P.N, P.n))
    X, U, LAM = _c(X), _c(U), _c(LAM)
    ut = _d(_c(UT)) if UT is not None else None
    lib.ref_kkt(C.ptr, _d(_c(x0)), _d(xr), st, _d(X), _d(U), _d(LAM), ut,
                _d(KX), _d(KU), _d(KL))
    return KX, KU, KL


def norms(P: Problem, KX, KU, KL):
    lib = _load()
    C = _Ctx(P)
    rs = ctypes.c_double(); rp = ctypes.c_double()
    lib.ref_norms(C.ptr, _d(_c(KX)), _d(_c(KU)), _d(_c(KL)), ctypes.byref(rs), ctypes.byref(rp))
    return rs.value, rp.value


def residual(P: Problem, x0, xref, X, U, LAM):
    """(r_scaled, r_paper) of a trajectory (ut = u)."""
    return norms(P, *kkt(P, x0, xref, X, U, LAM))


def stage_solve(P: Problem, x, lam, b1, b2, b3, n_sw=2, n_schur=2, u=None):
    """Lower layer of one stage; u: the stage's inputs (needed with an input box)."""
    lib = _load()
    C = _Ctx(P)
    dx = np.zeros(P.n); du = np.zeros(P.m); dl = np.zeros(P.n)
    lib.ref_stage_solve(C.ptr, _d(_c(x)), _d(_c(lam)), None if u is None else _d(_c(u)),
                        _d(_c(b1)), _d(_c(b2)), _d(_c(b3)), n_sw, n_schur, _d(dx), _d(du),
                        _d(dl))
    return dx, du, dl


def alpha_max(P: Problem, U, DU):
    """Fraction-to-the-boundary step (eq. eq_alphamax) for inputs U and steps DU [N][m]."""
    lib = _load()
    C = _Ctx(P)
    return lib.ref_alpha_max(C.ptr, _d(_c(U)), _d(_c(DU)))


def iterate(P: Problem, x0, xref, X, U, LAM, n_sw=2, n_schur=2):
    """One upper iteration: (Xn, Un, LAMn, r_scaled(S^k), r_paper(S^k))."""
    lib = _load()
    C = _Ctx(P)
    xr, st = _xref(P, xref)
    X, U, LAM = _c(X), _c(U), _c(LAM)
    Xn = np.zeros_like(X); Un = np.zeros_like(U); Ln = np.zeros_like(LAM)
    rs = ctypes.c_double(); rp = ctypes.c_double()
    lib.ref_iterate(C.ptr, _d(_c(x0)), _d(xr), st, _d(X), _d(U), _d(LAM), _d(Xn), _d(Un),
                    _d(Ln), n_sw, n_schur, ctypes.byref(rs), ctypes.byref(rp))
    return Xn, Un, Ln, rs.value, rp.value


STATUS = {0: "converged", 1: "max_iter", 2: "nonfinite"}


UPPER = {"jacobi": 0, "fgs": 1, "bgs": 2, "sgs": 3}


def gs_sweep(P: Problem, x0, xref, X, U, LAM, direction: int, n_sw=2, n_schur=2, UT=None,
             omega=1.0):
    """One Gauss-Seidel sweep (direction +1 forward, -1 backward) on copies;
    returns the new (X, U, LAM). UT: regularization reference (default: each
    stage's input at its visit). omega: over-relaxation of each stage's step
    (SOR, Sec. 4.4)."""
    lib = _load()
    C = _Ctx(P)
    xr, st = _xref(P, xref)
    X, U, LAM = _c(X).copy(), _c(U).copy(), _c(LAM).copy()
    ut = None if UT is None else _d(_c(UT))
    lib.ref_gs_sweep(C.ptr, _d(_c(x0)), _d(xr), st, _d(X), _d(U), _d(LAM), ut, int(direction),
                     n_sw, n_schur, float(omega))
    return X, U, LAM


def solve(P: Problem, x0, xref, start=None, tol=1e-6, max_iter=2000, n_sw=2, n_schur=2,
          trace=False, upper="jacobi", omega=1.0):
    """Run the upper iteration from ``start`` (default cold) to r_scaled <= tol.

    upper: "jacobi" (eq. 1st_jacobi), "fgs" (eq. fgs), "bgs" or "sgs" (eq. sgs);
    omega: over-relaxation of the Gauss-Seidel sweeps (SOR / SSOR, Sec. 4.4).
    Returns a dict with X, U, LAM (the last evaluated iterate S^k), iters = k,
    r_scaled, r_paper, status and, if ``trace``, rhist[0..k].
    """
    lib = _load()
    C = _Ctx(P)
    xr, st = _xref(P, xref)
    X, U, LAM = cold_start(P, x0) if start is None else start
    X, U, LAM = _c(X).copy(), _c(feasible_inputs(P, U)), _c(LAM).copy()
    it = ctypes.c_int(); rs = ctypes.c_double(); rp = ctypes.c_double()
    hist = np.zeros(max_iter + 1) if trace else None
    if UPPER[upper] == 0 and omega != 1.0:
        raise ValueError("over-relaxation applies to the Gauss-Seidel sweeps")
    if UPPER[upper] == 0:
        status = lib.ref_solve(C.ptr, _d(_c(x0)), _d(xr), st, _d(X), _d(U), _d(LAM), tol,
                               max_iter, n_sw, n_schur, ctypes.byref(it), ctypes.byref(rs),
                               ctypes.byref(rp), _d(hist) if trace else None)
    else:
        status = lib.ref_solve_gs(C.ptr, _d(_c(x0)), _d(xr), st, _d(X), _d(U), _d(LAM),
                                  UPPER[upper], tol, max_iter, n_sw, n_schur, ctypes.byref(it),
                                  ctypes.byref(rs), ctypes.byref(rp),
                                  _d(hist) if trace else None, float(omega))
    out = dict(X=X, U=U, LAM=LAM, iters=it.value, r_scaled=rs.value, r_paper=rp.value,
               status=STATUS[status])
    if trace:
        out["rhist"] = hist[:it.value + 1]
    return out


def threads() -> int:
    """OpenMP threads the C reference uses (OMP_NUM_THREADS or all cores)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        return int(env)
    return os.cpu_count() or 1
