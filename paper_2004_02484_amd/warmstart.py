"""Learned warm start: a patch-encoder network predicting the input trajectory.

For each actuator of the input lattice the network reads a window of (x0,
xref) around it and predicts that actuator's inputs over the horizon. The
predicted inputs are handed to the solver as a u-only warm start: the library
builds the states by the backward-Euler model and the costates by the adjoint
recursion, compares the residual with the cold start's (fallback) and
iterates. The network is trained on solutions computed by the solver itself.

The optimal inputs depend on the initial state and the reference almost
linearly; the part that is not linear comes mostly from pointwise products
(the conductivity depends on the temperature, so the model's response and
its adjoint carry products of the state with itself and with the reference).
The window rows therefore hold five feature planes of the scaled fields
xt = x0/0.1 - 1 and rt = xref/0.3: xt, rt, xt^2 - 1/3, xt rt, rt^2 - 1/3.

Layers (run by the library's network object, nmpc_net_*; this module only
holds its handle, allocates torch device tensors and calls the C ABI):

    X  = features(x0, xref)                     rows: instance x actuator
    H1 = relu(X W1 + b1)                        window conv (32x32, stride 16)
    H2 = relu(H1 W2 + b2)                       1x1 conv
    H3 = relu(H2 W3 + b3)                       1x1 conv
    Y  = H3 W4 + b4 + X Ws[p]                   1x1 conv + per-actuator linear map
    u  = 4 Y                                    [instance][stage][actuator]

The hidden layers run on bf16 operands (fp32 accumulation) on the matrix
cores. The per-actuator map Ws[p] (p: the row's actuator; the domain is not
translation invariant, so each actuator has its own) carries most of the
prediction and runs on fp32 operands, also on the matrix cores.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Dict, Optional

import numpy as np

from . import _binding as B

U_SCALE = 4.0          # targets are u / U_SCALE
_vp = ctypes.c_void_p


def _lib():
    lib = B._load()
    if not getattr(lib, "_net_typed", False):
        i32, i64, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
        lib.nmpc_gemm_bf16.argtypes = [i32, i32, i32, i32, i32, _vp, i32, _vp, i32, f32, _vp, i32,
                                       _vp, i32, _vp, i32, _vp]
        lib.nmpc_gemm_f32.argtypes = [i32, i32, i32, i32, _vp, i32, i64, _vp, i32, i64, f32, _vp,
                                      i32, i64, i32, i32, _vp, _vp]
        lib.nmpc_gemm_f64.argtypes = [i32, i32, i32, i32, _vp, i32, i64, _vp, i32, i64,
                                      ctypes.c_double, ctypes.c_double, _vp, _vp, i32, i64, i32, _vp]
        lib.nmpc_gemm_f32_acc64.argtypes = [i32, i32, i32, i32, _vp, i32, i64, _vp, i32, i64,
                                            ctypes.c_double, _vp, i32, i64, i32, _vp]
        lib.nmpc_ls_prepare.argtypes = [_vp, i32, i32, i64, ctypes.c_double, _vp, i64, i32, _vp]
        lib.nmpc_net_features.argtypes = [_vp, _vp, i32, i32, i32, i32, i32, _vp, _vp, i32, _vp]
        lib.nmpc_relu_grad.argtypes = [_vp, _vp, _vp, i64, _vp]
        lib.nmpc_colsum.argtypes = [_vp, i32, i32, i32, _vp, _vp]
        lib.nmpc_mse_grad.argtypes = [_vp, i32, _vp, i32, i32, i32, f32, _vp, _vp, i32, _vp, _vp]
        lib.nmpc_adam.argtypes = [_vp, _vp, _vp, _vp, _vp, i64, f32, f32, f32, f32, f32, i32, _vp]
        lib.nmpc_to_bf16.argtypes = [_vp, _vp, i64, _vp]
        lib.nmpc_pack_inputs.argtypes = [_vp, i32, i32, i32, f32, _vp, i32, _vp]
        lib.nmpc_unpack_inputs.argtypes = [_vp, i32, i32, i32, i32, f32, _vp, _vp]
        for f in ("nmpc_gemm_bf16", "nmpc_gemm_f32", "nmpc_gemm_f64", "nmpc_gemm_f32_acc64",
                  "nmpc_ls_prepare", "nmpc_net_features", "nmpc_relu_grad", "nmpc_colsum",
                  "nmpc_mse_grad", "nmpc_adam", "nmpc_to_bf16", "nmpc_pack_inputs",
                  "nmpc_unpack_inputs"):
            getattr(lib, f).restype = ctypes.c_int
        lib._net_typed = True
    return lib


def _ck(rc, where):
    if rc != B.NMPC_OK:
        raise B.NmpcError(rc, where)


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def gemm(A, B_, M, N, K, *, ta=0, tb=0, lda=None, ldb=None, C=None, ldc=None, beta=0.0,
         bias=None, relu=False, Cb=None, ldcb=None):
    """C (fp32) / Cb (bf16) = op(A) op(B) [+ beta C] [+ bias] [ReLU] on the matrix cores."""
    lda = lda if lda is not None else (M if ta else K)
    ldb = ldb if ldb is not None else (K if tb else N)
    ldc = ldc if ldc is not None else N
    ldcb = ldcb if ldcb is not None else N
    _ck(_lib().nmpc_gemm_bf16(ta, tb, M, N, K, _p(A), lda, _p(B_), ldb, beta, _p(C), ldc,
                              _p(bias), 1 if relu else 0, _p(Cb), ldcb, _stream()),
        "nmpc_gemm_bf16")


def gemm_f32(A, B_, M, N, K, C, *, ta=0, lda, ldb, ldc, sa=0, sb=0, sc=0, groups=1, beta=0.0,
             ksplit=1, work=None):
    """C_g = beta C_g + op(A_g) B_g on fp32 operands for groups g (X_g = X + g sx);
    ksplit > 1 cuts K in parts summed in a fixed order (work: groups*ksplit*M*N floats)."""
    _ck(_lib().nmpc_gemm_f32(ta, M, N, K, _p(A), lda, sa, _p(B_), ldb, sb, beta, _p(C), ldc, sc,
                             groups, ksplit, _p(work), _stream()), "nmpc_gemm_f32")


def gemm_f64(A, B_, M, N, K, C, *, ta=0, lda, ldb, ldc, sa=0, sb=0, sc=0, groups=1, alpha=1.0,
             beta=0.0, Cin=None):
    """C_g = alpha op(A_g) B_g + beta Cin_g on fp64 operands (Cin defaults to C)."""
    _ck(_lib().nmpc_gemm_f64(ta, M, N, K, _p(A), lda, sa, _p(B_), ldb, sb, alpha, beta, _p(Cin),
                             _p(C), ldc, sc, groups, _stream()), "nmpc_gemm_f64")


def gemm_f32_acc64(A, B_, M, N, K, C, *, ta=0, lda, ldb, ldc, sa=0, sb=0, sc=0, groups=1,
                   beta=0.0):
    """C_g (fp64) = op(A_g) B_g + beta C_g with fp32 operands, fp64 products and sums."""
    _ck(_lib().nmpc_gemm_f32_acc64(ta, M, N, K, _p(A), lda, sa, _p(B_), ldb, sb, beta, _p(C), ldc,
                                   sc, groups, _stream()), "nmpc_gemm_f32_acc64")


def ls_prepare(G, X, n, groups, ridge_rel):
    """Ridge on the diagonals of G [groups][n][n] and X = I / trace (Newton-Schulz start)."""
    _ck(_lib().nmpc_ls_prepare(_p(G), n, n, n * n, ridge_rel, _p(X), n * n, groups, _stream()),
        "nmpc_ls_prepare")


def to_bf16(x, y=None):
    import torch
    y = torch.empty(x.shape, dtype=torch.int16, device=x.device) if y is None else y
    _ck(_lib().nmpc_to_bf16(_p(x), _p(y), x.numel(), _stream()), "nmpc_to_bf16")
    return y


def bf16_to_float(y):
    """Host-side view of bf16 bit patterns as float32 (tests, checkpoints)."""
    a = y.detach().cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return a.view(np.float32)


class nmpc_net_config(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("ns", ctypes.c_int32), ("lattice", ctypes.c_int32),
                ("win", ctypes.c_int32), ("hidden", ctypes.c_int32), ("planes", ctypes.c_int32)]


def _net_lib():
    lib = _lib()
    if not getattr(lib, "_netobj_typed", False):
        i32, i64, f32, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_uint32
        fp = ctypes.POINTER(ctypes.c_float)
        lib.nmpc_net_create.argtypes = [ctypes.POINTER(nmpc_net_config), ctypes.c_uint64, i32,
                                        ctypes.POINTER(_vp)]
        lib.nmpc_net_forward.argtypes = [_vp, i32, _vp, _vp, _vp, _vp]
        lib.nmpc_net_backward.argtypes = [_vp, i32, _vp, _vp, _vp, fp, _vp]
        lib.nmpc_net_adam_step.argtypes = [_vp, f32, f32, f32, f32, f32, u32, _vp]
        lib.nmpc_net_train_step.argtypes = [_vp, i32, _vp, _vp, _vp, f32, f32, u32, fp, _vp]
        lib.nmpc_net_get.argtypes = [_vp, ctypes.c_char_p, _vp, i64]
        lib.nmpc_net_set.argtypes = [_vp, ctypes.c_char_p, _vp, i64, i32, _vp]
        lib.nmpc_net_num_params.argtypes = [_vp]
        lib.nmpc_net_num_params.restype = i64
        lib.nmpc_net_save.argtypes = [_vp, ctypes.c_char_p]
        lib.nmpc_net_load.argtypes = [_vp, ctypes.c_char_p]
        lib.nmpc_net_destroy.argtypes = [_vp]
        lib.nmpc_net_destroy.restype = None
        for f in ("nmpc_net_create", "nmpc_net_forward", "nmpc_net_backward", "nmpc_net_adam_step",
                  "nmpc_net_train_step", "nmpc_net_get", "nmpc_net_set", "nmpc_net_save",
                  "nmpc_net_load"):
            getattr(lib, f).restype = ctypes.c_int
        lib._netobj_typed = True
    return lib


PARAMS = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4", "Ws")


class PatchNet:
    """Patch encoder for an ns x ns grid with an L x L actuator lattice and N
    stages: a handle of the library's network object (nmpc_net_*), which holds
    the parameters, gradients, optimizer state and activations on the device
    and runs every layer in the library's kernels."""

    PLANES = 5
    KSPLIT = 8      # K parts of the per-actuator map (few output tiles, long K)

    def __init__(self, N: int = 40, ns: int = 64, lattice: int = 4, win: int = 32,
                 hidden: int = 512, seed: int = 0, device: str = "cuda", max_count: int = 256):
        self.N, self.ns, self.L, self.win, self.H = N, ns, lattice, win, hidden
        self.m = lattice * lattice
        self.K0 = self.PLANES * win * win + self.m
        self.K0p = (self.K0 + 31) // 32 * 32
        self.device = device
        self.meta = {}
        self.seed = seed
        self.max_count = max_count
        self.cfg = nmpc_net_config(N, ns, lattice, win, hidden, self.PLANES)
        self.hd = self._create(max_count)
        self.last_count = 0

    def _create(self, max_count):
        hd = _vp()
        _ck(_net_lib().nmpc_net_create(ctypes.byref(self.cfg), self.seed, max_count,
                                       ctypes.byref(hd)), "nmpc_net_create")
        return hd

    def _ensure(self, count):
        """Room for `count` instances (the object is rebuilt with the same parameters)."""
        if count <= self.max_count:
            return
        st = self.state()
        old = self.hd
        self.max_count = count
        self.hd = self._create(count)
        _net_lib().nmpc_net_destroy(old)
        self.load_state(st)

    def shape(self, name):
        K0, H, N, m = self.K0p, self.H, self.N, self.m
        return {"W1": (K0, H), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (H, H), "b3": (H,),
                "W4": (H, N), "b4": (N if H > 0 else 0,), "Ws": (m, K0, N)}[name]

    def num_params(self) -> int:
        return int(_net_lib().nmpc_net_num_params(self.hd))

    # ------------------------------------------------------------ passes

    def predict(self, x0, xref, out=None):
        """Predicted input trajectories u [count][N][m] (float64, device)."""
        import torch
        count = x0.shape[0]
        self._ensure(count)
        u = out if out is not None else torch.empty((count, self.N, self.m), dtype=torch.float64,
                                                     device=x0.device)
        _ck(_net_lib().nmpc_net_forward(self.hd, count, _p(x0), _p(xref), _p(u), _stream()),
            "nmpc_net_forward")
        self.last_count = count
        return u

    def backward(self, x0, xref, u_target) -> float:
        """Forward and backward pass; the gradients stay in the object
        (``grad(name)``). Returns the mean squared error of the scaled inputs."""
        count = x0.shape[0]
        self._ensure(count)
        loss = ctypes.c_float()
        _ck(_net_lib().nmpc_net_backward(self.hd, count, _p(x0), _p(xref), _p(u_target),
                                         ctypes.byref(loss), _stream()), "nmpc_net_backward")
        self.last_count = count
        return float(loss.value)

    def train_step(self, x0, xref, u_target, lr=1e-3, wd=0.0, frozen=()) -> float:
        count = x0.shape[0]
        self._ensure(count)
        mask = sum(1 << PARAMS.index(k) for k in frozen)
        loss = ctypes.c_float()
        _ck(_net_lib().nmpc_net_train_step(self.hd, count, _p(x0), _p(xref), _p(u_target), lr, wd,
                                           mask, ctypes.byref(loss), _stream()),
            "nmpc_net_train_step")
        self.last_count = count
        return float(loss.value)

    # ------------------------------------------------------------ access

    def get(self, name, rows=None):
        """Host copy of a parameter, a gradient ("g" + name) or an activation
        of the last pass (rows of its instances; bf16 buffers as float32)."""
        if name in PARAMS or (name[0] == "g" and name[1:] in PARAMS):
            shape = self.shape(name if name in PARAMS else name[1:])
            a = np.empty(shape, dtype=np.float32)
        else:
            rows = self.last_count * self.m if rows is None else rows
            width = {"X": self.K0p, "Xf": self.K0p, "Y": self.N, "T": self.N, "dY": self.N,
                     "dYb": self.N}.get(name, self.H)
            if name.startswith("Wb"):
                shape = self.shape("W" + name[2:])
            else:
                shape = (rows, width)
            bf = name == "X" or name.startswith("Wb") or name.endswith("b")
            a = np.empty(shape, dtype=np.uint16 if bf else np.float32)
        if a.size:
            _ck(_net_lib().nmpc_net_get(self.hd, name.encode(), a.ctypes.data, a.size),
                "nmpc_net_get")
        if a.dtype == np.uint16:
            a = (a.astype(np.uint32) << 16).view(np.float32)
        return a

    def set_param(self, name, value):
        """Replace a parameter from a host array or a float32 device tensor."""
        import torch
        n = int(np.prod(self.shape(name)))
        if isinstance(value, torch.Tensor) and value.is_cuda:
            v = value.to(torch.float32).contiguous()
            _ck(_net_lib().nmpc_net_set(self.hd, name.encode(), _p(v), n, 1, _stream()),
                "nmpc_net_set")
        else:
            v = np.ascontiguousarray(value, dtype=np.float32)
            _ck(_net_lib().nmpc_net_set(self.hd, name.encode(), v.ctypes.data, n, 0, _stream()),
                "nmpc_net_set")

    def grad(self, name):
        return self.get("g" + name)

    # ------------------------------------------------------------ fitting

    def fit_linear(self, x0, xref, u, batch=256, ridge_rel=1e-6, iters=40):
        """Set the per-actuator map Ws to the minimizer of the squared error of
        X Ws[p] against u / U_SCALE over all rows (the hidden path contributes
        nothing while W4 and b4 are zero): Gram matrices G_p = X_p^T X_p and
        X_p^T T_p of the fp32 feature rows with fp64 sums, a relative ridge,
        G_p^{-1} by Newton-Schulz iteration in fp64, then Ws[p] = G_p^{-1} X_p^T T_p.
        Returns the Frobenius norm of I - G X of the last iterate per actuator."""
        import torch
        count = x0.shape[0]
        K0, m, N = self.K0p, self.m, self.N
        f64 = dict(dtype=torch.float64, device=self.device)
        G = torch.zeros((m, K0, K0), **f64)
        R = torch.zeros((m, K0, N), **f64)
        Xf = torch.empty((batch * m, K0), dtype=torch.float32, device=self.device)
        T = torch.empty((batch * m, N), dtype=torch.float32, device=self.device)
        for k in range(0, count, batch):
            c = min(batch, count - k)
            _ck(_lib().nmpc_net_features(_p(x0[k:k + c]), _p(xref[k:k + c]), c, self.ns, self.L,
                                         self.win, self.PLANES, _p(Xf), None, K0, _stream()),
                "nmpc_net_features")
            _ck(_lib().nmpc_pack_inputs(_p(u[k:k + c]), c, N, m, 1.0 / U_SCALE, _p(T), N,
                                        _stream()), "nmpc_pack_inputs")
            # group p: rows p, p + m, ... of the batch
            gemm_f32_acc64(Xf, Xf, K0, K0, c, G, ta=1, lda=m * K0, ldb=m * K0, ldc=K0,
                           sa=K0, sb=K0, sc=K0 * K0, groups=m, beta=1.0)
            gemm_f32_acc64(Xf, T, K0, N, c, R, ta=1, lda=m * K0, ldb=m * N, ldc=N,
                           sa=K0, sb=N, sc=K0 * N, groups=m, beta=1.0)
        X = torch.empty_like(G)
        ls_prepare(G, X, K0, m, ridge_rel)
        Tm = torch.empty_like(G)
        Xn = torch.empty_like(G)
        sq = dict(lda=K0, ldb=K0, ldc=K0, sa=K0 * K0, sb=K0 * K0, sc=K0 * K0, groups=m)
        for _ in range(iters):
            gemm_f64(G, X, K0, K0, K0, Tm, **sq)                            # T = G X
            gemm_f64(X, Tm, K0, K0, K0, Xn, alpha=-1.0, beta=2.0, Cin=X, **sq)   # 2X - X G X
            X, Xn = Xn, X
        gemm_f64(G, X, K0, K0, K0, Tm, **sq)
        W = torch.empty((m, K0, N), **f64)
        gemm_f64(X, R, K0, N, K0, W, lda=K0, ldb=N, ldc=N, sa=K0 * K0, sb=K0 * N, sc=K0 * N,
                 groups=m)
        self.set_param("Ws", W)
        eye = torch.eye(K0, **f64)
        return [float(torch.linalg.matrix_norm(eye - Tm[p])) for p in range(m)]

    # ------------------------------------------------------------ state

    def state(self) -> Dict[str, np.ndarray]:
        return {k: self.get(k) for k in PARAMS}

    def load_state(self, st: Dict[str, np.ndarray]):
        for k in PARAMS:
            if int(np.prod(self.shape(k))):
                self.set_param(k, np.asarray(st[k], dtype=np.float32))

    def save(self, path: str, meta: Optional[dict] = None):
        """Weights (fp32) + JSON header with the architecture and training facts."""
        header = {"format": "nmpc-patchnet-v2", "N": self.N, "ns": self.ns, "lattice": self.L,
                  "win": self.win, "hidden": self.H, "meta": meta or {}}
        np.savez_compressed(path, header=np.frombuffer(json.dumps(header).encode(), np.uint8),
                            **self.state())

    def save_bin(self, path: str):
        """The library's own weight file (nmpc_net_save)."""
        _ck(_net_lib().nmpc_net_save(self.hd, path.encode()), "nmpc_net_save")

    def load_bin(self, path: str):
        _ck(_net_lib().nmpc_net_load(self.hd, path.encode()), "nmpc_net_load")

    @classmethod
    def load(cls, path: str, device: str = "cuda", max_count: int = 256,
             mlp: bool = True) -> "PatchNet":
        """mlp=False builds the network without its hidden path (hidden = 0):
        the prediction is the per-actuator linear map alone."""
        z = np.load(path, allow_pickle=False)
        header = json.loads(bytes(z["header"]).decode())
        if header.get("format") != "nmpc-patchnet-v2":
            raise ValueError(f"{path}: not a patch-net checkpoint")
        net = cls(N=header["N"], ns=header["ns"], lattice=header["lattice"], win=header["win"],
                  hidden=header["hidden"] if mlp else 0, device=device, max_count=max_count)
        net.load_state({k: z[k] for k in PARAMS})
        net.meta = header["meta"]
        return net

    def close(self):
        if getattr(self, "hd", None):
            _net_lib().nmpc_net_destroy(self.hd)
            self.hd = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
