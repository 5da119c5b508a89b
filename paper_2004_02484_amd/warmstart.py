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

Layers (this module only allocates torch device tensors and calls the C ABI):

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


class PatchNet:
    """Patch encoder for an ns x ns grid with an L x L actuator lattice and N stages."""

    PLANES = 5
    KSPLIT = 8      # K parts of the per-actuator map (few output tiles, long K)

    def __init__(self, N: int = 40, ns: int = 64, lattice: int = 4, win: int = 32,
                 hidden: int = 512, seed: int = 0, device: str = "cuda"):
        import torch
        self.N, self.ns, self.L, self.win, self.H = N, ns, lattice, win, hidden
        self.m = lattice * lattice
        self.K0 = self.PLANES * win * win + self.m
        self.K0p = (self.K0 + 31) // 32 * 32
        self.device = device
        self.meta = {}
        rng = np.random.default_rng(seed)

        def he(fan_in, shape, gain=2.0):
            return rng.uniform(-1, 1, shape) * np.sqrt(3.0 * gain / fan_in)

        init = {
            "W1": he(self.K0, (self.K0p, hidden)), "b1": np.zeros(hidden),
            "W2": he(hidden, (hidden, hidden)), "b2": np.zeros(hidden),
            "W3": he(hidden, (hidden, hidden)), "b3": np.zeros(hidden),
            "W4": he(hidden, (hidden, N), gain=0.1), "b4": np.zeros(N),
            "Ws": np.zeros((self.m, self.K0p, N)),
        }
        init["W1"][self.K0:] = 0.0
        self.params: Dict[str, "torch.Tensor"] = {}
        for k, v in init.items():
            self.params[k] = torch.tensor(v, dtype=torch.float32, device=device)
        self._bf = {k: to_bf16(v) for k, v in self.params.items() if k.startswith("W") and k != "Ws"}
        self._opt = None
        self.step = 0

    # ------------------------------------------------------------ buffers

    def _alloc(self, rows):
        import torch
        key = rows
        if getattr(self, "_buf_rows", None) == key:
            return self._buf
        f = lambda *s: torch.empty(s, dtype=torch.float32, device=self.device)
        h = lambda *s: torch.empty(s, dtype=torch.int16, device=self.device)
        H, N = self.H, self.N
        self._buf = {
            "X": h(rows, self.K0p), "Xf": f(rows, self.K0p),
            "H1": f(rows, H), "H1b": h(rows, H), "H2": f(rows, H), "H2b": h(rows, H),
            "H3": f(rows, H), "H3b": h(rows, H), "Y": f(rows, N),
            "dY": f(rows, N), "dYb": h(rows, N), "T": f(rows, N), "sse": f(rows),
            "dH": f(rows, H), "dHb": h(rows, H), "work": f(self.KSPLIT * rows * N),
        }
        self._buf_rows = key
        return self._buf

    # ------------------------------------------------------------ forward

    def forward_rows(self, x0, xref):
        """Network output rows Y [count * m][N] (fp32) for device (x0, xref)."""
        count = x0.shape[0]
        rows = count * self.m
        b = self._alloc(rows)
        P, W = self.params, self._bf
        H, N, K0, m = self.H, self.N, self.K0p, self.m
        _ck(_lib().nmpc_net_features(_p(x0), _p(xref), count, self.ns, self.L, self.win,
                                     self.PLANES, _p(b["Xf"]), _p(b["X"]), K0, _stream()),
            "nmpc_net_features")
        gemm(b["X"], W["W1"], rows, H, K0, C=b["H1"], bias=P["b1"], relu=True, Cb=b["H1b"])
        gemm(b["H1b"], W["W2"], rows, H, H, C=b["H2"], bias=P["b2"], relu=True, Cb=b["H2b"])
        gemm(b["H2b"], W["W3"], rows, H, H, C=b["H3"], bias=P["b3"], relu=True, Cb=b["H3b"])
        gemm(b["H3b"], W["W4"], rows, N, H, C=b["Y"], bias=P["b4"])
        # per-actuator map: group p takes rows p, p + m, ... (row stride m K0)
        gemm_f32(b["Xf"], P["Ws"], count, N, K0, b["Y"], lda=m * K0, ldb=N, ldc=m * N,
                 sa=K0, sb=K0 * N, sc=N, groups=m, beta=1.0, ksplit=self.KSPLIT, work=b["work"])
        return b["Y"]

    def predict(self, x0, xref, out=None):
        """Predicted input trajectories u [count][N][m] (float64, device)."""
        import torch
        count = x0.shape[0]
        Y = self.forward_rows(x0, xref)
        u = out if out is not None else torch.empty((count, self.N, self.m), dtype=torch.float64,
                                                     device=self.device)
        _ck(_lib().nmpc_unpack_inputs(_p(Y), self.N, count, self.N, self.m, U_SCALE, _p(u),
                                      _stream()), "nmpc_unpack_inputs")
        return u

    # ------------------------------------------------------------ backward

    def loss_and_grads(self, x0, xref, u_target):
        """Mean squared error of Y against u_target / U_SCALE and the parameter
        gradients (fp32 tensors keyed like params)."""
        import torch
        count = x0.shape[0]
        rows = count * self.m
        Y = self.forward_rows(x0, xref)
        b = self._buf
        H, N, K0, m = self.H, self.N, self.K0p, self.m
        _ck(_lib().nmpc_pack_inputs(_p(u_target), count, N, m, 1.0 / U_SCALE, _p(b["T"]), N,
                                    _stream()), "nmpc_pack_inputs")
        scale = 2.0 / (rows * N)
        _ck(_lib().nmpc_mse_grad(_p(Y), N, _p(b["T"]), N, rows, N, scale, _p(b["dY"]), _p(b["dYb"]),
                                 N, _p(b["sse"]), _stream()), "nmpc_mse_grad")
        g = {k: torch.empty_like(v) for k, v in self.params.items()}
        W = self._bf
        lib = _lib()
        # output layer and the per-actuator map (fp32 dY)
        gemm(b["H3b"], b["dYb"], H, N, rows, ta=1, lda=H, ldb=N, C=g["W4"])
        gemm_f32(b["Xf"], b["dY"], K0, N, count, g["Ws"], ta=1, lda=m * K0, ldb=m * N, ldc=N,
                 sa=K0, sb=N, sc=K0 * N, groups=m)
        _ck(lib.nmpc_colsum(_p(b["dY"]), rows, N, N, _p(g["b4"]), _stream()), "nmpc_colsum")
        # hidden layers: dH_l = (dH_{l+1} W_{l+1}^T) * relu'(H_l)
        gemm(b["dYb"], W["W4"], rows, H, N, tb=1, ldb=N, C=b["dH"])
        for l, (hin, hout) in ((3, ("H2b", "H3")), (2, ("H1b", "H2")), (1, ("X", "H1"))):
            _ck(lib.nmpc_relu_grad(_p(b["dH"]), _p(b[hout]), _p(b["dHb"]), rows * H, _stream()),
                "nmpc_relu_grad")
            kin = K0 if hin == "X" else H
            gemm(b[hin], b["dHb"], kin, H, rows, ta=1, lda=kin, ldb=H, C=g[f"W{l}"])
            _ck(lib.nmpc_colsum(_p(b["dH"]), rows, H, H, _p(g[f"b{l}"]), _stream()), "nmpc_colsum")
            if l > 1:
                gemm(b["dHb"], W[f"W{l}"], rows, H, H, tb=1, ldb=H, C=b["dH"])
        loss = float(b["sse"].sum().item()) / (rows * N)
        return loss, g

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
        for k in range(0, count, batch):
            c = min(batch, count - k)
            b = self._alloc(c * m)
            _ck(_lib().nmpc_net_features(_p(x0[k:k + c]), _p(xref[k:k + c]), c, self.ns, self.L,
                                         self.win, self.PLANES, _p(b["Xf"]), None, K0, _stream()),
                "nmpc_net_features")
            _ck(_lib().nmpc_pack_inputs(_p(u[k:k + c]), c, N, m, 1.0 / U_SCALE, _p(b["T"]), N,
                                        _stream()), "nmpc_pack_inputs")
            # group p: rows p, p + m, ... of the batch
            gemm_f32_acc64(b["Xf"], b["Xf"], K0, K0, c, G, ta=1, lda=m * K0, ldb=m * K0, ldc=K0,
                           sa=K0, sb=K0, sc=K0 * K0, groups=m, beta=1.0)
            gemm_f32_acc64(b["Xf"], b["T"], K0, N, c, R, ta=1, lda=m * K0, ldb=m * N, ldc=N,
                           sa=K0, sb=N, sc=K0 * N, groups=m, beta=1.0)
        X = torch.empty_like(G)
        ls_prepare(G, X, K0, m, ridge_rel)
        T = torch.empty_like(G)
        Xn = torch.empty_like(G)
        sq = dict(lda=K0, ldb=K0, ldc=K0, sa=K0 * K0, sb=K0 * K0, sc=K0 * K0, groups=m)
        for _ in range(iters):
            gemm_f64(G, X, K0, K0, K0, T, **sq)                            # T = G X
            gemm_f64(X, T, K0, K0, K0, Xn, alpha=-1.0, beta=2.0, Cin=X, **sq)   # 2X - X G X
            X, Xn = Xn, X
        gemm_f64(G, X, K0, K0, K0, T, **sq)
        W = torch.empty((m, K0, N), **f64)
        gemm_f64(X, R, K0, N, K0, W, lda=K0, ldb=N, ldc=N, sa=K0 * K0, sb=K0 * N, sc=K0 * N,
                 groups=m)
        self.params["Ws"].copy_(W)
        eye = torch.eye(K0, **f64)
        return [float(torch.linalg.matrix_norm(eye - T[p])) for p in range(m)]

    def adam_step(self, grads, lr=1e-3, wd=0.0, b1=0.9, b2=0.999, eps=1e-8, frozen=()):
        import torch
        if self._opt is None:
            self._opt = {k: (torch.zeros_like(v), torch.zeros_like(v)) for k, v in self.params.items()}
        self.step += 1
        for k, w in self.params.items():
            if k in frozen:
                continue
            m, v = self._opt[k]
            _ck(_lib().nmpc_adam(_p(w), _p(grads[k]), _p(m), _p(v), _p(self._bf.get(k)), w.numel(),
                                 lr, b1, b2, eps, wd if k.startswith("W") else 0.0, self.step,
                                 _stream()), "nmpc_adam")

    # ------------------------------------------------------------ state

    def state(self) -> Dict[str, np.ndarray]:
        return {k: v.detach().cpu().numpy() for k, v in self.params.items()}

    def load_state(self, st: Dict[str, np.ndarray]):
        import torch
        for k in self.params:
            self.params[k] = torch.tensor(np.asarray(st[k], dtype=np.float32), device=self.device)
        self._bf = {k: to_bf16(v) for k, v in self.params.items() if k.startswith("W") and k != "Ws"}
        self._opt = None

    def save(self, path: str, meta: Optional[dict] = None):
        """Weights (fp32) + JSON header with the architecture and training facts."""
        header = {"format": "nmpc-patchnet-v2", "N": self.N, "ns": self.ns, "lattice": self.L,
                  "win": self.win, "hidden": self.H, "step": self.step, "meta": meta or {}}
        np.savez_compressed(path, header=np.frombuffer(json.dumps(header).encode(), np.uint8),
                            **self.state())

    @classmethod
    def load(cls, path: str, device: str = "cuda") -> "PatchNet":
        z = np.load(path, allow_pickle=False)
        header = json.loads(bytes(z["header"]).decode())
        if header.get("format") != "nmpc-patchnet-v2":
            raise ValueError(f"{path}: not a patch-net checkpoint")
        net = cls(N=header["N"], ns=header["ns"], lattice=header["lattice"], win=header["win"],
                  hidden=header["hidden"], device=device)
        net.load_state({k: z[k] for k in net.params})
        net.step = header["step"]
        net.meta = header["meta"]
        return net
