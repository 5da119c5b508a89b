"""Learned warm start: a patch-encoder network predicting the input trajectory.

For each actuator of the input lattice the network reads a window of (x0,
xref) around it and predicts that actuator's inputs over the horizon. The
predicted inputs are handed to the solver as a u-only warm start: the library
builds the states by the backward-Euler model and the costates by the adjoint
recursion, compares the residual with the cold start's (fallback) and
iterates. The network is trained on solutions computed by the solver itself.

Layers (each a GEMM on bf16 operands with fp32 accumulation, run by the
library's kernels; this module only allocates torch device tensors and calls
the C ABI):

    X  = windows(x0, xref)                      rows: instance x actuator
    H1 = relu(X W1 + b1)                        window conv (24x24, stride 16)
    H2 = relu(H1 W2 + b2)                       1x1 conv
    H3 = relu(H2 W3 + b3)                       1x1 conv
    Y  = H3 W4 + b4 + X Ws                      1x1 conv + linear skip conv
    u  = 4 Y                                    [instance][stage][actuator]

The skip product X Ws carries most of the prediction, so it runs on split
operands (X = Xhi + Xlo, Ws = Whi + Wlo, three bf16 products) for about 16
significant bits; the other layers use plain bf16 operands.
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
        lib.nmpc_net_windows.argtypes = [_vp, _vp, i32, i32, i32, i32, _vp, _vp, i32, _vp]
        lib.nmpc_split_bf16.argtypes = [_vp, _vp, _vp, i64, _vp]
        lib.nmpc_relu_grad.argtypes = [_vp, _vp, _vp, i64, _vp]
        lib.nmpc_colsum.argtypes = [_vp, i32, i32, i32, _vp, _vp]
        lib.nmpc_mse_grad.argtypes = [_vp, i32, _vp, i32, i32, i32, f32, _vp, _vp, i32, _vp, _vp]
        lib.nmpc_adam.argtypes = [_vp, _vp, _vp, _vp, _vp, i64, f32, f32, f32, f32, f32, i32, _vp]
        lib.nmpc_to_bf16.argtypes = [_vp, _vp, i64, _vp]
        lib.nmpc_pack_inputs.argtypes = [_vp, i32, i32, i32, f32, _vp, i32, _vp]
        lib.nmpc_unpack_inputs.argtypes = [_vp, i32, i32, i32, i32, f32, _vp, _vp]
        for f in ("nmpc_gemm_bf16", "nmpc_net_windows", "nmpc_split_bf16", "nmpc_relu_grad", "nmpc_colsum",
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

    def __init__(self, N: int = 40, ns: int = 64, lattice: int = 4, win: int = 24,
                 hidden: int = 512, seed: int = 0, device: str = "cuda"):
        import torch
        self.N, self.ns, self.L, self.win, self.H = N, ns, lattice, win, hidden
        self.m = lattice * lattice
        self.K0 = 2 * win * win + self.m
        self.K0p = (self.K0 + 31) // 32 * 32
        self.device = device
        rng = np.random.default_rng(seed)

        def he(fan_in, shape, gain=2.0):
            return rng.uniform(-1, 1, shape) * np.sqrt(3.0 * gain / fan_in)

        init = {
            "W1": he(self.K0, (self.K0p, hidden)), "b1": np.zeros(hidden),
            "W2": he(hidden, (hidden, hidden)), "b2": np.zeros(hidden),
            "W3": he(hidden, (hidden, hidden)), "b3": np.zeros(hidden),
            "W4": he(hidden, (hidden, N), gain=0.1), "b4": np.zeros(N),
            "Ws": np.zeros((self.K0p, N)),
        }
        init["W1"][self.K0:] = 0.0
        self.params: Dict[str, "torch.Tensor"] = {}
        for k, v in init.items():
            self.params[k] = torch.tensor(v, dtype=torch.float32, device=device)
        self._bf = {k: to_bf16(v) for k, v in self.params.items() if k.startswith("W")}
        self._split_ws()
        self._opt = None
        self.step = 0

    def _split_ws(self):
        import torch
        w = self.params["Ws"]
        hi = torch.empty(w.shape, dtype=torch.int16, device=self.device)
        lo = torch.empty_like(hi)
        _ck(_lib().nmpc_split_bf16(_p(w), _p(hi), _p(lo), w.numel(), _stream()), "nmpc_split_bf16")
        self._bf["Ws"], self._bf["Ws_lo"] = hi, lo

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
            "X": h(rows, self.K0p), "Xlo": h(rows, self.K0p),
            "H1": f(rows, H), "H1b": h(rows, H), "H2": f(rows, H), "H2b": h(rows, H),
            "H3": f(rows, H), "H3b": h(rows, H), "Y": f(rows, N),
            "dY": f(rows, N), "dYb": h(rows, N), "T": f(rows, N), "sse": f(rows),
            "dH": f(rows, H), "dHb": h(rows, H),
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
        _ck(_lib().nmpc_net_windows(_p(x0), _p(xref), count, self.ns, self.L, self.win,
                                    _p(b["X"]), _p(b["Xlo"]), self.K0p, _stream()),
            "nmpc_net_windows")
        H, N, K0 = self.H, self.N, self.K0p
        gemm(b["X"], W["W1"], rows, H, K0, C=b["H1"], bias=P["b1"], relu=True, Cb=b["H1b"])
        gemm(b["H1b"], W["W2"], rows, H, H, C=b["H2"], bias=P["b2"], relu=True, Cb=b["H2b"])
        gemm(b["H2b"], W["W3"], rows, H, H, C=b["H3"], bias=P["b3"], relu=True, Cb=b["H3b"])
        gemm(b["H3b"], W["W4"], rows, N, H, C=b["Y"], bias=P["b4"])
        gemm(b["X"], W["Ws"], rows, N, K0, C=b["Y"], beta=1.0)
        gemm(b["X"], W["Ws_lo"], rows, N, K0, C=b["Y"], beta=1.0)
        gemm(b["Xlo"], W["Ws"], rows, N, K0, C=b["Y"], beta=1.0)
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
        H, N, K0 = self.H, self.N, self.K0p
        _ck(_lib().nmpc_pack_inputs(_p(u_target), count, N, self.m, 1.0 / U_SCALE, _p(b["T"]), N,
                                    _stream()), "nmpc_pack_inputs")
        scale = 2.0 / (rows * N)
        _ck(_lib().nmpc_mse_grad(_p(Y), N, _p(b["T"]), N, rows, N, scale, _p(b["dY"]), _p(b["dYb"]),
                                 N, _p(b["sse"]), _stream()), "nmpc_mse_grad")
        g = {k: torch.empty_like(v) for k, v in self.params.items()}
        W = self._bf
        lib = _lib()
        # output layer and skip
        gemm(b["H3b"], b["dYb"], H, N, rows, ta=1, lda=H, ldb=N, C=g["W4"])
        gemm(b["X"], b["dYb"], K0, N, rows, ta=1, lda=K0, ldb=N, C=g["Ws"])
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

    def adam_step(self, grads, lr=1e-3, wd=0.0, b1=0.9, b2=0.999, eps=1e-8):
        import torch
        if self._opt is None:
            self._opt = {k: (torch.zeros_like(v), torch.zeros_like(v)) for k, v in self.params.items()}
        self.step += 1
        for k, w in self.params.items():
            m, v = self._opt[k]
            wb = None if k == "Ws" else self._bf.get(k)
            _ck(_lib().nmpc_adam(_p(w), _p(grads[k]), _p(m), _p(v), _p(wb), w.numel(),
                                 lr, b1, b2, eps, wd if k.startswith("W") else 0.0, self.step,
                                 _stream()), "nmpc_adam")
        self._split_ws()

    # ------------------------------------------------------------ state

    def state(self) -> Dict[str, np.ndarray]:
        return {k: v.detach().cpu().numpy() for k, v in self.params.items()}

    def load_state(self, st: Dict[str, np.ndarray]):
        import torch
        for k in self.params:
            self.params[k] = torch.tensor(np.asarray(st[k], dtype=np.float32), device=self.device)
        self._bf = {k: to_bf16(v) for k, v in self.params.items() if k.startswith("W")}
        self._split_ws()
        self._opt = None

    def save(self, path: str, meta: Optional[dict] = None):
        """Weights (fp32) + JSON header with the architecture and training facts."""
        header = {"format": "nmpc-patchnet-v1", "N": self.N, "ns": self.ns, "lattice": self.L,
                  "win": self.win, "hidden": self.H, "step": self.step, "meta": meta or {}}
        np.savez_compressed(path, header=np.frombuffer(json.dumps(header).encode(), np.uint8),
                            **self.state())

    @classmethod
    def load(cls, path: str, device: str = "cuda") -> "PatchNet":
        z = np.load(path, allow_pickle=False)
        header = json.loads(bytes(z["header"]).decode())
        if header.get("format") != "nmpc-patchnet-v1":
            raise ValueError(f"{path}: not a patch-net checkpoint")
        net = cls(N=header["N"], ns=header["ns"], lattice=header["lattice"], win=header["win"],
                  hidden=header["hidden"], device=device)
        net.load_state({k: z[k] for k in net.params})
        net.step = header["step"]
        net.meta = header["meta"]
        return net
