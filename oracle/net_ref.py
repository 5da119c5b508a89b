"""FP64 numpy reference of the warm-start patch encoder (test infrastructure).

Same layer structure as the library's network, written with numpy slicing and
matrix products: window rows of first- and second-order feature planes, three
ReLU layers and an output layer, plus a per-actuator linear map of the rows;
mean squared error and the hand-derived backward pass. Its
gradients are pinned against central differences of its own forward pass in
the CPU tests; the GPU kernels are compared against it.
"""
from __future__ import annotations

import numpy as np


def features(x0, xref, ns=64, lattice=4, win=32, planes=5, ld=None):
    """Rows [count * L^2][ld]: for each actuator, a win x win window (starting
    (win - ns/L)/2 nodes before its cell, zero outside the grid) of each
    feature plane of xt = x0/0.1 - 1 and rt = xref/0.3 -- xt, rt and, with
    planes = 5, xt^2 - 1/3, xt rt, rt^2 - 1/3 -- then a one-hot actuator
    index, then zero padding."""
    x0 = np.asarray(x0, float).reshape(-1, ns, ns)
    xref = np.asarray(xref, float).reshape(-1, ns, ns)
    count, L = x0.shape[0], lattice
    s = ns // L
    off = (win - s) // 2
    feat = planes * win * win
    ld = ld or feat + L * L
    out = np.zeros((count * L * L, ld))
    xt = x0 / 0.1 - 1.0
    rt = xref / 0.3
    fields = [xt, rt, xt * xt - 1.0 / 3.0, xt * rt, rt * rt - 1.0 / 3.0][:planes]
    pad = win + s
    big = np.zeros((count, planes, ns + 2 * pad, ns + 2 * pad))
    for c, f in enumerate(fields):
        big[:, c, pad:pad + ns, pad:pad + ns] = f
    for b in range(count):
        for p in range(L * L):
            y0 = (p // L) * s - off + pad
            x0_ = (p % L) * s - off + pad
            out[b * L * L + p, :feat] = big[b, :, y0:y0 + win, x0_:x0_ + win].reshape(-1)
            out[b * L * L + p, feat + p] = 1.0
    return out


def skip(Ws, X):
    """Per-actuator linear map: row r (actuator r mod m) times Ws[r mod m]."""
    m = Ws.shape[0]
    Y = np.empty((X.shape[0], Ws.shape[2]))
    for p in range(m):
        Y[p::m] = X[p::m] @ Ws[p]
    return Y


def forward(params, X, Xs=None):
    """Returns (Y, cache). params: W1 [K][H], b1, W2, b2, W3, b3, W4 [H][N],
    b4, Ws [m][K][N]. The hidden layers read X, the per-actuator linear map
    reads Xs (default X)."""
    p = params
    Xs = X if Xs is None else Xs
    z1 = X @ p["W1"] + p["b1"]; h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]; h2 = np.maximum(z2, 0.0)
    z3 = h2 @ p["W3"] + p["b3"]; h3 = np.maximum(z3, 0.0)
    Y = h3 @ p["W4"] + p["b4"] + skip(p["Ws"], Xs)
    return Y, (X, h1, h2, h3, Xs)


def mse(Y, T):
    return float(np.mean((Y - T) ** 2))


def backward(params, cache, Y, T):
    """Gradients of mse(Y, T) with respect to every parameter."""
    X, h1, h2, h3, Xs = cache
    p = params
    m = p["Ws"].shape[0]
    dY = 2.0 * (Y - T) / Y.size
    g = {"W4": h3.T @ dY, "b4": dY.sum(0),
         "Ws": np.stack([Xs[q::m].T @ dY[q::m] for q in range(m)])}
    d3 = (dY @ p["W4"].T) * (h3 > 0)
    g["W3"] = h2.T @ d3; g["b3"] = d3.sum(0)
    d2 = (d3 @ p["W3"].T) * (h2 > 0)
    g["W2"] = h1.T @ d2; g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"].T) * (h1 > 0)
    g["W1"] = X.T @ d1; g["b1"] = d1.sum(0)
    return g


def bf16_round(a):
    """Round float64 values to bfloat16 (nearest even) and return them as float64."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
