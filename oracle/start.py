"""Start built from an input trajectory (oracle; test infrastructure only).

Given inputs u_1..u_N, the states are the backward-Euler trajectory of the
model of eq. nlp, i.e. the state rows K^x_i = 0 of the KKT system of Sec. 3.2,
and the costates follow the adjoint recursion, the costate rows K^lam_i = 0
solved from the last stage down (lambda_{N+1} = 0). Only the input rows are
left nonzero. Each stage's nonlinear state equation is solved by Newton's
method, the linear costate equation by one solve, both with a sparse LU
factorisation (scipy), so the grids of the benchmark fit; ``dense.py`` holds
the dense form of the same state recursion for tiny grids.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from nmpc_inputs import Problem


def lap_sparse(P: Problem) -> sp.csr_matrix:
    """Central-difference Laplacian on the interior nodes (zero Dirichlet values),
    node (iy, ix) at index iy * nsx + ix."""
    def axis(ns, d):
        e = np.ones(ns)
        return sp.diags([e[:-1], -2.0 * e, e[:-1]], [-1, 0, 1]) / (d * d)
    Tx = axis(P.nsx, P.dx)
    if P.dim == 1:
        return Tx.tocsr()
    Ty = axis(P.nsy, P.dy)
    return (sp.kron(sp.identity(P.nsy), Tx) + sp.kron(Ty, sp.identity(P.nsx))).tocsr()


def _f_x(P: Problem, L, x):
    """Jacobian of f(u, x) = k(x) * (L x) + B u with respect to x:
    diag(k(x)) L + diag(k'(x) * (L x)), k(x) = k0 (1 + k1 x)."""
    k = P.k0 * (1.0 + P.k1 * x)
    return sp.diags(k) @ L + sp.diags(P.k0 * P.k1 * (L @ x))


def input_start(P: Problem, x0, xref, U):
    """(X, U, LAM) with K^x_i = 0 and K^lam_i = 0 for every stage.

    States: x_i - x_{i-1} - h f(u_i, x_i) = 0, Newton from x_{i-1} until the
    step is at the rounding level. Costates: (h f_x(x_i) - I)^T lambda_i =
    -(lambda_{i+1} + h q (x_i - xref_i)). xref: one vector, or one per stage.
    """
    L = lap_sparse(P)
    B = P.dense_B()
    I = sp.identity(P.n, format="csr")
    U = np.array(U, dtype=float).reshape(P.N, P.m)
    if P.tau > 0.0:   # strictly feasible start inside an input box (Sec. 4.2)
        d = 0.005 * (P.u_hi - P.u_lo)
        U = np.where(U < P.u_lo + d, P.u_lo + d, np.where(U > P.u_hi - d, P.u_hi - d, U))
    xref = np.asarray(xref, dtype=float)
    X = np.zeros((P.N, P.n))
    LAM = np.zeros((P.N, P.n))
    xp = np.asarray(x0, dtype=float).reshape(P.n)
    for i in range(P.N):
        bu = B @ U[i]
        x = xp.copy()
        for _ in range(60):
            k = P.k0 * (1.0 + P.k1 * x)
            g = x - xp - P.h * (k * (L @ x) + bu)
            step = spla.spsolve((I - P.h * _f_x(P, L, x)).tocsc(), g)
            x = x - step
            if np.max(np.abs(step)) <= 1e-15 * (1.0 + np.max(np.abs(x))):
                break
        X[i] = x
        xp = x
    nxt = np.zeros(P.n)
    for i in range(P.N - 1, -1, -1):
        xr = xref[i] if xref.ndim == 2 else xref
        A = (P.h * _f_x(P, L, X[i]) - I).T.tocsc()
        LAM[i] = spla.spsolve(A, -(nxt + P.h * P.q * (X[i] - xr)))
        nxt = LAM[i]
    return X, U.copy(), LAM
