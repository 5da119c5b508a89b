"""Oracle of the model engine's workloads (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module; it imports nothing from the product library. It computes, in plain
FP64 numpy/scipy, what the double-layer method computes for the further
members of the paper's PDE class (Sec. 2) that the model engine solves:

* ``plate`` -- the thin copper plate of Sec. 5: first order in time,
  ``w_t = alpha Lap w - beta (w - T_a) - rad (w^4 - T_a^4)`` with zero Neumann
  boundaries by fictitious points (eq. neumann / eq. dis_neumann with e = 0);
  the temperatures of the actuator nodes are the inputs, so those nodes are
  not states and enter the remaining nodes' stencils as ``alpha L_su u``;
* ``wave`` -- second order in time (eq. pde with a = 1): state x = (W, W_t)
  (eq. ode), ``W_tt + damp W_t = k(W) Lap W + B u``; the F_x and F_x^T
  solves of the lower layer eliminate v6 = h v7 - b6 and sweep the reduced
  system h grad_Wt g - I + h^2 grad_W g (eq. jaco2_sys);
* ``heat`` -- ``w_t = k(w) Lap w + B u`` with an arbitrary dense B.

Algorithm (Sec. 3-5, in the paper's order): KKT rows K_i of Sec. 3.2 with the
log barrier of eq. nlp_relaxed; upper layer eq. 1st_jacobi (or the
Gauss-Seidel sweeps of Sec. 4.4: eq. fgs, the backward sweep, eq. sgs) with
the fraction-to-the-boundary rule eq. alphamax; lower layer eq. step12 with
the Schur input iteration of Sec. 5.2 and point-Jacobi sweeps (Lemma
lemma_jaco) on F_x and F_x^T.

Vectors are compact: the plate's x holds its state nodes only (the grid nodes
without the actuator nodes, in node order); the wave's x is (W, W_t).
Pinned in ``tests/test_oracle_models.py``.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse as sp

from nmpc_inputs import ModelProblem


# --------------------------------------------------------------- operators

def axis_second_difference(M: int, d: float, boundary: str) -> sp.csr_matrix:
    """1D central second difference on M nodes with step d. Dirichlet: the
    nodes are interior points and the values outside are zero. Neumann: the
    nodes include both ends; the fictitious points w_{-1}, w_M are fixed by a
    zero central difference at the ends (w_{-1} = w_1, w_M = w_{M-2}), so the
    end rows read 2 (w_1 - w_0) / d^2."""
    A = sp.lil_matrix((M, M))
    for j in range(M):
        A[j, j] = -2.0
        for nb in (j - 1, j + 1):
            if 0 <= nb < M:
                A[j, nb] += 1.0
            elif boundary == "neumann" and M > 1:
                mirror = j + 1 if nb < 0 else j - 1       # the fictitious point's value
                A[j, mirror] += 1.0
    return (A / (d * d)).tocsr()


def grid_laplacian(P: ModelProblem) -> sp.csr_matrix:
    """Laplacian over all grid nodes (node iy * nsx + ix) by the 5-point
    stencil (3-point in 1D) with the problem's boundary rule."""
    Tx = axis_second_difference(P.nsx, P.dx, P.boundary)
    if P.nsy == 1:
        return Tx
    Ty = axis_second_difference(P.nsy, P.dy, P.boundary)
    return (sp.kron(sp.identity(P.nsy), Tx) + sp.kron(Ty, sp.identity(P.nsx))).tocsr()


class Ops:
    """The model's operators: state node list, L over the states, B (dense
    numpy matrices: the instances checked here are small)."""

    def __init__(self, P: ModelProblem):
        self.P = P
        L = grid_laplacian(P)
        if P.model == "plate":
            act = list(P.act)
            self.state = np.array([p for p in range(P.nodes) if p not in set(act)])
            self.act = np.array(act)
            self.L = L[self.state][:, self.state].toarray()
            self.B = (P.alpha * L[self.state][:, self.act]).toarray()
        else:
            self.state = np.arange(P.nodes)
            self.act = None
            self.L = L.toarray()
            self.B = np.asarray(P.B, dtype=np.float64)
        self.n = len(self.state)                       # spatial nodes that are states
        self.nx = 2 * self.n if P.model == "wave" else self.n
        self.m = self.B.shape[1]
        self.I = np.eye(self.n)

    # --- model functions
    def f(self, x, u):
        P = self.P
        if P.model == "plate":
            return (P.alpha * (self.L @ x) + self.B @ u - P.beta * (x - P.t_amb)
                    - P.rad * (x ** 4 - P.t_amb ** 4))
        if P.model == "heat":
            k = P.k0 * (1.0 + P.k1 * x)
            return k * (self.L @ x) + self.B @ u
        W, V = x[:self.n], x[self.n:]
        k = P.k0 * (1.0 + P.k1 * W)
        return np.concatenate([V, k * (self.L @ W) - P.damp * V + self.B @ u])

    def gw(self, W):
        """grad_W of k(W) Lap W (heat: grad_x f without B): diag(k) L + diag(k' L W)."""
        P = self.P
        k = P.k0 * (1.0 + P.k1 * W)
        return k[:, None] * self.L + np.diag(P.k0 * P.k1 * (self.L @ W))

    def fx(self, x):
        """grad_x f."""
        P = self.P
        if P.model == "plate":
            return P.alpha * self.L - np.diag(P.beta + 4.0 * P.rad * x ** 3)
        if P.model == "heat":
            return self.gw(x)
        n = self.n
        return np.block([[np.zeros((n, n)), self.I], [self.gw(x[:n]), -P.damp * self.I]])

    def fu(self):
        if self.P.model == "wave":
            return np.vstack([np.zeros((self.n, self.m)), self.B])
        return self.B

    def hxx(self, x, lam):
        """grad_xx^2 H: the cost's Hessian plus that of lam^T f."""
        P = self.P
        n = self.n
        if P.model == "plate":
            return np.diag(P.q - 12.0 * P.rad * x * x * lam)
        kp = P.k0 * P.k1
        if P.model == "heat":
            return P.q * self.I + kp * (lam[:, None] * self.L + self.L.T * lam[None, :])
        lv = lam[n:]
        Hww = P.q * self.I + kp * (lv[:, None] * self.L + self.L.T * lv[None, :])
        return scipy.linalg.block_diag(Hww, P.qv * self.I)

    def xref_vec(self, xref):
        """State reference (compact) from the given reference over the grid."""
        xref = np.asarray(xref, dtype=np.float64)
        if self.P.model == "wave":
            return np.concatenate([xref[:self.n], np.zeros(self.n)])
        return xref[self.state]

    def uref_vec(self, xref):
        """Input reference: the reference at the actuator nodes (plate), else 0."""
        if self.P.model == "plate":
            return np.asarray(xref, dtype=np.float64)[self.act]
        return np.zeros(self.m)

    def qdiag(self):
        P = self.P
        if P.model == "wave":
            return np.concatenate([np.full(self.n, P.q), np.full(self.n, P.qv)])
        return np.full(self.nx, P.q)


# ----------------------------------------------------------------- barrier

def barrier_grad(P: ModelProblem, u):
    if P.tau <= 0.0:
        return np.zeros_like(u)
    return -P.tau / (u - P.u_lo) + P.tau / (P.u_hi - u)


def barrier_hess(P: ModelProblem, u):
    if P.tau <= 0.0:
        return np.zeros_like(u)
    return P.tau / (u - P.u_lo) ** 2 + P.tau / (P.u_hi - u) ** 2


def alpha_max(P: ModelProblem, U, DU) -> float:
    """Fraction-to-the-boundary rule (eq. alphamax) for the step U - alpha DU:
    the largest alpha in (0, 1] with G(U - alpha DU) >= 0.005 G(U) for the box
    G = (u - u_lo, u_hi - u)."""
    if P.tau <= 0.0:
        return 1.0
    a = 1.0
    U = np.asarray(U).ravel()
    D = np.asarray(DU).ravel()
    pos, neg = D > 0, D < 0
    if pos.any():
        a = min(a, float(np.min(0.995 * (U[pos] - P.u_lo) / D[pos])))
    if neg.any():
        a = min(a, float(np.min(0.995 * (P.u_hi - U[neg]) / (-D[neg]))))
    return a


def feasible_inputs(P: ModelProblem, U):
    """Start inputs clipped to the box shrunk by 0.5 % of its width (strictly
    feasible S^0, Sec. 4.2); unchanged without a box."""
    U = np.array(U, dtype=np.float64)
    if P.tau > 0.0:
        d = 0.005 * (P.u_hi - P.u_lo)
        U = np.where(U < P.u_lo + d, P.u_lo + d, np.where(U > P.u_hi - d, P.u_hi - d, U))
    return U


# --------------------------------------------------------------------- KKT

def kkt_stage(ops: Ops, xp, x, u, lam, ln, ut, xr, ur):
    """K_i = (K^x, K^u, K^lambda) of one stage from x_{i-1} = xp, s_i = (x, u,
    lam), lambda_{i+1} = ln and the regularization reference ut."""
    P = ops.P
    kx = xp - x + P.h * ops.f(x, u)
    ku = P.h * (P.r * (u - ur) + ops.fu().T @ lam + barrier_grad(P, u)) + P.gamma * (u - ut)
    kl = ln - lam + P.h * (ops.qdiag() * (x - xr) + ops.fx(x).T @ lam)
    return kx, ku, kl


def kkt(ops: Ops, x0, xref, X, U, LAM, UT=None):
    """K_i (Sec. 3.2) for all stages: (KX [N][nx], KU [N][m], KL [N][nx]).
    x0: initial state (compact); UT: regularization reference u~ (default U:
    the gamma term vanishes)."""
    P = ops.P
    xr, ur = ops.xref_vec(xref), ops.uref_vec(xref)
    UT = U if UT is None else UT
    KX, KU, KL = np.zeros_like(X), np.zeros_like(U), np.zeros_like(LAM)
    for i in range(P.N):
        xp = x0 if i == 0 else X[i - 1]
        ln = LAM[i + 1] if i + 1 < P.N else np.zeros(ops.nx)
        KX[i], KU[i], KL[i] = kkt_stage(ops, xp, X[i], U[i], LAM[i], ln, UT[i], xr, ur)
    return KX, KU, KL


def norms(ops: Ops, KX, KU, KL):
    """(r_scaled, r_paper): r_paper = |K|_inf (the paper's stopping norm);
    r_scaled divides the input rows by h r and the costate rows by h."""
    P = ops.P
    ax, au, al = np.abs(KX).max(), np.abs(KU).max(), np.abs(KL).max()
    if not all(np.isfinite(v) for v in (ax, au, al)):
        return float("nan"), float("nan")
    return max(ax, au / (P.h * P.r), al / P.h), max(ax, au, al)


def residual(ops: Ops, x0, xref, X, U, LAM):
    return norms(ops, *kkt(ops, x0, xref, X, U, LAM))


# ------------------------------------------------------------- lower layer

def jacobi(A, c, n_sw: int):
    """n_sw point-Jacobi sweeps on A y = c from y = 0 (Lemma lemma_jaco)."""
    d = np.diag(A).copy()
    O = A - np.diag(d)
    y = np.zeros_like(c)
    for _ in range(n_sw):
        y = (c - O @ y) / d
    return y


def solve_fx(ops: Ops, x, c, n_sw, transpose=False):
    """Approximate solve of F_x v = c (or F_x^T v = c), F_x = h grad_x f - I,
    by point-Jacobi sweeps; for the second-order model through the reduced
    system of eq. jaco2_sys after eliminating v6."""
    P = ops.P
    h = P.h
    if P.model != "wave":
        Fx = h * ops.fx(x) - np.eye(ops.nx)
        return jacobi(Fx.T if transpose else Fx, c, n_sw)
    n = ops.n
    G = ops.gw(x[:n])
    b6, b7 = c[:n], c[n:]
    M = -(1.0 + h * P.damp) * ops.I + h * h * (G.T if transpose else G)
    if not transpose:
        # -v6 + h v7 = b6; h G v6 + (-h damp - 1) v7 = b7
        v7 = jacobi(M, b7 + h * (G @ b6), n_sw)
        v6 = h * v7 - b6
    else:
        # -v6 + h G^T v7 = b6; h v6 + (-h damp - 1) v7 = b7
        v7 = jacobi(M, b7 + h * b6, n_sw)
        v6 = h * (G.T @ v7) - b6
    return np.concatenate([v6, v7])


def stage_solve(ops: Ops, x, u, lam, b1, b2, b3, n_sw=2, n_schur=2):
    """Lower layer of one stage (Sec. 4.3, eq. step12 with the Schur input
    iteration of Sec. 5.2 from v3 = 0): returns (dx, du, dlam) ~ D_i^{-1} K_i
    for the right-hand side (b1, b2, b3) = (K^x, K^lambda, K^u)."""
    P = ops.P
    h = P.h
    Fu = h * ops.fu()
    Axx = h * ops.hxx(x, lam)
    auu = h * (P.r + barrier_hess(P, u)) + P.gamma
    v3 = np.zeros(ops.m)
    for _ in range(n_schur):
        v5 = solve_fx(ops, x, Fu @ v3 - b1, n_sw)
        v4 = solve_fx(ops, x, -b2 - Axx @ v5, n_sw, transpose=True)
        v3 = (b3 + Fu.T @ v4) / auu
    v2 = solve_fx(ops, x, b1 - Fu @ v3, n_sw)
    v1 = solve_fx(ops, x, b2 - Axx @ v2, n_sw, transpose=True)
    return v2, v3, v1


# ------------------------------------------------------------- upper layer

def sweep(ops: Ops, x0, xref, S, UT, direction, n_sw=2, n_schur=2):
    """One pass of the upper layer from S = (X, U, LAM): direction 0 is the
    Jacobi step eq. 1st_jacobi (every stage from S), +1 a forward and -1 a
    backward Gauss-Seidel sweep (each stage from the trajectory in which the
    stages visited before hold their new values). UT: regularization
    reference. Returns the new trajectory (alpha = 1)."""
    P = ops.P
    X, U, LAM = (a.copy() for a in S)
    Xn, Un, Ln = (a.copy() for a in S)
    order = range(P.N) if direction >= 0 else range(P.N - 1, -1, -1)
    xr, ur = ops.xref_vec(xref), ops.uref_vec(xref)
    for i in order:
        src = (X, U, LAM) if direction == 0 else (Xn, Un, Ln)   # new values once visited
        xp = x0 if i == 0 else src[0][i - 1]
        ln = src[2][i + 1] if i + 1 < P.N else np.zeros(ops.nx)
        kx, ku, kl = kkt_stage(ops, xp, X[i], U[i], LAM[i], ln, UT[i], xr, ur)
        dx, du, dl = stage_solve(ops, X[i], U[i], LAM[i], kx, kl, ku, n_sw, n_schur)
        Xn[i] = X[i] - dx
        Un[i] = U[i] - du
        Ln[i] = LAM[i] - dl
    return Xn, Un, Ln


SWEEPS = {"jacobi": (0,), "fgs": (1,), "bgs": (-1,), "sgs": (-1, 1)}


def cold_start(ops: Ops, x0):
    P = ops.P
    return (np.tile(x0, (P.N, 1)), np.full((P.N, ops.m), P.u_cold), np.zeros((P.N, ops.nx)))


def iterate(ops: Ops, x0, xref, S, upper="jacobi", n_sw=2, n_schur=2):
    """One upper iteration S^j -> S^{j+1}. With an input box each pass of
    the variant (one for Jacobi, FGS and BGS, two for SGS) is cut by the
    fraction-to-the-boundary rule: S <- S + alpha (S_pass - S)."""
    P = ops.P
    cur = tuple(a.copy() for a in S)
    for d in SWEEPS[upper]:
        new = sweep(ops, x0, xref, cur, S[1], d, n_sw, n_schur)
        if P.tau > 0.0:
            a = alpha_max(P, cur[1], cur[1] - new[1])
            new = tuple(c + a * (nw - c) for c, nw in zip(cur, new))
        cur = new
    return cur


def solve(ops: Ops, x0, xref, start=None, upper="jacobi", tol=1e-6, max_iter=2000, n_sw=2,
          n_schur=2, residual_kind="scaled"):
    """The double-layer method from ``start`` (default: the cold start x_i =
    x0, u_i = u_cold, lambda_i = 0) until the chosen norm of K(S^k) is <= tol.
    Returns dict(X, U, LAM, iters, r_scaled, r_paper, status)."""
    S = cold_start(ops, x0) if start is None else tuple(np.array(a, dtype=float) for a in start)
    S = (S[0], feasible_inputs(ops.P, S[1]), S[2])
    k = 0
    while True:
        rs, rp = residual(ops, x0, xref, *S)
        r = rs if residual_kind == "scaled" else rp
        if not np.isfinite(r):
            status = "nonfinite"
            break
        if r <= tol:
            status = "converged"
            break
        if k >= max_iter:
            status = "max_iter"
            break
        S = iterate(ops, x0, xref, S, upper, n_sw, n_schur)
        k += 1
    return dict(X=S[0], U=S[1], LAM=S[2], iters=k, r_scaled=rs, r_paper=rp, status=status)


# ---------------------------------------------------------- grid <-> state

def state_x0(ops: Ops, x0_grid):
    """Compact initial state from the grid-ordered input (wave: [W; W_t])."""
    x0_grid = np.asarray(x0_grid, dtype=np.float64)
    if ops.P.model == "wave":
        return x0_grid.copy()
    return x0_grid[ops.state]


def to_grid(ops: Ops, X, U=None):
    """Trajectory over the grid nodes: the plate's actuator nodes take the
    inputs' values (the node temperatures), [N][nodes]; other models return
    X unchanged."""
    if ops.P.model != "plate":
        return np.array(X)
    G = np.zeros((X.shape[0], ops.P.nodes))
    G[:, ops.state] = X
    if U is not None:
        G[:, ops.act] = U
    return G
