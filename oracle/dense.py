"""Dense numpy forms of the NMPC KKT system (oracle O1; test infrastructure only).

Every function here builds explicit matrices for *tiny* instances so that the
quantities the paper defines can be checked by textbook linear algebra:

* ``kkt``            -- K_i of Sec. 3.2 (eq. KKT), from dense L and B.
* ``lagrangian``     -- the scalar whose gradient K is (cost of eq. nlp plus
                        lambda_i^T times the backward-Euler state equation).
* ``jacobian``       -- the block-tridiagonal Newton matrix of eq. KKT_sys
                        (diagonal blocks D_i, couplings M_L, M_U).
* ``newton``         -- Newton's method of Sec. 3.3 with alpha = 1.
* ``split_DLU``      -- D, L, U of Sec. 4.2 and the D-bar / D-tilde split of
                        eq. decom (Lemma lemma_rho0).
* ``lq_condensed``   -- for linear dynamics (k1 = 0), the exact optimum of the
                        quadratic program obtained by eliminating the states.
* ``nlp_reduced``    -- for nonlinear dynamics, the NLP optimum of eq. nlp by
                        direct minimization over u with states from implicit
                        (backward-Euler) simulation.

Vector ordering: stage-major s_i = (x_i, u_i, lambda_i); K_i = (state row,
input row, costate row) as printed in Sec. 3.2.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.optimize

from nmpc_inputs import Problem


def lap_matrix(P: Problem) -> np.ndarray:
    """Central-difference Laplacian on the interior nodes, zero Dirichlet values."""
    Tx = (np.diag(-2.0 * np.ones(P.nsx)) + np.diag(np.ones(P.nsx - 1), 1)
          + np.diag(np.ones(P.nsx - 1), -1)) / P.dx ** 2
    if P.dim == 1:
        return Tx
    Ty = (np.diag(-2.0 * np.ones(P.nsy)) + np.diag(np.ones(P.nsy - 1), 1)
          + np.diag(np.ones(P.nsy - 1), -1)) / P.dy ** 2
    return np.kron(np.eye(P.nsy), Tx) + np.kron(Ty, np.eye(P.nsx))


def _ref(P, xref, i):
    xref = np.asarray(xref)
    return xref[i] if xref.ndim == 2 else xref


def f_dyn(P: Problem, L, B, x, u):
    k = P.k0 * (1.0 + P.k1 * x)
    return k * (L @ x) + B @ u


def fx_mat(P: Problem, L, x):
    """grad_x f = diag(k(x)) L + diag(k' L x)."""
    k = P.k0 * (1.0 + P.k1 * x)
    return k[:, None] * L + np.diag(P.k0 * P.k1 * (L @ x))


def hxx_mat(P: Problem, L, lam):
    """grad_xx^2 H = q I + k' (diag(lam) L + L diag(lam))."""
    kp = P.k0 * P.k1
    return P.q * np.eye(L.shape[0]) + kp * (lam[:, None] * L + L * lam[None, :])


def barrier(P: Problem, u):
    """Phi(u) = -tau sum_j (ln(u_j - u_lo) + ln(u_hi - u_j)) (eq. nlp_relaxed with
    the input box as G); 0 without a box (tau = 0)."""
    if P.tau <= 0.0:
        return 0.0
    return -P.tau * float(np.sum(np.log(u - P.u_lo) + np.log(P.u_hi - u)))


def barrier_grad(P: Problem, u):
    if P.tau <= 0.0:
        return np.zeros_like(u)
    return -P.tau / (u - P.u_lo) + P.tau / (P.u_hi - u)


def barrier_hess(P: Problem, u):
    """Diagonal of the barrier's Hessian."""
    if P.tau <= 0.0:
        return np.zeros_like(u)
    return P.tau / (u - P.u_lo) ** 2 + P.tau / (P.u_hi - u) ** 2


def alpha_max(P: Problem, U, DU):
    """Largest alpha in (0, 1] with G(u - alpha du) >= 0.005 G(u) for every input
    (eq. eq_alphamax), by bisection on the rule itself (no closed form used)."""
    if P.tau <= 0.0:
        return 1.0
    U = np.asarray(U); DU = np.asarray(DU)

    def ok(a):
        un = U - a * DU
        return (np.all(un - P.u_lo >= 0.005 * (U - P.u_lo))
                and np.all(P.u_hi - un >= 0.005 * (P.u_hi - U)))
    if ok(1.0):
        return 1.0
    lo, hi = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if ok(mid) else (lo, mid)
    return lo


def kkt(P: Problem, x0, xref, X, U, LAM, UT=None):
    """(KX [N,n], KU [N,m], KL [N,n]); UT None means ut = u (gamma term zero)."""
    L = lap_matrix(P)
    B = P.dense_B()
    N = P.N
    KX = np.zeros((N, P.n)); KU = np.zeros((N, P.m)); KL = np.zeros((N, P.n))
    for i in range(N):
        xp = x0 if i == 0 else X[i - 1]
        x, u, lam = X[i], U[i], LAM[i]
        KX[i] = xp - x + P.h * f_dyn(P, L, B, x, u)
        reg = 0.0 if UT is None else P.gamma * (u - UT[i])
        KU[i] = P.h * (P.r * u + barrier_grad(P, u) + B.T @ lam) + reg
        lnext = LAM[i + 1] if i + 1 < N else np.zeros(P.n)
        KL[i] = lnext - lam + P.h * (P.q * (x - _ref(P, xref, i)) + fx_mat(P, L, x).T @ lam)
    return KX, KU, KL


def norms(P: Problem, KX, KU, KL):
    """(r_scaled, r_paper): r_paper = |K|_inf; r_scaled divides input rows by h r,
    costate rows by h."""
    rp = max(np.max(np.abs(KX)), np.max(np.abs(KU)), np.max(np.abs(KL)))
    rs = max(np.max(np.abs(KX)), np.max(np.abs(KU)) / (P.h * P.r), np.max(np.abs(KL)) / P.h)
    return rs, rp


def lagrangian(P: Problem, x0, xref, X, U, LAM, UT=None):
    """sum_i h (l_i + Phi(u_i)) + gamma/2 |u_i - ut_i|^2
    + lam_i^T (x_{i-1} - x_i + h f(u_i, x_i))."""
    L = lap_matrix(P)
    B = P.dense_B()
    tot = 0.0
    for i in range(P.N):
        xp = x0 if i == 0 else X[i - 1]
        d = X[i] - _ref(P, xref, i)
        tot += P.h * 0.5 * (P.q * d @ d + P.r * U[i] @ U[i]) + P.h * barrier(P, U[i])
        if UT is not None:
            e = U[i] - UT[i]
            tot += 0.5 * P.gamma * e @ e
        tot += LAM[i] @ (xp - X[i] + P.h * f_dyn(P, L, B, X[i], U[i]))
    return tot


def pack(X, U, LAM):
    return np.concatenate([np.concatenate([X[i], U[i], LAM[i]]) for i in range(X.shape[0])])


def unpack(P: Problem, S):
    w = 2 * P.n + P.m
    S = S.reshape(P.N, w)
    return S[:, :P.n].copy(), S[:, P.n:P.n + P.m].copy(), S[:, P.n + P.m:].copy()


def pack_K(KX, KU, KL):
    return pack(KX, KU, KL)


def stage_block(P: Problem, L, B, x, lam, gamma, u=None):
    """D_i = grad_{s_i} K_i (rows: state, input, costate; cols: x, u, lam); u: the
    stage's inputs (the barrier's Hessian; needed with an input box)."""
    n, m, h = P.n, P.m, P.h
    Fx = fx_mat(P, L, x)
    D = np.zeros((2 * n + m, 2 * n + m))
    D[:n, :n] = h * Fx - np.eye(n)
    D[:n, n:n + m] = h * B
    bh = np.zeros(m) if u is None else barrier_hess(P, np.asarray(u))
    D[n:n + m, n:n + m] = np.diag(h * (P.r + bh) + gamma)
    D[n:n + m, n + m:] = h * B.T
    D[n + m:, :n] = h * hxx_mat(P, L, lam)
    D[n + m:, n + m:] = h * Fx.T - np.eye(n)
    return D


def jacobian(P: Problem, X, U, LAM, gamma=None):
    """Full block-tridiagonal Jacobian of K (eq. KKT_sys)."""
    gamma = P.gamma if gamma is None else gamma
    L = lap_matrix(P)
    B = P.dense_B()
    n, m, N = P.n, P.m, P.N
    w = 2 * n + m
    J = np.zeros((N * w, N * w))
    for i in range(N):
        J[i * w:(i + 1) * w, i * w:(i + 1) * w] = stage_block(P, L, B, X[i], LAM[i], gamma, U[i])
        if i > 0:      # M_L: state row of stage i on x_{i-1}
            J[i * w:i * w + n, (i - 1) * w:(i - 1) * w + n] = np.eye(n)
        if i + 1 < N:  # M_U: costate row of stage i on lam_{i+1}
            J[i * w + n + m:(i + 1) * w, (i + 1) * w + n + m:(i + 2) * w] = np.eye(n)
    return J


def newton(P: Problem, x0, xref, X, U, LAM, tol=1e-13, max_it=30, gamma=0.0):
    """Newton's method on K = 0 (gamma = 0: the exact KKT Jacobian)."""
    S = pack(X, U, LAM)
    hist = []
    for _ in range(max_it):
        Xk, Uk, Lk = unpack(P, S)
        K = pack_K(*kkt(P, x0, xref, Xk, Uk, Lk))
        hist.append(float(np.max(np.abs(K))))
        if hist[-1] <= tol:
            break
        J = jacobian(P, Xk, Uk, Lk, gamma=gamma)
        S = S - np.linalg.solve(J, K)
    return unpack(P, S), hist


def split_DLU(P: Problem, X, U, LAM, gamma=None):
    """(D, L+U, Dbar): block diagonal, off-diagonal couplings, and D without h D-tilde."""
    gamma = P.gamma if gamma is None else gamma
    J = jacobian(P, X, U, LAM, gamma=gamma)
    n, m, N = P.n, P.m, P.N
    w = 2 * n + m
    D = np.zeros_like(J)
    for i in range(N):
        D[i * w:(i + 1) * w, i * w:(i + 1) * w] = J[i * w:(i + 1) * w, i * w:(i + 1) * w]
    LU = J - D
    Dbar = D.copy()
    for i in range(N):
        o = i * w
        Dbar[o:o + n, o + n:o + n + m] = 0.0          # h grad_u f
        Dbar[o + n:o + n + m, o + n + m:o + w] = 0.0  # h grad_u f^T
    return D, LU, Dbar


def lq_condensed(P: Problem, x0, xref):
    """Exact optimum of eq. nlp when f is affine (k1 = 0).

    States are eliminated through the backward-Euler recursion
    x_i = (I - h k0 L)^{-1} (x_{i-1} + h B u_i), giving x = Phi x0 + G u; the
    cost sum_i h (q/2 |x_i - xref|^2 + r/2 |u_i|^2) is then a least-squares
    problem in u. Returns (X, U).
    """
    assert P.k1 == 0.0
    L = lap_matrix(P)
    B = P.dense_B()
    n, m, N, h = P.n, P.m, P.N, P.h
    Minv = np.linalg.inv(np.eye(n) - h * P.k0 * L)
    Phi = np.zeros((N * n, n))
    G = np.zeros((N * n, N * m))
    A = np.eye(n)
    for i in range(N):
        A = Minv @ A
        Phi[i * n:(i + 1) * n] = A
        for j in range(i + 1):
            T = np.linalg.matrix_power(Minv, i - j + 1) @ (h * B)
            G[i * n:(i + 1) * n, j * m:(j + 1) * m] = T
    xr = np.concatenate([_ref(P, xref, i) for i in range(N)])
    # minimize q/2 |Phi x0 + G u - xr|^2 + r/2 |u|^2 (common factor h dropped)
    lhs = P.q * G.T @ G + P.r * np.eye(N * m)
    rhs = -P.q * G.T @ (Phi @ x0 - xr)
    u = np.linalg.solve(lhs, rhs)
    x = Phi @ x0 + G @ u
    return x.reshape(N, n), u.reshape(N, m)


def simulate_implicit(P: Problem, x0, U):
    """States of x_i = x_{i-1} + h f(u_i, x_i), each step solved by Newton to 1e-14."""
    L = lap_matrix(P)
    B = P.dense_B()
    X = np.zeros((P.N, P.n))
    xp = np.asarray(x0, dtype=float)
    for i in range(P.N):
        x = xp.copy()
        for _ in range(50):
            g = x - xp - P.h * f_dyn(P, L, B, x, U[i])
            if np.max(np.abs(g)) < 1e-15:
                break
            Jg = np.eye(P.n) - P.h * fx_mat(P, L, x)
            x = x - np.linalg.solve(Jg, g)
        X[i] = x
        xp = x
    return X


def nlp_reduced(P: Problem, x0, xref, U0=None):
    """Optimum of eq. nlp (no inequality constraints) by BFGS over u alone.

    The objective is the plain cost evaluated on implicitly simulated states;
    its gradient is taken by central differences, so no optimality-condition
    formula enters. Returns (X, U, result).
    """
    N, m = P.N, P.m

    def cost(uflat):
        U = uflat.reshape(N, m)
        X = simulate_implicit(P, x0, U)
        tot = 0.0
        for i in range(N):
            d = X[i] - _ref(P, xref, i)
            tot += P.h * 0.5 * (P.q * d @ d + P.r * U[i] @ U[i])
        return tot

    u0 = np.zeros(N * m) if U0 is None else np.asarray(U0, float).reshape(-1)
    scale = cost(u0) + 1e-30
    res = scipy.optimize.minimize(lambda v: cost(v) / scale, u0, method="BFGS",
                                  jac="3-point", options={"gtol": 1e-12, "maxiter": 2000})
    U = res.x.reshape(N, m)
    return simulate_implicit(P, x0, U), U, res
