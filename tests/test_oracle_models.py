"""Pins of the model engine's oracle (``oracle/models.py``) against what the
paper and the mathematics fix, on tiny instances (CPU only):

* the boundary rules of the stencil: discrete cosine (Neumann, fictitious
  points) and sine (Dirichlet) eigenpairs in closed form;
* K equals the central-difference gradient of the Lagrangian of eq.
  nlp_relaxed (signs, Jacobians, the barrier and the regularization);
* the stage blocks used by the lower layer equal the finite-difference
  Jacobian of K_i; Newton with those blocks converges quadratically and the
  double-layer fixed point (Jacobi, SGS) equals Newton's point;
* the lower layer with many sweeps equals the dense solve D_i^{-1} K_i, and
  the second-order model's v6 elimination (eq. jaco2_sys) equals the direct
  F_x / F_x^T solve;
* the plate's fixed point is the optimum of the relaxed NLP found by direct
  minimization over the inputs (states simulated by backward Euler);
* the fraction-to-the-boundary step (eq. alphamax) by bisection; Gauss-Seidel
  sweeps of a linear instance equal the block splitting formulas.
"""
import numpy as np
import pytest
import scipy.optimize

from nmpc_inputs import ModelProblem, gaussian_factors, make_plate_problem, make_wave_problem
from oracle import models as om


def tiny_plate(tau=1.0, gamma=0.05, rad=None, N=3):
    """5 x 5 Neumann grid, 4 actuator nodes, boxed inputs; constants scaled so
    that every term matters at this size."""
    P = make_plate_problem()
    return P.with_(nsx=5, nsy=5, N=N, h=2.0, act=[6, 8, 16, 18], tau=tau, gamma=gamma,
                   alpha=0.004, beta=2e-3, rad=P.rad * 1e3 if rad is None else rad)


def plate_instance(P, seed=0):
    rng = np.random.default_rng(seed)
    x0 = P.t_amb + rng.uniform(0, 60, P.nodes)
    xref = P.t_amb + 100 + rng.uniform(0, 150, P.nodes)
    return x0, xref


def tiny_wave(N=3, ns=4):
    g = gaussian_factors(ns, 2, 0.2)
    B = np.kron(g.T, g.T)
    h = (1.0 / (ns + 1)) * np.sqrt(0.3 / (4 * 1.5))
    return ModelProblem(model="wave", nsx=ns, nsy=ns, N=N, h=h, boundary="dirichlet", B=B,
                        q=1.0, qv=0.1, r=0.01, gamma=0.01 * h, k0=1.0, k1=0.5, damp=2.0)


def wave_instance(P, seed=0):
    rng = np.random.default_rng(seed)
    x0 = np.concatenate([rng.uniform(0, 0.2, P.nodes), rng.uniform(-0.1, 0.1, P.nodes)])
    return x0, rng.uniform(-0.3, 0.3, P.nodes)


def tiny_heat(N=3):
    rng = np.random.default_rng(4)
    B = rng.uniform(0, 1, (12, 3))
    h = 0.2 / (0.75 * 25)
    return ModelProblem(model="heat", nsx=4, nsy=3, N=N, h=h, boundary="dirichlet", B=B,
                        q=1.0, r=0.01, gamma=0.01 * h, k0=0.5, k1=0.5)


def heat_instance(P, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 0.2, P.nodes), rng.uniform(-0.3, 0.3, P.nodes)


CASES = {"plate": (tiny_plate, plate_instance), "wave": (tiny_wave, wave_instance),
         "heat": (tiny_heat, heat_instance)}


def setup(name, **kw):
    mk, inst = CASES[name]
    P = mk(**kw)
    ops = om.Ops(P)
    x0g, xref = inst(P)
    return P, ops, om.state_x0(ops, x0g), xref


def random_traj(ops, x0, seed=1):
    rng = np.random.default_rng(seed)
    P = ops.P
    X = np.tile(x0, (P.N, 1)) + rng.normal(size=(P.N, ops.nx)) * (3.0 if P.model == "plate" else 0.03)
    if P.tau > 0:
        U = rng.uniform(P.u_lo + 0.2 * (P.u_hi - P.u_lo), P.u_hi - 0.2 * (P.u_hi - P.u_lo),
                        (P.N, ops.m))
    else:
        U = rng.normal(size=(P.N, ops.m))
    L = rng.normal(size=(P.N, ops.nx)) * (50.0 if P.model == "plate" else 0.01)
    return X, U, L


# ---------------------------------------------------------------- stencils

@pytest.mark.parametrize("M", [2, 5, 13])
def test_neumann_second_difference_has_cosine_eigenpairs(M):
    d = 1.0 / (M - 1)
    A = om.axis_second_difference(M, d, "neumann")
    j = np.arange(M)
    for a in range(M):
        v = np.cos(np.pi * a * j / (M - 1))
        lam = -4.0 / d ** 2 * np.sin(np.pi * a / (2 * (M - 1))) ** 2
        np.testing.assert_allclose(A @ v, lam * v, atol=1e-9 / d ** 2)


def test_grid_laplacian_eigenpairs_both_boundaries():
    P = make_plate_problem().with_(nsx=6, nsy=4)
    L = om.grid_laplacian(P)
    ix, iy = np.meshgrid(np.arange(6), np.arange(4))
    for a, b in [(0, 0), (1, 2), (5, 3)]:
        v = (np.cos(np.pi * a * ix / 5) * np.cos(np.pi * b * iy / 3)).ravel()
        lam = -4 / P.dx ** 2 * np.sin(np.pi * a / 10) ** 2 - 4 / P.dy ** 2 * np.sin(np.pi * b / 6) ** 2
        np.testing.assert_allclose(L @ v, lam * v, atol=1e-9 * abs(lam) + 1e-9)
    W = tiny_wave()
    L = om.grid_laplacian(W)
    ix, iy = np.meshgrid(np.arange(1, 5), np.arange(1, 5))
    for a, b in [(1, 1), (2, 3)]:
        v = (np.sin(np.pi * a * ix * W.dx) * np.sin(np.pi * b * iy * W.dy)).ravel()
        lam = -4 / W.dx ** 2 * (np.sin(np.pi * a * W.dx / 2) ** 2 + np.sin(np.pi * b * W.dy / 2) ** 2)
        np.testing.assert_allclose(L @ v, lam * v, atol=1e-9 * abs(lam))


def test_plate_constant_field_is_stationary_without_losses():
    """A uniform temperature (states and actuators alike) has a zero Laplacian
    under zero-Neumann boundaries: alpha L_ss x + B u = 0."""
    P = make_plate_problem()
    ops = om.Ops(P)
    x = np.full(ops.n, 431.0)
    u = np.full(ops.m, 431.0)
    np.testing.assert_allclose(P.alpha * (ops.L @ x) + ops.B @ u, 0.0, atol=1e-12)
    assert ops.n == 153 and ops.m == 16


# ------------------------------------------------------------ KKT and blocks

def lagrangian(ops, x0, xref, X, U, LAM, UT):
    """sum_i h (l_i + Phi(u_i)) + gamma/2 |u_i - u~_i|^2 + lam_i^T (x_{i-1} - x_i + h f)."""
    P = ops.P
    xr, ur, qd = ops.xref_vec(xref), ops.uref_vec(xref), ops.qdiag()
    tot = 0.0
    for i in range(P.N):
        xp = x0 if i == 0 else X[i - 1]
        l = 0.5 * np.sum(qd * (X[i] - xr) ** 2) + 0.5 * P.r * np.sum((U[i] - ur) ** 2)
        phi = 0.0
        if P.tau > 0:
            phi = -P.tau * np.sum(np.log(U[i] - P.u_lo) + np.log(P.u_hi - U[i]))
        tot += P.h * (l + phi) + 0.5 * P.gamma * np.sum((U[i] - UT[i]) ** 2)
        tot += LAM[i] @ (xp - X[i] + P.h * ops.f(X[i], U[i]))
    return tot


@pytest.mark.parametrize("name", list(CASES))
def test_kkt_is_the_gradient_of_the_lagrangian(name):
    P, ops, x0, xref = setup(name)
    X, U, L = random_traj(ops, x0)
    UT = U + 0.01 * np.random.default_rng(3).normal(size=U.shape)
    KX, KU, KL = om.kkt(ops, x0, xref, X, U, L, UT)
    rng = np.random.default_rng(7)
    for arr, K in ((X, KL), (U, KU), (L, KX)):
        for _ in range(12):
            i, j = rng.integers(arr.shape[0]), rng.integers(arr.shape[1])
            e = 1e-5 * max(1.0, abs(arr[i, j]))
            arr[i, j] += e
            fp = lagrangian(ops, x0, xref, X, U, L, UT)
            arr[i, j] -= 2 * e
            fm = lagrangian(ops, x0, xref, X, U, L, UT)
            arr[i, j] += e
            g = (fp - fm) / (2 * e)
            assert abs(g - K[i, j]) <= 1e-6 * max(1.0, abs(K[i, j])) * (1e3 if P.model == "plate" else 1), (i, j, g, K[i, j])


def stage_block(ops, x, u, lam):
    """D_i = d K_i / d (x_i, u_i, lambda_i) (rows K^x, K^u, K^lambda) from the
    model's derivative functions."""
    P = ops.P
    h, nx, m = P.h, ops.nx, ops.m
    Fx = h * ops.fx(x) - np.eye(nx)
    Fu = h * ops.fu()
    Axx = h * ops.hxx(x, lam)
    Auu = np.diag(h * (P.r + om.barrier_hess(P, u)) + P.gamma)
    Z = np.zeros
    return np.block([[Fx, Fu, Z((nx, nx))],
                     [Z((m, nx)), Auu, Fu.T],
                     [Axx, Z((nx, m)), Fx.T]])


@pytest.mark.parametrize("name", list(CASES))
def test_stage_blocks_are_the_jacobian_of_k(name):
    P, ops, x0, xref = setup(name)
    X, U, L = random_traj(ops, x0)
    xr, ur = ops.xref_vec(xref), ops.uref_vec(xref)
    i = 1
    s = np.concatenate([X[i], U[i], L[i]])
    nx, m = ops.nx, ops.m

    def k_of(s):
        x, u, lam = s[:nx], s[nx:nx + m], s[nx + m:]
        kx, ku, kl = om.kkt_stage(ops, X[i - 1], x, u, lam, L[i + 1], U[i], xr, ur)
        return np.concatenate([kx, ku, kl])
    J = np.zeros((len(s), len(s)))
    for c in range(len(s)):
        e = 1e-6 * max(1.0, abs(s[c]))
        sp_, sm = s.copy(), s.copy()
        sp_[c] += e
        sm[c] -= e
        J[:, c] = (k_of(sp_) - k_of(sm)) / (2 * e)
    D = stage_block(ops, X[i], U[i], L[i])
    assert np.abs(J - D).max() <= 1e-5 * max(1.0, np.abs(D).max())


def newton(ops, x0, xref, S, iters=30):
    """Newton's method on the full KKT system (Sec. 3.3), block-tridiagonal
    matrix from the stage blocks and the identity couplings; returns the
    iterates' residual history and the solution."""
    P = ops.P
    nx, m = ops.nx, ops.m
    w = 2 * nx + m
    X, U, L = (a.copy() for a in S)
    hist = []
    for _ in range(iters):
        KX, KU, KL = om.kkt(ops, x0, xref, X, U, L)
        K = np.concatenate([np.concatenate([KX[i], KU[i], KL[i]]) for i in range(P.N)])
        hist.append(np.abs(K).max())
        if hist[-1] <= 1e-13 * max(1.0, np.abs(U).max()):
            break
        J = np.zeros((P.N * w, P.N * w))
        for i in range(P.N):
            J[i * w:(i + 1) * w, i * w:(i + 1) * w] = stage_block(ops, X[i], U[i], L[i]) - np.diag(
                np.concatenate([np.zeros(nx), np.full(m, P.gamma), np.zeros(nx)]))
            if i > 0:       # K^x_i depends on x_{i-1} with the identity
                J[i * w:i * w + nx, (i - 1) * w:(i - 1) * w + nx] = np.eye(nx)
            if i + 1 < P.N:   # K^lambda_i depends on lambda_{i+1} with the identity
                J[i * w + nx + m:(i + 1) * w, (i + 1) * w + nx + m:(i + 2) * w] = np.eye(nx)
        d = np.linalg.solve(J, K)
        for i in range(P.N):
            X[i] -= d[i * w:i * w + nx]
            U[i] -= d[i * w + nx:i * w + nx + m]
            L[i] -= d[i * w + nx + m:(i + 1) * w]
    return hist, (X, U, L)


@pytest.mark.parametrize("name", list(CASES))
def test_fixed_point_equals_newton_point(name):
    """gamma does not enter the fixed point (u~ = u^k): Newton on K with the
    gamma term dropped converges quadratically to the same point that the
    Jacobi and the SGS double-layer iterations reach."""
    P, ops, x0, xref = setup(name)
    # rounding floor of r_scaled: the plate's inputs sit near the box (barrier
    # Hessian ~1e4) at values ~700, so its K^u rows carry ~1e-10 of rounding
    tol = 1e-8 if P.model == "plate" else 1e-11
    o = om.solve(ops, x0, xref, upper="jacobi", tol=tol, max_iter=5000, n_sw=6, n_schur=4)
    assert o["status"] == "converged"
    # start near the point (inputs moved towards the box centre: stays feasible)
    U1 = o["U"] + 1e-5 * (P.u_cold - o["U"]) if P.tau > 0 else o["U"] * (1 + 1e-5)
    hist, (X, U, L) = newton(ops, x0, xref, (o["X"] + 0.0, U1, o["LAM"] * (1 + 1e-5)))
    assert hist[-1] <= 1e-9
    # quadratic convergence: few steps from a 1e-5 perturbation to the floor,
    # each at least squaring the relative residual (up to a constant)
    tail = [h for h in hist if h > 1e-9]
    assert len(tail) <= 5
    for a, b in zip(tail, tail[1:]):
        assert b <= 1e3 * a * a / hist[0] + 1e-9
    np.testing.assert_allclose(o["U"], U, rtol=0, atol=1e-8 * np.abs(U).max())
    s = om.solve(ops, x0, xref, upper="sgs", tol=tol, max_iter=5000)
    assert s["status"] == "converged" and s["iters"] < o["iters"]
    np.testing.assert_allclose(s["U"], U, rtol=0, atol=1e-8 * np.abs(U).max())
    if P.tau > 0:
        assert np.all(U > P.u_lo) and np.all(U < P.u_hi)


@pytest.mark.parametrize("name", list(CASES))
def test_lower_layer_with_many_sweeps_is_the_dense_stage_solve(name):
    P, ops, x0, xref = setup(name)
    X, U, L = random_traj(ops, x0)
    i = 1
    KX, KU, KL = om.kkt(ops, x0, xref, X, U, L)
    dx, du, dl = om.stage_solve(ops, X[i], U[i], L[i], KX[i], KL[i], KU[i], n_sw=400, n_schur=300)
    D = stage_block(ops, X[i], U[i], L[i])
    ref = np.linalg.solve(D, np.concatenate([KX[i], KU[i], KL[i]]))
    got = np.concatenate([dx, du, dl])
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
    # one sweep and no Schur step: dx = K^x / diag(F_x) (point Jacobi from zero)
    if P.model != "wave":
        dx1, du1, _ = om.stage_solve(ops, X[i], U[i], L[i], KX[i], KL[i], KU[i], n_sw=1, n_schur=0)
        Fx = P.h * ops.fx(X[i]) - np.eye(ops.nx)
        np.testing.assert_allclose(dx1, KX[i] / np.diag(Fx), rtol=1e-12)


def test_wave_elimination_equals_the_direct_solve():
    P, ops, x0, xref = setup("wave")
    X, U, L = random_traj(ops, x0)
    c = np.random.default_rng(2).normal(size=ops.nx)
    Fx = P.h * ops.fx(X[0]) - np.eye(ops.nx)
    np.testing.assert_allclose(om.solve_fx(ops, X[0], c, 200), np.linalg.solve(Fx, c), atol=1e-11)
    np.testing.assert_allclose(om.solve_fx(ops, X[0], c, 200, transpose=True),
                               np.linalg.solve(Fx.T, c), atol=1e-11)
    # the reduced matrix is diagonally dominant at this step (eq. jaco2_sys)
    n = ops.n
    M = -(1 + P.h * P.damp) * np.eye(n) + P.h ** 2 * ops.gw(X[0][:n])
    off = np.abs(M).sum(1) - np.abs(np.diag(M))
    assert np.all(off < np.abs(np.diag(M)))


def simulate_plate(ops, x0, U):
    """States of the backward-Euler model for inputs U (Newton per stage)."""
    P = ops.P
    X = np.zeros((P.N, ops.n))
    xp = x0.copy()
    for i in range(P.N):
        x = xp.copy()
        for _ in range(50):
            g = x - xp - P.h * ops.f(x, U[i])
            J = np.eye(ops.n) - P.h * ops.fx(x)
            st = np.linalg.solve(J, g)
            x -= st
            if np.abs(st).max() <= 1e-12 * np.abs(x).max():
                break
        X[i] = x
        xp = x
    return X


def test_plate_fixed_point_is_the_relaxed_nlp_optimum():
    """Direct minimization of sum_i h (l_i + Phi(u_i)) over the inputs, the
    states simulated by the backward-Euler model: no optimality formula is
    involved, so this pins the KKT rows, their signs and the barrier."""
    P, ops, x0, xref = setup("plate", tau=5.0, gamma=0.02)
    xr, ur = ops.xref_vec(xref), ops.uref_vec(xref)
    o = om.solve(ops, x0, xref, upper="sgs", tol=1e-8, max_iter=5000)
    assert o["status"] == "converged"

    def cost(v):
        U = v.reshape(P.N, ops.m)
        if np.any(U <= P.u_lo) or np.any(U >= P.u_hi):
            return np.inf
        X = simulate_plate(ops, x0, U)
        c = 0.0
        for i in range(P.N):
            c += P.h * (0.5 * P.q * np.sum((X[i] - xr) ** 2) + 0.5 * P.r * np.sum((U[i] - ur) ** 2)
                        - P.tau * np.sum(np.log(U[i] - P.u_lo) + np.log(P.u_hi - U[i])))
        return c
    v0 = np.full(P.N * ops.m, P.u_cold)
    res = scipy.optimize.minimize(cost, v0, method="Powell",
                                  options={"xtol": 1e-10, "ftol": 1e-14, "maxfev": 200000})
    res = scipy.optimize.minimize(cost, res.x, method="BFGS", options={"gtol": 1e-9})
    Uopt = res.x.reshape(P.N, ops.m)
    assert np.abs(Uopt - o["U"]).max() <= 1e-4 * np.abs(o["U"]).max()
    assert cost(o["U"].ravel()) <= res.fun + 1e-9 * abs(res.fun)


def test_alpha_max_is_the_largest_step_keeping_the_fraction_of_the_boundary():
    P = tiny_plate(tau=1.0)
    rng = np.random.default_rng(0)
    U = rng.uniform(P.u_lo + 10, P.u_hi - 10, (3, 4))
    D = rng.normal(size=(3, 4)) * 300

    def ok(a):
        Un = U - a * D
        return np.all(Un - P.u_lo >= 0.005 * (U - P.u_lo) - 1e-12) and \
            np.all(P.u_hi - Un >= 0.005 * (P.u_hi - U) - 1e-12)
    a = om.alpha_max(P, U, D)
    lo, hi = 0.0, 1.0
    if ok(1.0):
        assert a == 1.0
    else:
        for _ in range(80):
            mid = 0.5 * (lo + hi)
            lo, hi = (mid, hi) if ok(mid) else (lo, mid)
        assert abs(a - lo) <= 1e-12
    assert om.alpha_max(P.with_(tau=0.0), U, D) == 1.0


def test_gauss_seidel_sweeps_are_the_block_splittings():
    """Linear plate (no radiation, no box): with an exact lower layer a forward
    sweep is S - (D + L)^{-1} K, a backward one S - (D + U)^{-1} K, and SGS
    (backward then forward, u~ = u^k in both) equals their composition."""
    P, ops, x0, xref = setup("plate", tau=0.0, gamma=0.05, rad=0.0)
    X, U, L = random_traj(ops, x0)
    nx, m = ops.nx, ops.m
    w = 2 * nx + m

    def pack(S):
        return np.concatenate([np.concatenate([S[0][i], S[1][i], S[2][i]]) for i in range(P.N)])

    S = (X, U, L)
    KX, KU, KL = om.kkt(ops, x0, xref, X, U, L)
    K = np.concatenate([np.concatenate([KX[i], KU[i], KL[i]]) for i in range(P.N)])
    D = np.zeros((P.N * w, P.N * w)); Lo = np.zeros_like(D); Up = np.zeros_like(D)
    for i in range(P.N):
        D[i * w:(i + 1) * w, i * w:(i + 1) * w] = stage_block(ops, X[i], U[i], L[i])
        if i > 0:
            Lo[i * w:i * w + nx, (i - 1) * w:(i - 1) * w + nx] = np.eye(nx)
        if i + 1 < P.N:
            Up[i * w + nx + m:(i + 1) * w, (i + 1) * w + nx + m:(i + 2) * w] = np.eye(nx)
    big = dict(n_sw=400, n_schur=300)
    f = om.sweep(ops, x0, xref, S, U, 1, **big)
    np.testing.assert_allclose(pack(f), pack(S) - np.linalg.solve(D + Lo, K), atol=1e-8)
    b = om.sweep(ops, x0, xref, S, U, -1, **big)
    np.testing.assert_allclose(pack(b), pack(S) - np.linalg.solve(D + Up, K), atol=1e-8)
    sgs = om.iterate(ops, x0, xref, S, "sgs", **big)
    np.testing.assert_allclose(pack(sgs), pack(om.sweep(ops, x0, xref, b, U, 1, **big)), atol=1e-12)


def test_paper_plate_configuration_converges_inside_the_box():
    """The paper's setting (13 x 13, N = 20, tau = 100, gamma = 0.5, SGS, two
    Jacobi sweeps and two Schur steps, stop at |K|_inf < 1) converges from the
    ambient start with every input inside [T_a, T_a + 400]."""
    from nmpc_inputs import make_plate_instance
    P = make_plate_problem()
    ops = om.Ops(P)
    x0g, xref = make_plate_instance(P, 0, "slope")
    o = om.solve(ops, om.state_x0(ops, x0g), xref, upper="sgs", tol=1.0, residual_kind="paper",
                 max_iter=200)
    assert o["status"] == "converged" and o["r_paper"] < 1.0
    assert np.all(o["U"] > P.u_lo) and np.all(o["U"] < P.u_hi)
    assert o["iters"] <= 60
