"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test ties the oracle to something other than itself: closed-form
eigenpairs, finite differences of the Lagrangian, Newton's method with dense
LU, the exact optimum of the NLP (direct minimization, or the condensed QP in
the linear case), the nilpotency of Lemma lemma_rho0, and dense solves of the
stage blocks.
"""
import numpy as np
import pytest

from nmpc_inputs import gaussian_factors, make_instance, make_problem

import oracle
from oracle import dense


def tiny2d(nsx=4, nsy=3, N=3, gamma_rel=1.0, k1=0.5, lattice=2, sigma=0.25):
    P = make_problem("grid", ns=nsx, N=N, gamma_rel=gamma_rel, lattice=lattice)
    P = P.with_(nsy=nsy, gx=gaussian_factors(nsx, lattice, sigma),
                gy=gaussian_factors(nsy, lattice, sigma), k1=k1)
    P.gamma = gamma_rel * P.h * P.r
    return P


def tiny_data(P, seed=0, scale_lam=0.01):
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(0.0, 0.2, P.n)
    xref = rng.uniform(-0.3, 0.3, P.n)
    X = rng.normal(size=(P.N, P.n)) * 0.1
    U = rng.normal(size=(P.N, P.m))
    LAM = rng.normal(size=(P.N, P.n)) * scale_lam
    UT = rng.normal(size=(P.N, P.m))
    return x0, xref, X, U, LAM, UT


def fd_grad(fun, S, eps=1e-6):
    g = np.zeros_like(S)
    for t in range(S.size):
        Sp = S.copy(); Sp[t] += eps
        Sm = S.copy(); Sm[t] -= eps
        g[t] = (fun(Sp) - fun(Sm)) / (2 * eps)
    return g


# ---------------------------------------------------------------- P7: stencil

@pytest.mark.parametrize("a,b", [(1, 1), (2, 3), (4, 1)])
def test_stencil_eigenpairs(a, b):
    """L sin(pi a x) sin(pi b y) = mu (same), mu = -(4/dx^2) sin^2(pi a dx/2) - (4/dy^2) sin^2(pi b dy/2)."""
    P = tiny2d(nsx=6, nsy=5, N=1, k1=0.0).with_(k0=1.0)
    xs = (np.arange(P.nsx) + 1) * P.dx
    ys = (np.arange(P.nsy) + 1) * P.dy
    v = (np.sin(np.pi * b * ys)[:, None] * np.sin(np.pi * a * xs)[None, :]).reshape(-1)
    mu = -(4 / P.dx ** 2) * np.sin(np.pi * a * P.dx / 2) ** 2 - (4 / P.dy ** 2) * np.sin(np.pi * b * P.dy / 2) ** 2
    # state row with x0 = 0, u = 0, k = 1: KX_1 = -x_1 + h L x_1
    KX, _, _ = oracle.kkt(P, np.zeros(P.n), np.zeros(P.n), v[None, :], np.zeros((1, P.m)),
                          np.zeros((1, P.n)))
    Lv = (KX[0] + v) / P.h
    np.testing.assert_allclose(Lv, mu * v, atol=1e-9 * abs(mu))
    np.testing.assert_allclose(dense.lap_matrix(P) @ v, mu * v, atol=1e-9 * abs(mu))


def test_stencil_eigenpairs_1d():
    P = make_problem("c0").with_(N=1, k1=0.0, k0=1.0)
    j = np.arange(1, P.nsx + 1)
    for a in (1, 5, 16):
        v = np.sin(np.pi * a * j * P.dx)
        mu = -(4 / P.dx ** 2) * np.sin(np.pi * a * P.dx / 2) ** 2
        KX, _, _ = oracle.kkt(P, np.zeros(P.n), np.zeros(P.n), v[None], np.zeros((1, P.m)),
                              np.zeros((1, P.n)))
        np.testing.assert_allclose((KX[0] + v) / P.h, mu * v, atol=1e-9 * abs(mu))


# ------------------------------------------------- P3: K = grad of Lagrangian

@pytest.mark.parametrize("which", ["2d", "1d"])
def test_kkt_is_lagrangian_gradient(which):
    """K_i = (d/dlam_i, d/du_i, d/dx_i) of the Lagrangian of the relaxed problem."""
    if which == "2d":
        P = tiny2d()
    else:
        P = make_problem("c0", N=3)
    x0, xref, X, U, LAM, UT = tiny_data(P)
    KX, KU, KL = oracle.kkt(P, x0, xref, X, U, LAM, UT)
    S = dense.pack(X, U, LAM)
    g = fd_grad(lambda s: dense.lagrangian(P, x0, xref, *dense.unpack(P, s), UT), S)
    gX, gU, gL = dense.unpack(P, g)
    scale = max(np.abs(KX).max(), np.abs(KU).max(), np.abs(KL).max())
    assert np.abs(gL - KX).max() <= 1e-8 * scale
    assert np.abs(gU - KU).max() <= 1e-8 * scale
    assert np.abs(gX - KL).max() <= 1e-8 * scale


def test_time_varying_reference():
    """A per-stage reference enters stage i's costate row only."""
    P = tiny2d()
    x0, xref, X, U, LAM, _ = tiny_data(P)
    xr2 = np.stack([xref * (1 + 0.1 * i) for i in range(P.N)])
    a = oracle.kkt(P, x0, xr2, X, U, LAM)
    b = dense.kkt(P, x0, xr2, X, U, LAM)
    for p, q in zip(a, b):
        np.testing.assert_allclose(p, q, rtol=0, atol=1e-15)
    c = oracle.kkt(P, x0, xref, X, U, LAM)
    np.testing.assert_allclose(a[2][0], c[2][0], atol=1e-15)
    assert np.abs(a[2][1] - c[2][1]).max() > 1e-6


# ------------------------------------------- Newton matrix = Jacobian of K

def test_newton_matrix_is_kkt_jacobian():
    """eq. KKT_sys: diagonal blocks D_i = grad_{s_i} K_i, couplings M_L, M_U."""
    P = tiny2d()
    x0, xref, X, U, LAM, _ = tiny_data(P)
    J = dense.jacobian(P, X, U, LAM)
    S = dense.pack(X, U, LAM)
    UT = U.copy()  # regularization reference frozen at the linearization point

    def Kvec(s):
        return dense.pack(*oracle.kkt(P, x0, xref, *dense.unpack(P, s), UT))

    Jfd = np.zeros_like(J)
    eps = 1e-6
    for t in range(S.size):
        Sp = S.copy(); Sp[t] += eps
        Sm = S.copy(); Sm[t] -= eps
        Jfd[:, t] = (Kvec(Sp) - Kvec(Sm)) / (2 * eps)
    assert np.abs(Jfd - J).max() <= 1e-7 * np.abs(J).max()


# -------------------------------------------------------- P1: Newton + LU

@pytest.mark.parametrize("which", ["2d", "c0"])
def test_newton_quadratic_and_jacobi_fixed_point(which):
    P = tiny2d(N=4) if which == "2d" else make_problem("c0")
    if which == "2d":
        x0, xref = tiny_data(P)[:2]
    else:
        x0, xref = make_instance(P, 3)
    (Xn, Un, Ln), hist = dense.newton(P, x0, xref, *oracle.cold_start(P, x0))
    assert hist[-1] <= 1e-13
    # quadratic convergence: e_{k+1} <= C e_k^2 once in the basin
    ratios = [hist[k + 1] / hist[k] ** 2 for k in range(1, len(hist) - 1) if hist[k] > 1e-12]
    assert len(hist) <= 8 and max(ratios) < 1e4
    o = oracle.solve(P, x0, xref, tol=1e-13, max_iter=20000)
    assert o["status"] == "converged"
    np.testing.assert_allclose(o["U"], Un, atol=1e-9 * np.abs(Un).max())
    np.testing.assert_allclose(o["X"], Xn, atol=1e-11)
    np.testing.assert_allclose(o["LAM"], Ln, atol=1e-9 * np.abs(Ln).max())


# --------------------------------------------------- NLP optimum (eq. nlp)

def test_fixed_point_is_nlp_optimum():
    """The KKT point equals the minimizer of the cost over u, states simulated
    by backward Euler (no optimality formula involved)."""
    P = tiny2d(N=3)
    P.h = 0.02
    P.gamma = P.h * P.r
    x0, xref = tiny_data(P, seed=4)[:2]
    o = oracle.solve(P, x0, xref, tol=1e-13, max_iter=20000)
    assert o["status"] == "converged"
    Xm, Um, res = dense.nlp_reduced(P, x0, xref)
    assert np.abs(o["U"] - Um).max() <= 2e-5 * np.abs(Um).max()
    assert np.abs(o["X"] - Xm).max() <= 1e-7


# ----------------------------------------------- P2: linear-quadratic case

@pytest.mark.parametrize("which", ["2d", "c0"])
def test_lq_case_matches_condensed_qp(which):
    P = (tiny2d(N=5) if which == "2d" else make_problem("c0", N=6)).with_(k1=0.0)
    x0, xref = tiny_data(P, seed=2)[:2]
    Xq, Uq = dense.lq_condensed(P, x0, xref)
    o = oracle.solve(P, x0, xref, tol=1e-13, max_iter=20000)
    assert o["status"] == "converged"
    np.testing.assert_allclose(o["U"], Uq, atol=1e-9 * np.abs(Uq).max())
    np.testing.assert_allclose(o["X"], Xq, atol=1e-12)
    # KKT is affine: one Newton step from any start is exact
    (_, Un, _), hist = dense.newton(P, x0, xref, *oracle.cold_start(P, x0), max_it=2)
    assert hist[1] <= 1e-12 * max(hist[0], 1.0)


# ------------------------------------------------------- P4: nilpotency

@pytest.mark.parametrize("N", [2, 3, 5])
def test_dbar_coupling_is_nilpotent(N):
    """Lemma lemma_rho0: rho(Dbar^{-1}(L+U)) = 0. Exact form: the
    (2N-1)-th power vanishes (x errors move forward, lambda errors backward
    one stage per iteration, and the only x->lambda turn is inside a stage)."""
    P = tiny2d(N=N)
    x0, xref, X, U, LAM, _ = tiny_data(P, seed=5)
    _, LU, Dbar = dense.split_DLU(P, X, U, LAM)
    G = np.linalg.solve(Dbar, LU)
    nG = np.linalg.norm(G, 2)
    Gk = np.linalg.matrix_power(G, 2 * N - 1)
    assert np.linalg.norm(Gk, 2) <= 1e-10 * nG ** (2 * N - 1)
    Gk1 = np.linalg.matrix_power(G, 2 * N - 2)
    assert np.linalg.norm(Gk1, 2) > 1e-6 * nG ** (2 * N - 2)
    assert np.max(np.abs(np.linalg.eigvals(G))) < 1e-3


# ----------------------------------------------- P5: lower layer exactness

@pytest.mark.parametrize("which", ["2d", "c0"])
def test_lower_layer_many_sweeps_is_dense_block_solve(which):
    """Schur elimination + point Jacobi (eq. step12, coff) reproduce D_i^{-1} K_i
    when the sweep counts grow; D_i is taken by finite differences of K_i."""
    P = tiny2d() if which == "2d" else make_problem("c0", N=2)
    x0, xref, X, U, LAM, _ = tiny_data(P, seed=6)
    KX, KU, KL = oracle.kkt(P, x0, xref, X, U, LAM)
    i = 1
    dx, du, dl = oracle.stage_solve(P, X[i], LAM[i], KX[i], KL[i], KU[i], n_sw=400, n_schur=60)
    UT = U.copy()

    def Ki(si):
        X2, U2, L2 = X.copy(), U.copy(), LAM.copy()
        X2[i], U2[i], L2[i] = si[:P.n], si[P.n:P.n + P.m], si[P.n + P.m:]
        a, b, c = oracle.kkt(P, x0, xref, X2, U2, L2, UT)
        return np.concatenate([a[i], b[i], c[i]])

    s = np.concatenate([X[i], U[i], LAM[i]])
    D = np.zeros((s.size, s.size))
    for t in range(s.size):
        sp = s.copy(); sp[t] += 1e-6
        sm = s.copy(); sm[t] -= 1e-6
        D[:, t] = (Ki(sp) - Ki(sm)) / 2e-6
    ref = np.linalg.solve(D, np.concatenate([KX[i], KU[i], KL[i]]))
    got = np.concatenate([dx, du, dl])
    assert np.abs(got - ref).max() <= 1e-7 * np.abs(ref).max()
    # and the analytic block agrees with the finite-difference one
    Dan = dense.stage_block(P, dense.lap_matrix(P), P.dense_B(), X[i], LAM[i], P.gamma)
    assert np.abs(Dan - D).max() <= 1e-7 * np.abs(D).max()


def test_two_sweeps_are_the_stated_schedule():
    """With n_sw = 1 the F_x solve is y = c / diag(F_x); with zero Schur passes v3 = 0."""
    P = tiny2d()
    x0, xref, X, U, LAM, _ = tiny_data(P, seed=7)
    KX, KU, KL = oracle.kkt(P, x0, xref, X, U, LAM)
    i = 0
    dx, du, dl = oracle.stage_solve(P, X[i], LAM[i], KX[i], KL[i], KU[i], n_sw=1, n_schur=0)
    assert np.all(du == 0)
    Fx = P.h * dense.fx_mat(P, dense.lap_matrix(P), X[i]) - np.eye(P.n)
    np.testing.assert_allclose(dx, KX[i] / np.diag(Fx), rtol=1e-13)
    Axx = P.h * dense.hxx_mat(P, dense.lap_matrix(P), LAM[i])
    np.testing.assert_allclose(dl, (KL[i] - Axx @ dx) / np.diag(Fx), rtol=1e-12, atol=1e-18)


# ---------------------------------------- upper layer = block Jacobi (eq. 1st_jacobi)

def test_upper_iteration_is_block_jacobi_step():
    P = tiny2d(N=4)
    x0, xref, X, U, LAM, _ = tiny_data(P, seed=8)
    Xn, Un, Ln, rs, rp = oracle.iterate(P, x0, xref, X, U, LAM, n_sw=400, n_schur=60)
    D, LU, _ = dense.split_DLU(P, X, U, LAM)
    K = dense.pack(*dense.kkt(P, x0, xref, X, U, LAM))
    Sn = dense.pack(X, U, LAM) - np.linalg.solve(D, K)
    got = dense.pack(Xn, Un, Ln)
    assert np.abs(got - Sn).max() <= 1e-9 * np.abs(Sn).max()
    rs2, rp2 = dense.norms(P, *dense.kkt(P, x0, xref, X, U, LAM))
    assert abs(rs - rs2) <= 1e-12 * rs2 and abs(rp - rp2) <= 1e-12 * rp2


def test_single_stage_is_newton_step():
    """P10: N = 1 has L = U = 0, so one iteration with an exact lower layer and
    gamma = 0 is one Newton step."""
    P = tiny2d(N=1, gamma_rel=0.0)
    x0, xref, X, U, LAM, _ = tiny_data(P, seed=9)
    Xn, Un, Ln, _, _ = oracle.iterate(P, x0, xref, X, U, LAM, n_sw=400, n_schur=60)
    J = dense.jacobian(P, X, U, LAM, gamma=0.0)
    K = dense.pack(*dense.kkt(P, x0, xref, X, U, LAM))
    Sn = dense.pack(X, U, LAM) - np.linalg.solve(J, K)
    assert np.abs(dense.pack(Xn, Un, Ln) - Sn).max() <= 1e-9 * np.abs(Sn).max()


def test_fixed_point_independent_of_schedule():
    """gamma (with ut = u^k), n_sw and n_schur change the rate, not the solution."""
    P0 = make_problem("c0")
    x0, xref = make_instance(P0, 1)
    sols = []
    for g, nsw, nsc in [(1.0, 2, 2), (0.1, 1, 1), (0.0, 4, 3), (3.0, 2, 1)]:
        P = make_problem("c0", gamma_rel=g)
        o = oracle.solve(P, x0, xref, tol=1e-12, max_iter=20000, n_sw=nsw, n_schur=nsc)
        assert o["status"] == "converged"
        sols.append(o["U"])
    for s in sols[1:]:
        np.testing.assert_allclose(s, sols[0], atol=1e-9 * np.abs(sols[0]).max())


# ---------------------------------------------- P6: diagonal dominance

@pytest.mark.parametrize("name", ["c0", "g16"])
def test_point_jacobi_contracts(name):
    """Lemma lemma_jaco (element-wise): F_x is strictly diagonally dominant at
    the step sizes used, with the contraction bound 2d h k/dx^2 / (1 + 2d h k/dx^2)."""
    P = make_problem("c0") if name == "c0" else make_problem("grid", ns=16, N=4)
    x0, xref = make_instance(P, 0)
    o = oracle.solve(P, x0, xref, tol=1e-8, max_iter=20000)
    L = dense.lap_matrix(P)
    worst = 0.0
    for i in range(P.N):
        F = P.h * dense.fx_mat(P, L, o["X"][i]) - np.eye(P.n)
        d = np.abs(np.diag(F))
        off = np.abs(F).sum(1) - d
        offT = np.abs(F).sum(0) - d
        worst = max(worst, (off / d).max(), (offT / d).max())
    kmax = P.k0 * (1 + P.k1 * np.abs(o["X"]).max())
    c = (2 * P.dim) * P.h * kmax / P.dx ** 2
    assert worst < 1.0
    assert worst <= c / (1 + c) * 1.05


# ---------------------------------------------------------- P8: rho < 1

def test_rho_below_one_and_observed_rate():
    """Theorem theorem_cvg: rho(D*^{-1}(L+U)) < 1 for gamma > 0 and short T.

    With the regularization reference updated every iteration (ut = u^k, as in
    the paper's experiment) the gamma term of K vanishes identically, so the
    derivative of the iteration map at S* is D*^{-1}(gamma E_u - (L+U)), E_u
    the projector on the input rows; the residual of the exact-lower-layer
    iteration decays at that matrix's spectral radius (Lemma lemma_rate)."""
    P = tiny2d(nsx=5, nsy=5, N=4, lattice=2, sigma=0.2)
    x0, xref = tiny_data(P, seed=11)[:2]
    o = oracle.solve(P, x0, xref, tol=1e-14, max_iter=20000)
    D, LU, _ = dense.split_DLU(P, o["X"], o["U"], o["LAM"])
    rho = np.max(np.abs(np.linalg.eigvals(np.linalg.solve(D, LU))))
    assert 0.0 < rho < 1.0
    w = 2 * P.n + P.m
    E = np.zeros_like(D)
    for i in range(P.N):
        for j in range(P.m):
            E[i * w + P.n + j, i * w + P.n + j] = 1.0
    rho_k = np.max(np.abs(np.linalg.eigvals(np.linalg.solve(D, P.gamma * E - LU))))
    assert 0.0 < rho_k < 1.0
    t = oracle.solve(P, x0, xref, tol=1e-300, max_iter=200, n_sw=300, n_schur=40, trace=True)
    r = t["rhist"]
    k0 = int(np.argmax(r < 1e-3 * r[0]))
    span = 20
    assert k0 > 0 and r[k0 + span] > 1e-12 * r[0]
    rate = (r[k0 + span] / r[k0]) ** (1.0 / span)
    assert abs(rate - rho_k) <= 0.05 * rho_k


# ------------------------------------------------------ status handling

def test_nonfinite_and_noconv_status():
    P = make_problem("c0")
    x0, xref = make_instance(P, 0)
    X, U, L = oracle.cold_start(P, x0)
    U[3, 1] = np.nan
    o = oracle.solve(P, x0, xref, start=(X, U, L), tol=1e-6, max_iter=50)
    assert o["status"] == "nonfinite"
    o = oracle.solve(P, x0, xref, tol=1e-6, max_iter=3)
    assert o["status"] == "max_iter" and o["iters"] == 3


def test_c0_solution_satisfies_kkt():
    """P9: the returned iterate satisfies the KKT conditions to the tolerance,
    re-checked with the dense evaluation."""
    P = make_problem("c0")
    x0, xref = make_instance(P, 0)
    o = oracle.solve(P, x0, xref, tol=1e-6)
    assert o["status"] == "converged"
    rs, rp = dense.norms(P, *dense.kkt(P, x0, xref, o["X"], o["U"], o["LAM"]))
    assert rs <= 1e-6 and abs(rs - o["r_scaled"]) <= 1e-12


# ------------------------- Gauss-Seidel upper layers (Sec. 4.4, eq. fgs, eq. sgs)

def _tri_parts(J, P):
    """Block-diagonal D, strictly lower L and strictly upper U block parts of
    the stage-block-tridiagonal matrix J (J = D + L + U)."""
    w = 2 * P.n + P.m
    D = np.zeros_like(J); L = np.zeros_like(J); Up = np.zeros_like(J)
    for i in range(P.N):
        for k in range(P.N):
            blk = J[i * w:(i + 1) * w, k * w:(k + 1) * w]
            tgt = D if i == k else (L if k < i else Up)
            tgt[i * w:(i + 1) * w, k * w:(k + 1) * w] = blk
    return D, L, Up


@pytest.mark.parametrize("direction", [1, -1])
def test_gs_sweep_is_the_papers_fgs_bgs_step(direction):
    """A forward sweep equals S - (D^k + L)^{-1} K^k (eq. fgs), a backward one
    S - (D^k + U)^{-1} K^k, on a nonlinear instance: K_i is affine in x_{i-1}
    and lambda_{i+1} with identity coefficients and D_i depends on s_i only, so
    the sequential sweep and the block-triangular solve agree exactly."""
    P = tiny2d(N=4)
    x0, xref, X, U, LAM, _ = tiny_data(P, seed=21)
    Xn, Un, Ln = oracle.gs_sweep(P, x0, xref, X, U, LAM, direction, n_sw=400, n_schur=60)
    J = dense.jacobian(P, X, U, LAM)
    D, L, Up = _tri_parts(J, P)
    K = dense.pack(*dense.kkt(P, x0, xref, X, U, LAM))
    Sn = dense.pack(X, U, LAM) - np.linalg.solve(D + (L if direction > 0 else Up), K)
    got = dense.pack(Xn, Un, Ln)
    assert np.abs(got - Sn).max() <= 1e-9 * np.abs(Sn).max()
    # and it differs from the Jacobi step (the coupling is really used)
    Sj = dense.pack(X, U, LAM) - np.linalg.solve(D, K)
    assert np.abs(got - Sj).max() > 1e-6 * np.abs(Sn).max()


def test_sgs_iteration_is_eq_sgs_in_the_linear_case():
    """With k1 = 0 the blocks do not depend on S, and one SGS iteration (a
    backward sweep, then a forward sweep) equals eq. sgs:
    S - (D + L)^{-1} (K - U (D + U)^{-1} K)."""
    P = tiny2d(N=4, k1=0.0)
    x0, xref, X, U, LAM, _ = tiny_data(P, seed=22)
    o = oracle.solve(P, x0, xref, start=(X, U, LAM), tol=0.0, max_iter=1, n_sw=400,
                     n_schur=60, upper="sgs")
    J = dense.jacobian(P, X, U, LAM)
    D, L, Up = _tri_parts(J, P)
    K = dense.pack(*dense.kkt(P, x0, xref, X, U, LAM))
    Sn = dense.pack(X, U, LAM) - np.linalg.solve(D + L, K - Up @ np.linalg.solve(D + Up, K))
    got = dense.pack(o["X"], o["U"], o["LAM"])
    assert np.abs(got - Sn).max() <= 1e-9 * np.abs(Sn).max()


def test_fgs_rate_is_the_square_of_jacobis():
    """Theorem cor_cvg: the KKT matrix is block tridiagonal, hence consistently
    ordered, so rho((D + L)^{-1} U) = rho(D^{-1}(L + U))^2. Checked on the
    iteration matrices at the solution, and on the oracle's observed residual
    decay (linear case, gamma = 0, exact lower layer, where the FGS map is
    exactly affine)."""
    P = tiny2d(nsx=5, nsy=4, N=5, lattice=2, sigma=0.2, k1=0.0, gamma_rel=0.0)
    x0, xref = tiny_data(P, seed=23)[:2]
    o = oracle.solve(P, x0, xref, tol=1e-13, max_iter=20000)
    J = dense.jacobian(P, o["X"], o["U"], o["LAM"])
    D, L, Up = _tri_parts(J, P)
    rj = np.max(np.abs(np.linalg.eigvals(np.linalg.solve(D, L + Up))))
    rf = np.max(np.abs(np.linalg.eigvals(np.linalg.solve(D + L, Up))))
    rb = np.max(np.abs(np.linalg.eigvals(np.linalg.solve(D + Up, L))))
    assert 0.0 < rj < 1.0
    assert abs(rf - rj ** 2) <= 1e-8 and abs(rb - rj ** 2) <= 1e-8
    # the oracle's sweep map has exactly that iteration matrix: its columns by
    # differences (the map is affine here)
    X, U, LAM = o["X"], o["U"], o["LAM"]
    S0 = dense.pack(X, U, LAM)
    base = dense.pack(*oracle.gs_sweep(P, x0, xref, X, U, LAM, 1, n_sw=400, n_schur=60))
    G = np.zeros((S0.size, S0.size))
    for j in range(S0.size):
        e = np.zeros(S0.size); e[j] = 1e-3
        Xe, Ue, Le = dense.unpack(P, S0 + e)
        G[:, j] = (dense.pack(*oracle.gs_sweep(P, x0, xref, Xe, Ue, Le, 1, n_sw=400,
                                               n_schur=60)) - base) / 1e-3
    np.testing.assert_allclose(G, -np.linalg.solve(D + L, Up), atol=1e-8)
    # observed residual decay over many iterations (the dominant eigenvalues
    # are a complex pair, so single-step ratios oscillate)
    t = oracle.solve(P, x0, xref, tol=1e-300, max_iter=80, n_sw=300, n_schur=40, trace=True,
                     upper="fgs")
    r = t["rhist"]
    k0 = int(np.argmax(r < 1e-2 * r[0]))
    k1 = int(np.nonzero(r > 1e-11 * r[0])[0].max())
    assert k1 - k0 >= 15
    rate = (r[k1] / r[k0]) ** (1.0 / (k1 - k0))
    assert abs(rate - rj ** 2) <= 0.1 * rj ** 2


@pytest.mark.parametrize("upper", ["fgs", "bgs", "sgs"])
def test_gauss_seidel_fixed_point_is_jacobis(upper):
    """Same KKT point as the Jacobi upper layer (the splitting changes only the
    rate), in fewer iterations on the nonlinear 1D configuration."""
    P = make_problem("c0")
    x0, xref = make_instance(P, 3)
    oj = oracle.solve(P, x0, xref, tol=1e-12, max_iter=20000)
    og = oracle.solve(P, x0, xref, tol=1e-12, max_iter=20000, upper=upper)
    assert oj["status"] == og["status"] == "converged"
    np.testing.assert_allclose(og["U"], oj["U"], atol=1e-9 * np.abs(oj["U"]).max())
    assert og["iters"] < oj["iters"]


# ----------------------------------------- cold start: every stage the same

@pytest.mark.parametrize("which", ["tiny", "c1"])
def test_cold_start_rows_equal_at_every_stage(which):
    """The cold start (x_i = x0, u_i = 0, lambda_i = 0) with one reference for
    all stages has the same KKT rows at every stage: K^x_i = -h f(x0, 0) (the
    backward-Euler step from x_{i-1} = x0 at every stage, the initial state
    included), K^u_i = 0, and the costate row reduces to the stage-cost
    gradient (no costate terms). So one stage's residual is the whole start's,
    which the library's fallback check relies on. Checked against the dense
    reference's rows; a per-stage reference breaks the equality."""
    if which == "tiny":
        P = tiny2d(N=5)
        x0, xref, *_ = tiny_data(P, seed=3)
    else:
        P = make_problem("c1").with_(N=6)
        x0, xref = make_instance(P, 11)
    X, U, LAM = oracle.cold_start(P, x0)
    KX, KU, KL = oracle.kkt(P, x0, xref, X, U, LAM)
    dX, dU, dL = dense.kkt(P, x0, xref, X, U, LAM)
    np.testing.assert_allclose(KX, dX, rtol=0, atol=1e-13 * max(1.0, np.abs(dX).max()))
    np.testing.assert_allclose(KL, dL, rtol=0, atol=1e-13 * max(1.0, np.abs(dL).max()))
    assert np.abs(KU).max() == 0.0
    for i in range(1, P.N):
        np.testing.assert_array_equal(KX[i], KX[0])
        np.testing.assert_array_equal(KL[i], KL[0])
    assert np.abs(KX[0]).max() > 0 and np.abs(KL[0]).max() > 0
    rs_all, rp_all = oracle.norms(P, KX, KU, KL)
    rs_0, rp_0 = oracle.norms(P, KX[:1].repeat(P.N, 0), KU, KL[:1].repeat(P.N, 0))
    assert rs_all == rs_0 and rp_all == rp_0
    xr2 = np.stack([np.asarray(xref) * (1 + 0.1 * i) for i in range(P.N)])
    _, _, KL2 = oracle.kkt(P, x0, xr2, X, U, LAM)
    assert np.abs(KL2[1] - KL2[0]).max() > 0


# -------------------------------------------- SOR: over-relaxed sweeps (Sec. 4.4)

@pytest.mark.parametrize("direction", [1, -1])
@pytest.mark.parametrize("omega", [0.7, 1.3])
def test_sor_sweep_is_the_papers_relaxed_step(direction, omega):
    """A forward sweep with over-relaxation omega equals
    S - omega (D^k + omega L)^{-1} K^k (the paper's SOR step with alpha = 1),
    a backward one S - omega (D^k + omega U)^{-1} K^k, on a nonlinear instance
    (same reason as the plain sweep: K_i is affine in the neighbour stages with
    the coupling blocks as coefficients, D_i depends on s_i only)."""
    P = tiny2d(N=4)
    x0, xref, X, U, LAM, _ = tiny_data(P, seed=22)
    Xn, Un, Ln = oracle.gs_sweep(P, x0, xref, X, U, LAM, direction, n_sw=400, n_schur=60,
                                 omega=omega)
    J = dense.jacobian(P, X, U, LAM)
    D, L, Up = _tri_parts(J, P)
    K = dense.pack(*dense.kkt(P, x0, xref, X, U, LAM))
    C = L if direction > 0 else Up
    Sn = dense.pack(X, U, LAM) - omega * np.linalg.solve(D + omega * C, K)
    got = dense.pack(Xn, Un, Ln)
    assert np.abs(got - Sn).max() <= 1e-9 * np.abs(Sn).max()
    # omega = 1 is the plain sweep, bit for bit
    a = oracle.gs_sweep(P, x0, xref, X, U, LAM, direction, omega=1.0)
    b = oracle.gs_sweep(P, x0, xref, X, U, LAM, direction)
    for p, q in zip(a, b):
        np.testing.assert_array_equal(p, q)


@pytest.mark.parametrize("upper", ["fgs", "sgs"])
def test_sor_fixed_point_is_jacobis(upper):
    """Over-relaxation changes the rate, not the KKT point."""
    P = make_problem("c0")
    x0, xref = make_instance(P, 3)
    oj = oracle.solve(P, x0, xref, tol=1e-12, max_iter=20000)
    og = oracle.solve(P, x0, xref, tol=1e-12, max_iter=20000, upper=upper, omega=1.2)
    assert oj["status"] == og["status"] == "converged"
    np.testing.assert_allclose(og["U"], oj["U"], atol=1e-9 * np.abs(oj["U"]).max())
    with pytest.raises(ValueError):
        oracle.solve(P, x0, xref, omega=1.2)


# ----------------------------- input box: log barrier and the step rule (NEXT-2)

def boxed(P, tau=0.02, lo=-2.0, hi=3.0):
    return P.with_(tau=tau, u_lo=lo, u_hi=hi)


def box_data(P, seed=0):
    x0, xref, X, U, LAM, UT = tiny_data(P, seed)
    rng = np.random.default_rng(seed + 100)
    U = rng.uniform(P.u_lo + 0.1, P.u_hi - 0.1, U.shape)     # strictly inside the box
    UT = rng.uniform(P.u_lo + 0.1, P.u_hi - 0.1, U.shape)
    return x0, xref, X, U, LAM, UT


@pytest.mark.parametrize("which", ["2d", "1d"])
def test_box_kkt_is_lagrangian_gradient(which):
    """With the input box the KKT rows are still the gradient of the Lagrangian
    of the relaxed problem (eq. nlp_relaxed: stage cost h (l + Phi), Phi the
    log barrier of G = (u - u_lo, u_hi - u)); checked by central differences,
    and the C rows against the dense ones."""
    P = boxed(tiny2d() if which == "2d" else make_problem("c0", N=3))
    x0, xref, X, U, LAM, UT = box_data(P)
    KX, KU, KL = oracle.kkt(P, x0, xref, X, U, LAM, UT)
    dX, dU, dL = dense.kkt(P, x0, xref, X, U, LAM, UT)
    for a, b in ((KX, dX), (KU, dU), (KL, dL)):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * max(1.0, np.abs(b).max()))
    S = dense.pack(X, U, LAM)
    g = fd_grad(lambda s: dense.lagrangian(P, x0, xref, *dense.unpack(P, s), UT), S)
    gX, gU, gL = dense.unpack(P, g)
    scale = max(np.abs(KX).max(), np.abs(KU).max(), np.abs(KL).max())
    assert np.abs(gU - KU).max() <= 1e-8 * scale
    assert np.abs(gX - KL).max() <= 1e-8 * scale
    assert np.abs(gL - KX).max() <= 1e-8 * scale
    # the barrier really enters: without it the input rows differ
    KU0 = oracle.kkt(P.with_(tau=0.0), x0, xref, X, U, LAM, UT)[1]
    assert np.abs(KU0 - KU).max() > 1e-6 * scale


def test_box_newton_matrix_and_stage_solve():
    """The dense Newton matrix with the barrier's Hessian in A_uu is the
    Jacobian of K (finite differences), and the lower layer with many sweeps
    solves the stage block with that A_uu."""
    P = boxed(tiny2d())
    x0, xref, X, U, LAM, _ = box_data(P, seed=4)
    J = dense.jacobian(P, X, U, LAM)
    S = dense.pack(X, U, LAM)
    UT = U.copy()

    def Kvec(s):
        return dense.pack(*oracle.kkt(P, x0, xref, *dense.unpack(P, s), UT))

    Jfd = np.zeros_like(J)
    for t in range(S.size):
        Sp = S.copy(); Sp[t] += 1e-6
        Sm = S.copy(); Sm[t] -= 1e-6
        Jfd[:, t] = (Kvec(Sp) - Kvec(Sm)) / 2e-6
    assert np.abs(Jfd - J).max() <= 1e-7 * np.abs(J).max()
    KX, KU, KL = oracle.kkt(P, x0, xref, X, U, LAM)
    i = 1
    dx, du, dl = oracle.stage_solve(P, X[i], LAM[i], KX[i], KL[i], KU[i], n_sw=400, n_schur=60,
                                    u=U[i])
    w = 2 * P.n + P.m
    Di = J[i * w:(i + 1) * w, i * w:(i + 1) * w]
    ref = np.linalg.solve(Di, np.concatenate([KX[i], KU[i], KL[i]]))
    got = np.concatenate([dx, du, dl])
    assert np.abs(got - ref).max() <= 1e-7 * np.abs(ref).max()


def test_fraction_to_boundary_rule():
    """eq. eq_alphamax: the C closed form against bisection on the rule itself;
    the binding input lands exactly on G^{k+1} = 0.005 G^k."""
    P = boxed(tiny2d(N=2))
    U = np.array([[0.0, 1.0, 2.9, -1.9], [0.5, 0.5, 0.5, 0.5]])[:, :P.m]
    DU = np.array([[0.1, -3.0, 0.0, 0.0], [0.0, 0.0, 0.0, 0.0]])[:, :P.m]
    a = oracle.alpha_max(P, U, DU)
    assert a == pytest.approx(dense.alpha_max(P, U, DU), rel=1e-12)
    un = U - a * DU
    assert P.u_hi - un[0, 1] == pytest.approx(0.005 * (P.u_hi - U[0, 1]), rel=1e-12)
    assert oracle.alpha_max(P, U, DU * 1e-3) == 1.0
    assert oracle.alpha_max(P.with_(tau=0.0), U, DU) == 1.0


def test_box_solution_is_the_relaxed_optimum():
    """1D heat with a box that binds (the unconstrained inputs leave it): the
    Jacobi iteration with the barrier and the step rule converges, keeps every
    iterate strictly inside the box, and reaches the point where the dense
    Newton iteration with the same rule converges (K = 0 of the relaxed
    problem); the constrained inputs differ from the unconstrained ones."""
    P0 = make_problem("c0")
    x0, xref = make_instance(P0, 3)
    free = oracle.solve(P0, x0, xref, tol=1e-10, max_iter=20000)
    umax = np.abs(free["U"]).max()
    P = P0.with_(tau=1e-3 * P0.r * umax, u_lo=-0.5 * umax, u_hi=0.5 * umax)
    o = oracle.solve(P, x0, xref, tol=1e-9, max_iter=50000, trace=True)
    assert o["status"] == "converged"
    assert np.all(o["U"] > P.u_lo) and np.all(o["U"] < P.u_hi)
    assert np.abs(o["U"] - free["U"]).max() > 0.1 * umax
    # dense Newton with the fraction-to-boundary rule from the cold start
    Xc, Uc, Lc = oracle.cold_start(P, x0)
    S = dense.pack(Xc, Uc, Lc)
    for _ in range(200):
        Xk, Uk, Lk = dense.unpack(P, S)
        K = dense.pack_K(*dense.kkt(P, x0, xref, Xk, Uk, Lk))
        if np.abs(K).max() <= 1e-12:
            break
        d = np.linalg.solve(dense.jacobian(P, Xk, Uk, Lk, gamma=0.0), K)
        _, dU, _ = dense.unpack(P, d)
        S = S - dense.alpha_max(P, Uk, dU) * d
    Xn, Un, Ln = dense.unpack(P, S)
    assert np.abs(dense.pack_K(*dense.kkt(P, x0, xref, Xn, Un, Ln))).max() <= 1e-10
    np.testing.assert_allclose(o["U"], Un, rtol=0, atol=1e-6 * umax)


def _newton_box_point(P, x0, xref):
    """Dense Newton with the fraction-to-the-boundary rule from the cold start:
    the point where K of the relaxed problem vanishes."""
    Xc, Uc, Lc = oracle.cold_start(P, x0)
    S = dense.pack(Xc, Uc, Lc)
    for _ in range(200):
        Xk, Uk, Lk = dense.unpack(P, S)
        K = dense.pack_K(*dense.kkt(P, x0, xref, Xk, Uk, Lk))
        if np.abs(K).max() <= 1e-12:
            break
        d = np.linalg.solve(dense.jacobian(P, Xk, Uk, Lk, gamma=0.0), K)
        _, dU, _ = dense.unpack(P, d)
        S = S - dense.alpha_max(P, Uk, dU) * d
    return dense.unpack(P, S)


@pytest.mark.parametrize("upper", ["fgs", "bgs", "sgs"])
def test_box_gauss_seidel_reaches_the_relaxed_optimum(upper):
    """The Gauss-Seidel layers with the barrier and the step rule cut per
    sweep converge, strictly inside the box, to the dense Newton point of the
    relaxed problem (the same point as the Jacobi layer)."""
    P0 = make_problem("c0")
    x0, xref = make_instance(P0, 3)
    free = oracle.solve(P0, x0, xref, tol=1e-10, max_iter=20000)
    umax = np.abs(free["U"]).max()
    P = P0.with_(tau=1e-3 * P0.r * umax, u_lo=-0.5 * umax, u_hi=0.5 * umax)
    o = oracle.solve(P, x0, xref, tol=1e-9, max_iter=50000, upper=upper)
    assert o["status"] == "converged"
    assert np.all(o["U"] > P.u_lo) and np.all(o["U"] < P.u_hi)
    Xn, Un, Ln = _newton_box_point(P, x0, xref)
    np.testing.assert_allclose(o["U"], Un, rtol=0, atol=1e-6 * umax)


def test_box_sweep_is_cut_by_the_step_rule():
    """From a start next to the box's bounds with a weak barrier one forward
    sweep would leave the box; the iteration takes S + alpha (S_sweep - S)
    with alpha from the rule on the sweep's input step, every input keeping at
    least 0.005 of its distance to the bounds."""
    P0 = make_problem("c0")
    x0, xref = make_instance(P0, 3)
    free = oracle.solve(P0, x0, xref, tol=1e-10, max_iter=20000)
    umax = np.abs(free["U"]).max()
    P = P0.with_(tau=1e-5 * P0.r * umax, u_lo=-0.5 * umax, u_hi=0.5 * umax)
    U0 = np.clip(free["U"], 0.98 * P.u_lo, 0.98 * P.u_hi)
    S = (free["X"].copy(), U0, free["LAM"].copy())
    sw = oracle.gs_sweep(P, x0, xref, *S, +1)
    a = oracle.alpha_max(P, S[1], S[1] - sw[1])
    assert a < 0.5
    o = oracle.solve(P, x0, xref, start=tuple(v.copy() for v in S), tol=0.0, max_iter=1,
                     upper="fgs")
    for got, s0, s1 in zip((o["X"], o["U"], o["LAM"]), S, sw):
        np.testing.assert_allclose(got, s0 + a * (s1 - s0), rtol=1e-13, atol=1e-15)
    g_old = np.minimum(S[1] - P.u_lo, P.u_hi - S[1])
    g_new = np.minimum(o["U"] - P.u_lo, P.u_hi - o["U"])
    assert np.all(g_new >= 0.005 * g_old - 1e-15)
