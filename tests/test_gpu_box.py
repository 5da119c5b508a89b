"""Input box (log barrier of eq. nlp_relaxed, fraction-to-the-boundary step of
eq. eq_alphamax) on the GPU against the FP64 oracle."""
import numpy as np
import pytest

from nmpc_inputs import make_batch, make_instance, make_problem

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2004_02484_amd as m
    return m


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


def boxed_c0(seed=3, tau_rel=1e-3):
    """1D heat with a box at half the unconstrained inputs' range (it binds)."""
    P0 = make_problem("c0")
    x0, xref = make_instance(P0, seed)
    free = oracle.solve(P0, x0, xref, tol=1e-10, max_iter=20000)
    umax = np.abs(free["U"]).max()
    P = P0.with_(tau=tau_rel * P0.r * umax, u_lo=-0.5 * umax, u_hi=0.5 * umax)
    return P, x0, xref, free


def step_alpha(P, x0, xref, X, U, L):
    """alpha of the Jacobi step from (X, U, L) (oracle pieces)."""
    KX, KU, KL = oracle.kkt(P, x0, xref, X, U, L)
    DU = np.stack([oracle.stage_solve(P, X[i], L[i], KX[i], KL[i], KU[i], u=U[i])[1]
                   for i in range(P.N)])
    return oracle.alpha_max(P, U, DU)


def test_box_iterates_match_oracle(nm):
    """From the unconstrained solution clipped into the box (weak barrier) the
    first steps would leave it: the fraction-to-the-boundary rule cuts them
    (alpha < 1), and the GPU iterates follow the oracle's."""
    P, x0, xref, free = boxed_c0(tau_rel=1e-5)
    start = (free["X"].copy(), np.clip(free["U"], 0.98 * P.u_lo, 0.98 * P.u_hi),
             free["LAM"].copy())
    assert step_alpha(P, x0, xref, *start) < 0.1
    for k in (1, 2, 6):
        s = nm.Solver(P, tol=0.0, max_iter=k)
        rc, X, U, L, info = s.solve(x0, xref, warm=start)
        s.close()
        o = oracle.solve(P, x0, xref, start=tuple(a.copy() for a in start), tol=0.0, max_iter=k)
        assert rc == nm.NMPC_E_NOCONV and info["iters"] == k
        assert rel(U, o["U"]) <= 1e-10, (k, rel(U, o["U"]))
        assert rel(X, o["X"]) <= 1e-10 and rel(L, o["LAM"]) <= 1e-10
        assert np.all(U > P.u_lo) and np.all(U < P.u_hi)
    s = nm.Solver(P, tol=1e-8, max_iter=20000)
    rc, X, U, L, info = s.solve(x0, xref, warm=start)
    o = oracle.solve(P, x0, xref, start=tuple(a.copy() for a in start), tol=1e-8, max_iter=20000)
    assert rc == nm.NMPC_OK and o["status"] == "converged"
    assert abs(info["iters"] - o["iters"]) <= 1
    assert rel(U, o["U"]) <= 1e-6


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_box_solve_matches_oracle(nm, prec):
    P, x0, xref, free = boxed_c0(seed=5)
    precision = nm.NMPC_FP64 if prec == "fp64" else nm.NMPC_FP32_SWEEP
    s = nm.Solver(P, tol=1e-8, max_iter=20000, precision=precision)
    rc, X, U, L, info = s.solve(x0, xref)
    o = oracle.solve(P, x0, xref, tol=1e-8, max_iter=20000)
    assert rc == nm.NMPC_OK and o["status"] == "converged"
    if prec == "fp64":
        assert abs(info["iters"] - o["iters"]) <= 1
    ex = oracle.solve(P, x0, xref, tol=1e-12, max_iter=50000)
    err = rel(U, ex["U"])
    print(f"{prec}: iterations GPU {info['iters']}, oracle {o['iters']}, input error {err:.2e}")
    assert err <= (1e-6 if prec == "fp64" else 1e-4)
    assert np.all(U > P.u_lo) and np.all(U < P.u_hi)
    assert rel(U, free["U"]) > 0.1                   # the box changed the answer
    r_s, _ = oracle.residual(P, x0, xref, X, U, L)
    assert r_s <= 1e-8 * (1 if prec == "fp64" else 10)


def test_start_outside_the_box_is_moved_inside(nm):
    """A warm start whose inputs leave the box is clipped into it (strictly
    feasible S^0, Sec. 4.2; 0.5 % of the box width from each bound) before
    anything else runs: given starts and starts built from inputs, with the
    fallback check. Iterates equal the oracle's, which applies the same rule."""
    from oracle.start import input_start
    P, x0, xref, free = boxed_c0(seed=4, tau_rel=1e-4)
    U0 = free["U"] * 1.3                      # about a third of the entries outside
    assert np.mean((U0 <= P.u_lo) | (U0 >= P.u_hi)) > 0.2
    d = 0.005 * (P.u_hi - P.u_lo)
    np.testing.assert_array_equal(oracle.feasible_inputs(P, U0),
                                  np.clip(U0, P.u_lo + d, P.u_hi - d))
    start = (free["X"].copy(), U0, free["LAM"].copy())
    for k in (0, 1, 3):
        s = nm.Solver(P, tol=0.0, max_iter=k)
        rc, X, U, L, info = s.solve(x0, xref, warm=start)
        s.close()
        o = oracle.solve(P, x0, xref, start=tuple(a.copy() for a in start), tol=0.0, max_iter=k)
        assert rc == nm.NMPC_E_NOCONV and info["iters"] == k
        assert rel(U, o["U"]) <= 1e-10 and rel(X, o["X"]) <= 1e-10
        assert rel(L, o["LAM"]) <= 1e-10
        assert np.all(U > P.u_lo) and np.all(U < P.u_hi)
        assert np.isfinite(info["r_scaled"])
    # start built from the inputs alone (rollout), fallback on
    s = nm.Solver(P, tol=0.0, max_iter=0, fallback=1)
    rc, X, U, L, info = s.solve(x0, xref, warm=(None, U0, None))
    s.close()
    Xs, Us, Ls = input_start(P, x0, xref, U0)
    np.testing.assert_array_equal(U, Us)
    assert rel(X, Xs) <= 1e-8 and rel(L, Ls) <= 1e-8
    assert info["start_used"] == 2 and np.isfinite(info["r_scaled"])
    # and the solve from it reaches the oracle's solution inside the box
    s = nm.Solver(P, tol=1e-8, max_iter=20000)
    rc, X, U, L, info = s.solve(x0, xref, warm=start)
    ex = oracle.solve(P, x0, xref, tol=1e-12, max_iter=50000)
    assert rc == nm.NMPC_OK and rel(U, ex["U"]) <= 1e-6


def test_box_2d_batch_fp32(nm):
    """Small 2D batch with FP32 sweeps: every instance converges inside the box,
    matching the oracle's solution of each instance."""
    import torch
    P0 = make_problem("grid", ns=16, N=8, lattice=2)
    x0, xr = make_batch(P0, [1, 2, 3])
    free = [oracle.solve(P0, x0[b], xr[b], tol=1e-10, max_iter=20000) for b in range(3)]
    umax = max(np.abs(f["U"]).max() for f in free)
    P = P0.with_(tau=1e-3 * P0.r * umax, u_lo=-0.5 * umax, u_hi=0.5 * umax)
    s = nm.Solver(P, max_batch=3, tol=1e-7, max_iter=20000, precision=nm.NMPC_FP32_SWEEP)
    rc, X, U, L, infos = s.solve_batch(torch.tensor(x0, device="cuda"),
                                       torch.tensor(xr, device="cuda"))
    assert rc == nm.NMPC_OK
    for b in range(3):
        ex = oracle.solve(P, x0[b], xr[b], tol=1e-11, max_iter=50000)
        assert ex["status"] == "converged"
        Ub = U[b].cpu().numpy()
        assert rel(Ub, ex["U"]) <= 1e-4
        assert np.all(Ub > P.u_lo) and np.all(Ub < P.u_hi)


@pytest.mark.parametrize("upper", ["fgs", "bgs", "sgs"])
def test_box_gauss_seidel_iterates_match_oracle(nm, upper):
    """The Gauss-Seidel layers with the input box (the paper's pairing, SGS):
    from a start where the fraction-to-the-boundary rule cuts the sweeps, the
    GPU iterates follow the oracle's (each sweep cut, S + alpha (S_sweep -
    S)); converged, the inputs equal the oracle's solution."""
    code = {"fgs": nm.NMPC_UPPER_FGS, "bgs": nm.NMPC_UPPER_BGS, "sgs": nm.NMPC_UPPER_SGS}[upper]
    P, x0, xref, free = boxed_c0(tau_rel=1e-5)
    start = (free["X"].copy(), np.clip(free["U"], 0.98 * P.u_lo, 0.98 * P.u_hi),
             free["LAM"].copy())
    sw = oracle.gs_sweep(P, x0, xref, *start, 1 if upper == "fgs" else -1)
    assert oracle.alpha_max(P, start[1], start[1] - sw[1]) < 0.5    # the rule cuts
    for prec in ("fp64", "fp32"):
        precision = nm.NMPC_FP64 if prec == "fp64" else nm.NMPC_FP32_SWEEP
        for k in ((1, 2, 5) if prec == "fp64" else (3,)):
            s = nm.Solver(P, tol=0.0, max_iter=k, upper=code, precision=precision)
            rc, X, U, L, info = s.solve(x0, xref, warm=start)
            s.close()
            o = oracle.solve(P, x0, xref, start=tuple(a.copy() for a in start), tol=0.0,
                             max_iter=k, upper=upper)
            assert rc == nm.NMPC_E_NOCONV and info["iters"] == k
            bar = 1e-10 if prec == "fp64" else 1e-3
            assert rel(U, o["U"]) <= bar, (prec, k, rel(U, o["U"]))
            if prec == "fp64":
                assert rel(X, o["X"]) <= bar and rel(L, o["LAM"]) <= bar
            assert np.all(U > P.u_lo) and np.all(U < P.u_hi)
    s = nm.Solver(P, tol=1e-8, max_iter=20000, upper=code)
    rc, X, U, L, info = s.solve(x0, xref)
    o = oracle.solve(P, x0, xref, tol=1e-8, max_iter=20000, upper=upper)
    assert rc == nm.NMPC_OK and o["status"] == "converged"
    assert abs(info["iters"] - o["iters"]) <= 1
    ok = o if info["iters"] == o["iters"] else oracle.solve(P, x0, xref, tol=0.0,
                                                            max_iter=info["iters"], upper=upper)
    assert rel(U, ok["U"]) <= 1e-9
    ex = oracle.solve(P, x0, xref, tol=1e-12, max_iter=50000)
    assert rel(U, ex["U"]) <= 1e-6


def test_box_sgs_fp32_batch_2d(nm):
    """2D batch, SGS, FP32 sweeps with the final FP64 correction and the box:
    every instance converges inside the box to the oracle's exact solution."""
    import torch
    P0 = make_problem("grid", ns=16, N=8, lattice=2)
    x0, xr = make_batch(P0, [1, 2, 3])
    free = [oracle.solve(P0, x0[b], xr[b], tol=1e-10, max_iter=20000) for b in range(3)]
    umax = max(np.abs(f["U"]).max() for f in free)
    P = P0.with_(tau=1e-3 * P0.r * umax, u_lo=-0.5 * umax, u_hi=0.5 * umax)
    s = nm.Solver(P, max_batch=3, tol=1e-7, max_iter=20000, precision=nm.NMPC_FP32_SWEEP,
                  upper=nm.NMPC_UPPER_SGS)
    rc, X, U, L, infos = s.solve_batch(torch.tensor(x0, device="cuda"),
                                       torch.tensor(xr, device="cuda"))
    assert rc == nm.NMPC_OK
    for b in range(3):
        ex = oracle.solve(P, x0[b], xr[b], tol=1e-11, max_iter=50000, upper="sgs")
        assert ex["status"] == "converged"
        Ub = U[b].cpu().numpy()
        assert rel(Ub, ex["U"]) <= 1e-4
        assert np.all(Ub > P.u_lo) and np.all(Ub < P.u_hi)


def test_box_arguments_are_checked(nm):
    P, x0, xref, _ = boxed_c0()
    bad = P.with_(u_lo=0.1)                          # cold start u = 0 outside
    with pytest.raises(nm.NmpcError) as e:
        nm.Solver(bad)
    assert e.value.code == nm.NMPC_E_ARG


def test_box_streaming_path_matches_oracle(nm):
    """The streaming (multi-pass) path with the input box: barrier rows in
    K^u and A_uu, stage limits from the final input step, the step cut by the
    instance's alpha. Equal-k iterates equal the oracle's from a start where
    the rule cuts (1D and a 2D grid); converged FP32 sweeps meet the exact
    solution inside the box."""
    P, x0, xref, free = boxed_c0(tau_rel=1e-5)
    start = (free["X"].copy(), np.clip(free["U"], 0.98 * P.u_lo, 0.98 * P.u_hi),
             free["LAM"].copy())
    assert step_alpha(P, x0, xref, *start) < 0.1
    for k in (1, 3):
        s = nm.Solver(P, tol=0.0, max_iter=k, path=nm.NMPC_PATH_STREAM)
        rc, X, U, L, info = s.solve(x0, xref, warm=start)
        s.close()
        o = oracle.solve(P, x0, xref, start=tuple(a.copy() for a in start), tol=0.0, max_iter=k)
        assert rc == nm.NMPC_E_NOCONV and info["iters"] == k
        assert rel(U, o["U"]) <= 1e-10 and rel(X, o["X"]) <= 1e-10 and rel(L, o["LAM"]) <= 1e-10
    P0 = make_problem("grid", ns=40, N=4, lattice=4)
    x0b, xrb = make_instance(P0, 2)
    fr = oracle.solve(P0, x0b, xrb, tol=1e-8, max_iter=20000)
    umax = np.abs(fr["U"]).max()
    Pb = P0.with_(tau=1e-3 * P0.r * umax, u_lo=-0.5 * umax, u_hi=0.5 * umax)
    for k in (2, 5):
        s = nm.Solver(Pb, tol=0.0, max_iter=k, path=nm.NMPC_PATH_STREAM)
        rc, X, U, L, info = s.solve(x0b, xrb)
        s.close()
        o = oracle.solve(Pb, x0b, xrb, tol=0.0, max_iter=k)
        assert rel(U, o["U"]) <= 1e-10 and rel(X, o["X"]) <= 1e-10 and rel(L, o["LAM"]) <= 1e-10
    s = nm.Solver(Pb, tol=1e-7, max_iter=20000, path=nm.NMPC_PATH_STREAM,
                  precision=nm.NMPC_FP32_SWEEP)
    rc, X, U, L, info = s.solve(x0b, xrb)
    ex = oracle.solve(Pb, x0b, xrb, tol=1e-11, max_iter=50000)
    assert rc == nm.NMPC_OK and rel(U, ex["U"]) <= 1e-4
    assert np.all(U > Pb.u_lo) and np.all(U < Pb.u_hi)
    assert rel(U, fr["U"]) > 0.05     # the box changed the answer
