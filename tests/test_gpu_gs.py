"""GPU parity of the Gauss-Seidel upper layers (FGS, BGS, SGS) against the
CPU oracle's sweeps, through the C ABI.

Same start, same upper layer and schedule, equal iteration k: every
trajectory entry within 1e-10 relative (FP64 kernels; the only differences
are FP64 summation orders). Converged results against the oracle run to
r_scaled <= 1e-11, with the FP32-sweep bar of 1e-4 on the inputs.
"""
import numpy as np
import pytest

from nmpc_inputs import gaussian_factors, make_batch, make_instance, make_problem

import oracle

pytestmark = pytest.mark.gpu

REL = 1e-10
UPPERS = {"fgs": 1, "bgs": 2, "sgs": 3}


def rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def nm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2004_02484_amd as nm
    return nm


def shaped(nsx, nsy, N, lattice):
    P = make_problem("grid", ns=nsx, N=N, lattice=lattice)
    sigma = 0.05 if lattice == 4 else 0.2
    P = P.with_(nsy=nsy, gx=gaussian_factors(nsx, lattice, sigma),
                gy=gaussian_factors(nsy, lattice, sigma))
    P.h = 0.2 / (0.75 * max(nsx + 1, nsy + 1) ** 2)
    P.gamma = P.h * P.r
    return P


CASES = [("c0", None), ("13x37x6 L2", (13, 37, 6, 2)), ("48x40x5 L4", (48, 40, 5, 4)),
         ("64x64x3 L4", (64, 64, 3, 4)), ("7x16x1 L2", (7, 16, 1, 2))]


@pytest.mark.parametrize("upper", list(UPPERS))
@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_gs_iterates_match_oracle(nm, upper, case):
    spec = dict(CASES)[case]
    P = make_problem("c0") if spec is None else shaped(*spec)
    x0, xref = make_instance(P, 7)
    for k in (1, 3):
        s = nm.Solver(P, tol=0.0, max_iter=k, upper=UPPERS[upper])
        rc, X, U, L, info = s.solve(x0, xref)
        s.close()
        o = oracle.solve(P, x0, xref, tol=0.0, max_iter=k, upper=upper)
        assert rc == nm.NMPC_E_NOCONV and info["iters"] == k
        assert rel(X, o["X"]) <= REL, (k, rel(X, o["X"]))
        assert rel(U, o["U"]) <= REL, (k, rel(U, o["U"]))
        assert rel(L, o["LAM"]) <= REL, (k, rel(L, o["LAM"]))
        assert abs(info["r_scaled"] - o["r_scaled"]) <= 1e-9 * o["r_scaled"]
        assert abs(info["r_paper"] - o["r_paper"]) <= 1e-9 * o["r_paper"]


@pytest.mark.parametrize("upper", list(UPPERS))
def test_gs_converges_like_the_oracle_fp64(nm, upper):
    P = make_problem("c0")
    x0, xref = make_instance(P, 2)
    s = nm.Solver(P, tol=1e-8, max_iter=5000, upper=UPPERS[upper])
    rc, X, U, L, info = s.solve(x0, xref)
    o = oracle.solve(P, x0, xref, tol=1e-8, max_iter=5000, upper=upper)
    assert rc == nm.NMPC_OK and o["status"] == "converged"
    assert abs(info["iters"] - o["iters"]) <= 1
    ex = oracle.solve(P, x0, xref, tol=1e-12, max_iter=50000)
    assert rel(U, ex["U"]) <= 1e-6
    r_s, _ = oracle.residual(P, x0, xref, X, U, L)
    assert r_s <= 1e-8


def test_sgs_fp32_sweeps_c1_batch(nm):
    """C1 batch with FP32 sweeps and SGS: every instance converges, the
    inputs match the oracle's exact solution to 1e-4, and the iteration
    count is that of the oracle's SGS."""
    import torch
    P = make_problem("c1")
    seeds = [31, 32, 33, 34]
    x0, xr = make_batch(P, seeds)
    s = nm.Solver(P, max_batch=4, tol=1e-6, max_iter=3000, precision=nm.NMPC_FP32_SWEEP,
                  upper=nm.NMPC_UPPER_SGS)
    rc, X, U, L, infos = s.solve_batch(torch.tensor(x0, device="cuda"),
                                       torch.tensor(xr, device="cuda"))
    assert rc == nm.NMPC_OK
    o = oracle.solve(P, x0[0], xr[0], tol=1e-6, max_iter=3000, upper="sgs")
    its = [i["iters"] for i in infos]
    print(f"SGS iterations GPU {its}, oracle (first instance) {o['iters']}")
    assert abs(its[0] - o["iters"]) <= 2
    for b in (0, 3):
        ex = oracle.solve(P, x0[b], xr[b], tol=1e-11, max_iter=20000)
        err = rel(U[b].cpu().numpy(), ex["U"])
        print(f"instance {b}: control error vs exact {err:.2e}, "
              f"err_vs_fp64 {infos[b]['err_vs_fp64']:.2e}")
        assert err <= 1e-4
        assert 0.0 < infos[b]["err_vs_fp64"] <= 1e-4
        r_s, _ = oracle.residual(P, x0[b], xr[b], X[b].cpu().numpy(), U[b].cpu().numpy(),
                                 L[b].cpu().numpy())
        assert r_s <= 1e-6


def test_sgs_fp32_finish(nm):
    """fp32_finish = 1 with SGS: the solve returns the iterate whose test passed
    in the FP32 phase, one iteration before the default's FP64-corrected one;
    it passes the oracle's residual test and meets the FP32-sweep bar."""
    import torch
    P = make_problem("c1")
    x0, xr = make_batch(P, [35, 36])
    X0, XR = torch.tensor(x0, device="cuda"), torch.tensor(xr, device="cuda")
    runs = {}
    for fin in (0, 1):
        s = nm.Solver(P, max_batch=2, tol=1e-6, max_iter=3000, precision=nm.NMPC_FP32_SWEEP,
                      upper=nm.NMPC_UPPER_SGS, fp32_finish=fin)
        rc, X, U, L, infos = s.solve_batch(X0, XR)
        assert rc == nm.NMPC_OK
        runs[fin] = (X.cpu().numpy(), U.cpu().numpy(), L.cpu().numpy(), infos)
        s.close()
    X, U, L, infos = runs[1]
    for b in range(2):
        assert infos[b]["iters"] <= runs[0][3][b]["iters"] - 1
        r_s, _ = oracle.residual(P, x0[b], xr[b], X[b], U[b], L[b])
        assert r_s <= 1e-6
        ex = oracle.solve(P, x0[b], xr[b], tol=1e-11, max_iter=20000)
        err = rel(U[b], ex["U"])
        print(f"instance {b}: {infos[b]['iters']} iterations "
              f"(default {runs[0][3][b]['iters']}), control error vs exact {err:.2e}")
        assert err <= 1e-4
        assert infos[b]["err_vs_fp64"] == -1.0
        d = runs[0][3][b]
        assert 0.0 < d["err_vs_fp64"] <= 1e-4
        if d["iters"] == infos[b]["iters"] + 1:   # one FP64 sweep from the FP32 iterate
            step = np.abs(runs[0][1][b] - U[b]).max() / np.abs(runs[0][1][b]).max()
            assert abs(d["err_vs_fp64"] - step) <= 1e-6 * step


def test_sgs_batch_equals_single_solves(nm):
    import torch
    P = shaped(40, 33, 6, 4)
    x0, xr = make_batch(P, [1, 2, 3])
    s = nm.Solver(P, max_batch=3, tol=1e-7, max_iter=3000, upper=nm.NMPC_UPPER_SGS)
    rc, X, U, L, infos = s.solve_batch(torch.tensor(x0, device="cuda"),
                                       torch.tensor(xr, device="cuda"))
    assert rc == nm.NMPC_OK
    for b in range(3):
        rc1, X1, U1, L1, i1 = s.solve(x0[b], xr[b])
        assert i1["iters"] == infos[b]["iters"]
        np.testing.assert_array_equal(U1, U[b].cpu().numpy())
        np.testing.assert_array_equal(X1, X[b].cpu().numpy())


def test_sgs_with_starts_and_statuses(nm):
    P = make_problem("c0")
    x0, xref = make_instance(P, 4)
    ex = oracle.solve(P, x0, xref, tol=1e-12, max_iter=50000)
    s = nm.Solver(P, tol=1e-8, upper=nm.NMPC_UPPER_SGS)
    rc, X, U, L, info = s.solve(x0, xref, warm=(ex["X"], ex["U"], ex["LAM"]))
    assert rc == nm.NMPC_OK and info["iters"] == 0
    rc, X, U, L, info = s.solve(x0, xref, warm=(None, ex["U"] * (1 + 1e-3), None))
    assert rc == nm.NMPC_OK and info["start_used"] == 2
    bad = np.full_like(ex["U"], np.nan)
    s2 = nm.Solver(P, tol=1e-8, upper=nm.NMPC_UPPER_SGS)
    rc, X, U, L, info = s2.solve(x0, xref, warm=(ex["X"], bad, ex["LAM"]))
    assert rc == nm.NMPC_E_NONFINITE
    s3 = nm.Solver(P, tol=0.0, max_iter=3, upper=nm.NMPC_UPPER_SGS,
                   precision=nm.NMPC_FP32_SWEEP)
    rc, X, U, L, info = s3.solve(x0, xref)
    assert rc == nm.NMPC_E_NOCONV and info["iters"] == 3


def test_sgs_autotune_keeps_the_results(nm):
    import torch
    P = make_problem("grid", ns=64, N=6, lattice=4)
    x0, xr = make_batch(P, [5, 6])
    X0, XR = torch.tensor(x0, device="cuda"), torch.tensor(xr, device="cuda")
    s = nm.Solver(P, max_batch=2, tol=0.0, max_iter=4, precision=nm.NMPC_FP32_SWEEP,
                  upper=nm.NMPC_UPPER_SGS)
    _, _, U0, _, _ = s.solve_batch(X0, XR)
    U0 = U0.cpu().numpy()
    tr = s.autotune(X0, XR, iters=3)
    cfg = s.kernel_config()
    print(f"SGS tile rows {tr}, waves {cfg['waves']}")
    _, _, U1, _, _ = s.solve_batch(X0, XR)
    assert rel(U1.cpu().numpy(), U0) <= 1e-5


@pytest.mark.parametrize("upper", ["fgs", "bgs", "sgs"])
@pytest.mark.parametrize("omega", [0.8, 1.3])
def test_sor_iterates_match_oracle(nm, upper, omega):
    """Over-relaxed sweeps (SOR, backward SOR, SSOR): the first iterates match
    the oracle's relaxed sweeps, and the solve converges to the Jacobi fixed
    point with the oracle's iteration count."""
    P = shaped(13, 37, 6, 2)
    x0, xref = make_instance(P, 5)
    for k in (1, 3):
        s = nm.Solver(P, tol=0.0, max_iter=k, upper=UPPERS[upper], omega=omega)
        rc, X, U, L, info = s.solve(x0, xref)
        s.close()
        o = oracle.solve(P, x0, xref, tol=0.0, max_iter=k, upper=upper, omega=omega)
        assert rc == nm.NMPC_E_NOCONV and info["iters"] == k
        assert rel(X, o["X"]) <= REL and rel(U, o["U"]) <= REL and rel(L, o["LAM"]) <= REL
    s = nm.Solver(P, tol=1e-8, max_iter=5000, upper=UPPERS[upper], omega=omega)
    rc, X, U, L, info = s.solve(x0, xref)
    o = oracle.solve(P, x0, xref, tol=1e-8, max_iter=5000, upper=upper, omega=omega)
    assert rc == nm.NMPC_OK and o["status"] == "converged"
    assert abs(info["iters"] - o["iters"]) <= 1
    ex = oracle.solve(P, x0, xref, tol=1e-12, max_iter=50000)
    assert rel(U, ex["U"]) <= 1e-6
