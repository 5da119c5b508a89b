"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

Same start and schedule: iterate S^k must agree element by element (the only
differences are FP64 rounding order, e.g. in the B^T sums), so the bar is a
relative 1e-10 on every trajectory. Converged results are also compared with
the oracle run to r_scaled <= 1e-12 ("exact"), and the measured control error
is asserted against the FP64 (1e-6) and FP32-sweep (1e-4) bars.
"""
import numpy as np
import pytest

from nmpc_inputs import gaussian_factors, make_batch, make_instance, make_problem

import oracle

pytestmark = pytest.mark.gpu

REL = 1e-10


def rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def nm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2004_02484_amd as nm
    return nm


def ragged2d(nsx, nsy, N, lattice=2, sigma=0.2, gamma_rel=1.0):
    P = make_problem("grid", ns=nsx, N=N, lattice=lattice, gamma_rel=gamma_rel)
    P = P.with_(nsy=nsy, gx=gaussian_factors(nsx, lattice, sigma),
                gy=gaussian_factors(nsy, lattice, sigma))
    P.h = 0.2 / (0.75 * max(nsx + 1, nsy + 1) ** 2)
    P.gamma = gamma_rel * P.h * P.r
    return P


def check_same_iterate(P, x0, xref, k, nm, **opts):
    s = nm.Solver(P, tol=0.0, max_iter=k, **opts)
    rc, X, U, L, info = s.solve(x0, xref)
    s.close()
    o = oracle.solve(P, x0, xref, tol=0.0, max_iter=k,
                     n_sw=opts.get("n_sweep", 2), n_schur=opts.get("n_schur", 2))
    assert rc == nm.NMPC_E_NOCONV and info["iters"] == k
    assert rel(X, o["X"]) <= REL
    assert rel(L, o["LAM"]) <= REL if np.abs(o["LAM"]).max() > 0 else np.all(L == 0)
    assert rel(U, o["U"]) <= REL if np.abs(o["U"]).max() > 0 else np.all(U == 0)
    # the input rows h (r u + B^T lam) cancel; their B^T sums run in another
    # order on the GPU, so the norms carry a few ulps of the summands
    assert abs(info["r_scaled"] - o["r_scaled"]) <= 1e-9 * o["r_scaled"]
    assert abs(info["r_paper"] - o["r_paper"]) <= 1e-9 * o["r_paper"]


@pytest.mark.parametrize("k", [0, 1, 2, 7, 40])
def test_c0_iterates_match_oracle(nm, k):
    P = make_problem("c0")
    x0, xref = make_instance(P, 0)
    check_same_iterate(P, x0, xref, k, nm)


@pytest.mark.parametrize("k", [1, 3])
def test_c1_iterates_match_oracle(nm, k):
    P = make_problem("c1")
    x0, xref = make_instance(P, 1)
    check_same_iterate(P, x0, xref, k, nm)


@pytest.mark.parametrize("shape", [(13, 37, 6), (64, 5, 3), (7, 16, 4), (40, 64, 2), (57, 23, 3)])
def test_ragged_shapes_match_oracle(nm, shape):
    """Grids that leave lanes, rows and waves partly empty (ragged tails);
    57 columns: 4-column tiles whose last lanes are partly or wholly past the
    grid (the 16-byte accesses of those tiles mask them)."""
    nsx, nsy, N = shape
    P = ragged2d(nsx, nsy, N)
    x0, xref = make_instance(P, 5)
    check_same_iterate(P, x0, xref, 5, nm)


def test_partial_four_column_tiles_fp32_solve(nm):
    """FP32 sweeps with the final correction on a 57 x 23 grid (4-column
    tiles with lanes past the grid, partial rows): the returned trajectory
    meets the tolerance by the oracle's residual and the FP32-sweep bar
    against the oracle's exact solution."""
    P = ragged2d(57, 23, 4)
    x0, xref = make_instance(P, 6)
    s = nm.Solver(P, precision=nm.NMPC_FP32_SWEEP, tol=1e-6)
    rc, X, U, L, info = s.solve(x0, xref)
    s.close()
    assert rc == nm.NMPC_OK
    rs, _ = oracle.residual(P, x0, xref, X, U, L)
    ex = oracle.solve(P, x0, xref, tol=1e-12, max_iter=20000)
    err = np.abs(U - ex["U"]).max() / np.abs(ex["U"]).max()
    print(f"57 x 23: {info['iters']} iterations, oracle residual {rs:.2e}, control error {err:.2e}")
    assert rs <= 1e-6 and err <= 1e-4


@pytest.mark.parametrize("nsw,nsc", [(1, 0), (3, 1), (4, 3)])
def test_schedule_variants_match_oracle(nm, nsw, nsc):
    P = make_problem("grid", ns=24, N=5)
    x0, xref = make_instance(P, 2)
    check_same_iterate(P, x0, xref, 4, nm, n_sweep=nsw, n_schur=nsc)


def test_degenerate_single_node_single_stage(nm):
    P = make_problem("c0").with_(nsx=1, N=1, lx=1, gx=np.ones((1, 1)))
    x0 = np.array([0.1]); xref = np.array([0.3])
    check_same_iterate(P, x0, xref, 3, nm)
    s = nm.Solver(P)
    rc, X, U, L, info = s.solve(x0, xref)
    o = oracle.solve(P, x0, xref, tol=1e-6)
    assert rc == nm.NMPC_OK and info["iters"] == o["iters"]
    assert rel(U, o["U"]) <= REL


def oracle_at(P, x0, xref, o, k, **kw):
    """The oracle's iterate S^k: ``o`` itself when it stopped at k, else the
    oracle rerun without a tolerance for exactly k upper iterations (the two
    stopping tests may fall on either side of a threshold tie)."""
    if o["iters"] == k:
        return o
    return oracle.solve(P, x0, xref, tol=0.0, max_iter=k, **kw)


@pytest.mark.parametrize("name,seed", [("c0", 3), ("c1", 4)])
def test_converged_solution_matches_oracle(nm, name, seed):
    P = make_problem(name)
    x0, xref = make_instance(P, seed)
    s = nm.Solver(P)
    rc, X, U, L, info = s.solve(x0, xref)
    o = oracle.solve(P, x0, xref, tol=1e-6)
    assert rc == nm.NMPC_OK and o["status"] == "converged"
    assert abs(info["iters"] - o["iters"]) <= 1
    assert info["err_vs_fp64"] == 0.0     # an FP64 solve has no FP32 phase
    # element by element against the oracle's iterate of the same index, always
    ok = oracle_at(P, x0, xref, o, info["iters"])
    assert rel(X, ok["X"]) <= 1e-9 and rel(U, ok["U"]) <= 1e-9 and rel(L, ok["LAM"]) <= 1e-9
    err_oracle = rel(U, ok["U"])
    assert err_oracle <= 1e-6          # the FP64 bar against the oracle
    assert info["r_scaled"] <= 1e-6
    # the returned trajectory satisfies the KKT conditions (oracle re-check)
    rs, _ = oracle.residual(P, x0, xref, X, U, L)
    assert rs <= 1e-6 and abs(rs - info["r_scaled"]) <= 1e-9 * rs
    ex = oracle.solve(P, x0, xref, tol=1e-12, max_iter=20000)
    err = rel(U, ex["U"])
    print(f"{name}: iters {info['iters']} (oracle {o['iters']}), control rel. error vs the "
          f"oracle's S^k {err_oracle:.2e}, vs exact {err:.2e}")
    assert err <= 1e-4


@pytest.mark.parametrize("name,seed", [("c0", 3), ("c1", 4)])
def test_fp64_solution_meets_the_fp64_bar_against_the_exact_solution(nm, name, seed):
    """At tol 1e-9 the FP64 solve is within 1e-6 (relative, controls) of the
    oracle's exact solution (r_scaled <= 1e-12); at tol 1e-6 the distance to
    the exact solution is set by the tolerance (C0: about 2e-6), not by the
    GPU arithmetic, which the same-k comparison above bounds."""
    P = make_problem(name)
    x0, xref = make_instance(P, seed)
    s = nm.Solver(P, tol=1e-9, max_iter=20000)
    rc, X, U, L, info = s.solve(x0, xref)
    assert rc == nm.NMPC_OK
    ex = oracle.solve(P, x0, xref, tol=1e-12, max_iter=20000)
    err = rel(U, ex["U"])
    print(f"{name}: tol 1e-9, {info['iters']} iterations, control rel. error vs exact {err:.2e}")
    assert err <= 1e-6


def test_batch_matches_single_solves(nm):
    import torch
    P = make_problem("c1")
    seeds = [10, 11, 12]
    x0, xref = make_batch(P, seeds)
    s = nm.Solver(P, max_batch=4)
    rc, X, U, L, infos = s.solve_batch(torch.tensor(x0, device="cuda"),
                                       torch.tensor(xref, device="cuda"))
    assert rc == nm.NMPC_OK
    for b, sd in enumerate(seeds):
        o = oracle.solve(P, x0[b], xref[b], tol=1e-6)
        assert abs(infos[b]["iters"] - o["iters"]) <= 1
        ok = oracle_at(P, x0[b], xref[b], o, infos[b]["iters"])
        assert rel(U[b].cpu().numpy(), ok["U"]) <= 1e-9
        assert rel(X[b].cpu().numpy(), ok["X"]) <= 1e-9
        assert rel(L[b].cpu().numpy(), ok["LAM"]) <= 1e-9
    # graph replay length does not change the result
    s.set_options(check_every=1)
    rc2, X2, U2, L2, infos2 = s.solve_batch(torch.tensor(x0, device="cuda"),
                                            torch.tensor(xref, device="cuda"))
    assert torch.equal(U2, U) and torch.equal(X2, X) and torch.equal(L2, L)
    assert [i["iters"] for i in infos2] == [i["iters"] for i in infos]


@pytest.mark.parametrize("upper", ["jacobi", "sgs"])
def test_timing_counts_evaluation_only_units_apart(nm, upper):
    """The timing counters count a unit per stage visit that evaluates and
    updates, and apart from them the evaluation-only visits: the check of the
    FP64-corrected iterate of an FP32-sweep solve, one visit per stage of each
    instance. FP64 and fp32_finish solves have none."""
    import torch
    P = make_problem("c0")
    x0, xref = make_batch(P, [30, 31, 32])
    dx0, dxr = torch.tensor(x0, device="cuda"), torch.tensor(xref, device="cuda")
    up = {"jacobi": nm.NMPC_UPPER_JACOBI, "sgs": nm.NMPC_UPPER_SGS}[upper]
    for prec, fin, evals in ((nm.NMPC_FP32_SWEEP, 0, 3 * P.N), (nm.NMPC_FP64, 0, 0),
                             (nm.NMPC_FP32_SWEEP, 1, 0)):
        s = nm.Solver(P, max_batch=4, precision=prec, fp32_finish=fin, upper=up)
        s.timing_enable(True)
        rc, X, U, L, infos = s.solve_batch(dx0, dxr)
        tm = s.timing_read()
        s.close()
        assert rc == nm.NMPC_OK
        assert tm["eval_units"] == evals, (prec, fin, tm)
        if upper == "jacobi":
            # S^0 .. S^j evaluated with their (speculative) updates, plus the
            # FP64 step from S^j in the corrected variant (iters counts it)
            assert tm["units"] == sum((i["iters"] + 1) * P.N for i in infos), (prec, fin, tm)
        else:
            # two sweeps per SGS iteration after the first evaluation
            assert tm["units"] >= sum(2 * i["iters"] * P.N for i in infos), (prec, fin, tm)


def test_first_graph_sized_from_the_previous_solve_keeps_the_results(nm):
    """FP32-sweep Jacobi solves of one handle: the first graph of a solve is
    sized from the previous solve's iteration count (its FP32 launches, then
    the final FP64 correction's three). Whether the estimate is exact (the
    same warm solve again) or too short (a cold solve after a warm one), every
    result equals, bit for bit, that of a fresh handle, which runs the
    ordinary graphs."""
    import torch
    P = make_problem("c1")
    x0, xref = make_batch(P, [20, 21, 22])
    dx0, dxr = torch.tensor(x0, device="cuda"), torch.tensor(xref, device="cuda")
    opts = dict(max_batch=4, precision=nm.NMPC_FP32_SWEEP, check_every=16)

    def fresh(warm=None):
        s = nm.Solver(P, **opts)
        out = s.solve_batch(dx0, dxr, warm=warm)
        s.close()
        return out

    rc, Xc, Uc, Lc, ic = fresh()
    assert rc == nm.NMPC_OK
    rng = np.random.default_rng(4)   # a warm start: the solution with noisy inputs
    Up = (Uc * (1.0 + 1e-4 * torch.tensor(rng.standard_normal(Uc.shape), device="cuda"))).contiguous()
    warm = (Xc.clone(), Up, Lc.clone())
    rw, Xw, Uw, Lw, iw = fresh(warm)
    assert rw == nm.NMPC_OK
    assert max(i["iters"] for i in iw) + 4 <= 16 < max(i["iters"] for i in ic)
    s = nm.Solver(P, **opts)
    for want, w in (((Xw, Uw, Lw, iw), warm),       # sets the estimate
                    ((Xw, Uw, Lw, iw), warm),       # estimate exact
                    ((Xc, Uc, Lc, ic), None)):      # estimate too short
        rc, X, U, L, info = s.solve_batch(dx0, dxr, warm=w)
        assert rc == nm.NMPC_OK
        assert torch.equal(X, want[0]) and torch.equal(U, want[1]) and torch.equal(L, want[2])
        for a, b in zip(info, want[3]):
            assert (a["iters"], a["fp32_iters"], a["r_scaled"], a["err_vs_fp64"]) == \
                   (b["iters"], b["fp32_iters"], b["r_scaled"], b["err_vs_fp64"])


def test_residual_batch_matches_oracle(nm):
    import torch
    P = make_problem("c1")
    x0, xref = make_batch(P, [1, 2])
    rng = np.random.default_rng(0)
    X = rng.uniform(0, 0.2, (2, P.N, P.n)); U = rng.normal(size=(2, P.N, P.m))
    L = rng.normal(size=(2, P.N, P.n)) * 1e-3
    s = nm.Solver(P, max_batch=2)
    t = lambda a: torch.tensor(a, device="cuda")
    rs, rp = s.residual_batch(t(x0), t(xref), t(X), t(U), t(L))
    for b in range(2):
        ors, orp = oracle.residual(P, x0[b], xref[b], X[b], U[b], L[b])
        assert abs(rs[b] - ors) <= 1e-12 * ors and abs(rp[b] - orp) <= 1e-12 * orp


def test_fp32_sweeps_reach_fp64_fixed_point(nm):
    P = make_problem("c1")
    x0, xref = make_instance(P, 6)
    s = nm.Solver(P, precision=nm.NMPC_FP32_SWEEP)
    rc, X, U, L, info = s.solve(x0, xref)
    assert rc == nm.NMPC_OK and info["fp32_iters"] > 0 and info["r_scaled"] <= 1e-6
    rs, _ = oracle.residual(P, x0, xref, X, U, L)
    assert rs <= 1e-6
    ex = oracle.solve(P, x0, xref, tol=1e-12, max_iter=20000)
    err = rel(U, ex["U"])
    print(f"fp32 sweeps: iters {info['iters']} (fp32 {info['fp32_iters']}), "
          f"control rel. error vs exact {err:.2e}, err_vs_fp64 {info['err_vs_fp64']:.2e}")
    assert err <= 1e-4
    assert 0.0 < info["err_vs_fp64"] <= 1e-4


def test_fp32_finish_returns_the_fp32_phase_iterate(nm):
    """fp32_finish = 1: the solve ends where the FP32 phase's test passes, one
    upper iteration before the default (which then takes the FP64 correction
    step and tests its result). The returned iterate passes the oracle's FP64
    residual test and meets the FP32-sweep bar against the exact solution."""
    import torch
    P = make_problem("c1")
    x0s, xrefs = make_batch(P, [6, 9])
    X0, XR = torch.tensor(x0s, device="cuda"), torch.tensor(xrefs, device="cuda")
    runs = {}
    for fin in (0, 1):
        s = nm.Solver(P, max_batch=2, precision=nm.NMPC_FP32_SWEEP, fp32_finish=fin)
        rc, X, U, L, infos = s.solve_batch(X0, XR)
        assert rc == nm.NMPC_OK
        runs[fin] = (X.cpu().numpy(), U.cpu().numpy(), L.cpu().numpy(), infos)
        s.close()
    for b in range(2):
        X, U, L, infos = runs[1]
        i0, i1 = runs[0][3][b], infos[b]
        assert i1["iters"] <= i0["iters"] - 1 and i1["r_scaled"] <= 1e-6
        rs, _ = oracle.residual(P, x0s[b], xrefs[b], X[b], U[b], L[b])
        # the two residuals differ by the rounding of differently ordered sums
        assert rs <= 1e-6 and abs(rs - i1["r_scaled"]) <= 1e-12
        ex = oracle.solve(P, x0s[b], xrefs[b], tol=1e-12, max_iter=20000)
        err = rel(U[b], ex["U"])
        print(f"instance {b}: fp32_finish {i1['iters']} iterations (default {i0['iters']}), "
              f"control rel. error vs exact {err:.2e} (default {rel(runs[0][1][b], ex['U']):.2e}),"
              f" err_vs_fp64 {i0['err_vs_fp64']:.2e}")
        assert err <= 1e-4
        # err_vs_fp64: the default's FP64 correction step from the FP32-phase
        # iterate, which is what fp32_finish returns (same arithmetic up to it)
        assert i1["err_vs_fp64"] == -1.0
        if i0["iters"] == i1["iters"] + 1:
            step = np.abs(runs[0][1][b] - U[b]).max() / np.abs(runs[0][1][b]).max()
            assert abs(i0["err_vs_fp64"] - step) <= 1e-6 * step, (i0["err_vs_fp64"], step)
        assert 0.0 < i0["err_vs_fp64"] <= 1e-4


def test_warm_start_and_failure_statuses(nm):
    P = make_problem("c0")
    x0, xref = make_instance(P, 7)
    ex = oracle.solve(P, x0, xref, tol=1e-10)
    s = nm.Solver(P)
    rc, X, U, L, info = s.solve(x0, xref, warm=(ex["X"], ex["U"], ex["LAM"]))
    assert rc == nm.NMPC_OK and info["iters"] == 0
    np.testing.assert_array_equal(U, ex["U"])
    bad = ex["U"].copy(); bad[2, 1] = np.nan
    rc, X, U, L, info = s.solve(x0, xref, warm=(ex["X"], bad, ex["LAM"]))
    assert rc == nm.NMPC_E_NONFINITE and info["iters"] == 0
    s.set_options(max_iter=3)
    rc, X, U, L, info = s.solve(x0, xref)
    o = oracle.solve(P, x0, xref, tol=1e-6, max_iter=3)
    assert rc == nm.NMPC_E_NOCONV and info["iters"] == 3 and rel(U, o["U"]) <= REL


def test_time_varying_reference(nm):
    P = make_problem("c0")
    x0, xref = make_instance(P, 8)
    xr = np.stack([xref * (1.0 - 0.02 * i) for i in range(P.N)])
    s = nm.Solver(P, xref_per_stage=1, tol=0.0, max_iter=6)
    rc, X, U, L, info = s.solve(x0, xr)
    o = oracle.solve(P, x0, xr, tol=0.0, max_iter=6)
    assert rel(U, o["U"]) <= REL and rel(L, o["LAM"]) <= REL


@pytest.mark.parametrize("upper", [0, 3])
def test_widest_fused_grid(nm, upper):
    """96 x 96 (six columns and three rows per lane, 8 waves) on the fused
    path, Jacobi and SGS: equal iterate to the oracle at k = 2."""
    P = make_problem("grid", ns=96, N=3, lattice=4)
    x0, xref = make_instance(P, 12)
    s = nm.Solver(P, tol=0.0, max_iter=2, path=nm.NMPC_PATH_FUSED, upper=upper)
    assert s.kernel_config()["rows_per_lane"] == 3
    rc, X, U, L, info = s.solve(x0, xref)
    o = oracle.solve(P, x0, xref, tol=0.0, max_iter=2,
                     upper="jacobi" if upper == 0 else "sgs")
    assert rc == nm.NMPC_E_NOCONV and info["iters"] == 2
    assert rel(X, o["X"]) <= REL and rel(U, o["U"]) <= REL and rel(L, o["LAM"]) <= REL


def test_batch_count_outside_the_handle_is_refused(nm):
    """An empty batch and a batch beyond the handle's capacity are argument
    errors, reported before any device work (the outputs stay untouched)."""
    import torch
    P = make_problem("c0")
    s = nm.Solver(P, max_batch=2)
    n = P.nsx * P.nsy
    for count in (0, 3):
        x0 = torch.zeros((count, n), dtype=torch.float64, device="cuda")
        out = tuple(torch.full(sh, 7.0, dtype=torch.float64, device="cuda")
                    for sh in ((count, P.N, n), (count, P.N, P.m), (count, P.N, n)))
        with pytest.raises(nm.NmpcError) as e:
            s.solve_batch(x0, x0.clone(), out=out)
        assert e.value.code == nm.NMPC_E_ARG
        assert all(bool((o == 7.0).all()) for o in out)
    s.close()
