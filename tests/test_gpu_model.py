"""The model engine on the GPU (copper plate, second-order wave, dense-B heat)
against its oracle (``oracle/models.py``), through the C ABI.

Same start and schedule: the iterate S^k after k upper iterations must agree
element by element (FP64 on both sides; the only differences are the order of
the stencil and B^T sums), bar 1e-10 relative, with every upper layer and the
input box (barrier and fraction-to-the-boundary rule) active. Converged
solves: the GPU's iteration count is the oracle's (+-1 at threshold ties) and
the returned trajectory equals the oracle's iterate of the same index.
"""
import numpy as np
import pytest

from nmpc_inputs import (ModelProblem, gaussian_factors, make_plate_instance, make_plate_problem,
                         make_wave_instance, make_wave_problem)
from oracle import models as om

pytestmark = pytest.mark.gpu

REL = 1e-10
UPPERS = {"jacobi": 0, "fgs": 1, "bgs": 2, "sgs": 3}


@pytest.fixture(scope="module")
def nm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2004_02484_amd as m
    return m


def rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


def small_plate(N=4, tau=20.0):
    """7 x 7 Neumann plate with 4 actuator nodes, the paper's physics sped up
    (alpha x 20) so that the stencil matters at this size; box binding."""
    P = make_plate_problem()
    return P.with_(nsx=7, nsy=7, N=N, act=[16, 18, 30, 32], alpha=P.alpha * 20, tau=tau)


def dense_heat(nsx=9, nsy=6, N=4, m=3, seed=4):
    rng = np.random.default_rng(seed)
    B = rng.uniform(0, 1, (nsx * nsy, m))
    h = 0.2 / (0.75 * (max(nsx, nsy) + 1) ** 2)
    return ModelProblem(model="heat", nsx=nsx, nsy=nsy, N=N, h=h, boundary="dirichlet", B=B,
                        q=1.0, r=0.01, gamma=0.01 * h, k0=0.5, k1=0.5)


def instance(P, seed):
    if P.model == "plate":
        return make_plate_instance(P, seed)
    if P.model == "wave":
        return make_wave_instance(P, seed)
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 0.2, P.nodes), rng.uniform(-0.3, 0.3, P.nodes)


def gpu_solve(nm, P, x0, xref, warm=None, **opts):
    import torch
    s = nm.ModelSolver(P, max_batch=1, **opts)
    t = lambda a: torch.tensor(np.asarray(a)[None], device="cuda")
    w = None if warm is None else tuple(t(a) for a in warm)
    rc, X, U, L, info = s.solve_batch(t(x0), t(xref), warm=w)
    s.close()
    return rc, X[0].cpu().numpy(), U[0].cpu().numpy(), L[0].cpu().numpy(), info[0]


def compare(ops, o, X, U, L, bar):
    """GPU grid-layout trajectory against the oracle's compact one."""
    Xo = om.to_grid(ops, o["X"], o["U"])
    Lo = om.to_grid(ops, o["LAM"])
    assert rel(U, o["U"]) <= bar, ("u", rel(U, o["U"]))
    assert rel(X, Xo) <= bar, ("x", rel(X, Xo))
    if np.abs(Lo).max() > 0:
        assert rel(L, Lo) <= bar, ("lambda", rel(L, Lo))
    else:
        assert np.all(L == 0)


CASES = {
    "plate7": lambda: small_plate(),
    "plate13": lambda: make_plate_problem(),
    "wave6": lambda: make_wave_problem(ns=6, N=4),
    "heat9x6": lambda: dense_heat(),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("upper", list(UPPERS))
def test_model_iterates_match_oracle(nm, case, upper):
    P = CASES[case]()
    ops = om.Ops(P)
    x0, xref = instance(P, 3)
    for k in (0, 1, 3):
        rc, X, U, L, info = gpu_solve(nm, P, x0, xref, tol=0.0, max_iter=k, upper=UPPERS[upper])
        o = om.solve(ops, om.state_x0(ops, x0), xref, upper=upper, tol=0.0, max_iter=k)
        assert rc == nm.NMPC_E_NOCONV and info["iters"] == k
        compare(ops, o, X, U, L, REL)
        assert abs(info["r_scaled"] - o["r_scaled"]) <= 1e-9 * o["r_scaled"]
        assert abs(info["r_paper"] - o["r_paper"]) <= 1e-9 * o["r_paper"]
        if P.tau > 0:
            assert np.all(U > P.u_lo) and np.all(U < P.u_hi)


def test_plate_fraction_to_the_boundary_cuts_the_steps(nm):
    """From a start near the box's upper bound with a weak barrier the passes
    would leave the box: the rule cuts them and the GPU follows the oracle."""
    P = small_plate(tau=0.5)
    ops = om.Ops(P)
    x0, xref = instance(P, 5)
    free = om.solve(ops, om.state_x0(ops, x0), xref, upper="sgs", tol=1e-6, max_iter=400)
    U0 = np.clip(free["U"] + 60.0, P.u_lo + 5, P.u_hi - 1.0)
    X0 = om.to_grid(ops, free["X"], U0)
    L0 = om.to_grid(ops, free["LAM"])
    start = (X0, U0, L0)
    ostart = (free["X"], U0, free["LAM"])
    for upper in ("jacobi", "sgs"):
        S = ostart
        cut = False
        for _ in range(2):
            S2 = om.iterate(ops, om.state_x0(ops, x0), xref, S, upper)
            full = om.sweep(ops, om.state_x0(ops, x0), xref, S, S[1], 0 if upper == "jacobi" else -1)
            cut |= om.alpha_max(P, S[1], S[1] - full[1]) < 1.0
            S = S2
        assert cut
        for k in (1, 2, 4):
            rc, X, U, L, info = gpu_solve(nm, P, x0, xref, warm=start, tol=0.0, max_iter=k,
                                          upper=UPPERS[upper])
            o = om.solve(ops, om.state_x0(ops, x0), xref, start=ostart, upper=upper, tol=0.0,
                         max_iter=k)
            compare(ops, o, X, U, L, REL)
            assert np.all(U > P.u_lo) and np.all(U < P.u_hi)


@pytest.mark.parametrize("upper", ["sgs", "jacobi"])
def test_paper_plate_configuration_converges_like_the_oracle(nm, upper):
    """13 x 13, N = 20, tau = 100, gamma = 0.5, two sweeps and two Schur steps,
    stopping at the paper's |K|_inf < 1: same iteration count as the oracle
    (+-1), and the returned trajectory equals the oracle's iterate of that
    index; the inputs stay inside [T_a, T_a + 400]."""
    P = make_plate_problem()
    ops = om.Ops(P)
    x0, xref = make_plate_instance(P, 0, "slope")
    rc, X, U, L, info = gpu_solve(nm, P, x0, xref, tol=1.0, max_iter=500, upper=UPPERS[upper],
                                  residual=nm.NMPC_RES_PAPER)
    o = om.solve(ops, om.state_x0(ops, x0), xref, upper=upper, tol=1.0, residual_kind="paper",
                 max_iter=500)
    assert rc == nm.NMPC_OK and o["status"] == "converged" and info["r_paper"] < 1.0
    assert abs(info["iters"] - o["iters"]) <= 1
    if info["iters"] != o["iters"]:
        o = om.solve(ops, om.state_x0(ops, x0), xref, upper=upper, tol=0.0, max_iter=info["iters"])
    compare(ops, o, X, U, L, 1e-9)
    assert np.all(U > P.u_lo) and np.all(U < P.u_hi)
    print(f"plate {upper}: {info['iters']} iterations, |K|_inf {info['r_paper']:.3f}, "
          f"inputs {U.min():.1f}..{U.max():.1f} K")


@pytest.mark.parametrize("case", ["plate7", "wave6", "heat9x6"])
def test_model_converged_solution_matches_the_oracle(nm, case):
    P = CASES[case]()
    ops = om.Ops(P)
    x0, xref = instance(P, 7)
    tol = 1e-8 if P.model == "plate" else 1e-9
    rc, X, U, L, info = gpu_solve(nm, P, x0, xref, tol=tol, max_iter=5000, upper=3)
    o = om.solve(ops, om.state_x0(ops, x0), xref, upper="sgs", tol=tol, max_iter=5000)
    assert rc == nm.NMPC_OK and o["status"] == "converged"
    assert abs(info["iters"] - o["iters"]) <= 1
    if info["iters"] != o["iters"]:
        o = om.solve(ops, om.state_x0(ops, x0), xref, upper="sgs", tol=0.0, max_iter=info["iters"])
    compare(ops, o, X, U, L, 1e-9)
    rs, _ = om.residual(ops, om.state_x0(ops, x0), xref,
                        X[:, ops.state] if P.model == "plate" else X, U,
                        L[:, ops.state] if P.model == "plate" else L)
    assert rs <= tol


def test_model_residual_batch_matches_oracle(nm):
    import torch
    for P in (small_plate(), make_wave_problem(ns=5, N=3), dense_heat()):
        ops = om.Ops(P)
        x0, xref = instance(P, 1)
        rng = np.random.default_rng(2)
        o = om.solve(ops, om.state_x0(ops, x0), xref, upper="sgs", tol=0.0, max_iter=2)
        X = om.to_grid(ops, o["X"] * (1 + 1e-3 * rng.normal(size=o["X"].shape)), o["U"])
        L = om.to_grid(ops, o["LAM"] * (1 + 1e-2 * rng.normal(size=o["LAM"].shape)))
        U = o["U"]
        s = nm.ModelSolver(P)
        t = lambda a: torch.tensor(np.asarray(a)[None], device="cuda")
        rs, rp = s.residual_batch(t(x0), t(xref), t(X), t(U), t(L))
        s.close()
        Xc = X[:, ops.state] if P.model == "plate" else X
        Lc = L[:, ops.state] if P.model == "plate" else L
        ors, orp = om.residual(ops, om.state_x0(ops, x0), xref, Xc, U, Lc)
        assert abs(rs[0] - ors) <= 1e-11 * ors and abs(rp[0] - orp) <= 1e-11 * orp


def test_model_batch_statuses_and_warm_start(nm):
    """A batch: instance 0 cold, the converged solution given back returns at
    k = 0 bit for bit (a model without a box: inside one the given inputs are
    first moved 0.5 % of its width away from the bounds), a NaN start gives
    NMPC_E_NONFINITE; batch results equal single solves."""
    import torch
    P = dense_heat()
    ops = om.Ops(P)
    (x0a, xra), (x0b, xrb) = instance(P, 1), instance(P, 2)
    rc, X, U, L, info = gpu_solve(nm, P, x0a, xra, tol=1e-8, max_iter=3000, upper=3)
    assert rc == nm.NMPC_OK
    rc2, X2, U2, L2, info2 = gpu_solve(nm, P, x0a, xra, warm=(X, U, L), tol=1e-8, max_iter=3000,
                                       upper=3)
    assert rc2 == nm.NMPC_OK and info2["iters"] == 0
    np.testing.assert_array_equal(U2, U)
    bad = U.copy(); bad[1, 2] = np.nan
    rc3, *_, info3 = gpu_solve(nm, P, x0a, xra, warm=(X, bad, L), tol=1e-8, max_iter=30, upper=3)
    assert rc3 == nm.NMPC_E_NONFINITE and info3["status"] == nm.NMPC_E_NONFINITE
    s = nm.ModelSolver(P, max_batch=3, tol=1e-8, max_iter=3000, upper=3)
    t = lambda a: torch.tensor(np.asarray(a), device="cuda")
    rcb, Xb, Ub, Lb, infb = s.solve_batch(t(np.stack([x0a, x0b, x0a])), t(np.stack([xra, xrb, xra])))
    assert rcb == nm.NMPC_OK
    np.testing.assert_array_equal(Ub[0].cpu().numpy(), U)
    np.testing.assert_array_equal(Ub[2].cpu().numpy(), U)
    rcs, Xs, Us, Ls, infs = gpu_solve(nm, P, x0b, xrb, tol=1e-8, max_iter=3000, upper=3)
    np.testing.assert_array_equal(Ub[1].cpu().numpy(), Us)
    assert [i["iters"] for i in infb] == [info["iters"], infs["iters"], info["iters"]]


def test_model_rejects_what_it_does_not_cover(nm):
    P = small_plate()
    with pytest.raises(nm.NmpcError) as e:
        nm.ModelSolver(P, precision=nm.NMPC_FP32_SWEEP)
    assert e.value.code == nm.NMPC_E_UNSUPPORTED
    with pytest.raises(nm.NmpcError) as e:
        nm.ModelSolver(P.with_(act=[16, 16, 30, 32]))
    assert e.value.code == nm.NMPC_E_ARG
    with pytest.raises(nm.NmpcError) as e:
        nm.ModelSolver(P.with_(u_cold=P.u_lo))
    assert e.value.code == nm.NMPC_E_ARG
    with pytest.raises(nm.NmpcError) as e:
        nm.ModelSolver(make_wave_problem(ns=80, N=4))
    assert e.value.code == nm.NMPC_E_UNSUPPORTED


LARGE = {
    # node counts past 1024 and 2048 take the engine's 4- and 8-node-per-thread
    # kernels; 64 x 64 is its largest grid
    "heat64x64": (lambda: dense_heat(nsx=64, nsy=64, N=2, m=4), "jacobi"),
    "heat40x40": (lambda: dense_heat(nsx=40, nsy=40, N=2, m=4), "sgs"),
    "plate45": (lambda: make_plate_problem(ns=45, N=2), "sgs"),
    "wave40": (lambda: make_wave_problem(ns=40, N=2), "jacobi"),
}


@pytest.mark.parametrize("case", list(LARGE))
def test_model_largest_grids_match_oracle(nm, case):
    """The engine's multi-node-per-thread kernels (1,600 .. 4,096 nodes, the
    largest grid it takes) against the oracle at equal k."""
    make, upper = LARGE[case]
    P = make()
    ops = om.Ops(P)
    x0, xref = instance(P, 3)
    for k in (1, 2):
        rc, X, U, L, info = gpu_solve(nm, P, x0, xref, tol=0.0, max_iter=k, upper=UPPERS[upper])
        o = om.solve(ops, om.state_x0(ops, x0), xref, upper=upper, tol=0.0, max_iter=k)
        assert rc == nm.NMPC_E_NOCONV and info["iters"] == k
        compare(ops, o, X, U, L, REL)
        assert abs(info["r_scaled"] - o["r_scaled"]) <= 1e-9 * o["r_scaled"]


def test_model_grid_beyond_the_engine_is_refused(nm):
    with pytest.raises(nm.NmpcError) as e:
        nm.ModelSolver(dense_heat(nsx=65, nsy=64, N=2, m=4))
    assert e.value.code == nm.NMPC_E_UNSUPPORTED


def test_model_batch_count_outside_the_handle_is_refused(nm):
    import torch
    P = small_plate()
    s = nm.ModelSolver(P, max_batch=2)
    for count in (0, 3):
        x0 = torch.zeros((count, s.nx), dtype=torch.float64, device="cuda")
        xr = torch.zeros((count, P.nodes), dtype=torch.float64, device="cuda")
        with pytest.raises(nm.NmpcError) as e:
            s.solve_batch(x0, xr)
        assert e.value.code == nm.NMPC_E_ARG
    s.close()
