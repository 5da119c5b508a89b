"""GPU parity of ragged batches (instances of several grids and horizons in
one launch per upper iteration) and of the tile autotuners, against the CPU
oracle run instance by instance.

Equal-k comparisons use the FP64 kernels (relative 1e-10, as for the batch
kernel); converged comparisons use the FP32-sweep kernels against the oracle
run to r_scaled <= 1e-11 (control error <= 1e-4) and the zero-residual
invariant recomputed by the oracle on the returned trajectories.
"""
import numpy as np
import pytest

from nmpc_inputs import gaussian_factors, grid_h, make_instance, make_problem, ragged_specs

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


def cls2d(nsx, nsy, N):
    """2D class with the 4 x 4 Gaussian lattice (sigma 0.05), h from the finer axis."""
    P = make_problem("grid", ns=nsx, N=N, lattice=4)
    P = P.with_(nsy=nsy, gx=gaussian_factors(nsx, 4, 0.05), gy=gaussian_factors(nsy, 4, 0.05))
    P.h = grid_h(max(nsx, nsy))
    P.gamma = P.h * P.r
    return P


def dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


# classes with ragged tails: widths below, at and above a 16-lane row, heights
# that leave rows and waves empty, horizons from 1 up
SMALL = [(16, 16, 4), (33, 17, 3), (20, 48, 5), (64, 9, 2), (7, 7, 1), (48, 40, 3)]


def small_batch(order):
    classes = [cls2d(*c) for c in SMALL]
    inst = []
    for t, c in enumerate(order):
        x0, xr = make_instance(classes[c], 100 + t)
        inst.append((c, x0, xr))
    return classes, inst


@pytest.mark.parametrize("k", [1, 4])
def test_ragged_iterates_match_oracle(nm, k):
    order = [0, 1, 2, 3, 4, 5, 1, 0, 5]
    classes, inst = small_batch(order)
    rs = nm.RaggedSolver(classes, max_instances=16, tol=0.0, max_iter=k)
    rc, res, infos, _ = rs.solve(order, [dev(x) for _, x, _ in inst], [dev(r) for _, _, r in inst])
    assert rc == nm.NMPC_E_NOCONV
    for (c, x0, xr), (X, U, L), info in zip(inst, res, infos):
        o = oracle.solve(classes[c], x0, xr, tol=0.0, max_iter=k)
        assert info["iters"] == k and info["status"] == nm.NMPC_E_NOCONV
        assert rel(X.cpu().numpy(), o["X"]) <= REL
        assert rel(U.cpu().numpy(), o["U"]) <= REL
        assert rel(L.cpu().numpy(), o["LAM"]) <= REL
        assert abs(info["r_scaled"] - o["r_scaled"]) <= 1e-9 * o["r_scaled"]
    rs.close()


def test_ragged_equals_batch_solver_per_class(nm):
    """Each instance of a ragged batch gets the iterate the one-problem batch
    solver computes for it (equal k, relative 1e-11)."""
    order = [2, 0, 2, 5]
    classes, inst = small_batch(order)
    rs = nm.RaggedSolver(classes, max_instances=8, tol=0.0, max_iter=6)
    rc, res, infos, _ = rs.solve(order, [dev(x) for _, x, _ in inst], [dev(r) for _, _, r in inst])
    for (c, x0, xr), (X, U, L) in zip(inst, res):
        s = nm.Solver(classes[c], tol=0.0, max_iter=6)
        _, Xb, Ub, Lb, _ = s.solve(x0, xr)
        s.close()
        assert rel(U.cpu().numpy(), Ub) <= 1e-11
        assert rel(X.cpu().numpy(), Xb) <= 1e-11
        assert rel(L.cpu().numpy(), Lb) <= 1e-11


def test_ragged_fp32_converges_to_the_exact_solution(nm):
    order = [0, 1, 2, 3, 5]
    classes, inst = small_batch(order)
    rs = nm.RaggedSolver(classes, max_instances=8, tol=1e-6, max_iter=20000,
                         precision=nm.NMPC_FP32_SWEEP)
    rs.timing_enable(True)
    rc, res, infos, _ = rs.solve(order, [dev(x) for _, x, _ in inst], [dev(r) for _, _, r in inst])
    tm = rs.timing_read()
    assert rc == nm.NMPC_OK
    # every instance visits its stages once per iteration, once more for the
    # FP64 correction of the accepted FP32 iterate, and once for the
    # evaluation-only check of the corrected one, counted apart
    Ns = [classes[c].N for c in order]
    assert tm["units"] == sum((i["iters"] + 1) * n for i, n in zip(infos, Ns))
    assert tm["eval_units"] == sum(Ns)
    for (c, x0, xr), (X, U, L), info in zip(inst, res, infos):
        ex = oracle.solve(classes[c], x0, xr, tol=1e-11, max_iter=50000)
        assert ex["status"] == "converged"
        err = rel(U.cpu().numpy(), ex["U"])
        assert err <= 1e-4, (c, err)
        r_s, _ = oracle.residual(classes[c], x0, xr, X.cpu().numpy(), U.cpu().numpy(),
                                 L.cpu().numpy())
        assert r_s <= 1e-6 and info["r_scaled"] <= 1e-6
        assert 0.0 < info["err_vs_fp64"] <= 1e-4


def test_ragged_warm_start_given(nm):
    """A given (x, u, lambda) start that already satisfies the test returns at
    iteration 0 with exactly that trajectory."""
    import torch
    order = [0, 3]
    classes, inst = small_batch(order)
    exs = [oracle.solve(classes[c], x0, xr, tol=1e-11, max_iter=50000) for c, x0, xr in inst]
    rs = nm.RaggedSolver(classes, max_instances=4, tol=1e-6)
    warm = (torch.cat([dev(e["X"]).reshape(-1) for e in exs]),
            torch.cat([dev(e["U"]).reshape(-1) for e in exs]),
            torch.cat([dev(e["LAM"]).reshape(-1) for e in exs]))
    rc, res, infos, _ = rs.solve(order, [dev(x) for _, x, _ in inst], [dev(r) for _, _, r in inst],
                                 warm=warm)
    assert rc == nm.NMPC_OK
    for e, (X, U, L), info in zip(exs, res, infos):
        assert info["iters"] == 0
        np.testing.assert_array_equal(U.cpu().numpy(), e["U"])
        np.testing.assert_array_equal(X.cpu().numpy(), e["X"])


def test_ragged_autotune_keeps_the_results(nm):
    order = [0, 2, 5, 1]
    classes, inst = small_batch(order)
    x0 = [dev(x) for _, x, _ in inst]
    xr = [dev(r) for _, _, r in inst]
    rs = nm.RaggedSolver(classes, max_instances=8, tol=0.0, max_iter=5)
    w0 = rs.config(order)
    rc, res0, _, _ = rs.solve(order, x0, xr)
    U0 = [u.cpu().numpy() for _, u, _ in res0]
    w = rs.autotune(order, x0, xr, iters=4)
    assert w in (8, 12, 16) and rs.config(order) == w
    rc, res1, _, _ = rs.solve(order, x0, xr)
    for a, (_, u, _) in zip(U0, res1):
        assert rel(u.cpu().numpy(), a) <= 1e-10
    print(f"default {w0} waves, autotuned {w} waves")


def test_batch_autotune_keeps_the_results(nm):
    import torch
    P = make_problem("grid", ns=48, N=6, lattice=4)
    xs = [make_instance(P, s) for s in range(3)]
    X0 = dev(np.stack([x for x, _ in xs]))
    XR = dev(np.stack([r for _, r in xs]))
    s = nm.Solver(P, max_batch=3, tol=0.0, max_iter=5, precision=nm.NMPC_FP32_SWEEP)
    _, _, U0, _, _ = s.solve_batch(X0, XR)
    U0 = U0.cpu().numpy()
    tr = s.autotune(X0, XR, iters=4)
    assert tr >= 1
    _, _, U1, _, _ = s.solve_batch(X0, XR)
    # another tile height sums B^T in another order (FP32 lower layer)
    assert rel(U1.cpu().numpy(), U0) <= 1e-5
    print(f"tile rows chosen: {tr}")


def test_ragged_full_size_batch(nm):
    """512 instances of {32, 48, 64, 96}^2 grids and N in {20, 40, 60} in one
    launch per iteration (FP32 sweeps): every instance converges and the
    oracle's residual of sampled returned trajectories is within the test."""
    import torch
    specs = ragged_specs(512, seed=0)
    keys = sorted({(ns, N) for ns, N, _ in specs})
    classes = [make_problem("grid", ns=ns, N=N, lattice=4) for ns, N in keys]
    order = [keys.index((ns, N)) for ns, N, _ in specs]
    inst = [make_instance(classes[c], sd) for c, (_, _, sd) in zip(order, specs)]
    rs = nm.RaggedSolver(classes, max_instances=512, tol=1e-6, max_iter=5000,
                         precision=nm.NMPC_FP32_SWEEP)
    x0 = torch.cat([dev(x) for x, _ in inst])
    xr = torch.cat([dev(r) for _, r in inst])
    print(f"classes {keys}, default {rs.config(order)} waves", flush=True)
    rc, res, infos, _ = rs.solve(order, x0, xr)
    assert rc == nm.NMPC_OK
    it = np.array([i["iters"] for i in infos])
    print(f"iterations {it.min()}..{it.max()}", flush=True)
    for b in np.random.default_rng(0).choice(512, 6, replace=False):
        c = order[b]
        X, U, L = (t.cpu().numpy() for t in res[b])
        r_s, _ = oracle.residual(classes[c], inst[b][0], inst[b][1], X, U, L)
        assert r_s <= 1e-6, (b, keys[c], r_s)


def test_ragged_input_box_matches_oracle(nm):
    """Ragged batch whose classes carry input boxes (some classes none): at
    equal k every instance equals the oracle's Jacobi iterate with the barrier
    and the fraction-to-the-boundary rule (alpha global over the instance's
    stages); converged in FP32 sweeps, the inputs meet the oracle's exact
    solution inside each box."""
    order = [0, 1, 2, 5, 0, 3]
    classes, inst = small_batch(order)
    boxed = []
    for c, P in enumerate(classes):
        if c in (3,):             # no box for this class
            boxed.append(P)
            continue
        x0, xr = make_instance(P, 7)   # a box at 0.6 of one instance's input range
        free = oracle.solve(P, x0, xr, tol=1e-8, max_iter=20000)
        umax = np.abs(free["U"]).max()
        boxed.append(P.with_(tau=1e-4 * P.r * umax, u_lo=-0.6 * umax, u_hi=0.6 * umax))
    for k in (2, 6):
        rs = nm.RaggedSolver(boxed, max_instances=8, tol=0.0, max_iter=k)
        rc, res, infos, _ = rs.solve(order, [dev(x) for _, x, _ in inst],
                                     [dev(r) for _, _, r in inst])
        rs.close()
        for (c, x0, xr), (X, U, L), info in zip(inst, res, infos):
            o = oracle.solve(boxed[c], x0, xr, tol=0.0, max_iter=k)
            assert info["iters"] == k
            assert rel(U.cpu().numpy(), o["U"]) <= REL, (c, k, rel(U.cpu().numpy(), o["U"]))
            assert rel(X.cpu().numpy(), o["X"]) <= REL and rel(L.cpu().numpy(), o["LAM"]) <= REL
            if boxed[c].tau > 0:
                Uh = U.cpu().numpy()
                assert np.all(Uh > boxed[c].u_lo) and np.all(Uh < boxed[c].u_hi)
    rs = nm.RaggedSolver(boxed, max_instances=8, tol=1e-7, max_iter=20000,
                         precision=nm.NMPC_FP32_SWEEP)
    rc, res, infos, _ = rs.solve(order, [dev(x) for _, x, _ in inst], [dev(r) for _, _, r in inst])
    assert rc == nm.NMPC_OK
    for (c, x0, xr), (X, U, L), info in zip(inst, res, infos):
        ex = oracle.solve(boxed[c], x0, xr, tol=1e-11, max_iter=50000)
        assert ex["status"] == "converged"
        assert rel(U.cpu().numpy(), ex["U"]) <= 1e-4
