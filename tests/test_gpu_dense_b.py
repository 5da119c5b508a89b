"""Dense input matrix (nmpc_problem.b_kind = NMPC_B_DENSE) through nmpc_create:
the problem runs on the model engine's heat model; its iterates equal the C
oracle's (which always works with the dense B) at equal k, and a dense B that
equals a Kronecker lattice gives the Kronecker path's results."""
import numpy as np
import pytest

from nmpc_inputs import make_instance, make_problem

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2004_02484_amd as m
    return m


def rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


def random_dense(nsx=20, nsy=16, m=5, N=6, seed=3):
    """A non-separable dense B (each column a sum of two random bumps)."""
    P = make_problem("grid", ns=nsx, N=N, lattice=2)
    rng = np.random.default_rng(seed)
    ys, xs = np.meshgrid((np.arange(nsy) + 1.0) / (nsy + 1), (np.arange(nsx) + 1.0) / (nsx + 1),
                         indexing="ij")
    B = np.zeros((nsx * nsy, m))
    for j in range(m):
        for _ in range(2):
            cx, cy, s = rng.uniform(0.2, 0.8), rng.uniform(0.2, 0.8), rng.uniform(0.05, 0.2)
            B[:, j] += np.exp(-((xs - cx) ** 2 + (ys - cy) ** 2) / (2 * s * s)).ravel()
    return P.with_(nsy=nsy, lx=m, ly=1, gx=np.ones((m, nsx)), gy=np.ones((1, nsy)), B=B)


@pytest.mark.parametrize("k", [0, 1, 4])
def test_dense_b_iterates_match_oracle(nm, k):
    P = random_dense()
    x0, xref = make_instance(P.with_(B=None, lx=2, ly=2), 2)
    s = nm.Solver(P, tol=0.0, max_iter=k)
    rc, X, U, L, info = s.solve(x0, xref)
    s.close()
    o = oracle.solve(P, x0, xref, tol=0.0, max_iter=k)
    assert rc == nm.NMPC_E_NOCONV and info["iters"] == k
    assert rel(X, o["X"]) <= 1e-10
    if k > 0:
        assert rel(U, o["U"]) <= 1e-10 and rel(L, o["LAM"]) <= 1e-10
    assert abs(info["r_scaled"] - o["r_scaled"]) <= 1e-9 * o["r_scaled"]


@pytest.mark.parametrize("upper", [0, 3])
def test_dense_b_converged_equals_oracle(nm, upper):
    P = random_dense(N=5)
    x0, xref = make_instance(P.with_(B=None, lx=2, ly=2), 4)
    name = "jacobi" if upper == 0 else "sgs"
    s = nm.Solver(P, tol=1e-9, max_iter=20000, upper=upper)
    rc, X, U, L, info = s.solve(x0, xref)
    o = oracle.solve(P, x0, xref, tol=1e-9, max_iter=20000, upper=name)
    assert rc == nm.NMPC_OK and o["status"] == "converged"
    assert abs(info["iters"] - o["iters"]) <= 1
    if info["iters"] != o["iters"]:
        o = oracle.solve(P, x0, xref, tol=0.0, max_iter=info["iters"], upper=name)
    assert rel(U, o["U"]) <= 1e-9 and rel(X, o["X"]) <= 1e-9
    # the converged solution given back returns at k = 0
    rc, X2, U2, L2, info2 = s.solve(x0, xref, warm=(X, U, L))
    assert rc == nm.NMPC_OK and info2["iters"] == 0
    np.testing.assert_array_equal(U2, U)


def test_dense_b_equal_to_the_lattice_matches_the_kronecker_path(nm):
    import torch
    P = make_problem("grid", ns=24, N=5, lattice=2)
    Pd = P.with_(B=P.dense_B())
    x0s = []
    xrs = []
    for sd in (5, 6):
        a, b = make_instance(P, sd)
        x0s.append(a)
        xrs.append(b)
    t = lambda a: torch.tensor(np.stack(a), device="cuda")
    runs = []
    for Q in (P, Pd):
        s = nm.Solver(Q, max_batch=2, tol=0.0, max_iter=6)
        rc, X, U, L, infos = s.solve_batch(t(x0s), t(xrs))
        runs.append((X.cpu().numpy(), U.cpu().numpy(), L.cpu().numpy()))
        s.close()
    for a, b in zip(*runs):
        assert rel(b, a) <= 1e-11


def test_dense_b_1d_with_input_box(nm):
    P = make_problem("c0")
    free = oracle.solve(P, *make_instance(P, 3), tol=1e-10, max_iter=20000)
    umax = np.abs(free["U"]).max()
    Pd = P.with_(B=P.dense_B(), tau=1e-3 * P.r * umax, u_lo=-0.5 * umax, u_hi=0.5 * umax)
    x0, xref = make_instance(P, 3)
    for k in (1, 5):
        s = nm.Solver(Pd, tol=0.0, max_iter=k)
        rc, X, U, L, info = s.solve(x0, xref)
        o = oracle.solve(Pd, x0, xref, tol=0.0, max_iter=k)
        assert rel(U, o["U"]) <= 1e-10 and rel(X, o["X"]) <= 1e-10 and rel(L, o["LAM"]) <= 1e-10
        assert np.all(U > Pd.u_lo) and np.all(U < Pd.u_hi)


def test_dense_b_unsupported_calls(nm):
    import torch
    P = random_dense()
    with pytest.raises(nm.NmpcError) as e:
        nm.Solver(P, precision=nm.NMPC_FP32_SWEEP)
    assert e.value.code == nm.NMPC_E_UNSUPPORTED
    s = nm.Solver(P)
    x0, xref = make_instance(P.with_(B=None, lx=2, ly=2), 1)
    t = lambda a: torch.tensor(a[None], device="cuda")
    with pytest.raises(nm.NmpcError) as e:
        s.autotune(t(x0), t(xref))
    assert e.value.code == nm.NMPC_E_UNSUPPORTED
    with pytest.raises(nm.NmpcError) as e:
        s.solve(x0, xref, warm=(None, np.zeros((P.N, P.m)), None))
    assert e.value.code == nm.NMPC_E_UNSUPPORTED
