"""GPU tests of starts built from an input trajectory and of the fallback.

A start built from u must satisfy the state rows (backward-Euler model) and
the costate rows (adjoint recursion) of the KKT conditions, checked with the
oracle's KKT evaluation; only the input rows remain. From such a start the
iteration reaches the same solution as from the cold start.
"""
import numpy as np
import pytest

from nmpc_inputs import make_instance, make_problem

import oracle
from oracle.start import input_start

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2004_02484_amd as nm
    return nm


@pytest.fixture(scope="module")
def c1_case():
    P = make_problem("c1")
    x0, xref = make_instance(P, 21)
    ex = oracle.solve(P, x0, xref, tol=1e-11, max_iter=20000)
    assert ex["status"] == "converged"
    return P, x0, xref, ex


@pytest.mark.parametrize("name", ["c0", "c1"])
def test_input_built_start_satisfies_state_and_costate_rows(nm, name, c1_case):
    if name == "c1":
        P, x0, xref, ex = c1_case
    else:
        P = make_problem("c0")
        x0, xref = make_instance(P, 4)
        ex = oracle.solve(P, x0, xref, tol=1e-11, max_iter=20000)
    rng = np.random.default_rng(3)
    U = ex["U"] * (1.0 + 1e-2 * rng.standard_normal(ex["U"].shape))
    s = nm.Solver(P, tol=0.0, max_iter=0, warm_sweeps=40)
    rc, X, Uo, L, info = s.solve(x0, xref, warm=(None, U, None))
    assert rc == nm.NMPC_E_NOCONV and info["iters"] == 0 and info["start_used"] == 2
    np.testing.assert_array_equal(Uo, U)
    KX, KU, KL = oracle.kkt(P, x0, xref, X, Uo, L)
    assert np.abs(KX).max() <= 1e-12
    assert np.abs(KL).max() / P.h <= 1e-10
    # the input rows carry the perturbation: |K^u|/(h r) ~ |u - u*|
    assert np.abs(KU).max() / (P.h * P.r) > 1e-4


def test_input_start_converges_to_the_solution_faster(nm, c1_case):
    P, x0, xref, ex = c1_case
    rng = np.random.default_rng(4)
    U = ex["U"] * (1.0 + 1e-3 * rng.standard_normal(ex["U"].shape))
    s = nm.Solver(P)
    rc_c, Xc, Uc, Lc, info_c = s.solve(x0, xref)
    rc, X, Uw, L, info = s.solve(x0, xref, warm=(None, U, None))
    assert rc == nm.NMPC_OK and rc_c == nm.NMPC_OK
    err = np.abs(Uw - ex["U"]).max() / np.abs(ex["U"]).max()
    print(f"cold {info_c['iters']} iterations, start from u (1e-3 noise) {info['iters']}, "
          f"control rel. error vs exact {err:.2e}")
    assert info["iters"] < info_c["iters"] // 2
    assert err <= 1e-4
    rs, _ = oracle.residual(P, x0, xref, X, Uw, L)
    assert rs <= 1e-6


def test_fallback_keeps_the_better_start(nm, c1_case):
    P, x0, xref, ex = c1_case
    s = nm.Solver(P, fallback=1)
    bad = np.full_like(ex["U"], np.nan)
    rc, X, U, L, info = s.solve(x0, xref, warm=(None, bad, None))
    assert rc == nm.NMPC_OK and info["start_used"] == 0
    huge = np.full_like(ex["U"], 1e6)
    rc, X, U, L, info = s.solve(x0, xref, warm=(None, huge, None))
    assert rc == nm.NMPC_OK and info["start_used"] == 0
    good = ex["U"] * (1 + 1e-4)
    rc, X, U, L, info = s.solve(x0, xref, warm=(None, good, None))
    assert rc == nm.NMPC_OK and info["start_used"] == 2
    rc, X, U, L, info = s.solve(x0, xref, warm=(ex["X"], ex["U"], ex["LAM"]))
    assert rc == nm.NMPC_OK and info["start_used"] == 1 and info["iters"] == 0


def test_batch_input_start_with_fallback(nm, c1_case):
    import torch
    P, x0, xref, ex = c1_case
    B = 3
    X0 = torch.tensor(np.stack([x0] * B), device="cuda")
    XR = torch.tensor(np.stack([xref] * B), device="cuda")
    U = np.stack([ex["U"] * (1 + 1e-3), np.full_like(ex["U"], np.nan), ex["U"]])
    s = nm.Solver(P, max_batch=B, fallback=1)
    rc, X, Uo, L, infos = s.solve_batch(X0, XR, warm=(None, torch.tensor(U, device="cuda"), None))
    assert rc == nm.NMPC_OK
    assert [i["start_used"] for i in infos] == [2, 0, 2]
    for b in range(B):
        err = np.abs(Uo[b].cpu().numpy() - ex["U"]).max() / np.abs(ex["U"]).max()
        assert err <= 1e-4


@pytest.mark.parametrize("name,per_stage", [("c1", False), ("c1", True), ("c0", False),
                                             ("grid40", True)])
def test_fallback_decision_follows_the_start_residuals(nm, c1_case, name, per_stage):
    """The fallback compares the built start's residual (evaluated by the
    library while it builds the start) with the cold start's (stage 0 only
    when one reference serves all stages). Over a range of input scalings the
    choice must be the one the oracle's residuals of the two starts give;
    scalings whose two residuals lie within 25 % of each other are skipped.
    Cases: the 64 x 64 batch grid, 1D, and a 40 x 40 grid whose tiles end in
    a partial one."""
    if name == "c1":
        P, x0, xref, ex = c1_case
    else:
        P = make_problem("c0") if name == "c0" else make_problem("grid", ns=40, N=6, lattice=2)
        x0, xref = make_instance(P, 21)
        ex = oracle.solve(P, x0, xref, tol=1e-11, max_iter=50000)
        assert ex["status"] == "converged"
    xr = np.stack([xref * (1.0 + 0.05 * i / P.N) for i in range(P.N)]) if per_stage else xref
    rs_cold, _ = oracle.residual(P, x0, xr, *oracle.cold_start(P, x0))
    s = nm.Solver(P, fallback=1, tol=0.0, max_iter=0, xref_per_stage=int(per_stage))
    seen = set()
    for c in (0.5, 0.95, 1.0, 1.05, 2.0, 10.0):
        U = c * ex["U"]
        rs_in, _ = oracle.residual(P, x0, xr, *input_start(P, x0, xr, U))
        ratio = rs_in / rs_cold
        if 0.8 < ratio < 1.25:
            continue
        rc, X, Uo, L, info = s.solve(x0, xr, warm=(None, U, None))
        want = 2 if ratio < 1.0 else 0
        print(f"scale {c:g}: oracle residuals built {rs_in:.3e} cold {rs_cold:.3e}, "
              f"start used {info['start_used']}")
        assert rc == nm.NMPC_E_NOCONV and info["start_used"] == want, (c, ratio)
        seen.add(want)
    assert seen == {0, 2}


@pytest.mark.parametrize("sweeps,sweeps_lam,bar", [(14, 0, 1e-6), (24, 0, 1e-11), (10, 14, 3e-4)])
def test_rollout_matches_the_exact_input_start(nm, c1_case, sweeps, sweeps_lam, bar):
    """The start built on the GPU from u (Chebyshev-weighted point-Jacobi
    sweeps per stage; sweeps_lam > 0: that many for the costates) against the
    oracle's start solved to rounding. With the sweep matrices' spectral
    radius mu ~ 0.44 the weights reduce a stage's error by about 2 r^s, r =
    mu / (1 + sqrt(1 - mu^2)) ~ 0.23: ~3e-9 after 14 sweeps, ~8e-7 after 10,
    rounding after 24; the bars allow for the 40 stages passing their errors
    on (the costates inherit the states' error)."""
    P, x0, xref, ex = c1_case
    U = ex["U"] * (1.0 + 1e-2 * np.random.default_rng(8).standard_normal(ex["U"].shape))
    s = nm.Solver(P, tol=0.0, max_iter=0, warm_sweeps=sweeps, warm_sweeps_lambda=sweeps_lam)
    rc, X, Uo, L, info = s.solve(x0, xref, warm=(None, U, None))
    assert info["start_used"] == 2
    Xe, _, Le = input_start(P, x0, xref, U)
    ex_ = np.abs(X - Xe).max() / np.abs(Xe).max()
    el_ = np.abs(L - Le).max() / np.abs(Le).max()
    print(f"{sweeps}/{sweeps_lam} sweeps: state rel. error {ex_:.2e}, costate rel. error {el_:.2e}")
    assert ex_ <= bar and el_ <= bar
