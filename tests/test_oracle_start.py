"""Pins of the oracle's input-built start (``oracle/start.py``).

The start's states must be the backward-Euler trajectory of eq. nlp (checked
against the dense Newton simulation), its state and costate rows of the KKT
system of Sec. 3.2 must vanish (checked with the C oracle's KKT evaluation,
which shares no code with the sparse builder), and the exact optimum must be
reproduced from its own inputs (all KKT rows vanish there, and the start is
unique given u).
"""
import numpy as np
import pytest

from nmpc_inputs import make_instance, make_problem

import oracle
from oracle import dense
from oracle.start import input_start


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_states_match_the_dense_simulation():
    P = make_problem("c0")
    x0, xref = make_instance(P, 2)
    U = np.random.default_rng(5).normal(0.0, 2.0, (P.N, P.m))
    X, _, _ = input_start(P, x0, xref, U)
    assert _rel(X, dense.simulate_implicit(P, x0, U)) <= 1e-12


@pytest.mark.parametrize("case", ["c0", "grid"])
@pytest.mark.parametrize("per_stage", [False, True])
def test_state_and_costate_rows_vanish(case, per_stage):
    P = make_problem("c0") if case == "c0" else make_problem("grid", ns=12, N=6, lattice=2)
    x0, xref = make_instance(P, 3)
    xr = np.stack([xref * (1.0 + 0.3 * i / P.N) for i in range(P.N)]) if per_stage else xref
    U = np.random.default_rng(6).normal(0.0, 1.0, (P.N, P.m))
    X, Uo, LAM = input_start(P, x0, xr, U)
    KX, KU, KL = oracle.kkt(P, x0, xr, X, Uo, LAM)
    assert np.abs(KX).max() <= 1e-13
    assert np.abs(KL).max() <= 1e-13 * max(1.0, np.abs(LAM).max())
    assert np.abs(KU).max() > 1e-6   # the input rows are not solved


def test_the_optimum_is_reproduced_from_its_inputs():
    P = make_problem("c0")
    x0, xref = make_instance(P, 4)
    ex = oracle.solve(P, x0, xref, tol=1e-13, max_iter=50000)
    assert ex["status"] == "converged"
    X, U, LAM = input_start(P, x0, xref, ex["U"])
    assert _rel(X, ex["X"]) <= 1e-11 and _rel(LAM, ex["LAM"]) <= 1e-9
