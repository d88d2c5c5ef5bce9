"""The oracle's own float64 error sits far below every parity tolerance.

Parity asserts positions within 1e-5 (relative) and impulses within 1e-4 (relative, in
converged mode), and contact decisions bit for bit from float64 predicates.  At the first
contact frame of the 5^3-node cube drop, each oracle result is checked against its own
defining equation (oracle/fp64_errors.py): backward errors of the global, Delassus and
Schur solves at the level of float64 rounding, and forward-error estimates (one step of
iterative refinement) at least 1e6 times below the tolerance they serve.
"""
import pytest

from oracle import fp64_errors


@pytest.fixture(scope="module")
def table():
    return fp64_errors.cube_case(0)


def test_backward_errors_are_rounding_level(table):
    for k in ("global_backward", "delassus_backward", "schur_backward"):
        assert table[k] <= 64 * fp64_errors.EPS64, (k, table[k])


def test_forward_errors_far_below_tolerances(table):
    assert table["contacts"] > 0
    assert table["global_refine_rel"] <= 1e-11          # positions: 1e-5
    assert table["positions_refine_rel"] <= 1e-11       # positions: 1e-5
    assert table["schur_refine_rel"] <= 1e-10           # impulses: 1e-4
    assert table["schur_cond2"] * fp64_errors.EPS64 <= 1e-10


def test_residual_evaluation_error_below_threshold(table):
    # the NCP threshold is 1e-6 m; its float64 evaluation error is ~1e-19 m here
    assert table["ncp_eval_bound"] <= 1e-12
