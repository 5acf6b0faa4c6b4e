"""The stored 181 x 61 oracle solutions are roots of the oracle's residual.

They are written by tests/golden/make_working_solutions.py, which calls only
the oracle; this check re-evaluates F at the stored u (Section 3.1) so that a
stale or corrupted file cannot pass as a reference.
"""
import os

import numpy as np
import pytest

from oracle import residual as R
from paper_1709_08803_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("froude", [1.4])
def test_stored_solution_is_a_root_of_the_oracle_residual(froude):
    d = np.load(os.path.join(GOLDEN, f"working_181x61_F{froude}.npz"))
    p = W.working(froude)
    u = d["u"]
    assert u.shape == (p.n_unknowns,)
    F = R.residual(p, u)
    assert np.abs(F).max() <= float(d["ftol"])
    # a nontrivial wave field, below the limiting crest height F^2 / 2 (Section 4)
    zeta = R.reconstruct(p, u).zeta
    assert 0.01 < np.abs(zeta).max() < froude ** 2 / 2
