"""Full-domain solves with asymmetric bottoms (Section 3.1 with y_1 = -y_M; the
two offset bumps of Section 5.3) against the oracle's converged solution."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from paper_1709_08803_amd import workloads as W
from oracle import jfnk as OJ
from oracle import linear as Lin
from oracle import residual as R

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bim():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_1709_08803_amd import bim as B
    B.lib()
    return B


def offset_bumps(N=41, M=41, F=0.6):
    """The two-bump layout of the paper's asymmetric case -- bumps at (10, 10) and
    (0, -10) on x in [-7, 53], y in [-30, 30] -- scaled by 0.4 onto a small full
    mesh: bumps of height 0.2 at (4, 4) and (0, -4), x in [-7, 17], y in [-12, 12]."""
    d = 0.8 * math.sqrt(2.0)
    return W.make_problem(N, M, -7.0, 17.0, -12.0, 12.0, F,
                          [W.Bump(0.2, d, d, cx=4.0, cy=4.0), W.Bump(0.2, d, d, cx=0.0, cy=-4.0)],
                          half_domain=False, name=f"offset-bumps-{N}x{M}")


@pytest.fixture(scope="module")
def oracle_solution():
    p = offset_bumps()
    J = Lin.jacobian(p)
    u = W.uniform_stream(p) - np.linalg.solve(J, Lin.forcing(p))
    lu = sla.lu_factor(Lin.banded(p, J, Lin.band_halfwidth(p.M)))

    class Pre:
        def apply(self, r):
            return sla.lu_solve(lu, r)
    res = OJ.newton_krylov(p, u, precond=Pre(), ftol=1e-12)
    assert res.converged
    return p, res.u


@pytest.mark.parametrize("prec,storage,tol", [("fp64", "fp64", 1e-9), ("fp32c", "fp32", 1e-8)])
def test_full_domain_solve_matches_oracle(bim, oracle_solution, prec, storage, tol):
    p, uref = oracle_solution
    dp = bim.DeviceProblem(p)
    P = bim.Preconditioner(dp, storage=storage)
    u = bim.linear_start(dp, P, prec=prec, rtol=1e-4 if prec == "fp32c" else 0.0)
    rep = bim.solve(dp, u, P, ftol=1e-11, inner_prec=prec, precond_storage=storage)
    P.close()
    uu = u.cpu().numpy()
    a, b = R.reconstruct(p, uu), R.reconstruct(p, uref)
    dz = float(np.abs(a.zeta - b.zeta).max())
    dphi = float(np.abs(a.phi - b.phi).max())
    print(f"{p.name} {prec}: status {rep['status']} Newton {rep['newton_iters']} GMRES {rep['gmres_iters']} "
          f"max|dzeta| {dz:.2e} max|dphi| {dphi:.2e}")
    assert rep["status"] == 0
    assert dz <= tol and dphi <= tol
    # the asymmetric layout gives an asymmetric surface
    assert np.abs(a.zeta - a.zeta[::-1]).max() > 1e-3
    assert np.abs(R.residual(p, uu)).max() <= 1e-10
