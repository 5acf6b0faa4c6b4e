"""Solves with surface tension (Section 6) against the oracle's converged solution."""
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


def _oracle_solution(p):
    J = Lin.jacobian(p)
    u = W.uniform_stream(p) - np.linalg.solve(J, Lin.forcing(p))
    lu = sla.lu_factor(Lin.banded(p, J, Lin.band_halfwidth(p.M)))

    class Pre:
        def apply(self, r):
            return sla.lu_solve(lu, r)
    res = OJ.newton_krylov(p, u, precond=Pre(), ftol=1e-12)
    assert res.converged
    return res.u


CASES = [
    ("half-31x11-F1.4-tau0.1", lambda tau: W.make_problem(31, 11, -16, 16, 0, 10, 1.4, [W.Bump(0.1, 1.0, 1.0)], tau=tau), 0.1),
    ("full-41x25-F0.6-tau0.05", lambda tau: W.make_problem(41, 25, -8, 16, -8, 8, 0.6,
                                                            [W.Bump(0.15, 1.2, 1.2, cx=1.0, cy=2.0)],
                                                            half_domain=False, tau=tau), 0.05),
]


@pytest.mark.parametrize("name,mk,tau", CASES, ids=[c[0] for c in CASES])
def test_solve_with_surface_tension_matches_oracle(bim, name, mk, tau):
    p = mk(tau)
    uref = _oracle_solution(p)
    u0ref = _oracle_solution(mk(0.0))
    dzt = np.abs(R.reconstruct(p, uref).zeta - R.reconstruct(p, u0ref).zeta).max()
    print(f"{name}: tension changes the oracle's surface by {dzt:.3e}")
    assert dzt > 1e-3
    dp = bim.DeviceProblem(p)
    for prec, storage, tol in (("fp64", "fp64", 1e-9), ("fp32c", "fp32", 1e-8)):
        P = bim.Preconditioner(dp, storage=storage)
        u = bim.linear_start(dp, P, prec=prec, rtol=1e-4 if prec == "fp32c" else 0.0)
        rep = bim.solve(dp, u, P, ftol=1e-11, inner_prec=prec, precond_storage=storage)
        P.close()
        uu = u.cpu().numpy()
        dz = np.abs(R.reconstruct(p, uu).zeta - R.reconstruct(p, uref).zeta).max()
        dphi = np.abs(R.reconstruct(p, uu).phi - R.reconstruct(p, uref).phi).max()
        print(f"  {prec}: status {rep['status']} Newton {rep['newton_iters']} GMRES {rep['gmres_iters']} "
              f"max|dzeta| {dz:.2e} max|dphi| {dphi:.2e}")
        assert rep["status"] == 0 and dz <= tol and dphi <= tol
        assert np.abs(R.residual(p, uu)).max() <= 1e-10


def test_surface_tension_needs_four_rows(bim):
    p = W.make_problem(9, 3, -4, 4, 0, 2, 1.2, [], tau=0.1)
    dp = bim.DeviceProblem(p)
    u = torch.as_tensor(W.uniform_stream(p), device="cuda")
    with pytest.raises(bim.BimError):
        bim.residual(dp, u)
