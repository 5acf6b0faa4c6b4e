"""Pins of the surface-tension extension of the oracle (Section 6: a surface
tension term, tau times the mean curvature, in Bernoulli's equation; it alters
the top-left block of the Jacobian near its diagonal).

They fix the added term against mathematics and linear theory:
  * the discrete curvature converges at second order to the analytic one on
    every row, including the symmetry row and the outer edge;
  * the finite-difference Jacobian of the nonlinear residual with tau at the
    uniform stream equals the linear Jacobian J~(tau);
  * the discrete linear solution with tau converges to the Fourier solution of
    the linear problem with tau, which differs from the tau = 0 one by far more
    than that error (a planted sign error in the term fails the pin).
"""
import numpy as np
import pytest

from paper_1709_08803_amd import workloads as W
from oracle import fourier as Fo
from oracle import linear as Lin
from oracle import residual as R


def _analytic(p, amp=0.3):
    """u for zeta = amp cos(0.5 x) cos(0.35 y) (phi = psi = x) and the exact
    curvature at the collocation points."""
    X, Y = np.meshgrid(p.x(), p.y())
    u = W.uniform_stream(p)
    nb = (p.N + 1) * p.M
    blk = u[:nb].reshape(p.M, p.N + 1)
    blk[:, 0] = amp * np.cos(0.5 * p.x1) * np.cos(0.35 * p.y())
    blk[:, 1:] = -0.5 * amp * np.sin(0.5 * X) * np.cos(0.35 * Y)
    Xs, Ys = R.collocation_points(p)
    c, s_ = np.cos(0.5 * Xs), np.sin(0.5 * Xs)
    cy, sy = np.cos(0.35 * Ys), np.sin(0.35 * Ys)
    zx, zy = -0.5 * amp * s_ * cy, -0.35 * amp * c * sy
    zxx, zyy, zxy = -0.25 * amp * c * cy, -0.1225 * amp * c * cy, 0.175 * amp * s_ * sy
    q = 1 + zx * zx + zy * zy
    K = ((1 + zy * zy) * zxx - 2 * zx * zy * zxy + (1 + zx * zx) * zyy) / q ** 1.5
    return u, K


@pytest.mark.parametrize("half", [True, False])
def test_curvature_converges_second_order_on_every_row(half):
    errs = []
    for h in (0.25, 0.125, 0.0625):
        L = 6.0
        N, M = int(round(2 * L / h)) + 1, int(round((L if half else 2 * L) / h)) + 1
        p = W.make_problem(N, M, -L, L, 0.0 if half else -L, L, 0.8, [], half_domain=half, tau=0.1)
        u, K = _analytic(p)
        nf = R.reconstruct(p, u)
        e = np.abs(R.curvature(p, nf) - K)
        errs.append((e.max(), e[0].max(), e[-1].max()))
        # the residual's dynamic rows carry -tau K on top of the tau = 0 rows
        F1 = R.dynamic_rows(p, nf)
        p0 = W.make_problem(N, M, -L, L, 0.0 if half else -L, L, 0.8, [], half_domain=half)
        assert np.allclose(F1 - R.dynamic_rows(p0, nf), -0.1 * R.curvature(p, nf), atol=1e-14)
    errs = np.array(errs)
    for col in range(3):  # all rows, the first row, the outer edge (one-sided stencil)
        assert errs[1, col] < errs[0, col] / 3.0 and errs[2, col] < errs[1, col] / 3.0, errs[:, col]
    assert errs[2, 0] < 2e-5


def test_fd_jacobian_at_uniform_stream_equals_linear_jacobian_with_tau():
    for half in (True, False):
        p = W.make_problem(9, 6 if half else 7, -4, 4, 0.0 if half else -3.0, 3, 0.8, [], half_domain=half, tau=0.07)
        u0 = W.uniform_stream(p)
        J = Lin.jacobian(p)
        n = u0.size
        Jfd = np.empty((n, n))
        for c in range(n):
            e = np.zeros(n)
            e[c] = 1e-6
            Jfd[:, c] = (R.residual(p, u0 + e) - R.residual(p, u0 - e)) / 2e-6
        assert np.abs(Jfd - J).max() < 1e-7 * max(1.0, np.abs(J).max())
        # and tau does enter: the block (1,1) differs from the tau = 0 one
        p0 = W.make_problem(9, p.M, -4, 4, p.y1, 3, 0.8, [], half_domain=half)
        assert np.abs(J - Lin.jacobian(p0)).max() > 0.3


def _centreline(F, N, M, xlo, xhi, yhi, tau, eps=0.01):
    p = W.make_problem(N, M, xlo, xhi, 0, yhi, F, [W.Bump(eps, 1.0, 1.0)], tau=tau)
    nf = R.reconstruct(p, Lin.linear_start(p))
    return p.x(), nf.zeta[0] / eps


def _fft_centreline(F, xs, tau, eps=0.01, h=0.125, mu=0.01):
    x, y, z = Fo.linear_surface_fft(F, lambda X, Y: eps * np.exp(-(X * X + Y * Y)), 160.0, h, mu, tau=tau)
    return np.interp(xs, x, z[np.argmin(np.abs(y))]) / eps


def _tau_change(tau_discrete, tau_fourier=0.1, F=1.4):
    """The change that tau makes to the centreline of the discrete linear solution
    and of the Fourier solution (x in (-3, 8)), on two meshes of x in [-15, 30],
    y in [0, 15]: (relative error, correlation) per mesh."""
    out = []
    for N, M in ((46, 16), (91, 31)):
        xs, zb = _centreline(F, N, M, -15, 30, 15, tau_discrete)
        _, zb0 = _centreline(F, N, M, -15, 30, 15, 0.0)
        sel = (xs > -3) & (xs < 8)
        df = (_fft_centreline(F, xs, tau_fourier) - _fft_centreline(F, xs, 0.0))[sel]
        db = (zb - zb0)[sel]
        out.append((np.abs(db - df).max() / np.abs(df).max(),
                    float(db @ df / (np.linalg.norm(db) * np.linalg.norm(df)))))
    return out


def test_tau_change_of_discrete_linear_solution_converges_to_fourier():
    # supercritical (F = 1.4), tau = 0.1: the change of the discrete linear
    # solution due to surface tension converges to that of the Fourier solution
    (e1, c1), (e2, c2) = _tau_change(0.1)
    assert e2 < 0.7 * e1 and e2 < 0.45
    assert c2 > 0.9 and c2 > c1


def test_fourier_pin_rejects_the_opposite_sign_of_the_tension_term():
    (e1, c1), (e2, c2) = _tau_change(-0.1)
    assert c2 < 0.0 and e2 > 1.0


def test_preconditioner_with_tension_is_the_gravity_wave_one():
    # P leaves the whole tension term to the Krylov solver: with tau it is P of the same
    # problem without tau.  The reason: keeping -tau zeta*_xx in the slice block of (1,1)
    # makes that lower-triangular block a recurrence with a growing mode.
    mk = lambda tau: W.make_problem(31, 11, -16, 16, 0, 10, 1.4, [W.Bump(0.1, 1.0, 1.0)], tau=tau)
    p, p0 = mk(0.1), mk(0.0)
    hb = Lin.band_halfwidth(p.M)
    P, P0 = Lin.banded(p, Lin.jacobian(p), hb), Lin.banded(p0, Lin.jacobian(p0), hb)
    assert np.abs(P - P0).max() <= 1e-13 * np.abs(P0).max()
    s = p.N + 1
    slice0 = Lin.jacobian(p0)[s:2 * s, s:2 * s]
    with_xx = slice0.copy()
    with_xx[2:, :] -= p.tau * Lin.half_mesh_xx_map(p)[: p.N - 1, : s]
    assert np.abs(np.linalg.inv(slice0)).max() < 1e4
    assert np.abs(np.linalg.inv(with_xx)).max() > 1e15
