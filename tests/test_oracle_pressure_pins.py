"""Pins of the bottom-pressure and force oracle (Section 2.1, eq. (bottompressure)).

They fix it against Bernoulli's equation with the bottom kinematic condition,
the closed form of the undisturbed stream, adaptive 2-D quadrature of the force
integral and the mirror symmetry of a half domain.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_1709_08803_amd import workloads as W
from oracle import pressure as P
from oracle import residual as R


def test_pressure_is_bernoulli_with_bottom_kinematic_condition():
    # Phi_z eliminated by Phi_x beta_x + Phi_y beta_y = Phi_z on z = beta:
    # p must equal 1/2 - |grad Phi|^2 / 2 - beta / F^2 (eq. (finite_dynamic) with a pressure term).
    rng = np.random.default_rng(0)
    for _ in range(20):
        Px, Py, bx, by = rng.uniform(-1.2, 1.2, 4)
        beta = rng.uniform(-1.0, -0.5)
        F = rng.uniform(0.5, 2.0)
        Pz = Px * bx + Py * by
        psx, psy = Px + Pz * bx, Py + Pz * by
        got = P.pressure_from_gradient(beta, bx, by, psx, psy, F)
        ref = 0.5 - 0.5 * (Px * Px + Py * Py + Pz * Pz) - beta / F ** 2
        assert abs(got - ref) < 1e-13


def test_uniform_stream_over_flat_bottom():
    p = W.make_problem(31, 11, -16, 16, 0, 10, 0.7, [])
    pres = P.bottom_pressure(p, W.uniform_stream(p))
    assert np.abs(pres - 1.0 / 0.7 ** 2).max() < 1e-13
    assert np.abs(P.bottom_force(p, pres)).max() < 1e-12


def _analytic(p, bump, a=0.15):
    """u with psi = x + a sin(0.8 x) cos(0.5 (y - c)) and the exact integrand of the force."""
    c = 0.0  # even in y; the full-domain test moves the bump off the axis instead
    X, Y = np.meshgrid(p.x(), p.y())
    u = W.uniform_stream(p)
    nb = (p.N + 1) * p.M
    blk = u[2 * nb:].reshape(p.M, p.N + 1)
    blk[:, 0] = p.x1 + a * math.sin(0.8 * p.x1) * np.cos(0.5 * (p.y() - c))
    blk[:, 1:] = 1.0 + 0.8 * a * np.cos(0.8 * X) * np.cos(0.5 * (Y - c))

    def integrand(y, x, comp):
        g = bump.h * math.exp(-((x - bump.cx) ** 2 / bump.wx ** 2 + (y - bump.cy) ** 2 / bump.wy ** 2))
        beta = -1.0 + g
        bx = -2.0 * (x - bump.cx) / bump.wx ** 2 * g
        by = -2.0 * (y - bump.cy) / bump.wy ** 2 * g
        px = 1.0 + 0.8 * a * math.cos(0.8 * x) * math.cos(0.5 * (y - c))
        py = -0.5 * a * math.sin(0.8 * x) * math.sin(0.5 * (y - c))
        dp = P.pressure_from_gradient(beta, bx, by, px, py, p.froude) - 1.0 / p.froude ** 2
        return dp * (bx, by, -1.0)[comp]
    return u, integrand


@pytest.mark.parametrize("half", [True, False])
def test_force_converges_to_adaptive_quadrature(half):
    L, Ly = 4.0, 3.0
    bump = W.Bump(0.3, 1.2, 1.0, cx=0.3, cy=0.0 if half else 0.7)
    errs = []
    for h in (0.2, 0.1, 0.05):
        N, M = int(round(2 * L / h)) + 1, int(round((Ly if half else 2 * Ly) / h)) + 1
        p = W.make_problem(N, M, -L, L, 0.0 if half else -Ly, Ly, 0.9, [bump], half_domain=half)
        u, f = _analytic(p, bump)
        got = P.bottom_force(p, P.bottom_pressure(p, u))
        ref = np.array([integrate.dblquad(f, -L, L, -Ly, Ly, args=(k,), epsabs=1e-12, epsrel=1e-12)[0]
                        for k in range(3)])
        errs.append(np.abs(got - ref).max())
        assert abs(ref[0]) > 1e-3 and abs(ref[2]) > 1e-2
        if not half:
            assert abs(ref[1]) > 1e-3
    assert errs[1] < errs[0] / 2.8 and errs[2] < errs[1] / 3.3, errs  # second order
    assert errs[2] < 1e-4


def test_half_domain_pressure_equals_mirrored_full_domain():
    bump = W.Bump(0.2, 1.0, 1.0)
    ph = W.make_problem(21, 7, -10, 10, 0, 6, 0.8, [bump])
    pf = W.make_problem(21, 13, -10, 10, -6, 6, 0.8, [bump], half_domain=False)
    uh = W.perturbed_state(ph, 3)
    nbh, nbf = (ph.N + 1) * ph.M, (pf.N + 1) * pf.M
    uf = np.empty(3 * nbf)
    for f in range(3):
        bh = uh[f * nbh:(f + 1) * nbh].reshape(ph.M, ph.N + 1)
        uf[f * nbf:(f + 1) * nbf].reshape(pf.M, pf.N + 1)[:] = bh[np.abs(np.arange(pf.M) - 6)]
    a, b = P.bottom_pressure(ph, uh), P.bottom_pressure(pf, uf)
    assert np.abs(a - b[6:]).max() < 1e-13
    fa, fb = P.bottom_force(ph, a), P.bottom_force(pf, b)
    assert np.abs(fa - fb).max() < 1e-12 * (1 + np.abs(fb).max())
