"""Pins of the oracle's exact linear solution, eq. (exactsoln) of Section 4.1.

The quadrature of eq. (exactsoln) is checked against what fixes it from
outside the formula:
  * the linear problem solved by a 2-D FFT with the radiation condition
    imposed by a slow switch-on (damping mu); that solution converges to the
    radiation solution at first order in mu, so two dampings are extrapolated
    to mu -> 0 (Richardson) -- an independent method;
  * the radiation condition itself: zeta -> 0 far upstream;
  * zeta_x (differentiated under the integral signs) against central
    differences of zeta, including on x = 0 where |x| has its kink;
  * zeta even in y for a bump centred on y = 0.
A planted mistake in the pole's residue (dropped, or sign-flipped) must fail
the first two.
"""
import math

import numpy as np
import pytest

from oracle import fourier as Fo

EPS = 0.01  # bump height: the linear solution is proportional to it


def _fft_extrapolated(F, delta, pts):
    vals = {}
    for mu in (0.01, 0.005):
        x, y, z = Fo.linear_surface_fft(F, lambda X, Y: EPS * np.exp(-(X * X + Y * Y) / (2 * delta * delta)),
                                        160.0, 0.125, mu)
        vals[mu] = np.array([z[np.argmin(np.abs(y - py)), np.argmin(np.abs(x - px))] for px, py in pts])
    return 2.0 * vals[0.005] - vals[0.01]


def _exact(F, delta, pts, order=0):
    return Fo.exact_solution(F, [(EPS, delta, 0.0, 0.0)], [p[0] for p in pts], [p[1] for p in pts], order=order)


# (F, delta, points): the subcritical working bump and a supercritical one.
FFT_CASES = [
    (0.7, 1.0 / math.sqrt(2.0), ((-5.0, 0.0), (0.0, 0.0), (3.0, 0.0), (6.0, 0.0), (3.0, 2.0), (10.0, 3.0))),
    (1.4, 1.0 / math.sqrt(2.0), ((-5.0, 0.0), (-1.0, 0.0), (0.0, 0.0), (3.0, 0.0), (6.0, 0.0), (3.0, 2.0))),
]


def _fft_pin_holds(F, delta, pts):
    ex = _exact(F, delta, pts)
    ff = _fft_extrapolated(F, delta, pts)
    # the FFT's own error (periodic box of 320 x 320, O(mu^2)) is ~0.5 % of max|zeta| at these points
    return np.abs(ex - ff).max() <= 1.5e-2 * np.abs(ff).max(), ex, ff


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("F,delta,pts", FFT_CASES, ids=[f"F{c[0]}" for c in FFT_CASES])
def test_exact_matches_fft_extrapolated_to_no_damping(F, delta, pts):
    ok, ex, ff = _fft_pin_holds(F, delta, pts)
    assert ok, (ex, ff)


def _upstream_pin_holds(F):
    delta = 1.0 / math.sqrt(2.0)
    far = _exact(F, delta, ((-25.0, 0.0), (-25.0, 4.0)))
    near = _exact(F, delta, ((0.0, 0.0), (3.0, 0.0)))
    return np.abs(far).max() <= 0.01 * np.abs(near).max(), far, near


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("F", (0.7, 1.4))
def test_exact_vanishes_upstream(F):
    ok, far, near = _upstream_pin_holds(F)
    assert ok, (far, near)


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
def test_exact_derivative_matches_differences():
    F, delta, h = 0.6, 0.5, 1e-3
    for x, y in ((-2.0, 0.5), (0.0, 0.0), (0.0, 1.0), (1.5, 0.3), (4.0, 2.0)):
        zx = _exact(F, delta, ((x, y),), order=1)[0]
        zp, zm = _exact(F, delta, ((x + h, y), (x - h, y)))
        # central-difference truncation ~ zeta''' h^2 / 6 and the quadrature's 1e-10 / h
        assert abs(zx - (zp - zm) / (2 * h)) <= 2e-6 * EPS, (x, y, zx, (zp - zm) / (2 * h))


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
def test_exact_even_in_y():
    v = _exact(0.7, 0.5, ((2.0, 1.5), (2.0, -1.5), (-1.0, 3.0), (-1.0, -3.0)))
    assert abs(v[0] - v[1]) <= 1e-12 and abs(v[2] - v[3]) <= 1e-12


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("plant", ("drop", "flip"))
def test_planted_residue_mistakes_fail_the_pins(monkeypatch, plant):
    true = Fo.pole_residue
    if plant == "drop":
        monkeypatch.setattr(Fo, "pole_residue", lambda *a: 0.0)
    else:
        monkeypatch.setattr(Fo, "pole_residue", lambda *a: -true(*a))
    assert not _upstream_pin_holds(0.7)[0]
    assert not _fft_pin_holds(*FFT_CASES[0])[0]


def test_k_minus_tanh_series():
    # the series branch below 0.1 against the direct difference where that is still accurate,
    # and against its leading term k^3/3 where the direct difference has lost every digit
    for k in (0.05, 0.07, 0.0999):
        assert abs(Fo._k_minus_tanh(k) - (k - math.tanh(k))) <= 1e-12 * (k - math.tanh(k))
    for k in (1e-5, 1e-3):
        assert abs(Fo._k_minus_tanh(k) - k ** 3 / 3) <= 0.41 * k ** 5
    assert Fo._k_minus_tanh(0.1) == 0.1 - math.tanh(0.1)


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
def test_exact_supercritical_stable_under_k_truncation():
    # F > 1: the principal value next to small poles (psi just above psi_0) is formed without
    # cancellation, so the result does not move when the k-range is extended
    bt = Fo.bump_transform(EPS, 3.0)
    a = Fo.exact_solution_point(3.0, bt, 10.0, 0.0, kmax=Fo.bump_kmax(3.0))
    b = Fo.exact_solution_point(3.0, bt, 10.0, 0.0, kmax=5.0)
    assert abs(a - b) <= 1e-9 * EPS
