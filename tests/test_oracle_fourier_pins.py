"""Linear theory (Section 4.1) pins of the oracle's discrete linear solution."""
import math
import os

import numpy as np
import pytest

from paper_1709_08803_amd import workloads as W
from oracle import fourier as Fo
from oracle import linear as Lin
from oracle import residual as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")


def golden():
    vals = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            name, v = line.split()[:2]
            vals[name] = float(v)
    return vals


def test_printed_wavelengths_follow_from_dispersion_relation():
    g = golden()
    lam = 2 * math.pi / Fo.dispersion_root(0.6)
    assert abs(lam - g["wavelength_F0.6"]) < 0.005
    assert abs(4 * lam - g["inline_constructive_separation_linear"]) < 0.01
    assert abs(4.5 * lam - g["inline_destructive_separation_linear"]) < 0.01


def _centreline(F, N, M, xlo, xhi, yhi, eps=0.01):
    p = W.make_problem(N, M, xlo, xhi, 0, yhi, F, [W.Bump(eps, 1.0, 1.0)])
    nf = R.reconstruct(p, Lin.linear_start(p))
    return p.x(), nf.zeta[0] / eps


def _fft_centreline(F, xs, eps=0.01, h=0.25, mu=0.02):
    x, y, z = Fo.linear_surface_fft(F, lambda X, Y: eps * np.exp(-(X * X + Y * Y)), 160.0, h, mu)
    return np.interp(xs, x, z[np.argmin(np.abs(y))]) / eps


def test_discrete_linear_solution_matches_fourier_solution_supercritical():
    xs, zb = _centreline(1.4, 91, 31, -15, 30, 15)
    zf = _fft_centreline(1.4, xs)
    sel = (xs > -3) & (xs < 8)
    assert np.abs(zb - zf)[sel].max() < 0.12 * np.abs(zf[sel]).max()
    i0 = np.argmax(np.abs(zf[sel]))
    assert np.sign(zb[sel][i0]) == np.sign(zf[sel][i0])  # same sign at the main crest


def test_discrete_linear_solution_converges_to_fourier_solution_subcritical():
    errs = []
    for N, M in ((41, 13), (81, 25)):
        xs, zb = _centreline(0.7, N, M, -8, 12, 6)
        zf = _fft_centreline(0.7, xs, h=0.125, mu=0.01)
        sel = (xs > -3) & (xs < 8)
        errs.append(np.abs(zb - zf)[sel].max())
        near = (xs > -2.5) & (xs < 1.0)  # over the bump, before the wave train
        assert np.abs(zb - zf)[near].max() < 0.15 * np.abs(zf[near]).max()
    assert errs[1] < 0.6 * errs[0]
