"""Pins of the oracle residual against facts the paper and mathematics fix.

Each test names the passage it pins.  None of them re-types the oracle's own
formulas: they use an independent quadrature routine, Green's identity on
harmonic fields, symmetry, closed-form special cases, and the Jacobian entries
printed in Appendix B.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_1709_08803_amd import workloads as W
from oracle import residual as R
from harmonic import multipole_sources, field


# ---------------------------------------------------------------- S2 closed form (Section 3.1, I2'')
@pytest.mark.parametrize("seed", range(6))
def test_s2_closed_form_matches_adaptive_quadrature(seed):
    rng = np.random.default_rng(seed)
    zx, zy = rng.uniform(-0.8, 0.8, 2)
    A, B, C = 1 + zx * zx, 2 * zx * zy, 1 + zy * zy
    s1, s2 = -rng.uniform(1, 6), rng.uniform(1, 6)
    # include rectangles with an edge through the singular point (t1 = 0 / t2 = 0)
    t1 = 0.0 if seed % 3 == 0 else -rng.uniform(1, 6)
    t2 = 0.0 if seed % 3 == 1 else rng.uniform(1, 6)
    f = lambda t, s: 1.0 / math.sqrt(A * s * s + B * s * t + C * t * t)
    ref = 0.0
    # split at the singular point so the adaptive rule sees integrable corners
    for (a, b) in ((s1, 0.0), (0.0, s2)):
        for (c, d) in ((t1, 0.0), (0.0, t2)):
            if a < b and c < d:
                v, err = integrate.dblquad(f, a, b, c, d, epsabs=1e-13, epsrel=1e-13)
                ref += v
    got = R.s2_integral(np.array([A]), np.array([B]), np.array([C]), s1, s2, t1, t2)[0]
    assert abs(got - ref) <= 1e-10 * abs(ref)


def test_s2_closed_form_isotropic_square():
    # A = C = 1, B = 0: integral of 1/r over [-a,a]^2 = 8 a asinh(1) (polar closed form)
    a = 2.5
    got = R.s2_integral(np.array([1.0]), np.array([0.0]), np.array([1.0]), -a, a, -a, a)[0]
    assert abs(got - 8 * a * math.asinh(1.0)) < 1e-13


# ---------------------------------------------------------------- uniform stream and constants
def test_uniform_stream_gives_zero_residual():
    p = W.make_problem(31, 11, -16, 16, 0, 10, 0.7, [])
    F = R.residual(p, W.uniform_stream(p))
    assert np.abs(F).max() < 1e-12


def _rect_solid_angle(xs, ys, h, x1, x2, y1, y2):
    """Solid angle of the plate [x1,x2]x[y1,y2] seen from (xs, ys) at height h (closed form)."""
    F = lambda a, b: np.arctan(a * b / (h * np.sqrt(a * a + b * b + h * h)))
    return F(x2 - xs, y2 - ys) - F(x1 - xs, y2 - ys) - F(x2 - xs, y1 - ys) + F(x1 - xs, y1 - ys)


def test_constant_potential_shift_is_solid_angle_of_other_boundary():
    # phi = psi = x + c on flat boundaries: each BIE row is c (Omega - 2 pi), where
    # Omega is the solid angle the other boundary (a plate at distance 1, here the
    # truncated mirrored mesh) subtends; the 2 pi is that of the infinite plane.
    c = 0.3
    L, h = 12.0, 0.4
    p = W.make_problem(int(2 * L / h) + 1, int(L / h) + 1, -L, L, 0, L, 0.7, [])
    u = W.uniform_stream(p)
    nb = (p.N + 1) * p.M
    for f in (1, 2):
        u[f * nb:(f + 1) * nb].reshape(p.M, p.N + 1)[:, 0] += c
    F = R.residual(p, u)
    X, Y = R.collocation_points(p)
    omega = _rect_solid_angle(X, Y, 1.0, -L, L, -L, L)
    ref = c * (omega - 2 * math.pi)
    inner = (np.abs(X) < L - 3) & (Y < L - 3)  # away from the edges the trapezoid rule is O(h^2) exact
    for blk in (1, 2):
        rows = F[blk * nb:(blk + 1) * nb].reshape(p.M, p.N + 1)[:, 2:]
        assert np.abs(rows - ref)[(np.abs(X) < 4) & (Y < 4)].max() < 5e-4 * c
        assert np.abs(rows - ref)[inner].max() < 3e-3 * c
        assert np.abs(rows - ref).max() < 0.05 * c
    assert np.abs(ref[inner]).max() > 0.1 * c  # the truncation effect is resolved, not negligible


# ---------------------------------------------------------------- Green's identity on harmonic fields
def _harmonic_rows(L, h, zeta_amp=0.0, bump=0.0, half=True, plant=None):
    N, M = int(round(2 * L / h)) + 1, int(round(L / h)) + 1
    bumps = [W.Bump(bump, 1.5, 1.5)] if bump else []
    if half:
        p = W.make_problem(N, M, -L, L, 0.0, L, 0.7, bumps)
    else:
        p = W.make_problem(N, 2 * M - 1, -L, L, -L, L, 0.7, bumps, half_domain=False)
    X, Y = np.meshgrid(p.x(), p.y())
    g = zeta_amp * np.exp(-(X ** 2 + Y ** 2) / 4.0)
    zx, zy = g * (-X / 2.0), g * (-Y / 2.0)
    pos, q = multipole_sources(above=(0.6 + zeta_amp, 1.0 + zeta_amp), below=(-1.6, -2.0))
    uS, gxS, gyS, gzS = field(pos, q, X, Y, g)
    uB, gxB, gyB, gzB = field(pos, q, X, Y, p.beta)
    # single-layer slots: outward-normal flux per unit plan area (S), and its
    # negative on B, the slot that holds beta_x when u = Phi - x.
    sigS = -gxS * zx - gyS * zy + gzS
    sigB = gzB - gxB * p.beta_x - gyB * p.beta_y
    if plant == "bottom_single_layer_sign":
        sigB = -sigB
    gS, gB = R.Geometry(g, zx, zy), R.Geometry(p.beta, p.beta_x, p.beta_y)
    F2 = R.bie_rows(p, gS, uS, sigS, gB, uB, sigB, R.targets_from_nodes(p, gS, uS, sigS, "S"))
    F7 = R.bie_rows(p, gS, uS, sigS, gB, uB, sigB, R.targets_from_nodes(p, gB, uB, sigB, "B"))
    scale = 2 * math.pi * np.abs(uS).max()
    return np.abs(F2).max() / scale, np.abs(F7).max() / scale


def test_green_identity_flat_layer_converges():
    e1 = _harmonic_rows(10, 0.5)
    e2 = _harmonic_rows(10, 0.25)
    assert max(e2) < 0.03
    assert e2[0] < e1[0] / 2 and e2[1] < e1[1] / 2


def test_green_identity_rejects_printed_bottom_single_layer_sign():
    # the sign printed for I4 (+beta_x K2) violates Green's identity by O(1)
    e = _harmonic_rows(10, 0.25, plant="bottom_single_layer_sign")
    assert max(e) > 0.5


def test_green_identity_curved_boundaries_converges():
    e1 = _harmonic_rows(10, 0.5, zeta_amp=0.1, bump=0.2)
    e2 = _harmonic_rows(10, 0.25, zeta_amp=0.1, bump=0.2)
    assert max(e2) < 0.025
    assert e2[0] < e1[0] / 2 and e2[1] < e1[1]


def test_green_identity_full_domain():
    e = _harmonic_rows(8, 0.25, zeta_amp=0.1, bump=0.2, half=False)
    assert max(e) < 0.03


# ---------------------------------------------------------------- half domain == mirrored full domain
def test_half_domain_equals_full_domain_on_mirrored_data():
    ph = W.make_problem(21, 7, -10, 10, 0, 6, 0.8, [W.Bump(0.15, 1.2, 1.2)])
    pf = W.make_problem(21, 13, -10, 10, -6, 6, 0.8, [W.Bump(0.15, 1.2, 1.2)], half_domain=False)
    uh = W.perturbed_state(ph, 3)
    # mirror u: slices j of the full mesh are |j - 6| of the half mesh
    nbh, nbf = (ph.N + 1) * ph.M, (pf.N + 1) * pf.M
    uf = np.empty(3 * nbf)
    for f in range(3):
        bh = uh[f * nbh:(f + 1) * nbh].reshape(ph.M, ph.N + 1)
        uf[f * nbf:(f + 1) * nbf].reshape(pf.M, pf.N + 1)[:] = bh[np.abs(np.arange(pf.M) - 6)]
    Fh, Ff = R.residual(ph, uh), R.residual(pf, uf)
    for f in range(3):
        a = Fh[f * nbh:(f + 1) * nbh].reshape(ph.M, ph.N + 1)
        b = Ff[f * nbf:(f + 1) * nbf].reshape(pf.M, pf.N + 1)[6:]
        # the full domain's y-derivative on its central row is the central difference
        # of mirrored data, i.e. zero as on the half domain; all rows must agree
        assert np.abs(a - b).max() < 1e-12 * (1 + np.abs(a).max())


# ---------------------------------------------------------------- dynamic condition (eq. new_finite_dynamic)
def test_dynamic_row_is_bernoulli_with_kinematic_condition():
    # With Phi_z eliminated by the kinematic condition, the combined form must
    # equal 1/2 |grad Phi|^2 + zeta/F^2 - 1/2 (eq. finite_dynamic).
    rng = np.random.default_rng(0)
    p = W.make_problem(5, 4, -2, 2, 0, 3, 0.9, [])
    for _ in range(5):
        Px, Py, zx, zy, z = rng.uniform(-1, 1, 5)
        Pz = Px * zx + Py * zy
        phx, phy = Px + Pz * zx, Py + Pz * zy
        nf = R.NodeFields(*(np.full((4, 5), v) for v in (z, zx, zy, 0.0, phx, phy, 0.0, 0.0)))
        F1 = R.dynamic_rows(p, nf)
        ref = 0.5 * (Px * Px + Py * Py + Pz * Pz) + z / p.froude ** 2 - 0.5
        assert np.allclose(F1, ref, atol=1e-14)


# ---------------------------------------------------------------- Appendix B entries
def _fd_jacobian_rows(p, u, rows, cols, h=1e-6):
    J = np.zeros((len(rows), len(cols)))
    for c_i, c in enumerate(cols):
        e = np.zeros_like(u)
        e[c] = h
        J[:, c_i] = (R.residual_rows(p, u + e, rows) - R.residual_rows(p, u - e, rows)) / (2 * h)
    return J


def test_reconstruction_matches_appendix_b_dynamic_and_potential_entries():
    # Appendix B prints dF1/dphi_x = 1/2 at n = k, k+1; dF1/dzeta_x = dx/F^2 (1/2, 1.., 3/4, 1/4);
    # dF2/dphi_x = -pi dx, -2 pi dx.., -3 pi dx/2, -pi dx/2; dF2/dphi_1 = -2 pi.
    p = W.make_problem(9, 4, -4, 4, 0, 3, 0.8, [])
    u = W.uniform_stream(p)
    N, M, dx, F = p.N, p.M, p.dx, p.froude
    nb = (N + 1) * M
    l, k = 2, 4
    r1 = R.row_index(p, 0, l, k)
    r2 = R.row_index(p, 1, l, k)
    zcols = [l * (N + 1) + 1 + n for n in range(N)]
    pcols = [nb + l * (N + 1) + 1 + n for n in range(N)]
    J = _fd_jacobian_rows(p, u, [r1, r2], zcols + pcols + [l * (N + 1), nb + l * (N + 1)])
    pat = np.array([0.5, 1, 1, 1, 0.75, 0.25, 0, 0, 0]) * dx  # d zeta*_k / d zeta_x, k = 4 (0-based)
    assert np.allclose(J[0, :N], pat / F ** 2, atol=1e-8)
    assert np.allclose(J[0, N:2 * N], [0, 0, 0, 0, 0.5, 0.5, 0, 0, 0], atol=1e-8)
    assert abs(J[0, 2 * N] - 1 / F ** 2) < 1e-8
    assert np.allclose(J[1, N:2 * N], -2 * math.pi * pat, atol=1e-7)
    assert abs(J[1, 2 * N + 1] + 2 * math.pi) < 1e-7


def test_radiation_rows_match_appendix_b():
    p = W.tiny()
    u = W.perturbed_state(p, 5)
    nf = R.reconstruct(p, u)
    rad = R.radiation_rows(p, nf)
    x1, dx, n = p.x1, p.dx, p.n_decay
    # Appendix B prints the affine forms of F3..F6, F8, F9
    assert np.allclose(rad["F3"], x1 * nf.phi_x[:, 0] + n * nf.phi[:, 0] - x1 * (n + 1), atol=1e-13)
    assert np.allclose(rad["F4"], x1 / dx * nf.phi_x[:, 1] + (n - x1 / dx) * nf.phi_x[:, 0] - n, atol=1e-12)
    assert np.allclose(rad["F5"], x1 * nf.zeta_x[:, 0] + n * nf.zeta[:, 0], atol=1e-13)
    assert np.allclose(rad["F6"], x1 / dx * nf.zeta_x[:, 1] + (n - x1 / dx) * nf.zeta_x[:, 0], atol=1e-12)
    assert np.allclose(rad["F8"], x1 * nf.psi_x[:, 0] + n * nf.psi[:, 0] - x1 * (n + 1), atol=1e-13)
    assert np.allclose(rad["F9"], x1 / dx * nf.psi_x[:, 1] + (n - x1 / dx) * nf.psi_x[:, 0] - n, atol=1e-12)


def test_row_subset_matches_full_residual():
    p = W.tiny()
    u = W.perturbed_state(p, 2)
    F = R.residual(p, u)
    rows = np.random.default_rng(0).choice(F.size, 60, replace=False)
    assert np.array_equal(R.residual_rows(p, u, rows), F[rows])
