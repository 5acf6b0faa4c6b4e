"""Pins of the oracle's linearised system, Jacobian and preconditioner (Section 4, Appendices A and B)."""
import math

import numpy as np
import pytest

from paper_1709_08803_amd import workloads as W
from oracle import residual as R
from oracle import linear as Lin


@pytest.fixture(scope="module")
def small():
    p = W.make_problem(13, 5, -6, 6, 0, 4, 0.8, [])
    return p, Lin.jacobian(p)


def test_jacobian_equals_fd_jacobian_of_nonlinear_residual_at_uniform_stream(small):
    # Every nonlinear term that differs from its linearisation carries a factor
    # vanishing at the uniform stream over a flat bottom, so the nonlinear
    # Jacobian there is exactly J~ (Section 4.2).
    p, J = small
    u0 = W.uniform_stream(p)
    n, h = u0.size, 1e-5
    Jfd = np.empty_like(J)
    for c in range(n):
        e = np.zeros(n)
        e[c] = h
        Jfd[:, c] = (R.residual(p, u0 + e) - R.residual(p, u0 - e)) / (2 * h)
    assert np.abs(J - Jfd).max() < 1e-8


def test_forcing_is_nonlinear_residual_to_second_order_in_bump_height():
    errs = []
    for eps in (1e-3, 5e-4):
        p = W.make_problem(13, 5, -6, 6, 0, 4, 0.8, [W.Bump(eps, 1.0, 1.0)])
        errs.append(np.abs(R.residual(p, W.uniform_stream(p)) - Lin.forcing(p)).max())
    assert errs[1] < errs[0] / 3.5  # O(eps^2): halving eps quarters the difference


def test_block_identities_printed_in_section_4(small):
    # J~_23 = J~_32 and J~_22 = J~_33 (Section 4.2); J~_13 = 0; J~_11, J~_12,
    # J~_22 couple a slice only to itself.
    p, J = small
    nb = (p.N + 1) * p.M
    B = lambda i, j: J[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]
    assert np.array_equal(B(1, 2), B(2, 1))
    assert np.array_equal(B(1, 1), B(2, 2))
    assert not B(0, 2).any()
    sl = Lin.slice_of_index(p, np.arange(nb))
    off = sl[:, None] != sl[None, :]
    for (i, j) in ((0, 0), (0, 1), (1, 1)):
        assert not B(i, j)[off].any()
    colloc = (np.arange(nb) % (p.N + 1)) >= 2  # radiation rows have no long-range terms
    for (i, j) in ((1, 0), (1, 2), (2, 0)):
        blk = B(i, j)[colloc]
        assert np.abs(blk[off[colloc] & (np.arange(nb) % (p.N + 1) >= 1)[None, :]]).min() > 0  # dense


def test_appendix_b_potential_kernel_entries(small):
    # dF2/d(psi_x)_{n,m} printed: n=1: sum_{i>=2} dx/2 w K6; 1<n<N: dx/2 w K6(n) + dx sum_{i>n} w K6;
    # n=N: dx/2 w K6(N).  dF7/d(psi_x) printed: -pi dx (n=1), -2 pi dx, -3 pi dx/2 (n=k), -pi dx/2 (n=k+1).
    p, J = small
    N, M, dx = p.N, p.M, p.dx
    nb = (N + 1) * M
    K5, K6, K7, I5 = Lin.kernel_matrices(p)
    l, k, m = 2, 6, 1
    r = l * (N - 1) + k
    row2 = nb + l * (N + 1) + 2 + k
    wK6 = K6[r].reshape(M, N)[m]
    expect = np.array([dx / 2 * wK6[1:].sum()] + [dx / 2 * wK6[n] + dx * wK6[n + 1:].sum() for n in range(1, N - 1)]
                      + [dx / 2 * wK6[N - 1]])
    got = J[row2, 2 * nb + m * (N + 1) + 1: 2 * nb + m * (N + 1) + 1 + N]
    assert np.allclose(got, expect, rtol=1e-13, atol=1e-15)
    row7 = 2 * nb + l * (N + 1) + 2 + k
    got7 = J[row7, 2 * nb + l * (N + 1) + 1: 2 * nb + l * (N + 1) + 1 + N]
    exp7 = -math.pi * dx * np.array([1.0] + [2.0] * (k - 1) + [1.5, 0.5] + [0.0] * (N - k - 2))
    assert np.allclose(got7, exp7, atol=1e-13)
    # and the entries Appendix B misprints: dF2/dpsi_1 is sum_i w K6 (printed 0);
    # dF7/dzeta_x is +w K7 for every slice (printed -w K5 on slice l only)
    assert abs(J[row2, 2 * nb + m * (N + 1)] - wK6.sum()) < 1e-13
    assert np.allclose(J[row7, m * (N + 1) + 1: m * (N + 1) + 1 + N], K7[r].reshape(M, N)[m], atol=1e-14)


def test_band_and_block_lu_structure_of_appendix_a():
    # Banding the four dense blocks and factoring P in 3x3 blocks leaves exactly
    # two dense factor blocks, L32 and U33 (Appendix A, figure of the factored P).
    p = W.make_problem(13, 9, -6, 6, 0, 8, 0.8, [])
    pc = Lin.Preconditioner(p, hb=1)
    P, nb = pc.P, (p.N + 1) * p.M
    B = lambda i, j: P[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]
    inv = np.linalg.inv
    U11, U12 = B(0, 0), B(0, 1)
    L21 = B(1, 0) @ inv(U11)
    U22 = B(1, 1) - L21 @ U12
    L31 = B(2, 0) @ inv(U11)
    L32 = (B(2, 1) - L31 @ U12) @ inv(U22)
    U33 = B(2, 2) - L32 @ B(1, 2)
    sl = Lin.slice_of_index(p, np.arange(nb))
    far = np.abs(sl[:, None] - sl[None, :]) > 2  # beyond the band of products of banded blocks
    tiny = 1e-12
    for name, X in (("L21", L21), ("U22", U22), ("L31", L31)):
        assert np.abs(X[far]).max() < tiny, name
    for name, X in (("L32", L32), ("U33", U33)):
        assert np.abs(X[far]).max() > 1e-6, name


def test_preconditioner_solves_its_system():
    p = W.tiny(0.7)
    pc = Lin.Preconditioner(p)
    r = np.random.default_rng(0).standard_normal(p.n_unknowns)
    z = pc.apply(r)
    assert np.abs(pc.matvec(z) - r).max() < 1e-10 * np.abs(r).max()
    assert pc.hb == 1


def test_linear_start_solves_linear_system_and_is_second_order_accurate():
    res = []
    for eps in (0.02, 0.01):
        p = W.make_problem(31, 11, -16, 16, 0, 10, 0.7, [W.Bump(eps, 1.0, 1.0)])
        J, f0 = Lin.jacobian(p), Lin.forcing(p)
        ul = Lin.linear_start(p, J, f0)
        assert np.abs(Lin.F_lin(p, ul, J, f0)).max() < 1e-11
        res.append(np.abs(R.residual(p, ul)).max())
    # the nonlinear residual of the linear solution is O(eps^2)
    assert 3.3 < res[0] / res[1] < 4.7


@pytest.mark.parametrize("N,M,hb", [(31, 11, 1), (21, 9, 2), (13, 7, 3)])
def test_banded_matvec_equals_dense_banded_jacobian(N, M, hb):
    p = W.make_problem(N, M, -10, 10, 0, 6, 0.8, [W.Bump(0.1, 1, 1)])
    pc = Lin.Preconditioner(p, hb=hb)
    z = np.random.default_rng(1).standard_normal(p.n_unknowns)
    a, b = pc.matvec(z), Lin.banded_matvec(p, z, hb)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
