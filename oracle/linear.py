"""Oracle for the linearised system, its Jacobian and the block-banded preconditioner.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain FP64 with dense
numpy/scipy matrices; meant for small meshes.

  * F_lin(u): the discrete linear problem of Section 4.2 (eqs. (linear_integral)
    and (linear_dynamic2)) in the form of Appendix B, with the same
    reconstruction, collocation and radiation rows as the nonlinear residual,
    the mirror image on a half domain, and the bottom single-layer sign reading
    (density -beta_x) used for the nonlinear residual.
  * J~ = dF_lin/du: F_lin is affine in u, and J~ is composed here from the
    linear maps u -> (node values, node x-derivatives, half-mesh values and
    x-derivatives) and the kernel matrices K5, K6, K7 (Appendix B).  The
    entries printed in Appendix B are used only as test values; several of
    them are misprinted (see the tests).
  * P: J~ with its four dense blocks (2,1), (2,3), (3,1), (3,2) kept only for
    slice pairs |m - l| <= h_b (Appendix A: a band of b blocks of size
    (N+1) x (N+1) in each block row; Reading: the band is centred, h_b = max(1, round(M/20)), i.e.
    b = 2 h_b + 1 ~ M/10 as in Table 1).
  * Surface tension (Section 6, tau != 0): the linearised dynamic row gains
    -tau (zeta_xx* + zeta_yy*) (the linear part of -tau K), which adds entries
    near the diagonal of block (1,1) -- within the slice, and coupling each
    slice to its neighbours through zeta_yy.  Reading (the paper leaves surface
    tension to future work and gives no preconditioner for it): P is the
    preconditioner of the problem without surface tension, the whole tension
    term being left to the Krylov solver.  Any part of -tau zeta_xx* kept in
    block (1,1) turns the slice block, lower triangular in x (the radiation rows
    F5, F6 fix the upstream end and each dynamic row the next slope), into a
    recurrence with a growing mode -- capillary waves travel upstream -- whose
    inverse overflows (31 x 11, F = 1.4, tau = 0.1: max |(P11 slice)^-1| ~ 1e24,
    so a factorisation that eliminates block 1 first breaks down).  Without it
    GMRES needs more iterations (to 1e-10 on the linear system at that mesh:
    298 against 176 with the in-slice zeta_xx* kept, 37 without tension).
  * P^-1 r by a dense LU solve of P (the definition); the block LU of
    Appendix A is one way of computing the same vector.
  * The linear start u_lin = u0 - J~^-1 F_lin(u0), u0 the uniform stream
    (Reading: "start from the linear solution" is the discrete linear solution
    on the same mesh).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import residual as R

TWO_PI = 2.0 * math.pi


def band_halfwidth(M: int) -> int:
    return max(1, int(round(M / 20.0)))


# ----------------------------------------------------------------------------- reconstruction maps
def reconstruction_maps(p):
    """Linear maps from one field block u_f ((N+1) M entries) to
    node values [NM], node x-derivatives [NM], half-mesh values [(N-1)M] and
    half-mesh x-derivatives [(N-1)M], each as a dense matrix."""
    N, M, dx = p.N, p.M, p.dx
    nb = (N + 1) * M
    # one slice: v = [f_1, fx_1..fx_N]; node i value = f_1 + dx * trapezoid weights
    Tn = np.zeros((N, N + 1))
    Tn[:, 0] = 1.0
    for i in range(1, N):
        Tn[i, 1:] = Tn[i - 1, 1:]
        Tn[i, 1 + i - 1] += 0.5 * dx
        Tn[i, 1 + i] += 0.5 * dx
    Dn = np.zeros((N, N + 1))
    Dn[:, 1:] = np.eye(N)
    Avg = 0.5 * (np.eye(N - 1, N) + np.eye(N - 1, N, 1))  # node -> half-mesh mean
    eyeM = np.eye(M)
    Pn = np.kron(eyeM, Tn)
    Dx = np.kron(eyeM, Dn)
    Pt = np.kron(eyeM, Avg @ Tn)
    Dt = np.kron(eyeM, Avg @ Dn)
    assert Pn.shape == (N * M, nb)
    return Pn, Dx, Pt, Dt


def Pt_slice(p):
    """Node values -> half-mesh values of one slice: [(N-1)][(N+1)] (the per-slice block of Pt)."""
    N, dx = p.N, p.dx
    Tn = np.zeros((N, N + 1))
    Tn[:, 0] = 1.0
    for i in range(1, N):
        Tn[i, 1:] = Tn[i - 1, 1:]
        Tn[i, 1 + i - 1] += 0.5 * dx
        Tn[i, 1 + i] += 0.5 * dx
    Avg = 0.5 * (np.eye(N - 1, N) + np.eye(N - 1, N, 1))
    return Avg @ Tn


def half_mesh_xx_map(p):
    """zeta_x unknowns -> zeta_xx at the half-mesh points, (zeta_x,k+1 - zeta_x,k) / dx, all slices."""
    N, M, dx = p.N, p.M, p.dx
    D = np.zeros((N - 1, N + 1))
    for k in range(N - 1):
        D[k, 1 + k] = -1.0 / dx
        D[k, 2 + k] = 1.0 / dx
    return np.kron(np.eye(M), D)


def second_y_difference(p):
    """[M][M] matrix of the node second y-differences of the residual's reading
    (oracle.residual.d2_dy2): interior, mirrored symmetry row, one-sided edges."""
    M, dy = p.M, p.dy
    Y = np.zeros((M, M))
    for j in range(1, M - 1):
        Y[j, j - 1:j + 2] = (1.0, -2.0, 1.0)
    Y[M - 1, M - 4:] = (-1.0, 4.0, -5.0, 2.0)
    if p.half_domain:
        Y[0, 0:2] = (-2.0, 2.0)
    else:
        Y[0, 0:4] = (2.0, -5.0, 4.0, -1.0)
    return Y / (dy * dy)


# ----------------------------------------------------------------------------- kernel matrices
def kernel_matrices(p):
    """w-weighted linear kernels summed over the y-images, [(N-1)M targets] x [NM nodes]:
    K5 = 1/r, K6 = (r^2+1)^(-3/2), K7 = (r^2+1)^(-1/2) (Appendix B), and the
    exact integral of K5 over the truncated (mirrored) rectangle per target."""
    N, M = p.N, p.M
    X, Y = R.collocation_points(p)
    xs, ys = X.reshape(-1), Y.reshape(-1)
    xn = np.tile(p.x(), M)
    yn = np.repeat(p.y(), N)
    ci = np.full(N, 1.0)
    ci[[0, -1]] = 0.5
    cj = np.full(M, 1.0)
    cj[[0, -1]] = 0.5
    w = p.dx * p.dy * np.outer(cj, ci).reshape(-1)
    K5 = np.zeros((xs.size, xn.size))
    K6 = np.zeros_like(K5)
    K7 = np.zeros_like(K5)
    for iota in ((1.0, -1.0) if p.half_domain else (1.0,)):
        s = xn[None, :] - xs[:, None]
        t = iota * yn[None, :] - ys[:, None]
        r2 = s * s + t * t
        K5 += w / np.sqrt(r2)
        K6 += w / (r2 + 1.0) ** 1.5
        K7 += w / np.sqrt(r2 + 1.0)
    xlo, xhi, ylo, yhi = R.integration_rectangle(p)
    one = np.ones(xs.size)
    I5 = R.s2_integral(one, 0 * one, one, xlo - xs, xhi - xs, ylo - ys, yhi - ys)
    return K5, K6, K7, I5


# ----------------------------------------------------------------------------- J~ and F_lin
def _row_positions(p):
    """Indices in F of: radiation rows (two per slice) and collocation rows, per block."""
    N, M = p.N, p.M
    nb = (N + 1) * M
    rad0 = np.array([l * (N + 1) for l in range(M)])
    rad1 = rad0 + 1
    col = np.array([l * (N + 1) + 2 + k for l in range(M) for k in range(N - 1)])
    return nb, rad0, rad1, col


def _radiation_block(p, with_value: bool):
    """Rows (F5,F6) on the f-block of its own field, as a [2M][(N+1)M] pair (A0, A1) and constants."""
    N, M, x1, dx, n = p.N, p.M, p.x1, p.dx, p.n_decay
    nb = (N + 1) * M
    A0 = np.zeros((M, nb))
    A1 = np.zeros((M, nb))
    for l in range(M):
        b = l * (N + 1)
        A0[l, b + 0] = n
        A0[l, b + 1] = x1
        A1[l, b + 1] = n - x1 / dx
        A1[l, b + 2] = x1 / dx
    return A0, A1


def jacobian(p, K=None) -> np.ndarray:
    """J~ = dF_lin/du, dense [3(N+1)M]^2, rows in the order of Appendix B."""
    N, M, F = p.N, p.M, p.froude
    nb, rad0, rad1, col = _row_positions(p)
    Pn, Dx, Pt, Dt = reconstruction_maps(p)
    K5, K6, K7, I5 = kernel_matrices(p) if K is None else K
    J = np.zeros((3 * nb, 3 * nb))
    A0, A1 = _radiation_block(p, False)
    Z, Ph, Ps = slice(0, nb), slice(nb, 2 * nb), slice(2 * nb, 3 * nb)
    for blk, cols in ((0, Z), (1, Ph), (2, Ps)):
        J[blk * nb + rad0, cols] = A0
        J[blk * nb + rad1, cols] = A1
    # F1 = phi*_x + zeta*/F^2 - 1 (- tau (zeta*_xx + zeta*_yy) with surface tension)
    J[col, Z] = Pt / (F * F)
    J[col, Ph] = Dt
    tau = getattr(p, "tau", 0.0)
    if tau != 0.0:
        J[col, Z] -= tau * (half_mesh_xx_map(p) + np.kron(second_y_difference(p), Pt_slice(p)))
    # F2 = K5 (zeta_x - zeta*_x) + zeta*_x I5 + K6 (psi - x) - beta terms - 2 pi (phi* - x*)
    J[nb + col, Z] = K5 @ Dx - (K5.sum(axis=1) - I5)[:, None] * Dt
    J[nb + col, Ph] = -TWO_PI * Pt
    J[nb + col, Ps] = K6 @ Pn
    # F7 = K7 zeta_x + K6 (phi - x) - beta terms - 2 pi (psi* - x*)
    J[2 * nb + col, Z] = K7 @ Dx
    J[2 * nb + col, Ph] = K6 @ Pn
    J[2 * nb + col, Ps] = -TWO_PI * Pt
    return J


def forcing(p, K=None) -> np.ndarray:
    """F_lin(u0) at the uniform stream: the terms of the linear rows driven by beta_x."""
    N, M = p.N, p.M
    nb, rad0, rad1, col = _row_positions(p)
    K5, K6, K7, I5 = kernel_matrices(p) if K is None else K
    bx = p.beta_x.reshape(-1)
    bxs = R.half_mesh(p.beta_x).reshape(-1)
    f = np.zeros(3 * nb)
    # surface rows: bottom single layer with density -beta_x
    f[nb + col] = -(K7 @ bx)
    # bottom rows: own single layer -beta_x with the subtraction of -beta*_x K5
    f[2 * nb + col] = -(K5 @ bx - K5.sum(axis=1) * bxs) - bxs * I5
    return f


def F_lin(p, u: np.ndarray, J=None, f0=None) -> np.ndarray:
    """The linear residual: affine, F_lin(u) = J~ (u - u0) + F_lin(u0)."""
    from paper_1709_08803_amd.workloads import uniform_stream
    J = jacobian(p) if J is None else J
    f0 = forcing(p) if f0 is None else f0
    return J @ (u - uniform_stream(p)) + f0


def linear_start(p, J=None, f0=None) -> np.ndarray:
    """Discrete linear solution u_lin = u0 - J~^-1 F_lin(u0)."""
    from paper_1709_08803_amd.workloads import uniform_stream
    J = jacobian(p) if J is None else J
    f0 = forcing(p) if f0 is None else f0
    return uniform_stream(p) - sla.solve(J, f0)


# ----------------------------------------------------------------------------- preconditioner
def slice_of_index(p, idx: np.ndarray) -> np.ndarray:
    """y-slice l of a position in u or F (both are ordered slice by slice within each block)."""
    nb = (p.N + 1) * p.M
    return (idx % nb) // (p.N + 1)


def banded(p, J: np.ndarray, hb: int) -> np.ndarray:
    """P: J~ with the dense blocks (2,1), (2,3), (3,1), (3,2) cut to slice band |m - l| <= hb;
    with surface tension, block (1,1) is that of the problem without it."""
    nb = (p.N + 1) * p.M
    P = J.copy()
    sl = slice_of_index(p, np.arange(nb))
    far = np.abs(sl[:, None] - sl[None, :]) > hb
    for (bi, bj) in ((1, 0), (1, 2), (2, 0), (2, 1)):
        blk = P[bi * nb:(bi + 1) * nb, bj * nb:(bj + 1) * nb]
        blk[far] = 0.0
    tau = getattr(p, "tau", 0.0)
    if tau != 0.0:  # block (1,1) of the problem without surface tension
        _, _, _, col = _row_positions(p)
        P[col, :nb] += tau * (half_mesh_xx_map(p) + np.kron(second_y_difference(p), Pt_slice(p)))
    return P


class Preconditioner:
    """P = banded J~ and its LU factors (dense; small meshes only)."""

    def __init__(self, p, hb: int = -1, J=None):
        self.hb = band_halfwidth(p.M) if hb < 0 else hb
        self.J = jacobian(p) if J is None else J
        self.P = banded(p, self.J, self.hb)
        self.lu = sla.lu_factor(self.P)

    def apply(self, r: np.ndarray) -> np.ndarray:
        """z = P^-1 r."""
        return sla.lu_solve(self.lu, r)

    def matvec(self, z: np.ndarray) -> np.ndarray:
        return self.P @ z


def banded_matvec(p, z: np.ndarray, hb: int) -> np.ndarray:
    """P z without forming P (any mesh size): the linear rows of Appendix B
    applied to z with the kernel sums restricted to source slices |m - l| <= hb
    (the singular-subtraction term of the K5 row uses the full row sum, as in J~)."""
    N, M, F, n, x1, dx = p.N, p.M, p.froude, p.n_decay, p.x1, p.dx
    nf = R.reconstruct(p, z)  # linear in z: node values and x-derivatives of each block
    nb = (N + 1) * M
    out = np.zeros(3 * nb)
    X, Y = R.collocation_points(p)
    xs, ys = X.reshape(M, N - 1), Y.reshape(M, N - 1)
    ci = np.full(N, 1.0)
    ci[[0, -1]] = 0.5
    xn = p.x()
    xlo, xhi, ylo, yhi = R.integration_rectangle(p)
    zeta_s = R.half_mesh(nf.zeta)
    zx_s = R.half_mesh(nf.zeta_x)
    phi_s = R.half_mesh(nf.phi)
    phx_s = R.half_mesh(nf.phi_x)
    psi_s = R.half_mesh(nf.psi)
    F1 = phx_s + zeta_s / (F * F)
    F2 = -TWO_PI * phi_s
    F7 = -TWO_PI * psi_s
    images = (1.0, -1.0) if p.half_domain else (1.0,)
    for l in range(M):
        s = xn[None, :] - xs[l][:, None]  # [N-1][N]
        rowsum = np.zeros(N - 1)
        for m in range(M):
            cm = 0.5 if m in (0, M - 1) else 1.0
            w = p.dx * p.dy * ci * cm
            k5 = np.zeros((N - 1, N))
            k6 = np.zeros_like(k5)
            k7 = np.zeros_like(k5)
            for iota in images:
                t = iota * p.y()[m] - ys[l][0]
                r2 = s * s + t * t
                k5 += w / np.sqrt(r2)
                k6 += w / (r2 + 1.0) ** 1.5
                k7 += w / np.sqrt(r2 + 1.0)
            rowsum += k5.sum(axis=1)
            if abs(m - l) <= hb:
                F2[l] += k5 @ nf.zeta_x[m] + k6 @ nf.psi[m]
                F7[l] += k7 @ nf.zeta_x[m] + k6 @ nf.phi[m]
        one = np.ones(N - 1)
        I5 = R.s2_integral(one, 0 * one, one, xlo - xs[l], xhi - xs[l], ylo - ys[l], yhi - ys[l])
        F2[l] -= zx_s[l] * (rowsum - I5)
    rad = {
        "F5": x1 * nf.zeta_x[:, 0] + n * nf.zeta[:, 0],
        "F6": x1 / dx * (nf.zeta_x[:, 1] - nf.zeta_x[:, 0]) + n * nf.zeta_x[:, 0],
        "F3": x1 * nf.phi_x[:, 0] + n * nf.phi[:, 0],
        "F4": x1 / dx * (nf.phi_x[:, 1] - nf.phi_x[:, 0]) + n * nf.phi_x[:, 0],
        "F8": x1 * nf.psi_x[:, 0] + n * nf.psi[:, 0],
        "F9": x1 / dx * (nf.psi_x[:, 1] - nf.psi_x[:, 0]) + n * nf.psi_x[:, 0],
    }
    return R.assemble(p, F1, F2, F7, rad)
