"""Oracle for the discrete nonlinear residual F(u) (Section 3.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain FP64; every
function below states the passage it follows.  Readings of passages that the
paper leaves open are marked "Reading:".

F(u) is built in these steps:
  1. unpack u and integrate the x-derivatives along each y-slice with the
     trapezoidal rule (Section 3.1, eq. (unknowns); the reconstruction is the one
     whose Jacobian Appendix B prints: d zeta*/d zeta_x = dx (1/2, 1, .., 3/4, 1/4));
  2. y-derivatives by finite differences (Reading: second-order central
     differences, one-sided three-point stencils at an outer edge, zero on the
     symmetry line y = 0 of a half domain);
  3. values at the half-mesh collocation points (x_{k+1/2}, y_l) as the mean of
     the two neighbouring nodes (Appendix B: d phi*_x / d phi_x = 1/2 at n = k, k+1);
  4. the boundary-integral rows on the free surface (F2) and on the bottom (F7)
     from the trapezoidal sums of K1, K2 with the S2 subtraction and the closed
     form of the S2 integral (Section 2.2 and Section 3.1);
  5. the dynamic condition (F1, eq. (new_finite_dynamic)) at the same points,
     with the surface-tension term of Section 6 when the problem's tau is not 0;
  6. the six radiation rows per slice (eqs. (scullen1)-(scullen6), discretised
     as in Appendix B);
  7. assembly in the row order printed in Appendix B.

Readings that fix signs (derived from Green's second identity with outward
normals, and pinned by tests on harmonic fields):
  * the bottom single layer enters with density -beta_x (the paper prints +);
  * on the bottom equation the target value psi* is subtracted from the bottom
    double layer (the surface on which the target lies), not from the free
    surface one; the free-surface double layer there is integrated as is.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional, Sequence

import numpy as np

from . import _clib

TWO_PI = 2.0 * math.pi


# ----------------------------------------------------------------------------- step 1
def unpack(p, u: np.ndarray) -> Dict[str, np.ndarray]:
    """Split u (eq. (unknowns)) into f_{1,j} [M] and (f_x)_{i,j} [M][N] per field."""
    N, M = p.N, p.M
    u = np.asarray(u, dtype=np.float64)
    assert u.shape == (3 * (N + 1) * M,)
    out = {}
    for f, name in enumerate(("zeta", "phi", "psi")):
        blk = u[f * (N + 1) * M:(f + 1) * (N + 1) * M].reshape(M, N + 1)
        out[name + "1"] = blk[:, 0].copy()
        out[name + "_x"] = blk[:, 1:].copy()
    return out


def integrate_x(f1: np.ndarray, fx: np.ndarray, dx: float) -> np.ndarray:
    """f_{i,j} = f_{1,j} + trapezoidal integral of f_x from x_1 to x_i (Section 3.1)."""
    M, N = fx.shape
    f = np.empty((M, N))
    f[:, 0] = f1
    for i in range(1, N):
        f[:, i] = f[:, i - 1] + 0.5 * dx * (fx[:, i - 1] + fx[:, i])
    return f


# ----------------------------------------------------------------------------- step 2
def d_dy(f: np.ndarray, dy: float, half: bool) -> np.ndarray:
    """y-derivative of a node field [M][N].

    Reading (the paper does not say how zeta_y and phi_y are obtained):
    central differences inside; (3 f_M - 4 f_{M-1} + f_{M-2}) / (2 dy) on the
    outer edge y_M; on a half domain the field is even in y, so the derivative
    on y = 0 is zero; on a full domain the mirror of the outer-edge stencil is
    used on y_1.
    """
    M = f.shape[0]
    g = np.empty_like(f)
    g[1:-1] = (f[2:] - f[:-2]) / (2.0 * dy)
    g[-1] = (3.0 * f[-1] - 4.0 * f[-2] + f[-3]) / (2.0 * dy)
    if half:
        g[0] = 0.0
    else:
        g[0] = (-3.0 * f[0] + 4.0 * f[1] - f[2]) / (2.0 * dy)
    return g


def d2_dy2(f: np.ndarray, dy: float, half: bool) -> np.ndarray:
    """Second y-derivative of a node field [M][N] (used by the surface-tension term).

    Reading (the paper only names the curvature term): second differences
    inside; on a half domain the field is even in y, so on y = 0 the mirror
    value f_2 stands for f_0; on an outer edge the one-sided second-order
    four-point stencil (2 f_M - 5 f_{M-1} + 4 f_{M-2} - f_{M-3}) / dy^2 (and its
    mirror on y_1 of a full domain).  Needs M >= 4.
    """
    g = np.empty_like(f)
    g[1:-1] = (f[2:] - 2.0 * f[1:-1] + f[:-2]) / (dy * dy)
    g[-1] = (2.0 * f[-1] - 5.0 * f[-2] + 4.0 * f[-3] - f[-4]) / (dy * dy)
    if half:
        g[0] = 2.0 * (f[1] - f[0]) / (dy * dy)
    else:
        g[0] = (2.0 * f[0] - 5.0 * f[1] + 4.0 * f[2] - f[3]) / (dy * dy)
    return g


@dataclasses.dataclass
class NodeFields:
    zeta: np.ndarray
    zeta_x: np.ndarray
    zeta_y: np.ndarray
    phi: np.ndarray
    phi_x: np.ndarray
    phi_y: np.ndarray
    psi: np.ndarray
    psi_x: np.ndarray


def reconstruct(p, u: np.ndarray) -> NodeFields:
    """Steps 1-2: node values of zeta, phi, psi and their x- and y-derivatives."""
    q = unpack(p, u)
    zeta = integrate_x(q["zeta1"], q["zeta_x"], p.dx)
    phi = integrate_x(q["phi1"], q["phi_x"], p.dx)
    psi = integrate_x(q["psi1"], q["psi_x"], p.dx)
    return NodeFields(zeta=zeta, zeta_x=q["zeta_x"], zeta_y=d_dy(zeta, p.dy, p.half_domain),
                      phi=phi, phi_x=q["phi_x"], phi_y=d_dy(phi, p.dy, p.half_domain),
                      psi=psi, psi_x=q["psi_x"])


# ----------------------------------------------------------------------------- step 3
def half_mesh(g: np.ndarray) -> np.ndarray:
    """Value at (x_{k+1/2}, y_l), k = 1..N-1, as the mean of nodes k and k+1."""
    return 0.5 * (g[:, :-1] + g[:, 1:])


# ----------------------------------------------------------------------------- step 4
def s2_integral(A, B, C, s1, s2, t1, t2):
    """Integral of (A s^2 + B s t + C t^2)^(-1/2) over [s1, s2] x [t1, t2].

    Uses the antiderivative printed in Section 3.1 (the closed form of I2''):
      G(s, t) = t/sqrt(A) ln(2As + Bt + 2 sqrt(A Q)) + s/sqrt(C) ln(2Ct + Bs + 2 sqrt(C Q)),
    evaluated at the four corners.  A term whose prefactor (t, resp. s) is zero
    is taken as zero, its limit (the logarithm may be singular there).
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)

    def G(s, t):
        s = np.broadcast_to(np.asarray(s, dtype=np.float64), A.shape)
        t = np.broadcast_to(np.asarray(t, dtype=np.float64), A.shape)
        Q = A * s * s + B * s * t + C * t * t
        out = np.zeros(A.shape)
        with np.errstate(divide="ignore", invalid="ignore"):
            a1 = t / np.sqrt(A) * np.log(2.0 * A * s + B * t + 2.0 * np.sqrt(A * Q))
            a2 = s / np.sqrt(C) * np.log(2.0 * C * t + B * s + 2.0 * np.sqrt(C * Q))
        out += np.where(t == 0.0, 0.0, a1)
        out += np.where(s == 0.0, 0.0, a2)
        return out

    return G(s2, t2) - G(s1, t2) - G(s2, t1) + G(s1, t1)


@dataclasses.dataclass
class Geometry:
    """A boundary z = a(x, y) on the node mesh: a, a_x, a_y [M][N]."""
    a: np.ndarray
    ax: np.ndarray
    ay: np.ndarray


@dataclasses.dataclass
class TargetSet:
    """Collocation points: position, elevation d, double-layer value D*, the
    quadratic form (A, B, C) of S2, the single-layer value sigma* that
    multiplies S2, and which surface the point lies on (0 = S, 1 = B)."""
    x: np.ndarray
    y: np.ndarray
    d: np.ndarray
    D: np.ndarray
    A: np.ndarray
    B: np.ndarray
    C: np.ndarray
    sigma: np.ndarray
    self_id: np.ndarray


def raw_sums(p, gS: Geometry, DS, sigS, gB: Geometry, DB, sigB, tg: TargetSet,
             absmode: bool = False) -> np.ndarray:
    """The five trapezoidal sums of bie_sums.c for every target, shape [T][5].

    absmode=True returns the sums of |term| instead (tolerance scales).
    """
    L = _clib.lib()
    c = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    arrs = [c(gS.a), c(gS.ax), c(gS.ay), c(DS), c(sigS), c(gB.a), c(gB.ax), c(gB.ay), c(DB), c(sigB)]
    tarr = [c(tg.x), c(tg.y), c(tg.d), c(tg.D), c(tg.A), c(tg.B), c(tg.C)]
    tself = np.ascontiguousarray(tg.self_id, dtype=np.int32)
    T = tarr[0].shape[0]
    out = np.zeros((T, 5))
    L.oracle_bie_sums(p.N, p.M, p.x1, p.dx, p.y1, p.dy, 1 if p.half_domain else 0,
                      *[_clib.dptr(a) for a in arrs], T, *[_clib.dptr(a) for a in tarr],
                      _clib.iptr(tself), 1 if absmode else 0, _clib.dptr(out))
    return out


def integration_rectangle(p):
    """The truncated domain: [x_1, x_N] x [y_1, y_M], mirrored to [-y_M, y_M] on a half domain."""
    xN = p.x1 + (p.N - 1) * p.dx
    yM = p.y1 + (p.M - 1) * p.dy
    ylo = -yM if p.half_domain else p.y1
    return p.x1, xN, ylo, yM


def bie_rows(p, gS: Geometry, DS, sigS, gB: Geometry, DB, sigB, tg: TargetSet) -> np.ndarray:
    """Boundary-integral rows 2 pi (D* ) = I1 + I2 + I3 + I4 as residuals (Section 2.2).

    For a target on S:  I1 + I2' + sigma* iint S2 + I3 + I4 - 2 pi D*,
    for a target on B:  the same equation with the target moved to the bottom.
    With the sums of raw_sums this is
      dlS + slS - dlB - slB - sigma* s2 + sigma* iint S2 - 2 pi D*,
    where the bottom terms carry the outward-normal signs of Green's identity
    (double layer -K1 as printed for I3; single layer with density -beta_x, the
    reading noted in the module docstring).
    """
    raw = raw_sums(p, gS, DS, sigS, gB, DB, sigB, tg)
    xlo, xhi, ylo, yhi = integration_rectangle(p)
    I2pp = s2_integral(tg.A, tg.B, tg.C, xlo - tg.x, xhi - tg.x, ylo - tg.y, yhi - tg.y)
    return (raw[:, 0] + raw[:, 1] - raw[:, 2] - raw[:, 3]
            - tg.sigma * raw[:, 4] + tg.sigma * I2pp - TWO_PI * tg.D)


def collocation_points(p):
    """Half-mesh points x*_k = x_1 + (k - 1/2) dx, y*_l = y_l as [M][N-1] arrays."""
    xs = p.x1 + (np.arange(p.N - 1) + 0.5) * p.dx
    ys = p.y1 + np.arange(p.M) * p.dy
    X, Y = np.meshgrid(xs, ys)
    return X, Y


def targets_from_nodes(p, g: Geometry, D: np.ndarray, sig_slot: np.ndarray, which: str) -> TargetSet:
    """Collocation data from node arrays of one boundary (Section 3.1, half-mesh points).

    g is the boundary the points lie on, D its double-layer value and sig_slot
    its single-layer slot (zeta_x on S, beta_x on B).  The value multiplying S2
    is the single-layer density as it enters the row: +slot on S, -slot on B.
    """
    X, Y = collocation_points(p)
    a, ax, ay = half_mesh(g.a), half_mesh(g.ax), half_mesh(g.ay)
    sign = 1.0 if which == "S" else -1.0
    f = lambda v: np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1))
    return TargetSet(x=f(X), y=f(Y), d=f(a), D=f(half_mesh(D)), A=f(1.0 + ax * ax), B=f(2.0 * ax * ay),
                     C=f(1.0 + ay * ay), sigma=f(sign * half_mesh(sig_slot)),
                     self_id=np.full(X.size, 0 if which == "S" else 1, dtype=np.int32))


def targets_from_fields(p, nf: NodeFields, which: str) -> TargetSet:
    """Target data for the surface rows (which='S') or the bottom rows (which='B')."""
    gS, DS, sigS, gB, DB, sigB = surface_and_bottom(p, nf)
    if which == "S":
        return targets_from_nodes(p, gS, DS, sigS, "S")
    return targets_from_nodes(p, gB, DB, sigB, "B")


def subset(tg: TargetSet, idx: np.ndarray) -> TargetSet:
    return TargetSet(**{k: np.ascontiguousarray(getattr(tg, k)[idx]) for k in
                        ("x", "y", "d", "D", "A", "B", "C", "sigma", "self_id")})


# ----------------------------------------------------------------------------- step 5
def curvature(p, nf: NodeFields) -> np.ndarray:
    """Twice the mean curvature of z = zeta at the half-mesh points,
    K = div(grad zeta / sqrt(1 + |grad zeta|^2))
      = [(1 + zy^2) zxx - 2 zx zy zxy + (1 + zx^2) zyy] / (1 + zx^2 + zy^2)^(3/2)
    (Section 6: surface tension times mean curvature enters Bernoulli's equation).
    Reading: zx*, zy* are the half-mesh means used by the dynamic condition; zxx*
    and zxy* the differences of the node zeta_x and zeta_y across the half-mesh
    cell, (g_{k+1} - g_k) / dx; zyy* the half-mesh mean of the node second
    y-differences (d2_dy2)."""
    zx, zy = half_mesh(nf.zeta_x), half_mesh(nf.zeta_y)
    zxx = (nf.zeta_x[:, 1:] - nf.zeta_x[:, :-1]) / p.dx
    zxy = (nf.zeta_y[:, 1:] - nf.zeta_y[:, :-1]) / p.dx
    zyy = half_mesh(d2_dy2(nf.zeta, p.dy, p.half_domain))
    q = 1.0 + zx * zx + zy * zy
    return ((1.0 + zy * zy) * zxx - 2.0 * zx * zy * zxy + (1.0 + zx * zx) * zyy) / (q * np.sqrt(q))


def dynamic_rows(p, nf: NodeFields) -> np.ndarray:
    """F1 at the half-mesh points: eq. (new_finite_dynamic) written as a residual,
    with the surface-tension term -tau K when tau != 0 (Section 6; tau = T / (rho U^2 H),
    the pressure jump T K across the surface)."""
    zx, zy = half_mesh(nf.zeta_x), half_mesh(nf.zeta_y)
    px, py = half_mesh(nf.phi_x), half_mesh(nf.phi_y)
    z = half_mesh(nf.zeta)
    kin = 0.5 * ((1.0 + zx * zx) * py * py + (1.0 + zy * zy) * px * px - 2.0 * zx * zy * px * py) \
        / (1.0 + zx * zx + zy * zy)
    F1 = kin + z / (p.froude * p.froude) - 0.5
    tau = getattr(p, "tau", 0.0)
    if tau != 0.0:
        F1 = F1 - tau * curvature(p, nf)
    return F1


# ----------------------------------------------------------------------------- step 6
def radiation_rows(p, nf: NodeFields) -> Dict[str, np.ndarray]:
    """F3..F6, F8, F9 per slice (eqs. (scullen1)-(scullen6) as in Appendix B).

    The second x-derivative at x_1 is the forward difference of f_x.
    """
    n, x1, dx = p.n_decay, p.x1, p.dx
    out = {}
    out["F5"] = x1 * nf.zeta_x[:, 0] + n * nf.zeta[:, 0]
    out["F6"] = x1 * (nf.zeta_x[:, 1] - nf.zeta_x[:, 0]) / dx + n * nf.zeta_x[:, 0]
    out["F3"] = x1 * (nf.phi_x[:, 0] - 1.0) + n * (nf.phi[:, 0] - x1)
    out["F4"] = x1 * (nf.phi_x[:, 1] - nf.phi_x[:, 0]) / dx + n * (nf.phi_x[:, 0] - 1.0)
    out["F8"] = x1 * (nf.psi_x[:, 0] - 1.0) + n * (nf.psi[:, 0] - x1)
    out["F9"] = x1 * (nf.psi_x[:, 1] - nf.psi_x[:, 0]) / dx + n * (nf.psi_x[:, 0] - 1.0)
    return out


# ----------------------------------------------------------------------------- step 7
def assemble(p, F1, F2, F7, rad) -> np.ndarray:
    """Row order of Appendix B: per slice [F5, F6, F1(.)], then [F3, F4, F2(.)], then [F8, F9, F7(.)]."""
    N, M = p.N, p.M
    out = np.empty(3 * (N + 1) * M)
    for blk, (ra, rb, rows) in enumerate((("F5", "F6", F1), ("F3", "F4", F2), ("F8", "F9", F7))):
        v = out[blk * (N + 1) * M:(blk + 1) * (N + 1) * M].reshape(M, N + 1)
        v[:, 0] = rad[ra]
        v[:, 1] = rad[rb]
        v[:, 2:] = rows.reshape(M, N - 1)
    return out


def surface_and_bottom(p, nf: NodeFields):
    """Geometry and layer densities of both boundaries.

    Free surface: double-layer value phi - x, single-layer density zeta_x.
    Bottom: double-layer value psi - x, single-layer slot beta_x (entering
    with a minus sign in bie_rows).
    """
    X = np.broadcast_to(p.x(), nf.zeta.shape)
    gS = Geometry(nf.zeta, nf.zeta_x, nf.zeta_y)
    gB = Geometry(p.beta, p.beta_x, p.beta_y)
    return gS, nf.phi - X, nf.zeta_x, gB, nf.psi - X, p.beta_x


def residual(p, u: np.ndarray) -> np.ndarray:
    """F(u), length 3 (N+1) M, in the order of Appendix B."""
    nf = reconstruct(p, u)
    gS, DS, sigS, gB, DB, sigB = surface_and_bottom(p, nf)
    F2 = bie_rows(p, gS, DS, sigS, gB, DB, sigB, targets_from_fields(p, nf, "S"))
    F7 = bie_rows(p, gS, DS, sigS, gB, DB, sigB, targets_from_fields(p, nf, "B"))
    return assemble(p, dynamic_rows(p, nf), F2, F7, radiation_rows(p, nf))


def row_index(p, block: int, l: int, k: int) -> int:
    """Position in F of the collocation row (k, l) (0-based) of block 0 (F1), 1 (F2) or 2 (F7)."""
    return block * (p.N + 1) * p.M + l * (p.N + 1) + 2 + k


def residual_rows(p, u: np.ndarray, rows: Sequence[int]) -> np.ndarray:
    """Selected entries of F(u) (any row kind), computing only the sums they need."""
    rows = np.asarray(rows, dtype=np.int64)
    nf = reconstruct(p, u)
    gS, DS, sigS, gB, DB, sigB = surface_and_bottom(p, nf)
    N, M = p.N, p.M
    nb = (N + 1) * M
    out = np.empty(rows.shape[0])
    F1 = dynamic_rows(p, nf).reshape(-1)
    rad = radiation_rows(p, nf)
    names = (("F5", "F6"), ("F3", "F4"), ("F8", "F9"))
    bie_needed = {1: [], 2: []}
    for q, r in enumerate(rows):
        blk, rem = divmod(int(r), nb)
        l, c = divmod(rem, N + 1)
        if c < 2:
            out[q] = rad[names[blk][c]][l]
        elif blk == 0:
            out[q] = F1[l * (N - 1) + c - 2]
        else:
            bie_needed[blk].append((q, l * (N - 1) + c - 2))
    for blk, which in ((1, "S"), (2, "B")):
        if bie_needed[blk]:
            qs = np.array([a for a, _ in bie_needed[blk]])
            ts = np.array([b for _, b in bie_needed[blk]])
            tg = subset(targets_from_fields(p, nf, which), ts)
            out[qs] = bie_rows(p, gS, DS, sigS, gB, DB, sigB, tg)
    return out


def term_magnitude_rows(p, u: np.ndarray, rows: Optional[Sequence[int]] = None) -> np.ndarray:
    """Scale of each row of F for comparison tolerances: 1 + sum of |terms|.

    Boundary-integral rows: the sums of |term| over all pairs plus
    |sigma*| (s2 + |iint S2|) + 2 pi |D*|.  Pointwise rows: 1 + the largest
    magnitude among their few terms (bounded by a generous constant).
    rows: only these entries (in that order), computing only the sums they need.
    """
    nf = reconstruct(p, u)
    gS, DS, sigS, gB, DB, sigB = surface_and_bottom(p, nf)
    N, M = p.N, p.M
    nb = (N + 1) * M
    sel = np.arange(3 * nb) if rows is None else np.asarray(rows, dtype=np.int64)
    scale = np.full(sel.shape[0], 1.0 + abs(p.x1) * 4.0 / p.dx)
    xlo, xhi, ylo, yhi = integration_rectangle(p)
    blk, rem = np.divmod(sel, nb)
    l, c = np.divmod(rem, N + 1)
    for b, which in ((1, "S"), (2, "B")):
        q = np.nonzero((blk == b) & (c >= 2))[0]
        if q.size == 0:
            continue
        tg = subset(targets_from_fields(p, nf, which), l[q] * (N - 1) + c[q] - 2)
        raw = raw_sums(p, gS, DS, sigS, gB, DB, sigB, tg, absmode=True)
        I2pp = s2_integral(tg.A, tg.B, tg.C, xlo - tg.x, xhi - tg.x, ylo - tg.y, yhi - tg.y)
        mag = raw[:, :4].sum(axis=1) + np.abs(tg.sigma) * (raw[:, 4] + np.abs(I2pp)) + TWO_PI * np.abs(tg.D)
        scale[q] = 1.0 + mag
    return scale
