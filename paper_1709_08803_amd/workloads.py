"""Seeded synthetic inputs for the free-surface boundary-integral problem.

This module holds only input generation: the mesh description, bottom
topographies of the Gaussian form of eq. (bottom) in Section 2.1 (and sums of
such bumps), the uniform-stream state, and seeded perturbations used as test
states.  It contains none of the method's arithmetic (no kernels, no
quadrature, no residual) so that both the GPU path and the CPU oracle can draw
identical inputs from it without sharing any of the computation.

Layout conventions (shared interface, Section 3.1, eq. (unknowns)):
  * node arrays are [M][N] (row j = y_j, column i = x_i, x fastest), float64;
  * the unknown vector u has 3 (N+1) M entries: for each field f in
    (zeta, phi, psi) a block of M slices, slice j = [f_{1,j}, (f_x)_{1..N,j}].
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

RADIATION_DECAY = 0.05  # upstream decay rate n of the radiation condition (Section 3.1)


@dataclasses.dataclass
class Problem:
    """One discrete problem: mesh, Froude number and bottom topography.

    x_i = x1 + i dx (i = 0..N-1), y_j = y1 + j dy (j = 0..M-1).
    half_domain = True means the data are even in y about y = 0 and only
    y >= 0 is stored (y1 must be 0); the mirror half is implied.
    beta, beta_x, beta_y are node arrays [M][N] of the bottom z = beta(x, y).
    tau is the surface-tension parameter T / (rho U^2 H) (0: gravity waves only).
    """
    N: int
    M: int
    x1: float
    dx: float
    y1: float
    dy: float
    froude: float
    beta: np.ndarray
    beta_x: np.ndarray
    beta_y: np.ndarray
    half_domain: bool = True
    n_decay: float = RADIATION_DECAY
    name: str = ""
    tau: float = 0.0

    @property
    def n_unknowns(self) -> int:
        return 3 * (self.N + 1) * self.M

    @property
    def n_block(self) -> int:
        return (self.N + 1) * self.M

    def x(self) -> np.ndarray:
        return self.x1 + self.dx * np.arange(self.N)

    def y(self) -> np.ndarray:
        return self.y1 + self.dy * np.arange(self.M)

    def pairs_per_eval(self) -> int:
        """Collocation-point x source-node x image interactions of one residual."""
        images = 2 if self.half_domain else 1
        return 2 * (self.N - 1) * self.M * 2 * self.N * self.M * images


# ---------------------------------------------------------------- topography
@dataclasses.dataclass
class Bump:
    """beta + 1 contribution  h * exp(-((x-cx)^2/wx^2 + (y-cy)^2/wy^2)).

    wy = inf gives a transverse ridge uniform in y.  With wx = wy = sqrt(2)
    delta this is the Gaussian of eq. (bottom) with epsilon = h.
    """
    h: float
    wx: float
    wy: float
    cx: float = 0.0
    cy: float = 0.0


def topography(bumps: Sequence[Bump], x: np.ndarray, y: np.ndarray,
               mirror: bool) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """beta, beta_x, beta_y on the node grid (analytic derivatives).

    mirror=True adds the image of every bump with cy != 0 at -cy, so that the
    field is even in y (required on a half domain).
    """
    X, Y = np.meshgrid(x, y)  # [M][N]
    b = np.full_like(X, -1.0)
    bx = np.zeros_like(X)
    by = np.zeros_like(X)
    terms = list(bumps)
    if mirror:
        terms = terms + [dataclasses.replace(t, cy=-t.cy) for t in bumps if t.cy != 0.0]
    for t in terms:
        ax = (X - t.cx) / t.wx
        if math.isinf(t.wy):
            ay = np.zeros_like(Y)
            gy = np.zeros_like(Y)
        else:
            ay = (Y - t.cy) / t.wy
            gy = -2.0 * (Y - t.cy) / (t.wy * t.wy)
        g = t.h * np.exp(-(ax * ax + ay * ay))
        b += g
        bx += g * (-2.0 * (X - t.cx) / (t.wx * t.wx))
        by += g * gy
    return b, bx, by


def make_problem(N: int, M: int, xlo: float, xhi: float, ylo: float, yhi: float,
                 froude: float, bumps: Sequence[Bump], half_domain: bool = True,
                 name: str = "", tau: float = 0.0) -> Problem:
    dx = (xhi - xlo) / (N - 1)
    dy = (yhi - ylo) / (M - 1)
    if half_domain and ylo != 0.0:
        raise ValueError("a half domain starts at y = 0")
    x = xlo + dx * np.arange(N)
    y = ylo + dy * np.arange(M)
    b, bx, by = topography(bumps, x, y, mirror=half_domain)
    return Problem(N=N, M=M, x1=xlo, dx=dx, y1=ylo, dy=dy, froude=froude,
                   beta=b, beta_x=bx, beta_y=by, half_domain=half_domain, name=name, tau=tau)


# ---------------------------------------------------------------- named workloads
def tiny(froude: float = 0.7) -> Problem:
    """31 x 11 half domain, x in [-16, 16], y in [0, 10], bump 0.1 exp(-(x^2+y^2))."""
    return make_problem(31, 11, -16.0, 16.0, 0.0, 10.0, froude,
                        [Bump(0.1, 1.0, 1.0)], name="tiny-31x11")


def working(froude: float = 0.7, N: int = 181, M: int = 61) -> Problem:
    """181 x 61 half domain, x in [-30, 30], y in [0, 20], bump 0.2 exp(-(x^2+y^2))."""
    return make_problem(N, M, -30.0, 30.0, 0.0, 20.0, froude,
                        [Bump(0.2, 1.0, 1.0)], name=f"working-{N}x{M}")


def sweep_instances(count: int, seed: int, n_choices: Optional[Sequence[int]] = None,
                    fixed_n: Optional[int] = None, domain: Tuple[float, float, float] = (-30.0, 30.0, 20.0),
                    height: Tuple[float, float] = (0.05, 0.3), froude: Tuple[float, float] = (0.5, 2.0),
                    width: Tuple[float, float] = (0.5, 2.0), kinds: Sequence[int] = (0, 1, 2)) -> List[Problem]:
    """Seeded parameter sweep: uneven grids, F ~ U[0.5, 2], three topography kinds.

    Grids: N drawn from {61, 64, ..., 181} (N = 1 mod 3), M = (N-1)/3 + 1 over
    x in [-30, 30], y in [0, 20] (so dx = dy).  fixed_n forces one grid size;
    domain = (x_lo, x_hi, y_hi), height, froude and width ranges and the set of
    topography kinds override the defaults.
    Topography kinds: a single Gaussian h exp(-(x^2+y^2)/w^2); a transverse
    ridge h exp(-x^2/w^2); two inline bumps at (0, 0) and (d, 0); with
    h ~ U[0.05, 0.3], w ~ U[0.5, 2], d ~ U[4, 12].
    """
    rng = np.random.default_rng(seed)
    if n_choices is None:
        n_choices = list(range(61, 182, 3))
    out = []
    for c in range(count):
        N = int(fixed_n) if fixed_n is not None else int(rng.choice(n_choices))
        M = (N - 1) // 3 + 1
        F = float(rng.uniform(*froude))
        kind = int(kinds[int(rng.integers(0, len(kinds)))])
        h = float(rng.uniform(*height))
        w = float(rng.uniform(*width))
        d = float(rng.uniform(4.0, 12.0))
        if kind == 0:
            bumps = [Bump(h, w, w)]
        elif kind == 1:
            bumps = [Bump(h, w, math.inf)]
        else:
            bumps = [Bump(h, w, w), Bump(h, w, w, cx=d)]
        out.append(make_problem(N, M, domain[0], domain[1], 0.0, domain[2], F, bumps,
                                name=f"sweep{seed}-{c}-k{kind}-{N}x{M}"))
    return out


# ---------------------------------------------------------------- states
def uniform_stream(p: Problem) -> np.ndarray:
    """u for zeta = 0, phi = psi = x (undisturbed stream) in the layout above."""
    N, M = p.N, p.M
    u = np.zeros(3 * (N + 1) * M)
    for f in (1, 2):
        blk = u[f * (N + 1) * M:(f + 1) * (N + 1) * M].reshape(M, N + 1)
        blk[:, 0] = p.x1
        blk[:, 1:] = 1.0
    return u


def perturbed_state(p: Problem, seed: int, amp: float = 0.05) -> np.ndarray:
    """Uniform stream plus a seeded smooth wave-like perturbation (even in y).

    zeta_x, phi_x - 1, psi_x - 1 get sums of a few decaying cosine wave packets
    of amplitude ~amp; the upstream values get small offsets.  Used only as a
    realistic, reproducible evaluation point of the residual.
    """
    rng = np.random.default_rng(seed)
    N, M = p.N, p.M
    X, Y = np.meshgrid(p.x(), p.y())
    u = uniform_stream(p)
    for f in range(3):
        fx = np.zeros_like(X)
        for _ in range(3):
            a = amp * rng.uniform(0.3, 1.0) * (0.5 if f == 2 else 1.0)
            k = rng.uniform(0.8, 2.5)
            ky = rng.uniform(0.0, 1.0)
            x0 = rng.uniform(-5.0, 5.0)
            s = rng.uniform(3.0, 8.0)
            fx += a * np.cos(k * X + rng.uniform(0, 2 * np.pi)) * np.cos(ky * Y) \
                * np.exp(-((X - x0) ** 2 + Y ** 2) / (s * s))
        blk = u[f * (N + 1) * M:(f + 1) * (N + 1) * M].reshape(M, N + 1)
        blk[:, 1:] += fx
        blk[:, 0] += amp * 0.1 * rng.uniform(-1.0, 1.0)
    return u


def random_direction(p: Problem, seed: int) -> np.ndarray:
    """A seeded unit-scale direction vector (for Jacobian-vector products)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(p.n_unknowns)
