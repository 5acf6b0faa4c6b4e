"""Oracle of the bottom pressure and the force on the topography (Section 2.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain FP64.

Once the discrete problem is solved, Bernoulli's equation on the bottom
z = beta(x, y) gives the pressure there from the bottom potential psi, the way
eq. (new_finite_dynamic) gives the free-surface condition from phi (Section 2.1,
eq. (bottompressure)):
    p = 1/2 - 1/2 [(1 + b_x^2) psi_y^2 + (1 + b_y^2) psi_x^2 - 2 b_x b_y psi_x psi_y]
              / (1 + b_x^2 + b_y^2) - beta / F^2.
The paper notes that the total force on the topography follows by integrating
this pressure over the bottom; it gives no discrete rule.  Readings:
  * psi at the nodes is the trapezoidal x-integral of the unknowns and psi_y the
    y-difference of it, exactly as for phi in the residual (the same
    reconstruction, step 1-2 of oracle.residual);
  * the fluid pushes on the bottom along the fluid's outward normal there,
    (beta_x, beta_y, -1) / sqrt(1 + |grad beta|^2), and the area element is
    sqrt(1 + |grad beta|^2) dx dy, so the force is the plan-area integral of
    p (beta_x, beta_y, -1);
  * the undisturbed pressure of the uniform stream on the flat bottom, 1 / F^2,
    is subtracted before integrating (its integral over the flat part only
    measures the size of the truncated domain);
  * the plan-area integral is the trapezoidal rule on the mesh (weights
    dx dy c_i c_j), over the mirrored mesh on a half domain (twice the half sum,
    the symmetry row counted once; the y-force is zero there by symmetry).
"""
from __future__ import annotations

import numpy as np

from . import residual as R


def pressure_from_gradient(beta, bx, by, psi_x, psi_y, froude):
    """eq. (bottompressure) at points where the bottom slopes and psi's derivatives are known."""
    kin = 0.5 * ((1.0 + bx * bx) * psi_y * psi_y + (1.0 + by * by) * psi_x * psi_x
                 - 2.0 * bx * by * psi_x * psi_y) / (1.0 + bx * bx + by * by)
    return 0.5 - kin - beta / (froude * froude)


def bottom_pressure(p, u: np.ndarray) -> np.ndarray:
    """p at the bottom nodes [M][N] for the unknown vector u."""
    nf = R.reconstruct(p, u)
    psi_y = R.d_dy(nf.psi, p.dy, p.half_domain)
    return pressure_from_gradient(p.beta, p.beta_x, p.beta_y, nf.psi_x, psi_y, p.froude)


def trapezoid_weights(p) -> np.ndarray:
    """dx dy c_i c_j on the node mesh, c = 1/2 on the edges (Section 3.1)."""
    ci = np.ones(p.N)
    ci[[0, -1]] = 0.5
    cj = np.ones(p.M)
    cj[[0, -1]] = 0.5
    return p.dx * p.dy * np.outer(cj, ci)


def bottom_force(p, pres: np.ndarray) -> np.ndarray:
    """(Fx, Fy, Fz): the plan-area integral of (p - 1/F^2) (beta_x, beta_y, -1)."""
    w = trapezoid_weights(p)
    dp = pres - 1.0 / (p.froude * p.froude)
    f = np.array([(w * dp * p.beta_x).sum(), (w * dp * p.beta_y).sum(), -(w * dp).sum()])
    if p.half_domain:
        f = 2.0 * f
        f[1] = 0.0
    return f
