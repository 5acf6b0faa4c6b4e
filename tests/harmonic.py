"""Harmonic test fields for Green's-identity checks of the boundary-integral rows.

u(X) = sum_m q_m / |X - X_m| with all sources outside the fluid layer
(above the free surface or below the bottom).  The charges cancel the first
three vertical moments, so u and its gradient decay like rho^-5 horizontally
and truncating the mesh costs little.
"""
import numpy as np


def multipole_sources(above=(0.6, 1.0), below=(-1.6, -2.0), xc=0.0):
    zs = np.array(list(above) + list(below), dtype=np.float64)
    # q_0 = 1; sum q = 0, sum q z = 0, sum q z^2 = 0 fix the other three.
    Amat = np.vstack([np.ones(3), zs[1:], zs[1:] ** 2])
    rhs = -np.array([1.0, zs[0], zs[0] ** 2])
    q = np.concatenate([[1.0], np.linalg.solve(Amat, rhs)])
    pos = np.stack([np.full(4, xc), np.zeros(4), zs], axis=1)
    return pos, q


def field(pos, q, X, Y, Z):
    """u and its gradient at the points (X, Y, Z) (same shapes)."""
    u = np.zeros_like(X)
    gx = np.zeros_like(X)
    gy = np.zeros_like(X)
    gz = np.zeros_like(X)
    for (px, py, pz), qm in zip(pos, q):
        rx, ry, rz = X - px, Y - py, Z - pz
        r = np.sqrt(rx * rx + ry * ry + rz * rz)
        u += qm / r
        r3 = r ** 3
        gx -= qm * rx / r3
        gy -= qm * ry / r3
        gz -= qm * rz / r3
    return u, gx, gy, gz
