"""Oracle solver: damped inexact Newton with right-preconditioned GMRES (Section 3.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, textbook
algorithms:
  * GMRES(m) with right preconditioning (Saad & Schultz): Arnoldi with modified
    Gram-Schmidt, Givens rotations, restarts from the true residual;
  * the Jacobian action J(u) v as the first-order difference quotient
    (F(u + h v) - F(u)) / h with h = sqrt(eps) (1 + |u|) / |v| (Reading: the
    paper asks only for "a sufficiently small shift");
  * Newton steps u <- u + mu du with mu halved until
    |F(u + mu du)|_2 <= (1 - 1e-4 mu) |F(u)|_2 (Reading of "a simple line
    search ... sufficient decrease").
Because the converged solution of F(u) = 0 does not depend on the route, the
solver settings only affect iteration counts.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

from . import residual as R


def gmres_right(A: Callable[[np.ndarray], np.ndarray], b: np.ndarray,
                Minv: Optional[Callable[[np.ndarray], np.ndarray]], rtol: float, restart: int = 30,
                max_restarts: int = 10):
    """Solve A x = b; returns (x, iterations, relative residual estimate)."""
    n = b.size
    Minv = Minv or (lambda v: v)
    x = np.zeros(n)
    r = b.copy()
    beta0 = np.linalg.norm(r)
    if beta0 == 0.0:
        return x, 0, 0.0
    beta = beta0
    its = 0
    rel = 1.0
    for cycle in range(max_restarts + 1):
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        jend = 0
        done = False
        for j in range(restart):
            Z[j] = Minv(V[j])
            w = A(Z[j])
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):  # apply previous rotations
                a, c = H[i, j], H[i + 1, j]
                H[i, j], H[i + 1, j] = cs[i] * a + sn[i] * c, -sn[i] * a + cs[i] * c
            a, c = H[j, j], H[j + 1, j]
            rr = math.hypot(a, c)
            cs[j], sn[j] = (a / rr, c / rr) if rr > 0 else (1.0, 0.0)
            H[j, j], H[j + 1, j] = rr, 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            jend = j + 1
            rel = abs(g[j + 1]) / beta0
            if rel <= rtol or H[j + 1, j] == 0.0 and rr == 0.0:
                done = True
                break
        y = np.linalg.solve(np.triu(H[:jend, :jend]), g[:jend])
        x = x + Z[:jend].T @ y
        if done or cycle == max_restarts:
            break
        r = b - A(x)
        beta = np.linalg.norm(r)
        rel = beta / beta0
        if rel <= rtol:
            break
    return x, its, rel


@dataclasses.dataclass
class NewtonResult:
    u: np.ndarray
    converged: bool
    newton_iters: int
    gmres_iters: int
    history: List[float]


def newton_krylov(p, u0: np.ndarray, precond=None, ftol: float = 1e-10, gmres_rtol: float = 1e-8,
                  restart: int = 30, max_restarts: int = 10, max_newton: int = 30,
                  max_backtracks: int = 20) -> NewtonResult:
    """Solve F(u) = 0 from u0 (Section 3.2).  precond: object with .apply(r) = P^-1 r, or None."""
    u = np.array(u0, dtype=np.float64)
    F = R.residual(p, u)
    fn = np.linalg.norm(F)
    hist = [float(np.abs(F).max())]
    gm = 0
    eps = 2.0 ** -52
    for k in range(max_newton + 1):
        if np.abs(F).max() <= ftol:
            return NewtonResult(u, True, k, gm, hist)
        if k == max_newton:
            break
        Fk, uk = F, u

        def Jv(v, uk=uk, Fk=Fk):
            nv = np.linalg.norm(v)
            if nv == 0.0:
                return np.zeros_like(v)
            h = math.sqrt(eps) * (1.0 + np.linalg.norm(uk)) / nv
            return (R.residual(p, uk + h * v) - Fk) / h

        du, its, _ = gmres_right(Jv, -F, precond.apply if precond is not None else None, gmres_rtol, restart,
                                 max_restarts)
        gm += its
        mu = 1.0
        for _ in range(max_backtracks + 1):
            ut = u + mu * du
            Ft = R.residual(p, ut)
            ft = np.linalg.norm(Ft)
            if np.isfinite(ft) and ft <= (1.0 - 1e-4 * mu) * fn:
                break
            mu *= 0.5
        else:
            return NewtonResult(u, False, k + 1, gm, hist)
        u, F, fn = ut, Ft, ft
        hist.append(float(np.abs(F).max()))
    return NewtonResult(u, False, max_newton, gm, hist)
