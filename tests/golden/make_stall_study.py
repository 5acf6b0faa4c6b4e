#!/usr/bin/env python3
"""Why Newton stalls for some subcritical problems: an oracle-only study.

Calls only the CPU oracle (and the shared input generators).  For the bump
0.2 exp(-(x^2+y^2)) at F = 0.7 on the working domain x in [-30, 30],
y in [0, 20] (half domain), on two meshes of that domain -- 61 x 21, where
Newton converges, and 91 x 31, where it stalls -- it runs damped Newton with
right-preconditioned GMRES from the discrete linear start (Section 3.2) and,
at the last iterate u, forms the Jacobian J(u) of the nonlinear residual by
central differences of F (Section 3.1) and the linear Jacobian J~ (Section 4.2),
and reports:
  * the Newton history of ||F||_inf and how Newton ended;
  * the smallest singular values of A = J(u) J~^-1 (A = I where the problem is
    linear; a value near zero means J(u) is singular in a direction J~ is not),
    and of J~ itself;
  * the share of F(u) along A's left singular vectors of those values.
Writes tests/golden/oracle_stall_study_F0.7.json.  About 15 minutes on 8 cores.

    python tests/golden/make_stall_study.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import scipy.linalg as sla  # noqa: E402

from oracle import jfnk as OJ  # noqa: E402
from oracle import linear as Lin  # noqa: E402
from oracle import residual as R  # noqa: E402
from paper_1709_08803_amd import workloads as W  # noqa: E402


def fd_jacobian(p, u, h=1e-6):
    n = u.size
    J = np.empty((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = h * max(1.0, abs(u[c]))
        J[:, c] = (R.residual(p, u + e) - R.residual(p, u - e)) / (2.0 * e[c])
    return J


def study(N, M, froude=0.7, k=6):
    p = W.working(froude, N, M)
    t0 = time.time()
    Jl = Lin.jacobian(p)
    u0 = W.uniform_stream(p) - np.linalg.solve(Jl, Lin.forcing(p))
    lu_p = sla.lu_factor(Lin.banded(p, Jl, Lin.band_halfwidth(p.M)))

    class Pre:
        def apply(self, r):
            return sla.lu_solve(lu_p, r)
    res = OJ.newton_krylov(p, u0, precond=Pre(), ftol=1e-11, max_newton=15)
    F = R.residual(p, res.u)
    print(f"{N}x{M}: Newton converged={res.converged} history {['%.2e' % h for h in res.history]} "
          f"({time.time() - t0:.0f} s)", flush=True)
    J = fd_jacobian(p, res.u)
    print(f"{N}x{M}: FD Jacobian formed ({time.time() - t0:.0f} s)", flush=True)
    A = J @ np.linalg.inv(Jl)
    U, S, Vt = np.linalg.svd(A)
    Sl = np.linalg.svd(Jl, compute_uv=False)
    proj = np.abs(U[:, -k:].T @ F) / np.linalg.norm(F)
    return dict(mesh=f"{N}x{M}", froude=froude, converged=bool(res.converged), newton_iters=res.newton_iters,
                gmres_iters=res.gmres_iters, history_inf=[float(h) for h in res.history],
                final_inf=float(np.abs(F).max()),
                smallest_singular_values_of_J_times_inverse_linear_J=[float(s) for s in S[-k:][::-1]],
                smallest_singular_values_of_linear_J=[float(s) for s in Sl[-k:][::-1]],
                share_of_F_along_those_left_vectors=[float(x) for x in proj[::-1]],
                seconds=time.time() - t0)


if __name__ == "__main__":
    recs = [study(61, 21), study(91, 31)]
    out = os.path.join(HERE, "oracle_stall_study_F0.7.json")
    with open(out, "w") as f:
        json.dump(dict(problem="half domain x in [-30, 30], y in [0, 20], bump 0.2 exp(-(x^2+y^2)), F = 0.7",
                       studies=recs), f, indent=1)
    print("wrote", out, flush=True)
