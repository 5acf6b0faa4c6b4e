#!/usr/bin/env python3
"""Write the oracle's converged solutions of the 181 x 61 working problems.

Calls only the CPU oracle (and the shared input generators): the discrete linear
start u_lin = u0 - J~^-1 F_lin(u0) by dense LU, then damped Newton with
right-preconditioned GMRES(30) (Section 3.2), preconditioned by the dense LU of
the slice-banded J~ (Section 4.2).  Stops at ||F||_inf <= 1e-11.

Output: tests/golden/working_181x61_F<F>.npz with the full unknown vector u
(FP64, 3 (N+1) M entries in the order of Section 3.1), the Newton history and
the band half-width used.  Needs about 20 GB of host memory and a few minutes
per Froude number on 8 cores.

    python tests/golden/make_working_solutions.py 1.4 [0.7 ...]
"""
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
from paper_1709_08803_amd import workloads as W  # noqa: E402

BAND = 10


class _LU:
    def __init__(self, lu):
        self.lu = lu

    def apply(self, r):
        return sla.lu_solve(self.lu, r)


def solve(froude: float, ftol: float = 1e-11):
    p = W.working(froude)
    t0 = time.time()
    J = Lin.jacobian(p)
    f0 = Lin.forcing(p)
    P = Lin.banded(p, J, BAND)
    print(f"F={froude}: J~ and banded P formed ({time.time() - t0:.0f} s)", flush=True)
    lu = sla.lu_factor(J, overwrite_a=True, check_finite=False)
    del J
    u = W.uniform_stream(p) - sla.lu_solve(lu, f0)
    del lu
    print(f"F={froude}: linear start ({time.time() - t0:.0f} s)", flush=True)
    pre = _LU(sla.lu_factor(P, overwrite_a=True, check_finite=False))
    del P
    print(f"F={froude}: preconditioner factored ({time.time() - t0:.0f} s)", flush=True)
    res = OJ.newton_krylov(p, u, precond=pre, ftol=ftol)
    print(f"F={froude}: converged={res.converged} newton={res.newton_iters} gmres={res.gmres_iters} "
          f"history={['%.2e' % h for h in res.history]} ({time.time() - t0:.0f} s)", flush=True)
    if not res.converged:
        raise SystemExit(f"the oracle did not converge at F={froude}")
    out = os.path.join(HERE, f"working_181x61_F{froude}.npz")
    np.savez_compressed(out, u=res.u, history=np.array(res.history), band=BAND, ftol=ftol,
                        newton_iters=res.newton_iters, gmres_iters=res.gmres_iters)
    print("wrote", out, flush=True)


if __name__ == "__main__":
    for a in sys.argv[1:] or ["1.4"]:
        solve(float(a))
