#!/usr/bin/env python3
"""Write the oracle's converged solutions of held-out problems of the learned-start
experiment at 121 x 41: the first problems of workloads.sweep_instances(count,
seed=2, fixed_n=121) (the test set of paper_1709_08803_amd.learned_start) that
the oracle's Newton solves to ||F||_inf <= 1e-11, two of them by default.

Calls only the CPU oracle (and the shared input generators): the discrete linear
start by dense LU, then damped Newton with right-preconditioned GMRES(30)
(Section 3.2), preconditioned by the dense LU of the slice-banded J~ (Section
4.2).  Output: tests/golden/learned_heldout_121x41.npz with, per stored
problem, its index in the sweep, its Froude number and its unknown vector.

    python tests/golden/make_learned_heldout.py [how_many]
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402
import scipy.linalg as sla  # noqa: E402

from oracle import jfnk as OJ  # noqa: E402
from oracle import linear as Lin  # noqa: E402
from paper_1709_08803_amd import workloads as W  # noqa: E402

BAND = 3  # h of the library's default band at M = 41 is round(41 / 6) = 7; the oracle's P only needs to be good


class _LU:
    def __init__(self, lu):
        self.lu = lu

    def apply(self, r):
        return sla.lu_solve(self.lu, r)


def main(how_many=2, scan=8):
    probs = W.sweep_instances(scan, seed=2, fixed_n=121)
    idx, fr, us = [], [], []
    for i, p in enumerate(probs):
        if len(idx) >= how_many:
            break
        t0 = time.time()
        J = Lin.jacobian(p)
        u = W.uniform_stream(p) - np.linalg.solve(J, Lin.forcing(p))
        pre = _LU(sla.lu_factor(Lin.banded(p, J, BAND)))
        del J
        res = OJ.newton_krylov(p, u, precond=pre, ftol=1e-11)
        print(f"problem {i} ({p.name}, F = {p.froude:.4f}): converged={res.converged} newton={res.newton_iters} "
              f"({time.time() - t0:.0f} s)", flush=True)
        if res.converged:
            idx.append(i)
            fr.append(p.froude)
            us.append(res.u)
    out = os.path.join(HERE, "learned_heldout_121x41.npz")
    np.savez_compressed(out, index=np.array(idx), froude=np.array(fr), u=np.array(us))
    print("wrote", out, idx, flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 2)
