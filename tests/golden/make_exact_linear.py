"""Writes oracle_exact_linear.json: the oracle's exact linear solution, eq.
(exactsoln) of Section 4.1, and its x-derivative at sampled nodes of the
meshes of the paper's linear solutions (Fig. 4(a,b): one bump, F = 0.6,
delta = 0.5 on [-7, 17] x [-12, 12]; Fig. 5(a,b): F = 3, delta = 3 on
[-21, 51] x [-36, 36]; Fig. 8(a,b): two bumps inline four linear wavelengths
apart, F = 0.6, delta = 0.5 on [-7, 53] x [-30, 30]; all 281 x 281), of the
181 x 61 half-domain working problem (F = 0.7, bump 0.2 exp(-(x^2 + y^2))) and
of a supercritical pair of off-axis bumps.  Calls only oracle/.

    python tests/golden/make_exact_linear.py
"""
import json
import math
import os
import sys
import time
import warnings

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
from oracle import fourier as Fo  # noqa: E402

warnings.simplefilter("ignore")


def case(name, F, bumps, N, M, xlo, xhi, ylo, yhi, nsample, seed):
    dx, dy = (xhi - xlo) / (N - 1), (yhi - ylo) / (M - 1)
    rng = np.random.default_rng(seed)
    idx = {(0, 0), (N - 1, 0), (0, M - 1), (N - 1, M - 1)}
    for b in bumps:  # the node nearest each bump centre (x - b1 = 0 where it lies on the mesh)
        idx.add((int(np.clip(round((b[2] - xlo) / dx), 0, N - 1)), int(np.clip(round((b[3] - ylo) / dy), 0, M - 1))))
    while len(idx) < nsample:
        idx.add((int(rng.integers(N)), int(rng.integers(M))))
    idx = sorted(idx)
    xs = [xlo + i * dx for i, _ in idx]
    ys = [ylo + j * dy for _, j in idx]
    t = time.time()
    z = Fo.exact_solution(F, bumps, xs, ys, order=0)
    zx = Fo.exact_solution(F, bumps, xs, ys, order=1)
    print(f"{name}: {len(idx)} points in {time.time() - t:.0f} s", flush=True)
    return {"name": name, "froude": F, "bumps": [list(b) for b in bumps], "N": N, "M": M, "x1": xlo, "dx": dx,
            "y1": ylo, "dy": dy, "i": [i for i, _ in idx], "j": [j for _, j in idx], "zeta": z.tolist(),
            "zeta_x": zx.tolist()}


def main():
    lam = 2 * math.pi / Fo.dispersion_root(0.6)
    cases = [
        case("fig4-281x281-F0.6", 0.6, [(0.1, 0.5, 0.0, 0.0)], 281, 281, -7.0, 17.0, -12.0, 12.0, 28, 1),
        case("fig5-281x281-F3", 3.0, [(0.1, 3.0, 0.0, 0.0)], 281, 281, -21.0, 51.0, -36.0, 36.0, 12, 2),
        case("fig8-inline-281x281-F0.6", 0.6, [(0.1, 0.5, 0.0, 0.0), (0.1, 0.5, 4 * lam, 0.0)], 281, 281,
             -7.0, 53.0, -30.0, 30.0, 16, 3),
        case("working-181x61-F0.7", 0.7, [(0.2, 1 / math.sqrt(2.0), 0.0, 0.0)], 181, 61, -30.0, 30.0, 0.0, 20.0,
             16, 4),
        case("pair-91x31-F1.4", 1.4, [(0.1, 0.7, 0.0, 2.0), (0.1, 0.7, 0.0, -2.0)], 91, 31, -16.0, 16.0, 0.0, 10.0,
             12, 5),
    ]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_exact_linear.json")
    with open(out, "w") as f:
        json.dump({"source": "oracle.fourier.exact_solution (eq. (exactsoln), Section 4.1)", "cases": cases}, f)
    print("wrote", out)


if __name__ == "__main__":
    main()
