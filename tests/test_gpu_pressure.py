"""Bottom pressure and force on the topography (bim_bottom_pressure) against the CPU oracle."""
import os

import numpy as np
import pytest

from paper_1709_08803_amd import workloads as W
from oracle import pressure as OP

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def bim():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_1709_08803_amd import bim as B
    B.lib()
    return B


def _compare(bim, p, u):
    print(f"case {p.name} N={p.N} M={p.M} half={p.half_domain}", flush=True)
    dp = bim.DeviceProblem(p, device="cuda:0")
    pres, force = bim.bottom_pressure(dp, torch.as_tensor(u, device="cuda:0"))
    torch.cuda.synchronize()
    ref = OP.bottom_pressure(p, u)
    fref = OP.bottom_force(p, ref)
    a, f = pres.cpu().numpy(), force.cpu().numpy()
    # psi is an x-integral of values of size |x1|: rounding of order 1e-15 |x1| in psi,
    # divided by 2 dy in psi_y; the rest is pointwise FP64
    perr = float(np.abs(a - ref).max())
    ferr = float(np.abs(f - fref).max() / (np.abs(fref).max() + 1e-300))
    print(f"  pressure max |dp| {perr:.2e}, force {f} vs {fref}, rel {ferr:.2e}", flush=True)
    assert perr <= 1e-12 * (1 + abs(p.x1) / p.dy)
    assert ferr <= 1e-11
    return f


def test_pressure_on_perturbed_states(bim):
    for p, seed in ((W.tiny(0.7), 1), (W.working(1.4), 2),
                    (W.make_problem(121, 41, -20, 20, 0, 13.33, 0.9, [W.Bump(0.2, 1.0, 1.0, cx=3.0)]), 3),
                    (W.make_problem(61, 41, -15, 15, -10, 10, 1.2,
                                    [W.Bump(0.2, 1.0, 1.0, cx=2.0, cy=3.0), W.Bump(0.15, 1.0, 1.0, cx=-4.0, cy=-5.0)],
                                    half_domain=False), 4),
                    (W.make_problem(3, 3, -1, 1, 0, 1, 0.8, [W.Bump(0.1, 1.0, 1.0)]), 5)):
        f = _compare(bim, p, W.perturbed_state(p, seed))
        if not p.half_domain:
            assert f[1] != 0.0


def test_pressure_at_the_stored_oracle_solution(bim):
    # the converged 181 x 61, F = 1.4 solution written by the oracle: the wave drag
    # on the bump is positive (a force along the stream) and the pressure at the
    # far upstream bottom is the undisturbed 1/F^2
    g = np.load(os.path.join(HERE, "golden", "working_181x61_F1.4.npz"))
    p = W.working(1.4)
    f = _compare(bim, p, g["u"])
    assert f[0] > 0.0
    pres = OP.bottom_pressure(p, g["u"])
    assert abs(pres[:, 0] - 1 / 1.4 ** 2).max() < 1e-2
