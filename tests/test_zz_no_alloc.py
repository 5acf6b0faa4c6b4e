"""bim_residual_noalloc (the residual with a fixed device scratch, no allocation)
against bim_residual and the CPU oracle, through the C ABI."""
import numpy as np
import pytest

from paper_1709_08803_amd import workloads as W
from oracle import residual as R

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bim():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_1709_08803_amd import bim as B
    B.lib()
    return B


def _sampled_rows(p, count, seed):
    rng = np.random.default_rng(seed)
    n = p.n_unknowns
    rows = rng.choice(n, count, replace=False)
    # always include the edge rows of both boundary-integral blocks
    edge = [R.row_index(p, b, l, k) for b in (1, 2) for l in (0, p.M - 1) for k in (0, p.N - 2)]
    return np.unique(np.concatenate([rows, edge]))


def _check_against_oracle(p, u, F, prec, rows):
    ref = R.residual_rows(p, u, rows)
    scale = R.term_magnitude_rows(p, u, rows)
    err = float((np.abs(F[rows] - ref) / scale).max())
    tol = 1e-12 if prec == "fp64" else 5e-7
    print(f"{p.name} {prec}: max |dF|/scale over {rows.size} rows {err:.2e} (tolerance {tol:.0e})", flush=True)
    assert err <= tol


def test_noalloc_matches_residual_on_successive_calls(bim):
    assert bim.residual_noalloc_max_bytes() == 64 << 20
    cases = [
        # a mesh whose default FP32C launch does not fit: fewer source chunks
        (W.make_problem(541, 181, -30.0, 30.0, 0.0, 20.0, 1.4, [W.Bump(0.2, 1.0, 1.0)], name="541x181"), "fp32c", 11),
        (W.working(0.7), "fp64", 1),
        (W.working(1.4), "fp32c", 2),
        (W.tiny(0.7), "fp64", 3),   # the second input smaller than the first
        (W.tiny(0.7), "fp32c", 4),
    ]
    for p, prec, seed in cases:
        print(f"case {p.name} {prec}", flush=True)
        dp = bim.DeviceProblem(p, device="cuda:0")
        u = W.perturbed_state(p, seed)
        ud = torch.as_tensor(u, device="cuda:0")
        F = torch.full_like(ud, float("nan"))
        bim.residual_noalloc(dp, ud, F, prec=prec)
        Fref = bim.residual(dp, ud, prec=prec)
        torch.cuda.synchronize()
        a, b = F.cpu().numpy(), Fref.cpu().numpy()
        assert np.all(np.isfinite(a))
        small = p.N * p.M < 50000
        if small:
            # same kernels, same launch: identical sums
            assert np.array_equal(a, b), float(np.abs(a - b).max())
            rows = np.arange(p.n_unknowns) if p.N < 100 else _sampled_rows(p, 400, seed)
        else:
            rows = _sampled_rows(p, 120, seed)
        _check_against_oracle(p, u, a, prec, rows)
        if not small:
            _check_against_oracle(p, u, b, prec, rows)


def test_noalloc_rejects_a_mesh_beyond_its_scratch(bim):
    p = W.make_problem(731, 244, -30.0, 30.0, 0.0, 20.0, 1.4, [W.Bump(0.2, 1.0, 1.0)])
    dp = bim.DeviceProblem(p, device="cuda:0")
    u = torch.zeros(p.n_unknowns, dtype=torch.float64, device="cuda:0")
    F = torch.empty_like(u)
    with pytest.raises(bim.BimError) as e:
        bim.residual_noalloc(dp, u, F)
    assert e.value.code == -1 and "too large" in str(e.value)
