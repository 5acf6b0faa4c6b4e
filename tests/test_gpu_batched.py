"""Batched residual: one persistent launch over problems of uneven size."""
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


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32c", 5e-7)])
def test_batched_residual_matches_oracle_per_instance(bim, prec, tol):
    probs = W.sweep_instances(6, seed=0, n_choices=[31, 34, 46, 61])
    probs.append(W.tiny(0.9))
    dps = [bim.DeviceProblem(p) for p in probs]
    us_h = [W.perturbed_state(p, 20 + i) for i, p in enumerate(probs)]
    us = [torch.as_tensor(u, device="cuda") for u in us_h]
    Fs = bim.residual_batched(dps, us, prec)
    torch.cuda.synchronize()
    for p, u, F in zip(probs, us_h, Fs):
        ref = R.residual(p, u)
        scale = R.term_magnitude_rows(p, u)
        err = (np.abs(F.cpu().numpy() - ref) / scale).max()
        print(p.name, prec, err)
        assert err <= tol


def test_batched_equals_single_with_same_split(bim):
    # with the same kernel variant and source split a problem's result does not
    # depend on the batch it runs in
    probs = W.sweep_instances(4, seed=3, n_choices=[31, 46])
    dps = [bim.DeviceProblem(p) for p in probs]
    us = [torch.as_tensor(W.perturbed_state(p, 5), device="cuda") for p in probs]
    a = bim.residual_batched(dps, us, "fp64")
    b = bim.residual_batched(dps[1:2], us[1:2], "fp64")
    c = bim.residual_batched(dps[::-1], us[::-1], "fp64")
    torch.cuda.synchronize()
    assert torch.equal(a[1], b[0])
    assert torch.equal(a[0], c[-1])


def test_batched_solve_matches_single_solves_and_oracle(bim):
    from oracle import jfnk as OJ
    from oracle import linear as Lin
    probs = W.sweep_instances(5, seed=1, n_choices=[31, 34, 37])
    dps = [bim.DeviceProblem(p) for p in probs]
    starts = [bim.linear_start(dp) for dp in dps]
    ub = [u.clone() for u in starts]
    rc, reps = bim.solve_batched(dps, ub, ftol=1e-11, check=False)
    for i, (p, dp) in enumerate(zip(probs, dps)):
        us = starts[i].clone()
        rep = bim.solve(dp, us, ftol=1e-11, check=False)
        print(p.name, "batched", reps[i]["status"], reps[i]["newton_iters"], reps[i]["gmres_iters"],
              "single", rep["status"], rep["newton_iters"], rep["gmres_iters"])
        if rep["status"] != 0:
            continue  # a failed instance must fail in both
        assert reps[i]["status"] == 0
        a, b = ub[i].cpu().numpy(), us.cpu().numpy()
        za, zb = R.reconstruct(p, a).zeta, R.reconstruct(p, b).zeta
        assert np.abs(za - zb).max() <= 1e-9
        assert np.abs(R.residual(p, a)).max() < 1e-9


def test_batched_solve_mixed_precision(bim):
    probs = W.sweep_instances(3, seed=2, n_choices=[31, 46])
    dps = [bim.DeviceProblem(p) for p in probs]
    us = [bim.linear_start(dp) for dp in dps]
    rc, reps = bim.solve_batched(dps, us, ftol=1e-10, inner_prec="fp32c", check=False)
    for p, u, r in zip(probs, us, reps):
        print(p.name, r["status"], r["newton_iters"], r["gmres_iters"])
        if r["status"] == 0:
            assert np.abs(R.residual(p, u.cpu().numpy())).max() < 1e-9


def test_batched_solve_switches_precision_like_sequential(bim):
    # per-instance switch to FP64 inner sums below ||F||_inf = 1e-5: the lockstep
    # batch takes the same decisions as the single solves
    probs = W.sweep_instances(4, seed=5, n_choices=[31, 46, 61], froude=(1.2, 1.8), height=(0.05, 0.15))
    dps = [bim.DeviceProblem(p) for p in probs]
    us = [bim.linear_start(dp) for dp in dps]
    ub = [u.clone() for u in us]
    opts = dict(ftol=1e-10, inner_prec="fp32c", fp64_below=1e-5)
    rc, reps = bim.solve_batched(dps, ub, check=False, **opts)
    for p, dp, u0, ubi, rb in zip(probs, dps, us, ub, reps):
        us_ = u0.clone()
        rs = bim.solve(dp, us_, check=False, **opts)
        print(p.name, rb["status"], rs["status"], rb["newton_iters"], rs["newton_iters"], rb["inner_residual_evals"],
              rs["inner_residual_evals"])
        assert rb["status"] == rs["status"]
        if rb["status"] == 0:
            assert rb["inner_residual_evals"] < rb["newton_iters"]
            assert (ubi - us_).abs().max().item() <= 1e-8
            assert np.abs(R.residual(p, ubi.cpu().numpy())).max() < 1e-9


def test_batched_solve_with_fp32_stored_preconditioners(bim):
    # the batched apply reads FP32-stored operators: the lockstep batch ends
    # where the single solves with the same preconditioner storage end
    probs = W.sweep_instances(3, seed=7, n_choices=[31, 46], froude=(1.2, 1.8), height=(0.05, 0.15))
    dps = [bim.DeviceProblem(p) for p in probs]
    us = [bim.linear_start(dp) for dp in dps]
    ub = [u.clone() for u in us]
    opts = dict(ftol=1e-10, inner_prec="fp32c", precond_storage="fp32")
    rc, reps = bim.solve_batched(dps, ub, check=False, **opts)
    for p, dp, u0, ubi, rb in zip(probs, dps, us, ub, reps):
        us_ = u0.clone()
        rs = bim.solve(dp, us_, check=False, **opts)
        print(p.name, rb["status"], rs["status"], rb["newton_iters"], rs["newton_iters"], rb["gmres_iters"],
              rs["gmres_iters"])
        assert rb["status"] == rs["status"]
        if rb["status"] == 0:
            assert (ubi - us_).abs().max().item() <= 1e-8
            assert np.abs(R.residual(p, ubi.cpu().numpy())).max() < 1e-9


def test_batched_graph_replay_equals_eager_execution(bim):
    # one captured round graph replayed every round against the same rounds
    # launched eagerly: identical iterates and decisions, bit for bit; the
    # batch includes a 121 x 41 mesh and runs the sweep configuration (FP32C
    # inner sums, FP32-stored preconditioners)
    from paper_1709_08803_amd import workloads as W2
    probs = W2.sweep_instances(5, seed=11, n_choices=[31, 46, 61, 121])
    probs.append(W2.make_problem(121, 41, -30.0, 30.0, 0.0, 20.0, 1.3, [W2.Bump(0.15, 1.2, 1.2)], name="gauss-121x41"))
    dps = [bim.DeviceProblem(p) for p in probs]
    starts = [bim.linear_start(dp, prec="fp32c", rtol=1e-4) for dp in dps]
    opts = dict(ftol=1e-10, inner_prec="fp32c", precond_storage="fp32", max_newton=10, stall_steps=4)
    ug = [u.clone() for u in starts]
    ue = [u.clone() for u in starts]
    rc_g, rep_g = bim.solve_batched(dps, ug, check=False, use_graphs=1, **opts)
    rc_e, rep_e = bim.solve_batched(dps, ue, check=False, use_graphs=0, **opts)
    assert rc_g == rc_e
    for p, a, b, ra, rb in zip(probs, ug, ue, rep_g, rep_e):
        print(p.name, ra["status"], ra["newton_iters"], ra["gmres_iters"], rb["newton_iters"], rb["gmres_iters"])
        assert torch.equal(a, b)
        for k in ("status", "newton_iters", "gmres_iters", "residual_evals", "jv_evals", "backtracks"):
            assert ra[k] == rb[k], k
        assert ra["history"] == rb["history"]
    big = len(probs) - 1
    assert rep_g[big]["status"] == 0
    assert np.abs(R.residual(probs[big], ug[big].cpu().numpy())).max() <= 1e-10


def test_batched_solve_rejects_shared_preconditioner_or_vector(bim):
    probs = W.sweep_instances(2, seed=3, n_choices=[31])
    dps = [bim.DeviceProblem(p) for p in probs]
    P = bim.Preconditioner(dps[0])
    us = [bim.linear_start(dp) for dp in dps]
    with pytest.raises(bim.BimError):
        bim.solve_batched(dps, us, Ps=[P, P])
    with pytest.raises(bim.BimError):
        bim.solve_batched(dps, [us[0], us[0]])
    P.close()
