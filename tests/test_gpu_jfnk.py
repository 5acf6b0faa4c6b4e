"""GPU linear start and JFNK solves (through the C ABI) against the oracle's solutions."""
import numpy as np
import pytest

from paper_1709_08803_amd import workloads as W
from oracle import jfnk as OJ
from oracle import linear as Lin
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


@pytest.mark.parametrize("F", [0.7, 1.4])
def test_linear_start_matches_oracle(bim, F):
    p = W.tiny(F)
    ref = Lin.linear_start(p)
    dp = bim.DeviceProblem(p)
    u = bim.linear_start(dp).cpu().numpy()
    err = np.abs(u - ref).max() / np.abs(ref).max()
    print("linear start rel err", err)
    assert err < 1e-9


ORACLE_CACHE = {}


def oracle_solution(p, key):
    if key not in ORACLE_CACHE:
        pc = Lin.Preconditioner(p)
        res = OJ.newton_krylov(p, Lin.linear_start(p, pc.J), pc, ftol=1e-12)
        assert res.converged
        ORACLE_CACHE[key] = res.u
    return ORACLE_CACHE[key]


@pytest.mark.parametrize("F,inner,tol", [(0.7, "fp64", 1e-9), (1.4, "fp64", 1e-9), (0.7, "fp32c", 1e-8),
                                         (1.4, "fp32c", 1e-8)])
def test_converged_solution_matches_oracle(bim, F, inner, tol):
    p = W.tiny(F)
    ref = oracle_solution(p, ("tiny", F))
    dp = bim.DeviceProblem(p)
    P = bim.Preconditioner(dp)
    u = bim.linear_start(dp, P)
    rep = bim.solve(dp, u, P, ftol=1e-12, inner_prec=inner)
    print(F, inner, rep)
    assert rep["status"] == 0
    uh = u.cpu().numpy()
    z_gpu = R.reconstruct(p, uh)
    z_ref = R.reconstruct(p, ref)
    dz = np.abs(z_gpu.zeta - z_ref.zeta).max()
    dphi = np.abs(z_gpu.phi - z_ref.phi).max()
    print("max |dzeta|", dz, "max |dphi|", dphi)
    assert dz <= tol and dphi <= 10 * tol
    # the oracle agrees that the GPU solution solves the discrete system
    assert np.abs(R.residual(p, uh)).max() < 1e-10
    # the reported extent of the solution: its largest elevation and smallest depth
    assert abs(rep["max_zeta"] - z_ref.zeta.max()) <= 1e-8
    assert abs(rep["min_depth"] - (z_ref.zeta - p.beta).min()) <= 1e-8


def test_solver_reports_nonconvergence_and_bad_input(bim):
    p = W.tiny(0.7)
    dp = bim.DeviceProblem(p)
    u = bim.linear_start(dp)
    rep = bim.solve(dp, u.clone(), max_newton=0)
    assert rep["status"] == 1  # BIM_NOT_CONVERGED
    bad = u.clone()
    bad[5] = float("nan")
    rep = bim.solve(dp, bad, check=False)
    assert rep["status"] == -4  # BIM_EDOMAIN


def test_solver_flags_unphysical_iterates(bim):
    # iterates above the limiting height F^2 / 2, or reaching the bottom, are reported as
    # BIM_UNPHYSICAL (3) with their extent, in place of the convergence status
    p = W.tiny(0.7)
    dp = bim.DeviceProblem(p)
    u = bim.linear_start(dp)
    s = p.N + 1
    for shift, what in ((p.froude ** 2, "crest"), (-2.0, "bottom")):
        v = u.clone()
        v.view(3, p.M, s)[0, :, 0] += shift  # zeta_1 of every row: the whole surface moves
        rep = bim.solve(dp, v, max_newton=0, check=False)
        print(what, rep["status"], rep["max_zeta"], rep["min_depth"])
        assert rep["status"] == 3
        if what == "crest":
            assert rep["max_zeta"] > 0.5 * p.froude ** 2
        else:
            assert rep["min_depth"] <= 0.0
    # the batched solver reports the same per instance
    v = u.clone()
    v.view(3, p.M, s)[0, :, 0] += p.froude ** 2
    rc, reps = bim.solve_batched([dp, dp], [u.clone(), v], max_newton=0, check=False)
    assert [r["status"] for r in reps] == [1, 3] and rc == 3


def test_unpreconditioned_gmres_needs_more_iterations(bim):
    # the preconditioner's purpose (Section 4.2): fewer Krylov iterations for the same Newton steps
    p = W.tiny(0.7)
    dp = bim.DeviceProblem(p)
    P = bim.Preconditioner(dp)
    u0 = bim.linear_start(dp, P)
    a = bim.solve(dp, u0.clone(), P, ftol=1e-9)
    b = bim.solve(dp, u0.clone(), None, ftol=1e-9, use_precond=0, max_restarts=40, check=False)
    print("with P", a["gmres_iters"], "without", b["gmres_iters"])
    assert a["status"] == 0
    assert b["gmres_iters"] > 3 * a["gmres_iters"]


def test_graph_replay_matches_eager_solve(bim):
    # every Arnoldi step is captured once and replayed across restarts and
    # Newton steps; the replays must reproduce the eager path bit for bit
    p = W.tiny(1.4)
    dp = bim.DeviceProblem(p)
    P = bim.Preconditioner(dp)
    u0 = bim.linear_start(dp, P)
    ua, ub = u0.clone(), u0.clone()
    ra = bim.solve(dp, ua, P, ftol=1e-12, restart=10, use_graphs=1)
    rb = bim.solve(dp, ub, P, ftol=1e-12, restart=10, use_graphs=0)
    assert ra["status"] == 0 and rb["status"] == 0
    assert ra["gmres_iters"] == rb["gmres_iters"] and ra["gmres_iters"] > 10  # restarts replayed graphs
    assert torch.equal(ua, ub)


GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


@pytest.mark.parametrize("inner,tol,storage,lin", [("fp64", 1e-9, "fp64", "fp64"), ("fp32c", 1e-8, "fp64", "fp64"),
                                                    ("fp32c", 1e-8, "fp32", "fp32c")],
                         ids=["fp64", "fp32c", "mixed-fp32-storage"])
def test_full_size_solution_matches_stored_oracle_solution(bim, inner, tol, storage, lin):
    # 181 x 61, F = 1.4: the oracle's converged solution (tests/golden/make_working_solutions.py);
    # the mixed case runs the FP32-stored P (its S^-1 formed by FP32 substitutions)
    # and the FP32C linear start
    p = W.working(1.4)
    ref = np.load(f"{GOLDEN}/working_181x61_F1.4.npz")["u"]
    dp = bim.DeviceProblem(p)
    P = bim.Preconditioner(dp, storage=storage)
    u = bim.linear_start(dp, P, rtol=1e-4 if lin == "fp32c" else 0.0, prec=lin)
    rep = bim.solve(dp, u, P, ftol=1e-11, inner_prec=inner)
    print(inner, {k: rep[k] for k in ("status", "newton_iters", "gmres_iters", "fnorm_inf", "time_ms")})
    assert rep["status"] == 0
    uh = u.cpu().numpy()
    z_gpu, z_ref = R.reconstruct(p, uh), R.reconstruct(p, ref)
    dz = np.abs(z_gpu.zeta - z_ref.zeta).max()
    dphi = np.abs(z_gpu.phi - z_ref.phi).max()
    print("max |dzeta|", dz, "max |dphi|", dphi)
    assert dz <= tol and dphi <= 10 * tol
    P.close()


@pytest.mark.parametrize("inner,tol,storage,lin", [("fp64", 1e-9, "fp64", "fp64"), ("fp32c", 1e-8, "fp32", "fp32c")],
                         ids=["fp64", "mixed-fp32-storage"])
def test_froude_07_on_the_domain_extended_upstream_matches_the_oracle(bim, inner, tol, storage, lin):
    # F = 0.7 has no solution on x in [-30, 30] at 181 x 61 (a fold of the truncated
    # problem); on x in [-40, 30] at the same spacing (211 x 61, pivot blocks of 212 for
    # the split inversion) it converges, to the oracle's stored solution
    p = W.make_problem(211, 61, -40.0, 30.0, 0.0, 20.0, 0.7, [W.Bump(0.2, 1.0, 1.0)])
    ref = np.load(f"{GOLDEN}/working_211x61_F0.7.npz")["u"]
    dp = bim.DeviceProblem(p)
    P = bim.Preconditioner(dp, storage=storage)
    u = bim.linear_start(dp, P, rtol=1e-4 if lin == "fp32c" else 0.0, prec=lin)
    rep = bim.solve(dp, u, P, ftol=1e-11, inner_prec=inner)
    print(inner, {k: rep[k] for k in ("status", "newton_iters", "gmres_iters", "fnorm_inf", "time_ms")})
    assert rep["status"] == 0
    uh = u.cpu().numpy()
    z_gpu, z_ref = R.reconstruct(p, uh), R.reconstruct(p, ref)
    dz = np.abs(z_gpu.zeta - z_ref.zeta).max()
    dphi = np.abs(z_gpu.phi - z_ref.phi).max()
    print("max |dzeta|", dz, "max |dphi|", dphi)
    assert dz <= tol and dphi <= 10 * tol
    P.close()


def test_stall_stop_ends_a_stagnating_solve(bim):
    # F = 0.7 on the 181 x 61 working domain stagnates near ||F|| = 3.7e-3 (in the
    # oracle as here); with stall_steps = 3 the solve stops as soon as ||F||_inf
    # has not halved over three Newton steps, instead of running to max_newton
    p = W.working(0.7)
    dp = bim.DeviceProblem(p)
    P = bim.Preconditioner(dp)
    u = bim.linear_start(dp, P)
    rep = bim.solve(dp, u, P, check=False, stall_steps=3, max_newton=30)
    h = rep["history"][: rep["newton_iters"] + 1]
    print(rep["status"], rep["newton_iters"], h)
    assert rep["status"] == 1  # BIM_NOT_CONVERGED
    k = rep["newton_iters"]
    assert 3 <= k < 30
    assert h[k] > 0.5 * h[k - 3]
    assert all(h[i] <= 0.5 * h[i - 3] for i in range(3, k))  # it did not stop earlier
    P.close()


@pytest.mark.parametrize("opts", [dict(fp64_below=1e-5), dict(fp32c_gmres_rtol=0.0), dict(fp32c_gmres_rtol=1e-4),
                                  dict()],
                         ids=["switch-to-fp64", "fp32c-strict-gmres", "fp32c-forcing-1e-4", "fp32c-default-forcing"])
def test_fp32c_solve_options_reach_the_fp64_solution(bim, opts):
    # FP32C inner sums with the precision switch or either GMRES tolerance:
    # the same FP64-converged discrete solution as the plain FP64 solve
    p = W.working(1.4, N=61, M=21)
    dp = bim.DeviceProblem(p)
    P = bim.Preconditioner(dp)
    u0 = bim.linear_start(dp, P)
    u64 = u0.clone()
    r64 = bim.solve(dp, u64, P, ftol=1e-11, inner_prec="fp64")
    u32 = u0.clone()
    r32 = bim.solve(dp, u32, P, ftol=1e-11, inner_prec="fp32c", **opts)
    print(opts, "fp64", r64["newton_iters"], r64["gmres_iters"], "fp32c", r32["newton_iters"], r32["gmres_iters"],
          "inner evals", r32["inner_residual_evals"])
    assert r64["status"] == 0 and r32["status"] == 0
    assert r32["fnorm_inf"] <= 1e-11
    assert (u32 - u64).abs().max().item() <= 1e-9
    if "fp64_below" in opts:  # the last steps ran with FP64 sums (no FP32C base evaluation)
        assert r32["inner_residual_evals"] < r32["newton_iters"]
    else:
        assert r32["inner_residual_evals"] == r32["newton_iters"]
    P.close()


def test_solver_rejects_bad_switch_threshold(bim):
    p = W.tiny(0.7)
    dp = bim.DeviceProblem(p)
    u = bim.linear_start(dp)
    rep = bim.solve(dp, u, check=False, inner_prec="fp32c", fp64_below=-1.0)
    assert rep["status"] == -1  # BIM_EINVAL


@pytest.mark.parametrize("inner", ["fp64", "fp32c"])
def test_fp32_stored_preconditioner_reaches_the_same_solution(bim, inner):
    # a preconditioner stored in FP32 (passed in, or built by the solver from
    # the option) changes GMRES's path, not the Newton residual: the same
    # discrete solution as the FP64-stored one, with about as many iterations
    p = W.working(1.4, N=61, M=21)
    dp = bim.DeviceProblem(p)
    P64 = bim.Preconditioner(dp)
    P32 = bim.Preconditioner(dp, storage="fp32")
    u0 = bim.linear_start(dp, P64)
    ua = u0.clone()
    ra = bim.solve(dp, ua, P64, ftol=1e-11, inner_prec=inner)
    ub = u0.clone()
    rb = bim.solve(dp, ub, P32, ftol=1e-11, inner_prec=inner)
    uc = u0.clone()
    rc = bim.solve(dp, uc, None, ftol=1e-11, inner_prec=inner, precond_storage="fp32")
    print(inner, "P64", ra["newton_iters"], ra["gmres_iters"], "P32", rb["newton_iters"], rb["gmres_iters"],
          "internal P32", rc["newton_iters"], rc["gmres_iters"])
    assert ra["status"] == 0 and rb["status"] == 0 and rc["status"] == 0
    assert (ub - ua).abs().max().item() <= 1e-9
    assert torch.equal(uc, ub)  # the internal FP32 build is the same operator
    assert rb["gmres_iters"] <= 1.2 * ra["gmres_iters"] + 2
    P64.close()
    P32.close()


def test_solver_rejects_unknown_precond_storage(bim):
    p = W.tiny(0.7)
    dp = bim.DeviceProblem(p)
    u = bim.linear_start(dp)
    rep = bim.solve(dp, u, check=False, precond_storage=2)
    assert rep["status"] == -1  # BIM_EINVAL


@pytest.mark.parametrize("F", [0.7, 1.4])
def test_fp32c_linear_start_seeds_the_same_newton_solve(bim, F):
    # the linear start with FP32C products to 1e-4: within the FP32C operator's
    # resolution of the FP64 start, and Newton from it ends at the same solution
    # in as many steps
    p = W.working(F, N=61, M=21) if F == 1.4 else W.tiny(F)
    dp = bim.DeviceProblem(p)
    P = bim.Preconditioner(dp)
    u64 = bim.linear_start(dp, P, rtol=1e-8)
    u32 = bim.linear_start(dp, P, rtol=1e-4, prec="fp32c")
    d = (u32 - u64).abs().max().item() / u64.abs().max().item()
    a, b = u64.clone(), u32.clone()
    ra = bim.solve(dp, a, P, ftol=1e-11, inner_prec="fp32c")
    rb = bim.solve(dp, b, P, ftol=1e-11, inner_prec="fp32c")
    print(F, "start rel diff", d, "newton", ra["newton_iters"], rb["newton_iters"], "gmres", ra["gmres_iters"],
          rb["gmres_iters"])
    assert d <= 1e-2
    assert ra["status"] == 0 and rb["status"] == 0
    assert abs(ra["newton_iters"] - rb["newton_iters"]) <= 1
    assert (a - b).abs().max().item() <= 1e-9
    P.close()


def test_linear_start_rejects_unknown_precision(bim):
    import ctypes
    p = W.tiny(0.7)
    dp = bim.DeviceProblem(p)
    u = torch.empty(dp.n, dtype=torch.float64, device="cuda")
    assert bim.lib().bim_linear_start_ex(dp.ref(), None, u.data_ptr(), 1e-8, 3, None) == -1
