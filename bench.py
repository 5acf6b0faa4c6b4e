#!/usr/bin/env python3
"""Benchmark of the boundary-integral JFNK hot path on one MI355X.

Workload: the 181 x 61 half-domain mesh over x in [-30, 30], y in [0, 20] with
the Gaussian bump 0.2 exp(-(x^2 + y^2)) and F = 0.7 (synthetic, seeded).
A timed step is one evaluation of the dense residual F(u) in FP64 through the
C ABI (unpack and x-integration, node and collocation records, all-pairs sums,
closed-form singular term, dynamic and radiation rows, assembly).  `value` is
pair-interactions per second (collocation point x source node x y-image).
The default warm-up is 100 evaluations (about 70 ms): a GPU that comes out of
idle runs its first tens of milliseconds of work at lower clocks (measured on
this workload: 0.720 ms per evaluation over the 50 evaluations after a
5-evaluation warm-up from idle, 0.670 ms once warm).  With the solver legs (the
default) the GPU is busy for seconds before the warm-up starts.

Also reported: the FP32-compensated evaluation, the all-pairs kernel's
roofline fraction from HIP events on the launch stream, the time to a converged
solve (preconditioner setup, linear start and JFNK with FP64 or FP32-compensated
inner sums and an FP64- or FP32-stored preconditioner, with the distance between
the solutions and, where a stored oracle solution of the same problem exists, to
it) at F = 0.6, 0.7 and 1.4, at F = 0.7 on the domain extended upstream to
x_1 = -40, and on a full domain with two offset bumps; the 64-instance batched
sweep (one persistent all-pairs launch per lockstep round, each round one
replayed HIP graph); the exact linear solution of eq. (exactsoln) on the
paper's 281 x 281 linear-solution meshes (its node contraction against the FP64
matrix peak) and Newton from the start it gives; the learned start at 121 x 41
(trained in the run on a few hundred sweep problems) against the linear start;
and the CPU oracle timed on a bounded sample of the same workload on this
host's cores.  The solver legs run
before the timed residual steps (their GPU work brings the clocks up; the timed
region is the K steps alone).
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

FLOP_PER_PAIR = 25.5       # algorithmic FLOP per pair (mean over the four boundary pairings)
PEAK_FP64_VECTOR = 78.6    # TFLOP/s, MI355X
PEAK_FP32_VECTOR = 157.3   # TFLOP/s, MI355X


def cpu_baseline(p, u, budget_s=15.0):
    """Time the plain CPU oracle's all-pairs sums on a growing sample of collocation rows."""
    import numpy as np
    from oracle import residual as R
    nf = R.reconstruct(p, u)
    gS, DS, sigS, gB, DB, sigB = R.surface_and_bottom(p, nf)
    tg = R.targets_from_fields(p, nf, "S")
    tb = R.targets_from_fields(p, nf, "B")
    pairs_per_target = 2 * p.N * p.M * (2 if p.half_domain else 1)
    rng = np.random.default_rng(0)
    n = 64
    spent, pairs = 0.0, 0
    while spent < budget_s:
        idx = rng.choice(tg.x.size, n, replace=False)
        t0 = time.perf_counter()
        R.bie_rows(p, gS, DS, sigS, gB, DB, sigB, R.subset(tg, idx))
        R.bie_rows(p, gS, DS, sigS, gB, DB, sigB, R.subset(tb, idx))
        dt = time.perf_counter() - t0
        spent += dt
        pairs += 2 * n * pairs_per_target
        n = min(tg.x.size, n * 2)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": pairs / spent, "unit": "pair-interactions/s", "cores": cores, "kind": "oracle",
            "sample": f"{pairs} pairs: random collocation rows of the 181x61 FP64 residual "
                      f"(surface and bottom), {spent:.1f} s"}


def measured_traffic():
    """HBM bytes per FP64 all-pairs launch from the committed counter runs, or None
    if the kernel source has changed since those counters were taken."""
    import hashlib
    path = os.path.join(HERE, "profiles", "k_allpairs_181x61_hbm_traffic.md")
    src = os.path.join(HERE, "paper_1709_08803_amd", "csrc", "residual.hip")
    try:
        fields = dict(line.split(": ", 1) for line in open(path).read().splitlines() if ": " in line)
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        if fields.get("source_sha256_prefix", "").strip() != sha:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None




def time_to_solution(B, W, np, torch, froude, ftol=1e-10, max_newton=15, problem=None, golden=None):
    """Wall time from the mesh to ||F||_inf <= ftol on the 181 x 61 problem at one F
    (or on `problem`, compared with the stored oracle solution `golden`).

    Each preconditioner storage (FP64, FP32) has its own setup and linear start;
    a leg's total is its storage's setup and linear start plus its solve.  A leg
    that does not converge is reported with its status and final ||F||_inf only:
    no speedup and no distance to another solution is formed from it."""
    p = problem if problem is not None else W.working(froude)
    dp = B.DeviceProblem(p)
    nb = (p.N + 1) * p.M
    res = {"froude": froude}
    # per preconditioner storage: the linear start's precision and GMRES tolerance
    #   fp64: FP64 products to 1e-8, the relative tolerance of every FP64 Newton
    #         step's GMRES (a tighter one changes no Newton count)
    #   fp32: FP32C products to 1e-4 (a looser start saves at most 2 ms at 181 x 61
    #         and has cost a Newton step)
    starts = {"fp64": ("fp64", 1e-8), "fp32": ("fp32c", 1e-4)}
    # leg: (preconditioner storage, solver options)
    #   fp64:         FP64 sums, FP64-stored P, FP64 linear start (plain FP64)
    #   fp32c:        FP32C sums with the library's GMRES tolerance for such steps
    #                 (1e-2, the contraction Newton reaches per FP32C step anyway),
    #                 FP32-stored P, FP32C linear start
    #   fp32c_p64:    FP32C sums, FP64-stored P and linear start
    #   fp32c_strict: FP32C sums with every GMRES solve at 1e-8, FP64-stored P
    #   fp64_rtol1e-2: FP64 sums and P with every GMRES solve at 1e-2, the
    #                 tolerance of the fp32c legs: separates what the looser
    #                 linear solves give from what the FP32C sums give
    legs = {"fp64": ("fp64", dict(inner_prec="fp64")),
            "fp32c": ("fp32", dict(inner_prec="fp32c")),
            "fp32c_p64": ("fp64", dict(inner_prec="fp32c")),
            "fp32c_strict": ("fp64", dict(inner_prec="fp32c", fp32c_gmres_rtol=0.0)),
            "fp64_rtol1e-2": ("fp64", dict(inner_prec="fp64", gmres_rtol=1e-2))}
    sols = {}
    for storage in ("fp64", "fp32"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P = B.Preconditioner(dp, storage=storage)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        lprec, lrtol = starts[storage]
        t0 = time.perf_counter()
        ulin = B.linear_start(dp, P, rtol=lrtol, prec=lprec)
        torch.cuda.synchronize()
        t_lin = time.perf_counter() - t0
        # the apply reads every stored array once: bytes ~ P.nbytes (less the
        # 4 n FP64 apply scratch); timed with events on the current stream
        r = torch.ones(dp.n, dtype=torch.float64, device="cuda")
        z = torch.empty_like(r)
        for _ in range(3):
            P.apply(r, out=z)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            P.apply(r, out=z)
        e1.record()
        torch.cuda.synchronize()
        apply_ms = e0.elapsed_time(e1) / 20
        apply_bytes = P.nbytes - 4 * 8 * (dp.n // 3)
        res[f"precond_{storage}"] = {"setup_ms": t_setup * 1e3, "linear_start_ms": t_lin * 1e3,
                                     "linear_start_prec": lprec, "linear_start_rtol": lrtol,
                                     "band_halfwidth": P.band, "bytes": P.nbytes, "apply_ms": apply_ms,
                                     "apply_GBps": apply_bytes / (apply_ms * 1e-3) / 1e9}
        for leg, (st, kw) in legs.items():
            if st != storage:
                continue
            u = ulin.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep = B.solve(dp, u, P, ftol=ftol, check=False, max_newton=max_newton, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            sols[leg] = u.cpu().numpy()
            res[leg] = {"precond_storage": storage, "status": rep["status"], "converged": rep["status"] == 0,
                        "solve_ms": dt * 1e3,
                        "total_ms": (dt + t_setup + t_lin) * 1e3, "newton": rep["newton_iters"],
                        "gmres": rep["gmres_iters"], "jv_evals": rep["jv_evals"],
                        "residual_evals": rep["residual_evals"], "fnorm_inf": rep["fnorm_inf"]}
        P.close()
    if res["fp64"]["converged"] and res["fp32c"]["converged"]:
        d = sols["fp32c"] - sols["fp64"]
        res["fp32c_vs_fp64"] = {"max_dzeta_x": float(np.abs(d[:nb]).max()),
                                "max_dphi_x": float(np.abs(d[nb:2 * nb]).max())}
    for leg in legs:
        if leg != "fp64" and res["fp64"]["converged"] and res[leg]["converged"]:
            res[f"speedup_{leg}"] = res["fp64"]["solve_ms"] / res[leg]["solve_ms"]
            res[f"speedup_{leg}_total"] = res["fp64"]["total_ms"] / res[leg]["total_ms"]
    # the mixed-precision leg against FP64 at the same GMRES tolerance
    if res["fp32c"]["converged"] and res["fp64_rtol1e-2"]["converged"]:
        res["speedup_fp32c_vs_fp64_rtol1e-2"] = res["fp64_rtol1e-2"]["solve_ms"] / res["fp32c"]["solve_ms"]
        res["speedup_fp32c_vs_fp64_rtol1e-2_total"] = res["fp64_rtol1e-2"]["total_ms"] / res["fp32c"]["total_ms"]
    gold = golden if problem is not None else os.path.join(HERE, "tests", "golden", f"working_181x61_F{froude}.npz")
    if gold and os.path.exists(gold):
        ref = np.load(gold)["u"]
        zr, pr = node_values(p, ref, 0), node_values(p, ref, 1)
        for leg, u in sols.items():
            if res[leg]["converged"]:
                res[leg]["max_dzeta_vs_oracle"] = float(np.abs(node_values(p, u, 0) - zr).max())
                res[leg]["max_dphi_vs_oracle"] = float(np.abs(node_values(p, u, 1) - pr).max())
    return res


def extended_domain(W):
    """The 181 x 61 working problem at F = 0.7 with the domain extended upstream to
    x_1 = -40 at the same spacing (211 x 61): on x in [-30, 30] Newton stalls where
    the discrete Jacobian becomes singular, on this domain it converges."""
    return W.make_problem(211, 61, -40.0, 30.0, 0.0, 20.0, 0.7, [W.Bump(0.2, 1.0, 1.0)], name="working-211x61-x1=-40")


def two_bump_full_domain(W, N=151):
    """The paper's asymmetric two-bump problem (bumps of eq. (bottom) with height
    0.2 and delta = 0.5 at (10, 10) and (0, -10); F = 0.6; x in [-7, 53],
    y in [-30, 30]) on a full N x N mesh."""
    import math
    d = 0.5 * math.sqrt(2.0)
    return W.make_problem(N, N, -7.0, 53.0, -30.0, 30.0, 0.6,
                          [W.Bump(0.2, d, d, cx=10.0, cy=10.0), W.Bump(0.2, d, d, cx=0.0, cy=-10.0)],
                          half_domain=False, name=f"two-bumps-full-{N}x{N}")


PEAK_FP64_MATRIX = 78.6   # TFLOP/s, MI355X dense FP64 MFMA


def exact_linear_legs(B, W, np, torch, reps=3, starts=True):
    """Exact linear solution of eq. (exactsoln) on the meshes of the paper's linear
    solutions (Figs. 4(a,b), 5(a,b), 8(a,b): 281 x 281), zeta and zeta_x, with the
    contraction kernel's time from HIP events on its stream; and Newton from the
    start it gives against the discrete linear start on the 181 x 61 problem."""
    import math
    k06 = 1.0 / 0.36
    for _ in range(100):  # root of k F^2 = tanh k at F = 0.6 (wavelength 2 pi / k): Newton from
        # k = 1 / F^2, where k F^2 - tanh k > 0, decreases monotonically to it (convex for k > 0)
        k06 -= (0.36 * k06 - math.tanh(k06)) / (0.36 - 1.0 / math.cosh(k06) ** 2)
    lam = 2.0 * math.pi / k06
    meshes = [("fig4-281x281-F0.6", 0.6, [(0.1, 0.5, 0.0, 0.0)], 281, 281, -7.0, 17.0, -12.0, 12.0),
              ("fig5-281x281-F3", 3.0, [(0.1, 3.0, 0.0, 0.0)], 281, 281, -21.0, 51.0, -36.0, 36.0),
              ("fig8-inline-281x281-F0.6", 0.6, [(0.1, 0.5, 0.0, 0.0), (0.1, 0.5, 4 * lam, 0.0)], 281, 281,
               -7.0, 53.0, -30.0, 30.0)]
    out = {"meshes": []}
    for name, F, bumps, N, M, xlo, xhi, ylo, yhi in meshes:
        dx, dy = (xhi - xlo) / (N - 1), (yhi - ylo) / (M - 1)
        best = None
        for _ in range(reps):
            z, zx, info = B.exact_linear(F, bumps, N, M, xlo, dx, ylo, dy, config={"timing": 1})
            if best is None or info["contract_ms"] < best["contract_ms"]:
                best = info
        flop = 4.0 * N * M * best["nodes"] * len(bumps)  # 2 outputs x one FMA per (target, node)
        ach = flop / (best["contract_ms"] * 1e-3) / 1e12
        out["meshes"].append({"name": name, "froude": F, "bumps": bumps, "mesh": f"{N}x{M}",
                              "nodes": best["nodes"], "psi_nodes": best["psi_nodes"], "kcut": best["kcut"],
                              "total_ms": best["total_ms"], "contract_ms": best["contract_ms"],
                              "contract_tflops": ach, "contract_frac_fp64_matrix_peak": ach / PEAK_FP64_MATRIX,
                              "max_abs_zeta": float(z.abs().max())})
    if not starts:
        return out
    # Newton from the exact linear solution's start against the discrete linear
    # start (the bottom here is a bump of the paper's form, whose transform the
    # exact solution needs): plain FP64 from both starts, and the mixed-precision
    # solve (FP32C sums, FP32-stored P) from the exact start; total_ms = setup of
    # P + start + solve, as in the time-to-solution legs
    starts = []
    for F in (1.4, 0.6):
        p = W.working(F)
        dp = B.DeviceProblem(p)
        row = {"froude": F}
        for storage in ("fp64", "fp32"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P = B.Preconditioner(dp, storage=storage)
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            kinds = ("linear", "exact") if storage == "fp64" else ("exact_fp32c",)
            for kind in kinds:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if kind == "linear":
                    u = B.linear_start(dp, P, rtol=1e-8, prec="fp64")
                else:
                    z, zx, _ = B.exact_linear(F, [(0.2, 1.0 / math.sqrt(2.0), 0.0, 0.0)], p.N, p.M, p.x1, p.dx,
                                              p.y1, p.dy)
                    u = B.exact_start(dp, z, zx)
                torch.cuda.synchronize()
                t_start = time.perf_counter() - t0
                F0 = B.residual(dp, u, "fp64")
                f0 = float(F0.abs().max())
                inner = "fp32c" if kind == "exact_fp32c" else "fp64"
                t0 = time.perf_counter()
                rep = B.solve(dp, u, P, ftol=1e-10, check=False, max_newton=15, inner_prec=inner)
                torch.cuda.synchronize()
                t_solve = time.perf_counter() - t0
                row[kind] = {"precond_storage": storage, "inner": inner, "setup_ms": t_setup * 1e3,
                             "start_ms": t_start * 1e3, "fnorm_inf_start": f0, "status": rep["status"],
                             "newton": rep["newton_iters"], "gmres": rep["gmres_iters"], "solve_ms": t_solve * 1e3,
                             "total_ms": (t_setup + t_start + t_solve) * 1e3}
                row[kind + "_u"] = u.cpu().numpy()
            P.close()
        nb = (p.N + 1) * p.M
        for kind in ("exact", "exact_fp32c"):
            if row["linear"]["status"] == 0 and row[kind]["status"] == 0:
                row[f"max_dzeta_x_{kind}_vs_linear_start"] = float(
                    np.abs(row["linear_u"][:nb] - row[kind + "_u"][:nb]).max())
        for kind in ("linear", "exact", "exact_fp32c"):
            del row[kind + "_u"]
        starts.append(row)
    out["newton_from_exact_start_181x61"] = starts
    return out


def learned_leg(n_train=384, n_test=16, epochs=100, hidden=512):
    """The learned start at 121 x 41 (M = (N-1)/3 + 1): a network trained in this
    run on n_train problems of the seeded sweep (their converged FP64 solutions
    from the batched solver), then Newton from the learned start against Newton
    from the discrete linear start on n_test held-out problems (a learned attempt
    that has not converged in 8 steps falls back to the linear start, its cost
    charged to the learned side).  Reported whether it gains or loses."""
    from paper_1709_08803_amd import learned_start as LS
    return LS.experiment(121, n_train, n_test, epochs, hidden=hidden, log=lambda m: None)


def node_values(p, u, f):
    """f-th field at the nodes from u (trapezoidal x-integration of f_x from f_1)."""
    import numpy as np
    nb = (p.N + 1) * p.M
    blk = u[f * nb:(f + 1) * nb].reshape(p.M, p.N + 1)
    fx = blk[:, 1:]
    steps = 0.5 * p.dx * (fx[:, 1:] + fx[:, :-1])
    return blk[:, :1] + np.concatenate([np.zeros((p.M, 1)), np.cumsum(steps, axis=1)], axis=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-solution legs")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 64-instance batched sweep")
    ap.add_argument("--no-exact", action="store_true", help="skip the exact linear solution legs")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-start leg (trains a network, ~1 min)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="first run a plain elementwise copy of MB megabytes (reads MB, writes MB), "
                         "the reference for scaling hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (row sharding of the residual "
              f"and the preconditioner across GPUs is not implemented).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1709_08803_amd import bim as B
    from paper_1709_08803_amd import workloads as W

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    # solver legs first: they are reported as well, and the seconds of GPU work
    # they take bring the GPU to its steady clocks before the residual is timed
    extra = {}
    t_start = time.perf_counter()

    def progress(what):  # one line per finished leg on stderr (the JSON line stays alone on stdout)
        print(f"[bench] {what} done at {time.perf_counter() - t_start:.1f} s", file=sys.stderr, flush=True)
    if not args.no_solve:
        extra["time_to_solution"] = []
        for f in (0.6, 0.7, 1.4):
            extra["time_to_solution"].append(time_to_solution(B, W, np, torch, f))
            progress(f"time to solution at F = {f}")
        gold = os.path.join(HERE, "tests", "golden", "working_211x61_F0.7.npz")
        extra["time_to_solution_extended_domain"] = dict(
            workload="F = 0.7 on x in [-40, 30], y in [0, 20] (211 x 61, same spacing and bump)",
            **time_to_solution(B, W, np, torch, 0.7, problem=extended_domain(W), golden=gold))
        progress("extended domain")
        pf = two_bump_full_domain(W)
        extra["time_to_solution_full_domain"] = dict(
            workload="two offset bumps (10, 10), (0, -10), height 0.2, delta 0.5, F = 0.6, full domain "
                     "x in [-7, 53], y in [-30, 30], 151 x 151",
            pairs_per_eval=pf.pairs_per_eval(), **time_to_solution(B, W, np, torch, 0.6, problem=pf))
        progress("full domain")
    if not args.no_sweep:
        from paper_1709_08803_amd import sweep as SW
        sw = SW.run(64, 0, "fp32c")
        sw["sweep"]["per_instance"] = [[r["name"], r["F"], r["status"], r["newton"], r["gmres"]]
                                       for r in sw["sweep"]["per_instance"]]
        extra["sweep"] = sw
        progress("sweep")
    if not args.no_exact:
        extra["exact_linear"] = exact_linear_legs(B, W, np, torch, starts=not args.no_solve)
        progress("exact linear solution")
    if not args.no_solve and not args.no_learned:
        extra["learned_start_121x41"] = learned_leg()
        progress("learned start")

    p = W.working(0.7)
    dp = B.DeviceProblem(p)
    u_host = W.perturbed_state(p, 11)
    u = torch.as_tensor(u_host, device="cuda")
    F = torch.empty_like(u)
    pairs = p.pairs_per_eval()

    for _ in range(args.warmup):
        B.residual(dp, u, "fp64", out=F)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.residual(dp, u, "fp64", out=F)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt / args.steps * 1e3
    value = pairs * args.steps / dt

    # dominant kernel: all-pairs sums, HIP events on the launch stream, right
    # after the timed steps
    k64, t64 = B.residual_timed(dp, u, "fp64", iters=max(5, args.steps // 2))
    k32, t32 = B.residual_timed(dp, u, "fp32c", iters=max(5, args.steps // 2))
    ach64 = pairs * FLOP_PER_PAIR / (k64 * 1e-3) / 1e12
    ach32 = pairs * FLOP_PER_PAIR / (k32 * 1e-3) / 1e12

    out = {
        "metric": "pair-interactions/s + time-to-converged-solve, 181x61 grid: FP64 vs mixed/learned",
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "residual F(u), 181x61 half domain, x in [-30,30], y in [0,20], "
                               "bump 0.2 exp(-(x^2+y^2)), F=0.7, FP64",
                   "pairs_per_eval": pairs},
        "roofline": {"bound": "alu", "achieved": ach64, "peak": PEAK_FP64_VECTOR, "unit": "TFLOP/s",
                     "frac": ach64 / PEAK_FP64_VECTOR, "traffic": measured_traffic(),
                     "kernel": "k_allpairs<double>", "kernel_ms": k64,
                     "flop_per_pair": FLOP_PER_PAIR},
        "fp32c": {"eval_ms": t32, "kernel_ms": k32, "pairs_per_s": pairs / (t32 * 1e-3),
                  "roofline": {"bound": "alu", "achieved": ach32, "peak": PEAK_FP32_VECTOR,
                               "unit": "TFLOP/s", "frac": ach32 / PEAK_FP32_VECTOR}},
        "fp64_eval_ms_events": t64,
        "residual_evals_per_s": 1e3 / ms_step,
    }
    out.update(extra)
    progress("timed residual steps")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, u_host)
        progress("CPU baseline")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
