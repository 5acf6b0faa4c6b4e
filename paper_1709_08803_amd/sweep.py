"""Parameter sweep over many uneven problems on one GPU.

    python -m paper_1709_08803_amd.sweep [--count 64] [--seed 0] [--inner fp32c] [--storage fp32]

Instances: the seeded sweep of workloads.sweep_instances (meshes N x M with N
in 61..181, M = (N-1)/3 + 1 over x in [-30, 30], y in [0, 20]; F ~ U[0.5, 2];
Gaussian, transverse-ridge and two-bump topographies).  Reports, as one JSON
line:
  * the batched residual: every instance's all-pairs sums in one persistent
    launch, aggregate pair-interactions/s in FP64 and FP32C, with the library's
    default launch shape and after the autotuner has picked one on the largest
    mesh (which the sweep's solves then use);
  * the sweep itself (Newton capped at 10 steps and stopped once ||F|| has not
    halved over 4 steps): preconditioner setup for every instance, linear starts,
    and the lockstep batched JFNK (inner sums in the chosen precision,
    preconditioners stored in FP32 or FP64), with
    per-instance status, Newton and GMRES counts; and the same instances solved
    one after another with jfnk_solve, for the batching speedup.
Only library calls do numerical work; this module times and reports.
"""
from __future__ import annotations

import argparse
import json
import time

import torch

from . import bim as B
from . import workloads as W


def _sync_time(fn, reps=1):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) / reps


def run(count: int = 64, seed: int = 0, inner: str = "fp32c", ftol: float = 1e-10, sequential: bool = True,
        max_newton: int = 10, stall_steps: int = 4, storage: str = "fp32", tune: bool = True) -> dict:
    probs = W.sweep_instances(count, seed)
    dps = [B.DeviceProblem(p) for p in probs]
    pairs = sum(p.pairs_per_eval() for p in probs)
    us = [torch.as_tensor(W.perturbed_state(p, 7), device="cuda") for p in probs]
    res = {"count": count, "seed": seed, "pairs_per_sweep_eval": pairs, "max_newton": max_newton,
           "stall_steps": stall_steps,
           "meshes": sorted({f"{p.N}x{p.M}" for p in probs})}
    for prec in ("fp64", "fp32c"):
        B.residual_batched(dps, us, prec)
        _, dt = _sync_time(lambda: B.residual_batched(dps, us, prec), reps=5)
        res[f"batched_residual_{prec}"] = {"ms": dt * 1e3, "pairs_per_s": pairs / dt}
    if tune:
        # the batched launch runs one kernel variant for all instances: the one the
        # autotuner picks on the largest mesh of the sweep (it then also serves the
        # batched solver, and every later call with that mesh)
        big = max(range(count), key=lambda i: probs[i].N * probs[i].M)
        for prec in ("fp64", "fp32c"):
            cfg, ms = B.tune_residual(dps[big], us[big], prec)
            B.residual_batched(dps, us, prec)
            _, dt = _sync_time(lambda: B.residual_batched(dps, us, prec), reps=5)
            res[f"batched_residual_{prec}_tuned"] = {"ms": dt * 1e3, "pairs_per_s": pairs / dt,
                                                     "tuned_on": f"{probs[big].N}x{probs[big].M}",
                                                     "config": list(cfg), "tuned_kernel_ms": ms}
    # the sweep: preconditioners, linear starts, lockstep JFNK
    Ps, t_setup = _sync_time(lambda: [B.Preconditioner(dp, storage=storage) for dp in dps])
    # linear starts in the inner precision (FP64: to 1e-8, the Newton steps' GMRES
    # tolerance; FP32C: to 1e-4, well above the level its products resolve)
    lrtol = 1e-4 if inner == "fp32c" else 1e-8
    ulin, t_lin = _sync_time(lambda: [B.linear_start(dp, P, rtol=lrtol, prec=inner) for dp, P in zip(dps, Ps)])
    ub = [u.clone() for u in ulin]
    (rc, reps), t_solve = _sync_time(lambda: B.solve_batched(dps, ub, Ps, check=False, ftol=ftol,
                                                            inner_prec=inner, max_newton=max_newton,
                                                            stall_steps=stall_steps))
    conv = [r["status"] == 0 for r in reps]
    # the same lockstep rounds launched eagerly instead of replaying the round graph
    ue = [u.clone() for u in ulin]
    (rc_e, reps_e), t_eager = _sync_time(lambda: B.solve_batched(dps, ue, Ps, check=False, ftol=ftol,
                                                                 inner_prec=inner, max_newton=max_newton,
                                                                 stall_steps=stall_steps, use_graphs=0))
    graph_same = all(torch.equal(a, b) for a, b in zip(ub, ue)) and \
        all(a["newton_iters"] == b["newton_iters"] and a["status"] == b["status"] for a, b in zip(reps, reps_e))
    res["sweep"] = {"inner": inner, "precond_storage": storage, "linear_start_rtol": lrtol,
                    "precond_setup_s": t_setup, "linear_starts_s": t_lin,
                    "batched_solve_s": t_solve, "batched_solve_eager_s": t_eager,
                    "graph_replay_equals_eager": bool(graph_same), "converged": int(sum(conv)),
                    "newton_total": int(sum(r["newton_iters"] for r in reps)),
                    "gmres_total": int(sum(r["gmres_iters"] for r in reps)),
                    "per_instance": [{"name": p.name, "F": round(p.froude, 4), "status": r["status"],
                                      "newton": r["newton_iters"], "gmres": r["gmres_iters"],
                                      "fnorm_inf": r["fnorm_inf"]} for p, r in zip(probs, reps)]}
    if sequential:
        useq = [u.clone() for u in ulin]
        seq, t_seq = _sync_time(lambda: [B.solve(dp, u, P, check=False, ftol=ftol, inner_prec=inner,
                                                 max_newton=max_newton, stall_steps=stall_steps)
                                        for dp, u, P in zip(dps, useq, Ps)])
        same = sum(1 for a, b in zip(reps, seq) if (a["status"] == 0) == (b["status"] == 0))
        dmax = max((float((x - y).abs().max()) for x, y, r in zip(ub, useq, reps) if r["status"] == 0),
                   default=0.0)
        res["sweep"].update({"sequential_solve_s": t_seq, "batching_speedup": t_seq / t_solve,
                             "sequential_converged": int(sum(r["status"] == 0 for r in seq)),
                             "same_outcome": same, "max_abs_diff_batched_vs_sequential": dmax})
    for P in Ps:
        P.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--inner", default="fp32c", choices=("fp64", "fp32c"))
    ap.add_argument("--storage", default="fp32", choices=("fp64", "fp32"))
    ap.add_argument("--no-sequential", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (library default launch shape)")
    args = ap.parse_args()
    print(json.dumps(run(args.count, args.seed, args.inner, sequential=not args.no_sequential,
                         storage=args.storage, tune=not args.no_tune)))


if __name__ == "__main__":
    main()
