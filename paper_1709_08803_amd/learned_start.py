"""Learned initial guess: data generation with the solver, training, evaluation.

The network (libbim's lg_* kernels) maps (F, bottom beta on the mesh) and,
optionally, the discrete linear start's (zeta_x, phi_x) to a correction of the
linear start's (zeta_x, phi_x).  Training data are converged solutions of the
method itself, produced here by the batched JFNK solver over seeded sweeps of
topographies and Froude numbers.  The evaluation runs Newton from the learned
start and from the linear start on held-out problems and compares iterations
and time; if Newton fails from the learned start the solve is repeated from
the linear start (the fallback), and that cost is charged to the learned side.
Every numerical step runs in the library; this module only orchestrates
(batches, epochs, bookkeeping).
"""
from __future__ import annotations

import dataclasses
import time
from typing import List

import numpy as np
import torch

from . import bim as B
from . import workloads as W


@dataclasses.dataclass
class Sample:
    problem: W.Problem
    X0: torch.Tensor       # bf16 bits [M][N][C0]
    ffeat: torch.Tensor    # [1]
    target: torch.Tensor   # FP32 [2 M N]: (u*_x - u_lin_x) / out_scale for zeta and phi
    newton_from_linear: int


def xplanes(p: W.Problem, u: np.ndarray) -> np.ndarray:
    """(zeta_x, phi_x) planes [2][M][N] of u."""
    nb = (p.N + 1) * p.M
    return np.stack([u[f * nb:(f + 1) * nb].reshape(p.M, p.N + 1)[:, 1:] for f in range(2)])


def generate(problems: List[W.Problem], net: B.LearnedNet, batch: int = 32, ftol: float = 1e-10,
             inner_prec: str = "fp32c", max_newton: int = 10, log=print) -> List[Sample]:
    """Solve every problem from its linear start (batched); keep the converged ones.

    Newton is capped at max_newton steps: the batch advances in lockstep, so a
    problem that does not converge would otherwise hold the whole batch.  The
    targets are converged on the FP64 residual (||F||_inf <= ftol) whatever the
    inner precision; one FP32-stored preconditioner per problem serves its
    linear start (FP64 products, as at inference) and its solve."""
    out: List[Sample] = []
    scale = net.arch.out_scale
    t0 = time.perf_counter()
    for b0 in range(0, len(problems), batch):
        probs = problems[b0:b0 + batch]
        dps = [B.DeviceProblem(p) for p in probs]
        Ps = [B.Preconditioner(dp, storage="fp32") for dp in dps]
        ulin = [B.linear_start(dp, P, rtol=1e-10) for dp, P in zip(dps, Ps)]
        us = [u.clone() for u in ulin]
        _, reps = B.solve_batched(dps, us, Ps, ftol=ftol, inner_prec=inner_prec, check=False,
                                  max_newton=max_newton, stall_steps=4)
        for P in Ps:
            P.close()
        for p, dp, ul, u, rep in zip(probs, dps, ulin, us, reps):
            if rep["status"] != 0:
                continue
            X0, f = net.make_input(dp, ul)
            tgt = ((xplanes(p, u.cpu().numpy()) - xplanes(p, ul.cpu().numpy())) / scale).astype(np.float32)
            out.append(Sample(p, X0, f, torch.as_tensor(tgt.reshape(-1), device=X0.device), rep["newton_iters"]))
        if log:
            log(f"  generated {len(out)}/{b0 + len(probs)} converged ({time.perf_counter() - t0:.1f} s)")
    return out


def stack(samples: List[Sample]):
    X = torch.stack([s.X0 for s in samples])
    F = torch.cat([s.ffeat for s in samples])
    T = torch.stack([s.target for s in samples])
    return X, F, T


def train(net: B.LearnedNet, samples: List[Sample], epochs: int = 100, batch: int = 32, lr: float = 1e-3,
          seed: int = 0, log=print) -> List[float]:
    """Adam on the mean-squared error of the correction, shuffled mini-batches."""
    X, F, T = stack(samples)
    n = len(samples)
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        perm = rng.permutation(n)
        tot = 0.0
        for b0 in range(0, n, batch):
            idx = torch.as_tensor(perm[b0:b0 + batch], device=X.device)
            loss = net.train_step(X[idx].contiguous(), F[idx].contiguous(), T[idx].contiguous(), lr)
            tot += loss * idx.numel()
        hist.append(tot / n)
        if log and (ep % max(1, epochs // 10) == 0 or ep == epochs - 1):
            log(f"  epoch {ep}: loss {hist[-1]:.4e}")
    return hist


def _timed_solve(dp, u, P, **opts):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = B.solve(dp, u, P, check=False, **opts)
    torch.cuda.synchronize()
    return rep, (time.perf_counter() - t0) * 1e3


def evaluate(net: B.LearnedNet, problems: List[W.Problem], ftol: float = 1e-10, inner_prec: str = "fp64",
             learned_max_newton: int = 8) -> dict:
    """Newton from the linear start and from the learned start on each problem.

    Times include building the start (the linear start's GMRES; for the learned
    start lg_infer_start, which computes the linear start itself and then runs
    the network) and, if Newton from the learned start has not converged within
    learned_max_newton steps, the fallback solve from that linear start.  The
    preconditioner is shared and not timed (it depends only on the mesh and F).
    """
    rows = []
    for p in problems:
        dp = B.DeviceProblem(p)
        P = B.Preconditioner(dp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ul = B.linear_start(dp, P)
        torch.cuda.synchronize()
        t_lin = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
        ulearn = net.infer_start(dp, P)
        torch.cuda.synchronize()
        t_learn = (time.perf_counter() - t0) * 1e3
        u1 = ul.clone()
        r1, ms1 = _timed_solve(dp, u1, P, ftol=ftol, inner_prec=inner_prec)
        u2 = ulearn.clone()
        r2, ms2 = _timed_solve(dp, u2, P, ftol=ftol, inner_prec=inner_prec, max_newton=learned_max_newton)
        newton2, fallback = r2["newton_iters"], False
        if r2["status"] != 0:
            fallback = True
            u2 = ul.clone()
            r2b, ms2b = _timed_solve(dp, u2, P, ftol=ftol, inner_prec=inner_prec)
            ms2 += ms2b
            newton2 += r2b["newton_iters"]
            r2 = dict(r2b, newton_iters=newton2, gmres_iters=r2["gmres_iters"] + r2b["gmres_iters"])
        dz = float(np.abs(xplanes(p, u1.cpu().numpy()) - xplanes(p, u2.cpu().numpy())).max())
        rows.append(dict(name=p.name, F=p.froude, linear_status=r1["status"], learned_status=r2["status"],
                         linear_newton=r1["newton_iters"], learned_newton=newton2,
                         linear_gmres=r1["gmres_iters"], learned_gmres=r2["gmres_iters"],
                         linear_ms=t_lin + ms1, learned_ms=t_learn + ms2, fallback=fallback,
                         linear_f0=r1["fnorm0_inf"], learned_f0=r2["fnorm0_inf"], dx_between_solutions=dz))
        P.close()
    ok = [r for r in rows if r["linear_status"] == 0 and r["learned_status"] == 0]
    summ = dict(n=len(rows), both_converged=len(ok), fallbacks=sum(r["fallback"] for r in rows))
    if ok:
        for m in ("newton", "gmres", "ms", "f0"):
            summ[f"linear_{m}_mean"] = float(np.mean([r[f"linear_{m}"] for r in ok]))
            summ[f"learned_{m}_mean"] = float(np.mean([r[f"learned_{m}"] for r in ok]))
        summ["max_dx_between_solutions"] = float(max(r["dx_between_solutions"] for r in ok))
    return dict(summary=summ, rows=rows)


def experiment(n_mesh: int = 121, n_train: int = 4096, n_test: int = 256, epochs: int = 100, batch: int = 64,
               train_seed: int = 1, test_seed: int = 2, in_linear: int = 1, hidden: int = 256, log=print,
               **sweep) -> dict:
    """Generate, train and evaluate on seeded sweeps at one mesh (N = n_mesh, M = (N-1)/3 + 1)."""
    M = (n_mesh - 1) // 3 + 1
    train_p = W.sweep_instances(n_train, seed=train_seed, fixed_n=n_mesh, **sweep)
    test_p = W.sweep_instances(n_test, seed=test_seed, fixed_n=n_mesh, **sweep)
    net = B.LearnedNet(n_mesh, M, seed=0, max_batch=batch, in_linear=in_linear, D3=hidden)
    t0 = time.perf_counter()
    data = generate(train_p, net, batch=batch, log=log)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    hist = train(net, data, epochs=epochs, batch=min(batch, 32), log=log)
    t_train = time.perf_counter() - t0
    ev = evaluate(net, test_p)
    net.close()
    return dict(mesh=f"{n_mesh}x{M}", n_train=n_train, converged_training=len(data), n_test=n_test,
                epochs=epochs, generate_s=t_gen, train_s=t_train, loss_first=hist[0], loss_last=hist[-1],
                summary=ev["summary"])


# Problem families for the experiment: "sweep" is the full parameter sweep of
# workloads.sweep_instances; "bumps" keeps Gaussian and two-bump bottoms with
# F in [0.8, 1.8], heights 0.1-0.3 and widths 0.7-1.5.
FAMILIES = {"sweep": {}, "bumps": dict(kinds=(0, 2), froude=(0.8, 1.8), height=(0.1, 0.3), width=(0.7, 1.5))}


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="learned-start experiment on a seeded sweep")
    ap.add_argument("--mesh", type=int, default=121, help="N (M = (N-1)/3 + 1)")
    ap.add_argument("--train", type=int, default=4096)
    ap.add_argument("--test", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--in-linear", type=int, default=1)
    ap.add_argument("--family", default="sweep", choices=sorted(FAMILIES))
    ap.add_argument("--hidden", type=int, default=256, help="width of the hidden fully connected layer")
    args = ap.parse_args()
    res = experiment(args.mesh, args.train, args.test, args.epochs, in_linear=args.in_linear, hidden=args.hidden,
                     log=lambda m: print(m, flush=True), **FAMILIES[args.family])
    res["family"] = args.family
    print(json.dumps(res))


if __name__ == "__main__":
    main()
