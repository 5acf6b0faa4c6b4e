"""Learned initial guess: data generation with the solver, training, evaluation.

The network (libbim's lg_* kernels) maps (F, bottom beta on the mesh) to a
correction of the discrete linear start in (zeta_x, phi_x).  Training data are
converged solutions of the method itself (FP64 JFNK), produced here by the
batched solver over seeded sweeps of topographies and Froude numbers; the
evaluation compares Newton solves from the learned start with solves from the
linear start on held-out problems.  Every numerical step runs in the library;
this module only orchestrates (batches, epochs, bookkeeping).
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np
import torch

from . import bim as B
from . import workloads as W


@dataclasses.dataclass
class Sample:
    problem: W.Problem
    X0: torch.Tensor       # bf16 bits [M][N][2]
    ffeat: torch.Tensor    # [1]
    target: torch.Tensor   # FP32 [2 M N]: (u*_x - u_lin_x) / out_scale for zeta and phi
    u_star: np.ndarray
    u_lin: np.ndarray


def _xblocks(p: W.Problem, u: np.ndarray) -> np.ndarray:
    """(zeta_x, phi_x) planes [2][M][N] of u."""
    nb = (p.N + 1) * p.M
    return np.stack([u[f * nb:(f + 1) * nb].reshape(p.M, p.N + 1)[:, 1:] for f in range(2)])


def generate(problems: List[W.Problem], net: B.LearnedNet, batch: int = 32, ftol: float = 1e-10,
             inner_prec: str = "fp64", log=print) -> List[Sample]:
    """Solve every problem from its linear start (batched); keep the converged ones."""
    out: List[Sample] = []
    scale = net.arch.out_scale
    t0 = time.perf_counter()
    for b0 in range(0, len(problems), batch):
        probs = problems[b0:b0 + batch]
        dps = [B.DeviceProblem(p) for p in probs]
        ulin = [B.linear_start(dp, rtol=1e-10) for dp in dps]
        us = [u.clone() for u in ulin]
        rc, reps = B.solve_batched(dps, us, ftol=ftol, inner_prec=inner_prec, check=False)
        for p, dp, ul, u, rep in zip(probs, dps, ulin, us, reps):
            if rep["status"] != 0:
                continue
            uh, lh = u.cpu().numpy(), ul.cpu().numpy()
            X0, f = net.make_input(dp, ul)
            tgt = ((_xblocks(p, uh) - _xblocks(p, lh)) / scale).astype(np.float32).reshape(-1)
            out.append(Sample(p, X0, f, torch.as_tensor(tgt, device=X0.device), uh, lh))
        log(f"  generated {len(out)}/{b0 + len(probs)} converged ({time.perf_counter() - t0:.1f} s)")
    return out


def stack(samples: List[Sample]):
    X = torch.stack([s.X0 for s in samples])
    F = torch.cat([s.ffeat for s in samples])
    T = torch.stack([s.target for s in samples])
    return X, F, T


def train(net: B.LearnedNet, samples: List[Sample], epochs: int = 100, batch: int = 32, lr: float = 1e-3,
          seed: int = 0, log=print) -> List[float]:
    X, F, T = stack(samples)
    n = len(samples)
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        perm = rng.permutation(n)
        tot = 0.0
        for b0 in range(0, n, batch):
            idx = torch.as_tensor(perm[b0:b0 + batch], device=X.device)
            if idx.numel() == 0:
                continue
            loss = net.train_step(X[idx].contiguous(), F[idx].contiguous(), T[idx].contiguous(), lr)
            tot += loss * idx.numel()
        hist.append(tot / n)
        if ep % max(1, epochs // 10) == 0 or ep == epochs - 1:
            log(f"  epoch {ep}: loss {hist[-1]:.4e}")
    return hist


def evaluate(net: B.LearnedNet, problems: List[W.Problem], ftol: float = 1e-10, inner_prec: str = "fp64") -> dict:
    """Newton solves from the linear start and from the learned start on each problem."""
    rows = []
    for p in problems:
        dp = B.DeviceProblem(p)
        P = B.Preconditioner(dp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ul = B.linear_start(dp, P, rtol=1e-10)
        t_lin = time.perf_counter() - t0
        t0 = time.perf_counter()
        ulearn = net.infer_start(dp, P)
        torch.cuda.synchronize()
        t_learn = time.perf_counter() - t0
        res = {}
        for name, u0, tstart in (("linear", ul, t_lin), ("learned", ulearn, t_learn)):
            u = u0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep = B.solve(dp, u, P, ftol=ftol, inner_prec=inner_prec, check=False)
            torch.cuda.synchronize()
            res[name] = dict(status=rep["status"], newton=rep["newton_iters"], gmres=rep["gmres_iters"],
                             f0=rep["fnorm0_inf"], ms=(time.perf_counter() - t0 + tstart) * 1e3, u=u.cpu().numpy())
        dz = float(np.abs(_xblocks(p, res["linear"]["u"]) - _xblocks(p, res["learned"]["u"])).max())
        rows.append(dict(name=p.name, F=p.froude, dz_between_starts=dz,
                         **{f"{k}_{m}": res[k][m] for k in res for m in ("status", "newton", "gmres", "f0", "ms")}))
        P.close()
    ok = [r for r in rows if r["linear_status"] == 0 and r["learned_status"] == 0]
    summ = dict(n=len(rows), both_converged=len(ok))
    if ok:
        for m in ("newton", "gmres", "ms", "f0"):
            summ[f"linear_{m}_mean"] = float(np.mean([r[f"linear_{m}"] for r in ok]))
            summ[f"learned_{m}_mean"] = float(np.mean([r[f"learned_{m}"] for r in ok]))
    return dict(summary=summ, rows=rows)
