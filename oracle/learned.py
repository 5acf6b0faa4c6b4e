"""Oracle of the learned-start network: plain FP64 forward and backward.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The network is the one
described for the learned initial guess: conv 3x3 stride 2 pad 1 (2 -> C1) +
ReLU, conv 3x3 stride 2 pad 1 (C1 -> C2) + ReLU, fully connected on [flattened,
F-feature] (-> D3) + ReLU, fully connected linear (-> 2 H W); mean-squared
error loss sum (Y - T)^2 / (2 B n).  NHWC layout; weights [fan_in][fan_out],
convolution fan_in ordered (ky, kx, c_in).

With bf16=True the operands that the GPU keeps in bf16 (inputs, weights,
activations, and the gradients fed to products) are rounded to bf16 here too,
so the remaining difference is only the accumulation order and precision.
"""
from __future__ import annotations

import numpy as np


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bf16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def out_hw(n: int) -> int:
    return (n + 1) // 2


def im2col(X: np.ndarray) -> np.ndarray:
    """X [B][H][W][C] -> [B*Ho*Wo][9C] for a 3x3, stride 2, pad 1 window."""
    B, H, W, C = X.shape
    Ho, Wo = out_hw(H), out_hw(W)
    Xp = np.zeros((B, H + 2, W + 2, C))
    Xp[:, 1:H + 1, 1:W + 1] = X
    cols = np.empty((B, Ho, Wo, 3, 3, C))
    for ky in range(3):
        for kx in range(3):
            cols[:, :, :, ky, kx, :] = Xp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :]
    return cols.reshape(B * Ho * Wo, 9 * C)


def col2im(dcols: np.ndarray, B: int, H: int, W: int, C: int) -> np.ndarray:
    """Adjoint of im2col."""
    Ho, Wo = out_hw(H), out_hw(W)
    d = dcols.reshape(B, Ho, Wo, 3, 3, C)
    dXp = np.zeros((B, H + 2, W + 2, C))
    for ky in range(3):
        for kx in range(3):
            dXp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :] += d[:, :, :, ky, kx, :]
    return dXp[:, 1:H + 1, 1:W + 1]


def forward(params, X0, ffeat, bf=True):
    """params: list of (W, b) per layer.  X0 [B][H][W][2], ffeat [B].  Returns (Y4, cache)."""
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    (W1, b1), (W2, b2), (W3, b3), (W4, b4) = params
    X0 = r(X0)
    B, H, Wd, _ = X0.shape
    C1, C2 = W1.shape[1], W2.shape[1]
    cols1 = im2col(X0)
    Y1 = cols1 @ r(W1) + b1
    A1 = r(np.maximum(Y1, 0.0))
    H1, W1d = out_hw(H), out_hw(Wd)
    cols2 = im2col(A1.reshape(B, H1, W1d, C1))
    Y2 = cols2 @ r(W2) + b2
    A2 = r(np.maximum(Y2, 0.0)).reshape(B, -1)
    A2p = np.concatenate([A2, r(np.asarray(ffeat, dtype=np.float64))[:, None]], axis=1)
    Y3 = A2p @ r(W3) + b3
    A3 = r(np.maximum(Y3, 0.0))
    Y4 = A3 @ r(W4) + b4
    cache = dict(cols1=cols1, Y1=Y1, A1=A1, cols2=cols2, Y2=Y2, A2p=A2p, Y3=Y3, A3=A3, shape=(B, H, Wd, H1, W1d, C1, C2))
    return Y4, cache


def loss_and_grad_out(Y4, T):
    B, n = Y4.shape
    d = Y4 - T
    return 0.5 * float((d * d).sum()) / (B * n), d / (B * n)


def backward(params, cache, dY4, bf=True):
    """Gradients [(gW, gb)] of the four layers for the output gradient dY4."""
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    (W1, b1), (W2, b2), (W3, b3), (W4, b4) = params
    B, H, Wd, H1, W1d, C1, C2 = cache["shape"]
    D2 = cache["A2p"].shape[1] - 1
    g4 = (cache["A3"].T @ r(dY4), dY4.sum(axis=0))
    dA3 = r(dY4) @ r(W4).T
    dY3 = dA3 * (cache["Y3"] > 0)
    g3 = (cache["A2p"].T @ r(dY3), dY3.sum(axis=0))
    dA2 = (r(dY3) @ r(W3).T)[:, :D2]
    dY2 = dA2.reshape(-1, C2) * (cache["Y2"] > 0)
    g2 = (cache["cols2"].T @ r(dY2), dY2.sum(axis=0))
    dcols2 = r(dY2) @ r(W2).T
    dA1 = col2im(dcols2, B, H1, W1d, C1).reshape(-1, C1)
    dY1 = dA1 * (cache["Y1"] > 0)
    g1 = (cache["cols1"].T @ r(dY1), dY1.sum(axis=0))
    return [g1, g2, g3, g4]
