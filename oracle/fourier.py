"""Linear-theory reference values (Section 4.1).  TEST INFRASTRUCTURE ONLY.

* dispersion_root(F): the positive root k of k F^2 = tanh k (transverse waves on
  the centreline, sec(psi) = 1); 2 pi / k is the wavelength quoted for F = 0.6.
* linear_surface_fft(F, bumps, ...): zeta of the linear problem (eqs.
  (linearLaplace)-(linear_radiation2)) by a 2-D Fourier transform.  In Fourier
  space the linear problem gives, with kappa = |k| and k1 = kappa cos(psi),
      zeta^ = k1^2 F^2 beta^ sech(kappa) / (k1^2 F^2 - kappa tanh(kappa)),
  the integrand of eq. (exactsoln).  The radiation condition (the path below
  the pole) is imposed by the classical device of a slow switch-on: i k1 is
  replaced by i k1 + mu with a small mu > 0, which damps waves downstream and
  removes them upstream; the transform is taken on a large periodic box.
  beta^ is the discrete transform of beta + 1 on the same box.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import optimize


def dispersion_root(F: float) -> float:
    """Positive root of k F^2 = tanh(k) (exists for F < 1)."""
    if F >= 1.0:
        raise ValueError("no transverse-wave root for F >= 1")
    return optimize.brentq(lambda k: k * F * F - math.tanh(k), 1e-6, 50.0 / (F * F))


def linear_surface_fft(F: float, bump_fn, half_length: float = 160.0, h: float = 0.25,
                       mu: float = 0.02, tau: float = 0.0):
    """Return (x, y, zeta) on a periodic box [-L, L)^2 with spacing h.

    bump_fn(X, Y) -> beta + 1 on the grid.  tau: surface tension (Section 6);
    the linear dynamic condition phi_x + zeta / F^2 - tau lap(zeta) = 1 makes
    1/F^2 into 1/F^2 + tau kappa^2 for each Fourier mode, so kappa tanh(kappa)
    in the denominator gains the factor 1 + tau F^2 kappa^2.
    """
    n = int(round(2 * half_length / h))
    x = -half_length + h * np.arange(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    b = bump_fn(X, Y)
    bh = np.fft.fft2(b)
    k = 2 * np.pi * np.fft.fftfreq(n, d=h)
    K1, K2 = np.meshgrid(k, k, indexing="xy")
    kap = np.sqrt(K1 * K1 + K2 * K2)
    sig = 1j * K1 + mu
    with np.errstate(invalid="ignore", divide="ignore"):
        th = np.where(kap > 0, np.tanh(kap), 0.0)
        sech = 1.0 / np.cosh(np.minimum(kap, 700.0))
        zh = sig * sig * F * F * bh * sech / (sig * sig * F * F + kap * th * (1.0 + tau * F * F * kap * kap))
    zh[0, 0] = F * F / (F * F - 1.0) * bh[0, 0]
    z = np.real(np.fft.ifft2(zh))
    return x, x, z
