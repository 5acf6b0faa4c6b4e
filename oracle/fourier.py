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
* exact_solution / exact_solution_point: eq. (exactsoln) itself, and its
  x-derivative, by adaptive quadrature (scipy.integrate.quad; the principal
  value with the Cauchy weight), for topographies that are sums of the
  Gaussian bumps of eq. (bottom).  Pins: tests/test_oracle_exact_pins.py
  (the FFT solution extrapolated to mu -> 0, decay upstream, differences of
  zeta against zeta_x, symmetry in y).
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


def gaussian_transform(eps: float, w: float):
    """Fourier transform of beta + 1 = eps exp(-(x^2 + y^2) / w^2) in polar form,
    beta~(k, psi) = eps pi w^2 exp(-k^2 w^2 / 4) (real and isotropic)."""
    return lambda k, psi: eps * math.pi * w * w * math.exp(-k * k * w * w / 4.0)


def bump_transform(eps: float, delta: float):
    """beta~ of one bump of eq. (bottom) centred at the origin,
    eps exp(-(x^2 + y^2) / (2 delta^2)): eps 2 pi delta^2 exp(-k^2 delta^2 / 2)."""
    return gaussian_transform(eps, math.sqrt(2.0) * delta)


def bump_kmax(delta: float, decay: float = 45.0) -> float:
    """k beyond which k^2 sech(k) beta~(k) of a bump of width delta is below
    exp(-decay) of its scale: the root of k + k^2 delta^2 / 2 = decay."""
    a = 0.5 * delta * delta
    return (-1.0 + math.sqrt(1.0 + 4.0 * a * decay)) / (2.0 * a)


def pole(F: float, psi: float) -> float:
    """k_1(psi): the positive root of k F^2 - sec^2(psi) tanh(k), or 0 if there is none."""
    sec2 = 1.0 / math.cos(psi) ** 2
    if F * F >= sec2:
        return 0.0
    g = lambda k: k * F * F - sec2 * math.tanh(k)
    hi = sec2 / (F * F) + 1.0
    return optimize.brentq(g, 1e-12, hi, xtol=1e-15, rtol=1e-15)


def _sech(k: float) -> float:
    e = math.exp(-k)
    return 2.0 * e / (1.0 + e * e)


def _k_minus_tanh(k: float) -> float:
    """k - tanh(k) without cancellation at small k: the Taylor series of tanh
    (k^3/3 - 2k^5/15 + 17k^7/315 - 62k^9/2835 + 1382k^11/155925 - ...) below 0.1."""
    if k >= 0.1:
        return k - math.tanh(k)
    k2 = k * k
    return k * k2 * (1.0 / 3 - k2 * (2.0 / 15 - k2 * (17.0 / 315 - k2 * (62.0 / 2835 - k2 * (1382.0 / 155925
                     - k2 * 21844.0 / 6081075)))))


def pole_residue(F: float, beta_t, psi: float, k1: float) -> float:
    """R(psi) = k_1^2 sech(k_1) beta~(k_1, psi) / (F^2 - sec^2(psi) sech^2(k_1)): the
    residue at k = k_1 of the k-integrand of eq. (exactsoln) without its cosine
    (the denominator is the k-derivative of k F^2 - sec^2(psi) tanh k there);
    0 where there is no pole (k1 = 0)."""
    if k1 <= 0.0:
        return 0.0
    sec2 = 1.0 / math.cos(psi) ** 2
    return k1 * k1 * _sech(k1) * beta_t(k1, psi) / (F * F - sec2 * _sech(k1) ** 2)


def exact_solution_point(F: float, beta_t, x: float, y: float, kmax: float = 14.0, order: int = 0) -> float:
    """zeta(x, y) (order 0) or zeta_x(x, y) (order 1) of eq. (exactsoln)
    (Section 4.1), by adaptive quadrature, for a topography whose transform
    beta~(k, psi) is real and even in psi (symmetric about x = 0 and y = 0).

    Reading of the path below the pole: the k-integral of the first term is its
    principal value plus pi R sin(k_1 X), X = |x| cos(psi) + y sin(psi), with
    R = k_1^2 sech(k_1) beta~(k_1) / (F^2 - sec^2(psi) sech^2(k_1)) the residue
    of the integrand's pole (the denominator is the k-derivative of
    k F^2 - sec^2(psi) tanh k at k_1).  That is the half-residue an indentation
    below the pole adds to the real part of exp(-i k X); its sign is the one for
    which zeta vanishes far upstream (the principal value alone, or the other
    sign, leaves a wave there).  The second term is the downstream wave H(x) as
    printed.  zeta_x differentiates both under the integral signs
    (d|x|/dx = sign(x), with sign(0) = 0 and H(0) = 1/2, the mean of the
    one-sided derivatives, which agree since zeta is smooth).
    kmax: truncation of the k-integrals (beta~ decays like a Gaussian).
    """
    from scipy import integrate

    F2 = F * F
    sgn = (x > 0) - (x < 0)
    psi0 = 0.0 if F < 1.0 else math.acos(1.0 / F)

    def residue(psi, k1):
        return pole_residue(F, beta_t, psi, k1)

    def inner(psi):
        c, s = math.cos(psi), math.sin(psi)
        sec2 = 1.0 / (c * c)
        X = abs(x) * c + y * s
        if order == 0:
            num = lambda k: k * k * _sech(k) * beta_t(k, psi) * math.cos(k * X)
        else:
            num = lambda k: -k * c * sgn * k * k * _sech(k) * beta_t(k, psi) * math.sin(k * X)
        # g = k F^2 - sec^2(psi) tanh k, written as k (F^2 - sec^2 psi) + sec^2 psi (k - tanh k):
        # near psi_0 (F > 1) both of k F^2 and sec^2 tanh k are much larger than g
        g = lambda k: k * (F2 - sec2) + sec2 * _k_minus_tanh(k)
        k1 = pole(F, psi)
        lim = max(200, int(6 * kmax * (abs(X) + 1)))
        if k1 <= 0.0 or k1 >= kmax:
            # no pole; for F > 1 just below psi_0, g / k nearly vanishes at k = 0 and the
            # integrand varies on the scale sqrt(3 (F^2 - sec^2 psi) / sec^2 psi)
            sig = math.sqrt(max(3.0 * (F2 - sec2) / sec2, 0.0))
            brk = [sig * 2.0 ** j for j in range(40) if 0.0 < sig * 2.0 ** j < kmax] or None
            v, _ = integrate.quad(lambda k: num(k) / g(k) if k > 0 else 0.0, 0.0, kmax, points=brk,
                                  limit=lim, epsabs=1e-13, epsrel=1e-11)
            return v
        # principal value: Cauchy weight 1 / (k - k1) times the regular factor num (k - k1) / g,
        # with g / (k - k1) = F^2 - sec^2 (tanh k - tanh k1) / (k - k1) and
        # tanh k - tanh k1 = tanh(k - k1) (1 - tanh k tanh k1) (no cancellation at the pole)
        t1 = math.tanh(k1)

        def reg(k):
            d = k - k1
            if k <= 0.0:
                return 0.0  # num ~ k^2 and g ~ k (F^2 - sec^2 psi) near k = 0
            q = F2 - sec2 * (1.0 - math.tanh(k) * t1) * (math.tanh(d) / d if d != 0.0 else 1.0)
            return num(k) / q
        # the principal value over [0, 2 k1] (symmetric about the pole) and the plain
        # integral beyond, split where the integrand's scale k1 ends
        k2 = min(2.0 * k1, kmax)
        v, _ = integrate.quad(reg, 0.0, k2, weight="cauchy", wvar=k1, limit=lim, epsabs=1e-13, epsrel=1e-11)
        if k2 < kmax:
            brk = [k1 * 2.0 ** j for j in range(2, 40) if k1 * 2.0 ** j < kmax] or None
            w, _ = integrate.quad(lambda k: num(k) / g(k), k2, kmax, points=brk, limit=lim,
                                  epsabs=1e-13, epsrel=1e-11)
            v += w
        if order == 0:
            return v + math.pi * residue(psi, k1) * math.sin(k1 * X)
        return v + math.pi * residue(psi, k1) * k1 * c * sgn * math.cos(k1 * X)

    pts = [-psi0, psi0] if psi0 > 0.0 else None
    first, _ = integrate.quad(inner, -math.pi / 2, math.pi / 2, points=pts, limit=400, epsabs=1e-12, epsrel=1e-10)
    out = F2 / (2.0 * math.pi ** 2) * first
    if x >= 0.0:
        def wave(psi):
            c, s = math.cos(psi), math.sin(psi)
            k1 = pole(F, psi)
            if order == 0:
                return residue(psi, k1) * math.sin(k1 * x * c) * math.cos(k1 * y * s)
            return residue(psi, k1) * k1 * c * math.cos(k1 * x * c) * math.cos(k1 * y * s)
        w, _ = integrate.quad(wave, psi0, math.pi / 2, limit=400, epsabs=1e-12, epsrel=1e-10)
        out -= (0.5 if x == 0.0 else 1.0) * 2.0 * F2 / math.pi * w
    return out


def exact_solution(F: float, bumps, xs, ys, order: int = 0) -> np.ndarray:
    """zeta (order 0) or zeta_x (order 1) of eq. (exactsoln) at the points
    (xs[i], ys[i]) for beta + 1 a sum of bumps of eq. (bottom), bumps =
    [(eps, delta, b1, b2), ...]: the linear problem is linear in beta + 1, so the
    solution is the sum of each bump's solution, shifted to its centre."""
    out = np.zeros(len(xs))
    for eps, delta, b1, b2 in bumps:
        bt = bump_transform(eps, delta)
        km = bump_kmax(delta)
        for i, (x, y) in enumerate(zip(xs, ys)):
            out[i] += exact_solution_point(F, bt, float(x) - b1, float(y) - b2, kmax=km, order=order)
    return out
