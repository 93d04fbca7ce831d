"""REXI coefficients from the Cauchy contour integral (oracle; test infrastructure).

Paper, Section 4.2 ("Rational approximation of exponential integrators"):
f(x) ~ sum_n beta_n / (x + alpha_n)  (the REXI sum), obtained from the Cauchy
integral (Eq. cauchy_contour_integral) on a circle Gamma = {R e^{i theta} + mu}
with the N-point trapezoidal rule, which gives Eq. (cauchy_alpha) and
Eq. (cauchy_beta):

    alpha_n = -(R e^{i theta_n} + mu)
    beta_n  = -(1/N) R e^{i theta_n} f(R e^{i theta_n} + mu)

Section 4.2.2 ("Numerical cancellation") fixes the circle by three points:
p_0 on the positive real axis and p_{+-1} = +-i y on the imaginary axis, giving
the radius r = (Re(p_0)^2 + Im(p_{-1})^2) / (2 Re(p_0)) and centre p_0 - r.

Readings (the paper is silent): theta_n = 2 pi (n + 1/2) / N for n = 0..N-1,
which makes the poles exact conjugate pairs with none on the real axis; the
radius written r and R in the same passage is one quantity.

The coefficients are evaluated with mpmath at 40 significant digits and rounded
once to complex128.
"""
from __future__ import annotations

import mpmath
import numpy as np

FN_EXP, FN_PSI1, FN_PSI2 = 0, 1, 2
_DPS = 40


def circle_from_points(p0: float, y: float) -> tuple[float, float]:
    """Radius r and (real) centre mu of the circle through p0, +iy, -iy.

    Section 4.2.2: r = (Re p0^2 + Im p_{-1}^2) / (2 Re p0), centre p0 - r.
    """
    if not (p0 > 0.0 and y > 0.0):
        raise ValueError("p0 and y must be positive")
    r = (p0 * p0 + y * y) / (2.0 * p0)
    return r, p0 - r


def _fn(fn: int, z):
    """f(z) for exp (psi_0) and the ETD functions psi_1, psi_2 (Section 4.3)."""
    if fn == FN_EXP:
        return mpmath.exp(z)
    if fn == FN_PSI1:
        return (mpmath.exp(z) - 1) / z
    if fn == FN_PSI2:
        return (mpmath.exp(z) - 1 - z) / (z * z)
    raise ValueError("unknown function id")


def coefficients_mp(fn: int, N: int, p0: float, y: float):
    """alpha_n, beta_n as mpmath complex numbers (Eq. cauchy_alpha / cauchy_beta)."""
    if N <= 0 or N % 2:
        raise ValueError("N must be a positive even integer")
    with mpmath.workdps(_DPS):
        P0 = mpmath.mpf(p0)
        Y = mpmath.mpf(y)
        r = (P0 * P0 + Y * Y) / (2 * P0)
        mu = P0 - r
        alpha, beta = [], []
        for n in range(N):
            theta = 2 * mpmath.pi * (n + mpmath.mpf(1) / 2) / N
            w = r * mpmath.expj(theta)          # R e^{i theta_n}
            z = w + mu                          # point on the contour
            alpha.append(-z)
            beta.append(-(w * _fn(fn, z)) / N)
        return alpha, beta, r, mu


def coefficients(fn: int, N: int, p0: float, y: float):
    """alpha, beta (complex128 arrays of length N), r, mu (floats).

    Same convention as the paper: f(x) ~ sum_n beta_n / (x + alpha_n).
    """
    a, b, r, mu = coefficients_mp(fn, N, p0, y)
    alpha = np.array([complex(v) for v in a], dtype=np.complex128)
    beta = np.array([complex(v) for v in b], dtype=np.complex128)
    return alpha, beta, float(r), float(mu)


def rexi_sum(alpha: np.ndarray, beta: np.ndarray, x) -> np.ndarray:
    """The scalar REXI sum  sum_n beta_n / (x + alpha_n)  in FP64, pole order."""
    x = np.atleast_1d(np.asarray(x, dtype=np.complex128))
    out = np.zeros_like(x)
    for a, b in zip(alpha, beta):
        out += b / (x + a)
    return out


def rexi_sum_mp(alpha_mp, beta_mp, x: complex):
    """The scalar REXI sum evaluated in mpmath (no rounding of the coefficients)."""
    with mpmath.workdps(_DPS):
        X = mpmath.mpc(x)
        return sum(b / (X + a) for a, b in zip(alpha_mp, beta_mp))


def kappa(alpha: np.ndarray, beta: np.ndarray, x) -> np.ndarray:
    """Condition number of the sum at x: sum_n |beta_n| / |x + alpha_n|.

    Section 4.2.2 discusses the cancellation in the sum; the rounding floor of any
    implementation of the sum is about unit-roundoff times this number.
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.complex128))
    return np.array([np.sum(np.abs(beta) / np.abs(xx + alpha)) for xx in x])
