"""Choice of the REXI contour (p0, y, N) for a target accuracy (host side).

The circle through p0 and +-iy (Section 4.2, Eq. for r and mu) must enclose the
spectrum of dt L, which lies on the imaginary segment i[-rho, rho] with
rho = dt (sqrt(g H L(L+1)) / a + 2 Omega).  Here y = sqrt(2) 1.05 rho.  Two
things bound the accuracy of the rational sum S(x) = sum_n beta_n / (x + alpha_n)
on that segment:

* the approximation error max_{|w| <= rho} |S(i w) - e^{i w}|, evaluated here
  in FP64 on a dense grid of w (it falls geometrically with N, faster for
  larger p0, until the trapezoidal rule aliases the growth of e^z on the
  circle);
* the rounding floor of the solve: the terms are as large as
  kappa(w) = sum_n |beta_n| / |i w + alpha_n| while their sum is O(1)
  (Section 4.2.2), so any evaluation in a precision with unit roundoff u loses
  about u kappa.  kappa grows like e^{p0}, which is why a reduced-precision
  solve needs a small p0 and then many more poles.

predicted_error() adds the two; choose() returns, over a grid of p0, the
contour with the fewest (even) poles whose prediction meets the target.
The coefficients come from the library's own rexi_coefficients.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import api

U = {0: 2.0 ** -53, 1: 2.0 ** -24}       # unit roundoff of the solve: FP64, FP32 (REXI_PREC_FP32_SOLVE)
P0_GRID = (2.0, 3.0, 4.0, 5.0, 6.0, 8.0, 10.0, 12.0, 14.0, 16.0, 20.0, 24.0, 28.0, 32.0)


def spectral_radius(L: int, dt: float, a=api.EARTH["a"], g=api.EARTH["g"], H=api.EARTH["H"],
                    Omega=api.EARTH["Omega"]) -> float:
    return dt * (math.sqrt(g * H * L * (L + 1.0)) / a + 2.0 * Omega)


def enclosing_y(rho: float) -> float:
    return math.sqrt(2.0) * 1.05 * rho


def _terms(alpha, beta, rho, npts):
    w = np.linspace(-rho, rho, npts)
    return w, beta[None, :] / (1j * w[:, None] + alpha[None, :])


def scalar_error(alpha, beta, rho: float, npts: int = 1601) -> float:
    """max over |w| <= rho of |S(i w) - e^{i w}|."""
    w, t = _terms(alpha, beta, rho, npts)
    return float(np.abs(t.sum(axis=1) - np.exp(1j * w)).max())


def kappa(alpha, beta, rho: float, npts: int = 401) -> float:
    """max over |w| <= rho of sum_n |beta_n| / |i w + alpha_n|."""
    _, t = _terms(alpha, beta, rho, npts)
    return float(np.abs(t).sum(axis=1).max())


def predicted_error(alpha, beta, rho: float, prec: int) -> float:
    return scalar_error(alpha, beta, rho) + U[prec & 1] * kappa(alpha, beta, rho)


@dataclass(frozen=True)
class Contour:
    p0: float
    y: float
    N: int
    predicted: float


def _predict(N: int, p0: float, y: float, rho: float, prec: int) -> float:
    alpha, beta, _, _ = api.rexi_coefficients(api.FN_EXP, N, p0, y)
    return predicted_error(alpha, beta, rho, prec)


def choose(L: int, dt: float, target: float, prec: int, p0_grid=P0_GRID, n_max: int = 4096) -> Contour | None:
    """The contour with the fewest poles whose predicted error is <= target
    (None if no p0 of the grid reaches it within n_max poles)."""
    rho = spectral_radius(L, dt)
    y = enclosing_y(rho)
    best = None
    for p0 in p0_grid:
        if _predict(n_max, p0, y, rho, prec) > target:
            continue
        lo, hi = 1, n_max // 2          # search N = 2 k, k in (lo, hi]
        if best is not None:
            hi = min(hi, best.N // 2)
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if _predict(2 * mid, p0, y, rho, prec) <= target:
                hi = mid
            else:
                lo = mid
        N = 2 * hi
        e = _predict(N, p0, y, rho, prec)
        if e <= target and (best is None or N < best.N):
            best = Contour(p0, y, N, e)
    return best


def best_p0(L: int, dt: float, N: int, prec: int, p0_grid=P0_GRID) -> Contour:
    """The p0 of the grid with the smallest predicted error at a fixed N."""
    rho = spectral_radius(L, dt)
    y = enclosing_y(rho)
    cands = [Contour(p0, y, N, _predict(N, p0, y, rho, prec)) for p0 in p0_grid]
    return min(cands, key=lambda c: c.predicted)
