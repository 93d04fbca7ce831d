"""Pins of the oracle's REXI coefficients (Section 4.2) against mathematics.

* the circle through p0 and +-iy, worked by hand for the paper's parameters;
* the exact trapezoidal-rule error of the Cauchy integral on a circle:
  with t = (x - mu) / r and theta_n = 2 pi (n + 1/2) / N, the N-point rule gives
  f(x) - t^N f(x) + O(t^{2N}) + O(r^N / N!) for entire f, so the REXI error at a
  point is a known closed form -- a wrong sign, offset or factor in alpha or beta
  breaks it;
* conjugate symmetry and the rounding floor of the FP64-rounded coefficients;
* the cancellation factor kappa(x) = sum |beta_n| / |x + alpha_n| (Section
  4.2.2) at the centre of the circle, where every |x + alpha_n| = r and the
  sum is the trapezoidal rule of e^{mu + r cos theta}: e^{mu} I_0(r) = e^{p0}
  i0e(r) up to the rule's aliasing terms 2 I_N(r) e^{mu}, and elsewhere an
  mpmath evaluation at 40 digits from the unrounded coefficients.
"""
import json
import os

import mpmath
import numpy as np
import pytest
import scipy.special

from oracle import rexi

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_rexi_params.json")


def test_paper_circle_by_hand():
    g = json.load(open(GOLD))
    r, mu = rexi.circle_from_points(g["p0"], g["y"])
    assert r == g["r_by_hand"]
    assert mu == g["mu_by_hand"]
    # the circle passes through p0 and +-iy
    assert abs(abs(g["p0"] - mu) - r) < 1e-12
    assert abs(abs(1j * g["y"] - mu) - r) < 1e-12


@pytest.mark.parametrize("fn", [rexi.FN_EXP, rexi.FN_PSI1, rexi.FN_PSI2])
@pytest.mark.parametrize("N,p0,y", [(128, 10.0, 30.0), (64, 6.0, 14.0)])
def test_trapezoid_error_closed_form(fn, N, p0, y):
    a, b, r, mu = rexi.coefficients_mp(fn, N, p0, y)
    f = {rexi.FN_EXP: lambda z: mpmath.exp(z),
         rexi.FN_PSI1: lambda z: (mpmath.exp(z) - 1) / z if z != 0 else mpmath.mpf(1),
         rexi.FN_PSI2: lambda z: (mpmath.exp(z) - 1 - z) / z ** 2 if z != 0 else mpmath.mpf(0.5)}[fn]
    with mpmath.workdps(40):
        for w in [0.0, 0.37 * y, -0.61 * y, 0.2 * y]:
            x = mpmath.mpc(0.013 * y, w) if fn else mpmath.mpc(0, w)
            approx = rexi.rexi_sum_mp(a, b, x)
            t = (x - mu) / r
            predicted = -(t ** N) * f(x)
            err = approx - f(x)
            assert abs(err - predicted) <= 2e-2 * abs(predicted), (w, err, predicted)


def test_conjugate_pairs_and_sum_at_zero():
    alpha, beta, r, mu = rexi.coefficients(rexi.FN_EXP, 128, 10.0, 30.0)
    N = alpha.size
    assert np.all(alpha[::-1] == np.conj(alpha))
    assert np.all(beta[::-1] == np.conj(beta))
    # no pole on the real axis
    assert np.min(np.abs(alpha.imag)) > 0
    # S(0) = sum beta / alpha = 1 up to the geometric error (mu/r)^N and rounding
    S0 = np.sum(beta / alpha)
    bound = (abs(mu) / r) ** N + 8 * np.finfo(float).eps * rexi.kappa(alpha, beta, 0.0)[0]
    assert abs(S0 - 1.0) <= bound


def test_fp64_coefficients_on_imaginary_interval():
    """Max |S(i w) - e^{i w}| over |w| <= rho with the coefficients rounded once to
    FP64: within the geometric bound plus a rounding floor of a few u * kappa."""
    p0, y, N = 10.0, 30.0, 128
    alpha, beta, r, mu = rexi.coefficients(rexi.FN_EXP, N, p0, y)
    rho = 6.098  # spectral radius of dt L for T31, dt = 3600 s
    w = np.linspace(-rho, rho, 801)
    err = np.abs(rexi.rexi_sum(alpha, beta, 1j * w) - np.exp(1j * w))
    geo = (np.abs(1j * w - mu) / r) ** N
    floor = 8 * np.finfo(float).eps * rexi.kappa(alpha, beta, 1j * w)
    assert np.all(err <= 1.05 * geo + floor)
    assert err.max() < 3e-12


@pytest.mark.parametrize("N,p0,y", [(128, 10.0, 30.0), (256, 8.0, 67.9), (800, 8.0, 67.91071976436587)])
def test_kappa_at_the_centre_closed_form(N, p0, y):
    """kappa(mu) = (1/N) sum_n e^{mu + r cos theta_n} = e^{p0} i0e(r) (I_0 scaled by
    e^{-r}; mu + r = p0), with aliasing terms below 2 I_N(r)/I_0(r) ~ 1e-30 here."""
    alpha, beta, r, mu = rexi.coefficients(rexi.FN_EXP, N, p0, y)
    got = rexi.kappa(alpha, beta, mu)[0]
    ref = np.exp(p0) * scipy.special.i0e(r)
    assert abs(got - ref) <= 1e-13 * ref * np.sqrt(N), (got, ref)


@pytest.mark.parametrize("x", [0.0, 3.1j, -5.7j, 2.0 + 1.0j])
def test_kappa_matches_mpmath(x):
    """kappa against a 40-digit evaluation on the unrounded coefficients."""
    a_mp, b_mp, _, _ = rexi.coefficients_mp(rexi.FN_EXP, 128, 10.0, 30.0)
    with mpmath.workdps(40):
        X = mpmath.mpc(x)
        ref = float(sum(abs(b) / abs(X + a) for a, b in zip(a_mp, b_mp)))
    alpha, beta, _, _ = rexi.coefficients(rexi.FN_EXP, 128, 10.0, 30.0)
    assert abs(rexi.kappa(alpha, beta, x)[0] - ref) <= 1e-13 * ref
