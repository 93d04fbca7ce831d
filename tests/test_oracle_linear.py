"""Pins of the oracle's REXI linear step (Eq. rexi) against mathematics.

* dense matrix exponential at T8 (and per order at T31): L is normal in the
  energy inner product, so in that norm the REXI error is bounded by the largest
  scalar REXI error at an eigenvalue of dt L;
* the closed-form solution of the non-rotating linear SWE per (l, m):
  h(t) = h0 cos(wt) - (H/w) delta0 sin(wt), delta(t) = delta0 cos(wt) + (w/H) h0 sin(wt),
  zeta(t) = zeta0, with w = sqrt(g H l(l+1)) / a;
* the l = 0 height couples to nothing: h00' = S(0) h00 with S(0) = sum beta/alpha;
* m = 0 coefficients of a real field stay real; energy is conserved to the
  REXI error.
"""
import cmath
import math

import numpy as np
import pytest

from oracle import linear, rexi
from oracle import operator as op
from oracle.operator import Params
from paper_1805_06557_amd.inputs import random_state


def _energy(U, L, p):
    l = np.array([l for m in range(L + 1) for l in range(m, L + 1)], dtype=float)
    e = p.g * np.abs(U[0]) ** 2
    nz = l > 0
    e[nz] += p.H * p.a ** 2 / (l[nz] * (l[nz] + 1)) * (np.abs(U[1][nz]) ** 2 + np.abs(U[2][nz]) ** 2)
    # m > 0 coefficients stand for the +-m pair of a real field
    m = np.array([m for m in range(L + 1) for l in range(m, L + 1)])
    return np.sum(np.where(m > 0, 2.0, 1.0) * e)


def _scalar_error_at_eigs(alpha, beta, L, dt, p):
    worst = 0.0
    for m in range(L + 1):
        ev = np.linalg.eigvals(dt * op.operator_matrix(m, L, p))
        err = np.abs(rexi.rexi_sum(alpha, beta, ev) - np.exp(ev))
        worst = max(worst, err.max())
    return worst


@pytest.mark.parametrize("L,dt,N,p0,y", [(8, 3600.0, 128, 10.0, 30.0), (8, 7200.0, 64, 6.0, 14.0)])
def test_rexi_against_dense_expm(L, dt, N, p0, y):
    p = Params()
    alpha, beta, r, mu = rexi.coefficients(rexi.FN_EXP, N, p0, y)
    U0 = random_state(L, 5)
    got = linear.rexi_linear_step(U0, alpha, beta, dt, L, p)
    ref = linear.expm_step(U0, dt, L, p)
    bound = _scalar_error_at_eigs(alpha, beta, L, dt, p)
    diff = got - ref
    # energy-norm error (the l = 0 parts of zeta, delta are zero in the input)
    err = np.sqrt(_energy(diff, L, p) / _energy(U0, L, p))
    floor = 16 * np.finfo(float).eps * rexi.kappa(alpha, beta, 0.0)[0]
    assert err <= 1.01 * bound + floor, (err, bound, floor)
    # and the error is not trivially zero: the approximation is genuinely REXI
    assert err > 0.01 * bound


def test_rexi_against_expm_per_order_T31():
    """C1 shapes: T31, dt = 3600 s, the paper's contour (p0 = 10, y = 30, N = 128)."""
    L, dt = 31, 3600.0
    p = Params()
    alpha, beta, _, _ = rexi.coefficients(rexi.FN_EXP, 128, 10.0, 30.0)
    U0 = random_state(L, 0)
    got = linear.rexi_linear_step(U0, alpha, beta, dt, L, p)
    ref = linear.expm_step(U0, dt, L, p)
    err = np.sqrt(_energy(got - ref, L, p) / _energy(U0, L, p))
    assert err < 5e-12


def test_nonrotating_closed_form():
    L, dt = 12, 5400.0
    p = Params(Omega=0.0)
    rho = op.spectral_radius_bound(L, dt, p)
    y = 1.5 * rho
    alpha, beta, r, mu = rexi.coefficients(rexi.FN_EXP, 96, 4.0, y)
    U0 = random_state(L, 9)
    got = linear.rexi_linear_step(U0, alpha, beta, dt, L, p)
    idx = 0
    for m in range(L + 1):
        for l in range(m, L + 1):
            h0, z0, d0 = U0[:, idx]
            if l == 0:
                want = (h0 - p.H * d0 * dt, z0, d0)      # w = 0 limit
            else:
                w = np.sqrt(p.g * p.H * l * (l + 1)) / p.a
                c, s = np.cos(w * dt), np.sin(w * dt)
                want = (h0 * c - p.H / w * d0 * s, z0, d0 * c + w / p.H * h0 * s)
            for f in range(3):
                scale = np.abs(U0[f]).max()
                assert abs(got[f, idx] - want[f]) <= 1e-11 * scale, (l, m, f)
            idx += 1


def test_l0_height_and_m0_realness():
    L, dt = 15, 3600.0
    p = Params()
    alpha, beta, r, mu = rexi.coefficients(rexi.FN_EXP, 128, 10.0, 30.0)
    U0 = random_state(L, 2)
    U0[0, 0] = 1234.5                         # h_00
    got = linear.rexi_linear_step(U0, alpha, beta, dt, L, p)
    S0 = np.sum(beta / alpha)
    kap = rexi.kappa(alpha, beta, 0.0)[0]
    assert abs(got[0, 0] / U0[0, 0] - S0) <= 4 * np.finfo(float).eps * kap
    assert abs(S0 - 1.0) <= (abs(mu) / r) ** 128 + 8 * np.finfo(float).eps * kap
    # m = 0 block is the first L + 1 entries of every field
    assert np.abs(got[:, : L + 1].imag).max() <= 1e-13 * np.abs(got).max()


def test_energy_conserved_to_rexi_error():
    L, dt = 20, 3600.0
    p = Params()
    alpha, beta, _, _ = rexi.coefficients(rexi.FN_EXP, 128, 10.0, 30.0)
    U0 = random_state(L, 4)
    got = linear.rexi_linear_step(U0, alpha, beta, dt, L, p)
    e0, e1 = _energy(U0, L, p), _energy(got, L, p)
    assert abs(e1 / e0 - 1.0) < 1e-11


def test_crank_nicolson_nonrotating_amplification():
    """Section 4.1: CN with a = 1/2 multiplies a gravity mode by (1 + i w dt/2)/(1 - i w dt/2)."""
    L, dt = 6, 1800.0
    p = Params(Omega=0.0)
    U0 = random_state(L, 1)
    got = linear.cn_step(U0, dt, L, p)
    # the mode (h, delta) along the eigenvector of +i w: delta = -i (w/H) h
    idx = op.mode_index(L, 4, 2)
    w = np.sqrt(p.g * p.H * 20) / p.a
    V = np.zeros_like(U0)
    V[0, idx] = 1.0
    V[2, idx] = -1j * w / p.H
    out = linear.cn_step(V, dt, L, p)
    amp = (1 + 0.5j * w * dt) / (1 - 0.5j * w * dt)
    np.testing.assert_allclose(out[:, idx], amp * V[:, idx], rtol=1e-13)
    assert np.all(np.isfinite(got))


def _psi(k, z):
    """psi_1, psi_2 at a scalar (series near 0, where dt L has its zero eigenvalues)."""
    if abs(z) < 1e-3:
        return sum(z ** j / math.factorial(j + k) for j in range(8))
    e = cmath.exp(z)
    return (e - 1) / z if k == 1 else (e - 1 - z) / (z * z)


@pytest.mark.parametrize("fn,k", [(rexi.FN_PSI1, 1), (rexi.FN_PSI2, 2)])
def test_psi_sums_against_augmented_expm(fn, k):
    """The REXI sums of psi_1, psi_2 applied through the banded solves reproduce
    psi_k(dt L) U0 from the augmented-matrix exponential (an independent
    definition), at T8, to the scalar error of the sum plus its rounding floor."""
    L, dt, N, p0, y = 8, 3600.0, 128, 10.0, 30.0
    p = Params()
    alpha, beta, _, _ = rexi.coefficients(fn, N, p0, y)
    U0 = random_state(L, 6)
    got = linear.rexi_linear_step(U0, alpha, beta, dt, L, p)
    ref = linear.psi_step(U0, dt, L, k, p)
    # scalar error of the psi_k sum at the eigenvalues of dt L
    worst = 0.0
    for m in range(L + 1):
        ev = np.linalg.eigvals(dt * op.operator_matrix(m, L, p))
        f = np.array([_psi(k, complex(e)) for e in ev])
        worst = max(worst, float(np.abs(rexi.rexi_sum(alpha, beta, ev) - f).max()))
    err = np.sqrt(_energy(got - ref, L, p) / _energy(U0, L, p))
    floor = 16 * np.finfo(float).eps * rexi.kappa(alpha, beta, 0.0)[0]
    assert err <= 1.01 * worst + floor, (err, worst, floor)
    # and psi_k is not exp: the two differ by O(1)
    assert np.sqrt(_energy(got - linear.expm_step(U0, dt, L, p), L, p) / _energy(U0, L, p)) > 1e-2


def test_term_magnitudes_closed_forms():
    """The per-entry sum of the term magnitudes of Eq. (rexi) (the rounding floor
    of Section 4.2.2).  Without rotation a mode (l, m) couples h and delta only:
    (dt A + alpha) restricted to (h, delta) is [[alpha, -dt H], [dt g N / a^2, alpha]]
    (N = l(l+1)), so an input h0 alone gives the terms beta (alpha, -dt g N/a^2) h0 /
    (alpha^2 + dt^2 g H N / a^2); h_00 alone gives kappa(0) |h_00|.  And the sum of
    magnitudes bounds the magnitude of the sum."""
    L, dt = 6, 1800.0
    p = Params(Omega=0.0)
    alpha, beta, _, _ = rexi.coefficients(rexi.FN_EXP, 64, 6.0, 14.0)
    U0 = np.zeros((3, op.n_modes(L)), dtype=np.complex128)
    l, m, h0 = 4, 2, 3.0 - 2.0j
    idx = op.mode_index(L, l, m)
    U0[0, idx] = h0
    U0[0, 0] = 7.5
    M = linear.rexi_term_magnitudes(U0, alpha, beta, dt, L, p)
    c = dt * dt * p.g * p.H * l * (l + 1) / p.a ** 2
    den = np.abs(alpha ** 2 + c)
    want_h = np.sum(np.abs(beta) * np.abs(alpha) / den) * abs(h0)
    want_d = np.sum(np.abs(beta) / den) * dt * p.g * l * (l + 1) / p.a ** 2 * abs(h0)
    assert abs(M[0, idx] - want_h) <= 1e-12 * want_h
    assert abs(M[2, idx] - want_d) <= 1e-12 * want_d
    assert M[1, idx] == 0.0
    assert abs(M[0, 0] - rexi.kappa(alpha, beta, 0.0)[0] * 7.5) <= 1e-12 * M[0, 0]
    # rotation on, a random state: |sum| <= sum |.| entry by entry
    U1 = random_state(L, 3)
    q = Params()
    got = linear.rexi_linear_step(U1, alpha, beta, dt, L, q)
    M1 = linear.rexi_term_magnitudes(U1, alpha, beta, dt, L, q)
    assert np.all(np.abs(got) <= M1 * (1 + 1e-12) + 1e-300)
