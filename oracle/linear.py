"""The REXI linear step (oracle; test infrastructure).

Paper, Section 4.2, Eq. (rexi):

    U(dt) = exp(dt L) U(0)  ~  sum_n beta_n (dt L + alpha_n)^{-1} U(0)

with alpha_n, beta_n from the Cauchy contour (Eq. cauchy_alpha / cauchy_beta).
L = L_g + L_c (the paper's ``l`` term, Table 1) acts on each zonal order m
separately, so for every pole n and every m the oracle assembles the full
3(L - m + 1) square system (dt A_m + alpha_n I) with unknowns interleaved
(h_k, zeta_k, delta_k) -- a band matrix with four sub- and four
super-diagonals -- and solves it with LAPACK's partially pivoted band solver.
The beta-weighted sum runs over n = 0..N-1 in order with Neumaier compensation
on the real and imaginary parts.

``expm_step`` is the exact exponential per m (scipy's dense expm), the reference
the REXI approximation is measured against (Section 4.2: exp(dt L) = Q exp(dt
Lambda) Q^{-1}).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .operator import Params, energy_scale, gather_m, mode_index, operator_matrix, scatter_m

KL = KU = 4


def _band(A: np.ndarray) -> np.ndarray:
    """LAPACK band storage ab[KU + i - j, j] = A[i, j]."""
    n = A.shape[0]
    ab = np.zeros((KL + KU + 1, n), dtype=A.dtype)
    for d in range(-KL, KU + 1):
        if abs(d) >= n:
            continue
        diag = np.diagonal(A, offset=d)
        if d >= 0:
            ab[KU - d, d:] = diag
        else:
            ab[KU - d, : n + d] = diag
    return ab


class _Neumaier:
    """Compensated running sum of complex vectors (real and imaginary parts separately)."""

    def __init__(self, n: int):
        self.s = np.zeros(n, dtype=np.complex128)
        self.c = np.zeros(n, dtype=np.complex128)

    @staticmethod
    def _step(s, c, x):
        t = s + x
        big = np.abs(s) >= np.abs(x)
        c = c + np.where(big, (s - t) + x, (x - t) + s)
        return t, c

    def add(self, x: np.ndarray) -> None:
        sr, cr = self._step(self.s.real, self.c.real, x.real)
        si, ci = self._step(self.s.imag, self.c.imag, x.imag)
        self.s = sr + 1j * si
        self.c = cr + 1j * ci

    def value(self) -> np.ndarray:
        return self.s + self.c


def rexi_step_m(u: np.ndarray, A: np.ndarray, alpha: np.ndarray, beta: np.ndarray,
                dt: float, d: np.ndarray) -> np.ndarray:
    """sum_n beta_n (dt A + alpha_n I)^{-1} u for one zonal order (Eq. rexi).

    Each system is solved in the energy-scaled unknowns y = D x (D = diag(d)):
    (dt D A D^{-1} + alpha_n I) y = D u, a diagonal equilibration that leaves the
    solution unchanged and keeps LAPACK's pivoting meaningful.
    """
    n = A.shape[0]
    dB = dt * (d[:, None] * A / d[None, :])
    du = d * u
    acc = _Neumaier(n)
    for a, b in zip(alpha, beta):
        M = dB + a * np.eye(n)
        y = scipy.linalg.solve_banded((KL, KU), _band(M), du)
        acc.add(b * y)
    return acc.value() / d


def rexi_term_magnitudes(U0: np.ndarray, alpha: np.ndarray, beta: np.ndarray, dt: float,
                         L: int, p: Params = Params(), orders=None) -> np.ndarray:
    """Per output entry, the sum over the poles of the magnitudes of the terms of
    Eq. (rexi): sum_n |beta_n| |((dt L + alpha_n)^{-1} U0)_j| (real array [3, modes]).

    Section 4.2.2: the terms of the sum are far larger than the result, so any
    evaluation with unit roundoff u carries an error of about u times this sum
    (the per-entry form of kappa; for U0 = h_00 alone it is kappa(0) |h_00|)."""
    M = np.zeros(U0.shape, dtype=np.float64)
    for m in (range(L + 1) if orders is None else orders):
        A = operator_matrix(m, L, p)
        d = energy_scale(m, L, p)
        n = A.shape[0]
        dB = dt * (d[:, None] * A / d[None, :])
        du = d * gather_m(U0, m, L)
        acc = np.zeros(n)
        for a, b in zip(alpha, beta):
            y = scipy.linalg.solve_banded((KL, KU), _band(dB + a * np.eye(n)), du)
            acc += np.abs(b) * np.abs(y)
        tmp = np.zeros(U0.shape, dtype=np.complex128)
        scatter_m(tmp, acc / d, m, L)
        s = mode_index(L, m, m)
        M[:, s:s + L - m + 1] = tmp[:, s:s + L - m + 1].real
    return M


def rexi_linear_step(U0: np.ndarray, alpha: np.ndarray, beta: np.ndarray, dt: float,
                     L: int, p: Params = Params(), orders=None) -> np.ndarray:
    """REXI approximation of exp(dt L) U0 for a state U0[3, modes] (h, zeta, delta).

    ``orders`` restricts the work to a subset of zonal orders (the other entries of
    the result are left zero); used for bounded samples at large truncations.
    """
    U1 = np.zeros_like(U0, dtype=np.complex128)
    for m in (range(L + 1) if orders is None else orders):
        A = operator_matrix(m, L, p)
        d = energy_scale(m, L, p)
        scatter_m(U1, rexi_step_m(gather_m(U0, m, L), A, alpha, beta, dt, d), m, L)
    return U1


def expm_step(U0: np.ndarray, dt: float, L: int, p: Params = Params()) -> np.ndarray:
    """exp(dt L) U0 by a dense matrix exponential per zonal order, taken in the
    energy-scaled unknowns: exp(dt A) = D^{-1} exp(dt D A D^{-1}) D."""
    U1 = np.zeros_like(U0, dtype=np.complex128)
    for m in range(L + 1):
        d = energy_scale(m, L, p)
        B = d[:, None] * operator_matrix(m, L, p) / d[None, :]
        E = scipy.linalg.expm(dt * B)
        scatter_m(U1, (E @ (d * gather_m(U0, m, L))) / d, m, L)
    return U1


def psi_step(U0: np.ndarray, dt: float, L: int, k: int, p: Params = Params()) -> np.ndarray:
    """psi_k(dt L) U0 for k = 1, 2 (psi_1(K) = K^-1 (e^K - I), psi_2(K) = K^-2 (e^K - I - K),
    Section 4.3) by one dense exponential per zonal order of the augmented matrix
    [[dt A, b, 0], [0, 0, 1], [0, 0, 0]], whose exponential carries psi_1(dt A) b and
    psi_2(dt A) b in its last two columns (energy-scaled unknowns as in expm_step)."""
    U1 = np.zeros_like(U0, dtype=np.complex128)
    for m in range(L + 1):
        d = energy_scale(m, L, p)
        B = d[:, None] * operator_matrix(m, L, p) / d[None, :]
        n = B.shape[0]
        M = np.zeros((n + 2, n + 2), dtype=np.complex128)
        M[:n, :n] = dt * B
        M[:n, n] = d * gather_m(U0, m, L)
        M[n, n + 1] = 1.0
        E = scipy.linalg.expm(M)
        scatter_m(U1, E[:n, n + k - 1] / d, m, L)
    return U1


def cn_step(U0: np.ndarray, dt: float, L: int, p: Params = Params(), a: float = 0.5) -> np.ndarray:
    """Crank-Nicolson (Section 4.1): (I - a dt L)^{-1} (I + (1 - a) dt L) U0."""
    U1 = np.zeros_like(U0, dtype=np.complex128)
    for m in range(L + 1):
        d = energy_scale(m, L, p)
        B = d[:, None] * operator_matrix(m, L, p) / d[None, :]
        I = np.eye(B.shape[0])
        rhs = (I + (1.0 - a) * dt * B) @ (d * gather_m(U0, m, L))
        y = scipy.linalg.solve_banded((KL, KU), _band(I - a * dt * B), rhs)
        scatter_m(U1, y / d, m, L)
    return U1
