"""Spherical-harmonic transforms on a Gauss grid (oracle; test infrastructure).

Paper, Section 3.2: pseudo-spectral discretisation with spherical harmonics;
non-linear terms are formed on the grid and transformed back and forth.  The
paper uses a library for the transforms and does not state its conventions, so
the conventions below are readings:

* Gauss-Legendre latitudes, mu_j = sin(phi_j) descending (north to south),
  weights summing to 2; longitudes lambda_k = 2 pi k / nlon.
* Pbar_lm normalised so that integral_{-1}^{1} Pbar_lm^2 dmu = 1, no
  Condon-Shortley phase.  A real field is
      f(lambda, mu) = sum_l Pbar_l0 Re f_l0 + 2 Re sum_{m>=1} sum_l f_lm Pbar_lm e^{i m lambda}
  and only m >= 0 is stored.
* Vector fields are carried as U = u cos(phi), V = v cos(phi).  With
  H_lm = (1 - mu^2) dPbar_lm/dmu:
      U_m = (1/a) sum_l [ -psi_lm H_lm + i m chi_lm Pbar_lm ]
      V_m = (1/a) sum_l [  i m psi_lm Pbar_lm + chi_lm H_lm ]
  and for a cos-weighted pair (A, B) with Fourier coefficients A_m, B_m:
      div_lm  = (1/a) sum_j w_j / (1 - mu_j^2) [ i m A_m Pbar_lm - B_m H_lm ]
      curl_lm = (1/a) sum_j w_j / (1 - mu_j^2) [ i m B_m Pbar_lm + A_m H_lm ]

Gauss nodes come from this module's own Newton iteration in colatitude (so that
sin(theta) keeps full relative accuracy near the poles); Pbar_lm comes from the
standard three-term recurrence in l with base-2 exponent tracking of the seed
Pbar_mm = c_m sin(theta)^m so that nothing underflows before it should.
"""
from __future__ import annotations

import numpy as np

from .operator import Params, mode_index, n_modes


def gauss_legendre(n: int):
    """Gauss-Legendre nodes (descending mu), sin(theta) and weights.

    Newton iteration on P_n(cos theta) in the colatitude theta for the northern
    half, seeded by the asymptotic guess theta_j = pi (j + 3/4) / (n + 1/2); the
    southern half is the mirror image (x -> -x), and for odd n the middle node is
    x = 0.  P_n is evaluated in terms of t = 1 - x = 2 sin^2(theta/2) with
    Reinsch's modification of the three-term recurrence (it carries the
    differences D_k = P_k - P_{k-1}), so nothing cancels near the pole.  The
    weight is w = 2 / ((1 - x^2) P_n'(x)^2) with
    (1 - x^2) P_n'(x) = n (P_{n-1} - x P_n) = n (t P_n - D_n).
    """
    half = n // 2

    def legendre_t(t):
        p = np.ones_like(t)               # P_0
        d = -t                            # D_1 = P_1 - P_0 = -t
        p = p + d                         # P_1
        for k in range(2, n + 1):
            d = ((k - 1) * d - (2 * k - 1) * t * p) / k
            p = p + d
        return p, d                       # P_n, D_n

    j = np.arange(half, dtype=np.float64)
    theta = np.pi * (j + 0.75) / (n + 0.5)
    for _ in range(100):
        t = 2.0 * np.sin(0.5 * theta) ** 2
        s = np.sin(theta)
        p, d = legendre_t(t)
        dpdtheta = -n * (t * p - d) / s   # d/dtheta P_n(cos theta)
        dtheta = p / dpdtheta
        theta = theta - dtheta
        if half == 0 or np.max(np.abs(dtheta)) < 1e-17:
            break
    t = 2.0 * np.sin(0.5 * theta) ** 2
    s = np.sin(theta)
    x = np.cos(theta)
    p, d = legendre_t(t)
    w = 2.0 * s * s / (n * (t * p - d)) ** 2
    if n % 2:
        # middle node x = 0 (t = 1):  (1 - x^2) P_n' = n P_{n-1}(0)
        q, dq = legendre_t(np.ones(1))
        xm, sm, wm = np.zeros(1), np.ones(1), 2.0 / (n * (q - dq)) ** 2
    else:
        xm = sm = wm = np.zeros(0)
    X = np.concatenate([x, xm, -x[::-1]])
    S = np.concatenate([s, sm, s[::-1]])
    W = np.concatenate([w, wm, w[::-1]])
    return X, S, W


def legendre_m(m: int, lmax: int, x: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Pbar_lm(x_j) for l = m..lmax as an array [lmax - m + 1, len(x)].

    Seed Pbar_mm = c_m s^m with c_0 = 1/sqrt(2), c_m = c_{m-1} sqrt((2m+1)/(2m));
    Pbar_{m+1,m} = sqrt(2m+3) x Pbar_mm;
    Pbar_lm = (x Pbar_{l-1,m} - eps_{l-1} Pbar_{l-2,m}) / eps_l.
    The seed is carried as mantissa * 2^e (e <= 0) until the values grow back
    into range, so nothing is lost to underflow that the true value would keep.
    """
    nl = lmax - m + 1
    out = np.zeros((nl, len(x)))
    log2c = -0.5 + 0.5 * np.sum(np.log2((2.0 * np.arange(1, m + 1) + 1) / (2.0 * np.arange(1, m + 1))))
    log2seed = log2c + m * np.log2(s)
    e = np.where(log2seed < -900.0, np.floor(log2seed), 0.0).astype(np.int64)
    v_prev = np.exp2(log2seed - e)                      # mantissa of Pbar_mm
    out[0] = np.ldexp(v_prev, e)
    if nl == 1:
        return out
    v_cur = np.sqrt(2.0 * m + 3.0) * x * v_prev         # mantissa of Pbar_{m+1,m}
    out[1] = np.ldexp(v_cur, e)
    for i in range(2, nl):
        l = m + i
        el = np.sqrt((l * l - m * m) / (4.0 * l * l - 1.0))
        elm1 = np.sqrt(((l - 1) ** 2 - m * m) / (4.0 * (l - 1) ** 2 - 1.0))
        v_next = (x * v_cur - elm1 * v_prev) / el
        v_prev, v_cur = v_cur, v_next
        big = (e < 0) & (np.abs(v_cur) > 2.0 ** 600)
        if np.any(big):
            sh = np.where(big, np.minimum(600, -e), 0)
            v_prev = np.ldexp(v_prev, -sh)
            v_cur = np.ldexp(v_cur, -sh)
            e = e + sh
        out[i] = np.ldexp(v_cur, e)
    return out


class Grid:
    """Gauss grid of nlat x nlon points for truncation L, with per-m tables."""

    def __init__(self, L: int, nlat: int, nlon: int, p: Params = Params()):
        if nlon <= 2 * L:
            raise ValueError("nlon must exceed 2L")
        if nlat <= L:
            raise ValueError("nlat must exceed L")
        self.L, self.nlat, self.nlon, self.p = L, nlat, nlon, p
        self.mu, self.sint, self.w = gauss_legendre(nlat)
        self.lam = 2.0 * np.pi * np.arange(nlon) / nlon
        self._P = {}
        self._H = {}

    def P(self, m: int) -> np.ndarray:
        """Pbar_lm(mu_j), l = m..L, shape [L - m + 1, nlat]."""
        if m not in self._P:
            self._tables(m)
        return self._P[m]

    def H(self, m: int) -> np.ndarray:
        """H_lm(mu_j) = (1 - mu^2) dPbar_lm/dmu, l = m..L, shape [L - m + 1, nlat].

        H_lm = -l eps_{l+1} Pbar_{l+1,m} + (l+1) eps_l Pbar_{l-1,m}.
        """
        if m not in self._H:
            self._tables(m)
        return self._H[m]

    def _tables(self, m: int) -> None:
        L = self.L
        Pe = legendre_m(m, L + 1, self.mu, self.sint)   # up to L+1 for H
        H = np.zeros((L - m + 1, self.nlat))
        for l in range(m, L + 1):
            i = l - m
            e1 = np.sqrt(((l + 1) ** 2 - m * m) / (4.0 * (l + 1) ** 2 - 1.0))
            H[i] = -l * e1 * Pe[i + 1]
            if l > m:
                e0 = np.sqrt((l * l - m * m) / (4.0 * l * l - 1.0))
                H[i] += (l + 1) * e0 * Pe[i - 1]
        self._P[m] = Pe[: L - m + 1]
        self._H[m] = H

    # -- scalar transforms -------------------------------------------------
    def _fourier_to_grid(self, F: np.ndarray) -> np.ndarray:
        """F[m, j] (m = 0..L) -> real grid [nlat, nlon]:  F_0 + 2 Re sum_m F_m e^{i m lambda}."""
        X = np.zeros((self.nlat, self.nlon // 2 + 1), dtype=np.complex128)
        X[:, : self.L + 1] = F.T
        return np.fft.irfft(X, n=self.nlon, axis=1) * self.nlon

    def _grid_to_fourier(self, f: np.ndarray) -> np.ndarray:
        """Real grid -> F[m, j] = (1/nlon) sum_k f_jk e^{-i m lambda_k}, m = 0..L."""
        X = np.fft.rfft(f, axis=1) / self.nlon
        return X[:, : self.L + 1].T.copy()

    def synthesis(self, spec: np.ndarray) -> np.ndarray:
        """Spectral [modes] complex -> grid [nlat, nlon] real."""
        L = self.L
        F = np.zeros((L + 1, self.nlat), dtype=np.complex128)
        for m in range(L + 1):
            s = mode_index(L, m, m)
            F[m] = spec[s: s + L - m + 1] @ self.P(m)
        return self._fourier_to_grid(F)

    def analysis(self, field: np.ndarray) -> np.ndarray:
        """Grid [nlat, nlon] real -> spectral [modes] complex (Gauss quadrature)."""
        L = self.L
        F = self._grid_to_fourier(field)
        out = np.zeros(n_modes(L), dtype=np.complex128)
        for m in range(L + 1):
            s = mode_index(L, m, m)
            out[s: s + L - m + 1] = self.P(m) @ (self.w * F[m])
        return out

    # -- vector transforms -------------------------------------------------
    def uv_from_psichi(self, psi: np.ndarray, chi: np.ndarray):
        """(psi, chi) spectral -> (U, V) = (u cos phi, v cos phi) on the grid."""
        L, a = self.L, self.p.a
        FU = np.zeros((L + 1, self.nlat), dtype=np.complex128)
        FV = np.zeros((L + 1, self.nlat), dtype=np.complex128)
        for m in range(L + 1):
            s = mode_index(L, m, m)
            ps = psi[s: s + L - m + 1]
            ch = chi[s: s + L - m + 1]
            P, H = self.P(m), self.H(m)
            FU[m] = (-(ps @ H) + 1j * m * (ch @ P)) / a
            FV[m] = (1j * m * (ps @ P) + (ch @ H)) / a
        return self._fourier_to_grid(FU), self._fourier_to_grid(FV)

    def div_curl(self, A: np.ndarray, B: np.ndarray):
        """Spectral divergence and curl of the vector whose cos-weighted
        components on the grid are (A, B)."""
        L, a = self.L, self.p.a
        FA = self._grid_to_fourier(A)
        FB = self._grid_to_fourier(B)
        wt = self.w / (self.sint ** 2)
        div = np.zeros(n_modes(L), dtype=np.complex128)
        curl = np.zeros(n_modes(L), dtype=np.complex128)
        for m in range(L + 1):
            s = mode_index(L, m, m)
            P, H = self.P(m), self.H(m)
            Am, Bm = wt * FA[m], wt * FB[m]
            div[s: s + L - m + 1] = (1j * m * (P @ Am) - (H @ Bm)) / a
            curl[s: s + L - m + 1] = (1j * m * (P @ Bm) + (H @ Am)) / a
        return div, curl


def degree_array(L: int) -> np.ndarray:
    """l for every stored mode, in m-major order."""
    out = np.empty(n_modes(L), dtype=np.int64)
    for m in range(L + 1):
        s = mode_index(L, m, m)
        out[s: s + L - m + 1] = np.arange(m, L + 1)
    return out


def order_array(L: int) -> np.ndarray:
    """m for every stored mode, in m-major order."""
    out = np.empty(n_modes(L), dtype=np.int64)
    for m in range(L + 1):
        s = mode_index(L, m, m)
        out[s: s + L - m + 1] = m
    return out


def inv_laplacian(spec: np.ndarray, L: int, a: float) -> np.ndarray:
    """lap^{-1} in spectral space: multiply by -a^2 / (l(l+1)); the l = 0 part is 0."""
    l = degree_array(L).astype(np.float64)
    out = np.zeros_like(spec)
    nz = l > 0
    out[nz] = -a * a * spec[nz] / (l[nz] * (l[nz] + 1.0))
    return out
