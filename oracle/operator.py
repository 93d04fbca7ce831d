"""The linear operator L = L_g + L_c of the shallow-water equations in
spherical-harmonic space (oracle; test infrastructure).

Paper, Section 3 (vorticity-divergence form and the split U_t = L_g U + L_c U + N(U)):

    L_g:  Phi'_t = -Phi_bar delta,         delta_t = -lap Phi'
    L_c:  zeta_t = -f delta - V.grad f,    delta_t = f zeta + k.(grad f x V)

with f = 2 Omega sin(phi).  The state here is (h, zeta, delta) with h = Phi'/g
and Phi_bar = g H.  The paper does not print the spectral form of L_c (it says
only that keeping L_c in the linear part turns the per-term solve from diagonal
into a banded one, Section 5.3).  It is derived here from the PDE with the
recurrences  mu P_l = eps_{l+1} P_{l+1} + eps_l P_{l-1}  and
(1 - mu^2) dP_l/dmu = -l eps_{l+1} P_{l+1} + (l+1) eps_l P_{l-1},
eps_l^m = sqrt((l^2 - m^2) / (4 l^2 - 1)), and psi = -a^2 zeta / (l(l+1)),
chi = -a^2 delta / (l(l+1)).  For degree k >= max(m, 1), with q_k = 2 Omega / (k(k+1))
and the e^{+i m lambda} convention:

    h_t[k]     = -H delta[k]
    zeta_t[k]  = i m q_k zeta[k]  - 2 Omega [ (k+1)/k eps_k delta[k-1] + k/(k+1) eps_{k+1} delta[k+1] ]
    delta_t[k] = g k(k+1)/a^2 h[k] + i m q_k delta[k]
                 + 2 Omega [ (k+1)/k eps_k zeta[k-1] + k/(k+1) eps_{k+1} zeta[k+1] ]

Couplings to degrees outside [max(m, 1), L] are dropped (Galerkin truncation;
the l = 0 parts of zeta and delta carry no flow).  The rows of zeta and delta at
k = 0 are zero.  This formula is checked in tests against a brute-force
grid-space evaluation of L_c through the oracle's own transforms.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Params:
    """Planet and layer constants (defaults: Earth, 10 km mean depth)."""
    a: float = 6.37122e6
    g: float = 9.80616
    H: float = 1.0e4
    Omega: float = 7.292e-5


def n_modes(L: int) -> int:
    """Number of (l, m) pairs with 0 <= m <= l <= L."""
    return (L + 1) * (L + 2) // 2


def mode_index(L: int, l: int, m: int) -> int:
    """m-major position of (l, m): all degrees of m = 0 first, then m = 1, ..."""
    return m * (2 * L + 3 - m) // 2 + (l - m)


def eps(l: int, m: int) -> float:
    """eps_l^m = sqrt((l^2 - m^2) / (4 l^2 - 1)); zero for l <= m."""
    if l <= m or l <= 0:
        return 0.0
    return float(np.sqrt((l * l - m * m) / (4.0 * l * l - 1.0)))


def operator_matrix(m: int, L: int, p: Params) -> np.ndarray:
    """Dense matrix of L restricted to zonal order m.

    Unknown ordering: (h_k, zeta_k, delta_k) for k = m, m+1, ..., L, i.e. entry
    3 (k - m) + f with f = 0 (h), 1 (zeta), 2 (delta).
    """
    n = L - m + 1
    A = np.zeros((3 * n, 3 * n), dtype=np.complex128)
    kmin = max(m, 1)
    for k in range(m, L + 1):
        i = k - m
        A[3 * i + 0, 3 * i + 2] = -p.H
        if k < 1:
            continue
        Nk = k * (k + 1)
        q = 2.0 * p.Omega / Nk
        A[3 * i + 1, 3 * i + 1] = 1j * m * q
        A[3 * i + 2, 3 * i + 2] = 1j * m * q
        A[3 * i + 2, 3 * i + 0] = p.g * Nk / (p.a * p.a)
        if k - 1 >= kmin:
            c = 2.0 * p.Omega * (k + 1) / k * eps(k, m)
            A[3 * i + 1, 3 * (i - 1) + 2] = -c
            A[3 * i + 2, 3 * (i - 1) + 1] = +c
        if k + 1 <= L:
            c = 2.0 * p.Omega * k / (k + 1) * eps(k + 1, m)
            A[3 * i + 1, 3 * (i + 1) + 2] = -c
            A[3 * i + 2, 3 * (i + 1) + 1] = +c
    return A


def energy_scale(m: int, L: int, p: Params) -> np.ndarray:
    """Square roots of the energy weights, in operator_matrix's unknown ordering.

    The linear SWE conserve g |h|^2 + H a^2 / (l(l+1)) (|zeta|^2 + |delta|^2)
    (per mode), so with D = diag(energy_scale) the matrix D A D^{-1} is
    skew-Hermitian (the l = 0 entries of zeta, delta, which carry no flow, get
    weight 1).  Working in these variables removes the 1e15 spread of scales
    between the h and the zeta/delta entries of A.
    """
    out = []
    for k in range(m, L + 1):
        N = k * (k + 1)
        s = p.a * np.sqrt(p.H / N) if N else 1.0
        out += [np.sqrt(p.g), s, s]
    return np.array(out)


def gather_m(U: np.ndarray, m: int, L: int) -> np.ndarray:
    """Interleaved vector (h_k, zeta_k, delta_k)_{k=m..L} from U[3, modes]."""
    s = mode_index(L, m, m)
    n = L - m + 1
    v = np.empty(3 * n, dtype=np.complex128)
    for f in range(3):
        v[f::3] = U[f, s:s + n]
    return v


def scatter_m(U: np.ndarray, v: np.ndarray, m: int, L: int) -> None:
    """Inverse of gather_m: write the interleaved vector back into U[3, modes]."""
    s = mode_index(L, m, m)
    n = L - m + 1
    for f in range(3):
        U[f, s:s + n] = v[f::3]


def apply(U: np.ndarray, L: int, p: Params) -> np.ndarray:
    """L U for a spectral state U[3, modes] (h, zeta, delta)."""
    out = np.zeros_like(U)
    for m in range(L + 1):
        scatter_m(out, operator_matrix(m, L, p) @ gather_m(U, m, L), m, L)
    return out


def spectral_radius_bound(L: int, dt: float, p: Params) -> float:
    """rho = dt (sqrt(g H L (L+1)) / a + 2 Omega): bounds |eigenvalues of dt L|.

    The gravity part has eigenvalues +-i sqrt(g H l(l+1)) / a; the Coriolis part
    adds at most 2 Omega in magnitude.  The REXI contour must enclose i[-rho, rho]
    (Section 4.2.1: the contour must enclose all relevant eigenvalues).
    """
    return dt * (np.sqrt(p.g * p.H * L * (L + 1)) / p.a + 2.0 * p.Omega)
