"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds no part of the method's arithmetic: it only draws random
spectral coefficients and projects a prescribed zonal-jet height profile onto
Legendre polynomials with numpy's own Gauss-Legendre routines.  Spectral arrays
are complex128 [3, modes] holding (h, zeta, delta) in m-major order
(index of (l, m) = m (2L + 3 - m) / 2 + (l - m)).

The paper's barotropic-instability initial condition and reference data are not
available; these fields stand in for them:
* ``random_state``: x_lm = A (l + 1)^-2 (xi_1 + i xi_2) / sqrt(2), xi ~ N(0, 1),
  real for m = 0, zero l = 0 part of zeta and delta.
* ``jet_state``: a mid-latitude zonal jet (height step of 100 m across
  45N, width pi/36, vorticity from geostrophic balance at f_0 = 2 Omega sin(pi/4))
  plus small random perturbations of the same spectral shape.
"""
from __future__ import annotations

import numpy as np

EARTH = dict(a=6.37122e6, g=9.80616, H=1.0e4, Omega=7.292e-5)


def n_modes(L: int) -> int:
    return (L + 1) * (L + 2) // 2


def _degrees_orders(L: int):
    ls, ms = [], []
    for m in range(L + 1):
        for l in range(m, L + 1):
            ls.append(l)
            ms.append(m)
    return np.array(ls), np.array(ms)


def random_field(L: int, rng: np.random.Generator, amp: float) -> np.ndarray:
    l, m = _degrees_orders(L)
    x = rng.standard_normal(l.size) + 1j * rng.standard_normal(l.size)
    x = amp * x / np.sqrt(2.0) / (l + 1.0) ** 2
    x[m == 0] = x[m == 0].real
    return x


def random_state(L: int, seed: int, amps=(100.0, 1.0e-5, 1.0e-5)) -> np.ndarray:
    """Random (h, zeta, delta) with amplitude (l+1)^-2."""
    rng = np.random.default_rng(seed)
    U = np.stack([random_field(L, rng, a) for a in amps])
    U[1, 0] = 0.0
    U[2, 0] = 0.0
    return U


def jet_state(L: int, seed: int, dh: float = 100.0, pert=(1.0, 1.0e-6, 1.0e-7),
              a: float = EARTH["a"], g: float = EARTH["g"], Omega: float = EARTH["Omega"]) -> np.ndarray:
    """Zonal jet plus random perturbation (see module docstring)."""
    x, w = np.polynomial.legendre.leggauss(2 * L + 8)
    phi = np.arcsin(x)
    h = -0.5 * dh * np.tanh((phi - np.pi / 4.0) / (np.pi / 36.0))
    V = np.polynomial.legendre.legvander(x, L)              # P_l(x), unnormalised
    ls = np.arange(L + 1)
    h_l0 = np.sqrt((2.0 * ls + 1.0) / 2.0) * (V.T @ (w * h))
    f0 = 2.0 * Omega * np.sin(np.pi / 4.0)
    z_l0 = -(g / f0) * ls * (ls + 1.0) / (a * a) * h_l0
    U = random_state(L, seed, amps=pert).astype(np.complex128)
    U[0, : L + 1] += h_l0          # m = 0 block occupies the first L + 1 entries
    U[1, : L + 1] += z_l0
    U[1, 0] = 0.0
    U[2, 0] = 0.0
    return U


def ensemble_members(count: int, seed: int, truncations=(63, 127, 255), pole_range=(100, 400)):
    """Mixed-truncation ensemble description: list of (L, N, seed) per member.

    Truncation drawn uniformly from ``truncations``; pole count N = 2 randint(lo, hi].
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        L = int(rng.choice(truncations))
        N = 2 * int(rng.integers(pole_range[0] + 1, pole_range[1] + 1))
        out.append((L, N, seed * 1000 + i))
    return out
