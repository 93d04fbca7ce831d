"""Non-linear terms, explicit RK2 and Strang splitting (oracle; test infrastructure).

Paper, Section 3 (the N(U) column of the split):

    N_Phi   = -V.grad Phi' - Phi' div V   = -div(Phi' V)
    N_zeta  = -div(zeta V)
    N_delta =  k.curl(zeta V) - lap (V.V / 2)

In h = Phi'/g variables N_h = -div(h V).  zeta is the relative vorticity (the
Coriolis terms belong to L here, the paper's ``l`` term of Table 1).  The
products are formed pointwise on the Gauss grid (pseudo-spectral, Section 3.2)
with velocities from psi = lap^{-1} zeta, chi = lap^{-1} delta.

Time stepping (Section 4.1 and Section 4.4):
* ``heun``: the second-order explicit Runge-Kutta method (``erk``, Table 2); the
  paper does not name the variant, Heun's method is the reading used here.
* ``strang_ver1``: N^{dt/2} o L^{dt} o N^{dt/2} (Section 4.4, version 1), with the
  linear part by REXI (Eq. rexi) -- scheme ``l_rexi_n_erk_ver1``.
"""
from __future__ import annotations

import numpy as np

from . import linear
from .operator import Params
from .sht import Grid, degree_array, inv_laplacian


def tendency(grid: Grid, U: np.ndarray) -> np.ndarray:
    """N(U) for a spectral state U[3, modes] = (h, zeta, delta)."""
    L, a = grid.L, grid.p.a
    h, zeta, delta = U
    psi = inv_laplacian(zeta, L, a)
    chi = inv_laplacian(delta, L, a)
    hg = grid.synthesis(h)
    zg = grid.synthesis(zeta)
    Ug, Vg = grid.uv_from_psichi(psi, chi)
    div_h, _ = grid.div_curl(hg * Ug, hg * Vg)
    div_z, curl_z = grid.div_curl(zg * Ug, zg * Vg)
    ke = (Ug * Ug + Vg * Vg) / (2.0 * (grid.sint[:, None] ** 2))
    ke_s = grid.analysis(ke)
    l = degree_array(L).astype(np.float64)
    out = np.empty_like(U, dtype=np.complex128)
    out[0] = -div_h
    out[1] = -div_z
    out[2] = curl_z + (l * (l + 1.0) / (a * a)) * ke_s       # -lap KE
    return out


def heun(grid: Grid, U: np.ndarray, tau: float, tend=None) -> np.ndarray:
    """U + tau/2 (N(U) + N(U + tau N(U))) (tend: another explicit right-hand side)."""
    f = tendency if tend is None else tend
    N0 = f(grid, U)
    N1 = f(grid, U + tau * N0)
    return U + 0.5 * tau * (N0 + N1)


def tendency_lc(grid: Grid, U: np.ndarray) -> np.ndarray:
    """N(U) + L_c U: the explicit part when only L_g is treated by REXI (Section 3
    splitting L = L_g + L_c); L_c is the Coriolis part of the spectral operator."""
    from dataclasses import replace

    from .operator import apply
    return tendency(grid, U) + apply(U, grid.L, grid.p) - apply(U, grid.L, replace(grid.p, Omega=0.0))


def strang_ver1(grid: Grid, U: np.ndarray, dt: float, alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """One step of l_rexi_n_erk_ver1: N^{dt/2} o REXI^{dt} o N^{dt/2}."""
    U = heun(grid, U, 0.5 * dt)
    U = linear.rexi_linear_step(U, alpha, beta, dt, grid.L, grid.p)
    return heun(grid, U, 0.5 * dt)


def split_step(grid: Grid, U: np.ndarray, dt: float, version: int, alpha=None, beta=None,
               lg: bool = False) -> np.ndarray:
    """One Strang-split step (Section 4.4) with Heun for N and, for the linear
    part, the REXI sum (alpha, beta given) or Crank-Nicolson (alpha None):
    version 1: N^{dt/2} o L^{dt} o N^{dt/2};  version 0: L^{dt/2} o N^{dt} o L^{dt/2}.
    lg: the linear part is L_g alone and L_c joins N (lg_rexi_lc_n_erk_ver1)."""
    from dataclasses import replace
    L = grid.L
    p = replace(grid.p, Omega=0.0) if lg else grid.p
    tend = tendency_lc if lg else None

    def lin(V, h):
        if alpha is None:
            return linear.cn_step(V, h, L, p)
        return linear.rexi_linear_step(V, alpha, beta, h, L, p)

    if version == 1:
        return heun(grid, lin(heun(grid, U, 0.5 * dt, tend), dt), 0.5 * dt, tend)
    return lin(heun(grid, lin(U, 0.5 * dt), dt, tend), 0.5 * dt)


def etdrk2(grid: Grid, U: np.ndarray, dt: float, alpha: np.ndarray, beta0: np.ndarray, beta1: np.ndarray,
           beta2: np.ndarray) -> np.ndarray:
    """One step of l_rexi_n_etdrk (Section 4.3, Eq. etdrk), the matrix functions
    psi_0, psi_1, psi_2 of dt L applied through their REXI sums on one contour:
      A = psi_0(dt L) U + dt psi_1(dt L) N(U),  U1 = A + dt psi_2(dt L) (N(A) - N(U))."""
    L, p = grid.L, grid.p
    N0 = tendency(grid, U)
    A = linear.rexi_linear_step(U, alpha, beta0, dt, L, p) + dt * linear.rexi_linear_step(N0, alpha, beta1, dt, L, p)
    NA = tendency(grid, A)
    return A + dt * linear.rexi_linear_step(NA - N0, alpha, beta2, dt, L, p)


def full_tendency(grid: Grid, U: np.ndarray) -> np.ndarray:
    """(L + N)(U): the whole right-hand side of Eq. (sw_compact)."""
    from .operator import apply
    return apply(U, grid.L, grid.p) + tendency(grid, U)


def rk4(grid: Grid, U: np.ndarray, dt: float, nsteps: int) -> np.ndarray:
    """Classical RK4 on the full system; the paper's reference solutions are RK4
    with a very small step (Section 5)."""
    for _ in range(nsteps):
        k1 = full_tendency(grid, U)
        k2 = full_tendency(grid, U + 0.5 * dt * k1)
        k3 = full_tendency(grid, U + 0.5 * dt * k2)
        k4 = full_tendency(grid, U + dt * k3)
        U = U + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return U
