"""Pins of the oracle's spectral operator L = L_g + L_c (Section 3).

* brute force: L_c applied through grid space (f = 2 Omega mu times the velocity,
  then divergence and curl by quadrature) on a grid fine enough for exact
  quadrature must equal the banded spectral formula;
* Omega = 0: eigenvalues are the gravity-wave frequencies +-i sqrt(g H l(l+1))/a;
* energy: L is skew-adjoint in the energy inner product
  g |h|^2 + H a^2 / (l(l+1)) (|zeta|^2 + |delta|^2)  (the linear SWE conserve energy);
* with delta = 0, the vorticity diagonal is the westward Rossby-Haurwitz phase
  speed 2 Omega / (l(l+1)) of the non-divergent barotropic wave on a sphere at rest;
* the eigenvalues of dt L lie inside the stated spectral-radius bound.
"""
import numpy as np
import pytest

from oracle import operator as op
from oracle.operator import Params
from oracle.sht import Grid, inv_laplacian
from paper_1805_06557_amd.inputs import random_state


def _grid_Lc(grid: Grid, U: np.ndarray) -> np.ndarray:
    """L_c U by grid-space evaluation: zeta_t = -div(f V), delta_t = curl(f V)."""
    L, p = grid.L, grid.p
    psi = inv_laplacian(U[1], L, p.a)
    chi = inv_laplacian(U[2], L, p.a)
    Ug, Vg = grid.uv_from_psichi(psi, chi)
    f = 2.0 * p.Omega * grid.mu[:, None]
    div, curl = grid.div_curl(f * Ug, f * Vg)
    out = np.zeros_like(U)
    out[1] = -div
    out[2] = curl
    return out


@pytest.mark.parametrize("L", [8, 13])
def test_coriolis_brute_force_grid(L):
    p = Params()
    grid = Grid(L, 2 * L + 4, 4 * L + 8, p)
    U = random_state(L, 11)
    ref = _grid_Lc(grid, U)
    # spectral operator with gravity switched off (g = H = 0 leaves L_c only)
    pc = Params(a=p.a, g=0.0, H=0.0, Omega=p.Omega)
    got = op.apply(U, L, pc)
    scale = np.abs(ref[1:]).max()
    np.testing.assert_allclose(got[0], 0.0, atol=0)
    np.testing.assert_allclose(got[1:], ref[1:], atol=1e-12 * scale)


def test_gravity_frequencies_without_rotation():
    p = Params(Omega=0.0)
    L = 8
    for m in range(L + 1):
        ev = np.linalg.eigvals(op.operator_matrix(m, L, p))
        want = []
        for l in range(m, L + 1):
            w = np.sqrt(p.g * p.H * l * (l + 1)) / p.a
            want += [1j * w, -1j * w, 0.0]
        key = lambda z: (round(z.imag * 1e9), round(z.real * 1e9))
        np.testing.assert_allclose(sorted(ev, key=key), sorted(want, key=key), atol=1e-18)


@pytest.mark.parametrize("L", [8, 31])
def test_energy_skew_adjoint(L):
    p = Params()
    for m in range(L + 1):
        A = op.operator_matrix(m, L, p)
        wts = []
        keep = []
        for k in range(m, L + 1):
            N = k * (k + 1)
            for f in range(3):
                if f == 0:
                    wts.append(p.g)
                    keep.append(True)
                else:
                    wts.append(p.H * p.a ** 2 / N if N else 1.0)
                    keep.append(N > 0)
        keep = np.array(keep)
        W = np.diag(np.array(wts)[keep])
        As = A[np.ix_(keep, keep)]
        S = W @ As + As.conj().T @ W
        assert np.abs(S).max() <= 1e-14 * np.abs(W @ As).max()


def test_rossby_haurwitz_phase_speed():
    p = Params()
    L = 10
    for m in range(1, L + 1):
        A = op.operator_matrix(m, L, p)
        for k in range(m, L + 1):
            i = 3 * (k - m) + 1
            c = A[i, i] / (1j * m)          # zeta ~ exp(i m (lambda + c t)): pattern moves west at c
            assert abs(c - 2 * p.Omega / (k * (k + 1))) < 1e-20


@pytest.mark.parametrize("L,dt", [(31, 3600.0), (20, 7200.0)])
def test_spectrum_inside_radius_bound(L, dt):
    p = Params()
    rho = op.spectral_radius_bound(L, dt, p)
    worst = 0.0
    for m in range(L + 1):
        ev = np.linalg.eigvals(dt * op.operator_matrix(m, L, p))
        assert np.abs(ev.real).max() < 1e-10 * rho
        worst = max(worst, np.abs(ev).max())
    assert worst <= rho
