"""Pins of the oracle's non-linear terms and time stepping (Section 3, Section 4).

* N vanishes for a fluid at rest with any height field;
* N_h has no l = 0 part (mass is conserved);
* solid-body zonal flow u = u0 cos(phi) with zonal h: N_h = N_zeta = 0 and
  N_delta = (2 u0^2 / a^2) P_2(mu), i.e. (2 u0^2 / a^2) sqrt(2/5) on Pbar_20;
* the geostrophically balanced solid-body flow (Williamson et al. test case 2,
  h = -(a Omega u0 + u0^2 / 2) mu^2 / g + const) is a steady state of the whole
  system: (L + N) U = 0 -- this ties the Coriolis operator, gravity and N together;
* Heun is second order; Strang version 1 (N^{dt/2} o REXI^{dt} o N^{dt/2}) is second
  order against a small-step RK4 solution of the whole system;
* RK4 itself: on a linear right-hand side one step is the degree-4 Taylor
  polynomial of the exponential.
"""
import numpy as np
import pytest

from oracle import nonlinear, rexi
from oracle.operator import Params, apply, mode_index, n_modes, spectral_radius_bound
from oracle.sht import Grid
from paper_1805_06557_amd.inputs import random_state


def _grid(L):
    return Grid(L, (3 * L + 3) // 2 + 1, 3 * L + 3 + (3 * L + 3) % 2)


def test_rest_state_has_no_tendency():
    L = 10
    g = _grid(L)
    U = random_state(L, 1)
    U[1:] = 0.0
    N = nonlinear.tendency(g, U)
    assert np.abs(N).max() == 0.0


def test_mass_conservation():
    L = 12
    g = _grid(L)
    U = random_state(L, 2)
    N = nonlinear.tendency(g, U)
    assert abs(N[0, 0]) <= 1e-15 * np.abs(N[0]).max()


def _solid_body(L, u0, p, h_profile=True):
    U = np.zeros((3, n_modes(L)), dtype=complex)
    U[1, mode_index(L, 1, 0)] = 2 * u0 / p.a * np.sqrt(2.0 / 3.0)
    if h_profile:
        # mu^2 = 1/3 + (2/3) P_2 = 1/3 sqrt(2) Pbar_00 + (2/3) sqrt(2/5) Pbar_20
        c = -(p.a * p.Omega * u0 + 0.5 * u0 ** 2) / p.g
        U[0, mode_index(L, 0, 0)] = c / 3.0 * np.sqrt(2.0)
        U[0, mode_index(L, 2, 0)] = c * 2.0 / 3.0 * np.sqrt(2.0 / 5.0)
    return U


def test_solid_body_closed_form():
    L = 10
    p = Params()
    g = _grid(L)
    u0 = 25.0
    U = _solid_body(L, u0, p)
    N = nonlinear.tendency(g, U)
    want = np.zeros_like(N)
    want[2, mode_index(L, 2, 0)] = 2 * u0 ** 2 / p.a ** 2 * np.sqrt(2.0 / 5.0)
    scale = abs(want[2, mode_index(L, 2, 0)])
    np.testing.assert_allclose(N[1:], want[1:], atol=1e-13 * scale)
    # N_h against the natural scale of its terms, |h| u0 / a
    np.testing.assert_allclose(N[0], 0.0, atol=1e-13 * np.abs(U[0]).max() * u0 / p.a)


def test_balanced_solid_body_is_steady():
    L = 10
    p = Params()
    g = _grid(L)
    u0 = 2 * np.pi * p.a / (12 * 86400.0)
    U = _solid_body(L, u0, p)
    LU = apply(U, L, p)
    T = LU + nonlinear.tendency(g, U)
    # zeta, delta: against the size of the balancing terms; h: against |h| u0 / a
    assert np.abs(T[1:]).max() <= 1e-13 * np.abs(LU[1:]).max()
    assert np.abs(T[0]).max() <= 1e-13 * np.abs(U[0]).max() * u0 / p.a
    assert np.abs(LU[2]).max() > 1e-12            # the balance is not trivial


def test_heun_second_order():
    L = 10
    g = _grid(L)
    U = random_state(L, 3, amps=(50.0, 2e-5, 2e-6))
    tau = 1800.0

    def run(n):
        V = U.copy()
        for _ in range(n):
            V = nonlinear.heun(g, V, tau / n)
        return V

    ref = run(64)
    e1 = np.abs(run(1) - ref).max()
    e2 = np.abs(run(2) - ref).max()
    assert 3.3 < e1 / e2 < 4.7


def test_strang_ver1_second_order():
    L = 8
    p = Params()
    g = _grid(L)
    U = random_state(L, 4, amps=(50.0, 2e-5, 2e-6))
    T = 2 * 3600.0
    ref = nonlinear.rk4(g, U, T / 160, 160)

    def run(n):
        dt = T / n
        rho = spectral_radius_bound(L, dt, p)
        a, b, _, _ = rexi.coefficients(rexi.FN_EXP, 128, 8.0, 1.5 * rho + 2.0)
        V = U.copy()
        for _ in range(n):
            V = nonlinear.strang_ver1(g, V, dt, a, b)
        return V

    e1 = np.abs(run(2)[0] - ref[0]).max()
    e2 = np.abs(run(4)[0] - ref[0]).max()
    assert 3.0 < e1 / e2 < 5.0, (e1, e2)


def test_etdrk2_second_order():
    """l_rexi_n_etdrk (Section 4.3) converges at second order to an RK4 reference."""
    L = 8
    p = Params()
    g = _grid(L)
    U = random_state(L, 4, amps=(50.0, 2e-5, 2e-6))
    T = 2 * 3600.0
    ref = nonlinear.rk4(g, U, T / 160, 160)

    def run(n):
        dt = T / n
        rho = spectral_radius_bound(L, dt, p)
        y = 1.5 * rho + 2.0
        a, b0, _, _ = rexi.coefficients(rexi.FN_EXP, 128, 8.0, y)
        _, b1, _, _ = rexi.coefficients(rexi.FN_PSI1, 128, 8.0, y)
        _, b2, _, _ = rexi.coefficients(rexi.FN_PSI2, 128, 8.0, y)
        V = U.copy()
        for _ in range(n):
            V = nonlinear.etdrk2(g, V, dt, a, b0, b1, b2)
        return V

    e1 = np.abs(run(2)[0] - ref[0]).max()
    e2 = np.abs(run(4)[0] - ref[0]).max()
    assert 3.0 < e1 / e2 < 5.0, (e1, e2)


@pytest.mark.parametrize("version,use_rexi", [(0, True), (1, False), (0, False)],
                         ids=["rexi-ver0", "cn-ver1", "cn-ver0"])
def test_split_schemes_second_order(version, use_rexi):
    """l_rexi_n_erk_ver0 and the Crank-Nicolson splittings l_irk_n_erk_ver0/1
    (Section 4.4) converge at second order to an RK4 reference."""
    L = 8
    p = Params()
    g = _grid(L)
    U = random_state(L, 4, amps=(50.0, 2e-5, 2e-6))
    T = 2 * 3600.0
    ref = nonlinear.rk4(g, U, T / 160, 160)

    def run(n):
        dt = T / n
        tl = dt if version == 1 else 0.5 * dt
        a = b = None
        if use_rexi:
            rho = spectral_radius_bound(L, tl, p)
            a, b, _, _ = rexi.coefficients(rexi.FN_EXP, 128, 8.0, 1.5 * rho + 2.0)
        V = U.copy()
        for _ in range(n):
            V = nonlinear.split_step(g, V, dt, version, a, b)
        return V

    e1 = np.abs(run(2)[0] - ref[0]).max()
    e2 = np.abs(run(4)[0] - ref[0]).max()
    assert 3.0 < e1 / e2 < 5.0, (e1, e2)


def test_split_ver1_with_rexi_is_strang_ver1():
    L = 8
    p = Params()
    g = _grid(L)
    U = random_state(L, 5, amps=(50.0, 2e-5, 2e-6))
    rho = spectral_radius_bound(L, 1800.0, p)
    a, b, _, _ = rexi.coefficients(rexi.FN_EXP, 64, 6.0, 1.5 * rho + 2.0)
    assert np.array_equal(nonlinear.split_step(g, U, 1800.0, 1, a, b), nonlinear.strang_ver1(g, U, 1800.0, a, b))


def test_lg_split_second_order():
    """lg_rexi_lc_n_erk_ver1 (REXI on L_g, L_c with N) converges at second order
    to the RK4 reference of the full equations: a wrong sign or factor in the
    Coriolis part moved to the explicit side would break it."""
    L = 8
    p = Params()
    g = _grid(L)
    U = random_state(L, 4, amps=(50.0, 2e-5, 2e-6))
    T = 2 * 3600.0
    ref = nonlinear.rk4(g, U, T / 160, 160)

    def run(n):
        dt = T / n
        rho = spectral_radius_bound(L, dt, p)
        a, b, _, _ = rexi.coefficients(rexi.FN_EXP, 128, 8.0, 1.5 * rho + 2.0)
        V = U.copy()
        for _ in range(n):
            V = nonlinear.split_step(g, V, dt, 1, a, b, lg=True)
        return V

    e1 = np.abs(run(2)[0] - ref[0]).max()
    e2 = np.abs(run(4)[0] - ref[0]).max()
    assert 3.0 < e1 / e2 < 5.0, (e1, e2)


def test_grid_coriolis_matches_spectral_operator():
    """The Coriolis part L_c U equals what the spectral operator's Omega terms
    give (the difference of apply with and without Omega), checked against a
    grid-space evaluation of -div(f V) and curl(f V) + nothing for h, f = 2 Omega mu."""
    from dataclasses import replace

    from oracle.operator import apply
    from oracle.sht import inv_laplacian
    L = 13
    p = Params()
    g = Grid(L, 2 * (L + 1), 4 * (L + 1), p)
    U = random_state(L, 12)
    lc = apply(U, L, p) - apply(U, L, replace(p, Omega=0.0))
    Ug, Vg = g.uv_from_psichi(inv_laplacian(U[1], L, p.a), inv_laplacian(U[2], L, p.a))
    f = 2.0 * p.Omega * g.mu[:, None]
    div_f, curl_f = g.div_curl(f * Ug, f * Vg)
    scale = np.abs(lc[1:]).max()
    assert np.abs(lc[0]).max() == 0.0
    assert np.abs(lc[1] - (-div_f)).max() <= 1e-12 * scale
    assert np.abs(lc[2] - curl_f).max() <= 1e-12 * scale


def test_rk4_on_a_linear_system_is_the_taylor_polynomial(monkeypatch):
    """For u' = A u one classical RK4 step equals sum_{k <= 4} (h A)^k u / k!
    (the four order conditions of the method's weights on linear problems);
    the oracle's RK4 is run with its right-hand side replaced by the linear
    operator alone, and compared with that polynomial built from repeated
    operator applications."""
    L = 8
    g = _grid(L)
    U = random_state(L, 21)
    monkeypatch.setattr(nonlinear, "full_tendency", lambda grid, V: apply(V, grid.L, grid.p))
    h = 900.0
    got = nonlinear.rk4(g, U, h, 1)
    term = U.copy()
    ref = U.copy()
    for k in range(1, 5):
        term = apply(term, L, g.p) * (h / k)
        ref = ref + term
    for f in range(3):
        assert np.abs(got[f] - ref[f]).max() <= 1e-13 * np.abs(ref[f]).max(), f
    # the fifth Taylor term, which the step must not contain, is far above the
    # tolerance in every field (a method of higher order would fail the check)
    fifth = apply(term, L, g.p) * (h / 5)
    for f in range(3):
        assert np.abs(fifth[f]).max() > 1e-8 * np.abs(ref[f]).max(), f
