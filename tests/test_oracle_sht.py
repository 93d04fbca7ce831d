"""Pins of the oracle's spherical-harmonic transforms (Section 3.2) against
library routines, closed forms and identities."""
import mpmath
import numpy as np
import pytest
import scipy.special

from oracle.operator import Params, mode_index, n_modes
from oracle.sht import Grid, gauss_legendre, inv_laplacian, legendre_m
from paper_1805_06557_amd.inputs import random_field


@pytest.mark.parametrize("n", [8, 17, 48, 96, 192])
def test_gauss_nodes_match_numpy(n):
    x, s, w = gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.all(np.diff(x) < 0)                      # north to south
    np.testing.assert_allclose(x, xr[::-1], atol=2e-15)
    # numpy's weights lose relative accuracy at the polar nodes as n grows
    np.testing.assert_allclose(w, wr[::-1], rtol=0, atol=5e-14)
    np.testing.assert_allclose(s, np.sqrt(1 - x * x), rtol=1e-12)
    assert abs(w.sum() - 2.0) < 1e-14


@pytest.mark.parametrize("n", [48, 192])
def test_gauss_weights_against_mpmath(n):
    x, s, w = gauss_legendre(n)
    # mirror symmetry, then the southern nodes against a 60-digit root polish
    np.testing.assert_array_equal(w, w[::-1])
    np.testing.assert_array_equal(x, -x[::-1])
    with mpmath.workdps(60):
        for j in [n // 2, n // 2 + 1, n - 8, n - 2, n - 1]:
            th = mpmath.findroot(lambda t: mpmath.legendre(n, mpmath.cos(t)),
                                 mpmath.acos(mpmath.mpf(x[j])), tol=1e-50, verify=False)
            X = mpmath.cos(th)
            W = 2 * mpmath.sin(th) ** 2 / (n * mpmath.legendre(n - 1, X)) ** 2
            assert abs(x[j] - float(X)) < 2e-16
            assert abs(w[j] / float(W) - 1) < 1e-14


def test_legendre_matches_scipy_lpmv():
    x, s, _ = gauss_legendre(24)
    for m in range(0, 12):
        P = legendre_m(m, 20, x, s)
        for l in range(m, 21):
            ref = scipy.special.lpmv(m, l, x) * (-1.0) ** m        # remove Condon-Shortley
            ref *= np.sqrt((2 * l + 1) / 2.0 * scipy.special.factorial(l - m) / scipy.special.factorial(l + m))
            np.testing.assert_allclose(P[l - m], ref, rtol=1e-11, atol=1e-13)


def test_legendre_closed_forms():
    x, s, _ = gauss_legendre(10)
    P0 = legendre_m(0, 1, x, s)
    P1 = legendre_m(1, 1, x, s)
    np.testing.assert_allclose(P0[0], np.full_like(x, np.sqrt(0.5)), rtol=1e-15)
    np.testing.assert_allclose(P0[1], np.sqrt(1.5) * x, rtol=1e-14)
    np.testing.assert_allclose(P1[0], np.sqrt(3.0) / 2.0 * s, rtol=1e-14)


def _pbar_exact(l, m, x):
    """Pbar_lm(x) from the explicit polynomial form of d^m/dx^m P_l in exact
    rational arithmetic, then (1 - x^2)^{m/2} and the normalisation in mpmath."""
    from fractions import Fraction
    from math import factorial
    X = Fraction(x)
    acc = Fraction(0)
    for k in range(0, (l - m) // 2 + 1):
        c = Fraction((-1) ** k * factorial(2 * l - 2 * k), 2 ** l * factorial(k) * factorial(l - k) * factorial(l - 2 * k))
        p = l - 2 * k
        acc += c * Fraction(factorial(p), factorial(p - m)) * X ** (p - m)
    with mpmath.workdps(60):
        v = mpmath.mpf(acc.numerator) / acc.denominator
        v *= mpmath.power(1 - mpmath.mpf(X.numerator) ** 2 / mpmath.mpf(X.denominator) ** 2, mpmath.mpf(m) / 2)
        v *= mpmath.sqrt((2 * l + 1) / mpmath.mpf(2) * mpmath.factorial(l - m) / mpmath.factorial(l + m))
        return v


def test_legendre_underflow_region_against_exact():
    """Near the pole at T511 the seed sin(theta)^m underflows double range; the
    exponent-tracked recurrence must still produce the right values once they
    grow back, and (near-)zeros only where the true value is below ~1e-300."""
    x, s, _ = gauss_legendre(768)
    # (node, order) pairs whose seed Pbar_mm lies below 1e-280 (outside double
    # range) while Pbar_{511,m} is back above 1e-240, plus one ordinary case
    for j, m in [(28, 350), (40, 400), (56, 450), (40, 200)]:
        P = legendre_m(m, 511, x[j:j + 1], s[j:j + 1])[:, 0]
        for l in sorted({m, m + 1, (m + 511) // 2, 500, 511}):
            if l < m or l > 511:
                continue
            ref = _pbar_exact(l, m, x[j])
            if abs(ref) < mpmath.mpf("1e-295"):
                assert abs(P[l - m]) < 1e-280
            else:
                assert abs(P[l - m] - float(ref)) <= 1e-11 * abs(float(ref)), (j, m, l, P[l - m], ref)


@pytest.mark.parametrize("L,nlat", [(8, 16), (31, 48), (63, 96)])
def test_orthonormality(L, nlat):
    g = Grid(L, nlat, 2 * nlat)
    for m in range(L + 1):
        P = g.P(m)
        G = (P * g.w) @ P.T
        np.testing.assert_allclose(G, np.eye(L - m + 1), atol=1e-13)


@pytest.mark.parametrize("L,nlat,nlon", [(8, 16, 32), (31, 48, 96)])
def test_roundtrip_and_realness(L, nlat, nlon):
    g = Grid(L, nlat, nlon)
    rng = np.random.default_rng(0)
    f = random_field(L, rng, 1.0)
    back = g.analysis(g.synthesis(f))
    np.testing.assert_allclose(back, f, atol=1e-14 * np.abs(f).max() * 10)
    # analysis of any real grid field gives real m = 0 coefficients
    field = rng.standard_normal((nlat, nlon))
    spec = g.analysis(field)
    assert np.max(np.abs(spec[: L + 1].imag)) < 1e-15


def test_div_curl_of_velocity_recovers_vorticity_divergence():
    L, nlat, nlon = 21, 33, 64
    p = Params()
    g = Grid(L, nlat, nlon, p)
    rng = np.random.default_rng(3)
    zeta = random_field(L, rng, 1e-5)
    delta = random_field(L, rng, 1e-5)
    zeta[0] = delta[0] = 0.0
    psi = inv_laplacian(zeta, L, p.a)
    chi = inv_laplacian(delta, L, p.a)
    U, V = g.uv_from_psichi(psi, chi)
    div, curl = g.div_curl(U, V)
    np.testing.assert_allclose(div, delta, atol=1e-13 * 1e-5)
    np.testing.assert_allclose(curl, zeta, atol=1e-13 * 1e-5)


def test_solid_body_velocity_closed_form():
    """zeta = 2 u0 mu / a is solid-body rotation u = u0 cos(phi), v = 0."""
    L, nlat, nlon = 10, 16, 32
    p = Params()
    g = Grid(L, nlat, nlon, p)
    u0 = 20.0
    zeta = np.zeros(n_modes(L), dtype=complex)
    zeta[mode_index(L, 1, 0)] = 2 * u0 / p.a * np.sqrt(2.0 / 3.0)   # mu = sqrt(2/3) Pbar_10
    psi = inv_laplacian(zeta, L, p.a)
    U, V = g.uv_from_psichi(psi, np.zeros_like(psi))
    cos2 = (g.sint ** 2)[:, None]
    np.testing.assert_allclose(U, u0 * cos2 * np.ones((1, nlon)), atol=1e-12 * u0)
    np.testing.assert_allclose(V, 0.0, atol=1e-12 * u0)


def _three_halves_grid(L):
    """Smallest Gauss grid on which products of two fields of truncation L are
    analysed without aliasing (Section 3.2): 2 nlat - 1 >= 3L in latitude,
    nlon > 3L (even) in longitude."""
    nlat = (3 * L + 2) // 2
    nlon = 3 * L + 1
    return nlat, nlon + nlon % 2


@pytest.mark.parametrize("L", [10, 21, 31])
def test_products_alias_free_on_three_halves_grid(L):
    """The pseudo-spectral N(U) (products h V, zeta V and V.V/2 formed on the
    grid, Section 3.2) on the 3/2-rule grid equals N(U) on a grid twice as fine
    in both directions: the Gauss quadrature of the vector terms, weighted by
    1/(1 - mu^2), is exact there as well.  The bar is rounding amplified by
    l(l+1) in the kinetic-energy term.  One latitude or two longitudes fewer
    must alias (the check can fail)."""
    from oracle import nonlinear as onl
    from paper_1805_06557_amd.inputs import random_state
    p = Params()
    nlat, nlon = _three_halves_grid(L)
    U = random_state(L, 5)
    fine = onl.tendency(Grid(L, 2 * nlat, 2 * nlon, p), U)

    def rel(t):
        return [float(np.abs(t[f] - fine[f]).max() / np.abs(fine[f]).max()) for f in range(3)]
    bar = max(1e-14, 1e-15 * L * (L + 1))
    assert max(rel(onl.tendency(Grid(L, nlat, nlon, p), U))) <= bar
    assert min(rel(onl.tendency(Grid(L, nlat - 1, nlon, p), U))) > 1e3 * bar
    assert min(rel(onl.tendency(Grid(L, nlat, nlon - 2, p), U))) > 1e3 * bar
    rng = np.random.default_rng(L)
    a, b = random_field(L, rng, 1.0), random_field(L, rng, 1.0)
    g1, g2 = Grid(L, nlat, nlon, p), Grid(L, 2 * nlat, 2 * nlon, p)
    s1 = g1.analysis(g1.synthesis(a) * g1.synthesis(b))
    s2 = g2.analysis(g2.synthesis(a) * g2.synthesis(b))
    assert np.abs(s1 - s2).max() <= 1e-14 * np.abs(s2).max()


def test_workload_grids_meet_three_halves_rule():
    from paper_1805_06557_amd import configs
    grids = [w for w in configs.ALL.values() if getattr(w, "nlat", 0)]
    assert grids
    for w in grids:
        if w.nlat:
            nlat, nlon = _three_halves_grid(w.L)
            assert w.nlat >= nlat and w.nlon >= nlon, w.name
