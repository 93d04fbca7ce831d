"""The host-side contour chooser (Section 4.2 coefficients, Section 4.2.2
cancellation) against the oracle: its error estimate is the oracle's brute-force
REXI sum on the same grid, and the stored equal-error contours of the T255
FP32-against-FP64 comparison are what the chooser returns, minimal in N."""
import numpy as np
import pytest

from oracle import rexi as orexi
from oracle.operator import Params, spectral_radius_bound
from paper_1805_06557_amd import configs, contour


def test_radius_matches_oracle_bound():
    for L, dt in [(31, 3600.0), (255, 3600.0), (511, 7200.0)]:
        assert abs(contour.spectral_radius(L, dt) - spectral_radius_bound(L, dt, Params())) < 1e-12


def test_scalar_error_and_kappa_match_oracle_brute_force():
    N, p0, y = 128, 10.0, 30.0
    rho = spectral_radius_bound(31, 3600.0, Params())
    a, b, _, _ = orexi.coefficients(orexi.FN_EXP, N, p0, y)
    w = np.linspace(-rho, rho, 1601)
    ref = np.abs(orexi.rexi_sum(a, b, 1j * w) - np.exp(1j * w)).max()
    la, lb, _, _ = contour.api.rexi_coefficients(contour.api.FN_EXP, N, p0, y)
    got = contour.scalar_error(la, lb, rho)
    kref = orexi.kappa(a, b, 1j * np.linspace(-rho, rho, 401)).max()
    # the two evaluations differ only by rounding (order of the sum, last bits of the coefficients)
    assert abs(got - ref) <= 1e-3 * ref + 8 * 2.0 ** -53 * kref
    assert abs(contour.kappa(la, lb, rho) - kref) <= 1e-12 * kref
    # far from the rounding floor they agree closely
    a, b, _, _ = orexi.coefficients(orexi.FN_EXP, 64, p0, y)
    la, lb, _, _ = contour.api.rexi_coefficients(contour.api.FN_EXP, 64, p0, y)
    ref = np.abs(orexi.rexi_sum(a, b, 1j * w) - np.exp(1j * w)).max()
    assert abs(contour.scalar_error(la, lb, rho) - ref) <= 1e-9 * ref


@pytest.mark.parametrize("w", [configs.T255_FP32_AT_E, configs.T255_FP64_AT_E], ids=lambda w: w.name)
def test_equal_error_contours(w):
    E = configs.EQUAL_ERROR_E
    c = contour.choose(w.L, w.dt, E, w.prec)
    assert (c.p0, c.N) == (w.p0, w.N)
    assert abs(c.y - w.y) < 1e-9
    rho = contour.spectral_radius(w.L, w.dt)
    # minimal: two poles fewer misses the target at the same shift
    a, b, _, _ = orexi.coefficients(orexi.FN_EXP, w.N - 2, w.p0, w.y)
    assert contour.predicted_error(a, b, rho, w.prec) > E
    # the oracle's own coefficients meet the target at the chosen N
    a, b, _, _ = orexi.coefficients(orexi.FN_EXP, w.N, w.p0, w.y)
    assert contour.predicted_error(a, b, rho, w.prec) <= E


def test_fp32_floor_needs_more_poles():
    """At E = 1e-4 the FP32 rounding floor u_32 kappa forces a small shift and
    about four times the poles of FP64 (T255, dt = 3600 s)."""
    assert configs.T255_FP32_AT_E.N > 3 * configs.T255_FP64_AT_E.N
    assert contour.choose(255, 3600.0, 1e-6, 1) is None
