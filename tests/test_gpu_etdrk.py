"""GPU parity of the ETD2RK step l_rexi_n_etdrk (Section 4.3, Eq. etdrk)
against the oracle's etdrk2 (its psi sums pinned to the augmented-matrix
exponential, its order pinned by convergence).  FP64 bar: every entry within
max(1e-12, 8 u kappa) of the oracle, relative to its field's largest entry,
kappa the largest condition number of the psi_0, psi_1, psi_2 sums on the
contour."""
import numpy as np
import pytest

from oracle import nonlinear as onl
from oracle import rexi as orexi
from oracle.operator import Params, spectral_radius_bound
from oracle.sht import Grid
from paper_1805_06557_amd.inputs import jet_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = np.finfo(np.float64).eps / 2


@pytest.mark.parametrize("L,nlat,nlon,dt,N,p0", [(31, 48, 96, 3600.0, 128, 10.0), (63, 96, 192, 1800.0, 160, 6.0)])
def test_etdrk2_step(L, nlat, nlon, dt, N, p0):
    from paper_1805_06557_amd import api
    p = Params()
    g = Grid(L, nlat, nlon, p)
    rho = spectral_radius_bound(L, dt, p)
    y = 30.0 if L == 31 else np.sqrt(2) * 1.05 * rho
    a, b0, _, _ = orexi.coefficients(orexi.FN_EXP, N, p0, y)
    _, b1, _, _ = orexi.coefficients(orexi.FN_PSI1, N, p0, y)
    _, b2, _, _ = orexi.coefficients(orexi.FN_PSI2, N, p0, y)
    U0 = jet_state(L, 4)
    ref = onl.etdrk2(g, U0, dt, a, b0, b1, b2)
    ctx = api.SWE(L, nlat, nlon)
    d0 = torch.from_numpy(U0).cuda()
    d1 = torch.empty_like(d0)
    ctx.etdrk2_step(a, b0, b1, b2, dt, d0, d1)
    got = d1.cpu().numpy()
    w = 1j * np.linspace(-rho, rho, 401)
    kap = max(float(orexi.kappa(a, b, w).max()) for b in (b0, b1, b2))
    tol = max(1e-12, 8 * U64 * kap)
    for f in range(3):
        scale = np.abs(ref[f]).max()
        assert np.abs(got[f] - ref[f]).max() <= tol * scale, (f, np.abs(got[f] - ref[f]).max() / scale, tol)
    # in place, and repeated calls reuse the three cached coefficient sets bit for bit
    ctx.etdrk2_step(a, b0, b1, b2, dt, d0, d0)
    assert np.array_equal(d0.cpu().numpy(), got)
    ctx.close()
