"""GPU parity of the comparison schemes built on the same kernels: the
Crank-Nicolson linear step (Section 4.1, implicit ``irk``; one real shift on the
chain solve) and the four Strang splittings of Section 4.4 (REXI or CN for
the linear part, version 0 or 1), against the oracle.  FP64 bar: 1e-12 of
each field's largest entry (CN: the one-shift solve is well conditioned,
|w| / |z - i w| <= 2), max(1e-12, 4 u kappa) with the REXI sums."""
import numpy as np
import pytest

from oracle import linear as olinear
from oracle import nonlinear as onl
from oracle import rexi as orexi
from oracle.operator import Params, spectral_radius_bound
from oracle.sht import Grid
from paper_1805_06557_amd.inputs import jet_state, random_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = np.finfo(np.float64).eps / 2


def _api():
    from paper_1805_06557_amd import api
    return api


def _close(got, ref, tol):
    for f in range(3):
        scale = np.abs(ref[f]).max()
        assert np.abs(got[f] - ref[f]).max() <= tol * scale, (f, np.abs(got[f] - ref[f]).max() / scale, tol)


@pytest.mark.parametrize("L,dt,prec", [(31, 3600.0, 0), (255, 3600.0, 0), (63, 7200.0, 1)],
                         ids=["T31", "T255", "T63-fp32"])
def test_cn_step(L, dt, prec):
    api = _api()
    U0 = random_state(L, 21)
    ref = olinear.cn_step(U0, dt, L, Params())
    ctx = api.SWE(L, prec=prec)
    d0 = torch.from_numpy(U0).cuda()
    d1 = torch.empty_like(d0)
    ctx.cn_step(dt, d0, d1)
    _close(d1.cpu().numpy(), ref, 1e-12 if prec == 0 else 64 * 2.0 ** -24)
    ctx.close()


@pytest.mark.parametrize("scheme", [0, 1, 2, 3], ids=["rexi-v1", "rexi-v0", "cn-v1", "cn-v0"])
def test_split_step(scheme):
    api = _api()
    L, nlat, nlon, dt = 31, 48, 96, 3600.0
    p = Params()
    g = Grid(L, nlat, nlon, p)
    U0 = jet_state(L, 6)
    version = 1 if scheme in (0, 2) else 0
    a = b = None
    tol = 1e-12
    if scheme in (0, 1):
        tl = dt if version == 1 else 0.5 * dt
        rho = spectral_radius_bound(L, tl, p)
        a, b, _, _ = orexi.coefficients(orexi.FN_EXP, 128, 8.0, np.sqrt(2) * 1.05 * rho)
        kap = float(orexi.kappa(a, b, 1j * np.linspace(-rho, rho, 401)).max())
        tol = max(1e-12, 4 * U64 * kap)
    ref = onl.split_step(g, U0, dt, version, a, b)
    ctx = api.SWE(L, nlat, nlon)
    d0 = torch.from_numpy(U0).cuda()
    d1 = torch.empty_like(d0)
    ctx.split_step(scheme, a, b, dt, d0, d1)
    got = d1.cpu().numpy()
    _close(got, ref, tol)
    if scheme == 0:
        d2 = torch.empty_like(d0)
        ctx.strang_step(a, b, dt, d0, d2)
        assert np.array_equal(d2.cpu().numpy(), got)
    ctx.close()


@pytest.mark.parametrize("L,dt,N,p0", [(31, 3600.0, 128, 10.0), (255, 3600.0, 800, 12.0)], ids=["T31", "T255"])
def test_rexi_lg_stage(L, dt, N, p0):
    """The gravity-wave REXI stage (per-degree sums, no banded solve) against the
    oracle's banded REXI solve with Omega = 0."""
    from dataclasses import replace
    api = _api()
    p = Params()
    rho = spectral_radius_bound(L, dt, p)
    y = 30.0 if L == 31 else np.sqrt(2) * 1.05 * rho
    a, b, _, _ = orexi.coefficients(orexi.FN_EXP, N, p0, y)
    U0 = random_state(L, 31)
    orders = None if L == 31 else [0, 1, 128, 255]
    ref = olinear.rexi_linear_step(U0, a, b, dt, L, replace(p, Omega=0.0), orders=orders)
    ctx = api.SWE(L)
    d0 = torch.from_numpy(U0).cuda()
    d1 = torch.empty_like(d0)
    ctx.rexi_lg_step(a, b, dt, d0, d1)
    got = d1.cpu().numpy()
    kap = float(orexi.kappa(a, b, 1j * np.linspace(-rho, rho, 401)).max())
    if orders is not None:
        from oracle.operator import mode_index
        idx = np.concatenate([np.arange(mode_index(L, m, m), mode_index(L, m, m) + L - m + 1) for m in orders])
        got, ref = got[:, idx], ref[:, idx]
    _close(got, ref, max(1e-12, 4 * U64 * kap))
    ctx.close()


def test_lg_split_step():
    api = _api()
    L, nlat, nlon, dt = 31, 48, 96, 3600.0
    p = Params()
    g = Grid(L, nlat, nlon, p)
    U0 = jet_state(L, 7)
    rho = spectral_radius_bound(L, dt, p)
    a, b, _, _ = orexi.coefficients(orexi.FN_EXP, 128, 8.0, np.sqrt(2) * 1.05 * rho)
    kap = float(orexi.kappa(a, b, 1j * np.linspace(-rho, rho, 401)).max())
    ref = onl.split_step(g, U0, dt, 1, a, b, lg=True)
    ctx = api.SWE(L, nlat, nlon)
    d0 = torch.from_numpy(U0).cuda()
    d1 = torch.empty_like(d0)
    ctx.split_step(api.SPLIT_LG_REXI_V1, a, b, dt, d0, d1)
    _close(d1.cpu().numpy(), ref, max(1e-12, 4 * U64 * kap))
    ctx.close()
