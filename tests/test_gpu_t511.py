"""The T511 workload (1536 x 768 Gauss grid, dt = 7200 s, N = 2000 poles, FP64):
the REXI stage on sampled zonal orders against the oracle (Eq. rexi; FP64 bar
max(1e-12, 4 u kappa) per field), and the transforms at full size through the
property Gauss quadrature guarantees for a band-limited field: analysis
inverts synthesis (to 1e-12 of the field's largest coefficient)."""
import numpy as np
import pytest

from oracle import linear as olinear
from oracle import rexi as orexi
from oracle.operator import Params, mode_index, spectral_radius_bound
from paper_1805_06557_amd.inputs import random_field, random_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = np.finfo(np.float64).eps / 2


def _api():
    from paper_1805_06557_amd import api
    return api


def test_t511_rexi_sampled_orders():
    from paper_1805_06557_amd import configs
    api = _api()
    w = configs.T511_FP64
    p = Params()
    alpha, beta, _, _ = orexi.coefficients(orexi.FN_EXP, w.N, w.p0, w.y)
    U0 = random_state(w.L, 9)
    orders = [400, 500, 511]      # the oracle solves order m in about 0.08 (L - m + 1) s here
    ref = olinear.rexi_linear_step(U0, alpha, beta, w.dt, w.L, p, orders=orders)
    ctx = api.SWE(w.L)
    d0 = torch.from_numpy(U0).cuda()
    d1 = torch.empty_like(d0)
    ctx.rexi_linear_step(alpha, beta, w.dt, d0, d1)
    got = d1.cpu().numpy()
    ctx.close()
    idx = np.concatenate([np.arange(mode_index(w.L, m, m), mode_index(w.L, m, m) + w.L - m + 1) for m in orders])
    kap = float(orexi.kappa(alpha, beta, 1j * np.linspace(-1, 1, 401) * spectral_radius_bound(w.L, w.dt, p)).max())
    tol = max(1e-12, 4 * U64 * kap)
    for f in range(3):
        scale = np.abs(ref[f, idx]).max()
        err = np.abs(got[f, idx] - ref[f, idx]).max()
        assert err <= tol * scale, (f, err / scale, tol)


def test_t511_transform_round_trip():
    api = _api()
    L, nlat, nlon = 511, 768, 1536
    rng = np.random.default_rng(11)
    nf = 2
    spec = np.stack([random_field(L, rng, 1.0) for _ in range(nf)])
    ctx = api.SWE(L, nlat, nlon)
    ds = torch.from_numpy(spec).cuda()
    dg = torch.empty((nf, nlat, nlon), dtype=torch.float64, device="cuda")
    ctx.sh_synthesis(ds, dg, nf)
    back = torch.empty_like(ds)
    ctx.sh_analysis(dg, back, nf)
    got = back.cpu().numpy()
    for f in range(nf):
        assert np.abs(got[f] - spec[f]).max() <= 1e-12 * np.abs(spec[f]).max()
    ctx.close()


def test_t511_strang_step_runs_finite():
    from paper_1805_06557_amd import configs
    from paper_1805_06557_amd.inputs import jet_state
    api = _api()
    w = configs.T511_FP64
    alpha, beta, _, _ = api.rexi_coefficients(api.FN_EXP, w.N, w.p0, w.y)
    ctx = api.SWE(w.L, w.nlat, w.nlon)
    U = torch.from_numpy(jet_state(w.L, w.seed)).cuda()
    V = torch.empty_like(U)
    ctx.strang_step(alpha, beta, w.dt, U, V)
    out = V.cpu().numpy()
    assert np.all(np.isfinite(out))
    # the mean height h_00 is left alone by the non-linear part (a divergence has
    # no l = 0 component) and multiplied by S(0) by the REXI stage, which equals
    # e^0 = 1 only up to the rational approximation's error at x = 0 plus its
    # rounding floor u kappa (kappa ~ 1e10 for this contour)
    h0 = U.cpu().numpy()[0, 0]
    a, b, _, _ = orexi.coefficients(orexi.FN_EXP, w.N, w.p0, w.y)
    s0 = complex(orexi.rexi_sum(a, b, 0.0)[0])
    kap0 = float(orexi.kappa(a, b, 0.0)[0])
    assert abs(out[0, 0] - s0 * h0) <= 8 * U64 * kap0 * abs(h0)
    assert abs(out[0, 0] - h0) <= (abs(s0 - 1.0) + 8 * U64 * kap0) * abs(h0)
    ctx.close()
