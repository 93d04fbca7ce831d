"""Device-side numeric status: a kernel that writes a non-finite value into an
output sets the context's flag word, and swe_sync reports REXI_ENUMERIC once
(naming the stage) and clears it.  The inputs are seeded with NaN or infinity
on the host: every kernel runs normally, only the values are invalid.  Also
the host-side refusals (a contour that leaves the chain systems without
diagonal dominance, Section 4.2.1) and the T511 jet, whose explicit stage
turns the state non-finite after some steps: the library reports it exactly
when the state holds a non-finite value."""
import numpy as np
import pytest

from oracle import rexi as orexi
from oracle.operator import Params, spectral_radius_bound
from paper_1805_06557_amd.inputs import jet_state, random_field, random_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _api():
    from paper_1805_06557_amd import api
    return api


def _expect_enumeric(api, ctx, word):
    with pytest.raises(api.RexiError) as ei:
        ctx.sync()
    assert ei.value.code == api.REXI_ENUMERIC
    assert word in str(ei.value), str(ei.value)
    ctx.sync()          # reported once, then clear


def test_rexi_stage_nan_input_is_reported():
    api = _api()
    ctx = api.SWE(31)
    a, b, _, _ = api.rexi_coefficients(api.FN_EXP, 128, 10.0, 30.0)
    U = random_state(31, 5)
    ctx.sync()
    d1 = torch.empty((3, api.n_modes(31)), dtype=torch.complex128, device="cuda")
    ctx.rexi_linear_step(a, b, 3600.0, torch.from_numpy(U).cuda(), d1)
    ctx.sync()                                     # finite input: nothing reported
    U[2, 40] = np.nan
    ctx.rexi_linear_step(a, b, 3600.0, torch.from_numpy(U).cuda(), d1)
    _expect_enumeric(api, ctx, "REXI")
    # the gravity-wave stage and the Crank-Nicolson step report through the same word
    ctx.rexi_lg_step(a, b, 3600.0, torch.from_numpy(U).cuda(), d1)
    _expect_enumeric(api, ctx, "REXI")
    ctx.cn_step(3600.0, torch.from_numpy(U).cuda(), d1)
    _expect_enumeric(api, ctx, "REXI")
    ctx.close()


@pytest.mark.parametrize("prec", [0, 2], ids=["fp64", "bf16-split"])
def test_nonlinear_and_transform_outputs_are_reported(prec):
    api = _api()
    L, nlat, nlon = 31, 48, 96
    ctx = api.SWE(L, nlat, nlon, prec=prec)
    U = jet_state(L, 3)
    d0 = torch.from_numpy(U).cuda()
    d1 = torch.empty_like(d0)
    ctx.nonlinear_step(600.0, d0, d1)
    ctx.sync()
    U[0, 5] = np.inf
    ctx.nonlinear_step(600.0, torch.from_numpy(U).cuda(), d1)
    _expect_enumeric(api, ctx, "non-linear")
    rng = np.random.default_rng(1)
    spec = random_field(L, rng, 1.0)[None, :].copy()
    spec[0, 3] = np.nan
    grid = torch.empty((1, nlat, nlon), dtype=torch.float64, device="cuda")
    ctx.sh_synthesis(torch.from_numpy(spec).cuda(), grid, 1)
    _expect_enumeric(api, ctx, "transform")
    g = rng.standard_normal((1, nlat, nlon))
    g[0, 7, 9] = np.nan
    out = torch.empty((1, api.n_modes(L)), dtype=torch.complex128, device="cuda")
    ctx.sh_analysis(torch.from_numpy(g).cuda(), out, 1)
    _expect_enumeric(api, ctx, "transform")
    ctx.close()


def test_contour_without_dominance_is_refused_before_launch():
    api = _api()
    L, dt = 8, 21600.0
    rho = spectral_radius_bound(L, dt, Params())
    a, b, _, _ = orexi.coefficients(orexi.FN_EXP, 64, 2.0, 1.02 * rho)
    ctx = api.SWE(L)
    U = torch.from_numpy(random_state(L, 2)).cuda()
    V = torch.zeros_like(U)
    with pytest.raises(api.RexiError) as ei:
        ctx.rexi_linear_step(a, b, dt, U, V)
    assert ei.value.code == api.REXI_ENUMERIC
    assert "diagonally dominant" in str(ei.value)
    ctx.sync()
    assert torch.count_nonzero(V).item() == 0      # nothing was enqueued
    ctx.close()


def test_t511_jet_blow_up_is_reported_when_it_happens():
    """The T511 jet at dt = 7200 s: after every Strang step the library reports
    a non-finite state if and only if the state holds one."""
    from paper_1805_06557_amd import configs
    api = _api()
    w = configs.T511_FP64
    alpha, beta, _, _ = api.rexi_coefficients(api.FN_EXP, w.N, w.p0, w.y)
    ctx = api.SWE(w.L, w.nlat, w.nlon)
    U = torch.from_numpy(jet_state(w.L, w.seed)).cuda()
    reported = None
    for s in range(20):
        ctx.strang_step(alpha, beta, w.dt, U, U)
        finite = bool(torch.isfinite(torch.view_as_real(U)).all())
        try:
            ctx.sync()
            flagged = False
        except api.RexiError as e:
            assert e.code == api.REXI_ENUMERIC
            flagged = True
        if reported is None:
            assert flagged == (not finite), (s, flagged, finite)
            if flagged:
                reported = s
                break
    print(f"T511 jet: non-finite state reported after step {reported}")
    ctx.close()
