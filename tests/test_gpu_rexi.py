"""GPU parity of rexi_linear_step against the oracle (Eq. rexi with L = L_g + L_c).

FP64 bar: every entry within max(1e-12, 4 u kappa) of the oracle, relative to
the largest entry of its field, where kappa = max_{|w|<=rho} sum |beta_n| /
|i w + alpha_n| is the condition number of the rational sum (the floor any
implementation of it has, Section 4.2.2).
FP32-solve bars (rounding model): the FP32 sweep makes a few roundings of
u_32 per row (the diagonal and right-hand side formed in FP32 from z and 1/z
rounded to FP32, the pivot with the unrefined hardware reciprocal, the two
elimination updates), each relative to the row's terms, and the diagonally
dominant chain spreads a row's perturbation to its neighbours with
geometrically decaying weight; the solutions are summed in FP64.  So an output
entry j carries about u_32 times M_j = sum_n |beta_n| |x_n,j| (the sum of the
magnitudes of its terms, oracle.linear.rexi_term_magnitudes): the bar is
16 u_32 M_j per entry (the roundings per row and their spread), and 3 u_32 kappa
of the field's largest entry per field (kappa as above bounds M_j / |U0|).
"""
import numpy as np
import pytest

from oracle import linear as olinear
from oracle import rexi as orexi
from oracle.operator import Params, mode_index, spectral_radius_bound
from paper_1805_06557_amd.inputs import random_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = np.finfo(np.float64).eps / 2
U32 = np.finfo(np.float32).eps / 2


def _api():
    from paper_1805_06557_amd import api
    return api


def _kappa_max(alpha, beta, rho):
    w = np.linspace(-rho, rho, 401)
    return float(orexi.kappa(alpha, beta, 1j * w).max())


def _run_gpu(L, alpha, beta, dt, U0, prec=0, seg_rows=0, solver=0, waves=0, poles_per_lane=0):
    api = _api()
    ctx = api.SWE(L, prec=prec)
    if seg_rows or solver or waves or poles_per_lane:
        ctx.set_tuning(solver=solver, seg_rows=seg_rows, waves=waves, poles_per_lane=poles_per_lane)
    d0 = torch.from_numpy(U0).cuda()
    d1 = torch.empty_like(d0)
    ctx.rexi_linear_step(alpha, beta, dt, d0, d1)
    torch.cuda.synchronize()
    out = d1.cpu().numpy()
    ctx.close()
    return out


def _assert_close(got, ref, tol, orders=None, L=None):
    if orders is not None:
        idx = np.concatenate([np.arange(mode_index(L, m, m), mode_index(L, m, m) + L - m + 1) for m in orders])
        got, ref = got[:, idx], ref[:, idx]
    for f in range(3):
        scale = np.abs(ref[f]).max()
        err = np.abs(got[f] - ref[f]).max()
        assert err <= tol * scale, (f, err / scale, tol)


CASES = [
    # name, L, N, dt, p0, y, seg_rows
    ("T31-paper-contour", 31, 128, 3600.0, 10.0, 30.0, 16),
    ("ragged-rows-and-poles", 20, 70, 3600.0, 8.0, 12.0, 16),
    ("checkpointed-segments", 45, 96, 3600.0, 8.0, 16.0, 16),
    ("smallest", 1, 4, 600.0, 1.0, 2.0, 16),
    ("single-pole-block-long-chain", 70, 64, 1800.0, 6.0, 9.0, 16),
]


@pytest.mark.parametrize("name,L,N,dt,p0,y,S", CASES, ids=[c[0] for c in CASES])
def test_fp64_parity(name, L, N, dt, p0, y, S):
    p = Params()
    rho = spectral_radius_bound(L, dt, p)
    assert y > rho
    alpha, beta, _, _ = orexi.coefficients(orexi.FN_EXP, N, p0, y)
    U0 = random_state(L, 100 + L)
    ref = olinear.rexi_linear_step(U0, alpha, beta, dt, L, p)
    got = _run_gpu(L, alpha, beta, dt, U0, seg_rows=S)
    tol = max(1e-12, 4 * U64 * _kappa_max(alpha, beta, rho))
    _assert_close(got, ref, tol)


def _assert_fp32(got, ref, M, kap, orders=None, L=None):
    """The two FP32-solve bars of the module docstring (per entry and per field)."""
    if orders is not None:
        idx = np.concatenate([np.arange(mode_index(L, m, m), mode_index(L, m, m) + L - m + 1) for m in orders])
        got, ref, M = got[:, idx], ref[:, idx], M[:, idx]
    per_entry = [float((np.abs(got[f] - ref[f]) / (16 * U32 * M[f] + 1e-300)).max()) for f in range(3)]
    per_field = [float(np.abs(got[f] - ref[f]).max() / (3 * U32 * kap * np.abs(ref[f]).max())) for f in range(3)]
    print("FP32 solve: error / bar per entry", per_entry, "per field", per_field)
    assert max(per_entry) <= 1.0, per_entry
    assert max(per_field) <= 1.0, per_field


def test_fp32_solve_parity_t31():
    L, N, dt = 31, 128, 3600.0
    p = Params()
    alpha, beta, _, _ = orexi.coefficients(orexi.FN_EXP, N, 10.0, 30.0)
    U0 = random_state(L, 7)
    ref = olinear.rexi_linear_step(U0, alpha, beta, dt, L, p)
    M = olinear.rexi_term_magnitudes(U0, alpha, beta, dt, L, p)
    got = _run_gpu(L, alpha, beta, dt, U0, prec=1)
    _assert_fp32(got, ref, M, _kappa_max(alpha, beta, spectral_radius_bound(L, dt, p)))


@pytest.mark.parametrize("prec", [0, 1])
def test_schedule_and_shape_do_not_change_bits(prec):
    """Every schedule (pivots recomputed, streamed from the cached factorization,
    or both), segment length and workgroup size performs the same operations in
    the same order on each (pole, row), and the pole sum is grouped the same
    way, so all give bit-identical results; repeated calls are bit-identical.
    N = 180 leaves 52 poles for the second wave of two poles per lane, which then
    runs with one pole per lane."""
    api = _api()
    L, N, dt = 57, 180, 3600.0
    alpha, beta, _, _ = orexi.coefficients(orexi.FN_EXP, N, 8.0, 16.0)
    U0 = random_state(L, 8)
    refs = []
    for P in (1, 2):
        ref = _run_gpu(L, alpha, beta, dt, U0, prec=prec, solver=api.SOLVER_FUSED, seg_rows=16, waves=1,
                       poles_per_lane=P)
        for solver in (api.SOLVER_FUSED, api.SOLVER_STREAM, api.SOLVER_HYBRID):
            for S in ((16, 32) if P == 1 else (8, 16)):
                for W in (1, 2, 4):
                    got = _run_gpu(L, alpha, beta, dt, U0, prec=prec, solver=solver, seg_rows=S, waves=W,
                                   poles_per_lane=P)
                    assert np.array_equal(got, ref), (P, solver, S, W)
        refs.append(ref)
    # two poles per lane regroup the pole sum: each lane adds its poles' weighted
    # outputs in the solve's precision before the FP64 sum over the wave
    scale = np.abs(refs[0]).max(axis=1, keepdims=True)
    if prec == 0:
        tol = 1e-13
    else:
        tol = 3 * U32 * _kappa_max(alpha, beta, spectral_radius_bound(L, dt, Params()))
    assert np.all(np.abs(refs[1] - refs[0]) <= tol * scale)


@pytest.mark.parametrize("solver", [2, 3])
def test_factor_cache_follows_coefficients(solver):
    """The cached factorization is reused while (alpha, beta, N, dt) stay the
    same and rebuilt when any of them or the precision changes."""
    api = _api()
    L = 40
    p = Params()
    a1, b1, _, _ = orexi.coefficients(orexi.FN_EXP, 96, 8.0, 16.0)
    a2, b2, _, _ = orexi.coefficients(orexi.FN_EXP, 128, 9.0, 20.0)
    U0 = random_state(L, 11)
    calls = [(a1, b1, 3600.0), (a1, b1, 3600.0), (a2, b2, 3600.0), (a2, b2, 1800.0), (a1, b1, 3600.0)]
    ctx = api.SWE(L)
    ctx.set_tuning(solver=solver)
    d0 = torch.from_numpy(U0).cuda()
    d1 = torch.empty_like(d0)
    for a, b, dt in calls:
        ctx.rexi_linear_step(a, b, dt, d0, d1)
        got = d1.cpu().numpy()
        fresh = _run_gpu(L, a, b, dt, U0, solver=api.SOLVER_FUSED)
        assert np.array_equal(got, fresh)
    ref = olinear.rexi_linear_step(U0, a1, b1, 3600.0, L, p)
    tol = max(1e-12, 4 * U64 * _kappa_max(a1, b1, spectral_radius_bound(L, 3600.0, p)))
    _assert_close(got, ref, tol)
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_t255_sampled_orders(prec):
    """Full T255 / N = 800 in the launch shape the benchmark uses (each
    schedule), checked on a sample of zonal orders the oracle solves one by one."""
    from paper_1805_06557_amd import configs
    api = _api()
    w = configs.T255_FP32 if prec else configs.T255_FP64
    p = Params()
    alpha, beta, _, _ = orexi.coefficients(orexi.FN_EXP, w.N, w.p0, w.y)
    U0 = random_state(w.L, 2)
    orders = [0, 1, 2, 97, 200, 254, 255]
    ref = olinear.rexi_linear_step(U0, alpha, beta, w.dt, w.L, p, orders=orders)
    kap = _kappa_max(alpha, beta, spectral_radius_bound(w.L, w.dt, p))
    M = olinear.rexi_term_magnitudes(U0, alpha, beta, w.dt, w.L, p, orders=orders) if prec else None
    outs = []
    for solver in (0, api.SOLVER_FUSED, api.SOLVER_STREAM, api.SOLVER_HYBRID):
        got = _run_gpu(w.L, alpha, beta, w.dt, U0, prec=prec, solver=solver)
        if prec:
            _assert_fp32(got, ref, M, kap, orders=orders, L=w.L)
        else:
            _assert_close(got, ref, max(1e-12, 4 * U64 * kap), orders=orders, L=w.L)
        outs.append(got)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_contour_not_enclosing_spectrum_is_rejected():
    api = _api()
    L, dt = 31, 3600.0
    alpha, beta, _, _ = orexi.coefficients(orexi.FN_EXP, 64, 2.0, 3.0)   # rho = 6.1 > y
    ctx = api.SWE(L)
    d0 = torch.zeros((3, api.n_modes(L)), dtype=torch.complex128, device="cuda")
    d1 = torch.empty_like(d0)
    with pytest.raises(api.RexiError) as ei:
        ctx.rexi_linear_step(alpha, beta, dt, d0, d1)
    assert ei.value.code == api.REXI_ENUMERIC
    with pytest.raises(api.RexiError) as ei:
        ctx.rexi_linear_step(alpha, beta, dt, d0, d0)
    assert ei.value.code == api.REXI_EINVAL
    ctx.close()
