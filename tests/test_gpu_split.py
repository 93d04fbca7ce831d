"""Split-precision (16-bit hi/lo on the matrix cores, FP32 accumulation) Legendre
stage against the FP64 oracle, in both modes: BF16 and FP16.

Rounding model (stated bars).  Every product a b is formed as
a_hi b_hi + a_hi b_lo + a_lo b_hi with |x - x_hi - x_lo| <= v |x|, v = 2^-16
for BF16 (two round-to-nearest steps of 8 significant bits) and 2^-22 for FP16
(11 significant bits), so a product is off by at most 3 v of its magnitude
(the dropped a_lo b_lo included); the FP32 accumulation of K terms adds at
most K 2^-24 of the sum of their magnitudes.  An output entry therefore
carries at most u_split(K) = 3 v + (K + 1) 2^-24 times the sum T of the
magnitudes of the products it adds (K = L + 2 table rows for the synthesis,
nlat/2 folded latitudes for the analysis).  In FP16 mode each column of the
data operand is scaled by a power of two that brings its largest entry into
[1/2, 1), and entries below FP16's smallest subnormal (2^-24 of the column's
largest) flush: at most 2^-24 of the column's largest entry per product more.
The transform tests hold every entry to this bound, with T computed from the
oracle's tables (tests/_oracle_helpers.py); the FFTs are FP64 and add
nothing at this level.  The non-linear tendency sums terms that largely cancel
(N_delta = curl(zeta V) + l(l+1)/a^2 KE for a balanced jet) and passes through
a synthesis, a product and an analysis, twice in a Heun step: a Heun step
U0 + tau/2 (N(U0) + N(U*)) is held entry by entry to 2 tau times the
first-order bound on the tendency's error (tests/_oracle_helpers.py,
tendency_error_bound: the synthesis errors propagated through the products
and the analysis, plus the analysis rounding; the factor 2 covers the two
evaluations, U* differing from U0 by tau N).

These worst-case bounds sit 10-1000 times above the errors rounding actually
makes (independent roundings partly cancel).  So every test also holds the GPU
to the rounding model's own error: the same transform or step computed on the
CPU with the split arithmetic emulated on the oracle's tables
(tests/_split_emulation.py: 16-bit hi/lo operands, three FP32 products, FP32
accumulation, the same parity folding and H combination).  The GPU's error
against the oracle, per field (largest entry and root mean square), must stay
within 4 times the emulation's: the two differ in summation order and in
where FP32 sums round, not in the model."""
import numpy as np
import pytest

from oracle import nonlinear as onl
from oracle.operator import Params, mode_index
from oracle.operator import n_modes as api_n_modes
from oracle.sht import Grid
from paper_1805_06557_amd.inputs import jet_state, random_field

from _oracle_helpers import analysis_term_sums, synthesis_term_sums, tendency_error_bound, term_scales
from _split_emulation import SplitGrid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SPLIT_UNIT = {"bf16": 2.0 ** -16, "fp16": 2.0 ** -22}


def u_split(L, nlat, mode="bf16"):
    """The bound for the longer of the two contractions (used by the Heun bars)."""
    return u_split_k(max(L + 2, nlat // 2), mode)


def u_split_k(K, mode):
    return 3 * SPLIT_UNIT[mode] + (K + 1) * 2.0 ** -24


def _flush_sums_synthesis(g, spec):
    """FP16 flush term per latitude: sum_m w_m (max_l |f_lm|) sum_l |Pbar_lm(mu_j)|."""
    L = g.L
    T = np.zeros(g.nlat)
    for m in range(L + 1):
        s = mode_index(L, m, m)
        T += (1.0 if m == 0 else 2.0) * np.abs(spec[s:s + L - m + 1]).max() * np.abs(g.P(m)).sum(axis=0)
    return T


def _flush_sums_analysis(g, field):
    """FP16 flush term per (l, m): (max_j w_j |F_m(mu_j)|) sum_j |Pbar_lm(mu_j)|."""
    L = g.L
    F = g._grid_to_fourier(field)
    T = np.zeros(api_n_modes(L))
    for m in range(L + 1):
        s = mode_index(L, m, m)
        T[s:s + L - m + 1] = (g.w * np.abs(F[m])).max() * np.abs(g.P(m)).sum(axis=1)
    return T


GRIDS = [(31, 48, 96), (63, 96, 192), (127, 192, 384)]
MODES = ["bf16", "fp16"]


def _prec(api, mode):
    return api.PREC_BF16_SPLIT if mode == "bf16" else api.PREC_FP16_SPLIT


def _api():
    from paper_1805_06557_amd import api
    return api


def _rel(got, ref):
    got, ref = np.atleast_2d(got), np.atleast_2d(ref)
    return [float(np.abs(got[f] - ref[f]).max() / np.abs(ref[f]).max()) for f in range(ref.shape[0])]


_term_scales = term_scales


def _heun_bound(g, U0, tau, mode):
    us, ua = u_split_k(g.L + 2, mode), u_split_k(g.nlat // 2, mode)
    return 2.0 * tau * tendency_error_bound(g, U0, us, ua)


def _check_heun(got, ref, bound, label):
    err = np.abs(got - ref)
    # entries whose bound is 0 (the l = 0 parts the operators leave exactly zero) must match exactly
    r = np.where(bound > 0, err / np.where(bound > 0, bound, 1.0), np.where(err > 0, np.inf, 0.0))
    print(label, "largest error / bound per field", r.max(axis=1).tolist())
    assert r.max() <= 1.0, r.max(axis=1).tolist()


MODEL_FACTOR = 4.0


def _model_check(got, ref, emu, label):
    """Per field: the GPU's largest and RMS error against the oracle within
    MODEL_FACTOR times the emulated split computation's."""
    got, ref, emu = (np.atleast_2d(x) for x in (got, ref, emu))
    e_g = np.abs(got - ref).max(axis=1)
    e_e = np.abs(emu - ref).max(axis=1)
    r_g = np.sqrt((np.abs(got - ref) ** 2).mean(axis=1))
    r_e = np.sqrt((np.abs(emu - ref) ** 2).mean(axis=1))
    print(label, "GPU / model error per field: largest", (e_g / e_e).tolist(), "rms", (r_g / r_e).tolist())
    assert np.all(e_g <= MODEL_FACTOR * e_e), (e_g / e_e).tolist()
    assert np.all(r_g <= MODEL_FACTOR * r_e), (r_g / r_e).tolist()


def _scaled(got, ref, scale):
    return [float(np.abs(got[f] - ref[f]).max() / scale[f]) for f in range(3)]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("L,nlat,nlon", GRIDS, ids=[f"T{g[0]}" for g in GRIDS])
def test_split_transforms(L, nlat, nlon, mode):
    """Every entry within the rounding bound of the module docstring."""
    api = _api()
    g = Grid(L, nlat, nlon, Params())
    rng = np.random.default_rng(300 + L)
    nf = 10                                    # more than one group of eight fields
    spec = np.stack([random_field(L, rng, 10.0 ** (k % 3)) for k in range(nf)])
    ctx = api.SWE(L, nlat, nlon, prec=_prec(api, mode))
    ds = torch.from_numpy(spec).cuda()
    dg = torch.empty((nf, nlat, nlon), dtype=torch.float64, device="cuda")
    ctx.sh_synthesis(ds, dg, nf)
    got = dg.cpu().numpy()
    us = u_split_k(L + 2, mode)
    worst = 0.0
    for f in range(nf):
        ref = g.synthesis(spec[f])
        bound = us * synthesis_term_sums(g, spec[f])
        if mode == "fp16":
            bound = bound + 2.0 ** -24 * _flush_sums_synthesis(g, spec[f])
        r = float((np.abs(got[f] - ref) / bound[:, None]).max())
        worst = max(worst, r)
        assert r <= 1.0, (f, r)
    print("synthesis", mode, L, "largest error / bound", worst, "field-relative", max(_rel(got.reshape(nf, -1),
          np.stack([g.synthesis(spec[f]) for f in range(nf)]).reshape(nf, -1))))
    sg = SplitGrid(L, nlat, nlon, Params(), mode)
    _model_check(got.reshape(nf, -1), np.stack([g.synthesis(spec[f]) for f in range(nf)]).reshape(nf, -1),
                 np.stack([sg.synthesis(spec[f]) for f in range(nf)]).reshape(nf, -1), f"T{L} synthesis {mode}")
    field = rng.standard_normal((nf, nlat, nlon))
    dso = torch.empty((nf, api.n_modes(L)), dtype=torch.complex128, device="cuda")
    ctx.sh_analysis(torch.from_numpy(field).cuda(), dso, nf)
    got = dso.cpu().numpy()
    ua = u_split_k(nlat // 2, mode)
    worst = 0.0
    for f in range(nf):
        ref = g.analysis(field[f])
        bound = ua * analysis_term_sums(g, field[f])
        if mode == "fp16":
            bound = bound + 2.0 ** -24 * _flush_sums_analysis(g, field[f])
        r = float((np.abs(got[f] - ref) / bound).max())
        worst = max(worst, r)
        assert r <= 1.0, (f, r)
    print("analysis", mode, L, "largest error / bound", worst)
    _model_check(got, np.stack([g.analysis(field[f]) for f in range(nf)]),
                 np.stack([sg.analysis(field[f]) for f in range(nf)]), f"T{L} analysis {mode}")
    ctx.sync()
    ctx.close()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("L,nlat,nlon", GRIDS[:2], ids=[f"T{g[0]}" for g in GRIDS[:2]])
def test_split_heun_increment(L, nlat, nlon, mode):
    api = _api()
    g = Grid(L, nlat, nlon, Params())
    U0 = jet_state(L, 3)
    tau = 900.0
    ref = onl.heun(g, U0, tau)
    ctx = api.SWE(L, nlat, nlon, prec=_prec(api, mode))
    d0 = torch.from_numpy(U0).cuda()
    d1 = torch.empty_like(d0)
    ctx.nonlinear_step(tau, d0, d1)
    got = d1.cpu().numpy()
    print("heun increment", mode, L, "relative to the increment", _rel(got - U0, ref - U0))
    _check_heun(got, ref, _heun_bound(g, U0, tau, mode), f"T{L} heun {mode}")
    emu = onl.heun(SplitGrid(L, nlat, nlon, Params(), mode), U0, tau)
    _model_check(got - U0, ref - U0, emu - U0, f"T{L} heun increment {mode}")
    ctx.close()


@pytest.fixture(scope="module")
def t255_heun_oracle():
    L, nlat, nlon = 255, 384, 768
    g = Grid(L, nlat, nlon, Params())
    U0 = jet_state(L, 2)
    return (g, U0, onl.heun(g, U0, 1800.0), {m: _heun_bound(g, U0, 1800.0, m) for m in MODES},
            {m: onl.heun(SplitGrid(L, nlat, nlon, Params(), m), U0, 1800.0) for m in MODES})


@pytest.mark.parametrize("mode", MODES)
def test_split_heun_t255_against_oracle(mode, t255_heun_oracle):
    """The T255 768 x 384 non-linear step (the workload's half step, tau = 1800 s)
    with the split Legendre stage against the oracle, per field, on the increment."""
    api = _api()
    g, U0, ref, bounds, emus = t255_heun_oracle
    L, nlat, nlon = g.L, g.nlat, g.nlon
    ctx = api.SWE(L, nlat, nlon, prec=_prec(api, mode))
    d0 = torch.from_numpy(U0).cuda()
    d1 = torch.empty_like(d0)
    ctx.nonlinear_step(1800.0, d0, d1)
    ctx.sync()
    got = d1.cpu().numpy()
    ctx.close()
    print("T255 heun increment vs oracle", mode, "relative to the increment", _rel(got - U0, ref - U0))
    _check_heun(got, ref, bounds[mode], f"T255 heun {mode}")
    _model_check(got - U0, ref - U0, emus[mode] - U0, f"T255 heun increment {mode}")


@pytest.fixture(scope="module")
def t511_heun_oracle():
    L, nlat, nlon = 511, 768, 1536
    g = Grid(L, nlat, nlon, Params())
    U0 = jet_state(L, 4)
    return (g, U0, onl.heun(g, U0, 900.0),
            {m: onl.heun(SplitGrid(L, nlat, nlon, Params(), m), U0, 900.0) for m in MODES})


@pytest.mark.parametrize("mode", MODES)
def test_split_t511_round_trip_and_step(mode, t511_heun_oracle):
    """T511 on 1536 x 768 (the analysis workgroup then needs more than 64 KB of
    LDS): synthesis then analysis of band-limited fields returns them to
    16 u_split(K) of each field's largest coefficient (Gauss quadrature makes
    the exact round trip the identity), and one non-linear step matches the
    oracle to the bar of the T255 case."""
    api = _api()
    L, nlat, nlon = 511, 768, 1536
    rng = np.random.default_rng(511)
    nf = 2
    spec = np.stack([random_field(L, rng, 1.0) for _ in range(nf)])
    ctx = api.SWE(L, nlat, nlon, prec=_prec(api, mode))
    ds = torch.from_numpy(spec).cuda()
    dg = torch.empty((nf, nlat, nlon), dtype=torch.float64, device="cuda")
    ctx.sh_synthesis(ds, dg, nf)
    back = torch.empty_like(ds)
    ctx.sh_analysis(dg, back, nf)
    e = _rel(back.cpu().numpy(), spec)
    print("T511 split round trip", mode, e)
    assert max(e) <= 16 * u_split(L, nlat, mode), e
    g, U0, ref, emus = t511_heun_oracle
    d0 = torch.from_numpy(U0).cuda()
    d1 = torch.empty_like(d0)
    ctx.nonlinear_step(900.0, d0, d1)
    ctx.sync()
    got = d1.cpu().numpy()
    print("T511 heun increment vs oracle", mode, "relative to the increment", _rel(got - U0, ref - U0))
    _model_check(got - U0, ref - U0, emus[mode] - U0, f"T511 heun increment {mode}")
    ctx.close()
