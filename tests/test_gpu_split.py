"""Split-precision (16-bit hi/lo on the matrix cores, FP32 accumulation) Legendre
stage against the FP64 oracle, in both modes: BF16 and FP16.

Stated tolerance: every product a b is formed as a_hi b_hi + a_hi b_lo + a_lo b_hi
with |x - x_hi - x_lo| <= v |x|, v = 2^-16 for BF16 (two round-to-nearest steps
of 8 significant bits) and 2^-22 for FP16 (11 significant bits; the data columns
are scaled by powers of two so that their largest entry lies in [1/2, 1), and
entries below FP16's smallest subnormal 2^-24 flush, an absolute 2^-25 of the
column's largest entry), so a product is off by at most 3 v of its magnitude
(the dropped a_lo b_lo included) plus 2^-24 of the largest; the FP32
accumulation over K = max(L + 1, nlat/2) terms adds K 2^-24.  An output thus
carries at most u_split(K) = 3 v + (K + 1) 2^-24 times the sum of the
magnitudes of its terms.  For these smooth and (l+1)^-2 spectra that sum
stays within 16 times the field's largest value, so the transforms' bar is
16 u_split(K) of each field's largest entry (measured errors, printed, are near
1e-5).  The non-linear tendency sums terms that largely cancel (N_delta =
curl(zeta V) + l(l+1)/a^2 KE for a balanced jet) and passes through a synthesis,
a product and an analysis, twice in a Heun step, so a Heun step's increment is
held to 24 u_split(K) of tau times the largest of the tendency's terms (div(hV)
for h, div(zeta V) for zeta, max(curl(zeta V), lap KE) for delta, from the
oracle's own pieces)."""
import numpy as np
import pytest

from oracle import nonlinear as onl
from oracle.operator import Params
from oracle.sht import Grid, degree_array, inv_laplacian
from paper_1805_06557_amd.inputs import jet_state, random_field

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SPLIT_UNIT = {"bf16": 2.0 ** -16, "fp16": 2.0 ** -22}


def u_split(L, nlat, mode="bf16"):
    return 3 * SPLIT_UNIT[mode] + (max(L + 1, nlat // 2) + 1) * 2.0 ** -24


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


def _term_scales(g, U):
    """Largest magnitude among the terms of each tendency component (oracle pieces)."""
    L, a = g.L, g.p.a
    h, zeta, delta = U
    hg, zg = g.synthesis(h), g.synthesis(zeta)
    Ug, Vg = g.uv_from_psichi(inv_laplacian(zeta, L, a), inv_laplacian(delta, L, a))
    div_h, _ = g.div_curl(hg * Ug, hg * Vg)
    div_z, curl_z = g.div_curl(zg * Ug, zg * Vg)
    ke = g.analysis((Ug * Ug + Vg * Vg) / (2.0 * (g.sint[:, None] ** 2)))
    l = degree_array(L).astype(np.float64)
    lap = (l * (l + 1.0) / (a * a)) * ke
    return np.array([np.abs(div_h).max(), np.abs(div_z).max(), max(np.abs(curl_z).max(), np.abs(lap).max())])


def _scaled(got, ref, scale):
    return [float(np.abs(got[f] - ref[f]).max() / scale[f]) for f in range(3)]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("L,nlat,nlon", GRIDS, ids=[f"T{g[0]}" for g in GRIDS])
def test_split_transforms(L, nlat, nlon, mode):
    api = _api()
    g = Grid(L, nlat, nlon, Params())
    rng = np.random.default_rng(300 + L)
    nf = 10                                    # more than one group of eight fields
    spec = np.stack([random_field(L, rng, 10.0 ** (k % 3)) for k in range(nf)])
    ctx = api.SWE(L, nlat, nlon, prec=_prec(api, mode))
    ds = torch.from_numpy(spec).cuda()
    dg = torch.empty((nf, nlat, nlon), dtype=torch.float64, device="cuda")
    ctx.sh_synthesis(ds, dg, nf)
    ref = np.stack([g.synthesis(spec[f]) for f in range(nf)]).reshape(nf, -1)
    e = _rel(dg.cpu().numpy().reshape(nf, -1), ref)
    print("synthesis", mode, L, max(e))
    assert max(e) <= 16 * u_split(L, nlat, mode), e
    field = rng.standard_normal((nf, nlat, nlon))
    dso = torch.empty((nf, api.n_modes(L)), dtype=torch.complex128, device="cuda")
    ctx.sh_analysis(torch.from_numpy(field).cuda(), dso, nf)
    refa = np.stack([g.analysis(field[f]) for f in range(nf)])
    e = _rel(dso.cpu().numpy(), refa)
    print("analysis", mode, L, max(e))
    assert max(e) <= 16 * u_split(L, nlat, mode), e
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
    e = _scaled(got - U0, ref - U0, tau * _term_scales(g, U0))
    print("heun increment", mode, L, e, "relative to the increment", _rel(got - U0, ref - U0))
    assert max(e) <= 24 * u_split(L, nlat, mode), e
    ctx.close()


@pytest.mark.parametrize("mode", MODES)
def test_split_matches_fp64_path_at_t255(mode):
    """The T255 768 x 384 non-linear step with the split Legendre stage against
    the FP64 path (itself pinned to the oracle), per field, on the increment."""
    api = _api()
    L, nlat, nlon = 255, 384, 768
    U0 = jet_state(L, 2)
    d0 = torch.from_numpy(U0).cuda()
    outs = []
    for prec in (0, _prec(api, mode)):
        ctx = api.SWE(L, nlat, nlon, prec=prec)
        d1 = torch.empty_like(d0)
        ctx.nonlinear_step(1800.0, d0, d1)
        outs.append(d1.cpu().numpy())
        ctx.close()
    g = Grid(L, nlat, nlon, Params())
    e = _scaled(outs[1] - U0, outs[0] - U0, 1800.0 * _term_scales(g, U0))
    print("T255 heun increment vs FP64 path", mode, e, "relative to the increment", _rel(outs[1] - U0, outs[0] - U0))
    assert max(e) <= 24 * u_split(L, nlat, mode), e


@pytest.mark.parametrize("mode", MODES)
def test_split_t511_round_trip_and_step(mode):
    """T511 on 1536 x 768 (the analysis workgroup then needs more than 64 KB of
    LDS): synthesis then analysis of band-limited fields returns them to
    16 u_split(K) of each field's largest coefficient (Gauss quadrature makes
    the exact round trip the identity), and one non-linear step matches the
    FP64 path (pinned to the oracle) to the bar of the T255 case."""
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
    U0 = jet_state(L, 4)
    d0 = torch.from_numpy(U0).cuda()
    outs = []
    for prec in (0, _prec(api, mode)):
        c = api.SWE(L, nlat, nlon, prec=prec)
        d1 = torch.empty_like(d0)
        c.nonlinear_step(900.0, d0, d1)
        outs.append(d1.cpu().numpy())
        c.close()
    g = Grid(L, nlat, nlon, Params())
    e = _scaled(outs[1] - U0, outs[0] - U0, 900.0 * _term_scales(g, U0))
    print("T511 heun increment vs FP64 path", mode, e, "relative to the increment", _rel(outs[1] - U0, outs[0] - U0))
    assert max(e) <= 24 * u_split(L, nlat, mode), e
    ctx.close()
