"""FP64 parity with the oracle at the sizes of the measured workloads, where
the longitude FFT runs at the lengths those workloads use (384 complex points
on the 768 x 384 grid of T255, 768 on the 1536 x 768 grid of T511) in every
mode of the ring kernel: inverse only (synthesis), forward only (analysis)
and the non-linear products (Heun step).  Section 3.2 (transforms), Section 3
(N(U)), Section 4.1 (Heun, ``erk``).

Bar: every compared entry of a transform within 1e-12 of the oracle relative
to the largest entry of its field.  A Heun step U1 = U0 + tau/2 (N(U0) + N(U*))
within max(1e-12, u_64 L(L+1)) of s_f = max(max |U1_f|, tau T_f) per field f,
T_f the largest of the tendency's terms (for the balanced jet the two terms of
N_delta nearly cancel, so the rounding of the step is relative to them, not to
their difference; and the l(l+1)/a^2 of N_delta's kinetic-energy term
multiplies the rounding of that term's analysis at degree l, up to L(L+1)
times a unit roundoff of the kinetic energy, while the field's largest
entries sit at low degree).  T511: the oracle transforms only sampled orders (its tables for
all 512 orders take seconds and 0.8 GB), except for the Heun step, which needs
the full tendency."""
import numpy as np
import pytest

from oracle import nonlinear as onl
from oracle.operator import Params, mode_index
from oracle.sht import Grid
from paper_1805_06557_amd.inputs import jet_state, random_field

from _oracle_helpers import term_scales

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _api():
    from paper_1805_06557_amd import api
    return api


def _rel_err(got, ref):
    got, ref = np.atleast_2d(got), np.atleast_2d(ref)
    return [float(np.abs(got[f] - ref[f]).max() / np.abs(ref[f]).max()) for f in range(ref.shape[0])]


def _heun_check(L, nlat, nlon, seed, tau, g=None):
    api = _api()
    g = g or Grid(L, nlat, nlon, Params())
    U0 = jet_state(L, seed)
    ref = onl.heun(g, U0, tau)
    ctx = api.SWE(L, nlat, nlon)
    d0 = torch.from_numpy(U0).cuda()
    d1 = torch.empty_like(d0)
    ctx.nonlinear_step(tau, d0, d1)
    ctx.sync()
    got = d1.cpu().numpy()
    ctx.close()
    scale = np.maximum(np.abs(ref).max(axis=1), tau * term_scales(g, U0))
    e = [float(np.abs(got[f] - ref[f]).max() / scale[f]) for f in range(3)]
    bar = max(1e-12, 2.0 ** -53 * L * (L + 1))
    print(f"T{L} Heun step vs oracle: per field {e} of max(|U1|, tau x largest term) (bar {bar:.3g}); "
          f"of |U1| {_rel_err(got, ref)}; of the increment {_rel_err(got - U0, ref - U0)}")
    assert max(e) <= bar, e


def test_t255_heun_step_fp64():
    """T255 on 768 x 384, tau = dt/2 = 1800 s (the half step of the T255 workloads)."""
    _heun_check(255, 384, 768, 2, 1800.0)


def test_t255_synthesis_and_analysis_fp64():
    api = _api()
    L, nlat, nlon, nf = 255, 384, 768, 3
    g = Grid(L, nlat, nlon, Params())
    rng = np.random.default_rng(255)
    spec = np.stack([random_field(L, rng, 10.0 ** k) for k in range(nf)])
    ctx = api.SWE(L, nlat, nlon)
    dg = torch.empty((nf, nlat, nlon), dtype=torch.float64, device="cuda")
    ctx.sh_synthesis(torch.from_numpy(spec).cuda(), dg, nf)
    ref = np.stack([g.synthesis(spec[f]) for f in range(nf)])
    e = _rel_err(dg.cpu().numpy().reshape(nf, -1), ref.reshape(nf, -1))
    print("T255 synthesis vs oracle", e)
    assert max(e) <= 1e-12, e
    field = rng.standard_normal((nf, nlat, nlon)) * np.array([1.0, 1e-5, 1e3])[:, None, None]
    ds = torch.empty((nf, api.n_modes(L)), dtype=torch.complex128, device="cuda")
    ctx.sh_analysis(torch.from_numpy(field).cuda(), ds, nf)
    ctx.sync()
    refa = np.stack([g.analysis(field[f]) for f in range(nf)])
    e = _rel_err(ds.cpu().numpy(), refa)
    print("T255 analysis vs oracle", e)
    assert max(e) <= 1e-12, e
    ctx.close()


T511_ORDERS = [0, 1, 2, 63, 255, 400, 509, 510, 511]


def _order_slice(L, m):
    s = mode_index(L, m, m)
    return slice(s, s + L - m + 1)


def test_t511_synthesis_sampled_orders_fp64():
    """A spectrum supported on sampled orders (all their degrees): the oracle's
    synthesis of exactly those orders against the GPU's, on the whole grid."""
    api = _api()
    L, nlat, nlon = 511, 768, 1536
    g = Grid(L, nlat, nlon, Params())
    rng = np.random.default_rng(511)
    full = random_field(L, rng, 1.0)
    spec = np.zeros_like(full)
    F = np.zeros((L + 1, nlat), dtype=np.complex128)
    for m in T511_ORDERS:
        sl = _order_slice(L, m)
        spec[sl] = full[sl] * (1.0 + 10.0 * m / L)     # the high orders no smaller than the low ones
        F[m] = spec[sl] @ g.P(m)
    ref = g._fourier_to_grid(F)
    ctx = api.SWE(L, nlat, nlon)
    dg = torch.empty((1, nlat, nlon), dtype=torch.float64, device="cuda")
    ctx.sh_synthesis(torch.from_numpy(spec[None, :].copy()).cuda(), dg, 1)
    ctx.sync()
    e = _rel_err(dg.cpu().numpy().reshape(1, -1), ref.reshape(1, -1))
    print("T511 synthesis (sampled orders) vs oracle", e)
    assert max(e) <= 1e-12, e
    ctx.close()


def test_t511_analysis_sampled_orders_fp64():
    """Analysis of an arbitrary grid field; the oracle's quadrature of the
    sampled orders against the GPU's coefficients of those orders."""
    api = _api()
    L, nlat, nlon, nf = 511, 768, 1536, 2
    g = Grid(L, nlat, nlon, Params())
    rng = np.random.default_rng(512)
    field = rng.standard_normal((nf, nlat, nlon))
    ctx = api.SWE(L, nlat, nlon)
    ds = torch.empty((nf, api.n_modes(L)), dtype=torch.complex128, device="cuda")
    ctx.sh_analysis(torch.from_numpy(field).cuda(), ds, nf)
    ctx.sync()
    got = ds.cpu().numpy()
    ctx.close()
    for f in range(nf):
        Fm = g._grid_to_fourier(field[f])
        ref = np.concatenate([g.P(m) @ (g.w * Fm[m]) for m in T511_ORDERS])
        idx = np.concatenate([np.arange(mode_index(L, m, m), mode_index(L, m, m) + L - m + 1) for m in T511_ORDERS])
        e = float(np.abs(got[f, idx] - ref).max() / np.abs(ref).max())
        print("T511 analysis (sampled orders) vs oracle, field", f, e)
        assert e <= 1e-12, e


def test_t511_heun_step_fp64():
    """T511 on 1536 x 768, tau = 900 s: the full oracle tendency (all orders)."""
    _heun_check(511, 768, 1536, 4, 900.0)


U32 = 2.0 ** -24
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def t255_strang_oracle():
    """The oracle's l_rexi_n_erk_ver1 step of the T255 workloads' jet state for
    both contours they use (p0 = 12: FP64 solves; p0 = 8: FP32 solves)."""
    from oracle import rexi as orexi
    from paper_1805_06557_amd import configs
    from _oracle_helpers import oracle_rexi_parallel
    p = Params()
    w64, w32 = configs.T255_FP64, configs.T255_FP32
    g = Grid(w64.L, w64.nlat, w64.nlon, p)
    U0 = jet_state(w64.L, w64.seed)
    A = onl.heun(g, U0, 0.5 * w64.dt)
    out = {"g": g, "U0": U0, "T": term_scales(g, U0)}
    for w in (w64, w32):
        a, b, _, _ = orexi.coefficients(orexi.FN_EXP, w.N, w.p0, w.y)
        R = oracle_rexi_parallel(A, a, b, w.dt, w.L, p)
        rho = w.dt * (np.sqrt(p.g * p.H * w.L * (w.L + 1)) / p.a + 2 * p.Omega)
        kap = float(orexi.kappa(a, b, 1j * np.linspace(-rho, rho, 401)).max())
        out[w.p0] = (a, b, onl.heun(g, R, 0.5 * w.dt), kap)
    return out


@pytest.mark.parametrize("name", ["T255-fp64", "T255-fp32", "T255-fp32-bf16", "T255-fp32-fp16"])
def test_t255_strang_step_against_oracle(name, t255_strang_oracle):
    """One l_rexi_n_erk_ver1 step of each T255 workload (768 x 384, dt = 3600 s,
    N = 800) against the oracle's step, per field.  FP64: max(1e-12, 4 u_64 kappa)
    of the field's largest entry (the REXI sum's floor).  FP32 solves:
    3 u_32 kappa of the field's largest entry (the REXI stage's per-field bar of
    test_gpu_rexi) plus, with a split Legendre stage, twice the split Heun bar
    (8 u_split(K) tau T_f per half step, test_gpu_split) for the two half steps."""
    from paper_1805_06557_amd import configs
    api = _api()
    w = configs.ALL[name]
    o = t255_strang_oracle
    a, b, ref, kap = o[w.p0]
    U0 = o["U0"]
    ctx = api.SWE(w.L, w.nlat, w.nlon, prec=w.prec)
    d0 = torch.from_numpy(U0).cuda()
    d1 = torch.empty_like(d0)
    ctx.strang_step(a, b, w.dt, d0, d1)
    ctx.sync()
    got = d1.cpu().numpy()
    ctx.close()
    fmax = np.abs(ref).max(axis=1)
    if w.prec == 0:
        bar = max(1e-12, 4 * U64 * kap) * fmax
    else:
        bar = 3 * U32 * kap * fmax
        if w.prec & (api.PREC_BF16_SPLIT | api.PREC_FP16_SPLIT):
            v = 2.0 ** -16 if w.prec & api.PREC_BF16_SPLIT else 2.0 ** -22
            us = 3 * v + (max(w.L + 2, w.nlat // 2) + 1) * U32
            bar = bar + 2 * 8 * us * (0.5 * w.dt) * o["T"]
    err = np.abs(got - ref).max(axis=1)
    linf = err / fmax
    l2 = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    print(f"{name} step vs oracle: linf {linf.tolist()} l2 {l2.tolist()} error / bar {(err / bar).tolist()}")
    assert np.all(err <= bar), (err / bar).tolist()
