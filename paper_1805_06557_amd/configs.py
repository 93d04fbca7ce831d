"""The workloads this library is measured and tested on.

Contour parameters: the T31 case uses the paper's own choice (p0 = 10,
p_{+-1} = +-30i, N = 128; Section 5).  For the others y = sqrt(2) 1.05 rho with
rho = dt (sqrt(g H L(L+1)) / a + 2 Omega) the spectral-radius bound of dt L,
and p0 is the shift that minimises the predicted error (scalar error
max_{|w|<=rho} |S(i w) - e^{i w}| plus unit roundoff times the sum's
cancellation factor) at the stated N for the solve precision, as the
library's rexi_choose_contour evaluates it (p0 trades the geometric error of
the trapezoidal rule against the cancellation of the sum, Section 4.2.2).
"""
from __future__ import annotations

from dataclasses import dataclass, field


@dataclass(frozen=True)
class Workload:
    name: str
    L: int
    nlat: int
    nlon: int
    dt: float
    N: int
    p0: float
    y: float
    steps: int = 1
    prec: int = 0           # REXI_PREC_* flags
    seed: int = 0
    desc: str = ""
    extra: dict = field(default_factory=dict)


T31_LINEAR = Workload(
    "T31-linear", L=31, nlat=0, nlon=0, dt=3600.0, N=128, p0=10.0, y=30.0, seed=0,
    desc="linear SWE, T31, one REXI step dt = 3600 s, N = 128 (paper's contour), FP64")

T127_NONLINEAR = Workload(
    "T127-nonlinear", L=127, nlat=192, nlon=384, dt=1800.0, N=400, p0=5.0, y=17.139645430207057,
    steps=24, seed=1,
    desc="nonlinear SWE, T127 on 384x192, dt = 1800 s, N = 400, 24 Strang steps, FP64")

T255_FP64 = Workload(
    "T255-fp64", L=255, nlat=384, nlon=768, dt=3600.0, N=800, p0=12.0, y=67.91071976436587,
    steps=4, seed=2,
    desc="nonlinear SWE, T255 on 768x384, dt = 3600 s, N = 800, FP64 solves")

T255_FP32 = Workload(
    "T255-fp32", L=255, nlat=384, nlon=768, dt=3600.0, N=800, p0=8.0, y=67.91071976436587,
    steps=4, prec=1, seed=2,
    desc="nonlinear SWE, T255 on 768x384, dt = 3600 s, N = 800, FP32 solves, FP64 beta sum")

T255_FP32_BF16 = Workload(
    "T255-fp32-bf16", L=255, nlat=384, nlon=768, dt=3600.0, N=800, p0=8.0, y=67.91071976436587,
    steps=4, prec=1 | 2, seed=2,
    desc="nonlinear SWE, T255 on 768x384, dt = 3600 s, N = 800, FP32 solves, FP64 beta sum, "
         "split-BF16 matrix-core Legendre stage")

T255_FP32_FP16 = Workload(
    "T255-fp32-fp16", L=255, nlat=384, nlon=768, dt=3600.0, N=800, p0=8.0, y=67.91071976436587,
    steps=4, prec=1 | 4, seed=2,
    desc="nonlinear SWE, T255 on 768x384, dt = 3600 s, N = 800, FP32 solves, FP64 beta sum, "
         "split-FP16 matrix-core Legendre stage")

# The jet at T511 and dt = 7200 s sees the explicit Heun stage at an advective
# Courant number near 2 and turns non-finite after about nine steps, so a bench
# run times one step (after one warm-up) there.
T511_FP64 = Workload(
    "T511-fp64", L=511, nlat=768, nlon=1536, dt=7200.0, N=2000, p0=24.0, y=270.3467676176863,
    steps=1, seed=4,
    desc="linear+nonlinear SWE, T511 on 1536x768, dt = 7200 s, N = 2000, FP64",
    extra={"max_steps": 1})

# T511 with the split-FP16 Legendre stage; the solves stay FP64 (at dt = 7200 s
# no FP32 contour reaches a useful error: rexi_choose_contour finds none).
T511_FP64_FP16 = Workload(
    "T511-fp64-fp16", L=511, nlat=768, nlon=1536, dt=7200.0, N=2000, p0=24.0, y=270.3467676176863,
    steps=1, prec=4, seed=4,
    desc="linear+nonlinear SWE, T511 on 1536x768, dt = 7200 s, N = 2000, FP64 solves, "
         "split-FP16 matrix-core Legendre stage",
    extra={"max_steps": 1})

ALL = {w.name: w for w in [T31_LINEAR, T127_NONLINEAR, T255_FP64, T255_FP32, T255_FP32_BF16, T255_FP32_FP16,
                           T511_FP64, T511_FP64_FP16]}


# FP32 against FP64 solves at one fixed accuracy: the T255 REXI stage
# (dt = 3600 s) at a target scalar error E = 1e-4 on |w| <= rho.  Each
# precision gets its own contour, the fewest poles whose predicted error
# (approximation error + unit roundoff x kappa) meets E over the p0 grid of
# rexi_choose_contour: FP32 needs a small shift (its rounding floor u_32 kappa grows
# like e^{p0}) and therefore many poles, FP64 reaches E with a large shift and
# few poles.
EQUAL_ERROR_E = 1e-4
T255_FP32_AT_E = Workload(
    "T255-fp32-at-E", L=255, nlat=0, nlon=0, dt=3600.0, N=776, p0=8.0, y=67.91071976436587, prec=1, seed=2,
    desc="REXI stage T255, dt = 3600 s, FP32 solves, contour chosen for E = 1e-4")
T255_FP64_AT_E = Workload(
    "T255-fp64-at-E", L=255, nlat=0, nlon=0, dt=3600.0, N=190, p0=28.0, y=67.91071976436587, prec=0, seed=2,
    desc="REXI stage T255, dt = 3600 s, FP64 solves, contour chosen for E = 1e-4")

# Ensemble of linear-SWE instances of mixed truncation (T63/T127/T255), pole
# counts N = 2 randint(100, 400], dt = 3600 s, FP32 solves with the FP64 pole
# sum; each member's p0 minimises its predicted error at its N.
ENSEMBLE = Workload(
    "ensemble-64", L=255, nlat=0, nlon=0, dt=3600.0, N=0, p0=0.0, y=0.0, prec=1, seed=3,
    desc="64 linear-SWE members, T63/T127/T255 mixed, N in [202, 800], one fused REXI launch",
    extra={"count": 64})

ALL.update({w.name: w for w in [T255_FP32_AT_E, T255_FP64_AT_E, ENSEMBLE]})


def ensemble_plan(count: int = 64, seed: int = 3, prec: int = 1, dt: float = 3600.0):
    """Members of the ensemble: list of dicts with L, N, p0, y, dt and the input seed
    (each member's shift from the library's rexi_choose_contour at its N)."""
    from . import api
    from .inputs import ensemble_members
    cache = {}
    out = []
    for L, N, s in ensemble_members(count, seed):
        if (L, N) not in cache:
            cache[(L, N)] = api.choose_contour(api.spectral_radius(L, dt), prec=prec, N_fixed=N)
        c = cache[(L, N)]
        out.append(dict(L=L, N=N, p0=c["p0"], y=c["y"], dt=dt, seed=s))
    return out
