"""The workloads this library is measured and tested on.

Contour parameters: the T31 case uses the paper's own choice (p0 = 10,
p_{+-1} = +-30i, N = 128; Section 5).  For the others y = sqrt(2) 1.05 rho with
rho = dt (sqrt(g H L(L+1)) / a + 2 Omega) the spectral-radius bound of dt L,
and p0 is the shift that minimises the scalar error max_{|w|<=rho}
|S(i w) - e^{i w}| at the stated N for the solve precision (p0 trades the
geometric error of the trapezoidal rule against the cancellation of the sum,
Section 4.2.2).
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

T511_FP64 = Workload(
    "T511-fp64", L=511, nlat=768, nlon=1536, dt=7200.0, N=2000, p0=24.0, y=270.3467676176863,
    steps=1, seed=4,
    desc="linear+nonlinear SWE, T511 on 1536x768, dt = 7200 s, N = 2000, FP64")

ALL = {w.name: w for w in [T31_LINEAR, T127_NONLINEAR, T255_FP64, T255_FP32, T511_FP64]}
