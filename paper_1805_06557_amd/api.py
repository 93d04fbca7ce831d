"""Python binding of the C-ABI: argument marshalling only.

Device memory and streams come from PyTorch (complex128 CUDA tensors for
spectral states, float64 for grids); every computation runs in the library's
HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib

REXI_OK, REXI_EINVAL, REXI_ENOMEM, REXI_EDEVICE, REXI_ENOTSUP, REXI_ENUMERIC = 0, -1, -2, -3, -4, -5
FN_EXP, FN_PSI1, FN_PSI2 = 0, 1, 2
PREC_FP64, PREC_FP32_SOLVE, PREC_BF16_SPLIT, PREC_FP16_SPLIT = 0, 1, 2, 4
KERNEL_SOLVE, KERNEL_REDUCE, KERNEL_LEG_SYNTH, KERNEL_RING, KERNEL_LEG_ANAL, KERNEL_FACTOR, KERNEL_LEG_FUSED = range(7)
SOLVER_FUSED, SOLVER_STREAM, SOLVER_HYBRID = 1, 2, 3
SPLIT_REXI_V1, SPLIT_REXI_V0, SPLIT_CN_V1, SPLIT_CN_V0, SPLIT_LG_REXI_V1 = 0, 1, 2, 3, 4
EARTH = dict(a=6.37122e6, g=9.80616, H=1.0e4, Omega=7.292e-5)


class RexiError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


def _check(rc: int, where: str) -> None:
    if rc != REXI_OK:
        raise RexiError(rc, where, _lib.load().rexi_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def n_modes(L: int) -> int:
    return (L + 1) * (L + 2) // 2


def rexi_coefficients(fn: int, N: int, p0: float, y: float):
    """alpha, beta (complex128 numpy arrays), r, mu -- see rexi_coefficients()."""
    alpha = np.zeros(2 * N)
    beta = np.zeros(2 * N)
    r = ctypes.c_double()
    mu = ctypes.c_double()
    _check(_lib.load().rexi_coefficients(fn, N, p0, y, _dptr(alpha), _dptr(beta), ctypes.byref(r),
                                         ctypes.byref(mu)), "rexi_coefficients")
    return alpha.view(np.complex128), beta.view(np.complex128), r.value, mu.value


def spectral_radius(L: int, dt: float, a: float = EARTH["a"], g: float = EARTH["g"], H: float = EARTH["H"],
                    Omega: float = EARTH["Omega"]) -> float:
    """rho bounding the spectrum of dt L -- see rexi_spectral_radius()."""
    rho = ctypes.c_double()
    _check(_lib.load().rexi_spectral_radius(L, float(dt), a, g, H, Omega, ctypes.byref(rho)), "rexi_spectral_radius")
    return rho.value


def check_contour(L: int, dt: float, alpha, beta, a: float = EARTH["a"], g: float = EARTH["g"],
                  H: float = EARTH["H"], Omega: float = EARTH["Omega"]) -> float:
    """The host checks of a coefficient set (rexi_check_contour); returns the
    dominance margin, raises RexiError when a check fails."""
    al = _host_coeffs(alpha)
    be = _host_coeffs(beta)
    if al.size != be.size:
        raise ValueError("alpha and beta differ in length")
    margin = ctypes.c_double(float("nan"))
    _check(_lib.load().rexi_check_contour(L, a, g, H, Omega, float(dt), _dptr(al), _dptr(be), al.size // 2,
                                          ctypes.byref(margin)), "rexi_check_contour")
    return margin.value


def contour_error(alpha, beta, rho: float, npts: int = 1601):
    """(approx, kappa) of a coefficient set on i[-rho, rho] -- see rexi_contour_error()."""
    al = _host_coeffs(alpha)
    be = _host_coeffs(beta)
    if al.size != be.size:
        raise ValueError("alpha and beta differ in length")
    e = ctypes.c_double()
    k = ctypes.c_double()
    _check(_lib.load().rexi_contour_error(_dptr(al), _dptr(be), al.size // 2, float(rho), int(npts), ctypes.byref(e),
                                          ctypes.byref(k)), "rexi_contour_error")
    return e.value, k.value


def choose_contour(rho: float, target: float = 0.0, prec: int = PREC_FP64, N_fixed: int = 0, p0_grid=None,
                   n_max: int = 4096):
    """dict(p0, y, N, predicted) -- see rexi_choose_contour()."""
    grid = None if p0_grid is None else np.ascontiguousarray(np.asarray(p0_grid, dtype=np.float64))
    p0, y, pred = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    N = ctypes.c_int()
    _check(_lib.load().rexi_choose_contour(float(rho), float(target), int(prec), int(N_fixed),
                                           None if grid is None else _dptr(grid), 0 if grid is None else grid.size,
                                           int(n_max), ctypes.byref(p0), ctypes.byref(y), ctypes.byref(N),
                                           ctypes.byref(pred)), "rexi_choose_contour")
    return dict(p0=p0.value, y=y.value, N=N.value, predicted=pred.value)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _state_ptr(t, L: int, nf: int, name: str):
    import torch
    if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
        raise ValueError(f"{name}: expected a contiguous complex128 CUDA tensor")
    if t.numel() != nf * n_modes(L):
        raise ValueError(f"{name}: expected {nf} x {n_modes(L)} complex entries, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _grid_ptr(t, nlat: int, nlon: int, nf: int, name: str):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name}: expected a contiguous float64 CUDA tensor")
    if t.numel() != nf * nlat * nlon:
        raise ValueError(f"{name}: expected {nf} x {nlat} x {nlon} entries, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _host_coeffs(c) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(c, dtype=np.complex128))
    return c.view(np.float64)


class SWE:
    """A library context (swe_ctx) for truncation L on an nlat x nlon Gauss grid."""

    def __init__(self, L: int, nlat: int = 0, nlon: int = 0, a: float = EARTH["a"], g: float = EARTH["g"],
                 H: float = EARTH["H"], Omega: float = EARTH["Omega"], prec: int = PREC_FP64):
        self.L, self.nlat, self.nlon, self.prec = L, nlat, nlon, prec
        self.a, self.g, self.H, self.Omega = a, g, H, Omega
        self.modes = n_modes(L)
        self._lib = _lib.load()
        h = ctypes.c_void_p()
        _check(self._lib.swe_create(L, nlat, nlon, a, g, H, Omega, prec, ctypes.byref(h)), "swe_create")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.swe_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_tuning(self, solver: int = 0, seg_rows: int = 0, waves: int = 0, poles_per_lane: int = 0) -> None:
        """Schedule (SOLVER_*) and launch shape of the REXI solve; 0 keeps a value."""
        _check(self._lib.swe_set_tuning(self._h, solver, seg_rows, waves, poles_per_lane), "swe_set_tuning")

    def set_fusion(self, enable: bool) -> None:
        """Fused split-precision transform launches (default on; same result bits)."""
        _check(self._lib.swe_set_fusion(self._h, 1 if enable else 0), "swe_set_fusion")

    def get_fusion(self) -> bool:
        v = ctypes.c_int()
        _check(self._lib.swe_get_fusion(self._h, ctypes.byref(v)), "swe_get_fusion")
        return bool(v.value)

    def get_tuning(self) -> dict:
        v = [ctypes.c_int() for _ in range(4)]
        _check(self._lib.swe_get_tuning(self._h, *[ctypes.byref(x) for x in v]), "swe_get_tuning")
        return dict(zip(("solver", "seg_rows", "waves", "poles_per_lane"), (x.value for x in v)))

    def autotune(self, alpha, beta, dt: float, U0, U1, reps: int = 3, stream=None) -> float:
        """Times every schedule and launch shape on this problem, keeps the fastest;
        returns the mean milliseconds of one REXI stage with it."""
        a = _host_coeffs(alpha)
        b = _host_coeffs(beta)
        ms = ctypes.c_double()
        _check(self._lib.swe_autotune(self._h, _dptr(a), _dptr(b), a.size // 2, float(dt),
                                      _state_ptr(U0, self.L, 3, "U0"), _state_ptr(U1, self.L, 3, "U1"), int(reps),
                                      _stream_handle(stream), ctypes.byref(ms)), "swe_autotune")
        return ms.value

    def rexi_linear_step(self, alpha, beta, dt: float, U0, U1, stream=None) -> None:
        a = _host_coeffs(alpha)
        b = _host_coeffs(beta)
        N = a.size // 2
        if b.size != a.size:
            raise ValueError("alpha and beta differ in length")
        _check(self._lib.rexi_linear_step(self._h, _dptr(a), _dptr(b), N, float(dt),
                                          _state_ptr(U0, self.L, 3, "U0"), _state_ptr(U1, self.L, 3, "U1"),
                                          _stream_handle(stream)), "rexi_linear_step")

    def rexi_lg_step(self, alpha, beta, dt: float, U0, U1, stream=None) -> None:
        """REXI stage of the gravity-wave part L_g alone (U1 may equal U0)."""
        a = _host_coeffs(alpha)
        b = _host_coeffs(beta)
        _check(self._lib.rexi_lg_step(self._h, _dptr(a), _dptr(b), a.size // 2, float(dt),
                                      _state_ptr(U0, self.L, 3, "U0"), _state_ptr(U1, self.L, 3, "U1"),
                                      _stream_handle(stream)), "rexi_lg_step")

    def rexi_lg_step_noalloc(self, alpha, beta, dt: float, U0, U1, stream=None) -> None:
        """rexi_lg_step without device allocation (scratch in the library's static array)."""
        a = _host_coeffs(alpha)
        b = _host_coeffs(beta)
        _check(self._lib.rexi_lg_step_noalloc(self._h, _dptr(a), _dptr(b), a.size // 2, float(dt),
                                              _state_ptr(U0, self.L, 3, "U0"), _state_ptr(U1, self.L, 3, "U1"),
                                              _stream_handle(stream)), "rexi_lg_step_noalloc")

    def sh_synthesis(self, spec, grid, nf: int, stream=None) -> None:
        _check(self._lib.sh_synthesis(self._h, _state_ptr(spec, self.L, nf, "spec"),
                                      _grid_ptr(grid, self.nlat, self.nlon, nf, "grid"), nf,
                                      _stream_handle(stream)), "sh_synthesis")

    def sh_analysis(self, grid, spec, nf: int, stream=None) -> None:
        _check(self._lib.sh_analysis(self._h, _grid_ptr(grid, self.nlat, self.nlon, nf, "grid"),
                                     _state_ptr(spec, self.L, nf, "spec"), nf, _stream_handle(stream)),
               "sh_analysis")

    def nonlinear_step(self, tau: float, U0, U1, stream=None) -> None:
        _check(self._lib.swe_nonlinear_step(self._h, float(tau), _state_ptr(U0, self.L, 3, "U0"),
                                            _state_ptr(U1, self.L, 3, "U1"), _stream_handle(stream)),
               "swe_nonlinear_step")

    def strang_step(self, alpha, beta, dt: float, U0, U1, stream=None) -> None:
        a = _host_coeffs(alpha)
        b = _host_coeffs(beta)
        _check(self._lib.swe_strang_step(self._h, _dptr(a), _dptr(b), a.size // 2, float(dt),
                                         _state_ptr(U0, self.L, 3, "U0"), _state_ptr(U1, self.L, 3, "U1"),
                                         _stream_handle(stream)), "swe_strang_step")

    def strang_steps(self, alpha, beta, dt: float, nsteps: int, U0, U1, stream=None) -> None:
        """nsteps Strang steps from U0, result in U1 (bit-identical to separate steps)."""
        a = _host_coeffs(alpha)
        b = _host_coeffs(beta)
        _check(self._lib.swe_strang_steps(self._h, _dptr(a), _dptr(b), a.size // 2, float(dt), int(nsteps),
                                          _state_ptr(U0, self.L, 3, "U0"), _state_ptr(U1, self.L, 3, "U1"),
                                          _stream_handle(stream)), "swe_strang_steps")

    def cn_step(self, dt: float, U0, U1, stream=None) -> None:
        """Crank-Nicolson step of the linear part (U0 and U1 must differ)."""
        _check(self._lib.swe_cn_step(self._h, float(dt), _state_ptr(U0, self.L, 3, "U0"),
                                     _state_ptr(U1, self.L, 3, "U1"), _stream_handle(stream)), "swe_cn_step")

    def split_step(self, scheme: int, alpha, beta, dt: float, U0, U1, stream=None) -> None:
        """One Strang-split step (SPLIT_*); alpha, beta may be None for the CN schemes."""
        if alpha is None:
            a = b = None
            N = 0
        else:
            a, b = _host_coeffs(alpha), _host_coeffs(beta)
            N = a.size // 2
        _check(self._lib.swe_split_step(self._h, int(scheme), None if a is None else _dptr(a),
                                        None if b is None else _dptr(b), N, float(dt),
                                        _state_ptr(U0, self.L, 3, "U0"), _state_ptr(U1, self.L, 3, "U1"),
                                        _stream_handle(stream)), "swe_split_step")

    def etdrk2_step(self, alpha, beta0, beta1, beta2, dt: float, U0, U1, stream=None) -> None:
        """One l_rexi_n_etdrk step; beta0/1/2: the psi_0/1/2 weights on the contour alpha."""
        a = _host_coeffs(alpha)
        b = [_host_coeffs(x) for x in (beta0, beta1, beta2)]
        if any(x.size != a.size for x in b):
            raise ValueError("alpha and the beta sets differ in length")
        _check(self._lib.swe_etdrk2_step(self._h, _dptr(a), _dptr(b[0]), _dptr(b[1]), _dptr(b[2]), a.size // 2,
                                         float(dt), _state_ptr(U0, self.L, 3, "U0"), _state_ptr(U1, self.L, 3, "U1"),
                                         _stream_handle(stream)), "swe_etdrk2_step")

    def profile(self, enable: bool) -> None:
        _check(self._lib.swe_profile(self._h, 1 if enable else 0), "swe_profile")

    def profile_kernels(self, kernels) -> None:
        """Record HIP events around the launches of the given kernel ids only."""
        mask = 0
        for k in kernels:
            mask |= 1 << int(k)
        _check(self._lib.swe_profile_kernels(self._h, mask), "swe_profile_kernels")

    def profile_read(self, kernel: int):
        """(total_ms, launches) recorded for one kernel since the last read."""
        ms = ctypes.c_double()
        n = ctypes.c_int()
        _check(self._lib.swe_profile_read(self._h, kernel, ctypes.byref(ms), ctypes.byref(n)),
               "swe_profile_read")
        return ms.value, n.value

    def sync(self) -> None:
        _check(self._lib.swe_sync(self._h), "swe_sync")


def rexi_linear_step_batched(members, stream=None) -> None:
    """members: sequence of (SWE, alpha, beta, dt, U0, U1); one ensemble REXI stage."""
    lib = _lib.load()
    arr = (_lib.RexiMember * len(members))()
    keep = []
    for i, (ctx, alpha, beta, dt, U0, U1) in enumerate(members):
        a = _host_coeffs(alpha)
        b = _host_coeffs(beta)
        if b.size != a.size:
            raise ValueError("alpha and beta differ in length")
        keep += [a, b]
        arr[i] = _lib.RexiMember(ctx.handle, _dptr(a), _dptr(b), a.size // 2, float(dt),
                                 _state_ptr(U0, ctx.L, 3, "U0"), _state_ptr(U1, ctx.L, 3, "U1"))
    _check(lib.rexi_linear_step_batched(arr, len(members), _stream_handle(stream)), "rexi_linear_step_batched")
