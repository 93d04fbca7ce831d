"""CPU emulation of the split-precision rounding model of the Legendre stage
(tests only).  The oracle's FP64 tables and transforms are kept; only the
Legendre contractions are replaced by the model: every operand x becomes
x_hi = t(x) and x_lo = t(x - x_hi) for the 16-bit type t (bfloat16 or float16,
round to nearest even), and a contraction sum_k a_k b_k becomes
A_hi B_hi + A_hi B_lo + A_lo B_hi with FP32 products and FP32 accumulation
(numpy float32 matrix products).  In float16 mode the data operand is rounded
to FP32, every column of it scaled by the power of two that brings its largest
magnitude into [1/2, 1), and the products unscaled afterwards.  The contractions are arranged as the
matrix-core stage arranges them: per zonal order m, degrees split by the
parity of l - m against the northern latitudes (the southern hemisphere by
the symmetry of Pbar), vector fields through Pbar rows up to degree L+1 with
H_l = hA_l Pbar_{l+1} + hB_l Pbar_{l-1} (hA_l = -l eps_{l+1}, hB_l = (l+1) eps_l)
moved onto the coefficients (synthesis) or combined after the products
(analysis).  SplitGrid(mode) is an oracle Grid whose four transform methods
follow this model, so oracle.nonlinear.tendency and heun on it give the error
that the rounding model predicts for a whole non-linear step."""
import numpy as np

from oracle.operator import mode_index, n_modes
from oracle.sht import Grid, legendre_m


def _round_bf16(x):
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _round_fp16(x):
    return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)


def split16(x, mode):
    r = _round_bf16 if mode == "bf16" else _round_fp16
    hi = r(x)
    lo = r(np.asarray(x, dtype=np.float64) - hi)
    return hi, lo


def _col_scale(B, mode):
    """Per-column power-of-two scale (float16 mode) of a real [K, C] operand."""
    if mode != "fp16":
        return np.ones(B.shape[1])
    mx = np.abs(B).max(axis=0)
    e = np.where(mx > 0, np.floor(np.log2(np.where(mx > 0, mx, 1.0))) + 1, 0)
    return np.exp2(-e)


def mm_split(A, B, mode):
    """A [M, K] (table) times B [K, C] (data), both real, in the split model.
    In float16 mode the data operand is rounded to FP32 before it is scaled and
    split (the kernels stage it in FP32 to find the column maxima)."""
    if mode == "fp16":
        B = np.asarray(B, dtype=np.float32).astype(np.float64)
    s = _col_scale(B, mode)
    Ah, Al = split16(A, mode)
    Bh, Bl = split16(B * s[None, :], mode)
    f32 = np.float32
    C = (Ah.astype(f32) @ Bh.astype(f32)) + (Ah.astype(f32) @ Bl.astype(f32)) + (Al.astype(f32) @ Bh.astype(f32))
    return C.astype(np.float64) / s[None, :]


def _cplx_cols(z):
    """complex [K, n] -> real [K, 2n] (re, im interleaved per column)"""
    out = np.empty((z.shape[0], 2 * z.shape[1]))
    out[:, 0::2] = z.real
    out[:, 1::2] = z.imag
    return out


def _from_cols(r):
    return r[:, 0::2] + 1j * r[:, 1::2]


class SplitGrid(Grid):
    def __init__(self, L, nlat, nlon, p, mode):
        super().__init__(L, nlat, nlon, p)
        self.mode = mode
        self.half = nlat // 2
        self._Pext = {}

    def Pext(self, m):
        """Pbar_lm, l = m .. L+1, at the northern latitudes [L - m + 2, half]."""
        if m not in self._Pext:
            self._Pext[m] = legendre_m(m, self.L + 1, self.mu[: self.half], self.sint[: self.half])
        return self._Pext[m]

    def _hAB(self, m):
        l = np.arange(m, self.L + 2, dtype=np.float64)

        def eps(ll):
            return np.where(ll > m, np.sqrt(np.maximum(ll * ll - m * m, 0) / (4.0 * ll * ll - 1.0)), 0.0)
        return -l * eps(l + 1), (l + 1) * eps(l)

    # -- synthesis: per order, coefficient rows (l - m, parity) x columns
    def _synth_rows(self, m, coef):
        """coef: complex [n_rows, ncol] for rows l = m .. (rows of Pext); returns
        F_m at all latitudes, complex [nlat, ncol]."""
        P = self.Pext(m)[: coef.shape[0]]
        parts = []
        for par in (0, 1):
            rows = np.arange(par, coef.shape[0], 2)
            if rows.size == 0:
                parts.append(np.zeros((self.half, coef.shape[1]), dtype=np.complex128))
                continue
            r = mm_split(P[rows].T, _cplx_cols(coef[rows]), self.mode)     # [half, 2 ncol]
            parts.append(_from_cols(r))
        north = parts[0] + parts[1]
        south = parts[0] - parts[1]
        return np.concatenate([north, south[::-1]], axis=0)

    def _to_grid(self, F):
        """F [L+1, nlat] per field -> grid"""
        return self._fourier_to_grid(F)

    def synthesis(self, spec):
        L = self.L
        F = np.zeros((L + 1, self.nlat), dtype=np.complex128)
        for m in range(L + 1):
            s = mode_index(L, m, m)
            F[m] = self._synth_rows(m, spec[s: s + L - m + 1, None])[:, 0]
        return self._to_grid(F)

    def uv_from_psichi(self, psi, chi):
        L, a = self.L, self.p.a
        FU = np.zeros((L + 1, self.nlat), dtype=np.complex128)
        FV = np.zeros((L + 1, self.nlat), dtype=np.complex128)
        for m in range(L + 1):
            s = mode_index(L, m, m)
            n = L - m + 1
            ps = np.zeros(n + 3, dtype=np.complex128)      # psi_{l}, l = m-1 .. L+2 (zero outside m .. L)
            ch = np.zeros(n + 3, dtype=np.complex128)
            ps[1:n + 1] = psi[s: s + n]
            ch[1:n + 1] = chi[s: s + n]
            hA, hB = self._hAB(m)                       # for l = m .. L+1
            hAp = np.concatenate([[0.0], hA])            # hA_{l-1} at row l (index shift)
            hBp = np.concatenate([hB[1:], [0.0, 0.0]])   # hB_{l+1} at row l
            i = np.arange(n + 1)                         # rows l = m .. L+1
            sumH_psi = hAp[i] * ps[i] + hBp[i] * ps[i + 2]
            sumH_chi = hAp[i] * ch[i] + hBp[i] * ch[i + 2]
            cU = (-sumH_psi + 1j * m * ch[i + 1]) / a
            cV = (1j * m * ps[i + 1] + sumH_chi) / a
            F = self._synth_rows(m, np.stack([cU, cV], axis=1))
            FU[m], FV[m] = F[:, 0], F[:, 1]
        return self._to_grid(FU), self._to_grid(FV)

    # -- analysis: per order, folded weighted Fourier data x Pbar rows
    def _anal_rows(self, m, Y, nrows):
        """Y: complex [nlat, ncol] (weights applied); returns sum_j Pbar_l(mu_j) Y_j
        for l = m .. m + nrows - 1, complex [nrows, ncol]."""
        P = self.Pext(m)[:nrows]
        hN = Y[: self.half]
        hS = Y[self.nlat - 1: self.nlat - 1 - self.half: -1]
        out = np.zeros((nrows, Y.shape[1]), dtype=np.complex128)
        for par in (0, 1):
            rows = np.arange(par, nrows, 2)
            if rows.size == 0:
                continue
            fold = hN + hS if par == 0 else hN - hS
            out[rows] = _from_cols(mm_split(P[rows], _cplx_cols(fold), self.mode))
        return out

    def analysis(self, field):
        L = self.L
        F = self._grid_to_fourier(field)
        out = np.zeros(n_modes(L), dtype=np.complex128)
        for m in range(L + 1):
            s = mode_index(L, m, m)
            out[s: s + L - m + 1] = self._anal_rows(m, (self.w * F[m])[:, None], L - m + 1)[:, 0]
        return out

    def div_curl(self, A, B):
        L, a = self.L, self.p.a
        FA = self._grid_to_fourier(A)
        FB = self._grid_to_fourier(B)
        wd = self.w / (a * self.sint ** 2)
        div = np.zeros(n_modes(L), dtype=np.complex128)
        curl = np.zeros(n_modes(L), dtype=np.complex128)
        for m in range(L + 1):
            s = mode_index(L, m, m)
            n = L - m + 1
            # P terms: data m A and m B (the factor i applied after); H terms: rows up to L+1
            Y = np.stack([m * wd * FA[m], m * wd * FB[m], wd * FA[m], wd * FB[m]], axis=1)
            Z = self._anal_rows(m, Y, n + 1)
            hA, hB = self._hAB(m)
            hA, hB = hA[:n], hB[:n]

            def H(col):
                up = Z[1: n + 1, col]
                dn = np.concatenate([[0.0], Z[: n - 1, col]])
                return hA * up + hB * dn
            div[s: s + n] = 1j * Z[:n, 0] - H(3)
            curl[s: s + n] = 1j * Z[:n, 1] + H(2)
        return div, curl
