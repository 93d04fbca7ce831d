// Spherical-harmonic transforms and the non-linear tendency on the device.
//
// Spectral -> grid:  F_m(mu_j) = sum_l f_lm Pbar_lm(mu_j) (Legendre synthesis),
//                    f(lambda_k, mu_j) = Re F_0 + 2 Re sum_{m>=1} F_m e^{i m lambda_k}.
// Grid -> spectral:  F_m(mu_j) = (1/nlon) sum_k f e^{-i m lambda_k},
//                    f_lm = sum_j w_j Pbar_lm(mu_j) F_m(mu_j) (Gauss quadrature).
// Vector fields travel as U = u cos(phi), V = v cos(phi):
//   U_m = (1/a) sum_l [-psi H + i m chi Pbar],  V_m = (1/a) sum_l [i m psi Pbar + chi H]
//   div  = (1/a) sum_j w_j/(1-mu_j^2) [i m A_m Pbar - B_m H]
//   curl = (1/a) sum_j w_j/(1-mu_j^2) [i m B_m Pbar + A_m H],  H = (1-mu^2) dPbar/dmu.
//
// Legendre stage: one lane per northern Gauss latitude, Pbar_lm generated on the
// fly by the three-term recurrence in l (no tables in memory), the southern
// latitude obtained from the parity Pbar_lm(-mu) = (-1)^{l-m} Pbar_lm(mu).  The
// seed Pbar_mm = c_m sin(theta)^m leaves double range near the poles at high m,
// so it is carried as mantissa * 2^e (e <= 0) and renormalised when the
// recurrence has grown back into range.  The analysis sums over latitudes
// through LDS (each lane writes its contributions for a few degrees, threads
// then read them transposed).
//
// Ring stage: one workgroup per latitude circle; the real FFTs of length nlon
// run as complex Stockham FFTs of length nlon/2 (radix 4, 2 and 3) in LDS, with
// the non-linear products formed pointwise between the inverse and forward
// transforms, so grid fields never go to HBM.
#include <type_traits>

#include "internal.h"

namespace rexi {
namespace {

constexpr int WAVE = 64;

// --------------------------------------------------------------- helpers --
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(__builtin_fma(a.x, b.x, -(a.y * b.y)), __builtin_fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 scale2(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// acc += c * p (complex times real)
__device__ __forceinline__ void caxpy(double2& acc, double2 c, double p) {
    acc.x = __builtin_fma(c.x, p, acc.x);
    acc.y = __builtin_fma(c.y, p, acc.y);
}

struct LegArgs {
    const LegCoef* __restrict__ rec;    // [modes]
    const double* __restrict__ aon;     // [L+2] a / (l(l+1))
    const double* __restrict__ noa2;    // [L+2] l(l+1) / a^2
    const double* __restrict__ mu;      // [half]
    const double* __restrict__ sint;    // [half]
    const double* __restrict__ w;       // [half]
    const double* __restrict__ seed_m;  // [L+1][half]
    const int* __restrict__ seed_e;     // [L+1][half]
    int L, nlat, half, modes;
    double a;
};

// Recurrence state of one lane: Pbar_{l-1}, Pbar_l in units of 2^e.
struct Rec {
    double pm, p;
    int e;
};

__device__ __forceinline__ Rec rec_start(const LegArgs& A, int m, int j) {
    Rec r;
    r.pm = 0.0;
    r.p = A.seed_m[static_cast<size_t>(m) * A.half + j];
    r.e = A.seed_e[static_cast<size_t>(m) * A.half + j];
    return r;
}

// Advances to degree l+1; returns Pbar_{l+1} and H_l (both in units of 2^e).
__device__ __forceinline__ void rec_step(const LegCoef& c, double mu, Rec& r, double& pn, double& h) {
    pn = __builtin_fma(c.A * mu, r.p, -(c.B * r.pm));
    h = __builtin_fma(c.hA, pn, c.hB * r.pm);
}

constexpr double kBig = 0x1p400;

// ================================================== Legendre synthesis ==
// KIND 0: one scalar field per block row (blockIdx.y = field), P pass only.
// KIND 1: the non-linear set: h, zeta (P pass) and U, V from psi, chi
//         (psi = -a^2 zeta / N, chi = -a^2 delta / N) -> 4 output fields.
struct SynArgs {
    LegArgs g;
    const double2* __restrict__ spec;   // KIND 0: [nf][modes]; KIND 1: state [3][modes]
    double2* __restrict__ four;         // [nfo][L+1][nlat]
};

// Per-degree data of one order m staged in LDS (double2 slots per degree):
// KIND 0: {A, B}, coefficient;  KIND 1: {A, B}, {hA, hB}, h, zeta, delta, {a/N, m a/N}.
template <int KIND>
struct SynStage {
    static constexpr int SLOTS = KIND == 0 ? 2 : 6;
};

template <int KIND>
__global__ __launch_bounds__(WAVE) void legendre_synth_kernel(SynArgs S) {
    extern __shared__ __align__(16) double2 stg[];
    constexpr int SL = SynStage<KIND>::SLOTS;
    const LegArgs& A = S.g;
    const int m = blockIdx.x;
    const int Lm = A.L - m + 1;
    const int jt = blockIdx.z * WAVE + threadIdx.x;
    const bool valid = jt < A.half;
    const int j = valid ? jt : A.half - 1;
    const double mu = A.mu[j];
    const int base = m * (2 * A.L + 3 - m) / 2;
    const double dm = static_cast<double>(m);
    {
        const double2* sp0 = S.spec + static_cast<size_t>(KIND == 0 ? blockIdx.y : 0) * A.modes + base;
        for (int i = threadIdx.x; i < Lm; i += WAVE) {
            const LegCoef c = A.rec[base + i];
            stg[i * SL + 0] = make_double2(c.A, c.B);
            if constexpr (KIND == 0) {
                stg[i * SL + 1] = sp0[i];
            } else {
                const double aon = A.aon[m + i];
                stg[i * SL + 1] = make_double2(c.hA, c.hB);
                stg[i * SL + 2] = sp0[i];
                stg[i * SL + 3] = sp0[i + A.modes];
                stg[i * SL + 4] = sp0[i + 2 * A.modes];
                stg[i * SL + 5] = make_double2(aon, dm * aon);
            }
        }
    }
    __syncthreads();
    constexpr int NACC = KIND == 0 ? 1 : 4;
    double2 E[NACC], O[NACC];
#pragma unroll
    for (int f = 0; f < NACC; ++f) E[f] = O[f] = make_double2(0.0, 0.0);
    Rec r = rec_start(A, m, j);

    auto degree = [&](int i, auto odd) {
        constexpr bool ODD = decltype(odd)::value;
        const double2* st = stg + i * SL;
        const double2 ab = st[0];
        const double pn = __builtin_fma(ab.x * mu, r.p, -(ab.y * r.pm));
        const double p = r.p;
        if constexpr (KIND == 0) {
            if (ODD) caxpy(O[0], st[1], p); else caxpy(E[0], st[1], p);
        } else {
            const double2 hab = st[1];
            const double h = __builtin_fma(hab.x, pn, hab.y * r.pm);
            const double2 ch = st[2], cz = st[3], cd = st[4], fac = st[5];
            const double hp = fac.x * h;         // (a/N) H
            const double pp = fac.y * p;         // (m a/N) Pbar
            if (ODD) { caxpy(O[0], ch, p); caxpy(O[1], cz, p); }
            else     { caxpy(E[0], ch, p); caxpy(E[1], cz, p); }
            // U: i m chi Pbar / a = -i delta P'  (parity of P);  -psi H / a = zeta H'  (parity of H)
            // V: i m psi Pbar / a = -i zeta P'   (parity of P);   chi H / a = -delta H' (parity of H)
            const double2 up = make_double2(cd.y * pp, -cd.x * pp);
            const double2 vp = make_double2(cz.y * pp, -cz.x * pp);
            const double2 uh = make_double2(cz.x * hp, cz.y * hp);
            const double2 vh = make_double2(-cd.x * hp, -cd.y * hp);
            if (ODD) {
                O[2] = cadd(O[2], up); E[2] = cadd(E[2], uh);
                O[3] = cadd(O[3], vp); E[3] = cadd(E[3], vh);
            } else {
                E[2] = cadd(E[2], up); O[2] = cadd(O[2], uh);
                E[3] = cadd(E[3], vp); O[3] = cadd(O[3], vh);
            }
        }
        r.pm = r.p;
        r.p = pn;
    };

    int i = 0;
    for (; i + 3 < Lm; i += 4) {
        degree(i, std::integral_constant<bool, false>{});
        degree(i + 1, std::integral_constant<bool, true>{});
        degree(i + 2, std::integral_constant<bool, false>{});
        degree(i + 3, std::integral_constant<bool, true>{});
        if (r.e < 0 && fabs(r.p) > kBig) {
            const int sh = min(400, -r.e);
            r.p = ldexp(r.p, -sh);
            r.pm = ldexp(r.pm, -sh);
            r.e += sh;
#pragma unroll
            for (int f = 0; f < NACC; ++f) {
                E[f] = make_double2(ldexp(E[f].x, -sh), ldexp(E[f].y, -sh));
                O[f] = make_double2(ldexp(O[f].x, -sh), ldexp(O[f].y, -sh));
            }
        }
    }
    for (; i < Lm; ++i) {
        if ((i & 1) == 0) degree(i, std::integral_constant<bool, false>{});
        else degree(i, std::integral_constant<bool, true>{});
    }
    if (!valid) return;
    for (int f = 0; f < NACC; ++f) {
        const size_t row = (static_cast<size_t>(KIND == 0 ? blockIdx.y : f) * (A.L + 1) + m) * A.nlat;
        const double2 n = make_double2(ldexp(E[f].x + O[f].x, r.e), ldexp(E[f].y + O[f].y, r.e));
        const double2 s = make_double2(ldexp(E[f].x - O[f].x, r.e), ldexp(E[f].y - O[f].y, r.e));
        S.four[row + jt] = n;
        S.four[row + (A.nlat - 1 - jt)] = s;
    }
}

// ==================================================== Legendre analysis ==
// KIND 0: one scalar field per block row: f_lm = sum_j w_j Pbar_lm F_m.
// KIND 1: the non-linear tendency from the Fourier coefficients of
//         hU, hV, zU, zV, KE (fields 0..4):
//   N_h = -div(hU, hV), N_zeta = -div(zU, zV), N_delta = curl(zU, zV) + l(l+1)/a^2 KE_lm,
//   followed by the Runge-Kutta update out = U0 + c0 N (+ c1 Nprev), and Nsave = N.
struct AnaArgs {
    LegArgs g;
    const double2* __restrict__ four;   // [nf][L+1][nlat]
    double2* __restrict__ spec;         // KIND 0: [nf][modes]
    // KIND 1 epilogue
    const double2* __restrict__ U0;     // [3][modes]
    const double2* __restrict__ Nprev;  // [3][modes] or nullptr
    double2* __restrict__ Nsave;        // [3][modes] or nullptr
    double2* __restrict__ out;          // [3][modes]
    double c0, c1;
};

template <int KIND>
struct AnaTraits {
    static constexpr int NC = KIND == 0 ? 2 : 6;       // doubles contributed per (l, j)
    static constexpr int NIN = KIND == 0 ? 1 : 5;      // complex input fields
};

// Folded, weighted inputs of one lane (units of 2^e): for each field,
// S = F(mu) + F(-mu) and D = F(mu) - F(-mu).
template <int KIND>
__device__ __forceinline__ void load_folded(const AnaArgs& P, int m, int j, int e, double2* Sv, double2* Dv) {
    const LegArgs& A = P.g;
    constexpr int NIN = AnaTraits<KIND>::NIN;
    const double sc = ldexp(1.0, e);
    const double wj = A.w[j];
    const double wdiv = wj / (A.a * A.sint[j] * A.sint[j]);
#pragma unroll
    for (int f = 0; f < NIN; ++f) {
        const int fld = KIND == 0 ? blockIdx.y : f;
        const size_t row = (static_cast<size_t>(fld) * (A.L + 1) + m) * A.nlat;
        const double2 n = P.four[row + j];
        const double2 s = P.four[row + (A.nlat - 1 - j)];
        const double wt = (KIND == 0 || f == 4) ? wj : wdiv;
        Sv[f] = scale2(cadd(n, s), wt * sc);
        Dv[f] = scale2(csub(n, s), wt * sc);
    }
}

constexpr int RED_STRIDE = 72;   // doubles per staged output row (64 lanes + pad: 4-cycle LDS reads)

template <int KIND, int D>
__global__ __launch_bounds__(512) void legendre_anal_kernel(AnaArgs P) {
    extern __shared__ __align__(16) double smem[];
    constexpr int NC = AnaTraits<KIND>::NC;
    constexpr int NIN = AnaTraits<KIND>::NIN;
    constexpr int NO = D * NC;                           // outputs per chunk
    constexpr int SL = KIND == 0 ? 1 : 3;                // staged double2 per degree
    const LegArgs& A = P.g;
    const int m = blockIdx.x;
    const int Lm = A.L - m + 1;
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1), wv = tid / WAVE;
    const int nthreads = blockDim.x;
    const int nw = nthreads / WAVE;
    const bool valid = tid < A.half;
    const int j = valid ? tid : A.half - 1;
    const double mu = A.mu[j];
    const int base = m * (2 * A.L + 3 - m) / 2;
    double* red = smem;                                                   // [nw][NO][RED_STRIDE]
    double2* stg = reinterpret_cast<double2*>(smem + static_cast<size_t>(nw) * NO * RED_STRIDE);
    for (int i = tid; i < Lm; i += nthreads) {
        const LegCoef c = A.rec[base + i];
        stg[i * SL] = make_double2(c.A, c.B);
        if constexpr (KIND == 1) {
            stg[i * SL + 1] = make_double2(c.hA, c.hB);
            stg[i * SL + 2] = make_double2(A.noa2[m + i], 0.0);
        }
    }
    Rec r = rec_start(A, m, j);
    double2 Sv[NIN], Dv[NIN];
    load_folded<KIND>(P, m, j, r.e, Sv, Dv);
    if (!valid) {
#pragma unroll
        for (int f = 0; f < NIN; ++f) Sv[f] = Dv[f] = make_double2(0.0, 0.0);
    }
    const double dm = static_cast<double>(m);
    // reduction: thread t -> output o = t / G, part g = t % G
    int G = 1;
    while (G * 2 * NO <= nthreads && G < 16) G *= 2;
    const int o_red = tid / G, g_red = tid % G;
    const int nvals = nthreads;                          // values per output
    double* myred = red + static_cast<size_t>(wv) * NO * RED_STRIDE;
    __syncthreads();

    for (int i0 = 0; i0 < Lm; i0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int i = i0 + d;
            double c[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) c[k] = 0.0;
            if (i < Lm) {
                const double2* st = stg + i * SL;
                const double2 ab = st[0];
                const double pn = __builtin_fma(ab.x * mu, r.p, -(ab.y * r.pm));
                const double p = r.p;
                const bool odd = d & 1;                  // l - m = i0 + d with i0 a multiple of D
                if constexpr (KIND == 0) {
                    const double2 x = odd ? Dv[0] : Sv[0];
                    c[0] = x.x * p;
                    c[1] = x.y * p;
                } else {
                    const double2 hab = st[1];
                    const double h = __builtin_fma(hab.x, pn, hab.y * r.pm);
                    // P terms take the fold of P's parity, H terms the opposite one
                    const double2 hU = odd ? Dv[0] : Sv[0], zU = odd ? Dv[2] : Sv[2];
                    const double2 zV = odd ? Dv[3] : Sv[3], ke = odd ? Dv[4] : Sv[4];
                    const double2 hVh = odd ? Sv[1] : Dv[1], zVh = odd ? Sv[3] : Dv[3];
                    const double2 zUh = odd ? Sv[2] : Dv[2];
                    const double pm2 = dm * p;                 // m Pbar
                    const double pk = st[2].x * p;             // l(l+1)/a^2 Pbar
                    // N_h = -(i m hU P - hV H)
                    c[0] = __builtin_fma(hU.y, pm2, hVh.x * h);
                    c[1] = __builtin_fma(-hU.x, pm2, hVh.y * h);
                    // N_zeta = -(i m zU P - zV H)
                    c[2] = __builtin_fma(zU.y, pm2, zVh.x * h);
                    c[3] = __builtin_fma(-zU.x, pm2, zVh.y * h);
                    // N_delta = i m zV P + zU H + l(l+1)/a^2 KE P
                    c[4] = __builtin_fma(-zV.y, pm2, __builtin_fma(zUh.x, h, ke.x * pk));
                    c[5] = __builtin_fma(zV.x, pm2, __builtin_fma(zUh.y, h, ke.y * pk));
                }
                r.pm = r.p;
                r.p = pn;
            }
#pragma unroll
            for (int k = 0; k < NC; ++k) myred[(d * NC + k) * RED_STRIDE + lane] = c[k];
        }
        // renormalise lanes whose recurrence has grown back into range
        if (r.e < 0 && fabs(r.p) > kBig) {
            const int sh = min(400, -r.e);
            r.p = ldexp(r.p, -sh);
            r.pm = ldexp(r.pm, -sh);
            r.e += sh;
            load_folded<KIND>(P, m, j, r.e, Sv, Dv);
            if (!valid) {
#pragma unroll
                for (int f = 0; f < NIN; ++f) Sv[f] = Dv[f] = make_double2(0.0, 0.0);
            }
        }
        __syncthreads();
        if (o_red < NO) {
            double s = 0.0;
            for (int v = g_red; v < nvals; v += G) {
                const int w2 = v / WAVE, ln = v % WAVE;
                s += red[(static_cast<size_t>(w2) * NO + o_red) * RED_STRIDE + ln];
            }
            for (int msk = 1; msk < G; msk <<= 1) s += __shfl_xor(s, msk, G);
            const int d = o_red / NC, k = o_red % NC;
            const int i = i0 + d;
            if (g_red == 0 && i < Lm) {
                const size_t idx = static_cast<size_t>(base) + i;
                if constexpr (KIND == 0) {
                    double* dst = reinterpret_cast<double*>(P.spec + static_cast<size_t>(blockIdx.y) * A.modes + idx);
                    dst[k] = s;
                } else {
                    const int f = k >> 1, part = k & 1;
                    const size_t e2 = (static_cast<size_t>(f) * A.modes + idx) * 2 + part;
                    double v = reinterpret_cast<const double*>(P.U0)[e2] + P.c0 * s;
                    if (P.Nprev) v += P.c1 * reinterpret_cast<const double*>(P.Nprev)[e2];
                    if (P.Nsave) reinterpret_cast<double*>(P.Nsave)[e2] = s;
                    reinterpret_cast<double*>(P.out)[e2] = v;
                }
            }
        }
        __syncthreads();
    }
}

// ============================================================ ring FFTs ==
struct RingArgs {
    const double* __restrict__ tw;     // [M] complex e^{-2 pi i k / M}
    const double* __restrict__ twr;    // [M] complex e^{-2 pi i k / nlon}
    const double* __restrict__ sint;   // [half]
    const int* __restrict__ radix;     // [npass]
    int npass, L, nlat, nlon, half;
    const double2* __restrict__ fin;   // [nf_in][L+1][nlat]
    double2* __restrict__ fout;        // [nf_out][L+1][nlat]
    const double* __restrict__ gin;    // grid input  [nf][nlat][nlon] (forward-only mode)
    double* __restrict__ gout;         // grid output [nf][nlat][nlon] (inverse-only mode)
    int nf;
};

// One Stockham pass of radix R over M complex points: src -> dst.
template <int R>
__device__ __forceinline__ void fft_pass(const double2* src, double2* dst, int M, int Ns, const double* tw,
                                         bool inverse) {
    const int nb = M / R;
    const int twstep = M / (Ns * R);
    for (int jb = threadIdx.x; jb < nb; jb += blockDim.x) {
        const int k = jb % Ns;
        double2 v[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            v[t] = src[jb + t * nb];
            if (t > 0) {
                const int ti = (t * k * twstep) % M;
                double2 wv = make_double2(tw[2 * ti], tw[2 * ti + 1]);
                if (inverse) wv.y = -wv.y;
                v[t] = cmul(v[t], wv);
            }
        }
        if constexpr (R == 2) {
            const double2 a = v[0], b = v[1];
            v[0] = cadd(a, b);
            v[1] = csub(a, b);
        } else if constexpr (R == 4) {
            const double2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
            const double2 b0 = cadd(v[1], v[3]), b1 = csub(v[1], v[3]);
            // multiply b1 by -i (forward) or +i (inverse)
            const double2 b1r = inverse ? make_double2(-b1.y, b1.x) : make_double2(b1.y, -b1.x);
            v[0] = cadd(a0, b0);
            v[2] = csub(a0, b0);
            v[1] = cadd(a1, b1r);
            v[3] = csub(a1, b1r);
        } else {  // R == 3
            const double c = -0.5;
            const double s = inverse ? 0.86602540378443864676 : -0.86602540378443864676;
            const double2 t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
            const double2 m1 = make_double2(__builtin_fma(c, t1.x, v[0].x), __builtin_fma(c, t1.y, v[0].y));
            const double2 m2 = make_double2(-s * t2.y, s * t2.x);   // i s t2
            v[0] = cadd(v[0], t1);
            v[1] = cadd(m1, m2);
            v[2] = csub(m1, m2);
        }
        const int base = (jb / Ns) * Ns * R + k;
#pragma unroll
        for (int t = 0; t < R; ++t) dst[base + t * Ns] = v[t];
    }
}

// Complex FFT of length M in LDS; returns the buffer holding the result.
__device__ double2* fft_lds(double2* a, double2* scratch, const RingArgs& A, bool inverse) {
    const int M = A.nlon / 2;
    int Ns = 1;
    double2* src = a;
    double2* dst = scratch;
    for (int p = 0; p < A.npass; ++p) {
        const int R = A.radix[p];
        if (R == 4) fft_pass<4>(src, dst, M, Ns, A.tw, inverse);
        else if (R == 2) fft_pass<2>(src, dst, M, Ns, A.tw, inverse);
        else fft_pass<3>(src, dst, M, Ns, A.tw, inverse);
        __syncthreads();
        Ns *= R;
        double2* t = src;
        src = dst;
        dst = t;
    }
    return src;
}

// Loads F_m (m <= L) of one latitude and builds the half-length spectrum Z of
// the inverse real FFT:  Z_k = (X_k + conj X_{M-k}) + i e^{2 pi i k/nlon} (X_k - conj X_{M-k}),
// X_0 taken real, X_k = 0 for k > L.
__device__ void load_inverse(const double2* fin_row, int nlat_stride, double2* z, const RingArgs& A) {
    const int M = A.nlon / 2;
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
        double2 xk = make_double2(0.0, 0.0), xr = make_double2(0.0, 0.0);
        if (k <= A.L) xk = fin_row[static_cast<size_t>(k) * nlat_stride];
        const int kr = M - k;                      // 1..M
        if (kr <= A.L && kr < M) xr = fin_row[static_cast<size_t>(kr) * nlat_stride];
        if (k == 0) xk.y = 0.0;
        const double2 xrc = conj2(xr);
        const double2 s = cadd(xk, xrc);
        const double2 d = csub(xk, xrc);
        const double2 wk = make_double2(A.twr[2 * k], -A.twr[2 * k + 1]);  // e^{+2 pi i k / nlon}
        const double2 t = cmul(wk, d);
        z[k] = make_double2(s.x - t.y, s.y + t.x);                             // s + i t
    }
}

// From Z = FFT_M(x viewed as complex), the coefficients F_m = X_m / nlon, m <= L:
// X_m = (Z_m + conj Z_{M-m})/2 - (i/2) e^{-2 pi i m/nlon} (Z_m - conj Z_{M-m}).
__device__ void store_forward(const double2* Z, double2* fout_row, int nlat_stride, const RingArgs& A) {
    const int M = A.nlon / 2;
    const double inv = 1.0 / static_cast<double>(A.nlon);
    for (int k = threadIdx.x; k <= A.L; k += blockDim.x) {
        const double2 zk = Z[k];
        const double2 zr = conj2(Z[k == 0 ? 0 : M - k]);
        const double2 s = cadd(zk, zr);
        const double2 d = csub(zk, zr);
        const double2 wk = make_double2(A.twr[2 * k], A.twr[2 * k + 1]);   // e^{-2 pi i k / nlon}
        const double2 t = cmul(wk, d);
        // X = s/2 - i t/2
        const double2 X = make_double2(0.5 * (s.x + t.y), 0.5 * (s.y - t.x));
        fout_row[static_cast<size_t>(k) * nlat_stride] = scale2(X, inv);
    }
}

// MODE 0: inverse only (Fourier -> grid), nf fields.
// MODE 1: forward only (grid -> Fourier), nf fields.
// MODE 2: non-linear products: inverse of h, zeta, U, V; forward of hU, hV, zU, zV, KE.
template <int MODE>
__global__ __launch_bounds__(256) void ring_kernel(RingArgs A) {
    extern __shared__ __align__(16) double2 lds[];
    const int M = A.nlon / 2;
    const int j = blockIdx.x;
    const size_t fstride = static_cast<size_t>(A.L + 1) * A.nlat;
    double2* scratch = lds;
    if constexpr (MODE == 0) {
        double2* a = lds + M;
        for (int f = 0; f < A.nf; ++f) {
            load_inverse(A.fin + f * fstride + j, A.nlat, a, A);
            __syncthreads();
            double2* res = fft_lds(a, scratch, A, true);
            double2* g = reinterpret_cast<double2*>(A.gout + (static_cast<size_t>(f) * A.nlat + j) * A.nlon);
            for (int k = threadIdx.x; k < M; k += blockDim.x) g[k] = res[k];
            __syncthreads();
        }
    } else if constexpr (MODE == 1) {
        double2* a = lds + M;
        for (int f = 0; f < A.nf; ++f) {
            const double2* g = reinterpret_cast<const double2*>(A.gin + (static_cast<size_t>(f) * A.nlat + j) * A.nlon);
            for (int k = threadIdx.x; k < M; k += blockDim.x) a[k] = g[k];
            __syncthreads();
            double2* res = fft_lds(a, scratch, A, false);
            store_forward(res, A.fout + f * fstride + j, A.nlat, A);
            __syncthreads();
        }
    } else {
        // arrays: 0 h, 1 zeta, 2 U, 3 V, 4 KE, 5 hV; scratch
        double2* arr[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) arr[i] = lds + (i + 1) * M;
        double2* grid[4];
        for (int f = 0; f < 4; ++f) {
            load_inverse(A.fin + f * fstride + j, A.nlat, arr[f], A);
            __syncthreads();
            double2* res = fft_lds(arr[f], scratch, A, true);
            if (res != arr[f]) {
                for (int k = threadIdx.x; k < M; k += blockDim.x) arr[f][k] = res[k];
                __syncthreads();
            }
            grid[f] = arr[f];
        }
        const int jn = j < A.half ? j : A.nlat - 1 - j;
        const double s = A.sint[jn];
        const double kefac = 0.5 / (s * s);
        double* h = reinterpret_cast<double*>(arr[0]);
        double* z = reinterpret_cast<double*>(arr[1]);
        const double* U = reinterpret_cast<const double*>(arr[2]);
        double* V = reinterpret_cast<double*>(arr[3]);
        double* ke = reinterpret_cast<double*>(arr[4]);
        double* hv = reinterpret_cast<double*>(arr[5]);
        for (int k = threadIdx.x; k < A.nlon; k += blockDim.x) {
            const double u = U[k], v = V[k], hh = h[k], zz = z[k];
            ke[k] = __builtin_fma(u, u, v * v) * kefac;
            hv[k] = hh * v;
            V[k] = zz * v;          // zeta V
            h[k] = hh * u;          // h U
            z[k] = zz * u;          // zeta U
        }
        __syncthreads();
        // forward transforms: hU (arr0) -> field 0, hV (arr5) -> 1, zU (arr1) -> 2, zV (arr3) -> 3, KE (arr4) -> 4
        const int src[5] = {0, 5, 1, 3, 4};
        for (int f = 0; f < 5; ++f) {
            double2* res = fft_lds(arr[src[f]], scratch, A, false);
            store_forward(res, A.fout + f * fstride + j, A.nlat, A);
            __syncthreads();
        }
        (void)grid;
    }
}

}  // namespace

// ------------------------------------------------------------ launchers --
static LegArgs leg_args(const swe_ctx* ctx) {
    LegArgs g;
    g.rec = ctx->d_rec;
    g.aon = ctx->d_aon;
    g.noa2 = ctx->d_noa2;
    g.mu = ctx->d_mu;
    g.sint = ctx->d_sint;
    g.w = ctx->d_w;
    g.seed_m = ctx->d_seed_m;
    g.seed_e = ctx->d_seed_e;
    g.L = ctx->L;
    g.nlat = ctx->nlat;
    g.half = ctx->nlat / 2;
    g.modes = ctx->modes;
    g.a = ctx->a;
    return g;
}

static RingArgs ring_args(const swe_ctx* ctx) {
    RingArgs r{};
    r.tw = ctx->d_tw;
    r.twr = ctx->d_twr;
    r.sint = ctx->d_sint;
    r.radix = ctx->d_radix;
    r.npass = ctx->npass;
    r.L = ctx->L;
    r.nlat = ctx->nlat;
    r.nlon = ctx->nlon;
    r.half = ctx->nlat / 2;
    return r;
}

// LDS of the analysis kernel: staged reduction rows + staged per-degree coefficients.
static size_t anal_lds_bytes(const swe_ctx* ctx, int kind) {
    const int nw = (ctx->nlat / 2 + WAVE - 1) / WAVE;
    const int D = kind == 0 ? 8 : (nw <= 3 ? 4 : 2);
    const int NC = kind == 0 ? AnaTraits<0>::NC : AnaTraits<1>::NC;
    const int SL = kind == 0 ? 1 : 3;
    return sizeof(double) * nw * D * NC * RED_STRIDE + sizeof(double2) * SL * (ctx->L + 1);
}

static int ring_lds_bytes(const swe_ctx* ctx, int mode) {
    const int M = ctx->nlon / 2;
    const int arrays = mode == 2 ? 7 : 2;
    return arrays * M * static_cast<int>(sizeof(double2));
}

static int allow_lds(const void* fn, size_t bytes, const char* what) {
    if (bytes <= 64 * 1024) return REXI_OK;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(REXI_ENOTSUP, std::string("swe_create: ") + what + " of this grid needs more LDS than available");
    }
    return REXI_OK;
}

int sht_configure_kernels(swe_ctx* ctx) {
    int rc;
    if ((rc = allow_lds(reinterpret_cast<const void*>(&ring_kernel<2>), ring_lds_bytes(ctx, 2),
                        "the longitude FFT")) != REXI_OK)
        return rc;
    if ((rc = allow_lds(reinterpret_cast<const void*>(&legendre_anal_kernel<1, 2>), anal_lds_bytes(ctx, 1),
                        "the Legendre analysis")) != REXI_OK)
        return rc;
    if ((rc = allow_lds(reinterpret_cast<const void*>(&legendre_anal_kernel<1, 4>), anal_lds_bytes(ctx, 1),
                        "the Legendre analysis")) != REXI_OK)
        return rc;
    return REXI_OK;
}

int launch_legendre_synth(swe_ctx* ctx, int kind, const double* spec, double* four, int nf, hipStream_t stream) {
    SynArgs S;
    S.g = leg_args(ctx);
    S.spec = reinterpret_cast<const double2*>(spec);
    S.four = reinterpret_cast<double2*>(four);
    const int tiles = (ctx->nlat / 2 + WAVE - 1) / WAVE;
    const int slot = prof_begin(ctx, REXI_KERNEL_LEG_SYNTH, stream);
    if (kind == 0) {
        const size_t lds = sizeof(double2) * SynStage<0>::SLOTS * (ctx->L + 1);
        hipLaunchKernelGGL(legendre_synth_kernel<0>, dim3(ctx->L + 1, nf, tiles), dim3(WAVE), lds, stream, S);
    } else {
        const size_t lds = sizeof(double2) * SynStage<1>::SLOTS * (ctx->L + 1);
        hipLaunchKernelGGL(legendre_synth_kernel<1>, dim3(ctx->L + 1, 1, tiles), dim3(WAVE), lds, stream, S);
    }
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_LEG_SYNTH, slot, stream);
    return REXI_OK;
}

int launch_legendre_anal(swe_ctx* ctx, int kind, const double* four, double* spec, int nf, const double* U0,
                         const double* Nprev, double* Nsave, double* out, double c0, double c1,
                         hipStream_t stream) {
    AnaArgs P;
    P.g = leg_args(ctx);
    P.four = reinterpret_cast<const double2*>(four);
    P.spec = reinterpret_cast<double2*>(spec);
    P.U0 = reinterpret_cast<const double2*>(U0);
    P.Nprev = reinterpret_cast<const double2*>(Nprev);
    P.Nsave = reinterpret_cast<double2*>(Nsave);
    P.out = reinterpret_cast<double2*>(out);
    P.c0 = c0;
    P.c1 = c1;
    const int half = ctx->nlat / 2;
    const int nw = (half + WAVE - 1) / WAVE;
    const int threads = nw * WAVE;
    if (threads > 512) return fail(REXI_ENOTSUP, "Legendre analysis: more than 512 northern latitudes");
    const int slot = prof_begin(ctx, REXI_KERNEL_LEG_ANAL, stream);
    if (kind == 0) {
        const size_t lds = anal_lds_bytes(ctx, 0);
        hipLaunchKernelGGL((legendre_anal_kernel<0, 8>), dim3(ctx->L + 1, nf), dim3(threads), lds, stream, P);
    } else if (nw <= 3) {
        const size_t lds = anal_lds_bytes(ctx, 1);
        hipLaunchKernelGGL((legendre_anal_kernel<1, 4>), dim3(ctx->L + 1, 1), dim3(threads), lds, stream, P);
    } else {
        const size_t lds = anal_lds_bytes(ctx, 1);
        hipLaunchKernelGGL((legendre_anal_kernel<1, 2>), dim3(ctx->L + 1, 1), dim3(threads), lds, stream, P);
    }
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_LEG_ANAL, slot, stream);
    return REXI_OK;
}

int launch_ring(swe_ctx* ctx, int mode, const double* fin, double* fout, const double* gin, double* gout, int nf,
                hipStream_t stream) {
    RingArgs R = ring_args(ctx);
    R.fin = reinterpret_cast<const double2*>(fin);
    R.fout = reinterpret_cast<double2*>(fout);
    R.gin = gin;
    R.gout = gout;
    R.nf = nf;
    const size_t lds = static_cast<size_t>(ring_lds_bytes(ctx, mode));
    const int slot = prof_begin(ctx, REXI_KERNEL_RING, stream);
    if (mode == 0) hipLaunchKernelGGL(ring_kernel<0>, dim3(ctx->nlat), dim3(256), lds, stream, R);
    else if (mode == 1) hipLaunchKernelGGL(ring_kernel<1>, dim3(ctx->nlat), dim3(256), lds, stream, R);
    else hipLaunchKernelGGL(ring_kernel<2>, dim3(ctx->nlat), dim3(256), lds, stream, R);
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_RING, slot, stream);
    return REXI_OK;
}

}  // namespace rexi
