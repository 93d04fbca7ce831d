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
// Ring stage: one workgroup per latitude circle; it sums the synthesis partials
// of each order into the ring's Fourier coefficients, the real FFTs of length
// nlon run as complex Stockham FFTs of length nlon/2 (radix 4, 2 and 3) in LDS,
// and the non-linear products are formed pointwise between the inverse and
// forward transforms, so grid fields never go to HBM.  Fourier coefficients in
// HBM are order-major ([field][m][latitude]): the Legendre kernels, whose lanes
// are latitudes, read and write them contiguously.
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
    const int* __restrict__ seg_m;      // [nseg]
    const int* __restrict__ seg_i0;     // [nseg]
    const int* __restrict__ seg_n;      // [nseg]
    const double* __restrict__ seed_pm; // [nseg][half]
    const double* __restrict__ seed_p;  // [nseg][half]
    const int* __restrict__ seed_e;     // [nseg][half]
    int L, nlat, half, modes, nseg;
    double a;
};

// Recurrence state of one latitude: Pbar_{l-1}, Pbar_l in units of 2^e.
struct Rec {
    double pm, p;
    int e;
};

__device__ __forceinline__ Rec rec_start(const LegArgs& A, int gs, int j) {
    const size_t k = static_cast<size_t>(gs) * A.half + j;
    Rec r;
    r.pm = A.seed_pm[k];
    r.p = A.seed_p[k];
    r.e = A.seed_e[k];
    return r;
}

constexpr double kBig = 0x1p400;

// Renormalises a recurrence that has grown back into double range; returns the shift.
__device__ __forceinline__ int rec_renorm(Rec& r) {
    if (r.e < 0 && fabs(r.p) > kBig) {
        const int sh = min(400, -r.e);
        r.p = ldexp(r.p, -sh);
        r.pm = ldexp(r.pm, -sh);
        r.e += sh;
        return sh;
    }
    return 0;
}

// ================================================== Legendre synthesis ==
// One wave per (degree segment, latitude tile); each lane carries NJ northern
// latitudes (independent recurrences: instruction-level parallelism).  Every
// segment writes a partial Fourier coefficient; the ring kernel adds the
// partials of an order in segment order.
// KIND 0: one scalar field per block row (blockIdx.y = field), P pass only.
// KIND 1: the non-linear set: h, zeta (P pass) and U, V from psi, chi
//         (psi = -a^2 zeta / N, chi = -a^2 delta / N) -> 4 output fields.
struct SynArgs {
    LegArgs g;
    const double2* __restrict__ spec;   // KIND 0: [nf][modes]; KIND 1: state [3][modes]
    double2* __restrict__ part;         // [nfo][nseg][nlat]
};

// Per-degree data staged in LDS (double2 slots per degree):
// KIND 0: {A, B}, coefficient;  KIND 1: {A, B}, {hA, hB}, h, zeta, delta, {a/N, m a/N}.
template <int KIND>
struct SynStage {
    static constexpr int SLOTS = KIND == 0 ? 2 : 6;
};

template <int KIND, int NJ>
__global__ __launch_bounds__(WAVE) void legendre_synth_kernel(SynArgs S) {
    __shared__ double2 stg[64 * SynStage<KIND>::SLOTS];
    constexpr int SL = SynStage<KIND>::SLOTS;
    constexpr int NACC = KIND == 0 ? 1 : 4;
    const LegArgs& A = S.g;
    const int gs = blockIdx.x;
    const int m = A.seg_m[gs], i0 = A.seg_i0[gs], n = A.seg_n[gs];
    const int base = m * (2 * A.L + 3 - m) / 2;
    const double dm = static_cast<double>(m);
    {
        const double2* sp0 = S.spec + static_cast<size_t>(KIND == 0 ? blockIdx.y : 0) * A.modes + base;
        for (int d = threadIdx.x; d < n; d += WAVE) {
            const int i = i0 + d;
            const LegCoef c = A.rec[base + i];
            stg[d * SL + 0] = make_double2(c.A, c.B);
            if constexpr (KIND == 0) {
                stg[d * SL + 1] = sp0[i];
            } else {
                const double aon = A.aon[m + i];
                stg[d * SL + 1] = make_double2(c.hA, c.hB);
                stg[d * SL + 2] = sp0[i];
                stg[d * SL + 3] = sp0[i + A.modes];
                stg[d * SL + 4] = sp0[i + 2 * A.modes];
                stg[d * SL + 5] = make_double2(aon, dm * aon);
            }
        }
    }
    double mu[NJ];
    int jq[NJ];
    Rec r[NJ];
    double2 E[NJ][NACC], O[NJ][NACC];
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
        jq[q] = (blockIdx.z * NJ + q) * WAVE + threadIdx.x;
        const int j = jq[q] < A.half ? jq[q] : A.half - 1;
        mu[q] = A.mu[j];
        r[q] = rec_start(A, gs, j);
#pragma unroll
        for (int f = 0; f < NACC; ++f) E[q][f] = O[q][f] = make_double2(0.0, 0.0);
    }
    __syncthreads();

    auto degree = [&](int d, auto odd) {
        constexpr bool ODD = decltype(odd)::value;
        const double2* st = stg + d * SL;
        const double2 ab = st[0];
        if constexpr (KIND == 0) {
            const double2 c = st[1];
#pragma unroll
            for (int q = 0; q < NJ; ++q) {
                const double pn = __builtin_fma(ab.x * mu[q], r[q].p, -(ab.y * r[q].pm));
                const double p = r[q].p;
                if (ODD) caxpy(O[q][0], c, p); else caxpy(E[q][0], c, p);
                r[q].pm = p;
                r[q].p = pn;
            }
        } else {
            const double2 hab = st[1], ch = st[2], cz = st[3], cd = st[4], fac = st[5];
#pragma unroll
            for (int q = 0; q < NJ; ++q) {
                const double pn = __builtin_fma(ab.x * mu[q], r[q].p, -(ab.y * r[q].pm));
                const double p = r[q].p;
                const double h = __builtin_fma(hab.x, pn, hab.y * r[q].pm);
                const double hp = fac.x * h;         // (a/N) H
                const double pp = fac.y * p;         // (m a/N) Pbar
                double2* Pp = ODD ? O[q] : E[q];     // accumulators with the parity of Pbar
                double2* Hp = ODD ? E[q] : O[q];     // accumulators with the parity of H
                caxpy(Pp[0], ch, p);
                caxpy(Pp[1], cz, p);
                // U: i m chi Pbar / a = -i delta P' (P parity); -psi H / a = zeta H' (H parity)
                Pp[2].x = __builtin_fma(cd.y, pp, Pp[2].x);
                Pp[2].y = __builtin_fma(-cd.x, pp, Pp[2].y);
                caxpy(Hp[2], cz, hp);
                // V: i m psi Pbar / a = -i zeta P' (P parity); chi H / a = -delta H' (H parity)
                Pp[3].x = __builtin_fma(cz.y, pp, Pp[3].x);
                Pp[3].y = __builtin_fma(-cz.x, pp, Pp[3].y);
                Hp[3].x = __builtin_fma(-cd.x, hp, Hp[3].x);
                Hp[3].y = __builtin_fma(-cd.y, hp, Hp[3].y);
                r[q].pm = p;
                r[q].p = pn;
            }
        }
    };

    // i0 is a multiple of the (even) segment length: the parity of l - m is that of d
    int d = 0;
    for (; d + 3 < n; d += 4) {
        degree(d, std::integral_constant<bool, false>{});
        degree(d + 1, std::integral_constant<bool, true>{});
        degree(d + 2, std::integral_constant<bool, false>{});
        degree(d + 3, std::integral_constant<bool, true>{});
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
            const int sh = rec_renorm(r[q]);
            if (sh) {
#pragma unroll
                for (int f = 0; f < NACC; ++f) {
                    E[q][f] = make_double2(ldexp(E[q][f].x, -sh), ldexp(E[q][f].y, -sh));
                    O[q][f] = make_double2(ldexp(O[q][f].x, -sh), ldexp(O[q][f].y, -sh));
                }
            }
        }
    }
    for (; d < n; ++d) {
        if ((d & 1) == 0) degree(d, std::integral_constant<bool, false>{});
        else degree(d, std::integral_constant<bool, true>{});
    }
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
        if (jq[q] >= A.half) continue;
#pragma unroll
        for (int f = 0; f < NACC; ++f) {
            const size_t row = (static_cast<size_t>(KIND == 0 ? blockIdx.y : f) * A.nseg + gs) * A.nlat;
            const double2 nn = make_double2(ldexp(E[q][f].x + O[q][f].x, r[q].e), ldexp(E[q][f].y + O[q][f].y, r[q].e));
            const double2 ss = make_double2(ldexp(E[q][f].x - O[q][f].x, r[q].e), ldexp(E[q][f].y - O[q][f].y, r[q].e));
            S.part[row + jq[q]] = nn;
            S.part[row + (A.nlat - 1 - jq[q])] = ss;
        }
    }
}

// ==================================================== Legendre analysis ==
// One workgroup per degree segment; NW waves, each lane carries NJ northern
// latitudes (latitude j = (q NW + wave) 64 + lane).  Per chunk of D degrees a
// lane adds the contributions of its latitudes, the workgroup sums the lanes
// through LDS (lane-major write, transposed read), and the sums are written.
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
    const double2* __restrict__ U0;     // [3][modes] or nullptr (zero)
    const double2* __restrict__ Nprev;  // [3][modes] or nullptr
    double2* __restrict__ Nsave;        // [3][modes] or nullptr
    double2* __restrict__ out;          // [3][modes]
    double c0, c1;
};

template <int KIND>
struct AnaTraits {
    static constexpr int NC = KIND == 0 ? 2 : 6;       // doubles contributed per (l, j)
    static constexpr int NIN = KIND == 0 ? 1 : 5;      // complex input fields
    static constexpr int D = KIND == 0 ? 16 : 8;       // degrees per reduction chunk
};

// Folded, weighted inputs of one latitude (units of 2^e): for each field,
// S = F(mu) + F(-mu) and D = F(mu) - F(-mu); zero for padding latitudes.
template <int KIND>
__device__ __forceinline__ void load_folded(const AnaArgs& P, int m, int j, bool valid, int e, double2* Sv,
                                            double2* Dv) {
    const LegArgs& A = P.g;
    constexpr int NIN = AnaTraits<KIND>::NIN;
    const double sc = valid ? ldexp(1.0, e) : 0.0;
    const double wj = A.w[j];
    const double wdiv = wj / (A.a * A.sint[j] * A.sint[j]);
#pragma unroll
    for (int f = 0; f < NIN; ++f) {
        const int fld = KIND == 0 ? blockIdx.y : f;
        const double2* fr = P.four + (static_cast<size_t>(fld) * (A.L + 1) + m) * A.nlat;
        const double2 nn = fr[j];
        const double2 ss = fr[A.nlat - 1 - j];
        const double wt = (KIND == 0 || f == 4) ? wj : wdiv;
        Sv[f] = scale2(cadd(nn, ss), wt * sc);
        Dv[f] = scale2(csub(nn, ss), wt * sc);
    }
}

constexpr int RED_STRIDE = 72;   // doubles per staged output row (64 lanes + pad)

template <int KIND, int NJ, int NW>
__global__ __launch_bounds__(NW * WAVE) void legendre_anal_kernel(AnaArgs P) {
    constexpr int NC = AnaTraits<KIND>::NC;
    constexpr int NIN = AnaTraits<KIND>::NIN;
    constexpr int D = AnaTraits<KIND>::D;
    constexpr int NO = D * NC;                           // outputs per chunk
    constexpr int SL = KIND == 0 ? 1 : 3;                // staged double2 per degree
    constexpr int T = NW * WAVE;
    __shared__ double red[NW * NO * RED_STRIDE];
    __shared__ double2 stg[64 * SL];
    const LegArgs& A = P.g;
    const int gs = blockIdx.x;
    const int m = A.seg_m[gs], i0 = A.seg_i0[gs], n = A.seg_n[gs];
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1), wv = tid / WAVE;
    const int base = m * (2 * A.L + 3 - m) / 2;
    for (int d = tid; d < n; d += T) {
        const LegCoef c = A.rec[base + i0 + d];
        stg[d * SL] = make_double2(c.A, c.B);
        if constexpr (KIND == 1) {
            stg[d * SL + 1] = make_double2(c.hA, c.hB);
            stg[d * SL + 2] = make_double2(A.noa2[m + i0 + d], 0.0);
        }
    }
    double mu[NJ];
    int jq[NJ];
    Rec r[NJ];
    double2 Sv[NJ][NIN], Dv[NJ][NIN];
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
        jq[q] = (q * NW + wv) * WAVE + lane;
        const bool valid = jq[q] < A.half;
        const int j = valid ? jq[q] : A.half - 1;
        mu[q] = A.mu[j];
        r[q] = rec_start(A, gs, j);
        load_folded<KIND>(P, m, j, valid, r[q].e, Sv[q], Dv[q]);
    }
    const double dm = static_cast<double>(m);
    // reduction: thread t -> output o = t / G, part g = t % G
    constexpr int G = (T >= 8 * NO) ? 8 : (T >= 4 * NO) ? 4 : (T >= 2 * NO) ? 2 : 1;
    constexpr int NV = T / G;                            // values summed by one thread
    const int o_red = tid / G, g_red = tid % G;
    double* myred = red + wv * NO * RED_STRIDE;
    __syncthreads();

    for (int c0 = 0; c0 < n; c0 += D) {
#pragma unroll
        for (int dd = 0; dd < D; ++dd) {
            const int d = c0 + dd;
            double c[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) c[k] = 0.0;
            if (d < n) {
                const double2* st = stg + d * SL;
                const double2 ab = st[0];
                const bool odd = dd & 1;                 // l - m = i0 + c0 + dd, i0 and c0 even
#pragma unroll
                for (int q = 0; q < NJ; ++q) {
                    const double pn = __builtin_fma(ab.x * mu[q], r[q].p, -(ab.y * r[q].pm));
                    const double p = r[q].p;
                    if constexpr (KIND == 0) {
                        const double2 x = odd ? Dv[q][0] : Sv[q][0];
                        c[0] = __builtin_fma(x.x, p, c[0]);
                        c[1] = __builtin_fma(x.y, p, c[1]);
                    } else {
                        const double2 hab = st[1];
                        const double h = __builtin_fma(hab.x, pn, hab.y * r[q].pm);
                        // P terms take the fold of P's parity, H terms the opposite one
                        const double2 hU = odd ? Dv[q][0] : Sv[q][0], zU = odd ? Dv[q][2] : Sv[q][2];
                        const double2 zV = odd ? Dv[q][3] : Sv[q][3], ke = odd ? Dv[q][4] : Sv[q][4];
                        const double2 hVh = odd ? Sv[q][1] : Dv[q][1], zVh = odd ? Sv[q][3] : Dv[q][3];
                        const double2 zUh = odd ? Sv[q][2] : Dv[q][2];
                        const double pm2 = dm * p;               // m Pbar
                        const double pk = st[2].x * p;           // l(l+1)/a^2 Pbar
                        // N_h = -(i m hU P - hV H)
                        c[0] = __builtin_fma(hU.y, pm2, __builtin_fma(hVh.x, h, c[0]));
                        c[1] = __builtin_fma(-hU.x, pm2, __builtin_fma(hVh.y, h, c[1]));
                        // N_zeta = -(i m zU P - zV H)
                        c[2] = __builtin_fma(zU.y, pm2, __builtin_fma(zVh.x, h, c[2]));
                        c[3] = __builtin_fma(-zU.x, pm2, __builtin_fma(zVh.y, h, c[3]));
                        // N_delta = i m zV P + zU H + l(l+1)/a^2 KE P
                        c[4] = __builtin_fma(-zV.y, pm2, __builtin_fma(zUh.x, h, __builtin_fma(ke.x, pk, c[4])));
                        c[5] = __builtin_fma(zV.x, pm2, __builtin_fma(zUh.y, h, __builtin_fma(ke.y, pk, c[5])));
                    }
                    r[q].pm = p;
                    r[q].p = pn;
                }
            }
#pragma unroll
            for (int k = 0; k < NC; ++k) myred[(dd * NC + k) * RED_STRIDE + lane] = c[k];
        }
        // renormalise latitudes whose recurrence has grown back into range
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
            if (rec_renorm(r[q])) {
                const bool valid = jq[q] < A.half;
                load_folded<KIND>(P, m, valid ? jq[q] : A.half - 1, valid, r[q].e, Sv[q], Dv[q]);
            }
        }
        __syncthreads();
        if (o_red < NO) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
            for (int v = 0; v < NV; v += 4) {
#define RED_AT(vv) red[(((g_red + (vv) * G) / WAVE) * NO + o_red) * RED_STRIDE + ((g_red + (vv) * G) % WAVE)]
                s0 += RED_AT(v);
                if (v + 1 < NV) s1 += RED_AT(v + 1);
                if (v + 2 < NV) s2 += RED_AT(v + 2);
                if (v + 3 < NV) s3 += RED_AT(v + 3);
#undef RED_AT
            }
            double s = (s0 + s1) + (s2 + s3);
#pragma unroll
            for (int msk = 1; msk < G; msk <<= 1) s += __shfl_xor(s, msk, G);
            const int dd = o_red / NC, k = o_red % NC;
            const int d = c0 + dd;
            if (g_red == 0 && d < n) {
                const size_t idx = static_cast<size_t>(base) + i0 + d;
                if constexpr (KIND == 0) {
                    double* dst = reinterpret_cast<double*>(P.spec + static_cast<size_t>(blockIdx.y) * A.modes + idx);
                    dst[k] = s;
                } else {
                    const int f = k >> 1, part = k & 1;
                    const size_t e2 = (static_cast<size_t>(f) * A.modes + idx) * 2 + part;
                    double v = __builtin_fma(P.c0, s, P.U0 ? reinterpret_cast<const double*>(P.U0)[e2] : 0.0);
                    if (P.Nprev) v = __builtin_fma(P.c1, reinterpret_cast<const double*>(P.Nprev)[e2], v);
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
    const double* __restrict__ mu;     // [half] sin(latitude), northern
    const int* __restrict__ radix;     // [npass]
    int npass, L, nlat, nlon, half;
    // inverse input: synthesis partials [nf_in][nseg][nlat]; the Fourier
    // coefficient F_m of a latitude is the sum over segments segbase[m] ..
    // segbase[m + 1] - 1
    const double2* __restrict__ part;
    const int* __restrict__ segbase;   // [L+2]
    int nseg;
    double2* __restrict__ fout;        // Fourier coefficients [nf_out][L+1][nlat] (order-major)
    const double* __restrict__ gin;    // grid input  [nf][nlat][nlon] (forward-only mode)
    double* __restrict__ gout;         // grid output [nf][nlat][nlon] (inverse-only mode)
    int nf;
    double two_omega;                  // mode 2: 2 Omega adds f = 2 Omega mu to zeta (absolute vorticity)
};

// One Stockham pass of radix R over M complex points, for narr arrays at once
// (one barrier per pass for all of them): src[a] -> dst[a].
template <int R>
__device__ __forceinline__ void fft_pass(double2* const* src, double2* const* dst, int narr, int M, int Ns,
                                         const double* tw, bool inverse) {
    const int nb = M / R;
    const int twstep = M / (Ns * R);
    const int total = nb * narr;
    for (int x = threadIdx.x; x < total; x += blockDim.x) {
        const int a = x / nb;
        const int jb = x - a * nb;
        const double2* sa = src[a];
        double2* da = dst[a];
        const int k = jb % Ns;
        double2 v[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            v[t] = sa[jb + t * nb];
            if (t > 0) {
                const int ti = (t * k * twstep) % M;
                double2 wv = make_double2(tw[2 * ti], tw[2 * ti + 1]);
                if (inverse) wv.y = -wv.y;
                v[t] = cmul(v[t], wv);
            }
        }
        if constexpr (R == 2) {
            const double2 a0 = v[0], b0 = v[1];
            v[0] = cadd(a0, b0);
            v[1] = csub(a0, b0);
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
        for (int t = 0; t < R; ++t) da[base + t * Ns] = v[t];
    }
}

constexpr int MAXB = 4;   // arrays transformed together

// Complex FFTs of length M of narr (<= MAXB) arrays in LDS, ping-ponging with
// the scratch arrays; res[a] receives the buffer holding the result of array a.
__device__ void fft_lds(double2* const* a, double2* const* scratch, int narr, const RingArgs& A, bool inverse,
                        double2** res) {
    const int M = A.nlon / 2;
    int Ns = 1;
    double2* src[MAXB];
    double2* dst[MAXB];
    for (int i = 0; i < MAXB; ++i) {
        src[i] = i < narr ? a[i] : a[0];
        dst[i] = i < narr ? scratch[i] : scratch[0];
    }
    for (int p = 0; p < A.npass; ++p) {
        const int R = A.radix[p];
        if (R == 4) fft_pass<4>(src, dst, narr, M, Ns, A.tw, inverse);
        else if (R == 2) fft_pass<2>(src, dst, narr, M, Ns, A.tw, inverse);
        else fft_pass<3>(src, dst, narr, M, Ns, A.tw, inverse);
        __syncthreads();
        Ns *= R;
        for (int i = 0; i < MAXB; ++i) {
            double2* t = src[i];
            src[i] = dst[i];
            dst[i] = t;
        }
    }
    for (int i = 0; i < narr; ++i) res[i] = src[i];
}

// Compile-time-length variant: the pass sequence (radix 4, then 2, then 3) is
// fixed by M, every index division is by a constant, and the twiddles are read
// from LDS.  The result is in `a` after an even number of passes, else in `scratch`.
template <int R, int M, int NS, bool INV>
__device__ __forceinline__ void fft_pass_ct(double2* const* src, double2* const* dst, int narr, const double2* tw) {
    constexpr int nb = M / R;
    constexpr int twstep = M / (NS * R);
    const int total = nb * narr;
    for (int x = threadIdx.x; x < total; x += blockDim.x) {
        const int a = x / nb;
        const int jb = x - a * nb;
        const double2* sa = src[a];
        double2* da = dst[a];
        const int k = jb % NS;
        double2 v[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            v[t] = sa[jb + t * nb];
            if (t > 0) {
                double2 wv = tw[t * k * twstep];
                if (INV) wv.y = -wv.y;
                v[t] = cmul(v[t], wv);
            }
        }
        if constexpr (R == 2) {
            const double2 a0 = v[0], b0 = v[1];
            v[0] = cadd(a0, b0);
            v[1] = csub(a0, b0);
        } else if constexpr (R == 4) {
            const double2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
            const double2 b0 = cadd(v[1], v[3]), b1 = csub(v[1], v[3]);
            const double2 b1r = INV ? make_double2(-b1.y, b1.x) : make_double2(b1.y, -b1.x);
            v[0] = cadd(a0, b0);
            v[2] = csub(a0, b0);
            v[1] = cadd(a1, b1r);
            v[3] = csub(a1, b1r);
        } else {
            constexpr double c = -0.5;
            constexpr double s = INV ? 0.86602540378443864676 : -0.86602540378443864676;
            const double2 t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
            const double2 m1 = make_double2(__builtin_fma(c, t1.x, v[0].x), __builtin_fma(c, t1.y, v[0].y));
            const double2 m2 = make_double2(-s * t2.y, s * t2.x);
            v[0] = cadd(v[0], t1);
            v[1] = cadd(m1, m2);
            v[2] = csub(m1, m2);
        }
        const int base = (jb / NS) * NS * R + k;
#pragma unroll
        for (int t = 0; t < R; ++t) da[base + t * NS] = v[t];
    }
}

template <int M, int NS, bool INV>
__device__ __forceinline__ int fft_passes_ct(double2* const* src, double2* const* dst, int narr, const double2* tw) {
    if constexpr (NS >= M) {
        return 0;
    } else {
        constexpr int rem = M / NS;
        constexpr int R = (rem % 4 == 0) ? 4 : (rem % 2 == 0) ? 2 : 3;
        static_assert(rem % R == 0, "FFT length must be 2^a 3^b");
        fft_pass_ct<R, M, NS, INV>(src, dst, narr, tw);
        __syncthreads();
        return 1 + fft_passes_ct<M, NS * R, INV>(dst, src, narr, tw);
    }
}

template <int M, bool INV>
__device__ __forceinline__ void fft_lds_ct(double2* const* a, double2* const* scratch, int narr, const double2* tw,
                                           double2** res) {
    double2* src[MAXB];
    double2* dst[MAXB];
    for (int i = 0; i < MAXB; ++i) {
        src[i] = i < narr ? a[i] : a[0];
        dst[i] = i < narr ? scratch[i] : scratch[0];
    }
    const int np = fft_passes_ct<M, 1, INV>(src, dst, narr, tw);
    for (int i = 0; i < narr; ++i) res[i] = (np & 1) ? dst[i] : src[i];
}

// Fourier coefficients F_m (m <= L) of latitude j for fields f0 .. f0 + nb - 1
// into the LDS rows x[b]: each the sum of its order's segment partials.
__device__ void load_coeffs(const RingArgs& A, int f0, int nb, int j, double2* const* x) {
    const int n = nb * (A.L + 1);
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int b = t / (A.L + 1), m = t - b * (A.L + 1);
        const double2* pf = A.part + static_cast<size_t>(f0 + b) * A.nseg * A.nlat + j;
        double2 acc = make_double2(0.0, 0.0);
        const int g1 = A.segbase[m + 1];
        for (int g = A.segbase[m]; g < g1; ++g) acc = cadd(acc, pf[static_cast<size_t>(g) * A.nlat]);
        x[b][m] = acc;
    }
}

// From the LDS row F_m (m <= L) of one latitude, the half-length spectrum Z of
// the inverse real FFT:
//   Z_k = (X_k + conj X_{M-k}) + i e^{2 pi i k/nlon} (X_k - conj X_{M-k}),
// X_0 taken real, X_k = 0 for k > L.
__device__ void load_inverse(const double2* frow, double2* z, const RingArgs& A) {
    const int M = A.nlon / 2;
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
        double2 xk = make_double2(0.0, 0.0), xr = make_double2(0.0, 0.0);
        if (k <= A.L) xk = frow[k];
        const int kr = M - k;                      // 1..M
        if (kr <= A.L && kr < M) xr = frow[kr];
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
// frow points at F_0 of the latitude; consecutive orders are nlat apart.
__device__ void store_forward(const double2* Z, double2* frow, const RingArgs& A) {
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
        frow[static_cast<size_t>(k) * A.nlat] = scale2(X, inv);
    }
}

// MODE 0: inverse only (Fourier -> grid), nf fields, MAXB at a time.
// MODE 1: forward only (grid -> Fourier), nf fields, MAXB at a time.
// MODE 2: non-linear products: inverse of h, zeta, U, V; pointwise
//         hU, hV, zU, zV, KE = (U^2 + V^2) / (2 cos^2 phi); forward of those five.
// LDS: 2 MAXB arrays of nlon/2 complex values.
// Transforms of `narr` arrays: compile-time length MC when nonzero, else runtime.
template <int MC>
__device__ __forceinline__ void ring_fft(double2* const* a, double2* const* scratch, int narr, const RingArgs& A,
                                         const double2* twl, bool inverse, double2** res) {
    if constexpr (MC > 0) {
        if (inverse) fft_lds_ct<MC, true>(a, scratch, narr, twl, res);
        else fft_lds_ct<MC, false>(a, scratch, narr, twl, res);
    } else {
        fft_lds(a, scratch, narr, A, inverse, res);
    }
}

// Workgroups are dispatched round-robin over the 8 XCDs: each XCD gets a
// contiguous band of latitudes, so the rings that share cache lines of the
// order-major buffers meet in one L2.
__device__ __forceinline__ int ring_of_block(int b, int nlat) {
    if (nlat % 8) return b;
    return (b % 8) * (nlat / 8) + b / 8;
}

template <int MODE, int MC>
__global__ __launch_bounds__(256) void ring_kernel(RingArgs A) {
    extern __shared__ __align__(16) double2 lds[];
    const int M = A.nlon / 2;
    const int j = ring_of_block(blockIdx.x, A.nlat);
    const size_t fstride = static_cast<size_t>(A.L + 1) * A.nlat;   // one field of [L+1][nlat]
    const size_t row = static_cast<size_t>(j);
    double2* arr[2 * MAXB];
#pragma unroll
    for (int i = 0; i < 2 * MAXB; ++i) arr[i] = lds + i * M;
    double2* res[MAXB];
    double2* twl = lds + 2 * MAXB * M;               // twiddles (compile-time lengths only)
    if constexpr (MC > 0) {
        for (int k = threadIdx.x; k < M; k += blockDim.x) twl[k] = make_double2(A.tw[2 * k], A.tw[2 * k + 1]);
    }
    if constexpr (MODE == 0) {
        for (int f0 = 0; f0 < A.nf; f0 += MAXB) {
            const int nb = min(MAXB, A.nf - f0);
            load_coeffs(A, f0, nb, j, arr + MAXB);
            __syncthreads();
            for (int b = 0; b < nb; ++b) load_inverse(arr[MAXB + b], arr[b], A);
            __syncthreads();
            ring_fft<MC>(arr, arr + MAXB, nb, A, twl, true, res);
            for (int b = 0; b < nb; ++b) {
                double2* g = reinterpret_cast<double2*>(A.gout + (static_cast<size_t>(f0 + b) * A.nlat + j) * A.nlon);
                for (int k = threadIdx.x; k < M; k += blockDim.x) g[k] = res[b][k];
            }
            __syncthreads();
        }
    } else if constexpr (MODE == 1) {
        for (int f0 = 0; f0 < A.nf; f0 += MAXB) {
            const int nb = min(MAXB, A.nf - f0);
            for (int b = 0; b < nb; ++b) {
                const double2* g =
                    reinterpret_cast<const double2*>(A.gin + (static_cast<size_t>(f0 + b) * A.nlat + j) * A.nlon);
                for (int k = threadIdx.x; k < M; k += blockDim.x) arr[b][k] = g[k];
            }
            __syncthreads();
            ring_fft<MC>(arr, arr + MAXB, nb, A, twl, false, res);
            for (int b = 0; b < nb; ++b) store_forward(res[b], A.fout + (f0 + b) * fstride + row, A);
            __syncthreads();
        }
    } else {
        load_coeffs(A, 0, 4, j, arr + MAXB);
        __syncthreads();
        for (int f = 0; f < 4; ++f) load_inverse(arr[MAXB + f], arr[f], A);
        __syncthreads();
        ring_fft<MC>(arr, arr + MAXB, 4, A, twl, true, res);
        // the four arrays not holding results are free
        double2* freea[MAXB];
        {
            int nfree = 0;
            for (int i = 0; i < 2 * MAXB; ++i) {
                bool used = false;
                for (int b = 0; b < MAXB; ++b) used |= (arr[i] == res[b]);
                if (!used) freea[nfree++] = arr[i];
            }
        }
        const int jn = j < A.half ? j : A.nlat - 1 - j;
        const double sn = A.sint[jn];
        const double kefac = 0.5 / (sn * sn);
        const double fcor = A.two_omega * (j < A.half ? A.mu[jn] : -A.mu[jn]);   // 0 unless L_c joins N
        double* h = reinterpret_cast<double*>(res[0]);
        double* z = reinterpret_cast<double*>(res[1]);
        const double* U = reinterpret_cast<const double*>(res[2]);
        double* V = reinterpret_cast<double*>(res[3]);
        double* ke = reinterpret_cast<double*>(freea[0]);
        double* hv = reinterpret_cast<double*>(freea[1]);
        for (int k = threadIdx.x; k < A.nlon; k += blockDim.x) {
            const double u = U[k], v = V[k], hh = h[k], zz = z[k] + fcor;
            ke[k] = __builtin_fma(u, u, v * v) * kefac;
            hv[k] = hh * v;
            V[k] = zz * v;          // zeta V
            h[k] = hh * u;          // h U
            z[k] = zz * u;          // zeta U
        }
        __syncthreads();
        // forward transforms in two batches: (hU, hV, zU) then (zV, KE);
        // output fields 0 hU, 1 hV, 2 zU, 3 zV, 4 KE
        {
            double2* in3[MAXB] = {res[0], freea[1], res[1], res[1]};
            double2* sc3[MAXB] = {res[2], freea[2], freea[3], freea[3]};
            double2* out3[MAXB];
            ring_fft<MC>(in3, sc3, 3, A, twl, false, out3);
            store_forward(out3[0], A.fout + 0 * fstride + row, A);
            store_forward(out3[1], A.fout + 1 * fstride + row, A);
            store_forward(out3[2], A.fout + 2 * fstride + row, A);
        }
        __syncthreads();   // batch 1 outputs are read before their arrays become scratch
        {
            double2* in2[MAXB] = {res[3], freea[0], res[3], res[3]};
            double2* sc2[MAXB] = {res[2], freea[2], res[2], res[2]};
            double2* out2[MAXB];
            ring_fft<MC>(in2, sc2, 2, A, twl, false, out2);
            store_forward(out2[0], A.fout + 3 * fstride + row, A);
            store_forward(out2[1], A.fout + 4 * fstride + row, A);
        }
    }
}

}  // namespace

namespace {
// out = x + a y over n doubles (spectral-state combinations of the time steppers).
__global__ __launch_bounds__(256) void axpy_kernel(double* out, const double* x, double a, const double* y, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = __builtin_fma(a, y[i], x[i]);
}
}  // namespace

int launch_axpy(double* out, const double* x, double a, const double* y, int n, hipStream_t stream) {
    hipLaunchKernelGGL(axpy_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, out, x, a, y, n);
    REXI_HIP(hipGetLastError());
    return REXI_OK;
}

// ------------------------------------------------------------ launchers --
static LegArgs leg_args(const swe_ctx* ctx) {
    LegArgs g;
    g.rec = ctx->d_rec;
    g.aon = ctx->d_aon;
    g.noa2 = ctx->d_noa2;
    g.mu = ctx->d_mu;
    g.sint = ctx->d_sint;
    g.w = ctx->d_w;
    g.seg_m = ctx->d_seg_m;
    g.seg_i0 = ctx->d_seg_i0;
    g.seg_n = ctx->d_seg_n;
    g.seed_pm = ctx->d_seed_pm;
    g.seed_p = ctx->d_seed_p;
    g.seed_e = ctx->d_seed_e;
    g.nseg = ctx->nseg;
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
    r.mu = ctx->d_mu;
    r.radix = ctx->d_radix;
    r.npass = ctx->npass;
    r.L = ctx->L;
    r.nlat = ctx->nlat;
    r.nlon = ctx->nlon;
    r.half = ctx->nlat / 2;
    return r;
}

static int ring_lds_bytes(const swe_ctx* ctx, int /*mode*/) {
    const int M = ctx->nlon / 2;
    return (2 * MAXB + 1) * M * static_cast<int>(sizeof(double2));
}

template <int MODE>
static const void* ring_fn(int M) {
    switch (M) {
        case 48: return reinterpret_cast<const void*>(&ring_kernel<MODE, 48>);
        case 96: return reinterpret_cast<const void*>(&ring_kernel<MODE, 96>);
        case 192: return reinterpret_cast<const void*>(&ring_kernel<MODE, 192>);
        case 384: return reinterpret_cast<const void*>(&ring_kernel<MODE, 384>);
        case 768: return reinterpret_cast<const void*>(&ring_kernel<MODE, 768>);
        default: return reinterpret_cast<const void*>(&ring_kernel<MODE, 0>);
    }
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
    const int M = ctx->nlon / 2;
    if ((rc = allow_lds(ring_fn<0>(M), ring_lds_bytes(ctx, 0), "the longitude FFT")) != REXI_OK) return rc;
    if ((rc = allow_lds(ring_fn<1>(M), ring_lds_bytes(ctx, 1), "the longitude FFT")) != REXI_OK) return rc;
    if ((rc = allow_lds(ring_fn<2>(M), ring_lds_bytes(ctx, 2), "the longitude FFT")) != REXI_OK) return rc;
    return REXI_OK;
}

// Latitudes per lane for the Legendre stages: enough to cover the hemisphere
// with one (synthesis) or at most two (analysis) waves, up to three.
static int lat_per_lane(const swe_ctx* ctx) {
    const int half = ctx->nlat / 2;
    return half <= WAVE ? 1 : (half <= 2 * WAVE ? 2 : 3);
}

int launch_legendre_synth(swe_ctx* ctx, int kind, const double* spec, double* part, int nf, hipStream_t stream) {
    SynArgs S;
    S.g = leg_args(ctx);
    S.spec = reinterpret_cast<const double2*>(spec);
    S.part = reinterpret_cast<double2*>(part);
    // one latitude per lane: more waves in flight (measured faster than 2 or 3 at T255)
    const int NJ = 1;
    const int tiles = (ctx->nlat / 2 + NJ * WAVE - 1) / (NJ * WAVE);
    const dim3 grid(ctx->nseg, kind == 0 ? nf : 1, tiles);
    const int slot = prof_begin(ctx, REXI_KERNEL_LEG_SYNTH, stream);
    if (kind == 0) {
        if (NJ == 1) hipLaunchKernelGGL((legendre_synth_kernel<0, 1>), grid, dim3(WAVE), 0, stream, S);
        else if (NJ == 2) hipLaunchKernelGGL((legendre_synth_kernel<0, 2>), grid, dim3(WAVE), 0, stream, S);
        else hipLaunchKernelGGL((legendre_synth_kernel<0, 3>), grid, dim3(WAVE), 0, stream, S);
    } else {
        if (NJ == 1) hipLaunchKernelGGL((legendre_synth_kernel<1, 1>), grid, dim3(WAVE), 0, stream, S);
        else if (NJ == 2) hipLaunchKernelGGL((legendre_synth_kernel<1, 2>), grid, dim3(WAVE), 0, stream, S);
        else hipLaunchKernelGGL((legendre_synth_kernel<1, 3>), grid, dim3(WAVE), 0, stream, S);
    }
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_LEG_SYNTH, slot, stream);
    return REXI_OK;
}

template <int KIND>
static void launch_anal_shape(int NJ, int NW, dim3 grid, const AnaArgs& P, hipStream_t stream) {
    if (NW == 1) {
        if (NJ == 1) hipLaunchKernelGGL((legendre_anal_kernel<KIND, 1, 1>), grid, dim3(WAVE), 0, stream, P);
        else if (NJ == 2) hipLaunchKernelGGL((legendre_anal_kernel<KIND, 2, 1>), grid, dim3(WAVE), 0, stream, P);
        else hipLaunchKernelGGL((legendre_anal_kernel<KIND, 3, 1>), grid, dim3(WAVE), 0, stream, P);
    } else {
        hipLaunchKernelGGL((legendre_anal_kernel<KIND, 3, 2>), grid, dim3(2 * WAVE), 0, stream, P);
    }
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
    const int NJ = lat_per_lane(ctx);
    const int NW = (half + NJ * WAVE - 1) / (NJ * WAVE);
    if (NW > 2) return fail(REXI_ENOTSUP, "Legendre analysis: more than 384 northern latitudes");
    const dim3 grid(ctx->nseg, kind == 0 ? nf : 1);
    const int slot = prof_begin(ctx, REXI_KERNEL_LEG_ANAL, stream);
    if (kind == 0) launch_anal_shape<0>(NJ, NW, grid, P, stream);
    else launch_anal_shape<1>(NJ, NW, grid, P, stream);
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_LEG_ANAL, slot, stream);
    return REXI_OK;
}

int launch_ring(swe_ctx* ctx, int mode, const double* part, const int* segbase, int nseg, double* fout,
                const double* gin, double* gout, int nf, hipStream_t stream, double two_omega) {
    RingArgs R = ring_args(ctx);
    R.two_omega = two_omega;
    R.part = reinterpret_cast<const double2*>(part);
    R.segbase = segbase;
    R.nseg = nseg;
    R.fout = reinterpret_cast<double2*>(fout);
    R.gin = gin;
    R.gout = gout;
    R.nf = nf;
    const size_t lds = static_cast<size_t>(ring_lds_bytes(ctx, mode));
    const int slot = prof_begin(ctx, REXI_KERNEL_RING, stream);
    const int M = ctx->nlon / 2;
    const void* fn = mode == 0 ? ring_fn<0>(M) : (mode == 1 ? ring_fn<1>(M) : ring_fn<2>(M));
    void* kargs[] = {&R};
    REXI_HIP(hipLaunchKernel(fn, dim3(ctx->nlat), dim3(256), kargs, lds, stream));
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_RING, slot, stream);
    return REXI_OK;
}

}  // namespace rexi
