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
    unsigned* status;                   // non-finite outputs set a STATUS_* flag
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
};

// Degrees per reduction chunk.  The non-linear analysis with two waves per
// workgroup (more than 192 northern latitudes) takes 4-degree chunks, whose
// lane sums need half the LDS, and asks for two waves per SIMD; with one wave
// the 8-degree chunk is faster.
template <int KIND, int NW>
constexpr int ana_chunk() { return KIND == 0 ? 16 : (NW == 2 ? 4 : 8); }
template <int KIND, int NW>
constexpr int ana_occupancy() { return KIND == 1 && NW == 2 ? 2 : 1; }

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
__global__ __launch_bounds__(NW * WAVE) __attribute__((amdgpu_waves_per_eu(ana_occupancy<KIND, NW>())))
void legendre_anal_kernel(AnaArgs P) {
    constexpr int NC = AnaTraits<KIND>::NC;
    constexpr int NIN = AnaTraits<KIND>::NIN;
    constexpr int D = ana_chunk<KIND, NW>();
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
        // KIND 1: the update's inputs U0 and Nprev of this thread's output in
        // the chunk, requested before the chunk's products so that their
        // latency overlaps them (the update itself keeps its order below)
        double u0v = 0.0, npv = 0.0;
        if constexpr (KIND == 1) {
            const int d = c0 + o_red / NC, k = o_red % NC;
            if (o_red < NO && g_red == 0 && d < n) {
                const size_t e2 = (static_cast<size_t>(k >> 1) * A.modes + base + i0 + d) * 2 + (k & 1);
                if (P.U0) u0v = reinterpret_cast<const double*>(P.U0)[e2];
                if (P.Nprev) npv = reinterpret_cast<const double*>(P.Nprev)[e2];
            }
        }
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
                    note_nonfinite(A.status, s, STATUS_TRANSFORM);
                    dst[k] = s;
                } else {
                    const int f = k >> 1, part = k & 1;
                    const size_t e2 = (static_cast<size_t>(f) * A.modes + idx) * 2 + part;
                    double v = __builtin_fma(P.c0, s, u0v);
                    if (P.Nprev) v = __builtin_fma(P.c1, npv, v);
                    if (P.Nsave) reinterpret_cast<double*>(P.Nsave)[e2] = s;
                    note_nonfinite(A.status, v, STATUS_NONLINEAR);
                    reinterpret_cast<double*>(P.out)[e2] = v;
                }
            }
        }
        __syncthreads();
    }
}

// ============================================================ ring FFTs ==
struct RingArgs {
    const double* __restrict__ tw;     // [M] complex: the twiddles of every FFT pass (ring_twiddles)
    const double* __restrict__ twr;    // [M] complex e^{-2 pi i k / nlon}
    const double* __restrict__ sint;   // [half]
    const double* __restrict__ mu;     // [half] sin(latitude), northern
    const int* __restrict__ radix;     // [npass]
    int npass, L, nlat, nlon, half;
    // inverse input: synthesis partials, element (field f, segment g,
    // latitude j) at f pfs + g pgs + j pjs ([nf_in][nseg][nlat], or
    // [nf_in][nlat][L+1] latitude-major); the Fourier coefficient F_m of a
    // latitude is the sum over segments segbase[m] .. segbase[m + 1] - 1
    const double2* __restrict__ part;
    const int* __restrict__ segbase;   // [L+2]; nullptr: one segment per order (segbase[m] = m)
    int nseg;
    long long pfs;
    int pgs, pjs;
    double2* __restrict__ fout;        // Fourier coefficients [nf_out][L+1][nlat] (order-major)
    const double* __restrict__ gin;    // grid input  [nf][nlat][nlon] (forward-only mode)
    double* __restrict__ gout;         // grid output [nf][nlat][nlon] (inverse-only mode)
    int nf;
    unsigned* status;                  // non-finite grid outputs set STATUS_TRANSFORM
    double two_omega;                  // mode 2: 2 Omega adds f = 2 Omega mu to zeta (absolute vorticity)
};

// LDS arrays hold one padding slot per 8 complex values, so that the strided
// accesses of a Stockham pass spread over the banks.
__device__ __forceinline__ int pad8(int e) { return e + (e >> 3); }
__host__ __device__ constexpr int padded_len(int M) { return M + (M >> 3) + 1; }

constexpr int RING_WAVES = 5;        // one wave per field of the forward transforms
constexpr int RING_MMAX_RT = 1024;   // longest FFT of the runtime-length path

// The lane index as a value the compiler cannot relate to other uses of it.
// Each pass indexes with its own copy: index arithmetic simplified under one
// pass's bound (jb < nb) must not be reused by a pass with a larger bound.
__device__ __forceinline__ int opaque_lane(int lane) {
    asm volatile("" : "+v"(lane));
    return lane;
}

// Makes the LDS writes of every lane of the wave visible to the other lanes'
// later reads (the wave's LDS operations execute in order; this stops the
// compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- small DFTs, natural order: X_k = sum_n v_n e^{-+ 2 pi i n k / R}
// (minus sign: forward; plus: INV)
template <bool INV>
__device__ __forceinline__ double2 mul_mi(double2 x) {   // x (-i) forward, x (+i) inverse
    return INV ? make_double2(-x.y, x.x) : make_double2(x.y, -x.x);
}

template <bool INV>
__device__ __forceinline__ void dft3(double2& a0, double2& a1, double2& a2) {
    constexpr double s = INV ? 0.86602540378443864676 : -0.86602540378443864676;
    const double2 t1 = cadd(a1, a2), t2 = csub(a1, a2);
    const double2 m1 = make_double2(__builtin_fma(-0.5, t1.x, a0.x), __builtin_fma(-0.5, t1.y, a0.y));
    const double2 m2 = make_double2(-s * t2.y, s * t2.x);   // i s t2
    a0 = cadd(a0, t1);
    a1 = cadd(m1, m2);
    a2 = csub(m1, m2);
}

template <bool INV>
__device__ __forceinline__ void dft4(double2& a0, double2& a1, double2& a2, double2& a3) {
    const double2 s0 = cadd(a0, a2), s1 = csub(a0, a2), s2 = cadd(a1, a3), s3 = mul_mi<INV>(csub(a1, a3));
    a0 = cadd(s0, s2);
    a2 = csub(s0, s2);
    a1 = cadd(s1, s3);
    a3 = csub(s1, s3);
}

template <int R, bool INV>
__device__ __forceinline__ void dft(double2* v) {
    if constexpr (R == 2) {
        const double2 t = v[0];
        v[0] = cadd(t, v[1]);
        v[1] = csub(t, v[1]);
    } else if constexpr (R == 3) {
        dft3<INV>(v[0], v[1], v[2]);
    } else if constexpr (R == 4) {
        dft4<INV>(v[0], v[1], v[2], v[3]);
    } else if constexpr (R == 6) {
        // X_k = E_k + w6^k O_k, X_{k+3} = E_k - w6^k O_k (E, O: 3-point DFTs of
        // the even and odd samples)
        double2 e0 = v[0], e1 = v[2], e2 = v[4], o0 = v[1], o1 = v[3], o2 = v[5];
        dft3<INV>(e0, e1, e2);
        dft3<INV>(o0, o1, o2);
        constexpr double h = 0.86602540378443864676;
        o1 = cmul(o1, make_double2(0.5, INV ? h : -h));
        o2 = cmul(o2, make_double2(-0.5, INV ? h : -h));
        v[0] = cadd(e0, o0);
        v[3] = csub(e0, o0);
        v[1] = cadd(e1, o1);
        v[4] = csub(e1, o1);
        v[2] = cadd(e2, o2);
        v[5] = csub(e2, o2);
    } else {
        static_assert(R == 8, "radix 2, 3, 4, 6 or 8");
        // X_k = E_k + w8^k O_k, X_{k+4} = E_k - w8^k O_k
        double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
        dft4<INV>(e0, e1, e2, e3);
        dft4<INV>(o0, o1, o2, o3);
        constexpr double c = 0.70710678118654752440;
        o1 = INV ? make_double2(c * (o1.x - o1.y), c * (o1.x + o1.y)) : make_double2(c * (o1.x + o1.y), c * (o1.y - o1.x));
        o2 = mul_mi<INV>(o2);
        o3 = INV ? make_double2(-c * (o3.x + o3.y), c * (o3.x - o3.y)) : make_double2(c * (o3.y - o3.x), -c * (o3.x + o3.y));
        v[0] = cadd(e0, o0);
        v[4] = csub(e0, o0);
        v[1] = cadd(e1, o1);
        v[5] = csub(e1, o1);
        v[2] = cadd(e2, o2);
        v[6] = csub(e2, o2);
        v[3] = cadd(e3, o3);
        v[7] = csub(e3, o3);
    }
}

// Radix of the next Stockham pass when rem = M / Ns points per sub-transform
// remain (host and device use the same rule).
__host__ __device__ constexpr int ring_radix(int rem) {
    return rem == 6 ? 6 : rem % 8 == 0 ? 8 : rem % 4 == 0 ? 4 : rem % 6 == 0 ? 6 : rem % 2 == 0 ? 2 : 3;
}

// One Stockham pass of radix R over the M complex values of the wave's LDS
// array x (padded), in place: every lane first reads all its butterflies'
// values and twiddles (lanes past the last butterfly read butterfly 0's and
// discard the result), then transforms them, then writes them.  Ns = product
// of the radices already applied; the pass's twiddles e^{-2 pi i t k / (Ns R)}
// are tw[Ns - 1 + (t - 1) Ns + k] (consecutive k, so consecutive lanes read
// consecutive entries).  MC, NSC: compile-time M and Ns (0: runtime).
template <int R, bool INV, int MC, int NSC>
__device__ __forceinline__ void wave_pass(double2* x, int Mr, int Nsr, const double2* tw, int lane) {
    const int M = MC > 0 ? MC : Mr;
    const int Ns = NSC > 0 ? NSC : Nsr;
    const int nb = M / R;
    constexpr int BPL = ((MC > 0 ? MC : RING_MMAX_RT) / R + WAVE - 1) / WAVE;   // butterflies per lane
    constexpr bool TW = NSC != 1;                                              // the first pass has none
    lane = opaque_lane(lane);
    double2 v[BPL][R], w[BPL][R];
#pragma unroll
    for (int b = 0; b < BPL; ++b) {
        const int jb0 = lane + b * WAVE;
        const int jb = jb0 < nb ? jb0 : 0;
        const int k = jb % Ns;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            v[b][t] = x[pad8(jb + t * nb)];
            if (TW && t > 0) w[b][t] = tw[Ns - 1 + (t - 1) * Ns + k];
        }
    }
    __builtin_amdgcn_sched_barrier(0);   // the reads stay ahead of the arithmetic
#pragma unroll
    for (int b = 0; b < BPL; ++b) {
        if (TW) {
#pragma unroll
            for (int t = 1; t < R; ++t) {
                double2 wt = w[b][t];
                if (INV) wt.y = -wt.y;
                v[b][t] = cmul(v[b][t], wt);
            }
        }
        dft<R, INV>(v[b]);
    }
    wave_sync();
#pragma unroll
    for (int b = 0; b < BPL; ++b) {
        const int jb = lane + b * WAVE;
        if (jb < nb) {
            const int k = jb % Ns;
            const int base = (jb / Ns) * Ns * R + k;
#pragma unroll
            for (int t = 0; t < R; ++t) x[pad8(base + t * Ns)] = v[b][t];
        }
    }
    wave_sync();
}

// Complex FFT of length M of the wave's array x: compile-time M ...
template <int M, int NS, bool INV>
__device__ __forceinline__ void wave_fft_ct(double2* x, const double2* tw, int lane) {
    if constexpr (NS < M) {
        constexpr int R = ring_radix(M / NS);
        static_assert((M / NS) % R == 0, "FFT length must be 2^a 3^b");
        wave_pass<R, INV, M, NS>(x, M, NS, tw, lane);
        wave_fft_ct<M, NS * R, INV>(x, tw, lane);
    }
}

// ... or runtime M (passes from the context's radix list).
template <bool INV>
__device__ void wave_fft_rt(double2* x, const RingArgs& A, const double2* tw, int lane) {
    const int M = A.nlon / 2;
    int Ns = 1;
    for (int p = 0; p < A.npass; ++p) {
        const int R = A.radix[p];
        if (R == 8) wave_pass<8, INV, 0, 0>(x, M, Ns, tw, lane);
        else if (R == 6) wave_pass<6, INV, 0, 0>(x, M, Ns, tw, lane);
        else if (R == 4) wave_pass<4, INV, 0, 0>(x, M, Ns, tw, lane);
        else if (R == 2) wave_pass<2, INV, 0, 0>(x, M, Ns, tw, lane);
        else wave_pass<3, INV, 0, 0>(x, M, Ns, tw, lane);
        Ns *= R;
    }
}

template <int MC, bool INV>
__device__ __forceinline__ void wave_fft(double2* x, const RingArgs& A, const double2* tw, int lane) {
    if constexpr (MC > 0) wave_fft_ct<MC, 1, INV>(x, tw, lane);
    else wave_fft_rt<INV>(x, A, tw, lane);
}

// Fourier coefficients F_m (m <= L) of field f at latitude j into the wave's
// array x: each the sum of its order's segment partials (the first segment of
// every order the lane holds is loaded before any is added).
template <int MC>
__device__ __forceinline__ void wave_load_coeffs(const RingArgs& A, int f, int j, double2* x, int lane) {
    const double2* pf = A.part + f * A.pfs + static_cast<long long>(j) * A.pjs;
    lane = opaque_lane(lane);
    if constexpr (MC > 0) {
        constexpr int MPL = (MC + WAVE - 1) / WAVE;   // orders per lane (L < M)
        double2 acc[MPL];
        int g0[MPL], g1[MPL];
        if (A.segbase) {                              // segment ranges, all loads first
#pragma unroll
            for (int i = 0; i < MPL; ++i) {
                const int m = min(lane + i * WAVE, A.L);
                g0[i] = A.segbase[m];
                g1[i] = A.segbase[m + 1];
            }
        } else {
#pragma unroll
            for (int i = 0; i < MPL; ++i) {
                const int m = lane + i * WAVE;
                g0[i] = m;
                g1[i] = m + 1;
            }
        }
#pragma unroll
        for (int i = 0; i < MPL; ++i) {
            if (lane + i * WAVE > A.L) g0[i] = g1[i] = 0;
        }
#pragma unroll
        for (int i = 0; i < MPL; ++i)
            acc[i] = g0[i] < g1[i] ? pf[static_cast<long long>(g0[i]) * A.pgs] : make_double2(0.0, 0.0);
        // the later segments, segment t of every order the lane holds at once
        // (one memory round trip per segment rank, not per segment); each
        // order's partials are still added in segment order
        int tmax = 0;
#pragma unroll
        for (int i = 0; i < MPL; ++i) tmax = max(tmax, g1[i] - g0[i]);
        for (int t = 1; t < tmax; ++t) {
            double2 v[MPL];
#pragma unroll
            for (int i = 0; i < MPL; ++i)
                v[i] = g0[i] + t < g1[i] ? pf[static_cast<long long>(g0[i] + t) * A.pgs] : make_double2(0.0, 0.0);
#pragma unroll
            for (int i = 0; i < MPL; ++i)
                if (g0[i] + t < g1[i]) acc[i] = cadd(acc[i], v[i]);
        }
#pragma unroll
        for (int i = 0; i < MPL; ++i) {
            const int m = lane + i * WAVE;
            if (m <= A.L) x[pad8(m)] = acc[i];
        }
    } else {
        for (int m = lane; m <= A.L; m += WAVE) {
            double2 acc = make_double2(0.0, 0.0);
            const int g1 = A.segbase ? A.segbase[m + 1] : m + 1;
            for (int g = A.segbase ? A.segbase[m] : m; g < g1; ++g) acc = cadd(acc, pf[static_cast<long long>(g) * A.pgs]);
            x[pad8(m)] = acc;
        }
    }
    wave_sync();
}

// In place on the wave's array: F_m (m <= L) -> the half-length spectrum Z of
// the inverse real FFT,
//   Z_k = (X_k + conj X_{M-k}) + i e^{2 pi i k/nlon} (X_k - conj X_{M-k}),
// X_0 taken real, X_k = 0 for k > L.  twr: e^{-2 pi i k / nlon} (padded).
template <int MC>
__device__ __forceinline__ void wave_pack_inverse(const RingArgs& A, double2* x, const double2* twr, int lane) {
    const int M = MC > 0 ? MC : A.nlon / 2;
    constexpr int KPL = ((MC > 0 ? MC : RING_MMAX_RT) + WAVE - 1) / WAVE;
    lane = opaque_lane(lane);
    // every read first, unconditionally (k and M - k stay inside the padded
    // array; entries of orders above L are replaced by zero afterwards)
    double2 xa[KPL], xb[KPL], tw[KPL];
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k0 = lane + i * WAVE;
        const int k = k0 < M ? k0 : 0;
        xa[i] = x[pad8(k)];
        xb[i] = x[pad8(M - k)];
        tw[i] = twr[k];
    }
    __builtin_amdgcn_sched_barrier(0);   // the reads stay ahead of the arithmetic
    double2 z[KPL];
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k0 = lane + i * WAVE;
        const int k = k0 < M ? k0 : 0;
        const int kr = M - k;                      // 1..M
        double2 xk = k <= A.L ? xa[i] : make_double2(0.0, 0.0);
        const double2 xr = (kr <= A.L && kr < M) ? xb[i] : make_double2(0.0, 0.0);
        if (k == 0) xk.y = 0.0;
        const double2 xrc = conj2(xr);
        const double2 sm = cadd(xk, xrc);
        const double2 df = csub(xk, xrc);
        const double2 tk = tw[i];
        const double2 t = cmul(make_double2(tk.x, -tk.y), df);   // e^{+2 pi i k / nlon} d
        z[i] = make_double2(sm.x - t.y, sm.y + t.x);             // s + i t
    }
    wave_sync();
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k = lane + i * WAVE;
        if (k < M) x[pad8(k)] = z[i];
    }
    wave_sync();
}

// From Z = FFT_M(grid row viewed as complex) in the wave's array, the
// coefficients F_m = X_m / nlon, m <= L,
//   X_m = (Z_m + conj Z_{M-m})/2 - (i/2) e^{-2 pi i m/nlon} (Z_m - conj Z_{M-m}),
// written to frow[m nlat] (order-major buffer).
template <int MC>
__device__ __forceinline__ void wave_store_forward(const RingArgs& A, const double2* x, const double2* twr,
                                                   double2* frow, int lane) {
    const int M = MC > 0 ? MC : A.nlon / 2;
    constexpr int KPL = ((MC > 0 ? MC : RING_MMAX_RT) + WAVE - 1) / WAVE;
    const double inv = 1.0 / static_cast<double>(A.nlon);
    lane = opaque_lane(lane);
    // every LDS read first (orders above L read order 0's entries, unused)
    double2 za[KPL], zb[KPL], tw[KPL];
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k0 = lane + i * WAVE;
        const int k = k0 <= A.L ? k0 : 0;
        za[i] = x[pad8(k)];
        zb[i] = x[pad8(k == 0 ? 0 : M - k)];
        tw[i] = twr[k];
    }
    __builtin_amdgcn_sched_barrier(0);   // the reads stay ahead of the arithmetic
    double2 X[KPL];
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const double2 zk = za[i];
        const double2 zr = conj2(zb[i]);
        const double2 sm = cadd(zk, zr);
        const double2 df = csub(zk, zr);
        const double2 t = cmul(tw[i], df);
        X[i] = scale2(make_double2(0.5 * (sm.x + t.y), 0.5 * (sm.y - t.x)), inv);   // (s/2 - i t/2) / nlon
    }
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k = lane + i * WAVE;
        if (k <= A.L) frow[static_cast<size_t>(k) * A.nlat] = X[i];
    }
}

// Workgroups are dispatched round-robin over the 8 XCDs: each XCD gets a
// contiguous band of latitudes, so the rings that share cache lines of the
// order-major buffers meet in one L2.
__device__ __forceinline__ int ring_of_block(int b, int nlat) {
    if (nlat % 8) return b;
    return (b % 8) * (nlat / 8) + b / 8;
}

// One workgroup per latitude ring, RING_WAVES waves, each transforming one
// field in its own LDS array with wave-local synchronisation only.
// MODE 0: inverse only (Fourier -> grid), nf fields.
// MODE 1: forward only (grid -> Fourier), nf fields.
// MODE 2: non-linear products: inverse of h, zeta, U, V (waves 0-3); pointwise
//         hU, hV, zU, zV, KE = (U^2 + V^2) / (2 cos^2 phi) (whole workgroup);
//         forward of those five (waves 0-4).
// LDS: RING_WAVES padded arrays of M complex values, then the pass twiddles
// and e^{-2 pi i k / nlon}, k < M.
template <int MODE, int MC>
__global__ __launch_bounds__(RING_WAVES * WAVE) void ring_kernel(RingArgs A) {
    extern __shared__ __align__(16) double2 lds[];
    const int M = MC > 0 ? MC : A.nlon / 2;
    const int PL = padded_len(M);
    const int j = ring_of_block(blockIdx.x, A.nlat);
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const size_t fstride = static_cast<size_t>(A.L + 1) * A.nlat;   // one field of [L+1][nlat]
    double2* tw = lds + RING_WAVES * PL;
    double2* twr = tw + M;
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
        tw[k] = make_double2(A.tw[2 * k], A.tw[2 * k + 1]);
        twr[k] = make_double2(A.twr[2 * k], A.twr[2 * k + 1]);
    }
    double2* x = lds + wv * PL;
    if constexpr (MODE == 0) {
        __syncthreads();
        for (int f = wv; f < A.nf; f += RING_WAVES) {
            wave_load_coeffs<MC>(A, f, j, x, lane);
            wave_pack_inverse<MC>(A, x, twr, lane);
            wave_fft<MC, true>(x, A, tw, lane);
            double2* g = reinterpret_cast<double2*>(A.gout + (static_cast<size_t>(f) * A.nlat + j) * A.nlon);
            for (int k = lane; k < M; k += WAVE) {
                const double2 v = x[pad8(k)];
                note_nonfinite(A.status, v.x + v.y, STATUS_TRANSFORM);
                g[k] = v;
            }
            wave_sync();
        }
    } else if constexpr (MODE == 1) {
        __syncthreads();
        for (int f = wv; f < A.nf; f += RING_WAVES) {
            const double2* g =
                reinterpret_cast<const double2*>(A.gin + (static_cast<size_t>(f) * A.nlat + j) * A.nlon);
            for (int k = lane; k < M; k += WAVE) x[pad8(k)] = g[k];
            wave_sync();
            wave_fft<MC, false>(x, A, tw, lane);
            wave_store_forward<MC>(A, x, twr, A.fout + f * fstride + j, lane);
            wave_sync();
        }
    } else {
        if (wv < 4) wave_load_coeffs<MC>(A, wv, j, x, lane);
        __syncthreads();                                   // twiddles
        if (wv < 4) {
            wave_pack_inverse<MC>(A, x, twr, lane);
            wave_fft<MC, true>(x, A, tw, lane);
        }
        __syncthreads();
        // grid values: complex slot e of an array holds the grid points 2e, 2e + 1
        const int jn = j < A.half ? j : A.nlat - 1 - j;
        const double sn = A.sint[jn];
        const double kefac = 0.5 / (sn * sn);
        const double fcor = A.two_omega * (j < A.half ? A.mu[jn] : -A.mu[jn]);   // 0 unless L_c joins N
        double2* ah = lds;                 // h  -> hU
        double2* az = lds + PL;            // zeta -> zeta U
        double2* aU = lds + 2 * PL;        // U  -> hV
        double2* aV = lds + 3 * PL;        // V  -> zeta V
        double2* ak = lds + 4 * PL;        //    -> KE
        for (int e = threadIdx.x; e < M; e += blockDim.x) {
            const int pe = pad8(e);
            const double2 u = aU[pe], v = aV[pe], hh = ah[pe], z0 = az[pe];
            const double2 zz = make_double2(z0.x + fcor, z0.y + fcor);
            ak[pe] = make_double2(__builtin_fma(u.x, u.x, v.x * v.x) * kefac, __builtin_fma(u.y, u.y, v.y * v.y) * kefac);
            aU[pe] = make_double2(hh.x * v.x, hh.y * v.y);
            aV[pe] = make_double2(zz.x * v.x, zz.y * v.y);
            ah[pe] = make_double2(hh.x * u.x, hh.y * u.y);
            az[pe] = make_double2(zz.x * u.x, zz.y * u.y);
        }
        __syncthreads();
        // output fields 0 hU, 1 hV, 2 zU, 3 zV, 4 KE: wave w transforms field w
        double2* xf = lds + (wv == 1 ? 2 : wv == 2 ? 1 : wv) * PL;
        wave_fft<MC, false>(xf, A, tw, lane);
        wave_store_forward<MC>(A, xf, twr, A.fout + wv * fstride + j, lane);
    }
}

}  // namespace

namespace {
// out = x + a y over n doubles (spectral-state combinations of the time steppers).
__global__ __launch_bounds__(256) void axpy_kernel(double* out, const double* x, double a, const double* y, int n,
                                                   unsigned* status, unsigned bit) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double v = __builtin_fma(a, y[i], x[i]);
        note_nonfinite(status, v, bit);
        out[i] = v;
    }
}
}  // namespace

int launch_axpy(double* out, const double* x, double a, const double* y, int n, unsigned* status, unsigned bit,
                hipStream_t stream) {
    hipLaunchKernelGGL(axpy_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, out, x, a, y, n, status, bit);
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
    g.status = ctx->d_status;
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
    r.status = ctx->d_status;
    return r;
}

static int ring_lds_bytes(const swe_ctx* ctx, int /*mode*/) {
    const int M = ctx->nlon / 2;
    return (RING_WAVES * padded_len(M) + 2 * M) * static_cast<int>(sizeof(double2));
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

int ring_twiddles(int M, const std::vector<int>& radix, std::vector<double>& tw) {
    // e^{-2 pi i t k / (Ns R)} = e^{-2 pi i (t k M / (Ns R)) / M}, from the
    // length-M table, at Ns - 1 + (t - 1) Ns + k for every pass (R, Ns)
    std::vector<double> full;
    build_twiddles(M, full);
    tw.assign(2 * static_cast<size_t>(M), 0.0);
    int Ns = 1;
    for (int R : radix) {
        const int twstep = M / (Ns * R);
        for (int t = 1; t < R; ++t)
            for (int k = 0; k < Ns; ++k) {
                const size_t dst = static_cast<size_t>(Ns - 1 + (t - 1) * Ns + k);
                const size_t src = static_cast<size_t>((t * k * twstep) % M);
                tw[2 * dst] = full[2 * src];
                tw[2 * dst + 1] = full[2 * src + 1];
            }
        Ns *= R;
    }
    return REXI_OK;
}

int ring_plan(int M, std::vector<int>& radix) {
    radix.clear();
    int rem = M;
    while (rem > 1) {
        const int R = ring_radix(rem);
        if (rem % R) return fail(REXI_EINVAL, "swe_create: nlon/2 must be of the form 2^a 3^b");
        radix.push_back(R);
        rem /= R;
    }
    return REXI_OK;
}

int sht_configure_kernels(swe_ctx* ctx) {
    int rc;
    const int M = ctx->nlon / 2;
    if (ring_fn<2>(M) == ring_fn<2>(0) && M > RING_MMAX_RT)
        return fail(REXI_ENOTSUP, "swe_create: nlon/2 beyond 1024 outside the compiled FFT lengths");
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
                const double* gin, double* gout, int nf, hipStream_t stream, double two_omega, bool lat_major) {
    RingArgs R = ring_args(ctx);
    R.two_omega = two_omega;
    R.part = reinterpret_cast<const double2*>(part);
    R.segbase = segbase;
    R.nseg = nseg;
    if (lat_major && (segbase || nseg != ctx->L + 1))
        return fail(REXI_EINVAL, "ring stage: latitude-major partials need one segment per order");
    R.pfs = static_cast<long long>(nseg) * ctx->nlat;
    R.pgs = lat_major ? 1 : ctx->nlat;
    R.pjs = lat_major ? nseg : 1;
    R.fout = reinterpret_cast<double2*>(fout);
    R.gin = gin;
    R.gout = gout;
    R.nf = nf;
    const size_t lds = static_cast<size_t>(ring_lds_bytes(ctx, mode));
    const int slot = prof_begin(ctx, REXI_KERNEL_RING, stream);
    const int M = ctx->nlon / 2;
    const void* fn = mode == 0 ? ring_fn<0>(M) : (mode == 1 ? ring_fn<1>(M) : ring_fn<2>(M));
    void* kargs[] = {&R};
    REXI_HIP(hipLaunchKernel(fn, dim3(ctx->nlat), dim3(RING_WAVES * WAVE), kargs, lds, stream));
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_RING, slot, stream);
    return REXI_OK;
}

}  // namespace rexi
