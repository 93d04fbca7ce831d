// Legendre stage on the matrix cores, split BF16 precision (REXI_PREC_BF16_SPLIT).
//
// For one zonal order m the Legendre transforms are dense products with the
// matrix T[l][j] = Pbar_lm(mu_j) (and H_lm(mu_j) = (1-mu_j^2) dPbar_lm/dmu for
// the vector fields) over the northern Gauss latitudes j (Section 3.2):
//   synthesis  F[j][c] = sum_l T[l][j] X[l][c]      (K = degrees)
//   analysis   O[l][c] = sum_j T[l][j] Y[j][c]      (K = latitudes)
// The degrees of each parity of l - m form their own row block (the southern
// hemisphere follows from Pbar(-mu) = (-1)^{l-m} Pbar(mu), H with the opposite
// sign), so a 16-row tile is all even or all odd.  T is tabulated once per
// context in two layouts, each in MFMA operand order (synthesis: M = latitude,
// K = degree; analysis: M = degree, K = latitude): every (tile, K step) is a
// contiguous block of 64 lanes x 16 bytes, so a wave reads one operand with one
// coalesced 1 KB load.  Every value x is stored as x_hi = bf16(x),
// x_lo = bf16(x - x_hi), interleaved in groups of four (hi[4], lo[4]); a
// product is accumulated in FP32 as a_hi b_hi + a_hi b_lo + a_lo b_hi with
// v_mfma_f32_16x16x16_bf16 (relative error about 2^-16 per product, plus FP32
// accumulation).  The table entries come from the same exponent-tracked FP64
// recurrence as the FP64 path, seeded per 64-degree segment.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace rexi {
namespace {

constexpr int WAVE = 64;
constexpr int KB_SYN = 8;    // table K steps loaded per batch, synthesis
constexpr int KB_ANA = 12;   // and analysis

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bf16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short bf16_bits(float x) {
    const unsigned u = __float_as_uint(x);
    return static_cast<unsigned short>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_value(unsigned short b) { return __uint_as_float(static_cast<unsigned>(b) << 16); }

// x -> (hi, lo), both bf16: hi = bf16(x), lo = bf16(x - hi) with the residual formed in FP64.
__device__ __forceinline__ void split_bf16(double x, unsigned short& hi, unsigned short& lo) {
    hi = bf16_bits(static_cast<float>(x));
    lo = bf16_bits(static_cast<float>(x - static_cast<double>(bf16_value(hi))));
}

// Element k of a row stored as groups of four (hi[4], lo[4]): offsets in shorts.
__device__ __forceinline__ int grp_hi(int k) { return (k >> 2) * 8 + (k & 3); }
__device__ __forceinline__ int grp_lo(int k) { return (k >> 2) * 8 + 4 + (k & 3); }

struct TabArgs {
    const int* __restrict__ seg_m;
    const int* __restrict__ seg_i0;
    const int* __restrict__ seg_n;
    const double* __restrict__ seed_pm;
    const double* __restrict__ seed_p;
    const int* __restrict__ seed_e;
    const LegCoef* __restrict__ rec;
    const double* __restrict__ mu;
    const long long* __restrict__ off;   // [L+2] start of order m in every table (shorts)
    const int* __restrict__ kp;          // [2 (L+1)] padded rows of (m, parity)
    unsigned short* __restrict__ p_syn;  // [m][parity][j][rows]  (rows in groups of 4)
    unsigned short* __restrict__ h_syn;
    unsigned short* __restrict__ p_ana;  // [m][parity][rows][j]  (latitudes in groups of 4)
    unsigned short* __restrict__ h_ana;
    int L, half, hpad, nseg;
};

// One thread per (degree segment, northern latitude): the FP64 recurrence of
// the segment, written to the four tables.  Padding rows and latitudes stay
// zero (the tables are cleared before).
__global__ __launch_bounds__(256) void leg_table_kernel(TabArgs A) {
    const int gs = blockIdx.x;
    const int j = blockIdx.y * blockDim.x + threadIdx.x;
    if (gs >= A.nseg || j >= A.half) return;
    const int m = A.seg_m[gs], i0 = A.seg_i0[gs], n = A.seg_n[gs];
    const int base = m * (2 * A.L + 3 - m) / 2;
    const size_t k = static_cast<size_t>(gs) * A.half + j;
    double pm = A.seed_pm[k], p = A.seed_p[k];
    const int e = A.seed_e[k];
    const double mu = A.mu[j];
    const int ke = A.kp[2 * m], ko = A.kp[2 * m + 1];
    for (int d = 0; d < n; ++d) {
        const int i = i0 + d;                       // l - m
        const LegCoef c = A.rec[base + i];
        const double pn = __builtin_fma(c.A * mu, p, -(c.B * pm));
        const double h = __builtin_fma(c.hA, pn, c.hB * pm);
        const double pv = ldexp(p, e), hv = ldexp(h, e);
        const int par = i & 1, r = i >> 1;
        const int K = par ? ko : ke;
        const long long blk = A.off[m] + (par ? static_cast<long long>(ke) * A.hpad * 2 : 0);
        unsigned short hi, lo;
        // operand order: each (tile, K step) holds 64 lanes x (hi[4], lo[4]), so a
        // wave's operand load is one contiguous 1 KB read
        // synthesis (M = latitude j, K = row r): lane (j % 16) + 16 ((r % 16) / 4), element r % 4
        const long long ps = blk + ((static_cast<long long>(j >> 4) * (K >> 4) + (r >> 4)) * 64 +
                                    (j & 15) + 16 * ((r & 15) >> 2)) * 8 + (r & 3);
        // analysis (M = row r, K = latitude j): lane (r % 16) + 16 ((j % 16) / 4), element j % 4
        const long long pa = blk + ((static_cast<long long>(r >> 4) * (A.hpad >> 4) + (j >> 4)) * 64 +
                                    (r & 15) + 16 * ((j & 15) >> 2)) * 8 + (j & 3);
        split_bf16(pv, hi, lo);
        A.p_syn[ps] = hi;
        A.p_syn[ps + 4] = lo;
        A.p_ana[pa] = hi;
        A.p_ana[pa + 4] = lo;
        split_bf16(hv, hi, lo);
        A.h_syn[ps] = hi;
        A.h_syn[ps + 4] = lo;
        A.h_ana[pa] = hi;
        A.h_ana[pa + 4] = lo;
        pm = p;
        p = pn;
    }
}

__device__ __forceinline__ void mfma3(f32x4& acc, const uint4& a, const uint4& b) {
    // a, b: (hi[4], lo[4]) as 16 bytes
    bf16x4 ah, al, bh, bl;
    __builtin_memcpy(&ah, &a.x, 8);
    __builtin_memcpy(&al, &a.z, 8);
    __builtin_memcpy(&bh, &b.x, 8);
    __builtin_memcpy(&bl, &b.z, 8);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
}

// v if in, else zero (component selects, so no load is made conditional)
__device__ __forceinline__ uint4 keep_if(bool in, const uint4 v) {
    return make_uint4(in ? v.x : 0u, in ? v.y : 0u, in ? v.z : 0u, in ? v.w : 0u);
}

struct MfmaArgs {
    const unsigned short* __restrict__ p_syn;
    const unsigned short* __restrict__ h_syn;
    const unsigned short* __restrict__ p_ana;
    const unsigned short* __restrict__ h_ana;
    const long long* __restrict__ off;
    const int* __restrict__ kp;
    const int* __restrict__ ablk;       // analysis workgroups: (m, first tile) pairs
    const double* __restrict__ aon;     // [L+2] a / (l(l+1))
    const double* __restrict__ noa2;    // [L+2] l(l+1) / a^2
    const double* __restrict__ sint;    // [half]
    const double* __restrict__ w;       // [half]
    int L, nlat, half, hpad, kmax, modes, nf;
    double a;
    // synthesis
    const double2* __restrict__ spec;   // KIND 0: [nf][modes]; KIND 1: state [3][modes]
    double2* __restrict__ four_out;     // [nfo][L+1][nlat]
    // analysis
    const double2* __restrict__ four_in;  // [nfi][L+1][nlat]
    double2* __restrict__ spec_out;       // KIND 0: [nf][modes]
    const double2* __restrict__ U0;       // KIND 1 epilogue, [3][modes]
    const double2* __restrict__ Nprev;
    double2* __restrict__ Nsave;
    double2* __restrict__ out;
    double c0, c1;
};

// ---------------------------------------------------------------- synthesis --
// Workgroup: order m = blockIdx.x, 4 waves = 4 tiles of 16 northern latitudes
// (tile 4 blockIdx.y + wave); KIND 0: fields 8 blockIdx.z .. 8 blockIdx.z + 7.
// LDS: the B operands X[parity][column][row] (rows in groups of four) for the
// Pbar product and (KIND 1) the H product.
template <int KIND>
__global__ __launch_bounds__(256) void leg_synth_mfma_kernel(MfmaArgs A) {
    extern __shared__ __align__(16) unsigned short xs[];
    const int m = blockIdx.x;
    const int ke = A.kp[2 * m], ko = A.kp[2 * m + 1];
    const int Lm = A.L - m + 1;
    const int base = m * (2 * A.L + 3 - m) / 2;
    const int rowlen = 2 * A.kmax;                  // shorts per LDS column row
    unsigned short* xp = xs;                        // [2][16][rowlen]
    unsigned short* xh = xs + 2 * 16 * rowlen;      // KIND 1 only
    const int f0 = KIND == 0 ? 8 * blockIdx.z : 0;
    const double dm = static_cast<double>(m);
    // stage: one thread per (parity, row) forms the row's 16 columns, zero where
    // there is no degree or column
    for (int rp = threadIdx.x; rp < 2 * A.kmax; rp += blockDim.x) {
        const int par = rp / A.kmax, r = rp - par * A.kmax;
        const int i = 2 * r + par;                  // l - m
        double vp[16], vh[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) vp[c] = vh[c] = 0.0;
        if (i < Lm) {
            const int l = m + i;
            if constexpr (KIND == 0) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (f0 + q < A.nf) {
                        const double2 v = A.spec[static_cast<size_t>(f0 + q) * A.modes + base + i];
                        vp[2 * q] = v.x;
                        vp[2 * q + 1] = v.y;
                    }
                }
            } else {
                const double2 ch = A.spec[base + i];
                const double2 cz = A.spec[A.modes + base + i];
                const double2 cd = A.spec[2 * A.modes + base + i];
                const double aon = A.aon[l], maon = dm * aon;
                // Pbar columns: h, zeta, U_P = -i delta m a/N, V_P = -i zeta m a/N
                // H columns (at the U, V positions): U_H = zeta a/N, V_H = -delta a/N
                vp[0] = ch.x;
                vp[1] = ch.y;
                vp[2] = cz.x;
                vp[3] = cz.y;
                vp[4] = cd.y * maon;
                vp[5] = -cd.x * maon;
                vp[6] = cz.y * maon;
                vp[7] = -cz.x * maon;
                vh[4] = cz.x * aon;
                vh[5] = cz.y * aon;
                vh[6] = -cd.x * aon;
                vh[7] = -cd.y * aon;
            }
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            unsigned short hi, lo;
            const int o = (par * 16 + c) * rowlen;
            split_bf16(vp[c], hi, lo);
            xp[o + grp_hi(r)] = hi;
            xp[o + grp_lo(r)] = lo;
            if constexpr (KIND == 1) {
                split_bf16(vh[c], hi, lo);
                xh[o + grp_hi(r)] = hi;
                xh[o + grp_lo(r)] = lo;
            }
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1);
    const int tile = blockIdx.y * 4 + threadIdx.x / WAVE;
    if (tile * 16 >= A.hpad) return;
    const int kq = lane >> 4;                       // K quarter of this lane
    f32x4 accP[2], accH[2];
#pragma unroll
    for (int par = 0; par < 2; ++par) {
        accP[par] = f32x4{0.f, 0.f, 0.f, 0.f};
        accH[par] = f32x4{0.f, 0.f, 0.f, 0.f};
        const int K = par ? ko : ke;
        const long long blk = A.off[m] + (par ? static_cast<long long>(ke) * A.hpad * 2 : 0);
        // operand blocks of this latitude tile: 64 lanes x 8 shorts per K step
        const unsigned short* ap = A.p_syn + blk + (static_cast<long long>(tile) * (K >> 4) * 64 + lane) * 8;
        const unsigned short* ah = A.h_syn + blk + (static_cast<long long>(tile) * (K >> 4) * 64 + lane) * 8;
        const unsigned short* bp = xp + (par * 16 + (lane & 15)) * rowlen;
        const unsigned short* bh = xh + (par * 16 + (lane & 15)) * rowlen;
        // table operands in batches of KB steps, all loads of a batch issued
        // before its products (a serial load-multiply chain leaves the
        // small-m workgroups, the longest ones, waiting on memory latency);
        // steps past the end reload the last block and multiply a zero operand
        const int nks = K >> 4;
        for (int k0 = 0; k0 < nks; k0 += KB_SYN) {
            uint4 a[KB_SYN], a2[KB_SYN];
#pragma unroll
            for (int u = 0; u < KB_SYN; ++u) {
                const int ks = min(k0 + u, nks - 1);
                a[u] = *reinterpret_cast<const uint4*>(ap + ks * 512);
                if constexpr (KIND == 1) a2[u] = *reinterpret_cast<const uint4*>(ah + ks * 512);
            }
            __builtin_amdgcn_sched_barrier(0);   // keep the batch's loads ahead of its products
#pragma unroll
            for (int u = 0; u < KB_SYN; ++u) {
                const bool in = k0 + u < nks;
                const int g = 4 * min(k0 + u, nks - 1) + kq;   // group of four rows for this lane
                const uint4 b = keep_if(in, *reinterpret_cast<const uint4*>(bp + 8 * g));
                mfma3(accP[par], a[u], b);
                if constexpr (KIND == 1) {
                    const uint4 b2 = keep_if(in, *reinterpret_cast<const uint4*>(bh + 8 * g));
                    mfma3(accH[par], a2[u], b2);
                }
            }
        }
    }
    // lane holds column c = lane % 16 of rows (latitudes) 4 (lane / 16) + t; the
    // imaginary part (odd column) moves to the real part's lane, which writes the
    // complex value into row (field, m) of the Fourier buffer [nfo][L+1][nlat]
    const int c = lane & 15;
    const int f = KIND == 0 ? f0 + (c >> 1) : (c >> 1);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float e = accP[0][t] + accH[1][t], o = accP[1][t] + accH[0][t];   // even, odd in mu
        const double vn = static_cast<double>(e) + static_cast<double>(o);
        const double vs = static_cast<double>(e) - static_cast<double>(o);
        const double vn_im = __shfl(vn, lane + 1 < WAVE ? lane + 1 : lane);
        const double vs_im = __shfl(vs, lane + 1 < WAVE ? lane + 1 : lane);
        const int j = tile * 16 + 4 * kq + t;
        const bool col_ok = (c & 1) == 0 && (KIND == 0 ? (f < A.nf) : (c < 8));
        if (!col_ok || j >= A.half) continue;
        double2* row = A.four_out + (static_cast<size_t>(f) * (A.L + 1) + m) * A.nlat;
        row[j] = make_double2(vn, vn_im);
        row[A.nlat - 1 - j] = make_double2(vs, vs_im);
    }
}

// ----------------------------------------------------------------- analysis --
// Workgroup: (order m, first tile t0) = ablk[blockIdx.x], 4 waves = row tiles
// t0 .. t0 + 3 of 16 degrees of one parity (even-parity tiles first), so an
// order with many degrees spreads over several workgroups.  LDS: the B
// operands Y[fold][column][latitude] (latitudes in groups of four), fold 0 =
// F(mu) + F(-mu), fold 1 = F(mu) - F(-mu), weighted.
// KIND 0: O = sum_j w_j Pbar F (fields 8 blockIdx.z ..).  KIND 1: the
// non-linear tendency from the Fourier coefficients of hU, hV, zU, zV, KE:
//   Pbar columns: m hU.y, -m hU.x, m zU.y, -m zU.x, -m zV.y, m zV.x, KE.x, KE.y
//   H columns:    hV.x, hV.y, zV.x, zV.y, zU.x, zU.y
// N_h = cols 0-1, N_zeta = cols 2-3, N_delta = cols 4-5 + l(l+1)/a^2 cols 6-7,
// then out = U0 + c0 N + c1 Nprev and Nsave = N (FP64).
template <int KIND>
__global__ __launch_bounds__(256) void leg_anal_mfma_kernel(MfmaArgs A) {
    extern __shared__ __align__(16) unsigned short ys[];
    const int m = A.ablk[2 * blockIdx.x], t0 = A.ablk[2 * blockIdx.x + 1];
    const int ke = A.kp[2 * m], ko = A.kp[2 * m + 1];
    const int Lm = A.L - m + 1;
    const int base = m * (2 * A.L + 3 - m) / 2;
    const int rowlen = 2 * A.hpad;
    unsigned short* yp = ys;                        // [2][16][rowlen]
    unsigned short* yh = ys + 2 * 16 * rowlen;      // KIND 1 only
    const int f0 = KIND == 0 ? 8 * blockIdx.z : 0;
    const double dm = static_cast<double>(m);
    // stage: one thread per northern latitude forms its 16 columns for both folds
    for (int j = threadIdx.x; j < A.hpad; j += blockDim.x) {
        double sp[16], dp[16], sh[16], dh[16];   // Pbar columns (fold S, D), H columns (fold S, D)
#pragma unroll
        for (int c = 0; c < 16; ++c) sp[c] = dp[c] = sh[c] = dh[c] = 0.0;
        if (j < A.half) {
            const double wj = A.w[j];
            auto fold = [&](int f, double wt, double2& S, double2& D) {
                const double2* fr = A.four_in + (static_cast<size_t>(f) * (A.L + 1) + m) * A.nlat;
                const double2 nn = fr[j];
                const double2 ss = fr[A.nlat - 1 - j];
                S = make_double2((nn.x + ss.x) * wt, (nn.y + ss.y) * wt);
                D = make_double2((nn.x - ss.x) * wt, (nn.y - ss.y) * wt);
            };
            if constexpr (KIND == 0) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (f0 + q < A.nf) {
                        double2 S, D;
                        fold(f0 + q, wj, S, D);
                        sp[2 * q] = S.x;
                        sp[2 * q + 1] = S.y;
                        dp[2 * q] = D.x;
                        dp[2 * q + 1] = D.y;
                    }
                }
            } else {
                const double wdiv = wj / (A.a * A.sint[j] * A.sint[j]);
                double2 hUs, hUd, hVs, hVd, zUs, zUd, zVs, zVd, kes, ked;
                fold(0, wdiv, hUs, hUd);
                fold(1, wdiv, hVs, hVd);
                fold(2, wdiv, zUs, zUd);
                fold(3, wdiv, zVs, zVd);
                fold(4, wj, kes, ked);
                sp[0] = dm * hUs.y;  dp[0] = dm * hUd.y;  sh[0] = hVs.x; dh[0] = hVd.x;
                sp[1] = -dm * hUs.x; dp[1] = -dm * hUd.x; sh[1] = hVs.y; dh[1] = hVd.y;
                sp[2] = dm * zUs.y;  dp[2] = dm * zUd.y;  sh[2] = zVs.x; dh[2] = zVd.x;
                sp[3] = -dm * zUs.x; dp[3] = -dm * zUd.x; sh[3] = zVs.y; dh[3] = zVd.y;
                sp[4] = -dm * zVs.y; dp[4] = -dm * zVd.y; sh[4] = zUs.x; dh[4] = zUd.x;
                sp[5] = dm * zVs.x;  dp[5] = dm * zVd.x;  sh[5] = zUs.y; dh[5] = zUd.y;
                sp[6] = kes.x;       dp[6] = ked.x;
                sp[7] = kes.y;       dp[7] = ked.y;
            }
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            unsigned short hi, lo;
            const int o0 = c * rowlen, o1 = (16 + c) * rowlen;
            split_bf16(sp[c], hi, lo);
            yp[o0 + grp_hi(j)] = hi;
            yp[o0 + grp_lo(j)] = lo;
            split_bf16(dp[c], hi, lo);
            yp[o1 + grp_hi(j)] = hi;
            yp[o1 + grp_lo(j)] = lo;
            if constexpr (KIND == 1) {
                split_bf16(sh[c], hi, lo);
                yh[o0 + grp_hi(j)] = hi;
                yh[o0 + grp_lo(j)] = lo;
                split_bf16(dh[c], hi, lo);
                yh[o1 + grp_hi(j)] = hi;
                yh[o1 + grp_lo(j)] = lo;
            }
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1);
    const int te = ke / 16, to = ko / 16;
    const int tile = t0 + static_cast<int>(threadIdx.x) / WAVE;
    if (tile < te + to) {
        const int par = tile < te ? 0 : 1;
        const int r0 = (par ? tile - te : tile) * 16;
        const long long blk = A.off[m] + (par ? static_cast<long long>(ke) * A.hpad * 2 : 0);
        const int kq = lane >> 4;
        // operand blocks of this row tile: 64 lanes x 8 shorts per K step
        const unsigned short* ap = A.p_ana + blk + (static_cast<long long>(r0 >> 4) * (A.hpad >> 4) * 64 + lane) * 8;
        const unsigned short* ah = A.h_ana + blk + (static_cast<long long>(r0 >> 4) * (A.hpad >> 4) * 64 + lane) * 8;
        // Pbar of parity par pairs with fold par; H (opposite parity) with fold 1 - par
        const unsigned short* bp = yp + (par * 16 + (lane & 15)) * rowlen;
        const unsigned short* bh = yh + ((1 - par) * 16 + (lane & 15)) * rowlen;
        f32x4 accP = {0.f, 0.f, 0.f, 0.f}, accH = {0.f, 0.f, 0.f, 0.f};
        // table operands in batches of KB steps (loads first, then products)
        const int nks = A.hpad >> 4;
        for (int k0 = 0; k0 < nks; k0 += KB_ANA) {
            uint4 a[KB_ANA], a2[KB_ANA];
#pragma unroll
            for (int u = 0; u < KB_ANA; ++u) {
                const int js = min(k0 + u, nks - 1);
                a[u] = *reinterpret_cast<const uint4*>(ap + js * 512);
                if constexpr (KIND == 1) a2[u] = *reinterpret_cast<const uint4*>(ah + js * 512);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < KB_ANA; ++u) {
                const bool in = k0 + u < nks;
                const int g = 4 * min(k0 + u, nks - 1) + kq;
                const uint4 b = keep_if(in, *reinterpret_cast<const uint4*>(bp + 8 * g));
                mfma3(accP, a[u], b);
                if constexpr (KIND == 1) {
                    const uint4 b2 = keep_if(in, *reinterpret_cast<const uint4*>(bh + 8 * g));
                    mfma3(accH, a2[u], b2);
                }
            }
        }
        const int c = lane & 15;
        float ke_t[4];
        if constexpr (KIND == 1) {
            // the KE columns 6, 7 are added to columns 4, 5 (same rows, two lanes up)
#pragma unroll
            for (int t = 0; t < 4; ++t) ke_t[t] = __shfl(accP[t], lane + 2 < WAVE ? lane + 2 : lane);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int r = r0 + 4 * kq + t;
            const int i = 2 * r + par;                  // l - m
            if (i >= Lm) continue;
            const size_t idx = static_cast<size_t>(base) + i;
            if constexpr (KIND == 0) {
                const int f = f0 + (c >> 1);
                if (f >= A.nf) continue;
                reinterpret_cast<double*>(A.spec_out + static_cast<size_t>(f) * A.modes + idx)[c & 1] =
                    static_cast<double>(accP[t]);
            } else {
                if (c >= 6) continue;
                double v = static_cast<double>(accP[t]) + static_cast<double>(accH[t]);
                if (c >= 4) v = __builtin_fma(A.noa2[m + i], static_cast<double>(ke_t[t]), v);
                const int f = c >> 1, part = c & 1;
                const size_t e2 = (static_cast<size_t>(f) * A.modes + idx) * 2 + part;
                double o = __builtin_fma(A.c0, v, A.U0 ? reinterpret_cast<const double*>(A.U0)[e2] : 0.0);
                if (A.Nprev) o = __builtin_fma(A.c1, reinterpret_cast<const double*>(A.Nprev)[e2], o);
                if (A.Nsave) reinterpret_cast<double*>(A.Nsave)[e2] = v;
                reinterpret_cast<double*>(A.out)[e2] = o;
            }
        }
    }
}

MfmaArgs mfma_args(const swe_ctx* ctx) {
    MfmaArgs A{};
    A.p_syn = ctx->d_tab_psyn;
    A.h_syn = ctx->d_tab_hsyn;
    A.p_ana = ctx->d_tab_pana;
    A.h_ana = ctx->d_tab_hana;
    A.off = ctx->d_tab_off;
    A.kp = ctx->d_tab_kp;
    A.ablk = ctx->d_tab_ablk;
    A.aon = ctx->d_aon;
    A.noa2 = ctx->d_noa2;
    A.sint = ctx->d_sint;
    A.w = ctx->d_w;
    A.L = ctx->L;
    A.nlat = ctx->nlat;
    A.half = ctx->nlat / 2;
    A.hpad = ctx->tab_hpad;
    A.kmax = ctx->tab_kmax;
    A.modes = ctx->modes;
    A.a = ctx->a;
    return A;
}

int allow_dyn_lds(const void* fn, size_t bytes) {
    if (bytes > 160 * 1024) return fail(REXI_ENOTSUP, "split-precision Legendre: LDS need exceeds 160 KB");
    if (bytes > 64 * 1024 &&
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(REXI_ENOTSUP, "split-precision Legendre: LDS need exceeds the device limit");
    }
    return REXI_OK;
}

}  // namespace

int build_split_tables(swe_ctx* ctx, hipStream_t stream) {
    TabArgs T;
    T.seg_m = ctx->d_seg_m;
    T.seg_i0 = ctx->d_seg_i0;
    T.seg_n = ctx->d_seg_n;
    T.seed_pm = ctx->d_seed_pm;
    T.seed_p = ctx->d_seed_p;
    T.seed_e = ctx->d_seed_e;
    T.rec = ctx->d_rec;
    T.mu = ctx->d_mu;
    T.off = ctx->d_tab_off;
    T.kp = ctx->d_tab_kp;
    T.p_syn = ctx->d_tab_psyn;
    T.h_syn = ctx->d_tab_hsyn;
    T.p_ana = ctx->d_tab_pana;
    T.h_ana = ctx->d_tab_hana;
    T.L = ctx->L;
    T.half = ctx->nlat / 2;
    T.hpad = ctx->tab_hpad;
    T.nseg = ctx->nseg;
    const size_t bytes = sizeof(unsigned short) * static_cast<size_t>(ctx->tab_len);
    for (unsigned short* p : {ctx->d_tab_psyn, ctx->d_tab_hsyn, ctx->d_tab_pana, ctx->d_tab_hana})
        REXI_HIP(hipMemsetAsync(p, 0, bytes, stream));
    hipLaunchKernelGGL(leg_table_kernel, dim3(ctx->nseg, (T.half + 255) / 256), dim3(256), 0, stream, T);
    REXI_HIP(hipGetLastError());
    return REXI_OK;
}

int launch_legendre_synth_split(swe_ctx* ctx, int kind, const double* spec, double* four, int nf,
                                hipStream_t stream) {
    MfmaArgs A = mfma_args(ctx);
    A.spec = reinterpret_cast<const double2*>(spec);
    A.four_out = reinterpret_cast<double2*>(four);
    A.nf = nf;
    const size_t lds = sizeof(unsigned short) * 2 * 16 * 2 * static_cast<size_t>(A.kmax) * (kind == 0 ? 1 : 2);
    const int tiles = A.hpad / 16;
    const dim3 grid(ctx->L + 1, (tiles + 3) / 4, kind == 0 ? (nf + 7) / 8 : 1);
    int rc;
    const void* fn = kind == 0 ? reinterpret_cast<const void*>(&leg_synth_mfma_kernel<0>)
                               : reinterpret_cast<const void*>(&leg_synth_mfma_kernel<1>);
    if ((rc = allow_dyn_lds(fn, lds)) != REXI_OK) return rc;
    const int slot = prof_begin(ctx, REXI_KERNEL_LEG_SYNTH, stream);
    if (kind == 0)
        hipLaunchKernelGGL(leg_synth_mfma_kernel<0>, grid, dim3(256), lds, stream, A);
    else
        hipLaunchKernelGGL(leg_synth_mfma_kernel<1>, grid, dim3(256), lds, stream, A);
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_LEG_SYNTH, slot, stream);
    return REXI_OK;
}

int launch_legendre_anal_split(swe_ctx* ctx, int kind, const double* four, double* spec, int nf, const double* U0,
                               const double* Nprev, double* Nsave, double* out, double c0, double c1,
                               hipStream_t stream) {
    MfmaArgs A = mfma_args(ctx);
    A.four_in = reinterpret_cast<const double2*>(four);
    A.spec_out = reinterpret_cast<double2*>(spec);
    A.U0 = reinterpret_cast<const double2*>(U0);
    A.Nprev = reinterpret_cast<const double2*>(Nprev);
    A.Nsave = reinterpret_cast<double2*>(Nsave);
    A.out = reinterpret_cast<double2*>(out);
    A.c0 = c0;
    A.c1 = c1;
    A.nf = nf;
    const size_t lds = sizeof(unsigned short) * 2 * 16 * 2 * static_cast<size_t>(A.hpad) * (kind == 0 ? 1 : 2);
    const dim3 grid(ctx->tab_nablk, 1, kind == 0 ? (nf + 7) / 8 : 1);
    int rc;
    const void* fn = kind == 0 ? reinterpret_cast<const void*>(&leg_anal_mfma_kernel<0>)
                               : reinterpret_cast<const void*>(&leg_anal_mfma_kernel<1>);
    if ((rc = allow_dyn_lds(fn, lds)) != REXI_OK) return rc;
    const int slot = prof_begin(ctx, REXI_KERNEL_LEG_ANAL, stream);
    if (kind == 0)
        hipLaunchKernelGGL(leg_anal_mfma_kernel<0>, grid, dim3(256), lds, stream, A);
    else
        hipLaunchKernelGGL(leg_anal_mfma_kernel<1>, grid, dim3(256), lds, stream, A);
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_LEG_ANAL, slot, stream);
    return REXI_OK;
}

}  // namespace rexi
