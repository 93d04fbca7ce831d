// Legendre stage on the matrix cores, split 16-bit precision: BF16
// (REXI_PREC_BF16_SPLIT) or FP16 (REXI_PREC_FP16_SPLIT).
//
// For one zonal order m the Legendre transforms are dense products with the
// matrix T[l][j] = Pbar_lm(mu_j) over the northern Gauss latitudes j
// (Section 3.2):
//   synthesis  F[j][c] = sum_l T[l][j] X[l][c]      (K = degrees)
//   analysis   O[l][c] = sum_j T[l][j] Y[j][c]      (K = latitudes)
// The vector fields also need H_lm = (1-mu^2) dPbar_lm/dmu, which the degree
// recurrence gives as H_l = hA_l Pbar_{l+1} + hB_l Pbar_{l-1}.  No H table is
// kept: the synthesis moves the two terms onto the coefficients
// (sum_l H_l X_l = sum_l Pbar_l (hA_{l-1} X_{l-1} + hB_{l+1} X_{l+1})), and the
// analysis forms sum_j Pbar_l Y_j for every degree up to L+1 and combines the
// rows l+1 and l-1 afterwards.  The degrees of each parity of l - m form their
// own row block (the southern hemisphere follows from
// Pbar(-mu) = (-1)^{l-m} Pbar(mu)), so a 16-row tile is all even or all odd.
// T is tabulated once per context, degrees m .. L+1, in two layouts, each in
// MFMA operand order (synthesis: M = latitude, K = degree; analysis: M =
// degree, K = latitude): every (tile, K step) is a contiguous block of 64 lanes
// x 16 bytes, so a wave reads one operand with one coalesced 1 KB load.  Every
// value x is stored as x_hi = t(x), x_lo = t(x - x_hi) for the 16-bit type t,
// interleaved in groups of four (hi[4], lo[4]); a product is accumulated in
// FP32 as a_hi b_hi + a_hi b_lo + a_lo b_hi with v_mfma_f32_16x16x16_bf16 or
// _f16 (relative error about 2^-16 per product for BF16, 2^-22 for FP16, plus
// FP32 accumulation).  FP16's exponent range is narrow, so in FP16 mode every
// column of the data operand is scaled by a power of two that brings its
// largest magnitude into [1/2, 1) (exact; undone on the FP32 sums), and the
// table entries (|Pbar| < 64) fit as they are.  The table entries
// come from the same exponent-tracked FP64 recurrence as the FP64 path, seeded
// per 64-degree segment.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace rexi {
namespace {

constexpr int WAVE = 64;
constexpr int KB_SYN = 9;    // table K steps loaded per batch, synthesis (T255: one batch)
constexpr int KB_ANA = 12;   // and analysis
constexpr int SYN_THREADS = 256;   // synthesis block size (4 latitude tiles)
constexpr int ANA_WAVES = 16;      // analysis (and per-order synthesis) waves per workgroup
constexpr int ANA_THREADS = ANA_WAVES * WAVE;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
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

// x -> (hi, lo), both fp16: hi = fp16(x), lo = fp16(x - hi), residual in FP64.
__device__ __forceinline__ void split_f16(double x, unsigned short& hi, unsigned short& lo) {
    const _Float16 h = static_cast<_Float16>(x);
    const _Float16 l = static_cast<_Float16>(x - static_cast<double>(h));
    __builtin_memcpy(&hi, &h, 2);
    __builtin_memcpy(&lo, &l, 2);
}

// The 16-bit operand type of a split Legendre stage.
struct Bf16 {};
struct F16 {};

template <class E>
__device__ __forceinline__ void split16(double x, unsigned short& hi, unsigned short& lo) {
    if constexpr (std::is_same<E, F16>::value) split_f16(x, hi, lo); else split_bf16(x, hi, lo);
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
    unsigned short* __restrict__ p_ana;  // [m][parity][rows][j]  (latitudes in groups of 4)
    int L, half, hpad, nseg;
};

// Pbar_lm(mu_j) (row i = l - m) into both tables, split into 16-bit hi and lo.
template <class E>
__device__ __forceinline__ void put_entry(const TabArgs& A, int m, int i, int j, double v) {
    const int ke = A.kp[2 * m], ko = A.kp[2 * m + 1];
    const int par = i & 1, r = i >> 1;
    const int K = par ? ko : ke;
    const long long blk = A.off[m] + (par ? static_cast<long long>(ke) * A.hpad * 2 : 0);
    // operand order: each (tile, K step) holds 64 lanes x (hi[4], lo[4]), so a
    // wave's operand load is one contiguous 1 KB read
    // synthesis (M = latitude j, K = row r): lane (j % 16) + 16 ((r % 16) / 4), element r % 4
    const long long ps = blk + ((static_cast<long long>(j >> 4) * (K >> 4) + (r >> 4)) * 64 + (j & 15) +
                                16 * ((r & 15) >> 2)) * 8 + (r & 3);
    // analysis (M = row r, K = latitude j): lane (r % 16) + 16 ((j % 16) / 4), element j % 4
    const long long pa = blk + ((static_cast<long long>(r >> 4) * (A.hpad >> 4) + (j >> 4)) * 64 + (r & 15) +
                                16 * ((j & 15) >> 2)) * 8 + (j & 3);
    unsigned short hi, lo;
    split16<E>(v, hi, lo);
    A.p_syn[ps] = hi;
    A.p_syn[ps + 4] = lo;
    A.p_ana[pa] = hi;
    A.p_ana[pa + 4] = lo;
}

// One thread per (degree segment, northern latitude): the FP64 recurrence of
// the segment, written to both tables; the last segment of an order also
// writes degree L+1.  Padding rows and latitudes stay zero (the tables are
// cleared before).
template <class E>
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
    for (int d = 0; d < n; ++d) {
        const LegCoef c = A.rec[base + i0 + d];
        const double pn = __builtin_fma(c.A * mu, p, -(c.B * pm));
        put_entry<E>(A, m, i0 + d, j, ldexp(p, e));
        pm = p;
        p = pn;
    }
    if (i0 + n == A.L - m + 1) put_entry<E>(A, m, i0 + n, j, ldexp(p, e));
}

template <class E>
__device__ __forceinline__ void mfma3(f32x4& acc, const uint4& a, const uint4& b) {
    // a, b: (hi[4], lo[4]) as 16 bytes
    if constexpr (std::is_same<E, F16>::value) {
        f16x4 ah, al, bh, bl;
        __builtin_memcpy(&ah, &a.x, 8);
        __builtin_memcpy(&al, &a.z, 8);
        __builtin_memcpy(&bh, &b.x, 8);
        __builtin_memcpy(&bl, &b.z, 8);
        acc = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16f16(al, bh, acc, 0, 0, 0);
    } else {
        bf16x4 ah, al, bh, bl;
        __builtin_memcpy(&ah, &a.x, 8);
        __builtin_memcpy(&al, &a.z, 8);
        __builtin_memcpy(&bh, &b.x, 8);
        __builtin_memcpy(&bl, &b.z, 8);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
    }
}

// Per-column power-of-two scales of the data operand (FP16 mode): cmax holds
// this thread's largest |value| per column; the workgroup's maxima go through
// red ([waves][16] floats) and every thread receives sc[c] = 2^-e with
// max |column c| in [2^(e-1), 2^e) (1 for an all-zero column).  Columns NC ..
// 15 are known to be zero and are not reduced.
template <int NC, int NT>
__device__ __forceinline__ void column_scales(float* cmax, float* red, float* sc) {
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    constexpr int nw = NT / WAVE;
#pragma unroll
    for (int c = NC; c < 16; ++c) cmax[c] = 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        float v = cmax[c];
#pragma unroll
        for (int msk = 1; msk < WAVE; msk <<= 1) v = fmaxf(v, __shfl_xor(v, msk));
        cmax[c] = v;
    }
    if (lane < 16) {
        float v = 0.f;
#pragma unroll
        for (int c = 0; c < 16; ++c) v = lane == c ? cmax[c] : v;
        red[wv * 16 + lane] = v;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        float v = 0.f;
        for (int w = 0; w < nw; ++w) v = fmaxf(v, red[w * 16 + threadIdx.x]);
        int e = 0;
        if (v > 0.f) (void)frexpf(v, &e);
        sc[threadIdx.x] = ldexpf(1.0f, -max(e, -100));   // columns below 2^-101 stay unscaled
    }
    __syncthreads();
}

// Shorts per LDS row of a B operand holding n K-values (hi, lo): 4n bytes
// plus 16, so that the rows the 16 column lanes of a quarter-wave read start
// an odd number of 16-byte bank groups apart (no bank conflicts).
__host__ __device__ constexpr int lds_row(int n) { return 2 * n + 8; }

// v if in, else zero (component selects, so no load is made conditional)
__device__ __forceinline__ uint4 keep_if(bool in, const uint4 v) {
    return make_uint4(in ? v.x : 0u, in ? v.y : 0u, in ? v.z : 0u, in ? v.w : 0u);
}

struct MfmaArgs {
    const unsigned short* __restrict__ p_syn;
    const unsigned short* __restrict__ p_ana;
    const long long* __restrict__ off;
    const int* __restrict__ kp;
    const LegCoef* __restrict__ rec;    // [modes] recurrence and H coefficients
    const double* __restrict__ aon;     // [L+2] a / (l(l+1))
    const double* __restrict__ noa2;    // [L+2] l(l+1) / a^2
    const double* __restrict__ sint;    // [half]
    const double* __restrict__ w;       // [half]
    int L, nlat, half, hpad, kmax, modes, nf;
    double a;
    // synthesis
    const double2* __restrict__ spec;   // KIND 0: [nf][modes]; KIND 1: state [3][modes]
    double2* __restrict__ four_out;     // element (field, m, latitude) at f ofs + m oms + j ojs
    long long ofs;
    int oms, ojs;
    int xcd_blocks;                     // KIND 1: orders dealt to the XCDs in blocks of 8 (split_item)
    // analysis
    const double2* __restrict__ four_in;  // [nfi][L+1][nlat]
    double2* __restrict__ spec_out;       // KIND 0: [nf][modes]
    const double2* __restrict__ U0;       // KIND 1 epilogue, [3][modes]
    const double2* __restrict__ Nprev;
    double2* __restrict__ Nsave;
    double2* __restrict__ out;
    double c0, c1;
    unsigned* status;                     // non-finite outputs set a STATUS_* flag
    int ntg, ng;                          // KIND 0: latitude-tile groups, 8-field groups (split_item)
    int zreg;                             // analysis: bytes of the zs region (the fused kernel's us follows)
};

// The (order m, latitude-tile group, 8-field group) of a workgroup.  KIND 1
// (one-dimensional grid of (L+1) ntg workgroups): with xcd_blocks, the
// workgroups of each block of 8 consecutive orders run on one XCD (workgroup b
// runs on XCD b mod 8), so that the latitude-major Fourier rows they write
// together (8 orders = one 128-byte line) are completed in that XCD's L2; the
// blocks are dealt to the XCDs in snake order (x, 15 - x, 16 + x, ...) so that
// long and short orders mix on every XCD; otherwise b = m + (L+1) tg.
// KIND 0: a one-dimensional grid in which the ng
// field groups of one (order, tile group) pair p share an XCD (workgroup b runs
// on XCD b mod 8) and are dispatched within a window of 8 ng workgroups, so the
// table tiles they all read come from HBM once and then from that XCD's L2:
// b = 8 (ng (p / 8) + g) + p mod 8, pairs ordered by order (longest first).
// Returns false for the padding workgroups of the last window.
template <int KIND>
__device__ __forceinline__ bool split_item(const MfmaArgs& A, int& m, int& tg, int& g) {
    if constexpr (KIND == 1) {
        const int b = blockIdx.x;
        g = 0;
        if (A.xcd_blocks) {
            const int x = b & 7, i = b >> 3;            // XCD, slot on it
            const int per = 8 * A.ntg;                  // workgroups per block of 8 orders
            const int kb = i / per, r = i - kb * per;   // the XCD's kb-th block
            const int blk = (kb & 1) ? (kb + 1) * 8 - 1 - x : kb * 8 + x;
            m = blk * 8 + (r & 7);
            tg = r >> 3;
        } else {
            m = b % (A.L + 1);
            tg = b / (A.L + 1);
        }
        return true;
    } else {
        const int b = blockIdx.x;
        const int slot = b >> 3;
        g = slot % A.ng;
        const int p = 8 * (slot / A.ng) + (b & 7);
        m = p / A.ntg;
        tg = p - m * A.ntg;
        return m <= A.L;
    }
}

__host__ __device__ constexpr int split_grid_size(int pairs, int ng) { return (pairs + 7) / 8 * 8 * ng; }

// The 16 B-operand columns of synthesis staging row i = l - m of the state
// (i <= Lm = L - m + 1; zero where there is no degree or column): h and zeta
// (Pbar columns 0-3) and U, V (columns 4-7),
//   U_l = -i m delta_l a/N_l + hA_{l-1} zeta_{l-1} a/N_{l-1} + hB_{l+1} zeta_{l+1} a/N_{l+1},
//   V_l = -i m zeta_l a/N_l - hA_{l-1} delta_{l-1} a/N_{l-1} - hB_{l+1} delta_{l+1} a/N_{l+1}
// (N_l = l(l+1)), from v = (h, zeta, delta)_l, (zeta, delta)_{l-1},
// (zeta, delta)_{l+1} and s = a/N_l, hA_{l-1}, a/N_{l-1}, hB_{l+1}, a/N_{l+1}.
__device__ __forceinline__ void state_row_values(const double2* v, const double* s, int i, int Lm, double dm,
                                                 double* vp) {
#pragma unroll
    for (int c = 0; c < 16; ++c) vp[c] = 0.0;
    if (i > Lm) return;
    double2 U = make_double2(0.0, 0.0), V = make_double2(0.0, 0.0);
    if (i < Lm) {
        const double2 ch = v[0], cz = v[1], cd = v[2];
        const double maon = dm * s[0];
        vp[0] = ch.x;
        vp[1] = ch.y;
        vp[2] = cz.x;
        vp[3] = cz.y;
        U = make_double2(cd.y * maon, -cd.x * maon);
        V = make_double2(cz.y * maon, -cz.x * maon);
    }
    if (i >= 1) {                           // hA_{l-1} H-term of degree l-1
        const double t = s[1] * s[2];
        const double2 cz = v[3], cd = v[4];
        U = make_double2(__builtin_fma(t, cz.x, U.x), __builtin_fma(t, cz.y, U.y));
        V = make_double2(__builtin_fma(-t, cd.x, V.x), __builtin_fma(-t, cd.y, V.y));
    }
    if (i + 1 < Lm) {                       // hB_{l+1} H-term of degree l+1
        const double t = s[3] * s[4];
        const double2 cz = v[5], cd = v[6];
        U = make_double2(__builtin_fma(t, cz.x, U.x), __builtin_fma(t, cz.y, U.y));
        V = make_double2(__builtin_fma(-t, cd.x, V.x), __builtin_fma(-t, cd.y, V.y));
    }
    vp[4] = U.x;
    vp[5] = U.y;
    vp[6] = V.x;
    vp[7] = V.y;
}

// The synthesis table operands of one latitude tile of order m, per parity:
// ap[par] = first K step's block (64 lanes x 8 shorts per K step), nks[par]
// K steps; load_syn_batch reads KB_SYN steps from k0 (steps past the end
// reload the last block, which is not multiplied).
struct SynTile {
    const unsigned short* ap[2];
    int nks[2];
};

__device__ __forceinline__ SynTile syn_tile_ptrs(const MfmaArgs& A, int m, int tile, int lane) {
    SynTile T;
    const int ke = A.kp[2 * m], ko = A.kp[2 * m + 1];
    T.nks[0] = ke >> 4;
    T.nks[1] = ko >> 4;
    const long long off_m = A.off[m];
#pragma unroll
    for (int par = 0; par < 2; ++par) {
        const long long blk = off_m + (par ? static_cast<long long>(ke) * A.hpad * 2 : 0);
        T.ap[par] = A.p_syn + blk + (static_cast<long long>(tile) * T.nks[par] * 64 + lane) * 8;
    }
    return T;
}

__device__ __forceinline__ void load_syn_batch(const SynTile& T, int par, int k0, uint4* a) {
#pragma unroll
    for (int u = 0; u < KB_SYN; ++u) {
        const int ks = min(k0 + u, T.nks[par] - 1);
        a[u] = *reinterpret_cast<const uint4*>(T.ap[par] + ks * 512);
    }
}

// Products and Fourier output of one latitude tile of order m, both parities:
// xp is the B operand in LDS ([2][16][rowlen], rows in groups of four), pre
// the first table batch of each parity (requested by the caller), sc the
// column scales (FP16 mode).  Lane (c = lane % 16, K quarter kq) holds column
// c of latitudes 4 kq + t; the imaginary part (odd column) moves to the real
// part's lane, which writes the complex value of (field, m, latitude) at
// f ofs + m oms + j ojs, north and south (Pbar(-mu) = (-1)^(l-m) Pbar(mu)).
template <int KIND, class E, bool LAZY1 = false>
__device__ __forceinline__ void synth_tile(const MfmaArgs& A, int m, int tile, int f0, const SynTile& T,
                                           uint4 (&pre)[2][KB_SYN], const unsigned short* xp, int rowlen,
                                           const float* sc, int lane) {
    constexpr bool SCALED = std::is_same<E, F16>::value;
    const int kq = lane >> 4;
    f32x4 acc[2];
#pragma unroll
    for (int par = 0; par < 2; ++par) {
        acc[par] = f32x4{0.f, 0.f, 0.f, 0.f};
        const unsigned short* bp = xp + (par * 16 + (lane & 15)) * rowlen;
        // LAZY1: the odd parity's first batch is requested here, after the
        // even products (fewer registers live)
        if (LAZY1 && par == 1) load_syn_batch(T, 1, 0, pre[1]);
        // table operands in batches of KB steps, all loads of a batch issued
        // before its products (a serial load-multiply chain leaves the
        // small-m workgroups, the longest ones, waiting on memory latency);
        // pre[par] holds the current batch
        for (int k0 = 0; k0 < T.nks[par]; k0 += KB_SYN) {
            if (k0 > 0) load_syn_batch(T, par, k0, pre[par]);
            const uint4* a = pre[par];
            __builtin_amdgcn_sched_barrier(0);   // keep the batch's loads ahead of its products
#pragma unroll
            for (int u = 0; u < KB_SYN; ++u) {
                if (k0 + u < T.nks[par]) {                  // uniform: no products past the end
                    const int g = 4 * (k0 + u) + kq;        // group of four rows for this lane
                    const uint4 b = *reinterpret_cast<const uint4*>(bp + 8 * g);
                    mfma3<E>(acc[par], a[u], b);
                }
            }
        }
    }
    const int c = lane & 15;
    const int f = KIND == 0 ? f0 + (c >> 1) : (c >> 1);
    const double unscale = SCALED ? 1.0 / static_cast<double>(sc[c]) : 1.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float e = acc[0][t], o = acc[1][t];   // even, odd in mu
        const double vn = (static_cast<double>(e) + static_cast<double>(o)) * unscale;
        const double vs = (static_cast<double>(e) - static_cast<double>(o)) * unscale;
        const double vn_im = __shfl(vn, lane + 1 < WAVE ? lane + 1 : lane);
        const double vs_im = __shfl(vs, lane + 1 < WAVE ? lane + 1 : lane);
        const int j = tile * 16 + 4 * kq + t;
        const bool col_ok = (c & 1) == 0 && (KIND == 0 ? (f < A.nf) : (c < 8));
        if (!col_ok || j >= A.half) continue;
        double2* row = A.four_out + f * A.ofs + static_cast<long long>(m) * A.oms;
        row[static_cast<long long>(j) * A.ojs] = make_double2(vn, vn_im);
        row[static_cast<long long>(A.nlat - 1 - j) * A.ojs] = make_double2(vs, vs_im);
    }
}

// ---------------------------------------------------------------- synthesis --
// Workgroup (split_item): order m, 4 waves = 4 tiles of 16 northern latitudes
// (tile 4 tg + wave); KIND 0: fields 8 g .. 8 g + 7.
// LDS: the B operand X[parity][column][row] (rows in groups of four).
// KIND 1 columns: h, zeta, U, V (real and imaginary parts), with
//   U_l = -i m delta_l a/N_l + hA_{l-1} zeta_{l-1} a/N_{l-1} + hB_{l+1} zeta_{l+1} a/N_{l+1},
//   V_l = -i m zeta_l a/N_l - hA_{l-1} delta_{l-1} a/N_{l-1} - hB_{l+1} delta_{l+1} a/N_{l+1}
// (N_l = l(l+1)), rows up to degree L+1.
template <int KIND, class E>
__global__ __launch_bounds__(SYN_THREADS) void leg_synth_mfma_kernel(MfmaArgs A) {
    extern __shared__ __align__(16) unsigned short xs[];
    constexpr bool SCALED = std::is_same<E, F16>::value;
    __shared__ float sred[4 * 16], sc[16];
    int m, tg, g;
    if (!split_item<KIND>(A, m, tg, g)) return;
    const int Lm = A.L - m + 1;
    const int base = m * (2 * A.L + 3 - m) / 2;
    const int rowlen = lds_row(A.kmax);             // shorts per LDS column row
    unsigned short* xp = xs;                        // [2][16][rowlen]
    const int f0 = 8 * g;
    const double dm = static_cast<double>(m);
    const int lane = threadIdx.x & (WAVE - 1);
    const int tile = tg * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);   // wave-uniform
    const bool active = tile * 16 < A.hpad;
    // The first table batch of the even parity is requested before the
    // staging and that of the odd parity after it, so that their memory
    // latency overlaps the staging's and the even products (both before the
    // staging would hold too many registers for three workgroups per CU).
    const SynTile T = syn_tile_ptrs(A, m, active ? tile : 0, lane);
    uint4 pre[2][KB_SYN];
    if (active) load_syn_batch(T, 0, 0, pre[0]);
    // Staging row rp = (parity, row r), degree l = m + 2 r + parity.  Its
    // inputs are loaded with indices clamped into the order (straight-line
    // code, so that the loads of a thread's rows are in flight together);
    // row_values then forms the 16 column values, zero where there is no
    // degree or column.
    struct RowIn {
        double2 v[8];   // KIND 0: fields f0 .. f0+7; KIND 1: (h, zeta, delta)_l, (zeta, delta)_{l-1}, (zeta, delta)_{l+1}
        double s[5];    // KIND 1: a/N_l, hA_{l-1}, a/N_{l-1}, hB_{l+1}, a/N_{l+1}
    };
    auto row_load = [&](int rp, RowIn& in) {
        const int par = rp / A.kmax, r = rp - par * A.kmax;
        const int i = 2 * r + par;                  // l - m
        const int ic = min(i, Lm - 1);
        if constexpr (KIND == 0) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int fq = min(f0 + q, A.nf - 1);
                in.v[q] = A.spec[static_cast<size_t>(fq) * A.modes + base + ic];
            }
        } else {
            const int id = max(min(i - 1, Lm - 1), 0), iu = min(i + 1, Lm - 1);
            in.v[0] = A.spec[base + ic];
            in.v[1] = A.spec[A.modes + base + ic];
            in.v[2] = A.spec[2 * A.modes + base + ic];
            in.v[3] = A.spec[A.modes + base + id];
            in.v[4] = A.spec[2 * A.modes + base + id];
            in.v[5] = A.spec[A.modes + base + iu];
            in.v[6] = A.spec[2 * A.modes + base + iu];
            in.s[0] = A.aon[m + ic];
            in.s[1] = A.rec[base + id].hA;
            in.s[2] = A.aon[m + id];
            in.s[3] = A.rec[base + iu].hB;
            in.s[4] = A.aon[m + iu];
        }
    };
    auto row_values = [&](int rp, const RowIn& in, double* vp) {
        const int par = rp / A.kmax, r = rp - par * A.kmax;
        const int i = 2 * r + par;                  // l - m
        if constexpr (KIND == 0) {
#pragma unroll
            for (int c = 0; c < 16; ++c) vp[c] = 0.0;
            if (i < Lm) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (f0 + q < A.nf) {
                        vp[2 * q] = in.v[q].x;
                        vp[2 * q + 1] = in.v[q].y;
                    }
                }
            }
        } else {
            state_row_values(in.v, in.s, i, Lm, dm, vp);
        }
    };
    // every thread takes rows rp and rp + SYN_THREADS of each 2 SYN_THREADS
    const int nrows = 2 * A.kmax;
    constexpr int bd = SYN_THREADS;
    if constexpr (SCALED) {
        // the values go to LDS as FP32 (24 bits, more than the split keeps)
        // with their column maxima; then they are scaled and split
        float* stage = reinterpret_cast<float*>(xs + 2 * 16 * rowlen);   // [16][2 kmax]
        float cmax[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) cmax[c] = 0.f;
        auto put = [&](int rp, const RowIn& in) {
            double vp[16];
            row_values(rp, in, vp);
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const float v = static_cast<float>(vp[c]);
                stage[c * 2 * A.kmax + rp] = v;
                cmax[c] = fmaxf(cmax[c], fabsf(v));
            }
        };
        for (int rp = threadIdx.x; rp < nrows; rp += 2 * bd) {
            RowIn in0, in1;
            row_load(rp, in0);
            row_load(min(rp + bd, nrows - 1), in1);
            put(rp, in0);
            if (rp + bd < nrows) put(rp + bd, in1);
        }
        if (active) load_syn_batch(T, 1, 0, pre[1]);
        column_scales<KIND == 0 ? 16 : 8, SYN_THREADS>(cmax, sred, sc);
        for (int rp = threadIdx.x; rp < nrows; rp += bd) {
            const int par = rp / A.kmax, r = rp - par * A.kmax;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                unsigned short hi, lo;
                const int o = (par * 16 + c) * rowlen;
                split16<E>(static_cast<double>(stage[c * 2 * A.kmax + rp] * sc[c]), hi, lo);
                xp[o + grp_hi(r)] = hi;
                xp[o + grp_lo(r)] = lo;
            }
        }
    } else {
        // stage: the row's 16 columns, split, into the B operand
        auto put = [&](int rp, const RowIn& in) {
            const int par = rp / A.kmax, r = rp - par * A.kmax;
            double vp[16];
            row_values(rp, in, vp);
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                unsigned short hi, lo;
                const int o = (par * 16 + c) * rowlen;
                split16<E>(vp[c], hi, lo);
                xp[o + grp_hi(r)] = hi;
                xp[o + grp_lo(r)] = lo;
            }
        };
        for (int rp = threadIdx.x; rp < nrows; rp += 2 * bd) {
            RowIn in0, in1;
            row_load(rp, in0);
            row_load(min(rp + bd, nrows - 1), in1);
            put(rp, in0);
            if (rp + bd < nrows) put(rp + bd, in1);
        }
    }
    if (!SCALED && active) load_syn_batch(T, 1, 0, pre[1]);
    __syncthreads();
    if (!active) return;
    synth_tile<KIND, E>(A, m, tile, f0, T, pre, xp, rowlen, sc, lane);
}

// The synthesis factors of staging row rp = (parity, row r), degree
// l = m + 2 r + parity (indices clamped into the order): a/N_l, hA_{l-1},
// a/N_{l-1}, hB_{l+1}, a/N_{l+1}.
__device__ __forceinline__ void syn_factors(const MfmaArgs& A, int m, int rp, double* sf) {
    const int Lm = A.L - m + 1;
    const int base = m * (2 * A.L + 3 - m) / 2;
    const int par = rp / A.kmax, r = rp - par * A.kmax;
    const int i = 2 * r + par;
    const int ic = min(i, Lm - 1), id = max(min(i - 1, Lm - 1), 0), iu = min(i + 1, Lm - 1);
    sf[0] = A.aon[m + ic];
    sf[1] = A.rec[base + id].hA;
    sf[2] = A.aon[m + id];
    sf[3] = A.rec[base + iu].hB;
    sf[4] = A.aon[m + iu];
}

// Synthesis of the state of order m for every latitude by a workgroup of
// ANA_THREADS threads, from its coefficients us in LDS ([L-m+1][3] complex:
// h, zeta, delta; complete before the call).  syn_s holds the synthesis
// factors of the thread's first staging row (syn_factors, threads < 2 kmax).
// LDS: the B operand goes to ys ([2][16][lds_row(kmax)] shorts), FP16 mode
// stages FP32 values in zs ([16][2 kmax] floats); sred and sc take the column
// scales.  The waves take the latitude tiles in turn; the Fourier coefficients
// go to four_out (f ofs + m oms + j ojs).
template <class E>
__device__ void synth_state_block(const MfmaArgs& A, int m, const double* us, const double* syn_s,
                                  unsigned short* ys, float* zs, float* sred, float* sc) {
    constexpr bool SCALED = std::is_same<E, F16>::value;
    const int Lm = A.L - m + 1;
    const double dm = static_cast<double>(m);
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int ntile = A.hpad / 16;
    SynTile T = syn_tile_ptrs(A, m, wv < ntile ? wv : 0, lane);
    uint4 pre[2][KB_SYN];
    // staging row rp = (parity, row r), degree l = m + 2 r + parity, from us
    const int srow = lds_row(A.kmax);
    unsigned short* xp = ys;                   // [2][16][srow]
    auto row_in = [&](int rp, double2* v) {
        const int par = rp / A.kmax, r = rp - par * A.kmax;
        const int i = 2 * r + par;
        const int ic = min(i, Lm - 1), id = max(min(i - 1, Lm - 1), 0), iu = min(i + 1, Lm - 1);
        const double2* u2 = reinterpret_cast<const double2*>(us);   // [Lm][3] complex
        v[0] = u2[3 * ic];
        v[1] = u2[3 * ic + 1];
        v[2] = u2[3 * ic + 2];
        v[3] = u2[3 * id + 1];
        v[4] = u2[3 * id + 2];
        v[5] = u2[3 * iu + 1];
        v[6] = u2[3 * iu + 2];
        return i;
    };
    if constexpr (SCALED) {
        float* stage = zs;                     // [16][2 kmax] FP32
        float cmax[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) cmax[c] = 0.f;
        for (int rp = threadIdx.x; rp < 2 * A.kmax; rp += ANA_THREADS) {
            double sf[5], vp[16];
            double2 v[7];
            if (rp == static_cast<int>(threadIdx.x)) {
#pragma unroll
                for (int q = 0; q < 5; ++q) sf[q] = syn_s[q];
            } else {
                syn_factors(A, m, rp, sf);
            }
            const int i = row_in(rp, v);
            state_row_values(v, sf, i, Lm, dm, vp);
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const float fv = static_cast<float>(vp[c]);
                stage[c * 2 * A.kmax + rp] = fv;
                cmax[c] = fmaxf(cmax[c], fabsf(fv));
            }
        }
        column_scales<8, ANA_THREADS>(cmax, sred, sc);
        for (int rp = threadIdx.x; rp < 2 * A.kmax; rp += ANA_THREADS) {
            const int par = rp / A.kmax, r = rp - par * A.kmax;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                unsigned short hi, lo;
                const int o = (par * 16 + c) * srow;
                split16<E>(static_cast<double>(stage[c * 2 * A.kmax + rp] * sc[c]), hi, lo);
                xp[o + grp_hi(r)] = hi;
                xp[o + grp_lo(r)] = lo;
            }
        }
    } else {
        for (int rp = threadIdx.x; rp < 2 * A.kmax; rp += ANA_THREADS) {
            double sf[5], vp[16];
            double2 v[7];
            if (rp == static_cast<int>(threadIdx.x)) {
#pragma unroll
                for (int q = 0; q < 5; ++q) sf[q] = syn_s[q];
            } else {
                syn_factors(A, m, rp, sf);
            }
            const int i = row_in(rp, v);
            state_row_values(v, sf, i, Lm, dm, vp);
            const int par = rp / A.kmax, r = rp - par * A.kmax;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                unsigned short hi, lo;
                const int o = (par * 16 + c) * srow;
                split16<E>(vp[c], hi, lo);
                xp[o + grp_hi(r)] = hi;
                xp[o + grp_lo(r)] = lo;
            }
        }
    }
    // the even parity's first table batch of the wave's first tile
    if (wv < ntile) load_syn_batch(T, 0, 0, pre[0]);
    __syncthreads();
    for (int tile = wv; tile < ntile; tile += ANA_WAVES) {
        if (tile != wv) {
            T = syn_tile_ptrs(A, m, tile, lane);
            load_syn_batch(T, 0, 0, pre[0]);
        }
        synth_tile<1, E, true>(A, m, tile, 0, T, pre, xp, srow, sc, lane);
    }
}

// ----------------------------------------------------------------- analysis --
// Workgroup (split_item, one tile group): order m, ANA_WAVES waves taking the row tiles of 16
// degrees of one parity (even-parity tiles first) in turn.  LDS: the B operand
// Y[fold][column][latitude] (latitudes in groups of four), fold 0 =
// F(mu) + F(-mu), fold 1 = F(mu) - F(-mu), weighted; rows of a parity pair
// with the fold of that parity.  KIND 0: O = sum_j w_j Pbar F (fields
// 8 g ..), written from the accumulators.  KIND 1: the non-linear
// tendency from the Fourier coefficients of hU, hV, zU, zV, KE:
//   columns 0-7 (Pbar terms): m hU.y, -m hU.x, m zU.y, -m zU.x, -m zV.y, m zV.x, KE.x, KE.y
//   columns 8-13 (H terms):   hV.x, hV.y, zV.x, zV.y, zU.x, zU.y
// The products Z[l][c] of every degree up to L+1 go to LDS; then output
// column k (0-5) of degree l is
//   Z[l][k] + hA_l Z[l+1][8+k] + hB_l Z[l-1][8+k] (+ l(l+1)/a^2 Z[l][k+2], k >= 4)
// giving N_h (k 0-1), N_zeta (2-3), N_delta (4-5); then out = U0 + c0 N + c1 Nprev
// and Nsave = N (FP64).

// FUSE (KIND 1 only): the workgroup then synthesises the outputs of its order
// for the next evaluation (the stage-1 state of a Heun step): they stay in LDS
// (us, [L-m+1][6] doubles, after zs), the synthesis B operand is staged from
// them into the region of yp (kmax <= hpad) and the waves take the latitude
// tiles in turn; the Fourier coefficients go latitude-major to four_out (A.ofs,
// A.oms, A.ojs) and out is written only if non-null.
template <int KIND, class E, bool FUSE = false>
__global__ __launch_bounds__(ANA_WAVES * WAVE) void leg_anal_mfma_kernel(MfmaArgs A) {
    extern __shared__ __align__(16) unsigned short ys[];
    constexpr bool SCALED = std::is_same<E, F16>::value;
    static_assert(!FUSE || KIND == 1, "only the state's analysis is fused with a synthesis");
    __shared__ float sred[ANA_WAVES * 16], sc[16];
    int m, tg, g;
    if (!split_item<KIND>(A, m, tg, g)) return;
    const int ke = A.kp[2 * m], ko = A.kp[2 * m + 1];
    const int Lm = A.L - m + 1;
    const int base = m * (2 * A.L + 3 - m) / 2;
    const int rowlen = lds_row(A.hpad);
    unsigned short* yp = ys;                                        // [2][16][rowlen]
    float* zs = reinterpret_cast<float*>(ys + 2 * 16 * rowlen);     // KIND 1: [2][kmax][16]
    double* us = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(zs) + A.zreg);   // FUSE
    const int f0 = 8 * g;
    const double dm = static_cast<double>(m);
    // FUSE: the synthesis staging's per-degree factors of the thread's first
    // staging row (a/N and the H coefficients), requested now
    double syn_s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (FUSE) {
        if (static_cast<int>(threadIdx.x) < 2 * A.kmax) syn_factors(A, m, threadIdx.x, syn_s);
    }
    // KIND 1: the epilogue's inputs that do not depend on the products (H
    // coefficients, l(l+1)/a^2, U0 + c1 Nprev) of the thread's first EPI items
    // (degree, output column) are requested before anything else
    constexpr int EPI = 2;
    double pre_hA[EPI], pre_hB[EPI], pre_nk[EPI], pre_ob[EPI];
    auto epi_inputs = [&](int it, double& hA, double& hB, double& nk, double& ob) {
        const int i = it / 6, k = it - i * 6;
        hA = A.rec[base + i].hA;
        hB = A.rec[base + i].hB;
        nk = A.noa2[m + i];
        const size_t e2 = (static_cast<size_t>(k >> 1) * A.modes + base + i) * 2 + (k & 1);
        ob = A.U0 ? reinterpret_cast<const double*>(A.U0)[e2] : 0.0;
        if (A.Nprev) ob = __builtin_fma(A.c1, reinterpret_cast<const double*>(A.Nprev)[e2], ob);
    };
    if constexpr (KIND == 1) {
#pragma unroll
        for (int q = 0; q < EPI; ++q) {
            const int it = threadIdx.x + q * static_cast<int>(blockDim.x);
            pre_hA[q] = pre_hB[q] = pre_nk[q] = pre_ob[q] = 0.0;
            if (it < Lm * 6) epi_inputs(it, pre_hA[q], pre_hB[q], pre_nk[q], pre_ob[q]);
        }
    }
    // staging item it = (latitude j, input field q): that field's columns for
    // both folds (zero for padding latitudes and absent fields), handed to
    // emit(column, S-fold value, D-fold value)
    constexpr int NFLD = KIND == 0 ? 8 : 5;
    auto stage_item = [&](int it, auto&& emit) {
        const int j = it / NFLD, q = it - j * NFLD;
        double2 S = make_double2(0.0, 0.0), D = make_double2(0.0, 0.0);
        const int fld = KIND == 0 ? f0 + q : q;
        if (j < A.half && (KIND == 1 || fld < A.nf)) {
            const double wj = A.w[j];
            const double wt = (KIND == 0 || q == 4) ? wj : wj / (A.a * A.sint[j] * A.sint[j]);
            const double2* fr = A.four_in + (static_cast<size_t>(fld) * (A.L + 1) + m) * A.nlat;
            const double2 nn = fr[j];
            const double2 ss = fr[A.nlat - 1 - j];
            S = make_double2((nn.x + ss.x) * wt, (nn.y + ss.y) * wt);
            D = make_double2((nn.x - ss.x) * wt, (nn.y - ss.y) * wt);
        }
        // (column, S-fold value, D-fold value) of this field
        if constexpr (KIND == 0) {
            emit(j, 2 * q, S.x, D.x);
            emit(j, 2 * q + 1, S.y, D.y);
        } else {
            if (q == 0) {          // hU: Pbar columns 0, 1
                emit(j, 0, dm * S.y, dm * D.y);
                emit(j, 1, -dm * S.x, -dm * D.x);
            } else if (q == 1) {   // hV: H columns 8, 9
                emit(j, 8, S.x, D.x);
                emit(j, 9, S.y, D.y);
            } else if (q == 2) {   // zU: Pbar columns 2, 3; H columns 12, 13
                emit(j, 2, dm * S.y, dm * D.y);
                emit(j, 3, -dm * S.x, -dm * D.x);
                emit(j, 12, S.x, D.x);
                emit(j, 13, S.y, D.y);
            } else if (q == 3) {   // zV: Pbar columns 4, 5; H columns 10, 11
                emit(j, 4, -dm * S.y, -dm * D.y);
                emit(j, 5, dm * S.x, dm * D.x);
                emit(j, 10, S.x, D.x);
                emit(j, 11, S.y, D.y);
            } else {               // KE: Pbar columns 6, 7; columns 14, 15 stay zero
                emit(j, 6, S.x, D.x);
                emit(j, 7, S.y, D.y);
                emit(j, 14, 0.0, 0.0);
                emit(j, 15, 0.0, 0.0);
            }
        }
    };
    if constexpr (SCALED) {
        // the values go to LDS as FP32 (24 bits, more than the split keeps)
        // with their column maxima; then they are scaled and split.  The FP32
        // buffer [16][2][hpad] shares the region of zs, which is written only
        // after the products.
        float* stage = zs;
        float cmax[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) cmax[k] = 0.f;
        for (int it = threadIdx.x; it < A.hpad * NFLD; it += blockDim.x)
            stage_item(it, [&](int j, int col, double vs, double vd) {
                const float s0 = static_cast<float>(vs), s1 = static_cast<float>(vd);
                stage[(col * 2) * A.hpad + j] = s0;
                stage[(col * 2 + 1) * A.hpad + j] = s1;
                const float v = fmaxf(fabsf(s0), fabsf(s1));
#pragma unroll
                for (int k = 0; k < 16; ++k) cmax[k] = col == k ? fmaxf(cmax[k], v) : cmax[k];
            });
        column_scales<KIND == 0 ? 16 : 14, ANA_THREADS>(cmax, sred, sc);
        for (int it = threadIdx.x; it < A.hpad * 16; it += blockDim.x) {
            const int col = it / A.hpad, j = it - col * A.hpad;
            unsigned short hi, lo;
            const int o0 = col * rowlen, o1 = (16 + col) * rowlen;
            split16<E>(static_cast<double>(stage[(col * 2) * A.hpad + j] * sc[col]), hi, lo);
            yp[o0 + grp_hi(j)] = hi;
            yp[o0 + grp_lo(j)] = lo;
            split16<E>(static_cast<double>(stage[(col * 2 + 1) * A.hpad + j] * sc[col]), hi, lo);
            yp[o1 + grp_hi(j)] = hi;
            yp[o1 + grp_lo(j)] = lo;
        }
        __syncthreads();   // stage (= zs) is free again only after every split
    } else {
        for (int it = threadIdx.x; it < A.hpad * NFLD; it += blockDim.x)
            stage_item(it, [&](int j, int col, double vs, double vd) {
                unsigned short hi, lo;
                const int o0 = col * rowlen, o1 = (16 + col) * rowlen;
                split16<E>(vs, hi, lo);
                yp[o0 + grp_hi(j)] = hi;
                yp[o0 + grp_lo(j)] = lo;
                split16<E>(vd, hi, lo);
                yp[o1 + grp_hi(j)] = hi;
                yp[o1 + grp_lo(j)] = lo;
            });
    }
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1);
    const int te = ke / 16, to = ko / 16;
    const int kq = lane >> 4;
    const int c = lane & 15;
    for (int tile = threadIdx.x / WAVE; tile < te + to; tile += ANA_WAVES) {
        const int par = tile < te ? 0 : 1;
        const int r0 = (par ? tile - te : tile) * 16;
        const long long blk = A.off[m] + (par ? static_cast<long long>(ke) * A.hpad * 2 : 0);
        // operand blocks of this row tile: 64 lanes x 8 shorts per K step
        const unsigned short* ap = A.p_ana + blk + (static_cast<long long>(r0 >> 4) * (A.hpad >> 4) * 64 + lane) * 8;
        const unsigned short* bp = yp + (par * 16 + c) * rowlen;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        // table operands in batches of KB steps (loads first, then products)
        const int nks = A.hpad >> 4;
        for (int k0 = 0; k0 < nks; k0 += KB_ANA) {
            uint4 a[KB_ANA];
#pragma unroll
            for (int u = 0; u < KB_ANA; ++u) {
                const int js = min(k0 + u, nks - 1);
                a[u] = *reinterpret_cast<const uint4*>(ap + js * 512);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < KB_ANA; ++u) {
                const bool in = k0 + u < nks;
                const int g = 4 * min(k0 + u, nks - 1) + kq;
                const uint4 b = keep_if(in, *reinterpret_cast<const uint4*>(bp + 8 * g));
                mfma3<E>(acc, a[u], b);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int r = r0 + 4 * kq + t;
            const int i = 2 * r + par;                  // l - m
            if constexpr (KIND == 0) {
                const int f = f0 + (c >> 1);
                if (i >= Lm || f >= A.nf) continue;
                const double v = static_cast<double>(acc[t]) / (SCALED ? static_cast<double>(sc[c]) : 1.0);
                note_nonfinite(A.status, v, STATUS_TRANSFORM);
                reinterpret_cast<double*>(A.spec_out + static_cast<size_t>(f) * A.modes + base + i)[c & 1] = v;
            } else {
                zs[(par * A.kmax + r) * 16 + c] = acc[t];
            }
        }
    }
    if constexpr (KIND == 1) {
        __syncthreads();
        // one thread per (degree, output column)
        auto finish = [&](int it, double hA, double hB, double nk, double ob) {
            const int i = it / 6, k = it - i * 6;
            const float* zrow = zs + ((i & 1) * A.kmax + (i >> 1)) * 16;
            const float* zup = zs + (((i + 1) & 1) * A.kmax + ((i + 1) >> 1)) * 16;   // degree l+1 (<= L+1)
            // undo the column scales (1 unless FP16)
            const double uP = SCALED ? 1.0 / static_cast<double>(sc[k]) : 1.0;
            const double uH = SCALED ? 1.0 / static_cast<double>(sc[8 + k]) : 1.0;
            double v = static_cast<double>(zrow[k]) * uP;
            double hsum = hA * static_cast<double>(zup[8 + k]);
            if (i >= 1) {
                const float* zdn = zs + (((i - 1) & 1) * A.kmax + ((i - 1) >> 1)) * 16;
                hsum = __builtin_fma(hB, static_cast<double>(zdn[8 + k]), hsum);
            }
            v = __builtin_fma(hsum, uH, v);
            if (k >= 4) {
                const double uK = SCALED ? 1.0 / static_cast<double>(sc[k + 2]) : 1.0;
                v = __builtin_fma(nk * uK, static_cast<double>(zrow[k + 2]), v);
            }
            const size_t e2 = (static_cast<size_t>(k >> 1) * A.modes + base + i) * 2 + (k & 1);
            if (A.Nsave) reinterpret_cast<double*>(A.Nsave)[e2] = v;
            const double o = __builtin_fma(A.c0, v, ob);
            note_nonfinite(A.status, o, STATUS_NONLINEAR);
            if (FUSE) us[it] = o;                       // it = 6 i + k
            if (!FUSE || A.out) reinterpret_cast<double*>(A.out)[e2] = o;
        };
#pragma unroll
        for (int q = 0; q < EPI; ++q) {
            const int it = threadIdx.x + q * static_cast<int>(blockDim.x);
            if (it < Lm * 6) finish(it, pre_hA[q], pre_hB[q], pre_nk[q], pre_ob[q]);
        }
        for (int it = threadIdx.x + EPI * static_cast<int>(blockDim.x); it < Lm * 6; it += blockDim.x) {
            double hA, hB, nk, ob;
            epi_inputs(it, hA, hB, nk, ob);
            finish(it, hA, hB, nk, ob);
        }
    }
    if constexpr (FUSE) {
        __syncthreads();   // us complete; yp, zs and sc free
        synth_state_block<E>(A, m, us, syn_s, ys, zs, sred, sc);
    }
}

// The REXI stage's pole sum fused with the synthesis of its result (split
// precision): the workgroup of order m sums the pole-wave partials of its
// order's coefficients (sum_parts, the order of the separate reduction),
// writes them to U1, keeps them in LDS and synthesises them for every
// latitude (synth_state_block).  Order of workgroups as split_item<1>.
// LDS: [2][16][lds_row(kmax)] shorts, then A.zreg bytes (FP16 staging), then
// us ([L+1][3] complex).
template <class E>
__global__ __launch_bounds__(ANA_THREADS) void leg_sum_synth_mfma_kernel(MfmaArgs A, const double2* __restrict__ part,
                                                                         int nparts, double2* __restrict__ U1) {
    extern __shared__ __align__(16) unsigned short ys[];
    __shared__ float sred[ANA_WAVES * 16], sc[16];
    int m, tg, g;
    if (!split_item<1>(A, m, tg, g)) return;
    const int Lm = A.L - m + 1;
    const int base = m * (2 * A.L + 3 - m) / 2;
    float* zs = reinterpret_cast<float*>(ys + 2 * 16 * lds_row(A.kmax));
    double* us = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(zs) + A.zreg);
    double syn_s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (static_cast<int>(threadIdx.x) < 2 * A.kmax) syn_factors(A, m, threadIdx.x, syn_s);
    double2* u2 = reinterpret_cast<double2*>(us);
    for (int it = threadIdx.x; it < 3 * Lm; it += ANA_THREADS) {
        const int i = it / 3, f = it - 3 * i;
        const int e = f * A.modes + base + i;
        const double2 v = sum_parts(part, 3 * A.modes, nparts, e);
        note_nonfinite(A.status, v.x + v.y, STATUS_REXI);
        U1[e] = v;
        u2[it] = v;
    }
    __syncthreads();
    synth_state_block<E>(A, m, us, syn_s, ys, zs, sred, sc);
}

MfmaArgs mfma_args(const swe_ctx* ctx) {
    MfmaArgs A{};
    A.p_syn = ctx->d_tab_psyn;
    A.p_ana = ctx->d_tab_pana;
    A.off = ctx->d_tab_off;
    A.kp = ctx->d_tab_kp;
    A.rec = ctx->d_rec;
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
    A.status = ctx->d_status;
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
    T.p_ana = ctx->d_tab_pana;
    T.L = ctx->L;
    T.half = ctx->nlat / 2;
    T.hpad = ctx->tab_hpad;
    T.nseg = ctx->nseg;
    const size_t bytes = sizeof(unsigned short) * static_cast<size_t>(ctx->tab_len);
    for (unsigned short* p : {ctx->d_tab_psyn, ctx->d_tab_pana}) REXI_HIP(hipMemsetAsync(p, 0, bytes, stream));
    if (ctx->prec & REXI_PREC_FP16_SPLIT)
        hipLaunchKernelGGL(leg_table_kernel<F16>, dim3(ctx->nseg, (T.half + 255) / 256), dim3(256), 0, stream, T);
    else
        hipLaunchKernelGGL(leg_table_kernel<Bf16>, dim3(ctx->nseg, (T.half + 255) / 256), dim3(256), 0, stream, T);
    REXI_HIP(hipGetLastError());
    return REXI_OK;
}

int launch_legendre_synth_split(swe_ctx* ctx, int kind, const double* spec, double* four, int nf,
                                hipStream_t stream) {
    MfmaArgs A = mfma_args(ctx);
    A.spec = reinterpret_cast<const double2*>(spec);
    A.four_out = reinterpret_cast<double2*>(four);
    A.nf = nf;
    size_t lds = sizeof(unsigned short) * 2 * 16 * static_cast<size_t>(lds_row(A.kmax));
    if (ctx->prec & REXI_PREC_FP16_SPLIT) lds += sizeof(float) * 16 * 2 * static_cast<size_t>(A.kmax);
    const int tiles = A.hpad / 16;
    A.ntg = (tiles + 3) / 4;
    A.ng = (nf + 7) / 8;
    // kind 0 order-major [nf][L+1][nlat], kind 1 latitude-major [3][nlat][L+1]
    A.ofs = static_cast<long long>(ctx->L + 1) * ctx->nlat;
    A.oms = kind == 0 ? ctx->nlat : 1;
    A.ojs = kind == 0 ? 1 : ctx->L + 1;
    A.xcd_blocks = (ctx->L + 1) % 64 == 0;
    const dim3 grid = kind == 0 ? dim3(split_grid_size((ctx->L + 1) * A.ntg, A.ng)) : dim3((ctx->L + 1) * A.ntg);
    const bool f16 = (ctx->prec & REXI_PREC_FP16_SPLIT) != 0;
    const void* fn = kind == 0 ? (f16 ? reinterpret_cast<const void*>(&leg_synth_mfma_kernel<0, F16>)
                                      : reinterpret_cast<const void*>(&leg_synth_mfma_kernel<0, Bf16>))
                               : (f16 ? reinterpret_cast<const void*>(&leg_synth_mfma_kernel<1, F16>)
                                      : reinterpret_cast<const void*>(&leg_synth_mfma_kernel<1, Bf16>));
    int rc;
    if ((rc = allow_dyn_lds(fn, lds)) != REXI_OK) return rc;
    const int slot = prof_begin(ctx, REXI_KERNEL_LEG_SYNTH, stream);
    void* kargs[] = {&A};
    REXI_HIP(hipLaunchKernel(fn, grid, dim3(SYN_THREADS), kargs, lds, stream));
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
    size_t lds = sizeof(unsigned short) * 2 * 16 * static_cast<size_t>(lds_row(A.hpad));
    // zs (products, kind 1) and the FP16 mode's FP32 staging share one region
    size_t zbytes = kind == 1 ? sizeof(float) * 2 * 16 * static_cast<size_t>(A.kmax) : 0;
    if (ctx->prec & REXI_PREC_FP16_SPLIT) zbytes = std::max(zbytes, sizeof(float) * 16 * 2 * static_cast<size_t>(A.hpad));
    lds += zbytes;
    A.zreg = static_cast<int>(zbytes);
    A.ntg = 1;
    A.ng = (nf + 7) / 8;
    const dim3 grid = kind == 0 ? dim3(split_grid_size(ctx->L + 1, A.ng)) : dim3(ctx->L + 1, 1, 1);
    const bool f16 = (ctx->prec & REXI_PREC_FP16_SPLIT) != 0;
    const void* fn = kind == 0 ? (f16 ? reinterpret_cast<const void*>(&leg_anal_mfma_kernel<0, F16>)
                                      : reinterpret_cast<const void*>(&leg_anal_mfma_kernel<0, Bf16>))
                               : (f16 ? reinterpret_cast<const void*>(&leg_anal_mfma_kernel<1, F16>)
                                      : reinterpret_cast<const void*>(&leg_anal_mfma_kernel<1, Bf16>));
    int rc;
    if ((rc = allow_dyn_lds(fn, lds)) != REXI_OK) return rc;
    const int slot = prof_begin(ctx, REXI_KERNEL_LEG_ANAL, stream);
    void* kargs[] = {&A};
    REXI_HIP(hipLaunchKernel(fn, grid, dim3(ANA_THREADS), kargs, lds, stream));
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_LEG_ANAL, slot, stream);
    return REXI_OK;
}

int fused_anal_synth_supported(const swe_ctx* ctx) { return ctx->tab_kmax <= ctx->tab_hpad; }

int launch_legendre_anal_synth_split(swe_ctx* ctx, const double* four, const double* U0, const double* Nprev,
                                     double* Nsave, double* out, double c0, double c1, double* four_next,
                                     hipStream_t stream) {
    if (!fused_anal_synth_supported(ctx))
        return fail(REXI_ENOTSUP, "fused analysis and synthesis: degree rows exceed the latitude rows");
    MfmaArgs A = mfma_args(ctx);
    A.four_in = reinterpret_cast<const double2*>(four);
    A.U0 = reinterpret_cast<const double2*>(U0);
    A.Nprev = reinterpret_cast<const double2*>(Nprev);
    A.Nsave = reinterpret_cast<double2*>(Nsave);
    A.out = reinterpret_cast<double2*>(out);
    A.c0 = c0;
    A.c1 = c1;
    A.nf = 3;
    // the synthesis output of the state: latitude-major [3][nlat][L+1]
    A.four_out = reinterpret_cast<double2*>(four_next);
    A.ofs = static_cast<long long>(ctx->L + 1) * ctx->nlat;
    A.oms = 1;
    A.ojs = ctx->L + 1;
    A.ntg = 1;
    A.ng = 1;
    A.xcd_blocks = (ctx->L + 1) % 64 == 0;
    size_t lds = sizeof(unsigned short) * 2 * 16 * static_cast<size_t>(lds_row(A.hpad));
    size_t zbytes = sizeof(float) * 2 * 16 * static_cast<size_t>(A.kmax);
    if (ctx->prec & REXI_PREC_FP16_SPLIT) zbytes = std::max(zbytes, sizeof(float) * 16 * 2 * static_cast<size_t>(A.hpad));
    zbytes = (zbytes + 15) / 16 * 16;
    A.zreg = static_cast<int>(zbytes);
    lds += zbytes + sizeof(double) * 6 * static_cast<size_t>(ctx->L + 1);
    const bool f16 = (ctx->prec & REXI_PREC_FP16_SPLIT) != 0;
    const void* fn = f16 ? reinterpret_cast<const void*>(&leg_anal_mfma_kernel<1, F16, true>)
                         : reinterpret_cast<const void*>(&leg_anal_mfma_kernel<1, Bf16, true>);
    int rc;
    if ((rc = allow_dyn_lds(fn, lds)) != REXI_OK) return rc;
    const int slot = prof_begin(ctx, REXI_KERNEL_LEG_FUSED, stream);
    void* kargs[] = {&A};
    REXI_HIP(hipLaunchKernel(fn, dim3(ctx->L + 1), dim3(ANA_THREADS), kargs, lds, stream));
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_LEG_FUSED, slot, stream);
    return REXI_OK;
}

int launch_rexi_sum_synth_split(swe_ctx* ctx, const double* part, int nparts, double* U1, double* four_next,
                                hipStream_t stream) {
    if (nparts < 1) return fail(REXI_EINVAL, "pole sum and synthesis: no partial sums");
    MfmaArgs A = mfma_args(ctx);
    A.nf = 3;
    A.four_out = reinterpret_cast<double2*>(four_next);
    A.ofs = static_cast<long long>(ctx->L + 1) * ctx->nlat;
    A.oms = 1;
    A.ojs = ctx->L + 1;
    A.ntg = 1;
    A.ng = 1;
    A.xcd_blocks = (ctx->L + 1) % 64 == 0;
    size_t lds = sizeof(unsigned short) * 2 * 16 * static_cast<size_t>(lds_row(A.kmax));
    size_t zbytes = (ctx->prec & REXI_PREC_FP16_SPLIT) ? sizeof(float) * 16 * 2 * static_cast<size_t>(A.kmax) : 0;
    zbytes = (zbytes + 15) / 16 * 16;
    A.zreg = static_cast<int>(zbytes);
    lds += zbytes + sizeof(double) * 6 * static_cast<size_t>(ctx->L + 1);
    const bool f16 = (ctx->prec & REXI_PREC_FP16_SPLIT) != 0;
    const void* fn = f16 ? reinterpret_cast<const void*>(&leg_sum_synth_mfma_kernel<F16>)
                         : reinterpret_cast<const void*>(&leg_sum_synth_mfma_kernel<Bf16>);
    int rc;
    if ((rc = allow_dyn_lds(fn, lds)) != REXI_OK) return rc;
    const double2* p = reinterpret_cast<const double2*>(part);
    double2* u = reinterpret_cast<double2*>(U1);
    const int slot = prof_begin(ctx, REXI_KERNEL_REDUCE, stream);
    void* kargs[] = {&A, &p, &nparts, &u};
    REXI_HIP(hipLaunchKernel(fn, dim3(ctx->L + 1), dim3(ANA_THREADS), kargs, lds, stream));
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_REDUCE, slot, stream);
    return REXI_OK;
}

}  // namespace rexi
