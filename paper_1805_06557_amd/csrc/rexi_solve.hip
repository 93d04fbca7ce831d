// REXI linear stage on the device: for every pole n and zonal order m the
// shifted system (z_n I - dt L_m) y = u0 (z_n = -alpha_n), reduced to two
// complex tridiagonal chains by eliminating h, solved by an unpivoted Thomas
// sweep, and the weighted sum  U1 = sum_n w_n y_n  (w_n = -beta_n), which is
// the paper's Eq. (rexi) with L = L_g + L_c.
//
// Chain form (derived from the spectral operator; degree k = m + j on row j):
//   delta row: [z - i dt s_k + dt^2 H gN_k / z] delta_k
//              - dt (cm_k zeta_{k-1} + cp_k zeta_{k+1}) = r_delta + dt gN_k r_h / z
//   zeta row:  [z - i dt s_k] zeta_k + dt (cm_k delta_{k-1} + cp_k delta_{k+1}) = r_zeta
//   h_k = (r_h - dt H delta_k) / z
// Chain c = 0 holds (delta_m, zeta_{m+1}, delta_{m+2}, ...), chain c = 1 holds
// (zeta_m, delta_{m+1}, ...).
//
// Mapping: one wave per (m, chain, block of 64 P poles); lane l carries P
// poles, so every table value and right-hand side is wave-uniform (read by
// broadcast from the chain's row records, staged once per workgroup in LDS)
// and the per-lane work is a sequential sweep over l.  The chain is cut into
// segments of S rows: a first forward sweep keeps only the state entering each
// segment (a checkpoint in a global workspace, read back once); the backward
// pass then re-sweeps one segment at a time into registers and back-substitutes
// through it.  The pivots of the re-sweep are recomputed (FUSED) or read from a
// factorization cached per coefficient set and dt (STREAM, HYBRID); every
// schedule performs the same operations on each (pole, row), so all agree bit
// for bit.  The sum over the poles of a wave is formed in FP64 in a fixed order:
// lane-local over its P poles, then in LDS (write lane-major, read transposed,
// finish with a 3-step butterfly).  Pole waves write partial sums that a second
// kernel adds in pole-wave order, so results are bit-reproducible.  The file is
// compiled without automatic FMA contraction and every fused multiply-add is
// written out, so all inlined copies of a step perform the same rounding.
#include <algorithm>
#include <cstring>
#include <type_traits>
#include <utility>
#include <vector>

#include "internal.h"

namespace rexi {
namespace {

constexpr int WAVE = 64;

template <typename T>
struct Cx {
    T x, y;
};

__device__ __forceinline__ double rcp_refined(double n) {
    double r = __builtin_amdgcn_rcp(n);
    double e = __builtin_fma(-n, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-n, r, 1.0);
    return __builtin_fma(r, e, r);
}

// FP32: the hardware reciprocal (about 1 ulp) is used as is; the pivot then
// carries a relative error of a few u_32, within the FP32 sweep's own rounding.
__device__ __forceinline__ float rcp_refined(float n) { return __builtin_amdgcn_rcpf(n); }

// Lane 0's value of v, held in scalar registers.
__device__ __forceinline__ double wave_uniform(double v) {
    const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<int>(u & 0xffffffffu)));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<int>(u >> 32)));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Orders the LDS accesses of one wave (its lanes exchange data through a
// wave-private LDS region): LDS operations of a wave complete in order, so a
// compiler-level fence plus a wave barrier suffices.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Uniform data of one chain row, formed for every call from the state, dt and
// the per-mode coefficients (by the fused solve itself, in LDS, or by
// rexi_rows_kernel in HBM in chain order, record 2 base(m) + c Lm + j), so that
// the sweeps read one record per row and do no wave-uniform arithmetic.
struct RowRec {
    double a;          // coupling to row j-1, signed for the row type, times dt
    double ac;         // a_j c_{j-1}: the product of this row's a and the previous row's c (0 for j = 0)
    double dts;        // dt m q_k
    double g2;         // dt^2 H g k(k+1)/a^2  (delta rows; 0 for zeta rows)
    double tx, ty;     // dt g k(k+1)/a^2 r_h   (delta rows; 0 for zeta rows)
    double rx, ry;     // right-hand side r_delta or r_zeta
    double c;          // coupling to row j+1, signed for the row type, times dt
    double hx, hy;     // r_h (delta rows)
    double pad;
};
static_assert(sizeof(RowRec) == 96, "RowRec layout");

// The FP32 solve's record: the same quantities rounded once to FP32 (48 B, so a
// chain's records take half the LDS and half the broadcast reads).  The first
// 32 bytes hold everything the forward sweep reads.
struct RowRec32 {
    float a, ac, dts, g2, tx, ty, rx, ry, c, hx, hy;
    float pad;
};
static_assert(sizeof(RowRec32) == 48, "RowRec32 layout");

template <typename T>
using RecT = typename std::conditional<std::is_same<T, float>::value, RowRec32, RowRec>::type;

// The delta and zeta records of degree k = m + j (one per chain).
__device__ __forceinline__ RowRec32 round_rec(const RowRec& r) {
    RowRec32 q;
    q.a = static_cast<float>(r.a);
    q.ac = static_cast<float>(r.ac);
    q.c = static_cast<float>(r.c);
    q.dts = static_cast<float>(r.dts);
    q.tx = static_cast<float>(r.tx);
    q.ty = static_cast<float>(r.ty);
    q.rx = static_cast<float>(r.rx);
    q.ry = static_cast<float>(r.ry);
    q.g2 = static_cast<float>(r.g2);
    q.hx = static_cast<float>(r.hx);
    q.hy = static_cast<float>(r.hy);
    q.pad = 0.0f;
    return q;
}

// a_j c_{j-1} of row j >= 1 (degree k = m + j, coefficients cf; the previous
// degree's coefficients cfp).  The rows of a chain alternate between delta rows
// (couplings -dt cm, -dt cp) and zeta rows (dt cm, dt cp), so the product is
// -(dt cm_k)(dt cp_{k-1}) in either chain, the same bits as the product of the
// two rows' signed couplings.
__device__ __forceinline__ double coupling_product(const ModeCoef& cf, const ModeCoef& cfp, double dt) {
    return -((dt * cf.cm) * (dt * cfp.cp));
}

// The delta row (coupled to h) and the zeta row of degree k = m + j.
__device__ __forceinline__ RowRec delta_row(const ModeCoef& cf, double ac, double2 rh, double2 rd, double dt, double H) {
    RowRec d;
    d.a = -dt * cf.cm;
    d.ac = ac;
    d.c = -dt * cf.cp;
    d.dts = dt * cf.s;
    d.g2 = dt * dt * H * cf.gN;
    d.tx = dt * cf.gN * rh.x;
    d.ty = dt * cf.gN * rh.y;
    d.rx = rd.x;
    d.ry = rd.y;
    d.hx = rh.x;
    d.hy = rh.y;
    d.pad = 0.0;
    return d;
}

__device__ __forceinline__ RowRec zeta_row(const ModeCoef& cf, double ac, double2 rz, double dt) {
    RowRec z;
    z.a = dt * cf.cm;
    z.ac = ac;
    z.c = dt * cf.cp;
    z.dts = dt * cf.s;
    z.g2 = 0.0;
    z.tx = z.ty = 0.0;
    z.rx = rz.x;
    z.ry = rz.y;
    z.hx = z.hy = 0.0;
    z.pad = 0.0;
    return z;
}

__device__ __forceinline__ void build_row_pair(const double2* __restrict__ U0, const ModeCoef* __restrict__ coef,
                                               RowRec* __restrict__ rec, RowRec32* __restrict__ rec32, int L,
                                               int modes, double dt, double H, int m, int j) {
    const int base = m * (2 * L + 3 - m) / 2;
    const int idx = base + j;
    const int Lm = L - m + 1;
    const ModeCoef cf = coef[idx];
    const double ac = j > 0 ? coupling_product(cf, coef[idx - 1], dt) : 0.0;
    const int cd = j & 1;                                   // chain in which row j is a delta row
    const RowRec d = delta_row(cf, ac, U0[idx], U0[2 * modes + idx], dt, H);
    rec[2 * base + cd * Lm + j] = d;
    rec32[2 * base + cd * Lm + j] = round_rec(d);
    const RowRec z = zeta_row(cf, ac, U0[modes + idx], dt);
    rec[2 * base + (1 - cd) * Lm + j] = z;
    rec32[2 * base + (1 - cd) * Lm + j] = round_rec(z);
}


// One workgroup per order m (blockIdx.x), threads over the degrees.
__global__ __launch_bounds__(256) void rexi_rows_kernel(const double2* __restrict__ U0, const ModeCoef* __restrict__ coef,
                                                        RowRec* __restrict__ rec, RowRec32* __restrict__ rec32, int L,
                                                        int modes, double dt, double H) {
    const int m = blockIdx.x;
    for (int j = threadIdx.x; j < L - m + 1; j += blockDim.x)
        build_row_pair(U0, coef, rec, rec32, L, modes, dt, H, m, j);
}

// Ensemble form: member blockIdx.y.
struct RowsArgs {
    const double2* U0;
    const ModeCoef* coef;
    RowRec* rec;
    RowRec32* rec32;
    int L, modes;
    double dt, H;
};

__global__ __launch_bounds__(256) void rexi_rows_batched_kernel(const RowsArgs* __restrict__ args) {
    const RowsArgs a = args[blockIdx.y];
    const int m = blockIdx.x;
    if (m > a.L) return;
    for (int j = threadIdx.x; j < a.L - m + 1; j += blockDim.x)
        build_row_pair(a.U0, a.coef, a.rec, a.rec32, a.L, a.modes, a.dt, a.H, m, j);
}

struct SolveArgs {
    const RowRec* __restrict__ rec;     // [2 modes] chain-ordered row records
    const RowRec32* __restrict__ rec32; // the same rounded to FP32
    double2* __restrict__ out;          // [pole waves][3][modes] partial sums (one per wave of 64 poles)
    const PoleData* __restrict__ poles; // [N]
    const void* __restrict__ fact;      // cached pivots [2 modes][npad] complex T (STREAM, HYBRID)
    void* __restrict__ ckpt;            // segment-start states [tasks][pole waves][nck_max][CKW][P][64] complex T
    int L, modes, N, npb, npad;         // npb: workgroups per chain; npad: N rounded up to 64 P
    int nck_max, rec_bytes;             // per-wave checkpoints; LDS bytes of the records
    double dtH;
    // the fused schedule builds its chain's row records itself from these
    const double2* __restrict__ U0;     // [3][modes] state
    const ModeCoef* __restrict__ coef;  // [modes]
    double dt, H;
    unsigned* status;                   // non-finite outputs set STATUS_REXI
};

struct Lane {
    PoleData p;
    double wzr, wzi;   // w / z
    float zrf, zif;    // z in FP32
    float zirf, ziif;  // 1/z in FP32
    float wrf, wif;    // w in FP32 (the FP32 solve's weighting)
    float wzrf, wzif;  // w / z in FP32
};

template <typename T>
__host__ __device__ __forceinline__ const RecT<T>* chain_records(const SolveArgs& A, int row0) {
    if constexpr (std::is_same<T, float>::value) return A.rec32 + row0; else return A.rec + row0;
}

// Right-hand side d = r + t/z of a row (zeta rows have t = 0).  FP64 solve: in
// FP64.  FP32 solve: in FP32 from the rounded record (a rounding of the
// right-hand side by u_32 relative to its terms, which the FP32 solve's own
// backward error already contains).
template <typename T, bool DELTA>
__device__ __forceinline__ void row_rhs(const RecT<T>& R, const Lane& ln, T& dR, T& dI) {
    if constexpr (std::is_same<T, float>::value) {
        if constexpr (DELTA) {
            dR = __builtin_fmaf(ln.zirf, R.tx, __builtin_fmaf(-ln.ziif, R.ty, R.rx));
            dI = __builtin_fmaf(ln.zirf, R.ty, __builtin_fmaf(ln.ziif, R.tx, R.ry));
        } else {
            dR = R.rx;
            dI = R.ry;
        }
    } else {
        if constexpr (DELTA) {
            dR = __builtin_fma(ln.p.zir, R.tx, __builtin_fma(-ln.p.zii, R.ty, R.rx));
            dI = __builtin_fma(ln.p.zir, R.ty, __builtin_fma(ln.p.zii, R.tx, R.ry));
        } else {
            dR = R.rx;
            dI = R.ry;
        }
    }
}

template <typename T>
__device__ __forceinline__ T coupling_a(const RecT<T>& R) { return R.a; }
template <typename T>
__device__ __forceinline__ T coupling_c(const RecT<T>& R) { return R.c; }

// Pivot of a row: p_j = 1/(b_j - a_j c'_{j-1}) with c'_{j-1} = c_{j-1} p_{j-1},
// formed as b_j - (a_j c_{j-1}) p_{j-1} from the record's product ac, so that the
// recurrence runs on the pivots alone (c' = c p is formed only where the
// back-substitution needs it).  The diagonal b = z + g2/z - i dts (g2 = 0 for
// zeta rows) is formed in T; an FP32 diagonal is off by u_32 relative to
// |z| + g2/|z|, a backward error of the size the FP32 sweep makes anyway (the
// shifted systems are well conditioned: the poles stay at a distance y - rho
// from the spectrum).  pp: the previous row's pivot on entry, this row's on
// return.  Used by the factorization and by both sweeps of the fused schedule,
// so cached and recomputed pivots agree bit for bit.
template <typename T, bool DELTA>
__device__ __forceinline__ Cx<T> pivot_row(const RecT<T>& R, const Lane& ln, Cx<T>& pp) {
    T bR, bI;
    if constexpr (std::is_same<T, float>::value) {
        if constexpr (DELTA) {
            bR = __builtin_fmaf(R.g2, ln.zirf, ln.zrf);
            bI = __builtin_fmaf(R.g2, ln.ziif, ln.zif) - R.dts;
        } else {
            bR = ln.zrf;
            bI = ln.zif - R.dts;
        }
    } else {
        if constexpr (DELTA) {
            bR = __builtin_fma(R.g2, ln.p.zir, ln.p.zr);
            bI = __builtin_fma(R.g2, ln.p.zii, ln.p.zi) - R.dts;
        } else {
            bR = ln.p.zr;
            bI = ln.p.zi - R.dts;
        }
    }
    const T tac = R.ac;
    const T wr = fmaT(-tac, pp.x, bR);
    const T wi = fmaT(-tac, pp.y, bI);
    const T inv = rcp_refined(fmaT(wr, wr, wi * wi));
    const Cx<T> p{wr * inv, -wi * inv};
    pp = p;
    return p;
}

// c'_j = c_j p_j, the factor the back-substitution applies to x_{j+1}.
template <typename T>
__device__ __forceinline__ Cx<T> upper_factor(const RecT<T>& R, Cx<T> p) {
    const T tc = coupling_c<T>(R);
    return Cx<T>{tc * p.x, tc * p.y};
}

// The right-hand-side part of a forward step with pivot p: d' = (d - a d'_prev) p.
template <typename T, bool DELTA>
__device__ __forceinline__ void forward_rhs(const RecT<T>& R, const Lane& ln, Cx<T> p, Cx<T>& dp) {
    T dR, dI;
    row_rhs<T, DELTA>(R, ln, dR, dI);
    const T ta = coupling_a<T>(R);
    const T ur = fmaT(-ta, dp.x, dR);
    const T ui = fmaT(-ta, dp.y, dI);
    dp.x = fmaT(ur, p.x, -(ui * p.y));
    dp.y = fmaT(ur, p.y, ui * p.x);
}

// Sums the 6 staged slots over the 64 lanes of the wave and writes them.
// red: [6][64] double2.  Slot s < 4: chain row 4g + s; slots 4, 5: sum of
// (w/z) delta of the two delta rows of the group, from which
// h = sum_n (w_n/z_n) (t - dt H delta_n) = t swz - dt H sum_n (w_n/z_n) delta_n
// with swz the wave's sum of w/z and t the row's h right-hand side.
template <typename T, int C>
__device__ __forceinline__ void reduce_group(const SolveArgs& A, const RecT<T>* rc, double2 swz, double2* red,
                                             int lane, int pw, int base, int j0g, int Lm) {
    wave_sync();
    const int slot = lane >> 3, part = lane & 7;
    double sx = 0.0, sy = 0.0;
    if (slot < 6) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const double2 v = red[slot * WAVE + i * 8 + part];
            sx += v.x;
            sy += v.y;
        }
    }
#pragma unroll
    for (int msk = 1; msk < 8; msk <<= 1) {
        sx += __shfl_xor(sx, msk, 8);
        sy += __shfl_xor(sy, msk, 8);
    }
    if (part == 0 && slot < 6) {
        int q, field;
        if (slot < 4) {
            q = slot;
            field = ((q + C) & 1) == 0 ? 2 : 1;
        } else {
            q = 2 * (slot - 4) + C;
            field = 0;
        }
        const int j = j0g + q;
        if (j < Lm) {
            if (slot >= 4) {
                const double tx = static_cast<double>(rc[j].hx), ty = static_cast<double>(rc[j].hy);
                const double ax = __builtin_fma(tx, swz.x, -(ty * swz.y));
                const double ay = __builtin_fma(tx, swz.y, ty * swz.x);
                sx = __builtin_fma(-A.dtH, sx, ax);
                sy = __builtin_fma(-A.dtH, sy, ay);
            }
            note_nonfinite(A.status, sx + sy, STATUS_REXI);
            A.out[(pw * 3 + field) * A.modes + base + j] = make_double2(sx, sy);
        }
    }
    wave_sync();
}

// Back-substitution through one segment whose c'_j = c_j p_j and d'_j values cs
// and ds are in registers: x_j = d'_j - c'_j x_{j+1}; the weighted outputs of
// the lane's P poles are added in pole order, then summed over the wave.
template <typename T, int S, int C, int P>
__device__ __forceinline__ void back_segment(const SolveArgs& A, const Lane* ln, const RecT<T>* rc, int j0, int Lm,
                                             int base, int pw, int lane, const Cx<T> (*cs)[S],
                                             const Cx<T> (*ds)[S], Cx<T>* vnext, double2 swz, double2* red) {
    static_for<0, S / 4>([&](auto G) {
        constexpr int g = S / 4 - 1 - decltype(G)::value;
        static_for<0, 4>([&](auto Qi) {
            constexpr int q = 3 - decltype(Qi)::value;
            constexpr int jj = 4 * g + q;
            constexpr bool DELTA = ((jj + C) & 1) == 0;
            const int j = j0 + jj;
            const bool live = j < Lm;
            // weighted outputs of the lane's poles, added in pole order: in the
            // solve's precision (an FP32 product and sum adds one rounding of
            // u_32 to terms that carry the FP32 sweep's few u_32), then widened
            // for the FP64 sum over the wave
            T sx = T(0), sy = T(0), hx = T(0), hy = T(0);
#pragma unroll
            for (int k = 0; k < P; ++k) {
                Cx<T> v{T(0), T(0)};
                if (live) {
                    const Cx<T> cpj = cs[k][jj];
                    v.x = fmaT(-cpj.x, vnext[k].x, fmaT(cpj.y, vnext[k].y, ds[k][jj].x));
                    v.y = fmaT(-cpj.x, vnext[k].y, fmaT(-cpj.y, vnext[k].x, ds[k][jj].y));
                    vnext[k] = v;
                }
                T wr, wi, wzr, wzi;
                if constexpr (std::is_same<T, float>::value) {
                    wr = ln[k].wrf;
                    wi = ln[k].wif;
                    wzr = ln[k].wzrf;
                    wzi = ln[k].wzif;
                } else {
                    wr = ln[k].p.wr;
                    wi = ln[k].p.wi;
                    wzr = ln[k].wzr;
                    wzi = ln[k].wzi;
                }
                const T ox = fmaT(wr, v.x, -(wi * v.y));
                const T oy = fmaT(wr, v.y, wi * v.x);
                sx = k ? sx + ox : ox;
                sy = k ? sy + oy : oy;
                if constexpr (DELTA) {
                    // (w/z) delta; v = 0 past the chain's end
                    const T gx = fmaT(wzr, v.x, -(wzi * v.y));
                    const T gy = fmaT(wzr, v.y, wzi * v.x);
                    hx = k ? hx + gx : gx;
                    hy = k ? hy + gy : gy;
                }
            }
            red[q * WAVE + lane] = make_double2(static_cast<double>(sx), static_cast<double>(sy));
            if constexpr (DELTA)
                red[(4 + (q >> 1)) * WAVE + lane] = make_double2(static_cast<double>(hx), static_cast<double>(hy));
        });
        reduce_group<T, C>(A, rc, swz, red, lane, pw, base, j0 + 4 * g, Lm);
    });
}

// Schedules of the two sweeps.  FUSED: both sweeps compute the pivots (the
// forward sweep keeps d' and the previous pivot at segment starts; the backward
// pass recomputes each segment from them).  STREAM: both sweeps read the pivots
// of the cached factorization.  HYBRID: the forward sweep reads them and keeps
// the previous pivot at segment starts; the backward pass recomputes each
// segment's pivots.
enum Sched { FUSED = 0, STREAM = 1, HYBRID = 2 };

template <int SCHED>
constexpr int ckpt_words() { return SCHED == STREAM ? 1 : 2; }

// One wave solves one chain for up to 64 PS poles (PS: the launch's poles per
// lane): lane l carries poles 64 PS pw + 64 k + l, k < P, whose sweeps share
// every row record and are interleaved row by row.  P = PS except in the last
// pole wave when at most 64 poles are left there (P = 1: no lane sweeps a
// padding pole next to a real one).  Checkpoints and partial sums are laid out
// for PS.
template <typename T, int S, int C, int SCHED, int P, int PS>
__device__ __forceinline__ void solve_chain(const SolveArgs& A, int task, int m, int pb, unsigned char* smem) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x / WAVE;
    const int nw = blockDim.x / WAVE;
    const int pw = pb * nw + wv;                 // pole wave: poles 64 PS pw .. 64 PS (pw + 1) - 1
    const int Lm = A.L - m + 1;
    const int base = m * (2 * A.L + 3 - m) / 2;
    const int nseg = (Lm + S - 1) / S;
    constexpr int CKW = ckpt_words<SCHED>();

    // the chain's row records, shared by all waves of the block: built here from
    // the state and the mode coefficients (fused schedule; row j of chain C is
    // a delta row when j and C have the same parity), else copied from the
    // records the factorization was built from
    RecT<T>* rc = reinterpret_cast<RecT<T>*>(smem);
    if constexpr (SCHED == FUSED) {
        for (int j = threadIdx.x; j < Lm; j += blockDim.x) {
            const int idx = base + j;
            const ModeCoef cf = A.coef[idx];
            const double ac = j > 0 ? coupling_product(cf, A.coef[idx - 1], A.dt) : 0.0;
            const RowRec r = ((j & 1) == C) ? delta_row(cf, ac, A.U0[idx], A.U0[2 * A.modes + idx], A.dt, A.H)
                                            : zeta_row(cf, ac, A.U0[A.modes + idx], A.dt);
            if constexpr (std::is_same<T, float>::value) rc[j] = round_rec(r); else rc[j] = r;
        }
    } else {
        static_assert(sizeof(RecT<T>) % sizeof(uint4) == 0, "records are copied in 16-byte units");
        const uint4* src = reinterpret_cast<const uint4*>(chain_records<T>(A, 2 * base + C * Lm));
        uint4* dst = reinterpret_cast<uint4*>(rc);
        const int nq = Lm * static_cast<int>(sizeof(RecT<T>) / sizeof(uint4));
        for (int i = threadIdx.x; i < nq; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    // whole waves of padding poles have nothing to do
    if (pw * WAVE * PS >= A.N) return;

    Lane ln[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int n = pw * WAVE * PS + k * WAVE + lane;
        ln[k].p = A.poles[n < A.N ? n : 0];
        if (n >= A.N) ln[k].p.wr = ln[k].p.wi = 0.0;   // padding lanes add nothing
        ln[k].wzr = __builtin_fma(ln[k].p.wr, ln[k].p.zir, -(ln[k].p.wi * ln[k].p.zii));
        ln[k].wzi = __builtin_fma(ln[k].p.wr, ln[k].p.zii, ln[k].p.wi * ln[k].p.zir);
        ln[k].wrf = static_cast<float>(ln[k].p.wr);
        ln[k].wif = static_cast<float>(ln[k].p.wi);
        ln[k].wzrf = static_cast<float>(ln[k].wzr);
        ln[k].wzif = static_cast<float>(ln[k].wzi);
        ln[k].zrf = static_cast<float>(ln[k].p.zr);
        ln[k].zif = static_cast<float>(ln[k].p.zi);
        ln[k].zirf = static_cast<float>(ln[k].p.zir);
        ln[k].ziif = static_cast<float>(ln[k].p.zii);
    }
    // sum of w/z over the wave's poles (lane-local in pole order, then an xor
    // butterfly: every lane ends with the same bits, as each step adds the same
    // two values)
    double2 swz = make_double2(ln[0].wzr, ln[0].wzi);
#pragma unroll
    for (int k = 1; k < P; ++k) {
        swz.x += ln[k].wzr;
        swz.y += ln[k].wzi;
    }
#pragma unroll
    for (int msk = 1; msk < WAVE; msk <<= 1) {
        swz.x += __shfl_xor(swz.x, msk);
        swz.y += __shfl_xor(swz.y, msk);
    }
    swz = make_double2(wave_uniform(swz.x), wave_uniform(swz.y));   // scalar registers

    double2* red = reinterpret_cast<double2*>(smem + static_cast<size_t>(A.rec_bytes) +
                                              static_cast<size_t>(wv) * sizeof(double2) * 6 * WAVE);
    // segment-start states of this wave: [nck_max][CKW][P][64]
    Cx<T>* ck = reinterpret_cast<Cx<T>*>(A.ckpt) +
                (static_cast<size_t>(task) * A.npb * nw + pw) * A.nck_max * CKW * PS * WAVE + lane;
    // cached pivots of this chain: row j, pole n at fact[(row0 + j) npad + n]
    const Cx<T>* fact = reinterpret_cast<const Cx<T>*>(A.fact) + static_cast<size_t>(2 * base + C * Lm) * A.npad +
                        pw * PS * WAVE + lane;

    // the recurrence state: the previous row's pivot pp and d'
    Cx<T> pp[P], dp[P];
#pragma unroll
    for (int k = 0; k < P; ++k) pp[k] = dp[k] = Cx<T>{T(0), T(0)};
    // per segment row: the pivot p_j, replaced by c'_j = c_j p_j once the row's
    // d'_j is formed (the back-substitution needs only c'_j and d'_j)
    Cx<T> ps[P][S], ds[P][S];
    // forward sweep over the full segments, keeping the state entering each later one
    for (int seg = 0; seg < nseg - 1; ++seg) {
        if (seg > 0) {
            Cx<T>* c0 = ck + static_cast<size_t>((seg - 1) * CKW) * P * WAVE;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                c0[k * WAVE] = dp[k];
                if constexpr (CKW == 2) c0[(P + k) * WAVE] = pp[k];
            }
        }
        const RecT<T>* rs = rc + seg * S;
        if constexpr (SCHED == FUSED) {
            static_for<0, S>([&](auto Q) {
                constexpr int jj = decltype(Q)::value;
                constexpr bool DELTA = ((jj + C) & 1) == 0;
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    const Cx<T> p = pivot_row<T, DELTA>(rs[jj], ln[k], pp[k]);
                    forward_rhs<T, DELTA>(rs[jj], ln[k], p, dp[k]);
                }
            });
        } else {
            const Cx<T>* fseg = fact + static_cast<size_t>(seg * S) * A.npad;
            static_for<0, S>([&](auto Q) {
                constexpr int jj = decltype(Q)::value;
#pragma unroll
                for (int k = 0; k < P; ++k) ps[k][jj] = fseg[static_cast<size_t>(jj) * A.npad + k * WAVE];
            });
            static_for<0, S>([&](auto Q) {
                constexpr int jj = decltype(Q)::value;
                constexpr bool DELTA = ((jj + C) & 1) == 0;
#pragma unroll
                for (int k = 0; k < P; ++k) forward_rhs<T, DELTA>(rs[jj], ln[k], ps[k][jj], dp[k]);
            });
            if constexpr (SCHED == HYBRID) {
#pragma unroll
                for (int k = 0; k < P; ++k) pp[k] = ps[k][S - 1];
            }
        }
    }
    // the last segment is swept into registers and back-substituted at once
    Cx<T> vnext[P];
#pragma unroll
    for (int k = 0; k < P; ++k) vnext[k] = Cx<T>{T(0), T(0)};
    {
        const int j0 = (nseg - 1) * S;
        const Cx<T>* fseg = fact + static_cast<size_t>(j0) * A.npad;
        static_for<0, S>([&](auto Q) {
            constexpr int jj = decltype(Q)::value;
            constexpr bool DELTA = ((jj + C) & 1) == 0;
            if (j0 + jj < Lm) {
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    if constexpr (SCHED == STREAM) {
                        const Cx<T> p = fseg[static_cast<size_t>(jj) * A.npad + k * WAVE];
                        forward_rhs<T, DELTA>(rc[j0 + jj], ln[k], p, dp[k]);
                        ps[k][jj] = upper_factor<T>(rc[j0 + jj], p);
                    } else {
                        const Cx<T> p = pivot_row<T, DELTA>(rc[j0 + jj], ln[k], pp[k]);
                        forward_rhs<T, DELTA>(rc[j0 + jj], ln[k], p, dp[k]);
                        ps[k][jj] = upper_factor<T>(rc[j0 + jj], p);
                    }
                    ds[k][jj] = dp[k];
                }
            }
        });
        back_segment<T, S, C, P>(A, ln, rc, j0, Lm, base, pw, lane, ps, ds, vnext, swz, red);
    }
    // earlier segments: rebuild pivots and d' from the checkpoint, then back-substitute
    for (int seg = nseg - 2; seg >= 0; --seg) {
        const int j0 = seg * S;
        Cx<T> d[P], c[P];   // d' and the pivot of the row before the segment
#pragma unroll
        for (int k = 0; k < P; ++k) {
            d[k] = c[k] = Cx<T>{T(0), T(0)};
            if (seg > 0) {
                const Cx<T>* c0 = ck + static_cast<size_t>((seg - 1) * CKW) * P * WAVE;
                d[k] = c0[k * WAVE];
                if constexpr (CKW == 2) c[k] = c0[(P + k) * WAVE];
            }
        }
        if constexpr (SCHED == STREAM) {
            const Cx<T>* fseg = fact + static_cast<size_t>(j0) * A.npad;
            static_for<0, S>([&](auto Q) {
                constexpr int jj = decltype(Q)::value;
#pragma unroll
                for (int k = 0; k < P; ++k) ps[k][jj] = fseg[static_cast<size_t>(jj) * A.npad + k * WAVE];
            });
        }
        static_for<0, S>([&](auto Q) {
            constexpr int jj = decltype(Q)::value;
            constexpr bool DELTA = ((jj + C) & 1) == 0;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                if constexpr (SCHED == STREAM) {
                    forward_rhs<T, DELTA>(rc[j0 + jj], ln[k], ps[k][jj], d[k]);
                    ps[k][jj] = upper_factor<T>(rc[j0 + jj], ps[k][jj]);
                } else {
                    const Cx<T> p = pivot_row<T, DELTA>(rc[j0 + jj], ln[k], c[k]);
                    forward_rhs<T, DELTA>(rc[j0 + jj], ln[k], p, d[k]);
                    ps[k][jj] = upper_factor<T>(rc[j0 + jj], p);   // c'_j
                }
                ds[k][jj] = d[k];
            }
        });
        back_segment<T, S, C, P>(A, ln, rc, j0, Lm, base, pw, lane, ps, ds, vnext, swz, red);
    }
}

// Waves per SIMD the register allocation must allow: two where the segment
// registers (pivot and d' of S rows for P poles) take at most 128 VGPRs.
template <typename T, int S, int P>
constexpr int chain_occupancy() { return sizeof(T) * S * P <= 128 ? 2 : 1; }

// The chain of `task` for the pole waves of block pb: with two poles per lane,
// a last pole wave holding at most 64 poles runs with one pole per lane.
template <typename T, int S, int SCHED, int P>
__device__ __forceinline__ void solve_task(const SolveArgs& A, int task, int pb, unsigned char* smem) {
    const int m = task >> 1;
    const int pw = pb * static_cast<int>(blockDim.x / WAVE) + static_cast<int>(threadIdx.x / WAVE);
    const bool tail = P == 2 && pw * WAVE * P + WAVE >= A.N;
    if (task & 1) {
        if (tail) solve_chain<T, S, 1, SCHED, 1, P>(A, task, m, pb, smem);
        else solve_chain<T, S, 1, SCHED, P, P>(A, task, m, pb, smem);
    } else {
        if (tail) solve_chain<T, S, 0, SCHED, 1, P>(A, task, m, pb, smem);
        else solve_chain<T, S, 0, SCHED, P, P>(A, task, m, pb, smem);
    }
}

template <typename T, int S, int SCHED, int P>
__global__ __launch_bounds__(4 * WAVE) __attribute__((amdgpu_waves_per_eu(chain_occupancy<T, S, P>())))
void rexi_chain_kernel(SolveArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int task = blockIdx.x / A.npb;      // task = 2 m + chain: longest chains first
    const int pb = blockIdx.x - task * A.npb;
    solve_task<T, S, SCHED, P>(A, task, pb, smem);
}

// Ensemble form: one launch over the work items (member, task, pole block) of
// several independent problems of the same precision and launch shape; the
// host orders the items longest chain first.
template <typename T, int S, int SCHED, int P>
__global__ __launch_bounds__(4 * WAVE) __attribute__((amdgpu_waves_per_eu(chain_occupancy<T, S, P>())))
void rexi_chain_batched_kernel(const SolveArgs* __restrict__ args, const int4* __restrict__ items) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int4 it = items[blockIdx.x];
    const SolveArgs A = args[it.x];
    solve_task<T, S, SCHED, P>(A, it.y, it.z, smem);
}

// Factorization: the pivots of every chain row for every pole (padding lanes up
// to npad use pole 0), stored at fact[(chain row) npad + pole].  One thread per
// pole, one workgroup per (task, block of poles); depends on z, dt and the
// operator only, so it is reused while they stay the same.
template <typename T>
__global__ __launch_bounds__(256) void rexi_factor_kernel(const RecT<T>* __restrict__ rec,
                                                          const PoleData* __restrict__ poles, Cx<T>* __restrict__ fact,
                                                          int L, int N, int npad, int fpb) {
    const int task = blockIdx.x / fpb;
    const int n = (blockIdx.x - task * fpb) * blockDim.x + threadIdx.x;
    if (n >= npad) return;
    const int m = task >> 1, C = task & 1;
    const int Lm = L - m + 1;
    const int base = m * (2 * L + 3 - m) / 2;
    Lane ln;
    ln.p = poles[n < N ? n : 0];
    ln.zrf = static_cast<float>(ln.p.zr);
    ln.zif = static_cast<float>(ln.p.zi);
    ln.zirf = static_cast<float>(ln.p.zir);
    ln.ziif = static_cast<float>(ln.p.zii);
    const RecT<T>* rc = rec + 2 * base + C * Lm;
    Cx<T>* out = fact + static_cast<size_t>(2 * base + C * Lm) * npad + n;
    Cx<T> pp{T(0), T(0)};
    for (int j = 0; j < Lm; ++j) {
        const RecT<T> R = rc[j];
        const Cx<T> p = ((j + C) & 1) == 0 ? pivot_row<T, true>(R, ln, pp) : pivot_row<T, false>(R, ln, pp);
        out[static_cast<size_t>(j) * npad] = p;
    }
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const double2* __restrict__ part,
                                                           double2* __restrict__ U1, int count, int nparts,
                                                           unsigned* status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const double2 v = sum_parts(part, count, nparts, i);
    note_nonfinite(status, v.x + v.y, STATUS_REXI);
    U1[i] = v;
}

// Ensemble form: member blockIdx.y (count = 0: the member has one pole wave
// and its solve wrote U1 directly).
struct SumArgs {
    const double2* part;
    double2* U1;
    int count, nparts;
    unsigned* status;
};

__global__ __launch_bounds__(256) void sum_partials_batched_kernel(const SumArgs* __restrict__ args) {
    const SumArgs a = args[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.count) return;
    const double2 v = sum_parts(a.part, a.count, a.nparts, i);
    note_nonfinite(a.status, v.x + v.y, STATUS_REXI);
    a.U1[i] = v;
}

// The factorization cache of a context: reserve_factors sizes it (dropping a
// cache of another size), build_factors fills it from the row records of the
// current call when it is not valid for the cached coefficient set, dt and T.
template <typename T>
int reserve_factors(swe_ctx* ctx, const SolveArgs& A) {
    const size_t bytes = sizeof(Cx<T>) * 2 * static_cast<size_t>(A.modes) * A.npad;
    if (bytes > ctx->fact_cap) {
        if (ctx->d_fact) REXI_HIP(hipFree(ctx->d_fact));
        ctx->d_fact = nullptr;
        ctx->fact_cap = 0;
        ctx->fact_valid = false;
        if (hipMalloc(&ctx->d_fact, bytes) != hipSuccess)
            return fail(REXI_ENOMEM, "rexi solve: cannot allocate the factorization cache");
        ctx->fact_cap = bytes;
    }
    return REXI_OK;
}

template <typename T>
int build_factors(swe_ctx* ctx, const SolveArgs& A, hipStream_t stream) {
    const int tprec = std::is_same<T, float>::value ? 1 : 2;
    if (ctx->fact_valid && ctx->fact_prec == tprec && ctx->fact_key == ctx->poles_key) return REXI_OK;
    const int threads = 256;
    const int fpb = (A.npad + threads - 1) / threads;
    const unsigned blocks = static_cast<unsigned>(2 * (A.L + 1) * fpb);
    const int slot = prof_begin(ctx, REXI_KERNEL_FACTOR, stream);
    hipLaunchKernelGGL((rexi_factor_kernel<T>), dim3(blocks), dim3(threads), 0, stream, chain_records<T>(A, 0), A.poles,
                       reinterpret_cast<Cx<T>*>(ctx->d_fact), A.L, A.N, A.npad, fpb);
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_FACTOR, slot, stream);
    ctx->fact_valid = true;
    ctx->fact_key = ctx->poles_key;
    ctx->fact_prec = tprec;
    return REXI_OK;
}

// Fills the shape-dependent fields of A and makes sure the context's
// factorization cache (STREAM, HYBRID; filled later by build_factors, once the
// row records of the call exist) and checkpoint workspace are allocated.
template <typename T, int S, int SCHED, int P>
int configure(swe_ctx* ctx, SolveArgs& A, int waves, hipStream_t stream) {
    const int nseg = (A.L + 1 + S - 1) / S;
    A.nck_max = nseg > 2 ? nseg - 2 : 0;
    A.rec_bytes = static_cast<int>(sizeof(RecT<T>)) * (A.L + 1);
    A.npb = (A.N + WAVE * P * waves - 1) / (WAVE * P * waves);
    constexpr int CKW = ckpt_words<SCHED>();
    if (SCHED != FUSED) {
        const int rc = reserve_factors<T>(ctx, A);
        if (rc != REXI_OK) return rc;
        A.fact = ctx->d_fact;
    }
    // segment-start states: one slot per (task, pole wave, checkpoint)
    const size_t ck_bytes = sizeof(Cx<T>) * 2 * static_cast<size_t>(A.L + 1) * A.npb * waves *
                            static_cast<size_t>(A.nck_max > 0 ? A.nck_max : 1) * CKW * P * WAVE;
    if (ck_bytes > ctx->ckpt_cap) {
        if (ctx->d_ckpt) REXI_HIP(hipFree(ctx->d_ckpt));
        ctx->d_ckpt = nullptr;
        ctx->ckpt_cap = 0;
        if (hipMalloc(&ctx->d_ckpt, ck_bytes) != hipSuccess)
            return fail(REXI_ENOMEM, "rexi solve: cannot allocate the checkpoint workspace");
        ctx->ckpt_cap = ck_bytes;
    }
    A.ckpt = ctx->d_ckpt;
    return REXI_OK;
}

template <typename KernelFn>
int prepare_lds(KernelFn* fn, size_t lds) {
    if (lds > 160 * 1024) return fail(REXI_ENOTSUP, "rexi solve: LDS need exceeds 160 KB; lower waves");
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                static_cast<int>(lds)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(REXI_ENOTSUP, "rexi solve: LDS need exceeds the device limit; lower waves");
        }
    }
    return REXI_OK;
}

template <typename T, int S, int SCHED, int P>
int launch_typed(swe_ctx* ctx, SolveArgs A, int waves, hipStream_t stream) {
    int rc = configure<T, S, SCHED, P>(ctx, A, waves, stream);
    if (rc != REXI_OK) return rc;
    if (SCHED != FUSED && (rc = build_factors<T>(ctx, A, stream)) != REXI_OK) return rc;
    const size_t lds = static_cast<size_t>(A.rec_bytes) + sizeof(double2) * 6 * WAVE * waves;
    if ((rc = prepare_lds(&rexi_chain_kernel<T, S, SCHED, P>, lds)) != REXI_OK) return rc;
    const unsigned blocks = static_cast<unsigned>(2 * (A.L + 1) * A.npb);
    const int slot = prof_begin(ctx, REXI_KERNEL_SOLVE, stream);
    hipLaunchKernelGGL((rexi_chain_kernel<T, S, SCHED, P>), dim3(blocks), dim3(WAVE * waves), lds, stream, A);
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_SOLVE, slot, stream);
    return REXI_OK;
}

// ---- ensemble launch ---------------------------------------------------------

// Device copy of an ensemble's per-member arguments and work items, kept in the
// first member's context and re-uploaded only when the key changes.
struct BatchPlan {
    uint64_t key = 0;
    void* d_args = nullptr;     // SolveArgs[count]
    void* d_rows = nullptr;     // RowsArgs[count]
    void* d_sum = nullptr;      // SumArgs[count]
    void* d_items = nullptr;    // int4[nitems]
    size_t args_cap = 0, items_cap = 0;
    int nitems = 0, max_count = 0, max_modes = 0, max_L = 0;
    size_t lds = 0;
};

uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
    return h;
}

template <typename T, int S, int SCHED, int P>
int launch_batched_typed(const BatchMember* mem, int count, const Tuning& t, hipStream_t stream, SolveArgs* A,
                         BatchPlan& plan) {
    const int waves = t.waves;
    int rc;
    size_t rec_max = 0;
    for (int i = 0; i < count; ++i) {
        if ((rc = configure<T, S, SCHED, P>(mem[i].ctx, A[i], waves, stream)) != REXI_OK) return rc;
        rec_max = std::max(rec_max, static_cast<size_t>(A[i].rec_bytes));
    }
    for (int i = 0; i < count; ++i) A[i].rec_bytes = static_cast<int>(rec_max);
    const size_t lds = rec_max + sizeof(double2) * 6 * WAVE * waves;
    if ((rc = prepare_lds(&rexi_chain_batched_kernel<T, S, SCHED, P>, lds)) != REXI_OK) return rc;

    uint64_t key = 1469598103934665603ULL;
    key = mix(key, static_cast<uint64_t>(count));
    key = mix(key, static_cast<uint64_t>(t.solver * 1000 + t.seg_rows * 10 + t.poles_per_lane) * 8 + waves);
    for (int i = 0; i < count; ++i) {
        const unsigned char* b = reinterpret_cast<const unsigned char*>(&A[i]);
        for (size_t k = 0; k < sizeof(SolveArgs); k += 8) {
            uint64_t v = 0;
            std::memcpy(&v, b + k, std::min<size_t>(8, sizeof(SolveArgs) - k));
            key = mix(key, v);
        }
        key = mix(key, reinterpret_cast<uintptr_t>(mem[i].U0));
        key = mix(key, reinterpret_cast<uintptr_t>(mem[i].U1));
        uint64_t dtb;
        std::memcpy(&dtb, &mem[i].dt, 8);
        key = mix(key, dtb);
    }
    if (key != plan.key || !plan.d_args) {
        // work items, longest chains first (ties: member order, then task, then pole block)
        std::vector<int4> items;
        for (int i = 0; i < count; ++i)
            for (int task = 0; task < 2 * (A[i].L + 1); ++task)
                for (int pb = 0; pb < A[i].npb; ++pb) items.push_back(make_int4(i, task, pb, A[i].L - (task >> 1) + 1));
        std::stable_sort(items.begin(), items.end(), [](const int4& a, const int4& b) { return a.w > b.w; });
        std::vector<RowsArgs> rows(count);
        std::vector<SumArgs> sums(count);
        int max_modes = 0, max_L = 0;
        for (int i = 0; i < count; ++i) {
            swe_ctx* c = mem[i].ctx;
            rows[i] = RowsArgs{reinterpret_cast<const double2*>(mem[i].U0), c->d_coef,
                               reinterpret_cast<RowRec*>(c->d_rows), reinterpret_cast<RowRec32*>(c->d_rows32), c->L,
                               c->modes, mem[i].dt, c->H};
            const int nparts = (mem[i].N + WAVE * P - 1) / (WAVE * P);
            sums[i] = SumArgs{reinterpret_cast<const double2*>(c->d_partial), reinterpret_cast<double2*>(mem[i].U1),
                              nparts > 1 ? 3 * c->modes : 0, nparts, c->d_status};
            max_modes = std::max(max_modes, c->modes);
            max_L = std::max(max_L, c->L);
        }
        const size_t abytes = (sizeof(SolveArgs) + sizeof(RowsArgs) + sizeof(SumArgs)) * count;
        if (abytes > plan.args_cap) {
            for (void** p : {&plan.d_args, &plan.d_rows, &plan.d_sum}) {
                if (*p) REXI_HIP(hipFree(*p));
                *p = nullptr;
            }
            plan.args_cap = 0;
            if (hipMalloc(&plan.d_args, sizeof(SolveArgs) * count) != hipSuccess ||
                hipMalloc(&plan.d_rows, sizeof(RowsArgs) * count) != hipSuccess ||
                hipMalloc(&plan.d_sum, sizeof(SumArgs) * count) != hipSuccess)
                return fail(REXI_ENOMEM, "rexi_linear_step_batched: cannot allocate the ensemble plan");
            plan.args_cap = abytes;
        }
        if (sizeof(int4) * items.size() > plan.items_cap) {
            if (plan.d_items) REXI_HIP(hipFree(plan.d_items));
            plan.d_items = nullptr;
            plan.items_cap = 0;
            if (hipMalloc(&plan.d_items, sizeof(int4) * items.size()) != hipSuccess)
                return fail(REXI_ENOMEM, "rexi_linear_step_batched: cannot allocate the work items");
            plan.items_cap = sizeof(int4) * items.size();
        }
        // host arrays die at return: copy synchronously with respect to the host
        REXI_HIP(hipMemcpyAsync(plan.d_args, A, sizeof(SolveArgs) * count, hipMemcpyHostToDevice, stream));
        REXI_HIP(hipMemcpyAsync(plan.d_rows, rows.data(), sizeof(RowsArgs) * count, hipMemcpyHostToDevice, stream));
        REXI_HIP(hipMemcpyAsync(plan.d_sum, sums.data(), sizeof(SumArgs) * count, hipMemcpyHostToDevice, stream));
        REXI_HIP(hipMemcpyAsync(plan.d_items, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice, stream));
        REXI_HIP(hipStreamSynchronize(stream));
        plan.key = key;
        plan.nitems = static_cast<int>(items.size());
        plan.max_count = count;
        plan.max_modes = max_modes;
        plan.max_L = max_L;
    }
    swe_ctx* c0 = mem[0].ctx;
    if (SCHED != FUSED) {
        hipLaunchKernelGGL(rexi_rows_batched_kernel, dim3(plan.max_L + 1, count), dim3(256), 0, stream,
                           reinterpret_cast<const RowsArgs*>(plan.d_rows));
        REXI_HIP(hipGetLastError());
    }
    if (SCHED != FUSED) {
        // factorizations that are missing are built now that the row records exist
        for (int i = 0; i < count; ++i)
            if ((rc = build_factors<T>(mem[i].ctx, A[i], stream)) != REXI_OK) return rc;
    }
    const int slot = prof_begin(c0, REXI_KERNEL_SOLVE, stream);
    hipLaunchKernelGGL((rexi_chain_batched_kernel<T, S, SCHED, P>), dim3(plan.nitems), dim3(WAVE * waves), lds,
                       stream, reinterpret_cast<const SolveArgs*>(plan.d_args),
                       reinterpret_cast<const int4*>(plan.d_items));
    REXI_HIP(hipGetLastError());
    prof_end(c0, REXI_KERNEL_SOLVE, slot, stream);
    {
        const int threads = 256;
        const int slot2 = prof_begin(c0, REXI_KERNEL_REDUCE, stream);
        hipLaunchKernelGGL(sum_partials_batched_kernel, dim3((3 * plan.max_modes + threads - 1) / threads, count),
                           dim3(threads), 0, stream, reinterpret_cast<const SumArgs*>(plan.d_sum));
        REXI_HIP(hipGetLastError());
        prof_end(c0, REXI_KERNEL_REDUCE, slot2, stream);
    }
    return REXI_OK;
}

template <typename T, int S, int P>
int batched_sched(const BatchMember* mem, int count, const Tuning& t, hipStream_t stream, SolveArgs* A,
                  BatchPlan& plan) {
    switch (t.solver) {
        case REXI_SOLVER_STREAM: return launch_batched_typed<T, S, STREAM, P>(mem, count, t, stream, A, plan);
        case REXI_SOLVER_HYBRID: return launch_batched_typed<T, S, HYBRID, P>(mem, count, t, stream, A, plan);
        default: return launch_batched_typed<T, S, FUSED, P>(mem, count, t, stream, A, plan);
    }
}

template <typename T>
int batched_shape(const BatchMember* mem, int count, const Tuning& t, hipStream_t stream, SolveArgs* A,
                  BatchPlan& plan) {
    if (t.poles_per_lane == 2) {
        if (t.seg_rows == 8) return batched_sched<T, 8, 2>(mem, count, t, stream, A, plan);
        if (t.seg_rows == 16) return batched_sched<T, 16, 2>(mem, count, t, stream, A, plan);
    } else {
        if (t.seg_rows == 16) return batched_sched<T, 16, 1>(mem, count, t, stream, A, plan);
        if (t.seg_rows == 32) return batched_sched<T, 32, 1>(mem, count, t, stream, A, plan);
    }
    return fail(REXI_ENOTSUP, "rexi solve: seg_rows must be 16 or 32 with one pole per lane, 8 or 16 with two");
}

template <typename T, int S, int P>
int launch_sched(swe_ctx* ctx, const SolveArgs& A, int waves, int sched, hipStream_t stream) {
    switch (sched) {
        case REXI_SOLVER_STREAM: return launch_typed<T, S, STREAM, P>(ctx, A, waves, stream);
        case REXI_SOLVER_HYBRID: return launch_typed<T, S, HYBRID, P>(ctx, A, waves, stream);
        default: return launch_typed<T, S, FUSED, P>(ctx, A, waves, stream);
    }
}

// Supported shapes: one pole per lane with 16- or 32-row segments, two poles
// per lane with 8- or 16-row segments (the segment registers of 32 rows for two
// poles would not fit).
template <typename T>
int launch_shape(swe_ctx* ctx, const SolveArgs& A, const Tuning& t, hipStream_t stream) {
    if (t.poles_per_lane == 2) {
        if (t.seg_rows == 8) return launch_sched<T, 8, 2>(ctx, A, t.waves, t.solver, stream);
        if (t.seg_rows == 16) return launch_sched<T, 16, 2>(ctx, A, t.waves, t.solver, stream);
    } else {
        if (t.seg_rows == 16) return launch_sched<T, 16, 1>(ctx, A, t.waves, t.solver, stream);
        if (t.seg_rows == 32) return launch_sched<T, 32, 1>(ctx, A, t.waves, t.solver, stream);
    }
    return fail(REXI_ENOTSUP, "rexi solve: seg_rows must be 16 or 32 with one pole per lane, 8 or 16 with two");
}

// Shape-independent arguments of one member's solve; allocates the row records
// and (for more than one pole wave) the partial sums.
int base_args(swe_ctx* ctx, int N, double dt, const double* U0, const double* U1, int P, SolveArgs& A, int& nparts) {
    if (!ctx->d_rows) {
        if (hipMalloc(&ctx->d_rows, sizeof(RowRec) * 2 * static_cast<size_t>(ctx->modes)) != hipSuccess ||
            hipMalloc(&ctx->d_rows32, sizeof(RowRec32) * 2 * static_cast<size_t>(ctx->modes)) != hipSuccess)
            return fail(REXI_ENOMEM, "rexi solve: cannot allocate row records");
    }
    A.rec = reinterpret_cast<const RowRec*>(ctx->d_rows);
    A.rec32 = reinterpret_cast<const RowRec32*>(ctx->d_rows32);
    A.poles = ctx->d_poles;
    A.L = ctx->L;
    A.modes = ctx->modes;
    A.N = N;
    // the factorization layout pads the pole axis to whole pairs of waves for every launch shape
    A.npad = (N + 2 * WAVE - 1) / (2 * WAVE) * (2 * WAVE);
    nparts = (N + WAVE * P - 1) / (WAVE * P);          // pole waves that produce partial sums
    A.dtH = dt * ctx->H;
    A.U0 = reinterpret_cast<const double2*>(U0);
    A.coef = ctx->d_coef;
    A.dt = dt;
    A.H = ctx->H;
    A.fact = nullptr;
    A.ckpt = nullptr;
    A.npb = A.nck_max = A.rec_bytes = 0;
    A.status = ctx->d_status;
    const size_t count = static_cast<size_t>(3) * ctx->modes;
    if (nparts == 1) {
        A.out = reinterpret_cast<double2*>(const_cast<double*>(U1));
    } else {
        const size_t need = 2 * count * nparts;
        if (need > ctx->partial_cap) {
            if (ctx->d_partial) REXI_HIP(hipFree(ctx->d_partial));
            ctx->d_partial = nullptr;
            ctx->partial_cap = 0;
            if (hipMalloc(&ctx->d_partial, need * sizeof(double)) != hipSuccess)
                return fail(REXI_ENOMEM, "rexi solve: cannot allocate partial sums");
            ctx->partial_cap = need;
        }
        A.out = reinterpret_cast<double2*>(ctx->d_partial);
    }
    return REXI_OK;
}

}  // namespace

int launch_rexi_solve(swe_ctx* ctx, int N, double dt, const double* U0, double* U1, hipStream_t stream) {
    int nparts = 0;
    int rc = launch_rexi_chain(ctx, N, dt, U0, U1, &nparts, stream);
    if (rc != REXI_OK) return rc;
    return nparts > 1 ? launch_rexi_sum(ctx, nparts, U1, stream) : REXI_OK;
}

int launch_rexi_sum(swe_ctx* ctx, int nparts, double* U1, hipStream_t stream) {
    const int threads = 256;
    const int count = 3 * ctx->modes;
    const unsigned blocks = static_cast<unsigned>((count + threads - 1) / threads);
    const int slot = prof_begin(ctx, REXI_KERNEL_REDUCE, stream);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(blocks), dim3(threads), 0, stream,
                       reinterpret_cast<const double2*>(ctx->d_partial), reinterpret_cast<double2*>(U1), count,
                       nparts, ctx->d_status);
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_REDUCE, slot, stream);
    return REXI_OK;
}

int launch_rexi_chain(swe_ctx* ctx, int N, double dt, const double* U0, double* U1, int* nparts_out,
                      hipStream_t stream) {
    SolveArgs A;
    int nparts = 0;
    int rc = base_args(ctx, N, dt, U0, U1, ctx->tune.poles_per_lane, A, nparts);
    if (rc != REXI_OK) return rc;
    *nparts_out = nparts;
    if (ctx->tune.solver == REXI_SOLVER_STREAM || ctx->tune.solver == REXI_SOLVER_HYBRID) {
        // the streaming schedules read (and factorize) records built in HBM
        hipLaunchKernelGGL(rexi_rows_kernel, dim3(ctx->L + 1), dim3(256), 0, stream,
                           reinterpret_cast<const double2*>(U0), ctx->d_coef, reinterpret_cast<RowRec*>(ctx->d_rows),
                           reinterpret_cast<RowRec32*>(ctx->d_rows32), ctx->L, ctx->modes, dt, ctx->H);
        REXI_HIP(hipGetLastError());
    }
    const bool fp32 = (ctx->prec & REXI_PREC_FP32_SOLVE) != 0;
    return fp32 ? launch_shape<float>(ctx, A, ctx->tune, stream) : launch_shape<double>(ctx, A, ctx->tune, stream);
}

namespace {

// REXI sums of the gravity-wave part alone.  L_g leaves zeta alone and couples
// (h_l, delta_l) of one degree: (z - dt L_g) = [[z, dt H], [-dt gN_l, z]], gN_l =
// g l(l+1)/a^2, so sum_n w_n (z_n - dt L_g)^-1 = [[A_l, -dt H B_l], [dt gN_l B_l, A_l]]
// with A_l = sum w z / (z^2 + c_l), B_l = sum w / (z^2 + c_l), c_l = dt^2 H gN_l.
// One workgroup per degree l (l = L + 1 gives S(0) = sum w / z for zeta);
// each thread sums a strided share of the poles with compensation, then the
// workgroup adds the 256 shares in a fixed tree.
__global__ __launch_bounds__(256) void lg_sums_kernel(const PoleData* __restrict__ poles, int N, int L, double c1,
                                                      double2* __restrict__ AB) {
    __shared__ double red[4][256];
    const int l = blockIdx.x;
    const double c = l <= L ? c1 * l * (l + 1.0) : 0.0;
    double s[4] = {0.0, 0.0, 0.0, 0.0}, e[4] = {0.0, 0.0, 0.0, 0.0};
    auto add = [&](int k, double v) {
        const double t = s[k] + v;
        e[k] += (fabs(s[k]) >= fabs(v)) ? (s[k] - t) + v : (v - t) + s[k];
        s[k] = t;
    };
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const PoleData q = poles[n];
        // d = z^2 + c, then w / d and w z / d
        const double dr = __builtin_fma(q.zr, q.zr, __builtin_fma(-q.zi, q.zi, c));
        const double di = 2.0 * q.zr * q.zi;
        const double den = __builtin_fma(dr, dr, di * di);
        const double ir = dr / den, ii = -di / den;                 // 1 / d
        const double br = __builtin_fma(q.wr, ir, -(q.wi * ii));    // w / d
        const double bi = __builtin_fma(q.wr, ii, q.wi * ir);
        const double ar = __builtin_fma(br, q.zr, -(bi * q.zi));    // w z / d
        const double ai = __builtin_fma(br, q.zi, bi * q.zr);
        add(0, ar);
        add(1, ai);
        add(2, br);
        add(3, bi);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = s[k] + e[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
#pragma unroll
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        AB[2 * l] = make_double2(red[0][0], red[1][0]);
        AB[2 * l + 1] = make_double2(red[2][0], red[3][0]);
    }
}

// U1 = (sum over poles) U0 per mode; one workgroup per order m.  U1 may equal U0.
__global__ __launch_bounds__(256) void lg_apply_kernel(const double2* U0, double2* U1, const double2* __restrict__ AB,
                                                       int L, int modes, double dtH, double dtg_a2, unsigned* status) {
    const int m = blockIdx.x;
    const int base = m * (2 * L + 3 - m) / 2;
    const double2 S0 = AB[2 * (L + 1)];
    for (int j = threadIdx.x; j < L - m + 1; j += blockDim.x) {
        const int l = m + j, idx = base + j;
        const double2 A = AB[2 * l], B = AB[2 * l + 1];
        const double2 h = U0[idx], z = U0[modes + idx], d = U0[2 * modes + idx];
        const double gn = dtg_a2 * l * (l + 1.0);                    // dt g l(l+1)/a^2
        const double2 hb = make_double2(-dtH * B.x, -dtH * B.y);     // -dt H B
        const double2 db = make_double2(gn * B.x, gn * B.y);         // dt gN B
        const double2 h1 = make_double2(__builtin_fma(A.x, h.x, -(A.y * h.y)) + __builtin_fma(hb.x, d.x, -(hb.y * d.y)),
                                        __builtin_fma(A.x, h.y, A.y * h.x) + __builtin_fma(hb.x, d.y, hb.y * d.x));
        const double2 d1 = make_double2(__builtin_fma(db.x, h.x, -(db.y * h.y)) + __builtin_fma(A.x, d.x, -(A.y * d.y)),
                                        __builtin_fma(db.x, h.y, db.y * h.x) + __builtin_fma(A.x, d.y, A.y * d.x));
        const double2 z1 = make_double2(__builtin_fma(S0.x, z.x, -(S0.y * z.y)), __builtin_fma(S0.x, z.y, S0.y * z.x));
        note_nonfinite(status, (h1.x + h1.y) + (z1.x + z1.y) + (d1.x + d1.y), STATUS_REXI);
        U1[idx] = h1;
        U1[modes + idx] = z1;
        U1[2 * modes + idx] = d1;
    }
}

}  // namespace

int launch_rexi_lg_on(swe_ctx* ctx, const PoleData* poles, void* sums, int N, double dt, const double* U0,
                      double* U1, hipStream_t stream) {
    const double c1 = dt * dt * ctx->H * ctx->g / (ctx->a * ctx->a);
    hipLaunchKernelGGL(lg_sums_kernel, dim3(ctx->L + 2), dim3(256), 0, stream, poles, N, ctx->L, c1,
                       reinterpret_cast<double2*>(sums));
    REXI_HIP(hipGetLastError());
    hipLaunchKernelGGL(lg_apply_kernel, dim3(ctx->L + 1), dim3(256), 0, stream, reinterpret_cast<const double2*>(U0),
                       reinterpret_cast<double2*>(U1), reinterpret_cast<const double2*>(sums), ctx->L,
                       ctx->modes, dt * ctx->H, dt * ctx->g / (ctx->a * ctx->a), ctx->d_status);
    REXI_HIP(hipGetLastError());
    return REXI_OK;
}

int launch_rexi_lg(swe_ctx* ctx, int N, double dt, const double* U0, double* U1, hipStream_t stream) {
    if (!ctx->d_lgsum) {
        if (hipMalloc(&ctx->d_lgsum, lg_sums_bytes(ctx->L)) != hipSuccess)
            return fail(REXI_ENOMEM, "rexi_lg_step: cannot allocate the per-degree sums");
    }
    const int slot = prof_begin(ctx, REXI_KERNEL_SOLVE, stream);
    const int rc = launch_rexi_lg_on(ctx, ctx->d_poles, ctx->d_lgsum, N, dt, U0, U1, stream);
    prof_end(ctx, REXI_KERNEL_SOLVE, slot, stream);
    return rc;
}

int launch_rexi_batched(const BatchMember* mem, int count, hipStream_t stream) {
    swe_ctx* c0 = mem[0].ctx;
    const Tuning t = c0->tune;
    std::vector<SolveArgs> A(count);
    for (int i = 0; i < count; ++i) {
        int nparts = 0;
        const int rc = base_args(mem[i].ctx, mem[i].N, mem[i].dt, mem[i].U0, mem[i].U1, t.poles_per_lane, A[i], nparts);
        if (rc != REXI_OK) return rc;
    }
    if (!c0->batch) c0->batch = new BatchPlan();
    BatchPlan& plan = *static_cast<BatchPlan*>(c0->batch);
    const bool fp32 = (c0->prec & REXI_PREC_FP32_SOLVE) != 0;
    return fp32 ? batched_shape<float>(mem, count, t, stream, A.data(), plan)
                : batched_shape<double>(mem, count, t, stream, A.data(), plan);
}

void free_batch_plan(swe_ctx* ctx) {
    if (!ctx->batch) return;
    BatchPlan* p = static_cast<BatchPlan*>(ctx->batch);
    for (void* q : {p->d_args, p->d_rows, p->d_sum, p->d_items})
        if (q) (void)hipFree(q);
    delete p;
    ctx->batch = nullptr;
}

}  // namespace rexi
