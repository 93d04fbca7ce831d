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
// Mapping: one wave per (m, chain, block of 64 poles); lane = pole, so every
// table value and right-hand side is wave-uniform (scalar loads) and the
// per-lane work is a sequential sweep over l.  The chain is cut into segments
// of S rows: a first forward sweep keeps only the state entering each segment
// (a checkpoint in LDS); the backward pass then re-sweeps one segment at a
// time into registers and back-substitutes through it.  The sum over the
// 64 poles of a wave is formed in LDS (write lane-major, read transposed,
// finish with a 3-step butterfly), in FP64, in a fixed order.  Blocks of
// poles write partial sums that a second kernel adds in pole-block order,
// so results are bit-reproducible.  The file is compiled without automatic
// FMA contraction and every fused multiply-add is written out, so all inlined
// copies of a step perform the same rounding.
#include <type_traits>
#include <utility>

#include "internal.h"

namespace rexi {
namespace {

constexpr int WAVE = 64;
constexpr int RED_SLOTS = 8;  // staging slots per reduction round (6 used)

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

__device__ __forceinline__ float rcp_refined(float n) {
    float r = __builtin_amdgcn_rcpf(n);
    float e = __builtin_fmaf(-n, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

struct SolveArgs {
    const double2* __restrict__ U0;     // [3][modes]
    double2* __restrict__ out;          // [npb][3][modes]
    const PoleData* __restrict__ poles; // [N]
    const ModeCoef* __restrict__ coef;  // [modes]
    int L, modes, N, npb;
    double dt, dt2H, dtH;
};

struct Lane {
    PoleData p;
    double wzr, wzi;   // w / z
};

// One forward Thomas step on row j (degree k = m + j) of a chain.
template <typename T, bool DELTA>
__device__ __forceinline__ void forward_row(const SolveArgs& A, const Lane& ln, const ModeCoef* cf,
                                            const double2* uh, const double2* uz, const double2* ud,
                                            int j, Cx<T>& cp, Cx<T>& dp) {
    const ModeCoef c = cf[j];
    const double sgn = DELTA ? -A.dt : A.dt;
    const double a = sgn * c.cm;
    const double cc = sgn * c.cp;
    double br = ln.p.zr;
    double bi = __builtin_fma(-A.dt, c.s, ln.p.zi);
    double dr, di;
    if constexpr (DELTA) {
        const double2 rh = uh[j];
        const double2 rd = ud[j];
        const double g2 = A.dt2H * c.gN;
        br = __builtin_fma(g2, ln.p.zir, br);
        bi = __builtin_fma(g2, ln.p.zii, bi);
        const double g1 = A.dt * c.gN;
        const double tr = __builtin_fma(ln.p.zir, rh.x, -(ln.p.zii * rh.y));
        const double ti = __builtin_fma(ln.p.zir, rh.y, ln.p.zii * rh.x);
        dr = __builtin_fma(g1, tr, rd.x);
        di = __builtin_fma(g1, ti, rd.y);
    } else {
        const double2 rz = uz[j];
        dr = rz.x;
        di = rz.y;
    }
    const T ta = static_cast<T>(a);
    const T wr = fmaT(-ta, cp.x, static_cast<T>(br));
    const T wi = fmaT(-ta, cp.y, static_cast<T>(bi));
    const T inv = rcp_refined(fmaT(wr, wr, wi * wi));
    const T pr = wr * inv, pi = -wi * inv;
    const T ur = fmaT(-ta, dp.x, static_cast<T>(dr));
    const T ui = fmaT(-ta, dp.y, static_cast<T>(di));
    const T tc = static_cast<T>(cc);
    cp.x = tc * pr;
    cp.y = tc * pi;
    dp.x = fmaT(ur, pr, -(ui * pi));
    dp.y = fmaT(ur, pi, ui * pr);
}

// Sums the 6 staged slots over the 64 lanes of the wave and writes them.
// red: [RED_SLOTS][64] double2.  Slot s < 4: chain row 4g + s; slots 4, 5: h of
// the two delta rows of the group.
template <int C>
__device__ __forceinline__ void reduce_group(const SolveArgs& A, double2* red, int lane, int pb,
                                             int base, int j0g, int Lm) {
    __syncthreads();
    const int slot = lane >> 3, part = lane & 7;
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const double2 v = red[slot * WAVE + i * 8 + part];
        sx += v.x;
        sy += v.y;
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
        if (j < Lm) A.out[(pb * 3 + field) * A.modes + base + j] = make_double2(sx, sy);
    }
    __syncthreads();
}

template <typename T, int S, int C>
__device__ __forceinline__ void solve_segment(const SolveArgs& A, const Lane& ln, const ModeCoef* cf,
                                              const double2* uh, const double2* uz, const double2* ud,
                                              int seg, int Lm, int base, int pb, int lane, Cx<T> cp,
                                              Cx<T> dp, Cx<T>& vnext, double2* red) {
    Cx<T> cs[S], ds[S];
    const int j0 = seg * S;
    static_for<0, S>([&](auto Q) {
        constexpr int jj = decltype(Q)::value;
        constexpr bool DELTA = ((jj + C) & 1) == 0;
        if (j0 + jj < Lm) {
            forward_row<T, DELTA>(A, ln, cf, uh, uz, ud, j0 + jj, cp, dp);
            cs[jj] = cp;
            ds[jj] = dp;
        }
    });
    static_for<0, S / 4>([&](auto G) {
        constexpr int g = S / 4 - 1 - decltype(G)::value;
        static_for<0, 4>([&](auto Qi) {
            constexpr int q = 3 - decltype(Qi)::value;
            constexpr int jj = 4 * g + q;
            constexpr bool DELTA = ((jj + C) & 1) == 0;
            const int j = j0 + jj;
            Cx<T> v{T(0), T(0)};
            if (j < Lm) {
                v.x = ds[jj].x - fmaT(cs[jj].x, vnext.x, -(cs[jj].y * vnext.y));
                v.y = ds[jj].y - fmaT(cs[jj].x, vnext.y, cs[jj].y * vnext.x);
                vnext = v;
            }
            const double vx = static_cast<double>(v.x), vy = static_cast<double>(v.y);
            red[q * WAVE + lane] = make_double2(__builtin_fma(ln.p.wr, vx, -(ln.p.wi * vy)),
                                                __builtin_fma(ln.p.wr, vy, ln.p.wi * vx));
            if constexpr (DELTA) {
                double hx = 0.0, hy = 0.0;
                if (j < Lm) {
                    const double2 rh = uh[j];
                    const double tx = __builtin_fma(-A.dtH, vx, rh.x);
                    const double ty = __builtin_fma(-A.dtH, vy, rh.y);
                    hx = __builtin_fma(ln.wzr, tx, -(ln.wzi * ty));
                    hy = __builtin_fma(ln.wzr, ty, ln.wzi * tx);
                }
                red[(4 + (q >> 1)) * WAVE + lane] = make_double2(hx, hy);
            }
        });
        reduce_group<C>(A, red, lane, pb, base, j0 + 4 * g, Lm);
    });
}

template <typename T, int S, int C>
__device__ __forceinline__ void solve_chain(const SolveArgs& A, int m, int pb, unsigned char* smem) {
    const int lane = threadIdx.x;
    const int n = pb * WAVE + lane;
    Lane ln;
    ln.p = A.poles[n < A.N ? n : 0];
    if (n >= A.N) ln.p.wr = ln.p.wi = 0.0;   // padding lanes add nothing
    ln.wzr = __builtin_fma(ln.p.wr, ln.p.zir, -(ln.p.wi * ln.p.zii));
    ln.wzi = __builtin_fma(ln.p.wr, ln.p.zii, ln.p.wi * ln.p.zir);

    const int Lm = A.L - m + 1;
    const int base = m * (2 * A.L + 3 - m) / 2;
    const ModeCoef* cf = A.coef + base;
    const double2* uh = A.U0 + base;
    const double2* uz = uh + A.modes;
    const double2* ud = uz + A.modes;
    const int nseg = (Lm + S - 1) / S;

    Cx<T>* ck = reinterpret_cast<Cx<T>*>(smem);             // [nseg - 2][2][64]
    const int nck = nseg > 2 ? nseg - 2 : 0;
    double2* red = reinterpret_cast<double2*>(smem + sizeof(Cx<T>) * 2 * WAVE * nck);

    Cx<T> cp{T(0), T(0)}, dp{T(0), T(0)};
    for (int seg = 0; seg < nseg - 1; ++seg) {
        if (seg > 0) {
            ck[(2 * (seg - 1)) * WAVE + lane] = cp;
            ck[(2 * (seg - 1) + 1) * WAVE + lane] = dp;
        }
        const int j0 = seg * S;
        static_for<0, S>([&](auto Q) {
            constexpr int jj = decltype(Q)::value;
            constexpr bool DELTA = ((jj + C) & 1) == 0;
            forward_row<T, DELTA>(A, ln, cf, uh, uz, ud, j0 + jj, cp, dp);
        });
    }
    Cx<T> vnext{T(0), T(0)};
    solve_segment<T, S, C>(A, ln, cf, uh, uz, ud, nseg - 1, Lm, base, pb, lane, cp, dp, vnext, red);
    for (int seg = nseg - 2; seg >= 0; --seg) {
        if (seg > 0) {
            cp = ck[(2 * (seg - 1)) * WAVE + lane];
            dp = ck[(2 * (seg - 1) + 1) * WAVE + lane];
        } else {
            cp = Cx<T>{T(0), T(0)};
            dp = Cx<T>{T(0), T(0)};
        }
        solve_segment<T, S, C>(A, ln, cf, uh, uz, ud, seg, Lm, base, pb, lane, cp, dp, vnext, red);
    }
}

template <typename T, int S>
__global__ __launch_bounds__(WAVE) void rexi_chain_kernel(SolveArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int task = blockIdx.x / A.npb;      // task = 2 m + chain: longest chains first
    const int pb = blockIdx.x - task * A.npb;
    const int m = task >> 1;
    if (task & 1)
        solve_chain<T, S, 1>(A, m, pb, smem);
    else
        solve_chain<T, S, 0>(A, m, pb, smem);
}

// U1[i] = sum over pole blocks of part[pb][i], in block order, compensated.
__global__ __launch_bounds__(256) void sum_partials_kernel(const double2* __restrict__ part,
                                                           double2* __restrict__ U1, int count, int npb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double sx = 0.0, sy = 0.0, cx = 0.0, cy = 0.0;
    for (int b = 0; b < npb; ++b) {
        const double2 v = part[static_cast<size_t>(b) * count + i];
        double t = sx + v.x;
        cx += (fabs(sx) >= fabs(v.x)) ? (sx - t) + v.x : (v.x - t) + sx;
        sx = t;
        t = sy + v.y;
        cy += (fabs(sy) >= fabs(v.y)) ? (sy - t) + v.y : (v.y - t) + sy;
        sy = t;
    }
    U1[i] = make_double2(sx + cx, sy + cy);
}

template <typename T, int S>
size_t lds_bytes(int L) {
    const int nseg = (L + 1 + S - 1) / S;
    const int nck = nseg > 2 ? nseg - 2 : 0;
    return sizeof(Cx<T>) * 2 * WAVE * nck + sizeof(double2) * RED_SLOTS * WAVE;
}

template <typename T, int S>
int launch_typed(swe_ctx* ctx, const SolveArgs& A, hipStream_t stream) {
    const size_t lds = lds_bytes<T, S>(A.L);
    if (lds > 64 * 1024) return fail(REXI_ENOTSUP, "rexi solve: segment checkpoints exceed LDS; raise seg_rows");
    const unsigned blocks = static_cast<unsigned>(2 * (A.L + 1) * A.npb);
    const int slot = prof_begin(ctx, REXI_KERNEL_SOLVE, stream);
    hipLaunchKernelGGL((rexi_chain_kernel<T, S>), dim3(blocks), dim3(WAVE), lds, stream, A);
    REXI_HIP(hipGetLastError());
    prof_end(ctx, REXI_KERNEL_SOLVE, slot, stream);
    return REXI_OK;
}

}  // namespace

int launch_rexi_solve(swe_ctx* ctx, int N, double dt, const double* U0, double* U1, hipStream_t stream) {
    SolveArgs A;
    A.U0 = reinterpret_cast<const double2*>(U0);
    A.poles = ctx->d_poles;
    A.coef = ctx->d_coef;
    A.L = ctx->L;
    A.modes = ctx->modes;
    A.N = N;
    A.npb = (N + WAVE - 1) / WAVE;
    A.dt = dt;
    A.dtH = dt * ctx->H;
    A.dt2H = dt * dt * ctx->H;
    const size_t count = static_cast<size_t>(3) * ctx->modes;
    if (A.npb == 1) {
        A.out = reinterpret_cast<double2*>(U1);
    } else {
        const size_t need = 2 * count * A.npb;
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
    const bool fp32 = (ctx->prec & REXI_PREC_FP32_SOLVE) != 0;
    int rc;
    switch (ctx->tune.seg_rows) {
        case 8: rc = fp32 ? launch_typed<float, 8>(ctx, A, stream) : launch_typed<double, 8>(ctx, A, stream); break;
        case 32: rc = fp32 ? launch_typed<float, 32>(ctx, A, stream) : launch_typed<double, 32>(ctx, A, stream); break;
        default: rc = fp32 ? launch_typed<float, 16>(ctx, A, stream) : launch_typed<double, 16>(ctx, A, stream); break;
    }
    if (rc != REXI_OK) return rc;
    if (A.npb > 1) {
        const int threads = 256;
        const unsigned blocks = static_cast<unsigned>((count + threads - 1) / threads);
        const int slot = prof_begin(ctx, REXI_KERNEL_REDUCE, stream);
        hipLaunchKernelGGL(sum_partials_kernel, dim3(blocks), dim3(threads), 0, stream,
                           reinterpret_cast<const double2*>(ctx->d_partial), reinterpret_cast<double2*>(U1),
                           static_cast<int>(count), A.npb);
        REXI_HIP(hipGetLastError());
        prof_end(ctx, REXI_KERNEL_REDUCE, slot, stream);
    }
    return REXI_OK;
}

}  // namespace rexi
