// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "rexi_swe.h"

namespace rexi {

// ---------------------------------------------------------------- errors --
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define REXI_HIP(call)                                   \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return ::rexi::hip_fail(e_, #call); \
    } while (0)

// ------------------------------------------------------- host numerics --
inline int n_modes(int L) { return (L + 1) * (L + 2) / 2; }
inline int mode_index(int L, int l, int m) { return m * (2 * L + 3 - m) / 2 + (l - m); }

// Per-mode coefficients of the chain form of (z I - dt L), m-major like the
// spectral state.  For degree k of order m:
//   cm = 2 Omega (k+1)/k eps_k      coupling to degree k-1 (0 if k-1 < max(m,1))
//   cp = 2 Omega k/(k+1) eps_{k+1}  coupling to degree k+1 (0 if k = L)
//   s  = 2 Omega m / (k(k+1))       (0 for k = 0)
//   gN = g k(k+1) / a^2
struct ModeCoef {
    double cm, cp, s, gN;
};

void build_mode_coef(int L, double a, double g, double Omega, ModeCoef* out);

// Poles of one coefficient set in the form the solve kernel uses:
// z = -alpha (contour point), zi = 1/z, w = -beta, so that
//   sum_n beta_n (dt L + alpha_n)^{-1} u = sum_n w_n (z_n - dt L)^{-1} u.
struct PoleData {
    double zr, zi, zir, zii, wr, wi;
};

// Fills pd[0..N) from interleaved alpha/beta (1/z in extended precision).
void build_pole_data(const double* alpha, const double* beta, int N, PoleData* pd);

// Winding number of the closed polygon z_0 .. z_{N-1} around the point (x, y).
int winding_number(const PoleData* pd, int N, double x, double y);

// Smallest distance between a pole z_n and the segment i[-rho, rho].
double min_distance_to_segment(const PoleData* pd, int N, double rho);

// rho = dt (sqrt(g H L(L+1))/a + 2 Omega): bound on the spectrum of dt L.
double spectral_radius(int L, double dt, double a, double g, double H, double Omega);
// max_w |S(i w) - e^{i w}| (approx) and max_w sum |beta|/|i w + alpha| (kappa)
// over npts points of [-rho, rho]; either output may be NULL.
void contour_error(const double* alpha, const double* beta, int N, double rho, int npts, double* approx,
                   double* kappa);
// See rexi_choose_contour in rexi_swe.h.
int choose_contour(double rho, double target, int prec, int N_fixed, const double* grid, int n_grid, int n_max,
                   double* p0, double* y, int* N, double* predicted);

// Largest off-diagonal row sum of the chain form per unit dt for each degree:
// out[k] = max over the orders m <= k of |cm| + |cp| (see ModeCoef), k = 0..L.
void coupling_row_max(int L, double Omega, std::vector<double>& out);

// The operator a coefficient set is checked against.
struct OperatorBounds {
    int L;
    double a, g, H, Omega;
    const double* off;   // [L+1] coupling_row_max
};

// Host checks of a coefficient set before any launch: finite values; the
// poles wind once around the segment i[-rho, rho] that holds the spectrum of
// dt L (rho = dt (sqrt(g H L(L+1))/a + 2 Omega)) and keep a distance from it;
// with `chain`, every row of every chain system is strictly diagonally
// dominant (the condition under which the unpivoted elimination is stable).
// For degree k the orders m <= k give diagonal shifts dt m q_k in
// [0, dt 2 Omega/(k+1)], so a zeta-row diagonal z - i dt m q_k is at least the
// distance of z from the segment i[0, dt 2 Omega/(k+1)], and a delta-row
// diagonal z + dt^2 H gN_k / z - i dt m q_k at least the distance of
// z + dt^2 H gN_k / z from it; the row's off-diagonals sum to at most
// dt off[k].  *margin (may be NULL) receives the smallest ratio over poles and
// degrees (> 1 when every row is dominant).  `who` names the entry point in
// the error text.
int check_poles(const OperatorBounds& op, const PoleData* pd, int N, double dt, bool chain, const char* who,
                double* margin);

// Extended-precision REXI coefficients (see rexi_coefficients in rexi_swe.h).
int coefficients(int fn, int N, double p0, double y, double* alpha, double* beta,
                 double* r, double* mu);

// Three-term recurrence of the normalised associated Legendre functions for
// degree l of order m:  Pbar_{l+1} = A mu Pbar_l - B Pbar_{l-1}  (A = 1/eps_{l+1},
// B = eps_l/eps_{l+1}), and H_l = (1 - mu^2) dPbar_l/dmu = hA Pbar_{l+1} + hB Pbar_{l-1}
// (hA = -l eps_{l+1}, hB = (l+1) eps_l).
struct LegCoef {
    double A, B, hA, hB;
};

struct ShtHost {
    int half = 0;                          // nlat / 2
    std::vector<double> mu, sint, w;       // northern nodes (mu descending), sin(theta), weights
    std::vector<LegCoef> rec;              // [modes]
    std::vector<double> a_over_n;          // [L+2]: a / (l(l+1)), 0 for l = 0
    std::vector<double> n_over_a2;         // [L+2]: l(l+1) / a^2
    std::vector<long double> mu_ld, sint_ld;  // the same nodes in 80-bit
};

// Degree segments: the degrees l = m..L of every order are cut into runs of
// seg_len; each run restarts the recurrence from (Pbar_{k0-1}, Pbar_{k0}) at
// its first degree k0, stored as mantissas times 2^e (e <= 0, shared by the pair).
struct SegHost {
    int seg_len = 0, nseg = 0;
    std::vector<int> seg_m, seg_i0, seg_n;  // order, first degree offset l - m, degree count
    std::vector<int> segbase;               // [L+2] first segment of order m
    std::vector<double> seed_pm, seed_p;    // [nseg][half]
    std::vector<int> seed_e;                // [nseg][half]
};

void build_legendre_tables(int L, int nlat, double a, ShtHost& out);
void build_segments(int L, int seg_len, const ShtHost& sh, SegHost& out);
void build_twiddles(int M, std::vector<double>& tw);

// ------------------------------------------------------------- context --
struct Profiler {
    static constexpr int kCap = 4096;
    unsigned mask = 0;     // bit k: record kernel k
    hipEvent_t* start[REXI_KERNEL_COUNT] = {};
    hipEvent_t* stop[REXI_KERNEL_COUNT] = {};
    int count[REXI_KERNEL_COUNT] = {};
};

// Records the start event of `kernel` (if profiling) and returns its slot or -1.
int prof_begin(swe_ctx* ctx, int kernel, hipStream_t stream);
void prof_end(swe_ctx* ctx, int kernel, int slot, hipStream_t stream);

// One cached coefficient set on the device.
struct PoleSet {
    PoleData* d = nullptr;
    int cap = 0, n = 0;
    uint64_t key = 0;              // hash of alpha, beta, N and dt
    bool valid = false;
    bool chain_ok = false;         // the chain systems' dominance was checked for this set
    unsigned long long used = 0;   // last use, for replacement
};

struct Tuning {
    int solver = REXI_SOLVER_FUSED;   // sweep schedule (REXI_SOLVER_*)
    int seg_rows = 16;                // rows per register-resident segment (8, 16, 32)
    int waves = 4;                    // waves per workgroup (1, 2, 4)
    int poles_per_lane = 1;           // poles swept together by one lane (1, 2)
};

}  // namespace rexi

struct swe_ctx {
    int L = 0, nlat = 0, nlon = 0, prec = 0, device = 0, modes = 0;
    double a = 0, g = 0, H = 0, Omega = 0;
    std::vector<double> coup_max;      // [L+1] rexi::coupling_row_max(L, Omega)
    // non-finite results written by the context's kernels since the last
    // swe_sync (bit flags rexi::STATUS_*), set with vector atomics
    unsigned* d_status = nullptr;
    rexi::Tuning tune;
    bool fuse = true;                  // swe_set_fusion
    rexi::Profiler prof;

    // REXI tables
    rexi::ModeCoef* d_coef = nullptr;  // [modes]

    // cached coefficient sets (a few, so that schemes alternating between
    // several sums on one contour, such as ETD2RK's psi_0, psi_1, psi_2, do not
    // re-upload); d_poles / poles_key name the active one
    static constexpr int kPoleSets = 4;
    rexi::PoleSet pole_sets[kPoleSets];
    unsigned long long pole_clock = 0;
    rexi::PoleData* d_poles = nullptr;
    uint64_t poles_key = 0;

    // chain-ordered row records of the REXI solve, rebuilt per call [2 modes]
    // (FP64 and FP32 forms)
    void* d_rows = nullptr;
    void* d_rows32 = nullptr;
    // cached factorization: pivots of every chain row for every pole,
    // [2 modes][N rounded to 64] complex (FP32 or FP64), valid for the cached
    // coefficient set and dt
    void* d_fact = nullptr;
    size_t fact_cap = 0;
    bool fact_valid = false;
    uint64_t fact_key = 0;      // coefficient set (and dt) the pivots belong to
    int fact_prec = 0;          // 1: FP32 pivots, 2: FP64 pivots
    // per-degree sums of the gravity-wave REXI stage [L+2][2] complex
    void* d_lgsum = nullptr;
    // device copy of the last ensemble launched with this context first
    void* batch = nullptr;
    // segment-start states of the chain sweeps (per launch)
    void* d_ckpt = nullptr;
    size_t ckpt_cap = 0;

    // partial sums over pole blocks: [npb][3][modes] complex
    double* d_partial = nullptr;
    size_t partial_cap = 0;   // in doubles

    // spherical-harmonic transforms (grid contexts only)
    rexi::LegCoef* d_rec = nullptr;   // [modes]
    double* d_aon = nullptr;          // [L+2]
    double* d_noa2 = nullptr;         // [L+2]
    double* d_mu = nullptr;           // [nlat/2]
    double* d_sint = nullptr;         // [nlat/2]
    double* d_w = nullptr;            // [nlat/2]
    int nseg = 0;                     // degree segments over all orders
    int* d_seg_m = nullptr;           // [nseg]
    int* d_seg_i0 = nullptr;          // [nseg]
    int* d_seg_n = nullptr;           // [nseg]
    int* d_segbase = nullptr;         // [L+2]
    double* d_seed_pm = nullptr;      // [nseg][nlat/2]
    double* d_seed_p = nullptr;       // [nseg][nlat/2]
    int* d_seed_e = nullptr;          // [nseg][nlat/2]
    double* d_part = nullptr;         // synthesis partial sums [nf][nseg][nlat] complex
    size_t part_cap = 0;              // fields the partial buffer can hold
    double* d_tw = nullptr;           // [nlon/2] complex, pass twiddles of the longitude FFT
    double* d_twr = nullptr;          // [nlon/2] complex
    int* d_radix = nullptr;
    int npass = 0;
    double* d_fout = nullptr;         // Fourier coefficients of the forward FFTs [nf][L+1][nlat] complex
    size_t four_cap = 0;              // fields each Fourier buffer can hold
    double* d_ustar = nullptr;        // Runge-Kutta stage [3][modes]
    double* d_n0 = nullptr;           // first tendency [3][modes]
    // split-precision Legendre table (REXI_PREC_BF16_SPLIT or _FP16_SPLIT):
    // Pbar for degrees m .. L+1 as 16-bit (hi, lo) pairs in a latitude-major (synthesis) and a
    // degree-major (analysis) layout; order m starts at tab_off[m], each
    // (m, parity) block has tab_kp[2m + parity] rows (padded to 16) by tab_hpad
    // latitudes
    unsigned short* d_tab_psyn = nullptr;
    unsigned short* d_tab_pana = nullptr;
    long long* d_tab_off = nullptr;   // [L+2]
    int* d_tab_kp = nullptr;          // [2 (L+1)]
    int tab_hpad = 0, tab_kmax = 0;
    size_t tab_len = 0;               // shorts per table
    double* d_tmpA = nullptr;         // Strang intermediates [3][modes]
    double* d_tmpB = nullptr;
    double* d_tmpC = nullptr;         // swe_strang_steps: the state between steps
};

namespace rexi {

// Flags of ctx->d_status: which kind of output turned non-finite.
enum : unsigned { STATUS_REXI = 1u, STATUS_NONLINEAR = 2u, STATUS_TRANSFORM = 4u };

// Sets `bit` in *status when v is not finite (a rare path: one vector atomic).
__device__ __forceinline__ void note_nonfinite(unsigned* status, double v, unsigned bit) {
    if (!__builtin_isfinite(v)) atomicOr(status, bit);
}

// Sum over pole waves of part[pw][i] (pole waves of count entries each), in
// pole-wave order, with Neumaier compensation: the REXI stage's pole sum.
__device__ __forceinline__ double2 sum_parts(const double2* __restrict__ part, int count, int nparts, int i) {
    double sx = 0.0, sy = 0.0, cx = 0.0, cy = 0.0;
    for (int b = 0; b < nparts; ++b) {
        const double2 v = part[static_cast<size_t>(b) * count + i];
        double t = sx + v.x;
        cx += (fabs(sx) >= fabs(v.x)) ? (sx - t) + v.x : (v.x - t) + sx;
        sx = t;
        t = sy + v.y;
        cy += (fabs(sy) >= fabs(v.y)) ? (sy - t) + v.y : (v.y - t) + sy;
        sy = t;
    }
    return make_double2(sx + cx, sy + cy);
}

// Launches the chain solve + reduction for one REXI stage on `stream`.
int launch_rexi_solve(swe_ctx* ctx, int N, double dt, const double* U0, double* U1,
                      hipStream_t stream);
// The chain solve alone: *nparts receives the number of pole-wave partial sums
// it left in ctx->d_partial ([nparts][3 modes]); with one pole wave the solve
// wrote U1 itself (*nparts = 1).
int launch_rexi_chain(swe_ctx* ctx, int N, double dt, const double* U0, double* U1, int* nparts,
                      hipStream_t stream);
// U1 = the pole sum of the nparts partials the chain solve left (nparts > 1).
int launch_rexi_sum(swe_ctx* ctx, int nparts, double* U1, hipStream_t stream);

// One member of an ensemble REXI stage (poles already prepared in ctx).
struct BatchMember {
    swe_ctx* ctx;
    int N;
    double dt;
    const double* U0;
    double* U1;
};
// Launches the REXI stages of `count` members (same precision; launch shape of
// the first member's context) as one rows, one solve and one sum launch.
int launch_rexi_batched(const BatchMember* mem, int count, hipStream_t stream);
void free_batch_plan(swe_ctx* ctx);

// Spherical-harmonic transform stages (sht.hip).  kind 0: nf scalar fields;
// kind 1: the non-linear set (synthesis: h, zeta, U, V from a state;
// analysis: the tendency from hU, hV, zU, zV, KE with the Runge-Kutta update
// out = U0 + c0 N + c1 Nprev and, if Nsave, a copy of N).
int sht_configure_kernels(swe_ctx* ctx);
int launch_legendre_synth(swe_ctx* ctx, int kind, const double* spec, double* part, int nf, hipStream_t stream);
int launch_legendre_anal(swe_ctx* ctx, int kind, const double* four, double* spec, int nf, const double* U0,
                         const double* Nprev, double* Nsave, double* out, double c0, double c1,
                         hipStream_t stream);
// Split-precision (bf16 hi/lo, matrix-core) Legendre stage: tables and the two
// directions.  The synthesis writes the Fourier coefficients of kind 0 (nf
// fields) order-major [nf][L+1][nlat] and those of kind 1 (the state)
// latitude-major [3][nlat][L+1] (the ring kernel reads a latitude's orders
// contiguously); one partial per order either way (segbase = nullptr).
int build_split_tables(swe_ctx* ctx, hipStream_t stream);
int launch_legendre_synth_split(swe_ctx* ctx, int kind, const double* spec, double* four, int nf,
                                hipStream_t stream);
int launch_legendre_anal_split(swe_ctx* ctx, int kind, const double* four, double* spec, int nf, const double* U0,
                               const double* Nprev, double* Nsave, double* out, double c0, double c1,
                               hipStream_t stream);
// The state's analysis (kind 1) fused with the synthesis of its output:
// Nsave = N (if non-null), out = U0 + c0 N + c1 Nprev (Nprev may be null;
// out written only if non-null), and the Fourier coefficients of out,
// latitude-major, into four_next (as the kind-1 synthesis writes them).
// Needs the table's degree rows per parity to fit the latitude rows
// (fused_anal_synth_supported).
int fused_anal_synth_supported(const swe_ctx* ctx);
// The REXI stage's pole sum over nparts partials ([nparts][3 modes] complex)
// into U1, fused with the split synthesis of U1 into four_next (latitude-major,
// as the kind-1 synthesis writes it).
int launch_rexi_sum_synth_split(swe_ctx* ctx, const double* part, int nparts, double* U1, double* four_next,
                                hipStream_t stream);
int launch_legendre_anal_synth_split(swe_ctx* ctx, const double* four, const double* U0, const double* Nprev,
                                     double* Nsave, double* out, double c0, double c1, double* four_next,
                                     hipStream_t stream);
// The REXI stage of the gravity-wave part L_g alone (Coriolis-free): per degree
// l a 2x2 system in (h, delta), zeta multiplied by S(0); the sums over poles are
// formed once per degree.
int launch_rexi_lg(swe_ctx* ctx, int N, double dt, const double* U0, double* U1, hipStream_t stream);
// The same two launches on caller-provided buffers: poles [N] and the per-degree
// sums [L+2][2] complex (lg_sums_bytes(L) bytes); no allocation, no profiling.
inline size_t lg_sums_bytes(int L) { return sizeof(double) * 4 * static_cast<size_t>(L + 2); }
int launch_rexi_lg_on(swe_ctx* ctx, const PoleData* poles, void* sums, int N, double dt, const double* U0,
                      double* U1, hipStream_t stream);
// check_poles with the context's operator.
int check_poles(const swe_ctx* ctx, const PoleData* pd, int N, double dt, bool chain, const char* who);
// Cache key of a coefficient set (alpha, beta: 2N doubles each) and dt.
uint64_t pole_key(const double* alpha, const double* beta, int N, double dt);
// Allocation-free entry point support: resolves the device address of the
// library's static scratch array on `device` (once per device; call with the
// device current).
int noalloc_init_device(int device);
// out = x + a y over n doubles (out may equal x or y); non-finite outputs set
// `bit` in *status.
int launch_axpy(double* out, const double* x, double a, const double* y, int n, unsigned* status, unsigned bit,
                hipStream_t stream);
// Radix sequence of the longitude FFT of M = nlon/2 complex points.
int ring_plan(int M, std::vector<int>& radix);
// Twiddles of every pass of that plan, pass-major ([M] complex).
int ring_twiddles(int M, const std::vector<int>& radix, std::vector<double>& tw);
// mode 0: Fourier -> grid (nf fields); 1: grid -> Fourier; 2: non-linear products.
// The partials are [nf][nseg][nlat] (segment-major), or with lat_major
// [nf][nlat][L+1] (one per order, nseg = L+1, segbase = nullptr).
int launch_ring(swe_ctx* ctx, int mode, const double* part, const int* segbase, int nseg, double* fout,
                const double* gin, double* gout, int nf, hipStream_t stream, double two_omega = 0.0,
                bool lat_major = false);

}  // namespace rexi
