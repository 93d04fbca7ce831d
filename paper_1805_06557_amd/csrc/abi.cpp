// The C-ABI entry points: argument checks, context set-up, coefficient
// caching and the contour check, then the kernel launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <set>
#include <string>
#include <vector>

#include "internal.h"

namespace rexi {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? REXI_ENOMEM : REXI_EDEVICE;
}

namespace {

uint64_t fnv1a(const void* data, size_t bytes, uint64_t h) {
    const unsigned char* p = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < bytes; ++i) {
        h ^= p[i];
        h *= 1099511628211ULL;
    }
    return h;
}

}  // namespace

uint64_t pole_key(const double* alpha, const double* beta, int N, double dt) {
    uint64_t key = 1469598103934665603ULL;
    key = fnv1a(alpha, sizeof(double) * 2 * static_cast<size_t>(N), key);
    key = fnv1a(beta, sizeof(double) * 2 * static_cast<size_t>(N), key);
    key = fnv1a(&N, sizeof(N), key);
    key = fnv1a(&dt, sizeof(dt), key);
    return key;
}

int check_poles(const swe_ctx* ctx, const PoleData* pd, int N, double dt, bool chain, const char* who) {
    const OperatorBounds op{ctx->L, ctx->a, ctx->g, ctx->H, ctx->Omega, ctx->coup_max.data()};
    return check_poles(op, pd, N, dt, chain, who, nullptr);
}

namespace {

// RAII guard that makes the context's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Uploads a coefficient set into the cache slot and makes it the active one.
int activate_poles(swe_ctx* ctx, PoleSet* slot, const PoleData* pd, int N, uint64_t key, hipStream_t stream) {
    // replace the least recently used set; the device may still read it, so wait
    if (slot->valid) REXI_HIP(hipStreamSynchronize(stream));
    slot->valid = false;
    if (N > slot->cap) {
        if (slot->d) REXI_HIP(hipFree(slot->d));
        slot->d = nullptr;
        slot->cap = 0;
        if (hipMalloc(&slot->d, sizeof(PoleData) * N) != hipSuccess)
            return fail(REXI_ENOMEM, "rexi_linear_step: cannot allocate pole table");
        slot->cap = N;
    }
    // The host vector dies at return: copy synchronously with respect to the host.
    REXI_HIP(hipMemcpyAsync(slot->d, pd, sizeof(PoleData) * N, hipMemcpyHostToDevice, stream));
    REXI_HIP(hipStreamSynchronize(stream));
    slot->key = key;
    slot->n = N;
    slot->valid = true;
    slot->used = ctx->pole_clock;
    ctx->d_poles = slot->d;
    ctx->poles_key = key;
    return REXI_OK;
}

// The cache slot for a new set: the least recently used one (or an empty one).
PoleSet* pole_slot(swe_ctx* ctx, uint64_t key, int N, bool& hit) {
    ++ctx->pole_clock;
    PoleSet* slot = nullptr;
    hit = false;
    for (PoleSet& ps : ctx->pole_sets) {
        if (ps.valid && ps.key == key && ps.n == N) {
            ps.used = ctx->pole_clock;
            ctx->d_poles = ps.d;
            ctx->poles_key = key;
            hit = true;
            return &ps;
        }
        if (!slot || !ps.valid || (slot->valid && ps.used < slot->used)) slot = &ps;
    }
    return slot;
}

// Uploads (alpha, beta) if they differ from the cached set and checks that the
// poles enclose the spectrum of dt L (and, when `chain`, that the chain
// systems of the banded solve are diagonally dominant).
int prepare_poles(swe_ctx* ctx, const double* alpha, const double* beta, int N, double dt, bool chain,
                  const char* who, hipStream_t stream) {
    const uint64_t key = pole_key(alpha, beta, N, dt);
    bool hit = false;
    PoleSet* slot = pole_slot(ctx, key, N, hit);
    if (hit && (!chain || slot->chain_ok)) return REXI_OK;

    std::vector<PoleData> pd(N);
    build_pole_data(alpha, beta, N, pd.data());
    int rc = check_poles(ctx, pd.data(), N, dt, chain, who);
    if (rc != REXI_OK) return rc;
    if (hit) {
        slot->chain_ok = true;
        return REXI_OK;
    }
    if ((rc = activate_poles(ctx, slot, pd.data(), N, key, stream)) != REXI_OK) return rc;
    slot->chain_ok = chain;
    return REXI_OK;
}

template <typename T>
int upload(T** dst, const T* src, size_t count) {
    REXI_HIP(hipMalloc(dst, sizeof(T) * (count ? count : 1)));
    if (count) REXI_HIP(hipMemcpy(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice));
    return REXI_OK;
}

// Grid set-up: Gauss nodes, Legendre recurrence tables and seeds, FFT plan and workspaces.
int setup_sht(swe_ctx* ctx) {
    ShtHost h;
    build_legendre_tables(ctx->L, ctx->nlat, ctx->a, h);
    int rc;
    if ((rc = upload(&ctx->d_rec, h.rec.data(), h.rec.size())) != REXI_OK) return rc;
    if ((rc = upload(&ctx->d_aon, h.a_over_n.data(), h.a_over_n.size())) != REXI_OK) return rc;
    if ((rc = upload(&ctx->d_noa2, h.n_over_a2.data(), h.n_over_a2.size())) != REXI_OK) return rc;
    if ((rc = upload(&ctx->d_mu, h.mu.data(), h.mu.size())) != REXI_OK) return rc;
    if ((rc = upload(&ctx->d_sint, h.sint.data(), h.sint.size())) != REXI_OK) return rc;
    if ((rc = upload(&ctx->d_w, h.w.data(), h.w.size())) != REXI_OK) return rc;
    SegHost sg;
    build_segments(ctx->L, 64, h, sg);
    ctx->nseg = sg.nseg;
    if ((rc = upload(&ctx->d_seg_m, sg.seg_m.data(), sg.seg_m.size())) != REXI_OK) return rc;
    if ((rc = upload(&ctx->d_seg_i0, sg.seg_i0.data(), sg.seg_i0.size())) != REXI_OK) return rc;
    if ((rc = upload(&ctx->d_seg_n, sg.seg_n.data(), sg.seg_n.size())) != REXI_OK) return rc;
    if ((rc = upload(&ctx->d_segbase, sg.segbase.data(), sg.segbase.size())) != REXI_OK) return rc;
    if ((rc = upload(&ctx->d_seed_pm, sg.seed_pm.data(), sg.seed_pm.size())) != REXI_OK) return rc;
    if ((rc = upload(&ctx->d_seed_p, sg.seed_p.data(), sg.seed_p.size())) != REXI_OK) return rc;
    if ((rc = upload(&ctx->d_seed_e, sg.seed_e.data(), sg.seed_e.size())) != REXI_OK) return rc;
    if (ctx->prec & (REXI_PREC_BF16_SPLIT | REXI_PREC_FP16_SPLIT)) {
        // row blocks per (m, parity of l - m) for degrees m .. L+1, padded to 16;
        // latitudes padded to 16
        const int half = ctx->nlat / 2;
        ctx->tab_hpad = (half + 15) / 16 * 16;
        std::vector<int> kp(2 * (ctx->L + 1));
        std::vector<long long> off(ctx->L + 2, 0);
        int kmax = 16;
        for (int m = 0; m <= ctx->L; ++m) {
            const int Lm = ctx->L - m + 2;
            kp[2 * m] = ((Lm + 1) / 2 + 15) / 16 * 16;
            kp[2 * m + 1] = (Lm / 2 + 15) / 16 * 16;
            kmax = std::max(kmax, std::max(kp[2 * m], kp[2 * m + 1]));
            off[m + 1] = off[m] + static_cast<long long>(kp[2 * m] + kp[2 * m + 1]) * ctx->tab_hpad * 2;
        }
        ctx->tab_kmax = kmax;
        ctx->tab_len = static_cast<size_t>(off[ctx->L + 1]);
        if ((rc = upload(&ctx->d_tab_kp, kp.data(), kp.size())) != REXI_OK) return rc;
        if ((rc = upload(&ctx->d_tab_off, off.data(), off.size())) != REXI_OK) return rc;
        for (unsigned short** t : {&ctx->d_tab_psyn, &ctx->d_tab_pana})
            if (hipMalloc(reinterpret_cast<void**>(t), sizeof(unsigned short) * ctx->tab_len) != hipSuccess)
                return fail(REXI_ENOMEM, "swe_create: cannot allocate the split-precision Legendre tables");
        if ((rc = build_split_tables(ctx, nullptr)) != REXI_OK) return rc;
        REXI_HIP(hipStreamSynchronize(nullptr));
    }
    // FFT of nlon reals = complex FFT of M = nlon/2 points, M = 2^a 3^b
    const int M = ctx->nlon / 2;
    std::vector<int> radix;
    if ((rc = ring_plan(M, radix)) != REXI_OK) return rc;
    ctx->npass = static_cast<int>(radix.size());
    if ((rc = upload(&ctx->d_radix, radix.data(), radix.size())) != REXI_OK) return rc;
    std::vector<double> tw, twr;
    if ((rc = ring_twiddles(M, radix, tw)) != REXI_OK) return rc;
    build_twiddles(ctx->nlon, twr);
    twr.resize(2 * static_cast<size_t>(M));
    if ((rc = upload(&ctx->d_tw, tw.data(), tw.size())) != REXI_OK) return rc;
    if ((rc = upload(&ctx->d_twr, twr.data(), twr.size())) != REXI_OK) return rc;
    const size_t st = static_cast<size_t>(6) * ctx->modes;
    REXI_HIP(hipMalloc(&ctx->d_ustar, sizeof(double) * st));
    REXI_HIP(hipMalloc(&ctx->d_n0, sizeof(double) * st));
    REXI_HIP(hipMalloc(&ctx->d_tmpA, sizeof(double) * st));
    REXI_HIP(hipMalloc(&ctx->d_tmpB, sizeof(double) * st));
    REXI_HIP(hipMalloc(&ctx->d_tmpC, sizeof(double) * st));
    return sht_configure_kernels(ctx);
}

// Makes the synthesis-partial buffer ([nf][nseg][nlat]) and the Fourier
// buffer of the forward transforms ([nf][L+1][nlat]) hold at least nf fields.
int reserve_fourier(swe_ctx* ctx, int nf) {
    if (static_cast<size_t>(nf) <= ctx->four_cap) return REXI_OK;
    if (ctx->d_part) REXI_HIP(hipFree(ctx->d_part));
    if (ctx->d_fout) REXI_HIP(hipFree(ctx->d_fout));
    ctx->d_part = ctx->d_fout = nullptr;
    ctx->four_cap = 0;
    const size_t pbytes = sizeof(double) * 2 * static_cast<size_t>(nf) * ctx->nseg * ctx->nlat;
    const size_t fbytes = sizeof(double) * 2 * static_cast<size_t>(nf) * (ctx->L + 1) * ctx->nlat;
    if (hipMalloc(&ctx->d_part, pbytes) != hipSuccess || hipMalloc(&ctx->d_fout, fbytes) != hipSuccess)
        return fail(REXI_ENOMEM, "cannot allocate Fourier workspace");
    ctx->four_cap = static_cast<size_t>(nf);
    return REXI_OK;
}

// One Heun step dU/dt = N(U) over tau on `stream`.
bool split_legendre(const swe_ctx* ctx) { return (ctx->prec & (REXI_PREC_BF16_SPLIT | REXI_PREC_FP16_SPLIT)) != 0; }

// Spectral fields -> synthesis partials of the Fourier coefficients in
// ctx->d_part (per degree segment; one segment per order in the split path).
int to_fourier(swe_ctx* ctx, int kind, const double* spec, int nf, hipStream_t stream) {
    if (split_legendre(ctx)) return launch_legendre_synth_split(ctx, kind, spec, ctx->d_part, nf, stream);
    return launch_legendre_synth(ctx, kind, spec, ctx->d_part, nf, stream);
}

// Ring stage on the partials to_fourier left in ctx->d_part (mode 0: to the
// grid `gout`; mode 2: non-linear products into ctx->d_fout).
int ring_from_part(swe_ctx* ctx, int mode, double* gout, int nf, hipStream_t stream, double two_omega = 0.0) {
    const bool split = split_legendre(ctx);
    // the split synthesis of the state (kind 1, which mode 2 follows) is latitude-major
    return launch_ring(ctx, mode, ctx->d_part, split ? nullptr : ctx->d_segbase, split ? ctx->L + 1 : ctx->nseg,
                       ctx->d_fout, nullptr, gout, nf, stream, two_omega, split && mode == 2);
}

// Fourier coefficients (ctx->d_fout) -> spectral fields or the Runge-Kutta update.
int from_fourier(swe_ctx* ctx, int kind, double* spec, int nf, const double* U0, const double* Nprev, double* Nsave,
                 double* out, double c0, double c1, hipStream_t stream) {
    if (split_legendre(ctx))
        return launch_legendre_anal_split(ctx, kind, ctx->d_fout, spec, nf, U0, Nprev, Nsave, out, c0, c1, stream);
    return launch_legendre_anal(ctx, kind, ctx->d_fout, spec, nf, U0, Nprev, Nsave, out, c0, c1, stream);
}

// Nout = N(U): one evaluation of the non-linear tendency (with two_omega = 2 Omega:
// N + L_c, the Coriolis term formed on the grid through the absolute vorticity).
int tendency_eval(swe_ctx* ctx, const double* U, double* Nout, hipStream_t stream, double two_omega = 0.0) {
    int rc;
    if ((rc = reserve_fourier(ctx, 5)) != REXI_OK) return rc;
    if ((rc = to_fourier(ctx, 1, U, 3, stream)) != REXI_OK) return rc;
    if ((rc = ring_from_part(ctx, 2, nullptr, 0, stream, two_omega)) != REXI_OK) return rc;
    return from_fourier(ctx, 1, nullptr, 0, nullptr, nullptr, nullptr, Nout, 1.0, 0.0, stream);
}

// Crank-Nicolson over tau: (I - tau/2 L)^-1 (I + tau/2 L) U0 = -U0 + 4 (2 - tau L)^-1 U0,
// one real shift z = 2 with weight 4 on the chain solve.  U0 and U1 must differ.
int cn_linear(swe_ctx* ctx, double tau, const double* U0, double* U1, hipStream_t stream) {
    // the shift z = 2 lies 2 away from the spectrum segment: every chain diagonal
    // is at least 2 in modulus (see check_poles), the off-diagonals of a row sum
    // to at most tau coup_max[k]
    const double off = tau * *std::max_element(ctx->coup_max.begin(), ctx->coup_max.end());
    if (!(2.0 > off)) {
        char buf[200];
        std::snprintf(buf, sizeof buf,
                      "swe_cn_step: dt = %.6g is too long for the unpivoted chain elimination (off-diagonal "
                      "sum %.4g >= diagonal bound 2)", tau, off);
        return fail(REXI_ENUMERIC, buf);
    }
    uint64_t key = 0x43726e6b4e69636fULL;            // a tag no coefficient hash is expected to hit
    key = fnv1a(&tau, sizeof(tau), key);
    bool hit = false;
    PoleSet* slot = pole_slot(ctx, key, 1, hit);
    int rc;
    if (!hit) {
        PoleData pd{};
        pd.zr = 2.0;
        pd.zi = 0.0;
        pd.zir = 0.5;
        pd.zii = 0.0;
        pd.wr = 4.0;
        pd.wi = 0.0;
        if ((rc = activate_poles(ctx, slot, &pd, 1, key, stream)) != REXI_OK) return rc;
    }
    if ((rc = launch_rexi_solve(ctx, 1, tau, U0, U1, stream)) != REXI_OK) return rc;
    return launch_axpy(U1, U1, -1.0, U0, 6 * ctx->modes, ctx->d_status, STATUS_REXI, stream);
}

// synth_done: the synthesis of U0 is already in ctx->d_part (the pole sum of
// a REXI stage, or the previous step's last analysis, fused with it).
// synth_next (may be null): on input, ask for the synthesis of U1 to be left
// in ctx->d_part (the last analysis fused with it); on return, whether it was.
int heun_step(swe_ctx* ctx, double tau, const double* U0, double* U1, hipStream_t stream, double two_omega = 0.0,
              bool synth_done = false, bool* synth_next = nullptr) {
    int rc;
    if ((rc = reserve_fourier(ctx, 5)) != REXI_OK) return rc;
    // stage 1: U* = U0 + tau N(U0), keep N(U0)
    if (!synth_done && (rc = to_fourier(ctx, 1, U0, 3, stream)) != REXI_OK) return rc;
    if ((rc = ring_from_part(ctx, 2, nullptr, 0, stream, two_omega)) != REXI_OK) return rc;
    if (ctx->fuse && split_legendre(ctx) && fused_anal_synth_supported(ctx)) {
        // the analysis of each order synthesises its U* directly (one launch;
        // U* is not stored)
        if ((rc = launch_legendre_anal_synth_split(ctx, ctx->d_fout, U0, nullptr, ctx->d_n0, nullptr, tau, 0.0,
                                                   ctx->d_part, stream)) != REXI_OK)
            return rc;
    } else {
        if ((rc = from_fourier(ctx, 1, nullptr, 0, U0, nullptr, ctx->d_n0, ctx->d_ustar, tau, 0.0, stream)) !=
            REXI_OK)
            return rc;
        if ((rc = to_fourier(ctx, 1, ctx->d_ustar, 3, stream)) != REXI_OK) return rc;
    }
    // stage 2: U1 = U0 + tau/2 (N(U0) + N(U*))
    if ((rc = ring_from_part(ctx, 2, nullptr, 0, stream, two_omega)) != REXI_OK) return rc;
    if (synth_next && *synth_next && ctx->fuse && split_legendre(ctx) && fused_anal_synth_supported(ctx)) {
        // U1 is stored and also synthesised for the caller's next Heun step
        return launch_legendre_anal_synth_split(ctx, ctx->d_fout, U0, ctx->d_n0, nullptr, U1, 0.5 * tau, 0.5 * tau,
                                                ctx->d_part, stream);
    }
    if (synth_next) *synth_next = false;
    return from_fourier(ctx, 1, nullptr, 0, U0, ctx->d_n0, nullptr, U1, 0.5 * tau, 0.5 * tau, stream);
}

}  // namespace

int prof_begin(swe_ctx* ctx, int kernel, hipStream_t stream) {
    Profiler& p = ctx->prof;
    if (!(p.mask & (1u << kernel)) || p.count[kernel] >= Profiler::kCap) return -1;
    const int slot = p.count[kernel];
    if (!p.start[kernel]) {
        p.start[kernel] = new (std::nothrow) hipEvent_t[Profiler::kCap]();
        p.stop[kernel] = new (std::nothrow) hipEvent_t[Profiler::kCap]();
        if (!p.start[kernel] || !p.stop[kernel]) return -1;
    }
    if (!p.start[kernel][slot] && hipEventCreate(&p.start[kernel][slot]) != hipSuccess) return -1;
    if (!p.stop[kernel][slot] && hipEventCreate(&p.stop[kernel][slot]) != hipSuccess) return -1;
    if (hipEventRecord(p.start[kernel][slot], stream) != hipSuccess) return -1;
    return slot;
}

void prof_end(swe_ctx* ctx, int kernel, int slot, hipStream_t stream) {
    if (slot < 0) return;
    if (hipEventRecord(ctx->prof.stop[kernel][slot], stream) == hipSuccess) ctx->prof.count[kernel] = slot + 1;
}

bool valid_constants(double a, double g, double H, double Omega) {
    return a > 0 && g > 0 && H > 0 && Omega >= 0 && std::isfinite(a) && std::isfinite(g) && std::isfinite(H) &&
           std::isfinite(Omega);
}

}  // namespace rexi

using namespace rexi;

extern "C" {

const char* rexi_last_error(void) { return rexi::g_last_error.c_str(); }

int rexi_coefficients(int fn, int N, double p0, double y, double* alpha, double* beta, double* r,
                      double* mu) {
    return rexi::coefficients(fn, N, p0, y, alpha, beta, r, mu);
}

int rexi_check_contour(int L, double a, double g, double H, double Omega, double dt, const double* alpha,
                       const double* beta, int N, double* margin) {
    if (L < 1 || L > 1023) return fail(REXI_EINVAL, "rexi_check_contour: L must be in [1, 1023]");
    if (!valid_constants(a, g, H, Omega))
        return fail(REXI_EINVAL, "rexi_check_contour: a, g, H must be positive and Omega non-negative");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(REXI_EINVAL, "rexi_check_contour: dt must be positive");
    if (!alpha || !beta) return fail(REXI_EINVAL, "rexi_check_contour: NULL alpha or beta");
    if (N < 2 || (N & 1) || N > (1 << 20)) return fail(REXI_EINVAL, "rexi_check_contour: N must be even and in [2, 2^20]");
    std::vector<PoleData> pd(N);
    build_pole_data(alpha, beta, N, pd.data());
    std::vector<double> off;
    coupling_row_max(L, Omega, off);
    const OperatorBounds op{L, a, g, H, Omega, off.data()};
    return check_poles(op, pd.data(), N, dt, true, "rexi_check_contour", margin);
}

int rexi_spectral_radius(int L, double dt, double a, double g, double H, double Omega, double* rho) {
    if (!rho || L < 0 || !(dt > 0) || !std::isfinite(dt) || !valid_constants(a, g, H, Omega))
        return fail(REXI_EINVAL, "rexi_spectral_radius: bad argument");
    *rho = spectral_radius(L, dt, a, g, H, Omega);
    return REXI_OK;
}

int rexi_contour_error(const double* alpha, const double* beta, int N, double rho, int npts, double* approx,
                       double* kappa) {
    if (!alpha || !beta || !approx || !kappa) return fail(REXI_EINVAL, "rexi_contour_error: NULL argument");
    if (N < 1 || N > (1 << 20) || npts < 2 || npts > (1 << 20) || !(rho >= 0) || !std::isfinite(rho))
        return fail(REXI_EINVAL, "rexi_contour_error: bad N, npts or rho");
    contour_error(alpha, beta, N, rho, npts, approx, kappa);
    return REXI_OK;
}

int rexi_choose_contour(double rho, double target, int prec, int N_fixed, const double* p0_grid, int n_p0,
                        int n_max, double* p0, double* y, int* N, double* predicted) {
    if (!p0 || !y || !N || !predicted) return fail(REXI_EINVAL, "rexi_choose_contour: NULL output");
    if (!(rho > 0) || !std::isfinite(rho)) return fail(REXI_EINVAL, "rexi_choose_contour: rho must be positive");
    if (prec & ~(REXI_PREC_FP32_SOLVE | REXI_PREC_BF16_SPLIT | REXI_PREC_FP16_SPLIT))
        return fail(REXI_EINVAL, "rexi_choose_contour: unknown precision flags");
    if (p0_grid && (n_p0 < 1 || n_p0 > 1024)) return fail(REXI_EINVAL, "rexi_choose_contour: bad grid size");
    for (int i = 0; p0_grid && i < n_p0; ++i)
        if (!(p0_grid[i] > 0) || !std::isfinite(p0_grid[i]))
            return fail(REXI_EINVAL, "rexi_choose_contour: grid shifts must be positive");
    if (N_fixed < 0 || (N_fixed & 1) || N_fixed > (1 << 16))
        return fail(REXI_EINVAL, "rexi_choose_contour: N_fixed must be 0 or even and at most 65536");
    if (N_fixed == 0) {
        if (!(target > 0) || !std::isfinite(target)) return fail(REXI_EINVAL, "rexi_choose_contour: target must be positive");
        if (n_max < 2 || n_max > (1 << 16)) return fail(REXI_EINVAL, "rexi_choose_contour: n_max must be in [2, 65536]");
    }
    return choose_contour(rho, target, prec, N_fixed, p0_grid, n_p0, n_max, p0, y, N, predicted);
}

int swe_create(int L, int nlat, int nlon, double a, double g, double H, double Omega, int prec,
               swe_ctx** out) {
    if (!out) return fail(REXI_EINVAL, "swe_create: NULL output pointer");
    *out = nullptr;
    if (L < 1 || L > 1023) return fail(REXI_EINVAL, "swe_create: L must be in [1, 1023]");
    if (!valid_constants(a, g, H, Omega))
        return fail(REXI_EINVAL, "swe_create: a, g, H must be positive and Omega non-negative");
    const bool linear_only = nlat == 0 && nlon == 0;
    if (!linear_only) {
        if (nlat <= L || (nlat & 1)) return fail(REXI_EINVAL, "swe_create: nlat must be even and exceed L");
        if (nlon <= 2 * L || (nlon % 4)) return fail(REXI_EINVAL, "swe_create: nlon must exceed 2L and be a multiple of 4");
    }
    if (prec & ~(REXI_PREC_FP32_SOLVE | REXI_PREC_BF16_SPLIT | REXI_PREC_FP16_SPLIT))
        return fail(REXI_EINVAL, "swe_create: unknown precision flags");
    if ((prec & REXI_PREC_BF16_SPLIT) && (prec & REXI_PREC_FP16_SPLIT))
        return fail(REXI_EINVAL, "swe_create: BF16 and FP16 Legendre modes are exclusive");

    swe_ctx* ctx = new (std::nothrow) swe_ctx;
    if (!ctx) return fail(REXI_ENOMEM, "swe_create: out of host memory");
    ctx->L = L;
    ctx->nlat = nlat;
    ctx->nlon = nlon;
    ctx->prec = prec;
    // measured defaults (the autotuner refines them per problem): two poles per
    // lane, 8-row segments, 4 waves per workgroup in both precisions.  At T511
    // (512-row chains, N = 2000) the FP64 solve takes 1.98 ms with these against
    // 3.24 ms with one pole per lane, 16 rows and 2 waves: a long chain's records
    // leave LDS room for few workgroups per CU, so waves per workgroup count.
    ctx->tune.solver = REXI_SOLVER_FUSED;
    ctx->tune.poles_per_lane = 2;
    ctx->tune.seg_rows = 8;
    ctx->tune.waves = 4;
    ctx->a = a;
    ctx->g = g;
    ctx->H = H;
    ctx->Omega = Omega;
    ctx->modes = n_modes(L);
    coupling_row_max(L, Omega, ctx->coup_max);
    hipError_t e = hipGetDevice(&ctx->device);
    if (e != hipSuccess) {
        delete ctx;
        return hip_fail(e, "swe_create: hipGetDevice");
    }
    // the allocation-free entry point's scratch address on this device (a failure
    // here only disables that entry point, which retries and reports it)
    (void)noalloc_init_device(ctx->device);
    std::vector<ModeCoef> coef(ctx->modes);
    build_mode_coef(L, a, g, Omega, coef.data());
    e = hipMalloc(&ctx->d_coef, sizeof(ModeCoef) * ctx->modes);
    if (e == hipSuccess)
        e = hipMemcpy(ctx->d_coef, coef.data(), sizeof(ModeCoef) * ctx->modes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&ctx->d_status, sizeof(unsigned));
    if (e == hipSuccess) e = hipMemset(ctx->d_status, 0, sizeof(unsigned));
    if (e != hipSuccess) {
        swe_destroy(ctx);
        return hip_fail(e, "swe_create: uploading operator tables");
    }
    if (!linear_only) {
        const int rc = setup_sht(ctx);
        if (rc != REXI_OK) {
            const std::string msg = rexi_last_error();
            swe_destroy(ctx);
            return fail(rc, msg);
        }
    }
    *out = ctx;
    return REXI_OK;
}

int swe_destroy(swe_ctx* ctx) {
    if (!ctx) return REXI_OK;
    DeviceGuard guard(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->d_coef) (void)hipFree(ctx->d_coef);
    if (ctx->d_status) (void)hipFree(ctx->d_status);
    for (PoleSet& ps : ctx->pole_sets)
        if (ps.d) (void)hipFree(ps.d);
    if (ctx->d_partial) (void)hipFree(ctx->d_partial);
    if (ctx->d_rows) (void)hipFree(ctx->d_rows);
    if (ctx->d_rows32) (void)hipFree(ctx->d_rows32);
    if (ctx->d_fact) (void)hipFree(ctx->d_fact);
    if (ctx->d_ckpt) (void)hipFree(ctx->d_ckpt);
    if (ctx->d_lgsum) (void)hipFree(ctx->d_lgsum);
    free_batch_plan(ctx);
    void* sht_bufs[] = {ctx->d_rec, ctx->d_aon, ctx->d_noa2, ctx->d_mu, ctx->d_sint, ctx->d_w,
                        ctx->d_seg_m, ctx->d_seg_i0, ctx->d_seg_n, ctx->d_segbase, ctx->d_seed_pm,
                        ctx->d_seed_p, ctx->d_seed_e, ctx->d_tw, ctx->d_twr, ctx->d_radix, ctx->d_part,
                        ctx->d_fout, ctx->d_ustar, ctx->d_n0, ctx->d_tmpA, ctx->d_tmpB, ctx->d_tmpC, ctx->d_tab_psyn,
                        ctx->d_tab_pana, ctx->d_tab_off, ctx->d_tab_kp};
    for (void* p : sht_bufs)
        if (p) (void)hipFree(p);
    for (int k = 0; k < REXI_KERNEL_COUNT; ++k) {
        for (int i = 0; ctx->prof.start[k] && i < Profiler::kCap; ++i) {
            if (ctx->prof.start[k][i]) (void)hipEventDestroy(ctx->prof.start[k][i]);
            if (ctx->prof.stop[k][i]) (void)hipEventDestroy(ctx->prof.stop[k][i]);
        }
        delete[] ctx->prof.start[k];
        delete[] ctx->prof.stop[k];
    }
    delete ctx;
    return REXI_OK;
}

int swe_set_tuning(swe_ctx* ctx, int solver, int seg_rows, int waves, int poles_per_lane) {
    if (!ctx) return fail(REXI_EINVAL, "swe_set_tuning: NULL context");
    if (solver && solver != REXI_SOLVER_FUSED && solver != REXI_SOLVER_STREAM && solver != REXI_SOLVER_HYBRID)
        return fail(REXI_EINVAL, "swe_set_tuning: unknown solver schedule");
    if (seg_rows && seg_rows != 8 && seg_rows != 16 && seg_rows != 32)
        return fail(REXI_EINVAL, "swe_set_tuning: seg_rows must be 8, 16 or 32");
    if (waves && waves != 1 && waves != 2 && waves != 4)
        return fail(REXI_EINVAL, "swe_set_tuning: waves must be 1, 2 or 4");
    if (poles_per_lane && poles_per_lane != 1 && poles_per_lane != 2)
        return fail(REXI_EINVAL, "swe_set_tuning: poles_per_lane must be 1 or 2");
    if (solver) ctx->tune.solver = solver;
    if (poles_per_lane) ctx->tune.poles_per_lane = poles_per_lane;
    if (seg_rows) ctx->tune.seg_rows = seg_rows;
    if (waves) ctx->tune.waves = waves;
    return REXI_OK;
}

int swe_set_fusion(swe_ctx* ctx, int enable) {
    if (!ctx) return fail(REXI_EINVAL, "swe_set_fusion: NULL context");
    if (enable != 0 && enable != 1) return fail(REXI_EINVAL, "swe_set_fusion: enable must be 0 or 1");
    ctx->fuse = enable != 0;
    return REXI_OK;
}

int swe_get_fusion(swe_ctx* ctx, int* enable) {
    if (!ctx || !enable) return fail(REXI_EINVAL, "swe_get_fusion: NULL argument");
    *enable = ctx->fuse ? 1 : 0;
    return REXI_OK;
}

int rexi_linear_step(swe_ctx* ctx, const double* alpha, const double* beta, int N, double dt,
                     const double* U0, double* U1, hipStream_t stream) {
    if (!ctx) return fail(REXI_EINVAL, "rexi_linear_step: NULL context");
    if (!alpha || !beta || !U0 || !U1) return fail(REXI_EINVAL, "rexi_linear_step: NULL pointer");
    if (N < 2 || (N & 1) || N > (1 << 20)) return fail(REXI_EINVAL, "rexi_linear_step: N must be even and in [2, 2^20]");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(REXI_EINVAL, "rexi_linear_step: dt must be positive");
    const size_t bytes = sizeof(double) * 6 * ctx->modes;
    const char* a0 = reinterpret_cast<const char*>(U0);
    const char* a1 = reinterpret_cast<const char*>(U1);
    if (a0 < a1 + bytes && a1 < a0 + bytes) return fail(REXI_EINVAL, "rexi_linear_step: U0 and U1 overlap");
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(REXI_EDEVICE, "rexi_linear_step: cannot select the context's device");
    int rc = prepare_poles(ctx, alpha, beta, N, dt, true, "rexi_linear_step", stream);
    if (rc != REXI_OK) return rc;
    return launch_rexi_solve(ctx, N, dt, U0, U1, stream);
}

int rexi_lg_step(swe_ctx* ctx, const double* alpha, const double* beta, int N, double dt, const double* U0,
                 double* U1, hipStream_t stream) {
    if (!ctx) return fail(REXI_EINVAL, "rexi_lg_step: NULL context");
    if (!alpha || !beta || !U0 || !U1) return fail(REXI_EINVAL, "rexi_lg_step: NULL pointer");
    if (N < 2 || (N & 1) || N > (1 << 20)) return fail(REXI_EINVAL, "rexi_lg_step: N must be even and in [2, 2^20]");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(REXI_EINVAL, "rexi_lg_step: dt must be positive");
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(REXI_EDEVICE, "rexi_lg_step: cannot select the context's device");
    int rc = prepare_poles(ctx, alpha, beta, N, dt, false, "rexi_lg_step", stream);
    if (rc != REXI_OK) return rc;
    return launch_rexi_lg(ctx, N, dt, U0, U1, stream);
}

int rexi_linear_step_batched(const rexi_member* members, int count, hipStream_t stream) {
    if (!members || count < 1 || count > 4096)
        return fail(REXI_EINVAL, "rexi_linear_step_batched: need 1 to 4096 members");
    std::set<const swe_ctx*> seen;
    std::vector<BatchMember> mem(count);
    for (int i = 0; i < count; ++i) {
        const rexi_member& m = members[i];
        if (!m.ctx || !m.alpha || !m.beta || !m.U0 || !m.U1)
            return fail(REXI_EINVAL, "rexi_linear_step_batched: NULL context or pointer in a member");
        if (!seen.insert(m.ctx).second)
            return fail(REXI_EINVAL, "rexi_linear_step_batched: every member needs its own context");
        if (m.ctx->device != members[0].ctx->device ||
            ((m.ctx->prec ^ members[0].ctx->prec) & REXI_PREC_FP32_SOLVE))
            return fail(REXI_EINVAL, "rexi_linear_step_batched: members differ in device or solve precision");
        if (m.N < 2 || (m.N & 1) || m.N > (1 << 20))
            return fail(REXI_EINVAL, "rexi_linear_step_batched: N must be even and in [2, 2^20]");
        if (!(m.dt > 0) || !std::isfinite(m.dt)) return fail(REXI_EINVAL, "rexi_linear_step_batched: dt must be positive");
        const size_t bytes = sizeof(double) * 6 * m.ctx->modes;
        const char* a0 = reinterpret_cast<const char*>(m.U0);
        const char* a1 = reinterpret_cast<const char*>(m.U1);
        if (a0 < a1 + bytes && a1 < a0 + bytes) return fail(REXI_EINVAL, "rexi_linear_step_batched: U0 and U1 overlap");
        mem[i] = BatchMember{m.ctx, m.N, m.dt, m.U0, m.U1};
    }
    DeviceGuard guard(members[0].ctx->device);
    if (!guard.ok) return fail(REXI_EDEVICE, "rexi_linear_step_batched: cannot select the device");
    for (int i = 0; i < count; ++i) {
        const int rc = prepare_poles(members[i].ctx, members[i].alpha, members[i].beta, members[i].N,
                                     members[i].dt, true, "rexi_linear_step_batched", stream);
        if (rc != REXI_OK) return rc;
    }
    return launch_rexi_batched(mem.data(), count, stream);
}

int swe_get_tuning(swe_ctx* ctx, int* solver, int* seg_rows, int* waves, int* poles_per_lane) {
    if (!ctx || !solver || !seg_rows || !waves || !poles_per_lane)
        return fail(REXI_EINVAL, "swe_get_tuning: NULL argument");
    *solver = ctx->tune.solver;
    *seg_rows = ctx->tune.seg_rows;
    *waves = ctx->tune.waves;
    *poles_per_lane = ctx->tune.poles_per_lane;
    return REXI_OK;
}

int swe_autotune(swe_ctx* ctx, const double* alpha, const double* beta, int N, double dt, const double* U0,
                 double* U1, int reps, hipStream_t stream, double* best_ms) {
    if (!ctx) return fail(REXI_EINVAL, "swe_autotune: NULL context");
    if (reps < 1 || reps > 1000) return fail(REXI_EINVAL, "swe_autotune: reps must be in [1, 1000]");
    int rc = rexi_linear_step(ctx, alpha, beta, N, dt, U0, U1, stream);   // validates, prepares the poles
    if (rc != REXI_OK) return rc;
    DeviceGuard guard(ctx->device);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(REXI_EDEVICE, "swe_autotune: cannot create events");
    }
    const Tuning saved = ctx->tune;
    Tuning best = saved;
    double best_t = std::numeric_limits<double>::infinity();
    const int shapes[4][2] = {{1, 16}, {1, 32}, {2, 8}, {2, 16}};   // (poles per lane, segment rows)
    rc = REXI_OK;
    for (int solver = REXI_SOLVER_FUSED; solver <= REXI_SOLVER_HYBRID && rc == REXI_OK; ++solver) {
        for (const auto& sh : shapes) {
            for (int waves : {1, 2, 4}) {
                ctx->tune = Tuning{solver, sh[1], waves, sh[0]};
                int r = launch_rexi_solve(ctx, N, dt, U0, U1, stream);    // warm: builds a factorization
                if (r == REXI_ENOTSUP) continue;                          // shape does not fit this problem
                if (r != REXI_OK) { rc = r; break; }
                if (hipEventRecord(e0, stream) != hipSuccess) { rc = fail(REXI_EDEVICE, "swe_autotune: event"); break; }
                for (int i = 0; i < reps && r == REXI_OK; ++i) r = launch_rexi_solve(ctx, N, dt, U0, U1, stream);
                if (r != REXI_OK) { rc = r; break; }
                float ms = 0.0f;
                if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    rc = fail(REXI_EDEVICE, "swe_autotune: timing failed");
                    break;
                }
                if (ms < best_t) {
                    best_t = ms;
                    best = ctx->tune;
                }
            }
            if (rc != REXI_OK) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != REXI_OK) {
        ctx->tune = saved;
        return rc;
    }
    ctx->tune = best;
    if (best.solver == REXI_SOLVER_FUSED && ctx->d_fact) {
        // the winning schedule does not read the factorization: release it
        REXI_HIP(hipStreamSynchronize(stream));
        REXI_HIP(hipFree(ctx->d_fact));
        ctx->d_fact = nullptr;
        ctx->fact_cap = 0;
        ctx->fact_valid = false;
    }
    if (best_ms) *best_ms = best_t / reps;
    return REXI_OK;
}

int sh_synthesis(swe_ctx* ctx, const double* spec, double* grid, int nf, hipStream_t stream) {
    if (!ctx) return fail(REXI_EINVAL, "sh_synthesis: NULL context");
    if (!ctx->nlat) return fail(REXI_ENOTSUP, "sh_synthesis: linear-only context (no grid)");
    if (!spec || !grid || nf < 1 || nf > 64) return fail(REXI_EINVAL, "sh_synthesis: bad pointer or nf");
    DeviceGuard guard(ctx->device);
    int rc;
    if ((rc = reserve_fourier(ctx, nf)) != REXI_OK) return rc;
    if ((rc = to_fourier(ctx, 0, spec, nf, stream)) != REXI_OK) return rc;
    return ring_from_part(ctx, 0, grid, nf, stream);
}

int sh_analysis(swe_ctx* ctx, const double* grid, double* spec, int nf, hipStream_t stream) {
    if (!ctx) return fail(REXI_EINVAL, "sh_analysis: NULL context");
    if (!ctx->nlat) return fail(REXI_ENOTSUP, "sh_analysis: linear-only context (no grid)");
    if (!spec || !grid || nf < 1 || nf > 64) return fail(REXI_EINVAL, "sh_analysis: bad pointer or nf");
    DeviceGuard guard(ctx->device);
    int rc;
    if ((rc = reserve_fourier(ctx, nf)) != REXI_OK) return rc;
    if ((rc = launch_ring(ctx, 1, nullptr, nullptr, 0, ctx->d_fout, grid, nullptr, nf, stream)) != REXI_OK) return rc;
    return from_fourier(ctx, 0, spec, nf, nullptr, nullptr, nullptr, nullptr, 0.0, 0.0, stream);
}

int swe_nonlinear_step(swe_ctx* ctx, double tau, const double* U0, double* U1, hipStream_t stream) {
    if (!ctx) return fail(REXI_EINVAL, "swe_nonlinear_step: NULL context");
    if (!ctx->nlat) return fail(REXI_ENOTSUP, "swe_nonlinear_step: linear-only context (no grid)");
    if (!U0 || !U1) return fail(REXI_EINVAL, "swe_nonlinear_step: NULL state");
    if (!std::isfinite(tau)) return fail(REXI_EINVAL, "swe_nonlinear_step: tau must be finite");
    DeviceGuard guard(ctx->device);
    return heun_step(ctx, tau, U0, U1, stream);
}

namespace {
// One l_rexi_n_erk_ver1 step U0 -> U1 on prepared poles.  synth_done and
// synth_next as in heun_step (the synthesis of U0 already in ctx->d_part; the
// synthesis of U1 wanted there).
int strang_once(swe_ctx* ctx, int N, double dt, const double* U0, double* U1, hipStream_t stream, bool synth_done,
                bool* synth_next) {
    int rc;
    if ((rc = heun_step(ctx, 0.5 * dt, U0, ctx->d_tmpA, stream, 0.0, synth_done)) != REXI_OK) return rc;
    int nparts = 0;
    if ((rc = launch_rexi_chain(ctx, N, dt, ctx->d_tmpA, ctx->d_tmpB, &nparts, stream)) != REXI_OK) return rc;
    bool rexi_synth = false;
    if (nparts > 1 && ctx->fuse && split_legendre(ctx)) {
        // the pole sum of each order synthesises its result for the next Heun step
        if ((rc = reserve_fourier(ctx, 5)) != REXI_OK) return rc;
        if ((rc = launch_rexi_sum_synth_split(ctx, ctx->d_partial, nparts, ctx->d_tmpB, ctx->d_part, stream)) !=
            REXI_OK)
            return rc;
        rexi_synth = true;
    } else if (nparts > 1 && (rc = launch_rexi_sum(ctx, nparts, ctx->d_tmpB, stream)) != REXI_OK) {
        return rc;
    }
    return heun_step(ctx, 0.5 * dt, ctx->d_tmpB, U1, stream, 0.0, rexi_synth, synth_next);
}

int strang_checks(swe_ctx* ctx, const double* alpha, const double* beta, int N, double dt, const double* U0,
                  double* U1, const char* who) {
    if (!ctx) return fail(REXI_EINVAL, std::string(who) + ": NULL context");
    if (!ctx->nlat) return fail(REXI_ENOTSUP, std::string(who) + ": linear-only context (no grid)");
    if (!alpha || !beta || !U0 || !U1) return fail(REXI_EINVAL, std::string(who) + ": NULL pointer");
    if (N < 2 || (N & 1) || N > (1 << 20)) return fail(REXI_EINVAL, std::string(who) + ": N must be even and in [2, 2^20]");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(REXI_EINVAL, std::string(who) + ": dt must be positive");
    return REXI_OK;
}
}  // namespace

int swe_strang_step(swe_ctx* ctx, const double* alpha, const double* beta, int N, double dt,
                    const double* U0, double* U1, hipStream_t stream) {
    int rc;
    if ((rc = strang_checks(ctx, alpha, beta, N, dt, U0, U1, "swe_strang_step")) != REXI_OK) return rc;
    DeviceGuard guard(ctx->device);
    if ((rc = prepare_poles(ctx, alpha, beta, N, dt, true, "swe_strang_step", stream)) != REXI_OK) return rc;
    return strang_once(ctx, N, dt, U0, U1, stream, false, nullptr);
}

int swe_strang_steps(swe_ctx* ctx, const double* alpha, const double* beta, int N, double dt, int nsteps,
                     const double* U0, double* U1, hipStream_t stream) {
    int rc;
    if ((rc = strang_checks(ctx, alpha, beta, N, dt, U0, U1, "swe_strang_steps")) != REXI_OK) return rc;
    if (nsteps < 1) return fail(REXI_EINVAL, "swe_strang_steps: nsteps must be at least 1");
    DeviceGuard guard(ctx->device);
    if ((rc = prepare_poles(ctx, alpha, beta, N, dt, true, "swe_strang_steps", stream)) != REXI_OK) return rc;
    // step k writes U1 when nsteps - 1 - k is even, else the context's state
    // buffer, so that consecutive steps never share a buffer and the last
    // writes U1
    const double* src = U0;
    bool synth_done = false;
    for (int k = 0; k < nsteps; ++k) {
        double* dst = ((nsteps - 1 - k) % 2 == 0) ? U1 : ctx->d_tmpC;
        bool synth_next = k + 1 < nsteps;
        if ((rc = strang_once(ctx, N, dt, src, dst, stream, synth_done, &synth_next)) != REXI_OK) return rc;
        synth_done = synth_next;
        src = dst;
    }
    return REXI_OK;
}

int swe_cn_step(swe_ctx* ctx, double dt, const double* U0, double* U1, hipStream_t stream) {
    if (!ctx) return fail(REXI_EINVAL, "swe_cn_step: NULL context");
    if (!U0 || !U1) return fail(REXI_EINVAL, "swe_cn_step: NULL pointer");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(REXI_EINVAL, "swe_cn_step: dt must be positive");
    const size_t bytes = sizeof(double) * 6 * ctx->modes;
    const char* a0 = reinterpret_cast<const char*>(U0);
    const char* a1 = reinterpret_cast<const char*>(U1);
    if (a0 < a1 + bytes && a1 < a0 + bytes) return fail(REXI_EINVAL, "swe_cn_step: U0 and U1 overlap");
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(REXI_EDEVICE, "swe_cn_step: cannot select the context's device");
    return cn_linear(ctx, dt, U0, U1, stream);
}

int swe_split_step(swe_ctx* ctx, int scheme, const double* alpha, const double* beta, int N, double dt,
                   const double* U0, double* U1, hipStream_t stream) {
    if (!ctx) return fail(REXI_EINVAL, "swe_split_step: NULL context");
    if (!ctx->nlat) return fail(REXI_ENOTSUP, "swe_split_step: linear-only context (no grid)");
    if (scheme < REXI_SPLIT_REXI_V1 || scheme > REXI_SPLIT_LG_REXI_V1)
        return fail(REXI_EINVAL, "swe_split_step: unknown scheme");
    const bool lg = scheme == REXI_SPLIT_LG_REXI_V1;
    const bool rexi = scheme == REXI_SPLIT_REXI_V1 || scheme == REXI_SPLIT_REXI_V0 || lg;
    const bool v1 = scheme == REXI_SPLIT_REXI_V1 || scheme == REXI_SPLIT_CN_V1 || lg;
    const double two_omega = lg ? 2.0 * ctx->Omega : 0.0;   // L_c joins the explicit part
    if (!U0 || !U1 || (rexi && (!alpha || !beta))) return fail(REXI_EINVAL, "swe_split_step: NULL pointer");
    if (rexi && (N < 2 || (N & 1) || N > (1 << 20)))
        return fail(REXI_EINVAL, "swe_split_step: N must be even and in [2, 2^20]");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(REXI_EINVAL, "swe_split_step: dt must be positive");
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(REXI_EDEVICE, "swe_split_step: cannot select the context's device");
    const double tl = v1 ? dt : 0.5 * dt;   // step of the linear part
    int rc;
    auto linear = [&](const double* in, double* out) -> int {
        if (!rexi) return cn_linear(ctx, tl, in, out, stream);
        int r = prepare_poles(ctx, alpha, beta, N, tl, !lg, "swe_split_step", stream);
        if (r != REXI_OK) return r;
        return lg ? launch_rexi_lg(ctx, N, tl, in, out, stream) : launch_rexi_solve(ctx, N, tl, in, out, stream);
    };
    if (v1) {
        if ((rc = heun_step(ctx, 0.5 * dt, U0, ctx->d_tmpA, stream, two_omega)) != REXI_OK) return rc;
        if ((rc = linear(ctx->d_tmpA, ctx->d_tmpB)) != REXI_OK) return rc;
        return heun_step(ctx, 0.5 * dt, ctx->d_tmpB, U1, stream, two_omega);
    }
    if ((rc = linear(U0, ctx->d_tmpA)) != REXI_OK) return rc;
    if ((rc = heun_step(ctx, dt, ctx->d_tmpA, ctx->d_tmpB, stream)) != REXI_OK) return rc;
    return linear(ctx->d_tmpB, U1);
}

int swe_etdrk2_step(swe_ctx* ctx, const double* alpha, const double* beta0, const double* beta1,
                    const double* beta2, int N, double dt, const double* U0, double* U1, hipStream_t stream) {
    if (!ctx) return fail(REXI_EINVAL, "swe_etdrk2_step: NULL context");
    if (!ctx->nlat) return fail(REXI_ENOTSUP, "swe_etdrk2_step: linear-only context (no grid)");
    if (!alpha || !beta0 || !beta1 || !beta2 || !U0 || !U1) return fail(REXI_EINVAL, "swe_etdrk2_step: NULL pointer");
    if (N < 2 || (N & 1) || N > (1 << 20)) return fail(REXI_EINVAL, "swe_etdrk2_step: N must be even and in [2, 2^20]");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(REXI_EINVAL, "swe_etdrk2_step: dt must be positive");
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(REXI_EDEVICE, "swe_etdrk2_step: cannot select the context's device");
    // dt psi_1 and dt psi_2 as sums with the weights scaled by dt
    std::vector<double> b1(2 * static_cast<size_t>(N)), b2(2 * static_cast<size_t>(N));
    for (int i = 0; i < 2 * N; ++i) {
        b1[i] = dt * beta1[i];
        b2[i] = dt * beta2[i];
    }
    const int n = 6 * ctx->modes;
    int rc;
    // N0 = N(U0)
    if ((rc = tendency_eval(ctx, U0, ctx->d_n0, stream)) != REXI_OK) return rc;
    // A = psi_0(dt L) U0 + dt psi_1(dt L) N0
    if ((rc = prepare_poles(ctx, alpha, beta0, N, dt, true, "swe_etdrk2_step", stream)) != REXI_OK) return rc;
    if ((rc = launch_rexi_solve(ctx, N, dt, U0, ctx->d_tmpA, stream)) != REXI_OK) return rc;
    if ((rc = prepare_poles(ctx, alpha, b1.data(), N, dt, true, "swe_etdrk2_step", stream)) != REXI_OK) return rc;
    if ((rc = launch_rexi_solve(ctx, N, dt, ctx->d_n0, ctx->d_tmpB, stream)) != REXI_OK) return rc;
    if ((rc = launch_axpy(ctx->d_tmpA, ctx->d_tmpA, 1.0, ctx->d_tmpB, n, ctx->d_status, STATUS_REXI, stream)) != REXI_OK)
        return rc;
    // D = N(A) - N0
    if ((rc = tendency_eval(ctx, ctx->d_tmpA, ctx->d_ustar, stream)) != REXI_OK) return rc;
    if ((rc = launch_axpy(ctx->d_ustar, ctx->d_ustar, -1.0, ctx->d_n0, n, ctx->d_status, STATUS_NONLINEAR, stream)) !=
        REXI_OK)
        return rc;
    // U1 = A + dt psi_2(dt L) D
    if ((rc = prepare_poles(ctx, alpha, b2.data(), N, dt, true, "swe_etdrk2_step", stream)) != REXI_OK) return rc;
    if ((rc = launch_rexi_solve(ctx, N, dt, ctx->d_ustar, ctx->d_tmpB, stream)) != REXI_OK) return rc;
    return launch_axpy(U1, ctx->d_tmpA, 1.0, ctx->d_tmpB, n, ctx->d_status, STATUS_NONLINEAR, stream);
}

int swe_profile(swe_ctx* ctx, int enable) {
    if (!ctx) return fail(REXI_EINVAL, "swe_profile: NULL context");
    ctx->prof.mask = enable ? ~0u : 0u;
    return REXI_OK;
}

int swe_profile_kernels(swe_ctx* ctx, unsigned mask) {
    if (!ctx) return fail(REXI_EINVAL, "swe_profile_kernels: NULL context");
    ctx->prof.mask = mask;
    return REXI_OK;
}

int swe_profile_read(swe_ctx* ctx, int kernel, double* total_ms, int* launches) {
    if (!ctx || !total_ms || !launches) return fail(REXI_EINVAL, "swe_profile_read: NULL argument");
    if (kernel < 0 || kernel >= REXI_KERNEL_COUNT) return fail(REXI_EINVAL, "swe_profile_read: bad kernel id");
    DeviceGuard guard(ctx->device);
    Profiler& p = ctx->prof;
    double sum = 0.0;
    for (int i = 0; i < p.count[kernel]; ++i) {
        REXI_HIP(hipEventSynchronize(p.stop[kernel][i]));
        float ms = 0.0f;
        REXI_HIP(hipEventElapsedTime(&ms, p.start[kernel][i], p.stop[kernel][i]));
        sum += ms;
    }
    *total_ms = sum;
    *launches = p.count[kernel];
    p.count[kernel] = 0;
    return REXI_OK;
}

int swe_sync(swe_ctx* ctx) {
    if (!ctx) return fail(REXI_EINVAL, "swe_sync: NULL context");
    DeviceGuard guard(ctx->device);
    REXI_HIP(hipDeviceSynchronize());
    unsigned flags = 0;
    REXI_HIP(hipMemcpy(&flags, ctx->d_status, sizeof flags, hipMemcpyDeviceToHost));
    if (flags) {
        REXI_HIP(hipMemset(ctx->d_status, 0, sizeof flags));
        REXI_HIP(hipDeviceSynchronize());
        std::string what;
        if (flags & STATUS_REXI) what += " REXI/linear stage output;";
        if (flags & STATUS_NONLINEAR) what += " non-linear step output;";
        if (flags & STATUS_TRANSFORM) what += " transform output;";
        return fail(REXI_ENUMERIC, "swe_sync: non-finite values were written since the last swe_sync:" + what);
    }
    return REXI_OK;
}

}  // extern "C"
