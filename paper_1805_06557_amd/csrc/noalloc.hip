// Allocation-free variant of rexi_lg_step: the REXI stage of the gravity-wave
// part L_g (Section 3 splitting; per-degree pole sums applied per mode) for
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc).  Its two kernels are those
// of rexi_lg_step; the device memory they need besides the caller's state (the
// pole table and the per-degree sums) lives in one static device array of
// fixed size instead of context-owned allocations.
//
// The array is a file-scope __device__ variable: every device the library runs
// on holds its own copy until the process ends.  In host code its name is only
// a host-side stand-in, so the device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// handed to kernels and copies.
#include <cmath>
#include <mutex>

#include "internal.h"

namespace rexi {
namespace {

constexpr int kMaxPoles = 4096;        // N <= kMaxPoles
constexpr int kMaxL = 1023;            // the library's largest truncation
constexpr size_t kPoleBytes = sizeof(PoleData) * kMaxPoles;                   // 196 608 B
constexpr size_t kSumBytes = sizeof(double) * 4 * static_cast<size_t>(kMaxL + 2);   // 32 800 B
constexpr size_t kScratchBytes = kPoleBytes + kSumBytes;                      // 229 408 B
static_assert(kPoleBytes % 256 == 0, "the sums start 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;

// Host-side state per device: the scratch address, the coefficient set whose
// pole table the scratch holds, and the host staging table it was built in.
struct DeviceScratch {
    std::mutex mu;
    bool resolved = false;
    unsigned char* ptr = nullptr;     // device address of `scratch` on this device
    bool poles_valid = false;
    uint64_t poles_key = 0;
    PoleData host[kMaxPoles];
};

DeviceScratch g_dev[kMaxDevices];

// Resolves the scratch address of the current device; dev.mu must be held.
hipError_t resolve_locked(DeviceScratch& dev) {
    if (dev.resolved) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    dev.ptr = static_cast<unsigned char*>(p);
    dev.resolved = true;
    return hipSuccess;
}

}  // namespace

int noalloc_init_device(int device) {
    if (device < 0 || device >= kMaxDevices) return REXI_ENOTSUP;
    DeviceScratch& dev = g_dev[device];
    std::lock_guard<std::mutex> lock(dev.mu);
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) return REXI_EDEVICE;
    return resolve_locked(dev) == hipSuccess ? REXI_OK : REXI_EDEVICE;
}

}  // namespace rexi

using namespace rexi;

extern "C" int rexi_lg_step_noalloc(swe_ctx* ctx, const double* alpha, const double* beta, int N, double dt,
                                    const double* U0, double* U1, hipStream_t stream) {
    if (!ctx) return fail(REXI_EINVAL, "rexi_lg_step_noalloc: NULL context");
    if (!alpha || !beta || !U0 || !U1) return fail(REXI_EINVAL, "rexi_lg_step_noalloc: NULL pointer");
    if (N < 2 || (N & 1)) return fail(REXI_EINVAL, "rexi_lg_step_noalloc: N must be even and at least 2");
    if (N > kMaxPoles)
        return fail(REXI_EINVAL, "rexi_lg_step_noalloc: N exceeds the scratch limit of 4096 poles");
    if (ctx->L > kMaxL) return fail(REXI_EINVAL, "rexi_lg_step_noalloc: L exceeds the scratch limit of 1023");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(REXI_EINVAL, "rexi_lg_step_noalloc: dt must be positive");
    if (ctx->device < 0 || ctx->device >= kMaxDevices)
        return fail(REXI_ENOTSUP, "rexi_lg_step_noalloc: device index beyond the scratch table");
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return fail(REXI_EDEVICE, "rexi_lg_step_noalloc: hipGetDevice failed");
    if (prev != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(REXI_EDEVICE, "rexi_lg_step_noalloc: cannot select the context's device");
    struct Restore {
        int prev, cur;
        ~Restore() {
            if (prev >= 0 && prev != cur) (void)hipSetDevice(prev);
        }
    } restore{prev, ctx->device};

    DeviceScratch& dev = g_dev[ctx->device];
    std::lock_guard<std::mutex> lock(dev.mu);
    const hipError_t e = resolve_locked(dev);
    if (e != hipSuccess) return hip_fail(e, "rexi_lg_step_noalloc: hipGetSymbolAddress(scratch)");
    const uint64_t key = pole_key(alpha, beta, N, dt);
    if (!dev.poles_valid || dev.poles_key != key) {
        build_pole_data(alpha, beta, N, dev.host);
        const int rc = check_poles(ctx, dev.host, N, dt, false, "rexi_lg_step_noalloc");
        if (rc != REXI_OK) return rc;
        // ordered after earlier work on `stream`; the wait lets the next call
        // rebuild the host table
        dev.poles_valid = false;
        REXI_HIP(hipMemcpyAsync(dev.ptr, dev.host, sizeof(PoleData) * static_cast<size_t>(N),
                                hipMemcpyHostToDevice, stream));
        REXI_HIP(hipStreamSynchronize(stream));
        dev.poles_key = key;
        dev.poles_valid = true;
    }
    return launch_rexi_lg_on(ctx, reinterpret_cast<const PoleData*>(dev.ptr), dev.ptr + kPoleBytes, N, dt, U0, U1,
                             stream);
}
