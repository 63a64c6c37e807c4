// helm_precond_apply_noalloc: the FP32 EigT preconditioner for callers that cannot allocate device memory (code under
// stream capture, serving loops, harnesses that forbid allocation). The two complex64 staging vectors between the
// transforms and the z-solve live in one static device array, `scratch`, of NOALLOC_MAX_N * 2 complex64 values
// (32 MiB); the library resolves its address per device with hipGetSymbolAddress on the first call on that device
// and passes that address to the kernels. Every call on a device shares that device's array, so calls that overlap
// on one device (two streams, two threads) race.
#include <mutex>

#include "helm_internal.h"

namespace {
constexpr long long NOALLOC_MAX_N = 1LL << 21;   // 2^21 unknowns (e.g. 128^3)
constexpr int NOALLOC_MAX_DEVICES = 64;
}  // namespace

static __device__ __align__(256) float2 scratch[2 * NOALLOC_MAX_N];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The device address of `scratch` on `device` (made current for the query), resolved once per device.
hipError_t scratch_address(int device, float2 **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *out = static_cast<float2 *>(g_scratch_ptr[device]);
    return hipSuccess;
}

}  // namespace

extern "C" helm_status helm_precond_apply_noalloc(helm_ctx *ctx, const void *y_dev, void *z_dev) {
    if (!ctx) return HELM_EINVAL;
    helm::Ctx &c = ctx->c;
    if (!y_dev || !z_dev) { c.err = "NULL pointer"; return HELM_EINVAL; }
    if (c.n > NOALLOC_MAX_N) {
        c.err = "helm_precond_apply_noalloc: n = " + std::to_string(c.n) + " exceeds its maximum of " +
                std::to_string(NOALLOC_MAX_N) + " unknowns";
        return HELM_EINVAL;
    }
    if (c.device < 0 || c.device >= NOALLOC_MAX_DEVICES) { c.err = "device index out of range"; return HELM_EINVAL; }
    float2 *base = nullptr;
    const hipError_t e = scratch_address(c.device, &base);
    if (e != hipSuccess) {
        c.err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return HELM_EDEVICE;
    }
    return helm::eigt32_apply_ws(c, (const double2 *)y_dev, (double2 *)z_dev, base, base + NOALLOC_MAX_N);
}
