// Non-allocating variant of the Gram-Schmidt dot products (fvk_multidot) for
// callers that cannot allocate device memory while they run (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The block partials of the multi-dot reduction live in a file-scope device
// array of fixed size; each GPU holds its own copy until the process ends.
// Host code never passes the array's name to a kernel (on the host it is only
// a stand-in symbol): its device address is looked up once per device with
// hipGetSymbolAddress and that pointer is used for every launch.
#include <mutex>

#include "fvk_internal.h"

namespace {

// at most 1024 blocks (multidot_blocks) x 256 vectors of partial sums: 2 MiB
constexpr int kMaxVectors = 256;
constexpr size_t kScratchDoubles = size_t(1024) * kMaxVectors;

__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up once per
// device); nullptr and a message on failure
double *scratch_on_current_device(std::string *err) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        if (err) *err = "fvk_multidot_noalloc: no usable current device";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            if (err) *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_ptr[dev] = static_cast<double *>(p);
    }
    return g_ptr[dev];
}

}  // namespace

namespace fvk {

// called by fvk_create with the context's device current
bool noalloc_prepare(std::string *err) { return scratch_on_current_device(err) != nullptr; }

}  // namespace fvk

extern "C" {

fvk_status fvk_multidot_noalloc(fvk_ctx *ctx, const double *V, size_t ldv, int m,
                                const double *w, size_t n, double *out_dev) {
    if (!ctx || !V || !w || !out_dev || n == 0) return FVK_EINVAL;
    if (m < 1 || m > kMaxVectors) {
        ctx->err = "fvk_multidot_noalloc: m must be 1 .. 256";
        return FVK_EINVAL;
    }
    if (m > 1 && ldv < n) {
        ctx->err = "fvk_multidot_noalloc: ldv smaller than n";
        return FVK_EINVAL;
    }
    const int nb = fvk::multidot_blocks(n);
    if (size_t(nb) * size_t(m) > kScratchDoubles) {   // cannot happen: nb <= 1024
        ctx->err = "fvk_multidot_noalloc: partials exceed the static scratch";
        return FVK_EINVAL;
    }
    double *partials = scratch_on_current_device(&ctx->err);
    if (!partials) return FVK_EHIP;
    // every block writes all m of its partials and the reduction overwrites
    // out_dev, so nothing has to be cleared between calls
    fvk::launch_multidot(V, ldv, m, w, n, partials, nb, ctx->stream);
    fvk::launch_reduce_partials(partials, nb, m, out_dev, 0, ctx->stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        ctx->err = std::string("fvk_multidot_noalloc: ") + hipGetErrorString(e);
        return FVK_EHIP;
    }
    return FVK_OK;
}

}  // extern "C"
