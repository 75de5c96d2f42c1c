// A variant of mpmc_apply_poly that allocates nothing, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops,
// harnesses that forbid hipMalloc).  Its work vectors live in one file-scope
// device array of fixed size; every GPU the library runs on holds its own copy
// until the process ends.  The array's host-side name is not a device address:
// its address on each device is taken once with hipGetSymbolAddress (with that
// device current) and only that pointer reaches kernels.
#include <mutex>

#include "common.h"

namespace {

constexpr size_t kScratchBytes = 64ull << 20;   // the limit of mpmc_apply_poly_noalloc
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mtx;
std::map<int, void *> g_scratch;   // device -> address of its copy of scratch

}  // namespace

// Address of this device's scratch array (taken once per device, with the
// device current); nullptr on failure.
void *noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_mtx);
    const auto it = g_scratch.find(device);
    if (it != g_scratch.end()) return it->second;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != device && hipSetDevice(device) != hipSuccess) return nullptr;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) hipSetDevice(cur);
    if (e != hipSuccess || !ptr) return nullptr;
    g_scratch[device] = ptr;
    return ptr;
}

MPMC_API int mpmc_apply_poly_noalloc(mpmc_ctx *ctx, const mpmc_poly *p, const void *x, void *y, int nrhs, int prec) {
    if (!ctx) return MPMC_EINVAL;
    RET_IF(poly_validate(ctx, p));
    if (!x || !y || nrhs < 1) return set_err(ctx, MPMC_EINVAL, "mpmc_apply_poly_noalloc: bad argument");
    if (x == y) return set_err(ctx, MPMC_EINVAL, "mpmc_apply_poly_noalloc: x and y must not alias");
    if (prec != MPMC_FP64 && prec != MPMC_FP32)
        return set_err(ctx, MPMC_EINVAL, "mpmc_apply_poly_noalloc: FP64 or FP32 only");
    if (ctx->timing)
        return set_err(ctx, MPMC_ESTATE, "mpmc_apply_poly_noalloc: launch timing is on (it creates events)");
    const size_t vb = (vec_bytes(ctx, nrhs, prec) + 255) & ~(size_t)255;
    const int nbuf = poly_work_vectors(p);
    if ((size_t)nbuf * vb > kScratchBytes)
        return set_err(ctx, MPMC_EINVAL, "mpmc_apply_poly_noalloc: %d work vectors of %zu bytes exceed the %zu-byte limit",
                       nbuf, vb, kScratchBytes);
    char *base = (char *)noalloc_scratch(ctx->device);
    if (!base) return set_err(ctx, MPMC_EHIP, "mpmc_apply_poly_noalloc: no device address for the scratch array");
    void *buf[6];
    for (int i = 0; i < nbuf; ++i) buf[i] = base + (size_t)i * vb;
    return poly_apply_buf(ctx, p, x, y, nrhs, prec, buf);
}
