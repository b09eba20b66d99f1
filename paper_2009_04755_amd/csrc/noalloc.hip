// Allocation-free all-pairs entry point, for callers that cannot allocate device memory
// (code under stream capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The library's kernels take their workspace (prepared item copies, split-K partials, the
// work queue) from a context's slots.  Here those slots are carved, in call order, from one
// file-scope device array of ROCKET_NOALLOC_SCRATCH_BYTES; the kernels and host logic are
// the ones rocket_allpairs_ex runs.  Each device holds its own copy of the array until the
// process ends; its device address is taken once per device with hipGetSymbolAddress (the
// array's name in host code is only a host-side stand-in) and only that address is used.
#include <cstdio>
#include <mutex>

#include "common.hpp"

namespace {

constexpr int MAX_DEV = 64;

// The scratch buffer.  Zero-initialised at load; every call re-clears what must start at
// zero (queue counters, flags, histograms) with kernels or stream-ordered fills of its own.
__device__ __align__(256) char scratch[ROCKET_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu[MAX_DEV];
char *g_ptr[MAX_DEV] = {nullptr};        // device address of `scratch` on each device
rocket_ctx *g_ctx[MAX_DEV] = {nullptr};  // one internal arena-mode context per device

// Called with g_mu[dev] held and `dev` current.
rocket_status setup(int dev)
{
    if (g_ptr[dev] && g_ctx[dev]) return ROCKET_OK;
    rocket_ctx *ctx = nullptr;  // for the RK_HIP error path: report without a context
    void *p = nullptr;
    RK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return rk::fail(nullptr, ROCKET_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    rocket_ctx *c = nullptr;
    RK_TRY(rocket_create(&c, dev));
    c->arena = (char *)p;
    c->arena_cap = ROCKET_NOALLOC_SCRATCH_BYTES;
    g_ptr[dev] = (char *)p;
    g_ctx[dev] = c;
    return ROCKET_OK;
}

}  // namespace

extern "C" {

rocket_status rocket_allpairs_noalloc(const rocket_items *items, int64_t n, rocket_pair_fn fn, float *out,
                                      uint32_t *out_counts, void *stream)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return rk::hip_fail(nullptr, e, "hipGetDevice", __FILE__, __LINE__);
    if (dev < 0 || dev >= MAX_DEV) return rk::fail(nullptr, ROCKET_E_INVALID, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu[dev]);
    RK_TRY(setup(dev));
    rocket_ctx *ctx = g_ctx[dev];
    // Fresh layout for every call: no slot, plan or queue survives from the previous call,
    // so every buffer this call uses is carved (and re-initialised) by this call.
    for (auto &b : ctx->ws) b = rk::Buffer();
    ctx->arena = g_ptr[dev];
    ctx->arena_used = 0;
    ctx->ncc = rk::NccState();
    ctx->ovl = rk::OvlState();
    ctx->sp = rk::SpState();
    ctx->pce = rk::PceState();
    ctx->queue_owner = rk::QOWN_NONE;
    ctx->prepared_fn = 0;
    ctx->last_error.clear();
    rocket_status st = rocket_allpairs_ex(ctx, items, n, fn, out, out_counts, stream);
    if (st != ROCKET_OK) {
        // the internal context is not visible to the caller: its message (after the status
        // name that fail() put in front) becomes rocket_last_error(NULL)
        const std::string &m = ctx->last_error;
        const size_t c = m.find(": ");
        rk::fail(nullptr, st, c == std::string::npos ? m : m.substr(c + 2));
    }
    return st;
}

}  // extern "C"
