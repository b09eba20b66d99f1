// C ABI entry points, context and workspace management, queue upload.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "common.hpp"

namespace {

__global__ void k_fill_i32(int *p, int64_t n, int v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

rocket_ctx *g_default[64] = {nullptr};
std::mutex g_default_mu;
std::string g_null_error;

bool valid_fn(int fn) { return fn >= ROCKET_NCC_FP32 && fn <= ROCKET_PCE; }

}  // namespace

namespace rk {

rocket_status fail(rocket_ctx *ctx, rocket_status st, const std::string &msg)
{
    (ctx ? ctx->last_error : g_null_error) = std::string(rocket_status_str(st)) + ": " + msg;
    return st;
}

rocket_status hip_fail(rocket_ctx *ctx, hipError_t e, const char *what, const char *file, int line)
{
    char buf[512];
    snprintf(buf, sizeof buf, "%s failed with %s (%s) at %s:%d", what, hipGetErrorName(e), hipGetErrorString(e), file,
             line);
    return fail(ctx, e == hipErrorOutOfMemory ? ROCKET_E_OOM : ROCKET_E_HIP, buf);
}

int64_t ws_total(const rocket_ctx *ctx)
{
    int64_t t = 0;
    for (int k = 0; k < WS_COUNT; ++k) t += (int64_t)ctx->ws[k].bytes;
    return t;
}

rocket_status ws_get(rocket_ctx *ctx, Slot slot, size_t bytes, void **out)
{
    Buffer &b = ctx->ws[slot];
    if (bytes == 0) bytes = 256;
    if (ctx->arena) {
        // carve from the caller-provided arena: 256-byte aligned pieces in call order; a
        // slot that grows gets a new piece (its old contents are not kept, as with hipMalloc)
        if (b.bytes < bytes) {
            const size_t want = (bytes + 255) & ~(size_t)255;
            if (want > ctx->arena_cap - ctx->arena_used) {
                char buf[256];
                snprintf(buf, sizeof buf,
                         "the allocation-free entry point's scratch holds %zu bytes; this problem needs more "
                         "(%zu in use, %zu more requested)",
                         ctx->arena_cap, ctx->arena_used, want);
                return fail(ctx, ROCKET_E_OOM, buf);
            }
            b.ptr = ctx->arena + ctx->arena_used;
            b.bytes = want;
            ctx->arena_used += want;
        }
        *out = b.ptr;
        return ROCKET_OK;
    }
    if (b.bytes < bytes) {
        const size_t want = (bytes + (2u << 20) - 1) & ~(size_t)((2u << 20) - 1);
        const int64_t cap = ctx->opt[ROCKET_OPT_WORKSPACE_CAP];
        if (cap > 0 && ws_total(ctx) - (int64_t)b.bytes + (int64_t)want > cap)
            return fail(ctx, ROCKET_E_OOM, "workspace cap exceeded");
        if (b.ptr) {
            RK_HIP(hipFree(b.ptr));
            b.ptr = nullptr;
            b.bytes = 0;
        }
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, ROCKET_E_OOM, "hipMalloc of workspace failed");
        }
        b.ptr = p;
        b.bytes = want;
    }
    *out = b.ptr;
    return ROCKET_OK;
}

rocket_status upload_queue(rocket_ctx *ctx, hipStream_t s, QueueArgs *qa)
{
    const int64_t nitems = (int64_t)ctx->h_items.size();
    const int nseg = (int)ctx->h_seg.size() - 1;
    void *items = nullptr, *heads = nullptr, *seg = nullptr;
    RK_TRY(ws_get(ctx, WS_QUEUE_ITEMS, sizeof(int4) * (size_t)std::max<int64_t>(nitems, 1), &items));
    RK_TRY(ws_get(ctx, WS_QUEUE_HEADS, sizeof(int) * HEAD_STRIDE * MAX_SEG, &heads));
    RK_TRY(ws_get(ctx, WS_QUEUE_SEGS, sizeof(int) * (MAX_SEG + 1), &seg));
    if (nitems) RK_HIP(hipMemcpyAsync(items, ctx->h_items.data(), sizeof(int4) * nitems, hipMemcpyHostToDevice, s));
    RK_HIP(hipMemcpyAsync(seg, ctx->h_seg.data(), sizeof(int) * (nseg + 1), hipMemcpyHostToDevice, s));
    RK_HIP(hipStreamSynchronize(s));  // host staging vectors may be reused right after
    qa->items = (const int4 *)items;
    qa->heads = (int *)heads;
    qa->seg = (const int *)seg;
    qa->nseg = nseg;
    qa->ledger = nullptr;
    if (ctx->opt[ROCKET_OPT_LEDGER]) {
        void *led = nullptr;
        RK_TRY(ws_get(ctx, WS_LEDGER, sizeof(int) * (size_t)std::max<int64_t>(nitems, 1), &led));
        qa->ledger = (int *)led;
    }
    ctx->ledger_items = nitems;
    qa->trace = nullptr;
    ctx->trace_valid = false;
    if (ctx->opt[ROCKET_OPT_TRACE]) {
        void *tr = nullptr;
        RK_TRY(ws_get(ctx, WS_TRACE, 3 * sizeof(unsigned long long) * (size_t)std::max<int64_t>(nitems, 1), &tr));
        qa->trace = (unsigned long long *)tr;
        ctx->trace_valid = true;
    }
    return ROCKET_OK;
}

rocket_status reset_queue(rocket_ctx *ctx, hipStream_t s, const QueueArgs &qa)
{
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, s, qa.heads, (int64_t)HEAD_STRIDE * MAX_SEG, 0);
    RK_HIP(hipGetLastError());
    if (qa.ledger) {
        const int64_t n = std::max<int64_t>(ctx->ledger_items, 1);
        hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0, s,
                           qa.ledger, n, 0);
        RK_HIP(hipGetLastError());
    }
    if (qa.trace) {  // items never run keep zeros
        const int64_t n = 6 * std::max<int64_t>(ctx->ledger_items, 1);
        hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0, s,
                           (int *)qa.trace, n, 0);
        RK_HIP(hipGetLastError());
    }
    return ROCKET_OK;
}

rocket_status timing_begin(rocket_ctx *ctx, hipStream_t s)
{
    if (!ctx->opt[ROCKET_OPT_TIMING]) return ROCKET_OK;
    if (!ctx->ev_begin) {
        RK_HIP(hipEventCreate(&ctx->ev_begin));
        RK_HIP(hipEventCreate(&ctx->ev_end));
    }
    RK_HIP(hipEventRecord(ctx->ev_begin, s));
    return ROCKET_OK;
}

rocket_status timing_end(rocket_ctx *ctx, hipStream_t s)
{
    if (!ctx->opt[ROCKET_OPT_TIMING]) return ROCKET_OK;
    RK_HIP(hipEventRecord(ctx->ev_end, s));
    ctx->ev_pending = true;
    return ROCKET_OK;
}

int auto_grid(rocket_ctx *ctx, const void *kernel, int block, size_t dyn_lds, int64_t items)
{
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, dyn_lds) != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    int64_t g = ctx->opt[ROCKET_OPT_GRID] > 0 ? ctx->opt[ROCKET_OPT_GRID] : (int64_t)ctx->num_cu * per_cu;
    if (g > items) g = std::max<int64_t>(items, 1);
    return (int)g;
}

}  // namespace rk

extern "C" {

const char *rocket_status_str(rocket_status s)
{
    switch (s) {
    case ROCKET_OK: return "ROCKET_OK";
    case ROCKET_E_INVALID: return "ROCKET_E_INVALID";
    case ROCKET_E_UNSUPPORTED: return "ROCKET_E_UNSUPPORTED";
    case ROCKET_E_OOM: return "ROCKET_E_OOM";
    case ROCKET_E_HIP: return "ROCKET_E_HIP";
    case ROCKET_E_KEYRANGE: return "ROCKET_E_KEYRANGE";
    case ROCKET_E_UNSORTED: return "ROCKET_E_UNSORTED";
    case ROCKET_E_STATE: return "ROCKET_E_STATE";
    }
    return "ROCKET_E_UNKNOWN";
}

const char *rocket_last_error(const rocket_ctx *ctx) { return ctx ? ctx->last_error.c_str() : g_null_error.c_str(); }

rocket_status rocket_create(rocket_ctx **out, int device)
{
    if (!out) return rk::fail(nullptr, ROCKET_E_INVALID, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return rk::hip_fail(nullptr, e, "hipGetDeviceCount", __FILE__, __LINE__);
    if (device < 0 || device >= count) return rk::fail(nullptr, ROCKET_E_INVALID, "device out of range");
    rocket_ctx *c = new rocket_ctx();
    c->device = device;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        delete c;
        return rk::hip_fail(nullptr, e, "hipGetDeviceProperties", __FILE__, __LINE__);
    }
    c->num_cu = prop.multiProcessorCount;
    *out = c;
    return ROCKET_OK;
}

void rocket_destroy(rocket_ctx *ctx)
{
    if (!ctx) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &b : ctx->ws)
        if (b.ptr && !ctx->arena) (void)hipFree(b.ptr);
    if (ctx->ev_begin) (void)hipEventDestroy(ctx->ev_begin);
    if (ctx->ev_end) (void)hipEventDestroy(ctx->ev_end);
    rk::OocState &oc = ctx->ooc;
    if (oc.copy) (void)hipStreamDestroy(oc.copy);
    if (oc.start) (void)hipEventDestroy(oc.start);
    for (int k = 0; k < 2; ++k) {
        if (oc.copied[k]) (void)hipEventDestroy(oc.copied[k]);
        if (oc.freed[k]) (void)hipEventDestroy(oc.freed[k]);
    }
    rk::PceState &pc = ctx->pce;
    if (pc.side) (void)hipStreamDestroy(pc.side);
    for (hipEvent_t e : {pc.fork, pc.join, pc.staged[0], pc.staged[1], pc.consumed[0], pc.consumed[1]})
        if (e) (void)hipEventDestroy(e);
    (void)hipSetDevice(prev);
    delete ctx;
}

static rocket_status enter(rocket_ctx *ctx)
{
    if (!ctx) return rk::fail(nullptr, ROCKET_E_INVALID, "ctx is NULL");
    int cur = -1;
    RK_HIP(hipGetDevice(&cur));
    if (cur != ctx->device) RK_HIP(hipSetDevice(ctx->device));
    return ROCKET_OK;
}

rocket_status rocket_prepare(rocket_ctx *ctx, const rocket_items *items, int64_t n, rocket_pair_fn fn, void *stream)
{
    RK_TRY(enter(ctx));
    if (!items) return rk::fail(ctx, ROCKET_E_INVALID, "items is NULL");
    if (n < 0) return rk::fail(ctx, ROCKET_E_INVALID, "n < 0");
    if (!valid_fn(fn)) return rk::fail(ctx, ROCKET_E_UNSUPPORTED, "unknown pair function");
    hipStream_t s = (hipStream_t)stream;
    ctx->prepared_fn = 0;
    ctx->ovl.grad_ready = false;
    ctx->stats.cache_slots = 0;
    ctx->stats.cache_loads = 0;
    rocket_status st;
    switch (fn) {
    case ROCKET_NCC_FP32:
    case ROCKET_NCC_BF16X3:
    case ROCKET_NCC_BF16X6: st = rk::ncc_prepare(ctx, items, n, (int)fn, s); break;
    case ROCKET_GAUSS_OVERLAP: st = rk::ovl_prepare(ctx, items, n, 0, s); break;
    case ROCKET_GMM_L2: st = rk::ovl_prepare(ctx, items, n, items->point_cov ? rk::OVL_FULL_L2 : rk::OVL_GMM_L2, s); break;
    case ROCKET_GMM_BHATTACHARYA:
        st = rk::ovl_prepare(ctx, items, n, items->point_cov ? rk::OVL_FULL_BH : rk::OVL_GMM_BH, s);
        break;
    case ROCKET_SPARSE_COSINE: st = rk::sp_prepare(ctx, items, n, s); break;
    case ROCKET_PCE: st = rk::pce_prepare(ctx, items, n, s); break;
    default: st = ROCKET_E_UNSUPPORTED;
    }
    if (st == ROCKET_OK) ctx->prepared_fn = (int)fn;
    ctx->stats.n = n;
    ctx->stats.pairs = n * (n - 1) / 2;
    if (st == ROCKET_OK && ctx->opt[ROCKET_OPT_AUTOTUNE]) st = rk::autotune(ctx, s);
    ctx->stats.workspace_bytes = rk::ws_total(ctx);
    return st;
}

rocket_status rocket_compare(rocket_ctx *ctx, float *out, uint32_t *out_counts, void *stream)
{
    RK_TRY(enter(ctx));
    hipStream_t s = (hipStream_t)stream;
    const int fn = ctx->prepared_fn;
    if (!fn) return rk::fail(ctx, ROCKET_E_STATE, "compare without a successful prepare");
    if (!out && ctx->stats.pairs > 0) return rk::fail(ctx, ROCKET_E_INVALID, "out is NULL");
    rocket_status st;
    switch (fn) {
    case ROCKET_NCC_FP32:
    case ROCKET_NCC_BF16X3:
    case ROCKET_NCC_BF16X6: st = rk::ncc_compare(ctx, out, s); break;
    case ROCKET_GAUSS_OVERLAP:
    case ROCKET_GMM_L2:
    case ROCKET_GMM_BHATTACHARYA: st = rk::ovl_compare(ctx, out, nullptr, nullptr, nullptr, s); break;
    case ROCKET_SPARSE_COSINE: st = rk::sp_compare(ctx, out, out_counts, s); break;
    case ROCKET_PCE: st = rk::pce_compare(ctx, out, out_counts, s); break;
    default: st = ROCKET_E_STATE;
    }
    ctx->stats.workspace_bytes = rk::ws_total(ctx);
    return st;
}

rocket_status rocket_allpairs_ex(rocket_ctx *ctx, const rocket_items *items, int64_t n, rocket_pair_fn fn, float *out,
                                 uint32_t *out_counts, void *stream)
{
    RK_TRY(rocket_prepare(ctx, items, n, fn, stream));
    return rocket_compare(ctx, out, out_counts, stream);
}

rocket_status rocket_allpairs(const rocket_items *items, int64_t n, rocket_pair_fn fn, float *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return rk::hip_fail(nullptr, e, "hipGetDevice", __FILE__, __LINE__);
    if (dev < 0 || dev >= 64) return rk::fail(nullptr, ROCKET_E_INVALID, "device index out of range");
    rocket_ctx *ctx;
    {
        std::lock_guard<std::mutex> lk(g_default_mu);
        if (!g_default[dev]) {
            rocket_status st = rocket_create(&g_default[dev], dev);
            if (st != ROCKET_OK) return st;
        }
        ctx = g_default[dev];
    }
    RK_TRY(rocket_allpairs_ex(ctx, items, n, fn, out, nullptr, nullptr));
    RK_HIP(hipStreamSynchronize(nullptr));
    return ROCKET_OK;
}

rocket_status rocket_allpairs_host(rocket_ctx *ctx, const float *host_items, int64_t n, int64_t dim, int64_t ld,
                                   rocket_pair_fn fn, float *out, void *stream)
{
    RK_TRY(enter(ctx));
    if (fn != ROCKET_NCC_FP32 && fn != ROCKET_NCC_BF16X3 && fn != ROCKET_NCC_BF16X6)
        return rk::fail(ctx, ROCKET_E_UNSUPPORTED, "host-resident items: NCC pair functions only");
    ctx->prepared_fn = 0;  // the plane workspace is reused as the device cache
    ctx->trace_valid = false;
    ctx->ovl.grad_ready = false;
    rocket_status st = rk::ncc_allpairs_host(ctx, host_items, n, dim, ld, (int)fn, out, (hipStream_t)stream);
    ctx->stats.n = n;
    ctx->stats.pairs = n > 1 ? n * (n - 1) / 2 : 0;
    ctx->stats.workspace_bytes = rk::ws_total(ctx);
    return st;
}

rocket_status rocket_cv_build(rocket_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n, int K,
                              int64_t *cv_offsets, int64_t *keys, float *vals, int64_t capacity, void *stream)
{
    RK_TRY(enter(ctx));
    rocket_status st = rk::cv_build(ctx, residues, offsets, n, K, cv_offsets, keys, vals, capacity, (hipStream_t)stream);
    ctx->stats.workspace_bytes = rk::ws_total(ctx);
    return st;
}

rocket_status rocket_overlap_cost_grad(rocket_ctx *ctx, const rocket_items *clouds, int64_t n, const float *centroids,
                                       const float *params, float *out_cost, float *out_grad, void *stream)
{
    RK_TRY(enter(ctx));
    if (n < 0) return rk::fail(ctx, ROCKET_E_INVALID, "n < 0");
    const int64_t P = n * (n - 1) / 2;
    if (P > 0 && (!centroids || !params || !out_cost))
        return rk::fail(ctx, ROCKET_E_INVALID, "centroids, params and out_cost are required");
    hipStream_t s = (hipStream_t)stream;
    rk::OvlState &o = ctx->ovl;
    if (clouds) {
        ctx->prepared_fn = 0;
        RK_TRY(rk::ovl_prepare(ctx, clouds, n, 0, s));
        ctx->prepared_fn = ROCKET_GAUSS_OVERLAP;
        o.grad_ready = true;
    } else if (!(o.valid && o.grad_ready && o.mode == 0 && o.n == n)) {
        return rk::fail(ctx, ROCKET_E_STATE, "clouds is NULL but no clouds of this size were prepared by the previous "
                                             "rocket_overlap_cost_grad");
    }
    ctx->stats.n = n;
    ctx->stats.pairs = P;
    RK_TRY(rk::ovl_compare(ctx, out_cost, centroids, params, out_grad, s));
    ctx->stats.workspace_bytes = rk::ws_total(ctx);
    return ROCKET_OK;
}

rocket_status rocket_cost_grad(rocket_ctx *ctx, const rocket_items *items, int64_t n, rocket_pair_fn fn,
                               const float *centroids, const float *params, float *out_cost, float *out_grad,
                               void *stream)
{
    if (fn == ROCKET_GAUSS_OVERLAP)
        return rocket_overlap_cost_grad(ctx, items, n, centroids, params, out_cost, out_grad, stream);
    RK_TRY(enter(ctx));
    if (fn != ROCKET_GMM_L2 && fn != ROCKET_GMM_BHATTACHARYA)
        return rk::fail(ctx, ROCKET_E_UNSUPPORTED, "cost gradients exist for the three particle scores only");
    if (n < 0) return rk::fail(ctx, ROCKET_E_INVALID, "n < 0");
    const int64_t P = n * (n - 1) / 2;
    if (P > 0 && (!centroids || !params || !out_cost))
        return rk::fail(ctx, ROCKET_E_INVALID, "centroids, params and out_cost are required");
    hipStream_t s = (hipStream_t)stream;
    // full covariances, or the per-point-sigma kernel (isotropic points rotate onto themselves);
    // with items = NULL the previous preparation's kind is kept
    const bool full = items ? items->point_cov != nullptr : (ctx->ovl.mode == rk::OVL_FULL_L2 || ctx->ovl.mode == rk::OVL_FULL_BH);
    const int mode = fn == ROCKET_GMM_L2 ? (full ? rk::OVL_FULL_L2 : rk::OVL_GMM_L2)
                                         : (full ? rk::OVL_FULL_BH : rk::OVL_GMM_BH);
    rk::OvlState &o = ctx->ovl;
    if (items) {
        ctx->prepared_fn = 0;
        RK_TRY(rk::ovl_prepare(ctx, items, n, mode, s));
        ctx->prepared_fn = (int)fn;
        o.grad_ready = true;
    } else if (!(o.valid && o.grad_ready && o.mode == mode && o.n == n)) {
        return rk::fail(ctx, ROCKET_E_STATE, "items is NULL but no clouds of this size were prepared for this score "
                                             "by the previous rocket_cost_grad");
    }
    ctx->stats.n = n;
    ctx->stats.pairs = P;
    RK_TRY(rk::ovl_compare(ctx, out_cost, centroids, params, out_grad, s));
    ctx->stats.workspace_bytes = rk::ws_total(ctx);
    return ROCKET_OK;
}

rocket_status rocket_set_option(rocket_ctx *ctx, rocket_option opt, int64_t value)
{
    if (!ctx) return rk::fail(nullptr, ROCKET_E_INVALID, "ctx is NULL");
    if (opt < ROCKET_OPT_NCC_TILE || opt > ROCKET_OPT_TRACE) return rk::fail(ctx, ROCKET_E_UNSUPPORTED, "option");
    if (value < 0) return rk::fail(ctx, ROCKET_E_INVALID, "negative option value");
    if (opt == ROCKET_OPT_NCC_TILE && value != 0 && value != 64 && value != 128 && value != 256)
        return rk::fail(ctx, ROCKET_E_INVALID, "NCC tile must be 0, 64, 128 or 256");
    if (opt == ROCKET_OPT_NCC_KCHUNK && value % 16 != 0)
        return rk::fail(ctx, ROCKET_E_INVALID, "NCC K chunk must be a multiple of 16");
    if (opt == ROCKET_OPT_QUEUE_ORDER && value > 2) return rk::fail(ctx, ROCKET_E_INVALID, "queue order 0..2");
    if (opt == ROCKET_OPT_NCC_WAVES && value != 0 && value != 4 && value != 8)
        return rk::fail(ctx, ROCKET_E_INVALID, "NCC waves must be 0, 4 or 8");
    if (opt == ROCKET_OPT_OVL_VARIANT && value > 4) return rk::fail(ctx, ROCKET_E_INVALID, "overlap variant 0..4");
    if (opt == ROCKET_OPT_OVL_BLOCK && value > 64) return rk::fail(ctx, ROCKET_E_INVALID, "overlap block <= 64");
    if (opt == ROCKET_OPT_SP_LANES && value != 0 && value != 4 && value != 8)
        return rk::fail(ctx, ROCKET_E_INVALID, "sparse lanes per column must be 0, 4 or 8");
    if (opt == ROCKET_OPT_SP_CHUNK && ((value & (value - 1)) != 0 || value > ((int64_t)1 << 31)))
        return rk::fail(ctx, ROCKET_E_INVALID, "sparse chunk width must be 0 or a power of two up to 2^31");
    ctx->opt[opt] = value;
    return ROCKET_OK;
}

rocket_status rocket_get_option(const rocket_ctx *ctx, rocket_option opt, int64_t *value)
{
    if (!ctx || !value) return rk::fail(nullptr, ROCKET_E_INVALID, "NULL argument");
    if (opt < ROCKET_OPT_NCC_TILE || opt > ROCKET_OPT_TRACE) return ROCKET_E_UNSUPPORTED;
    *value = ctx->opt[opt];
    return ROCKET_OK;
}

rocket_status rocket_get_stats(const rocket_ctx *ctx, rocket_stats *out)
{
    if (!ctx || !out) return rk::fail(nullptr, ROCKET_E_INVALID, "NULL argument");
    *out = ctx->stats;
    out->kernel_ns = -1;
    if (ctx->ev_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(ctx->ev_end) == hipSuccess && hipEventElapsedTime(&ms, ctx->ev_begin, ctx->ev_end) == hipSuccess)
            out->kernel_ns = (int64_t)((double)ms * 1e6);
        else
            (void)hipGetLastError();
    }
    return ROCKET_OK;
}

rocket_status rocket_get_trace(rocket_ctx *ctx, rocket_trace_rec *out, int64_t cap, int64_t *count)
{
    if (!ctx || !count) return rk::fail(ctx, ROCKET_E_INVALID, "NULL argument");
    if (!ctx->opt[ROCKET_OPT_TRACE] || !ctx->trace_valid || !ctx->ws[rk::WS_TRACE].ptr ||
        !ctx->ws[rk::WS_QUEUE_ITEMS].ptr)
        return rk::fail(ctx, ROCKET_E_STATE, "no per-tile trace: set ROCKET_OPT_TRACE before a prepare whose compare "
                                             "runs a persistent queue");
    *count = ctx->ledger_items;
    if (!out || cap <= 0) return ROCKET_OK;
    const int64_t m = std::min(cap, ctx->ledger_items);
    if (m == 0) return ROCKET_OK;
    std::vector<unsigned long long> tr((size_t)(3 * m));
    std::vector<int4> items((size_t)m);
    RK_HIP(hipSetDevice(ctx->device));
    RK_HIP(hipDeviceSynchronize());
    RK_HIP(hipMemcpy(tr.data(), ctx->ws[rk::WS_TRACE].ptr, sizeof(unsigned long long) * tr.size(), hipMemcpyDeviceToHost));
    RK_HIP(hipMemcpy(items.data(), ctx->ws[rk::WS_QUEUE_ITEMS].ptr, sizeof(int4) * items.size(), hipMemcpyDeviceToHost));
    int khz = 0;
    RK_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device));
    if (khz <= 0) return rk::fail(ctx, ROCKET_E_HIP, "device wall clock rate unknown");
    unsigned long long t0 = ~0ull;
    for (int64_t k = 0; k < m; ++k)
        if (tr[3 * k] != 0) t0 = std::min(t0, tr[3 * k]);
    const double ns_per_tick = 1e6 / (double)khz;
    for (int64_t k = 0; k < m; ++k) {
        rocket_trace_rec &r = out[k];
        r.tile_i = items[k].x;
        r.tile_j = items[k].y;
        r.chunk = items[k].z;
        const bool ran = tr[3 * k] != 0;
        r.workgroup = ran ? (int32_t)tr[3 * k + 2] : -1;
        r.start_ns = ran ? (int64_t)((double)(tr[3 * k] - t0) * ns_per_tick) : -1;
        r.end_ns = ran && tr[3 * k + 1] >= tr[3 * k] ? (int64_t)((double)(tr[3 * k + 1] - t0) * ns_per_tick) : -1;
    }
    return ROCKET_OK;
}

rocket_status rocket_get_ledger(rocket_ctx *ctx, int32_t *out, int64_t cap, int64_t *count)
{
    RK_TRY(enter(ctx));
    if (!count) return rk::fail(ctx, ROCKET_E_INVALID, "count is NULL");
    *count = ctx->ledger_items;
    if (!ctx->opt[ROCKET_OPT_LEDGER] || !ctx->ws[rk::WS_LEDGER].ptr)
        return rk::fail(ctx, ROCKET_E_STATE, "ledger not enabled for the last compare");
    const int64_t m = std::min(cap, ctx->ledger_items);
    RK_HIP(hipDeviceSynchronize());
    if (m > 0) RK_HIP(hipMemcpy(out, ctx->ws[rk::WS_LEDGER].ptr, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
    return ROCKET_OK;
}

rocket_status rocket_autotune(rocket_ctx *ctx, void *stream)
{
    RK_TRY(enter(ctx));
    rocket_status st = rk::autotune(ctx, (hipStream_t)stream);
    ctx->stats.workspace_bytes = rk::ws_total(ctx);
    return st;
}

}  // extern "C"
