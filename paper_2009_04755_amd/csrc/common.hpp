// Internal declarations shared by the host library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rocket.h"

namespace rk {

// Named workspace slots owned by a context.
enum Slot {
    WS_QUEUE_ITEMS = 0,  // int4 work items
    WS_QUEUE_HEADS,      // per-segment pop counters
    WS_QUEUE_SEGS,       // segment boundaries
    WS_LEDGER,           // per-item pop counts (debug)
    WS_TRACE,            // per-item start, end and workgroup (ROCKET_OPT_TRACE)
    WS_FLAGS,            // device error flags
    WS_NCC_STATS,        // mean (f64), inverse norm (f32)
    WS_NCC_PLANES,       // split / centred operand planes
    WS_NCC_PARTIAL,      // split-K partial Gram tiles
    WS_NCC_TILES,        // tile list (bi, bj) for the epilogue
    WS_OOC_STAGE,        // two raw staging buffers for host-resident items
    WS_OVL_PACK,         // size-sorted packed clouds
    WS_OVL_META,         // per sorted cloud: offset, count, original index
    WS_OVL_SIG,          // packed scaled per-point deviations (GMM scores)
    WS_SP_KEYS,          // packed u32 keys
    WS_SP_META,          // flags, inverse norms, sorted order
    WS_SP_CHUNKS,        // band histogram over key micro-chunks + chunk counts
    WS_SP_CSHIFT,        // per band start of its chunk boundaries
    WS_SP_BOUNDS,        // chunk boundaries (units of 2^ulog keys)
    WS_SP_FINE,          // 64-key counts of micro-chunks that overflow a band's chunk
    WS_PCE_SPEC,         // PCE item spectra (complex f32, natural order)
    WS_PCE_STAGE,        // PCE staged transforms of one batch of pair-pairs (large images)
    WS_CV_K,             // dense K-string counts of a group of species (kept zeroed between calls)
    WS_CV_AUX,           // (K-1)- and (K-2)-string counts, chunk occupancy, totals
    WS_COUNT
};

struct Buffer {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// Work queue description handed to persistent kernels.
struct QueueArgs {
    const int4 *items;  // work items, grouped by segment
    int *heads;         // one counter per segment, HEAD_STRIDE ints apart
    const int *seg;     // nseg + 1 segment boundaries into items
    int *ledger;        // optional per-item pop counter
    int nseg;
    // optional per-item trace: start and end on the device wall clock, and the workgroup
    unsigned long long *trace = nullptr;
};
constexpr int HEAD_STRIDE = 32;  // 128 bytes between segment counters
constexpr int MAX_SEG = 8;       // one segment per XCD
enum { QOWN_NONE = 0, QOWN_NCC, QOWN_OVL, QOWN_SP, QOWN_PCE };

struct NccState {
    int64_t n = 0, dim = 0, ld = 0, n_pad = 0, d_pad = 0;
    int tile = 0, nkt = 0, kt_per_chunk = 0, nchunks = 0, waves = 4;
    int64_t tiles = 0, items = 0;
    const float *src = nullptr;
    int scheme = 0;
    // plan cache: the uploaded queue matches these parameters (unless a batched compare
    // has since replaced it with per-batch queues)
    QueueArgs qa{};
    bool queue_batched = false;
    int64_t pc_n = -1, pc_tile = -1, pc_nchunks = -1, pc_order = -1, pc_seed = -1, pc_ledger = -1;
    std::vector<int2> h_tiles;
};

// Cloud score modes: fixed-sigma overlap, per-point-sigma GMM L2 / Bhattacharya, and the
// same two scores for points with a full covariance (also the adjoint path of both).
enum { OVL_OVERLAP = 0, OVL_GMM_L2 = 1, OVL_GMM_BH = 2, OVL_FULL_L2 = 3, OVL_FULL_BH = 4 };

struct OvlState {
    int64_t n = 0, total = 0;
    const int64_t *offsets = nullptr;
    const float *xy = nullptr;
    double sigma = 0;
    int mode = 0;  // OVL_*
    int block = 0;
    int64_t tiles = 0, max_block_pts = 0;
    std::vector<int64_t> h_offsets;  // host copy of offsets
    std::vector<int> perm;           // sorted position -> original cloud
    QueueArgs qa{};
    int64_t pc_block = -1, pc_order = -1, pc_seed = -1, pc_ledger = -1;
    bool valid = false;
    bool grad_ready = false;  // prepared by rocket_overlap_cost_grad (reusable with clouds = NULL)
};

struct SpState {
    int64_t n = 0, total = 0;
    const int64_t *offsets = nullptr;
    const int64_t *keys = nullptr;
    const float *vals = nullptr;
    int wlog = 0, ulog = 0, lpc = 8;
    int64_t tiles = 0, nchunks_total = 0;
    std::vector<int64_t> h_offsets;
    std::vector<int> perm;
    const int64_t *cshift = nullptr;
    const int *bounds = nullptr;
    const float *inv_norm = nullptr;
    const int *dperm = nullptr;
    const uint32_t *k32 = nullptr;
    QueueArgs qa{};
    bool valid = false;
};

struct PceState {
    int64_t n = 0, tiles = 0;
    int L = 0;
    QueueArgs qa{};
    bool valid = false;
    bool big = false;  // H x W items through the staged multi-pass path
    int H = 0, W = 0;
    std::vector<int4> h_pp;  // pair-pairs (i, j, k, l) in tile order (staged path)
    // staged path, two staging buffers: the row pass of batch k + 1 (caller's stream) runs
    // while the column pass of batch k runs on `side`
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipEvent_t staged[2] = {nullptr, nullptr};    // row pass done: buffer k holds a batch
    hipEvent_t consumed[2] = {nullptr, nullptr};  // column/peak/PCE kernels done with buffer k
};

// Composition-vector builder: whether the dense K-string count array is all zeros.
struct CvState {
    bool clean = false;
    int K = 0;
    int64_t G = 0;
};

// Out-of-core state: copy stream and the events that order it against the compute stream.
struct OocState {
    hipStream_t copy = nullptr;
    hipEvent_t start = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr};  // raw block k landed in staging buffer k
    hipEvent_t freed[2] = {nullptr, nullptr};   // staging buffer k consumed by the split
};

}  // namespace rk

struct rocket_ctx {
    int device = 0;
    int num_cu = 256;
    int64_t opt[32] = {0};  // indexed by rocket_option
    rk::Buffer ws[rk::WS_COUNT];
    int prepared_fn = 0;
    int queue_owner = 0;  // which pair function's plan the device queue holds
    rk::NccState ncc;
    rk::OvlState ovl;
    rk::SpState sp;
    rk::OocState ooc;
    rk::CvState cv;
    rk::PceState pce;
    rocket_stats stats = {};
    int64_t ledger_items = 0;
    bool trace_valid = false;  // the trace slot holds the last compare's per-item records
    hipEvent_t ev_begin = nullptr, ev_end = nullptr;  // main-kernel timing (ROCKET_OPT_TIMING)
    bool ev_pending = false;
    std::string last_error;
    // host staging for queue uploads (kept to avoid re-allocation)
    std::vector<int4> h_items;
    std::vector<int> h_seg;
    // Arena mode (allocation-free entry point): when `arena` is set, workspace slots are
    // carved from [arena, arena + arena_cap) in call order instead of being allocated.
    char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    std::string tune_cache;  // autotuner cache file (empty: no cache)
};

namespace rk {

// Queue instrumentation in effect (ledger bit 0, trace bit 1): part of the key under which
// an uploaded queue is reused.
inline int64_t queue_flags(const rocket_ctx *ctx)
{
    return (ctx->opt[ROCKET_OPT_LEDGER] != 0 ? 1 : 0) | (ctx->opt[ROCKET_OPT_TRACE] != 0 ? 2 : 0);
}

rocket_status fail(rocket_ctx *ctx, rocket_status st, const std::string &msg);
rocket_status hip_fail(rocket_ctx *ctx, hipError_t e, const char *what, const char *file, int line);
rocket_status ws_get(rocket_ctx *ctx, Slot slot, size_t bytes, void **out);
int64_t ws_total(const rocket_ctx *ctx);
rocket_status upload_queue(rocket_ctx *ctx, hipStream_t s, QueueArgs *qa);
rocket_status reset_queue(rocket_ctx *ctx, hipStream_t s, const QueueArgs &qa);
int auto_grid(rocket_ctx *ctx, const void *kernel, int block, size_t dyn_lds, int64_t items);
// Bracket the main kernel launch with events when ROCKET_OPT_TIMING is set.
rocket_status timing_begin(rocket_ctx *ctx, hipStream_t s);
rocket_status timing_end(rocket_ctx *ctx, hipStream_t s);

// Planner (plan.cpp)
void plan_leaves(int64_t n, int64_t T, std::vector<int2> &out);
// Split `tiles` x `chunks` work items into per-XCD segments in chunk-major order.
void plan_chunked(const std::vector<int2> &tiles, int nchunks, int nseg, std::vector<int4> &items,
                  std::vector<int> &seg, int halves = 1);
// Cost-ordered (largest first) items dealt round-robin to segments.
void plan_lpt(const std::vector<int4> &items_in, const std::vector<double> &cost, int nseg,
              std::vector<int4> &items, std::vector<int> &seg);
void shuffle_items(std::vector<int4> &items, std::vector<int> &seg, uint64_t seed);
void single_segment(std::vector<int> &seg, int64_t nitems);

// Per pair-function modules.
rocket_status ncc_prepare(rocket_ctx *ctx, const rocket_items *it, int64_t n, int scheme, hipStream_t s);
rocket_status ncc_compare(rocket_ctx *ctx, float *out, hipStream_t s);
rocket_status ncc_allpairs_host(rocket_ctx *ctx, const float *host, int64_t n, int64_t dim, int64_t ld, int scheme,
                                float *out, hipStream_t s);
rocket_status ovl_prepare(rocket_ctx *ctx, const rocket_items *it, int64_t n, int mode, hipStream_t s);
rocket_status ovl_compare(rocket_ctx *ctx, float *out, const float *centroids, const float *params, float *grad,
                          hipStream_t s);
rocket_status ovl_autotune(rocket_ctx *ctx, hipStream_t s);
rocket_status ovl_replan_public(rocket_ctx *ctx, hipStream_t s);  // rebuild the cloud queue for the current options
// Autotuner for the prepared set (tune.cpp): cached or timed choice of the tile shape.
rocket_status autotune(rocket_ctx *ctx, hipStream_t s);
rocket_status sp_prepare(rocket_ctx *ctx, const rocket_items *it, int64_t n, hipStream_t s);
rocket_status sp_compare(rocket_ctx *ctx, float *out, uint32_t *counts, hipStream_t s);
rocket_status pce_prepare(rocket_ctx *ctx, const rocket_items *it, int64_t n, hipStream_t s);
rocket_status pce_compare(rocket_ctx *ctx, float *out, uint32_t *peak, hipStream_t s);
bool pce_big_shape(int64_t H, int64_t W);
rocket_status pce_big_prepare(rocket_ctx *ctx, const rocket_items *it, int64_t n, int H, int W, hipStream_t s);
rocket_status pce_big_compare(rocket_ctx *ctx, float *out, uint32_t *peak, int h, hipStream_t s);
rocket_status cv_build(rocket_ctx *ctx, const uint8_t *res, const int64_t *offsets, int64_t n, int K,
                       int64_t *cv_off, int64_t *keys, float *vals, int64_t capacity, hipStream_t s);

}  // namespace rk

#define RK_HIP(expr)                                                                  \
    do {                                                                              \
        hipError_t rk_e_ = (expr);                                                    \
        if (rk_e_ != hipSuccess) return rk::hip_fail(ctx, rk_e_, #expr, __FILE__, __LINE__); \
    } while (0)

#define RK_TRY(expr)                         \
    do {                                     \
        rocket_status rk_s_ = (expr);        \
        if (rk_s_ != ROCKET_OK) return rk_s_; \
    } while (0)
