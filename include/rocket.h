/*
 * rocket.h -- C ABI of the MI355X (gfx950) all-pairs library.
 *
 * The all-pairs problem (Section III of Heldens et al., "Rocket: Efficient and
 * Scalable All-Pairs Computations on Heterogeneous Platforms", arXiv 2009.04755):
 * for n items and a pair function f, compute f(l(i), l(j)) for every pair
 * 1 <= i < j <= n, where l(i) loads and pre-processes item i.  The paper splits l
 * into load / parse / host-to-device / GPU pre-process and f into GPU compare /
 * device-to-host / post-process (Section III, Fig. "pipeline").  This library is
 * the GPU part of that pipeline for one device:
 *
 *   rocket_prepare   the GPU pre-process stage of l for all n items at once;
 *   rocket_compare   the GPU compare stage of f for all n(n-1)/2 pairs, as one
 *                    persistent launch that pulls tiles of the pair matrix from an
 *                    on-device queue (Section IV-B's divide-and-conquer split and
 *                    work stealing, mapped onto the chip);
 *   rocket_allpairs  both, back to back;
 *   rocket_allpairs_host  the same for NCC items that stay in host memory and
 *                    pass through a fixed-size device cache (Section IV-A);
 *   rocket_cv_build  the GPU pre-process of the sparse application: protein
 *                    sequences to composition vectors (Section V-B).
 *
 * Three pair functions are provided, one per application of Section V:
 *   ROCKET_NCC_*          normalised cross-correlation of dense vectors (V-A);
 *   ROCKET_GAUSS_OVERLAP  Gaussian-mixture overlap of 2-D point clouds (V-C);
 *   ROCKET_SPARSE_COSINE  cosine of sparse key/value vectors plus the exact size
 *                         of the key intersection (V-B);
 *   ROCKET_GMM_L2, ROCKET_GMM_BHATTACHARYA  the two particle scores of V-C for
 *                         clouds whose points carry their own uncertainty;
 *   ROCKET_PCE            peak-to-correlation energy over all shifts (V-A variant);
 * and rocket_overlap_cost_grad gives the overlap cost's gradient with respect to a
 * rigid transform per pair (the registration optimiser of V-C).
 *
 * OUTPUT LAYOUT.  Results are written in the caller's item order as the packed
 * strict upper triangle, row-major: pair (i, j), i < j, lands at
 *     idx(i, j) = i*n - i*(i+1)/2 + (j - i - 1),   0 <= idx < P = n(n-1)/2.
 *
 * POINTERS AND OWNERSHIP.  Unless a comment says "host", every pointer is a DEVICE
 * pointer on the context's device.  The caller allocates and owns every input and
 * output; the library reads inputs and writes outputs only inside the work it
 * enqueues on the given stream and keeps no reference after that work completes
 * (rocket_compare re-reads the items passed to the last rocket_prepare, so they
 * must stay alive and unchanged until compare's work is done).  The context owns
 * its workspace (prepared item copies, split-K partials, work queue), grows it
 * with hipMalloc on demand and frees it in rocket_destroy.
 *
 * STREAMS.  `stream` is a hipStream_t passed as void* (NULL = the null stream).
 * Every call is stream-ordered; calls return once the work is enqueued, except
 * where a comment says the call synchronises.  A context must not be used from
 * two host threads at once; calls on one context must not overlap on the device
 * with different streams.  The staged PCE compare also runs kernels on a stream of
 * its own (created by rocket_prepare), forked from and joined back to `stream` with
 * events, so the call stays ordered on `stream` as a whole.
 *
 * ERRORS.  Every entry point returns a rocket_status.  Argument checks (null
 * pointers, negative sizes, ld < dim, unknown function) happen before anything is
 * enqueued.  Data checks that need the data (ragged offsets, sparse key order and
 * range) run on the device in rocket_prepare, which then synchronises once to read
 * the result.  After a failure the context stays usable; rocket_last_error
 * returns a message describing the most recent failure.
 */
#ifndef ROCKET_H
#define ROCKET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ROCKET_OK = 0,
    ROCKET_E_INVALID = -1,     /* bad argument: null pointer, negative size, ld < dim, bad offsets */
    ROCKET_E_UNSUPPORTED = -2, /* unknown pair function or option */
    ROCKET_E_OOM = -3,         /* workspace allocation failed (or exceeds ROCKET_OPT_WORKSPACE_CAP) */
    ROCKET_E_HIP = -4,         /* a HIP runtime call failed; see rocket_last_error */
    ROCKET_E_KEYRANGE = -5,    /* sparse key outside [0, 2^32 - 1) */
    ROCKET_E_UNSORTED = -6,    /* sparse keys of an item not strictly ascending */
    ROCKET_E_STATE = -7        /* rocket_compare without a matching rocket_prepare */
} rocket_status;

typedef enum {
    /* NCC (Section V-A): rho_ij = <a_i - mean a_i, a_j - mean a_j> / (|a_i - mean a_i| |a_j - mean a_j|).
     * Per-item mean and centred norm are reduced in FP64; the centred items are
     * compared as a Gram matrix on the matrix cores with FP32 accumulation:
     *   FP32   FP32 operands (v_mfma_f32_32x32x2_f32);
     *   BF16X3 each centred value x split into bf16 h + m (x ~ h + m), products
     *          h*h + h*m + m*h (bf16 MFMA);
     *   BF16X6 three-way split h + m + l, products h*h + h*m + m*h + h*l + l*h + m*m.
     * The Gram entry is rescaled by 1/(s_i s_j) in FP32.  A zero-variance item
     * gives NaN in all its pairs. */
    ROCKET_NCC_FP32 = 1,
    ROCKET_NCC_BF16X3 = 2,
    ROCKET_NCC_BF16X6 = 3,
    /* Gaussian overlap (Section V-C): C_ij = sum_k sum_l exp(-|x_k - y_l|^2 / (4 sigma^2)),
     * x the points of cloud i, y those of cloud j.  FP32 arithmetic, per-lane
     * partial sums reduced by a fixed wavefront tree.  An empty cloud gives 0. */
    ROCKET_GAUSS_OVERLAP = 4,
    /* Sparse cosine (Section V-B): cos_ij = sum_{k in K_i & K_j} v_ik v_jk / (|v_i| |v_j|),
     * norms over all entries of an item (FP64 reduction).  out_counts, when given,
     * receives |K_i & K_j| exactly.  A zero-norm item gives NaN; m_ij = 0 gives 0. */
    ROCKET_SPARSE_COSINE = 5,
    /* Per-localisation-uncertainty scores (Section V-C names the GMM L2 distance and the
     * Bhattacharya distance between particles).  Point k of cloud i is the isotropic
     * Gaussian N(x_k, s_k^2 I), point l of cloud j is N(y_l, t_l^2 I); v = s_k^2 + t_l^2,
     * D = |x_k - y_l|^2.
     *   GMM_L2:            sum_kl exp(-D / (2 v)) / (2 pi v), the cross term
     *                      integral of f_i f_j of the L2 distance between the mixtures;
     *   GMM_BHATTACHARYA:  sum_kl (2 s_k t_l / v) exp(-D / (4 v)), the sum of the
     *                      components' Bhattacharya coefficients.
     * FP32 with one reciprocal and one exp2 per term.  Deviations come from
     * point_sigma and must lie in [1e-18, 1e18] (checked in rocket_prepare, else
     * ROCKET_E_INVALID); the scalar sigma is ignored.  An empty cloud gives 0.
     * With point_cov set, every point carries a full covariance (S_k for cloud i, T_l for
     * cloud j; V = S_k + T_l, d = x_k - y_l) and the terms are the same integrals:
     *   GMM_L2:            exp(-d^T V^-1 d / 2) / (2 pi sqrt(det V)),
     *   GMM_BHATTACHARYA:  2 (det S_k det T_l)^(1/4) / sqrt(det V) exp(-d^T V^-1 d / 4);
     * one reciprocal square root and one exp2 per term.  Each covariance must be symmetric
     * positive definite with diagonal entries and determinant in [1e-36, 1e36] (checked in
     * rocket_prepare, else ROCKET_E_INVALID). */
    ROCKET_GMM_L2 = 6,
    ROCKET_GMM_BHATTACHARYA = 7,
    /* Peak-to-correlation energy over all cyclic shifts (the PCE variant of the forensics
     * comparison, Section V-A).  Items are H x W images flattened row-major (dense,
     * dim = H*W, ld >= dim), W = ROCKET_OPT_PCE_WIDTH (square if 0).  With a, b the two
     * items minus their means,
     *   C(s) = sum_x a(x + s) b(x)  (row index mod H, column index mod W),  s* = argmax C
     *   (smallest shift index r*W + c on ties),  PCE = C(s*)^2 (H W - |N|) / sum_{s outside N} C(s)^2,
     * N the (2h+1) x (2h+1) cyclic neighbourhood of s*, h = ROCKET_OPT_PCE_RADIUS (5 if 0),
     * h < min(H, W)/2.  Square items with L = 32, 64 or 128 run one f32 2-D FFT per pair
     * inside LDS; otherwise H and W must be in [16, 4096] (else
     * ROCKET_E_UNSUPPORTED) and the pair transforms are staged in HBM: two pairs per
     * complex 2-D FFT, a row pass, a column pass and a peak/energy pass over batches of
     * pair-pairs (ROCKET_OPT_PCE_BATCH).  A side that is not a power of two is transformed
     * by Bluestein's chirp convolution with FFTs of the next power of two >= 2*side - 1
     * (slower per value than a power-of-two side).  rocket_prepare transforms every item once
     * (FP64 mean and norm, f32 2-D FFT).  out_counts, when given, receives the peak shift
     * index r*W + c of s* (a(x) ~ b(x - s*)).  A constant item gives NaN. */
    ROCKET_PCE = 8
} rocket_pair_fn;

/* The item set.  Which fields are read depends on the pair function; unused
 * fields are ignored.  All pointers are device pointers. */
typedef struct {
    /* NCC: row-major float32 [n][ld]; item i is dense[i*ld .. i*ld + dim). */
    const float *dense;
    int64_t dim;
    int64_t ld;
    /* Ragged sets (overlap, sparse): item i owns entries offsets[i] .. offsets[i+1]-1;
     * int64 [n+1], offsets[0] = 0, non-decreasing. */
    const int64_t *offsets;
    /* Overlap: interleaved float32 (x, y) per point, [2 * offsets[n]]; sigma > 0. */
    const float *xy;
    double sigma;
    /* Sparse: int64 keys [offsets[n]], strictly ascending within an item and in
     * [0, 2^32 - 1); float32 values [offsets[n]]. */
    const int64_t *keys;
    const float *vals;
    /* GMM scores: float32 standard deviation per point, [offsets[n]], same order as xy. */
    const float *point_sigma;
    /* GMM scores with a full covariance per point: float32 (c_xx, c_xy, c_yy) per point,
     * [3 * offsets[n]], same order as xy; when set, point_sigma is ignored. */
    const float *point_cov;
} rocket_items;

typedef struct rocket_ctx rocket_ctx;

/* Create a context on HIP device `device` (host pointer out).  Allocates nothing on
 * the device until the first prepare. */
rocket_status rocket_create(rocket_ctx **out, int device);
/* Free the context and its workspace (synchronises the device first).  NULL is a no-op. */
void rocket_destroy(rocket_ctx *ctx);
/* Static, human-readable name of a status code. */
const char *rocket_status_str(rocket_status status);
/* Message for the most recent failure on ctx (or on the default contexts if ctx is
 * NULL); valid until the next call on that context. */
const char *rocket_last_error(const rocket_ctx *ctx);

/* Pre-process stage (the GPU part of l, Section III) for n items under pair function
 * fn, enqueued on `stream`.  Keeps what compare needs in the context's workspace. */
rocket_status rocket_prepare(rocket_ctx *ctx, const rocket_items *items, int64_t n, rocket_pair_fn fn,
                             void *stream);

/* Compare stage (the GPU part of f) for every pair of the last prepared set.
 * out: float32 [P] packed upper triangle (required when P > 0).
 * out_counts: uint32 [P] secondary result, may be NULL: intersection sizes (sparse cosine)
 * or peak shift indices (PCE); ignored by the other functions. */
rocket_status rocket_compare(rocket_ctx *ctx, float *out, uint32_t *out_counts, void *stream);

/* rocket_prepare followed by rocket_compare on `stream`. */
rocket_status rocket_allpairs_ex(rocket_ctx *ctx, const rocket_items *items, int64_t n, rocket_pair_fn fn,
                                 float *out, uint32_t *out_counts, void *stream);

/* The whole all-pairs evaluation on the calling thread's current device, with a
 * library-owned default context per device and the null stream; synchronises
 * before returning.  out: float32 [n(n-1)/2]. */
rocket_status rocket_allpairs(const rocket_items *items, int64_t n, rocket_pair_fn fn, float *out_upper_triangle);

/* Allocation-free all pairs, for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc).  Same items, pair
 * functions, outputs, stream semantics and results as rocket_allpairs_ex on a context with
 * default options, on the CURRENT device, but every workspace buffer (prepared item copies,
 * split-K partials, work queue, flags) is carved from one static device array of
 * ROCKET_NOALLOC_SCRATCH_BYTES per device, held until the process ends; the library then
 * calls no hipMalloc or hipFree.  The caller still passes (and owns) inputs and outputs.
 * A problem whose workspace does not fit fails with ROCKET_E_OOM and a message giving the
 * sizes (rocket_last_error(NULL)); `out` is then not written.  As in rocket_prepare, the
 * ragged and sparse functions read offsets to the host and synchronise during the call.
 * Every call on one device shares that device's array and the next call overwrites it:
 * calls whose work overlaps on one device (other streams, other host threads while work
 * is still in flight) race; host calls themselves are serialised per device. */
#define ROCKET_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
rocket_status rocket_allpairs_noalloc(const rocket_items *items, int64_t n, rocket_pair_fn fn, float *out,
                                      uint32_t *out_counts, void *stream);

/* Composition vectors (the GPU pre-process stage of Section V-B's application): for each
 * species, the K-string composition vector of Qi, Wang and Hao over its proteins,
 *     f(s) = n(s) / N_K,  f0(s) = f(s_1..s_{K-1}) f(s_2..s_K) / f(s_2..s_{K-1}),
 *     a(s) = (f(s) - f0(s)) / f0(s),
 * n(s) the occurrences of K-string s in windows of K residues inside one protein, N_k the
 * number of such windows of length k (FP64, rounded once to float32).  One entry per
 * K-string that occurs, keyed by its base-20 code (s_1 most significant), keys ascending.
 * residues: uint8 codes, 0..19 amino acids; any code >= 20 ends a protein (no window
 * spans it).  offsets: int64 [n+1], species s owns residues offsets[s]..offsets[s+1]-1.
 * K: 3..6.  Outputs form a ROCKET_SPARSE_COSINE item set: cv_offsets int64 [n+1], keys
 * int64 and vals float32 of `capacity` entries; capacity >= offsets[n] always suffices
 * (ROCKET_E_INVALID if the entries do not fit).  Reads offsets to the host and
 * synchronises once at the start and once at the end.  Workspace: dense counts of
 * 4 (20^K + 20^(K-1) + 20^(K-2)) bytes per species for a group of up to 64 species
 * (~257 MB per species at K = 6), the group sized to a quarter of the free device memory
 * and half of ROCKET_OPT_WORKSPACE_CAP when that is set; kept by the context. */
rocket_status rocket_cv_build(rocket_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n, int K,
                              int64_t *cv_offsets, int64_t *keys, float *vals, int64_t capacity, void *stream);

/* Out-of-core all pairs for the NCC functions: items stay in HOST memory (float32
 * [n][ld], row-major; page-locked memory lets copies run asynchronously) and pass
 * through a device cache (Section IV-A, first level) of ROCKET_OPT_CACHE_SLOTS slots,
 * each holding one block of `tile` items in split form.  Leaf tiles are visited in
 * divide-and-conquer order; a missing block evicts the least recently used slot not
 * needed by the same tile and is copied in on a separate stream, then centred and split
 * on `stream`, while earlier tiles compute.  `out` (device, P floats) receives exactly
 * what rocket_allpairs gives for the same items, options and pair function.
 * rocket_get_stats reports cache_slots and cache_loads.  Any set prepared on this
 * context is dropped (its workspace holds the cache).  The host array must stay alive
 * and unchanged until the enqueued work completes. */
rocket_status rocket_allpairs_host(rocket_ctx *ctx, const float *host_items /* host */, int64_t n, int64_t dim,
                                   int64_t ld, rocket_pair_fn fn, float *out, void *stream);

/* Registration gradient (Section V-C optimiser).  For every pair (i, j), i < j, and
 * its transform q = params[idx(i,j)] = (theta, tx, ty), the second cloud is moved as
 *     y'_l = R(theta) (y_l - c_j) + c_j + t,   c_j = centroids[j],
 * and the overlap cost C = sum_k sum_l exp(-|y'_l - x_k|^2 / (4 sigma^2)) is returned
 * with its gradient
 *     dC/dt     = -(1/(2 sigma^2)) sum w_kl (y'_l - x_k)
 *     dC/dtheta = -(1/(2 sigma^2)) sum w_kl <y'_l - x_k, dR/dtheta (y_l - c_j)>.
 * clouds: offsets + xy + sigma as for ROCKET_GAUSS_OVERLAP; this call prepares them (size
 * sort and packing, with one synchronisation).  clouds = NULL reuses the clouds prepared by
 * the previous rocket_overlap_cost_grad on this context (no other prepare in between, same
 * n): the caller guarantees that they are alive and unchanged, e.g. across the steps of one
 * descent; else ROCKET_E_STATE.
 * centroids: float32 [n][2].  params: float32 [P][3].  out_cost: float32 [P].
 * out_grad: float32 [P][3] (theta, tx, ty), may be NULL for cost only.
 * Outputs are in packed upper-triangle order.  Enqueued on `stream`. */
rocket_status rocket_overlap_cost_grad(rocket_ctx *ctx, const rocket_items *clouds, int64_t n,
                                       const float *centroids, const float *params, float *out_cost,
                                       float *out_grad, void *stream);

/* Registration gradient of any of the three particle scores (Section V-C: the optimiser
 * maximises the GMM L2 cross term or the Bhattacharya coefficient sum between particles
 * whose localisations carry an uncertainty, or the fixed-sigma overlap).  fn:
 * ROCKET_GAUSS_OVERLAP (exactly rocket_overlap_cost_grad), ROCKET_GMM_L2 or
 * ROCKET_GMM_BHATTACHARYA.  For the GMM scores the second cloud of pair (i, j) is moved by
 * q = params[idx(i,j)] = (theta, tx, ty) about c_j = centroids[j], points and covariances
 * alike (y'_l = R(y_l - c_j) + c_j + t, T'_l = R T_l R^T; isotropic deviations give
 * T_l = t_l^2 I), and out_cost / out_grad receive the score of the moved pair and its
 * gradient with respect to q.  With a = 1/2 (L2) or 1/4 (Bhattacharya), V = S_k + T'_l,
 * d = y'_l - x_k, u = V^-1 d, g = J R(y_l - c_j), W = J T'_l - T'_l J (J the 90-degree
 * rotation), each term w contributes
 *     dw/dt = -2 a w u,    dw/dtheta = w (-2 a g^T u + a u^T W u - tr(V^-1 W) / 2).
 * items: offsets + xy + point_sigma or point_cov as for the pair function; this call
 * prepares them (one synchronisation).  items = NULL reuses what the previous
 * rocket_cost_grad (or rocket_overlap_cost_grad) on this context prepared for the same fn
 * and n (no other prepare in between); the caller guarantees the clouds are alive and
 * unchanged; else ROCKET_E_STATE.  Other arguments and layouts as for
 * rocket_overlap_cost_grad.  FP32 arithmetic, per-lane partial sums reduced by a fixed
 * wavefront tree. */
rocket_status rocket_cost_grad(rocket_ctx *ctx, const rocket_items *items, int64_t n, rocket_pair_fn fn,
                               const float *centroids, const float *params, float *out_cost, float *out_grad,
                               void *stream);

/* Tunables.  0 means "choose automatically" for every option. */
typedef enum {
    ROCKET_OPT_NCC_TILE = 1,        /* NCC output tile edge: 64, 128 or 256 items */
    ROCKET_OPT_NCC_KCHUNK = 2,      /* NCC split-K chunk length, a multiple of 16 elements (0: enough chunks
                                       for ~2048 work items within [256, 2048]; for BF16x6 also at most
                                       2^32 / dim, since the matrix cores' accumulation error grows with
                                       chunk x dim relative to the pass bar) */
    ROCKET_OPT_GRID = 3,            /* persistent grid size in workgroups */
    ROCKET_OPT_QUEUE_ORDER = 4,     /* 0 planned (D&C order in per-XCD segments), 1 shuffled (by ROCKET_OPT_SEED),
                                       2 planned order in one segment */
    ROCKET_OPT_SEED = 5,            /* seed for the shuffled queue order */
    ROCKET_OPT_LEDGER = 6,          /* 1: record how often each work item is popped (rocket_get_ledger) */
    ROCKET_OPT_OVL_BLOCK = 7,       /* clouds: clouds per block of the tile grid (0: 8; 4 with full covariances), at most 64 */
    ROCKET_OPT_OVL_VARIANT = 8,     /* overlap: inner-loop variant 1..4: lanes x points per lane of cloud j =
                                       64x1, 32x2, 16x2, 16x4 */
    ROCKET_OPT_SP_LANES = 9,        /* sparse: lanes per column item, 4 or 8 (0: 4 when that leaves at least 8
                                       work items per CU, else 8); a work item covers
                                       1024 / lanes column items */
    ROCKET_OPT_SP_CHUNK = 10,       /* sparse: least micro-chunk width of the key-range cut, a power of two
                                       at most 2^31 (larger values: ROCKET_E_INVALID)
                                       (0: automatic, the smallest width giving at most 2^20 micro-chunks) */
    ROCKET_OPT_WORKSPACE_CAP = 11,  /* bytes; workspace growth beyond it fails with ROCKET_E_OOM.  The NCC
                                     * compare fits its split-K partials (K chunks x tile^2 floats per tile)
                                     * under it, or without a cap into half of the free device memory, by
                                     * running the leaf tiles in batches of one Gram launch + epilogue each
                                     * (same output bit for bit); E_OOM if one tile's partials do not fit */
    ROCKET_OPT_AUTOTUNE = 12,       /* 1: every rocket_prepare ends with rocket_autotune */
    ROCKET_OPT_TIMING = 13,         /* 1: bracket each compare's main persistent kernel with HIP events on the
                                       launch stream; rocket_get_stats reports its duration (for
                                       rocket_allpairs_host: the whole call's device work) */
    ROCKET_OPT_CACHE_SLOTS = 14,    /* rocket_allpairs_host: device cache slots, one block of `tile` items each
                                       (0: one per block, i.e. everything stays resident); at least 2 */
    ROCKET_OPT_PCE_RADIUS = 15,     /* ROCKET_PCE: half-width h of the excluded peak neighbourhood (0: 5); h < L/2 */
    ROCKET_OPT_NCC_WAVES = 16,      /* NCC Gram workgroup: 4 or 8 waves (0: 8 for tiles of 128 and 256; tiles of
                                       64 always use 4) */
    ROCKET_OPT_PCE_WIDTH = 17,      /* ROCKET_PCE: image width W (items are dim / W rows of W values); 0: square */
    ROCKET_OPT_PCE_BATCH = 18,      /* ROCKET_PCE, staged path: pair-pairs per batch of staged transforms (0: as
                                       many as 512 MiB holds; the cap and the arena bound it too).  Two
                                       staging buffers where the workspace holds two batches, the row pass of one
                                       batch overlapping the column pass of the other on a second stream of the
                                       context; one buffer and the caller's stream only in the allocation-free
                                       entry point */
    ROCKET_OPT_TRACE = 19           /* 1: the persistent kernels time-stamp every work item (rocket_get_trace); set
                                       before rocket_prepare, like ROCKET_OPT_LEDGER */
} rocket_option;

rocket_status rocket_set_option(rocket_ctx *ctx, rocket_option opt, int64_t value);
rocket_status rocket_get_option(const rocket_ctx *ctx, rocket_option opt, int64_t *value /* host */);

/* Facts about the last prepare/compare, for benchmarks and tests. */
typedef struct {
    int64_t n;               /* items */
    int64_t pairs;           /* n(n-1)/2 */
    int64_t tiles;           /* leaves of the divide-and-conquer split */
    int64_t work_items;      /* queue entries (tiles x split-K chunks, or tiles) */
    int64_t grid;            /* persistent workgroups launched */
    int64_t tile;            /* tile edge in items (NCC) or clouds/items per block */
    int64_t kchunk;          /* NCC split-K chunk length (0 otherwise) */
    int64_t workspace_bytes; /* device bytes currently held by the context */
    int64_t variant;         /* kernel variant in use: NCC pair function, overlap inner-loop variant, sparse
                                lanes per column item (a work item covers 1024 / variant column items),
                                PCE side L (one LDS tile per pair) or H * 10000 + W (staged path) */
    int64_t kernel_ns;       /* duration of the last main kernel (ROCKET_OPT_TIMING=1), else -1;
                                reading it waits for that kernel to finish */
    int64_t cache_slots;     /* rocket_allpairs_host: device cache slots used (0 otherwise) */
    int64_t cache_loads;     /* rocket_allpairs_host: block loads from host memory; the reload factor is
                                cache_loads / ceil(n / tile) (1 when every block is loaded once) */
    int64_t tune_us;         /* the last autotune's wall time in microseconds (0 if none ran) */
    int64_t tune_cached;     /* 1 when the last autotune applied a shape from the cache file */
} rocket_stats;

rocket_status rocket_get_stats(const rocket_ctx *ctx, rocket_stats *out /* host */);

/* Per-tile trace of the last compare that ran a persistent queue (Section IV-C's profiling
 * of when each job ran where), with ROCKET_OPT_TRACE set to 1 before its rocket_prepare.
 * One record per work item in queue order: its tile (block row, block column, NCC split-K
 * chunk or 0), the persistent workgroup that ran it (hardware places workgroup b on XCD
 * b mod 8) and its start and end on the device's constant-rate wall clock, in ns after the
 * earliest start.  A work item ends when its workgroup next pops the queue.  Items that did
 * not run have workgroup -1.  *count receives the number of work items; at most cap
 * records are written to out (host; NULL with cap 0 queries the count).  Synchronises the
 * device.  ROCKET_E_STATE without a trace (option unset, or a path without a queue: the
 * staged PCE path, the host-resident NCC path). */
typedef struct {
    int32_t tile_i, tile_j; /* block row and block column of the work item's tile */
    int32_t chunk;          /* NCC split-K chunk (0 for the other pair functions) */
    int32_t workgroup;      /* persistent workgroup that ran it, -1 if none */
    int64_t start_ns, end_ns;
} rocket_trace_rec;
rocket_status rocket_get_trace(rocket_ctx *ctx, rocket_trace_rec *out /* host */, int64_t cap, int64_t *count /* host */);

/* Copy the pop counts of the last compare (ROCKET_OPT_LEDGER=1) into host array out
 * [cap]; *count receives the number of work items.  Synchronises the device. */
rocket_status rocket_get_ledger(rocket_ctx *ctx, int32_t *out /* host */, int64_t cap, int64_t *count /* host */);

/* Autotuner of the tile shapes for the prepared set (the batching of uneven items into one
 * persistent launch, and the dense Gram tiles): every candidate is prepared and one whole
 * compare is timed with HIP events; the fastest is kept in the context's options (readable
 * with rocket_get_option) and the set is prepared with it.  Those options stay in effect for
 * later prepares on the context, whatever their size: set them back to 0 (the library's
 * defaults for each size) or tune again before preparing a set of another size.  Candidates:
 *   NCC:     tile {256, 128} (n >= 1536) or {128, 64}, waves {8, 4}, K chunk {default,
 *            default/2} (never longer than the default: FP32 accumulation in the matrix
 *            cores loses accuracy with chunk length);
 *   sparse:  lanes per column {4, 8} x micro-chunk width {automatic, twice that};
 *   clouds:  clouds per block {4, 8, 16} x inner-loop variant 1..4.
 * NCC tile / waves and the cloud shapes change only the schedule (same output bit for bit);
 * the K chunk and the sparse shapes change the FP32 summation order (results stay within
 * the pair function's accuracy).  With a cache file (rocket_set_tune_cache) the choice is
 * stored under (pair function, GPU architecture, log2 n in half steps, p50 / p90 item size
 * or log2 d) and reused by later calls with the same key without timing.  Synchronises;
 * allocates one scratch output when it times.  rocket_get_stats reports tune_us and
 * tune_cached.  A no-op for PCE.  ROCKET_OPT_AUTOTUNE=1 runs it at the end of every
 * rocket_prepare. */
rocket_status rocket_autotune(rocket_ctx *ctx, void *stream);

/* The autotuner's cache file (host path; NULL or "" disables the cache).  The file is
 * read at every rocket_autotune and rewritten (write to path.tmp, then rename) when a new
 * key is tuned. */
rocket_status rocket_set_tune_cache(rocket_ctx *ctx, const char *path /* host */);

/* Measurement aid for the VALU-bound rooflines (not part of the pair computation): issue
 * rates on `device`, in instructions per second over all lanes, of dependent chains of
 * FP32 FMA (v_fma_f32), v_exp_f32 and v_rcp_f32, eight independent chains per lane and
 * eight waves per SIMD of every CU, each timed with HIP events over one launch (~10 ms in
 * all).  Outputs are host doubles.  Allocates and frees a small sink buffer; synchronises. */
rocket_status rocket_probe_valu(int device, double *fma_per_s /* host */, double *exp2_per_s /* host */,
                                double *rcp_per_s /* host */);

/* Host-only planner, no device needed: the divide-and-conquer leaves for n items
 * with tiles of T items (Section IV-B: recursive quadrant split of the upper
 * triangle, empty quadrants skipped), in visiting order (top-left, top-right,
 * bottom-left, bottom-right).  Writes up to cap leaves to host arrays bi, bj and
 * returns the number of leaves (negative status on bad arguments). */
int64_t rocket_plan_tiles(int64_t n, int64_t T, int32_t *bi /* host */, int32_t *bj /* host */, int64_t cap);

/* Packed upper-triangle index of pair (i, j), i < j < n (host helper). */
int64_t rocket_pair_index(int64_t i, int64_t j, int64_t n);

#ifdef __cplusplus
}
#endif
#endif /* ROCKET_H */
