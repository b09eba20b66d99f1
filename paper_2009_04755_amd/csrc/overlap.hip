// Gaussian-overlap registration cost between 2-D point clouds (Section V-C compare kernel)
// and its adjoint with respect to a rigid transform, on gfx950.
//
//   C_ij = sum_k sum_l w_kl,  w_kl = exp(-|y'_l - x_k|^2 / (4 sigma^2)),
//   x = points of cloud i, y = points of cloud j, y' = y (cost) or R(theta)(y - c_j) + c_j + t (adjoint).
//   dC/dt     = -(1/(2 sigma^2)) sum_kl w_kl (y'_l - x_k)
//   dC/dtheta = -(1/(2 sigma^2)) sum_l < sum_k w_kl (y'_l - x_k), J R(theta)(y_l - c_j) >
//
// Clouds have uneven sizes.  Prepare sorts them by size (largest first) and packs them
// contiguously, so that a tile of T x T sorted clouds holds pairs of similar cost; tiles are
// queued largest estimated cost first (sum of N_a N_b) and dealt to per-XCD segments.  One
// persistent workgroup per CU stages the two cloud blocks of its tile in LDS and gives each
// pair to one wavefront: lanes own points of cloud j (S lanes x R registers per chunk, 64/S
// phases over the points of cloud i), every lane keeps FP32 partial sums, and the wavefront
// reduces them with a fixed xor-butterfly, so results do not depend on scheduling.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "common.hpp"
#include "queue.hpp"

namespace rk {
namespace {

constexpr int OVL_THREADS = 512;
constexpr int OVL_WAVES = OVL_THREADS / 64;
constexpr int OVL_MAX_BLOCK_PTS = 10000;  // per staged block (80 KB)

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Gather sorted clouds into one packed array: cloud s of the sorted order owns packed
// points coff[s] .. coff[s+1]-1.
__global__ void k_ovl_pack(const float2 *__restrict__ xy, const int64_t *__restrict__ offsets,
                           const int *__restrict__ perm, const int *__restrict__ coff, float2 *__restrict__ packed, int n)
{
    for (int s = blockIdx.x; s < n; s += gridDim.x) {
        const int64_t src = offsets[perm[s]];
        const int dst = coff[s], cnt = coff[s + 1] - coff[s];
        for (int k = threadIdx.x; k < cnt; k += blockDim.x) packed[dst + k] = xy[src + k];
    }
}

template <bool GRAD, int S, int R>
__global__ __launch_bounds__(OVL_THREADS, 1) void k_overlap(const float2 *__restrict__ pts, const int *__restrict__ coff,
                                                            const int *__restrict__ perm, int n, int T, float cexp,
                                                            QueueArgs q, float *__restrict__ out,
                                                            const float *__restrict__ cen,
                                                            const float *__restrict__ params, float *__restrict__ grad,
                                                            float gscale)
{
    constexpr int P = 64 / S;  // phases over the points of cloud i
    constexpr int CH = S * R;  // points of cloud j per chunk
    extern __shared__ float2 lds_pts[];
    __shared__ int s_item;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int slot = lane % S, phase = lane / S;

    for (;;) {
        const int it = queue_pop_wg(q, &s_item);
        if (it < 0) break;
        const int4 w = q.items[it];
        const int bI = w.x, bJ = w.y;
        const int a0 = bI * T, a1 = min(n, a0 + T), b0 = bJ * T, b1 = min(n, b0 + T);
        const bool diag = bI == bJ;
        // stage block I, then block J behind it (once on the diagonal)
        const int pI0 = coff[a0], pI1 = coff[a1];
        const int pJ0 = coff[b0], pJ1 = coff[b1];
        const int nI = pI1 - pI0, nJ = diag ? 0 : pJ1 - pJ0;
        for (int k = tid; k < nI; k += OVL_THREADS) lds_pts[k] = pts[pI0 + k];
        for (int k = tid; k < nJ; k += OVL_THREADS) lds_pts[nI + k] = pts[pJ0 + k];
        __syncthreads();

        const int na = a1 - a0, nb = b1 - b0;
        for (int p = wave; p < na * nb; p += OVL_WAVES) {
            const int a = a0 + p / nb, b = b0 + p % nb;
            if (a >= b) continue;  // diagonal tile: strict upper triangle only
            const int ia = perm[a], ib = perm[b];
            const int oi = min(ia, ib), oj = max(ia, ib);
            // cloud i (looped) and cloud j (in lanes) in LDS coordinates
            const int si = ia == oi ? a : b, sj = ia == oi ? b : a;
            const int base_i = si < b0 || diag ? coff[si] - pI0 : nI + coff[si] - pJ0;
            const int base_j = sj < b0 || diag ? coff[sj] - pI0 : nI + coff[sj] - pJ0;
            const int Ni = coff[si + 1] - coff[si], Nj = coff[sj + 1] - coff[sj];
            const int64_t pidx = (int64_t)oi * n - (int64_t)oi * (oi + 1) / 2 + (oj - oi - 1);

            float cx = 0.f, cy = 0.f, tx = 0.f, ty = 0.f;
            double dct = 1.0, dst = 0.0;
            if constexpr (GRAD) {
                const float th = params[3 * pidx];
                tx = params[3 * pidx + 1];
                ty = params[3 * pidx + 2];
                sincos((double)th, &dst, &dct);
                cx = cen[2 * oj];
                cy = cen[2 * oj + 1];
            }
            float accC = 0.f, accT = 0.f, accX = 0.f, accY = 0.f;
            for (int c0 = 0; c0 < Nj; c0 += CH) {
                // y'_l as an unevaluated FP32 pair (hi + lo): rounding the transformed point to
                // one FP32 would move every exponent by ~1250 |u| 2^-24, which is 1e-5 of a
                // term already at |u| ~ 0.25
                float yx[R], yy[R], lx[R], ly[R], vx[R], vy[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int l = c0 + r * S + slot;
                    if (l < Nj) {
                        const float2 y = lds_pts[base_j + l];
                        if constexpr (GRAD) {
                            // transform in FP64, rounded once to FP32
                            const double rx = (double)y.x - cx, ry = (double)y.y - cy;
                            const double ox = dct * rx - dst * ry, oy = dst * rx + dct * ry;
                            const double px = ox + cx + tx, py = oy + cy + ty;
                            yx[r] = (float)px;
                            yy[r] = (float)py;
                            lx[r] = (float)(px - (double)yx[r]);
                            ly[r] = (float)(py - (double)yy[r]);
                            vx[r] = (float)(-oy);
                            vy[r] = (float)ox;
                        } else {
                            yx[r] = y.x;
                            yy[r] = y.y;
                        }
                    } else {
                        yx[r] = 3.0e19f;  // far away: every term underflows to exactly 0
                        yy[r] = 3.0e19f;
                        lx[r] = ly[r] = 0.f;
                        vx[r] = 0.f;
                        vy[r] = 0.f;
                    }
                }
                float sc[R], sx[R], sy[R];
#pragma unroll
                for (int r = 0; r < R; ++r) sc[r] = sx[r] = sy[r] = 0.f;
                for (int k = phase; k < Ni; k += P) {
                    const float2 x = lds_pts[base_i + k];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        float ux = yx[r] - x.x, uy = yy[r] - x.y;
                        if constexpr (GRAD) {
                            ux += lx[r];
                            uy += ly[r];
                        }
                        const float d2 = fmaf(uy, uy, ux * ux);
                        const float wkl = __builtin_amdgcn_exp2f(-(d2 * cexp));
                        sc[r] += wkl;
                        if constexpr (GRAD) {
                            sx[r] = fmaf(wkl, ux, sx[r]);
                            sy[r] = fmaf(wkl, uy, sy[r]);
                        }
                    }
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    accC += sc[r];
                    if constexpr (GRAD) {
                        accX += sx[r];
                        accY += sy[r];
                        accT = fmaf(vx[r], sx[r], fmaf(vy[r], sy[r], accT));
                    }
                }
            }
            const float C = wave_sum(accC);
            if constexpr (GRAD) {
                const float GX = wave_sum(accX), GY = wave_sum(accY), GT = wave_sum(accT);
                if (lane == 0) {
                    out[pidx] = C;
                    if (grad) {
                        grad[3 * pidx] = gscale * GT;
                        grad[3 * pidx + 1] = gscale * GX;
                        grad[3 * pidx + 2] = gscale * GY;
                    }
                }
            } else {
                if (lane == 0) out[pidx] = C;
            }
        }
        __syncthreads();  // LDS is restaged for the next tile
    }
}

template <bool GRAD>
const void *ovl_kernel(int variant)
{
    switch (variant) {
    case 1: return (const void *)&k_overlap<GRAD, 64, 1>;
    case 2: return (const void *)&k_overlap<GRAD, 32, 2>;
    default: return (const void *)&k_overlap<GRAD, 16, 2>;
    }
}

template <bool GRAD>
void launch_ovl(int variant, int grid, size_t lds, hipStream_t s, const float2 *pts, const int *coff, const int *perm,
                int n, int T, float cexp, const QueueArgs &qa, float *out, const float *cen, const float *params,
                float *grad, float gscale)
{
    switch (variant) {
    case 1:
        hipLaunchKernelGGL((k_overlap<GRAD, 64, 1>), dim3(grid), dim3(OVL_THREADS), lds, s, pts, coff, perm, n, T,
                           cexp, qa, out, cen, params, grad, gscale);
        break;
    case 2:
        hipLaunchKernelGGL((k_overlap<GRAD, 32, 2>), dim3(grid), dim3(OVL_THREADS), lds, s, pts, coff, perm, n, T,
                           cexp, qa, out, cen, params, grad, gscale);
        break;
    default:
        hipLaunchKernelGGL((k_overlap<GRAD, 16, 2>), dim3(grid), dim3(OVL_THREADS), lds, s, pts, coff, perm, n, T,
                           cexp, qa, out, cen, params, grad, gscale);
        break;
    }
}

struct OvlDev {
    float2 *pts;
    int *coff, *perm;
};

OvlDev dev_ptrs(rocket_ctx *ctx, int64_t n)
{
    OvlDev d;
    d.pts = (float2 *)ctx->ws[WS_OVL_PACK].ptr;
    d.coff = (int *)ctx->ws[WS_OVL_META].ptr;
    d.perm = d.coff + ((n + 1 + 63) / 64) * 64;
    return d;
}

}  // namespace

// Build the tile queue for block size T over the sorted clouds: leaves of the
// divide-and-conquer split, largest estimated cost (sum of N_a N_b) first.
static void ovl_plan(rocket_ctx *ctx, int T, std::vector<int4> &items, std::vector<int> &seg, int64_t *max_block_pts,
                     std::vector<double> *costs_out = nullptr)
{
    OvlState &o = ctx->ovl;
    const int64_t n = o.n;
    std::vector<int2> leaves;
    plan_leaves(n, T, leaves);
    std::vector<int64_t> cnt(n);
    for (int64_t s = 0; s < n; ++s) cnt[s] = o.h_offsets[o.perm[s] + 1] - o.h_offsets[o.perm[s]];
    const int64_t nb = (n + T - 1) / T;
    std::vector<double> bsum(nb, 0.0);
    int64_t mx = 0;
    for (int64_t b = 0; b < nb; ++b) {
        int64_t pts = 0;
        for (int64_t s = b * T; s < std::min(n, (b + 1) * T); ++s) {
            bsum[b] += (double)cnt[s];
            pts += cnt[s];
        }
        mx = std::max(mx, pts);
    }
    *max_block_pts = mx;
    std::vector<int4> raw;
    std::vector<double> cost;
    raw.reserve(leaves.size());
    cost.reserve(leaves.size());
    for (size_t k = 0; k < leaves.size(); ++k) {
        const int bi = leaves[k].x, bj = leaves[k].y;
        double c;
        if (bi != bj) {
            c = bsum[bi] * bsum[bj];
        } else {  // strict upper triangle of the block: (S^2 - sum N^2) / 2
            double sq = 0;
            for (int64_t s = (int64_t)bi * T; s < std::min(n, (int64_t)(bi + 1) * T); ++s)
                sq += (double)cnt[s] * cnt[s];
            c = 0.5 * (bsum[bi] * bsum[bi] - sq);
        }
        raw.push_back(make_int4(bi, bj, 0, (int)k));
        cost.push_back(c + 64.0 * 64.0);  // per-pair overhead floor
    }
    if (costs_out) *costs_out = cost;
    const int64_t order = ctx->opt[ROCKET_OPT_QUEUE_ORDER];
    plan_lpt(raw, cost, MAX_SEG, items, seg);
    if (order == 1) shuffle_items(items, seg, (uint64_t)ctx->opt[ROCKET_OPT_SEED]);
    if (order == 2) single_segment(seg, (int64_t)items.size());
}

static int ovl_block(rocket_ctx *ctx) { return ctx->opt[ROCKET_OPT_OVL_BLOCK] ? (int)ctx->opt[ROCKET_OPT_OVL_BLOCK] : 16; }
static int ovl_variant(rocket_ctx *ctx)
{
    return ctx->opt[ROCKET_OPT_OVL_VARIANT] ? (int)ctx->opt[ROCKET_OPT_OVL_VARIANT] : 3;
}

static rocket_status ovl_replan(rocket_ctx *ctx, hipStream_t s)
{
    OvlState &o = ctx->ovl;
    int T = ovl_block(ctx);
    int64_t mx = 0;
    for (;;) {
        ovl_plan(ctx, T, ctx->h_items, ctx->h_seg, &mx);
        if (mx <= OVL_MAX_BLOCK_PTS || T == 1) break;
        T = std::max(1, T / 2);
    }
    if (mx > OVL_MAX_BLOCK_PTS) return fail(ctx, ROCKET_E_UNSUPPORTED, "a single cloud exceeds the LDS capacity");
    o.block = T;
    o.max_block_pts = mx;
    o.tiles = (int64_t)ctx->h_items.size();
    if (o.tiles > 0) RK_TRY(upload_queue(ctx, s, &o.qa));
    ctx->queue_owner = QOWN_OVL;
    o.pc_block = ovl_block(ctx);
    o.pc_order = ctx->opt[ROCKET_OPT_QUEUE_ORDER];
    o.pc_seed = ctx->opt[ROCKET_OPT_SEED];
    o.pc_ledger = ctx->opt[ROCKET_OPT_LEDGER];
    return ROCKET_OK;
}

rocket_status ovl_prepare(rocket_ctx *ctx, const rocket_items *it, int64_t n, hipStream_t s)
{
    OvlState &o = ctx->ovl;
    o.valid = false;
    if (n > 0 && (!it->offsets || !it->xy)) return fail(ctx, ROCKET_E_INVALID, "offsets or xy is NULL");
    if (!(it->sigma > 0.0) || !std::isfinite(it->sigma)) return fail(ctx, ROCKET_E_INVALID, "sigma must be > 0");
    if (n >= (1 << 30)) return fail(ctx, ROCKET_E_INVALID, "n too large");
    o.n = n;
    o.offsets = it->offsets;
    o.xy = it->xy;
    o.sigma = it->sigma;
    o.h_offsets.assign((size_t)n + 1, 0);
    if (n > 0) {
        RK_HIP(hipMemcpyAsync(o.h_offsets.data(), it->offsets, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s));
        RK_HIP(hipStreamSynchronize(s));
    }
    if (o.h_offsets[0] != 0) return fail(ctx, ROCKET_E_INVALID, "offsets[0] != 0");
    for (int64_t i = 0; i < n; ++i)
        if (o.h_offsets[i + 1] < o.h_offsets[i]) return fail(ctx, ROCKET_E_INVALID, "offsets decrease");
    o.total = o.h_offsets[n];
    if (o.total >= ((int64_t)1 << 31)) return fail(ctx, ROCKET_E_INVALID, "too many points");
    // size sort, largest first (stable)
    o.perm.resize(n);
    std::iota(o.perm.begin(), o.perm.end(), 0);
    std::stable_sort(o.perm.begin(), o.perm.end(), [&](int a, int b) {
        return o.h_offsets[a + 1] - o.h_offsets[a] > o.h_offsets[b + 1] - o.h_offsets[b];
    });
    std::vector<int> meta(((n + 1 + 63) / 64) * 64 + std::max<int64_t>(n, 1), 0);
    int acc = 0;
    for (int64_t s2 = 0; s2 < n; ++s2) {
        meta[s2] = acc;
        acc += (int)(o.h_offsets[o.perm[s2] + 1] - o.h_offsets[o.perm[s2]]);
    }
    meta[n] = acc;
    const size_t poff = ((n + 1 + 63) / 64) * 64;
    for (int64_t s2 = 0; s2 < n; ++s2) meta[poff + s2] = o.perm[s2];
    void *mp = nullptr, *pp = nullptr;
    RK_TRY(ws_get(ctx, WS_OVL_META, sizeof(int) * meta.size(), &mp));
    RK_TRY(ws_get(ctx, WS_OVL_PACK, sizeof(float2) * (size_t)std::max<int64_t>(o.total, 1), &pp));
    RK_HIP(hipMemcpyAsync(mp, meta.data(), sizeof(int) * meta.size(), hipMemcpyHostToDevice, s));
    if (n > 0) {
        const OvlDev d = dev_ptrs(ctx, n);
        hipLaunchKernelGGL(k_ovl_pack, dim3((unsigned)std::min<int64_t>(n, 65535)), dim3(256), 0, s,
                           (const float2 *)it->xy, it->offsets, d.perm, d.coff, d.pts, (int)n);
        RK_HIP(hipGetLastError());
    }
    RK_HIP(hipStreamSynchronize(s));  // meta staging vector goes out of scope
    RK_TRY(ovl_replan(ctx, s));
    if (ctx->opt[ROCKET_OPT_AUTOTUNE] && n >= 64) RK_TRY(ovl_autotune(ctx, s));
    ctx->stats.tiles = o.tiles;
    ctx->stats.work_items = o.tiles;
    ctx->stats.tile = o.block;
    ctx->stats.kchunk = 0;
    o.valid = true;
    return ROCKET_OK;
}

static rocket_status ovl_launch(rocket_ctx *ctx, hipStream_t s, float *out, const float *cen, const float *params,
                                float *grad, int variant)
{
    OvlState &o = ctx->ovl;
    const OvlDev d = dev_ptrs(ctx, o.n);
    const size_t lds = (size_t)2 * o.max_block_pts * sizeof(float2) + 16;
    const bool g = params != nullptr;
    const int grid = auto_grid(ctx, g ? ovl_kernel<true>(variant) : ovl_kernel<false>(variant), OVL_THREADS, lds,
                               o.tiles);
    ctx->stats.grid = grid;
    ctx->stats.variant = variant;
    RK_HIP(hipFuncSetAttribute(g ? ovl_kernel<true>(variant) : ovl_kernel<false>(variant),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    RK_TRY(reset_queue(ctx, s, o.qa));
    const float cexp = (float)(1.4426950408889634 / (4.0 * o.sigma * o.sigma));
    const float gscale = (float)(-1.0 / (2.0 * o.sigma * o.sigma));
    RK_TRY(timing_begin(ctx, s));
    if (g)
        launch_ovl<true>(variant, grid, lds, s, d.pts, d.coff, d.perm, (int)o.n, o.block, cexp, o.qa, out, cen, params,
                         grad, gscale);
    else
        launch_ovl<false>(variant, grid, lds, s, d.pts, d.coff, d.perm, (int)o.n, o.block, cexp, o.qa, out, nullptr,
                          nullptr, nullptr, gscale);
    RK_HIP(hipGetLastError());
    RK_TRY(timing_end(ctx, s));
    return ROCKET_OK;
}

rocket_status ovl_compare(rocket_ctx *ctx, float *out, const float *cen, const float *params, float *grad,
                          hipStream_t s)
{
    OvlState &o = ctx->ovl;
    if (!o.valid) return fail(ctx, ROCKET_E_STATE, "overlap set not prepared");
    if (o.n < 2 || o.tiles == 0) return ROCKET_OK;
    if (ctx->queue_owner != QOWN_OVL || o.pc_block != ovl_block(ctx) || o.pc_order != ctx->opt[ROCKET_OPT_QUEUE_ORDER] ||
        o.pc_seed != ctx->opt[ROCKET_OPT_SEED] || o.pc_ledger != ctx->opt[ROCKET_OPT_LEDGER])
        RK_TRY(ovl_replan(ctx, s));
    return ovl_launch(ctx, s, out, cen, params, grad, ovl_variant(ctx));
}

// Autotuner: time every (block size, inner-loop variant) candidate on the full prepared
// set's cost kernel and keep the fastest; the queue is rebuilt for each block size.
rocket_status ovl_autotune(rocket_ctx *ctx, hipStream_t s)
{
    OvlState &o = ctx->ovl;
    if (o.n < 2) return ROCKET_OK;
    const int64_t P = o.n * (o.n - 1) / 2;
    float *scratch = nullptr;
    RK_HIP(hipMalloc(&scratch, sizeof(float) * P));
    hipEvent_t e0, e1;
    RK_HIP(hipEventCreate(&e0));
    RK_HIP(hipEventCreate(&e1));
    const int64_t save_block = ctx->opt[ROCKET_OPT_OVL_BLOCK], save_var = ctx->opt[ROCKET_OPT_OVL_VARIANT];
    const int blocks[] = {8, 16, 32};
    float best = 1e30f;
    int best_b = 16, best_v = 3;
    rocket_status st = ROCKET_OK;
    for (int b : blocks) {
        ctx->opt[ROCKET_OPT_OVL_BLOCK] = b;
        if ((st = ovl_replan(ctx, s)) != ROCKET_OK) break;
        if (o.block != b) continue;  // block did not fit in LDS
        for (int v = 1; v <= 3; ++v) {
            if ((st = ovl_launch(ctx, s, scratch, nullptr, nullptr, nullptr, v)) != ROCKET_OK) break;  // warm-up
            (void)hipEventRecord(e0, s);
            if ((st = ovl_launch(ctx, s, scratch, nullptr, nullptr, nullptr, v)) != ROCKET_OK) break;
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) {
                best = ms;
                best_b = b;
                best_v = v;
            }
        }
        if (st != ROCKET_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(scratch);
    if (st != ROCKET_OK) {
        ctx->opt[ROCKET_OPT_OVL_BLOCK] = save_block;
        ctx->opt[ROCKET_OPT_OVL_VARIANT] = save_var;
        return st;
    }
    ctx->opt[ROCKET_OPT_OVL_BLOCK] = best_b;
    ctx->opt[ROCKET_OPT_OVL_VARIANT] = best_v;
    RK_TRY(ovl_replan(ctx, s));
    ctx->stats.tile = o.block;
    ctx->stats.variant = best_v;
    return ROCKET_OK;
}

}  // namespace rk
