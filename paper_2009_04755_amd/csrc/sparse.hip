// Cosine similarity of sparse key/value vectors with the exact key-intersection size
// (Section V-B compare kernel: the dot product of two sparse composition vectors), gfx950.
//
//   m_ij = |K_i & K_j|,  cos_ij = sum_{k in K_i & K_j} v_ik v_jk / (|v_i| |v_j|).
//
// Prepare validates the keys (strictly ascending per item, in [0, 2^32 - 1)), packs them to
// u32, reduces every item's L2 norm in FP64, and sorts items by nnz (largest first) so the
// streams processed side by side have similar lengths.  Work item = (band of RB=16 sorted
// row items) x (block of CB = 1024 / LPC sorted column items, LPC = 4 or 8 lanes per column).
// The key space is cut, per band, into
// chunks holding at most UMAX row entries (counted on a histogram of the band's keys over
// fixed-width micro-chunks; a micro-chunk wider than 64 keys that alone holds more than UMAX
// of a band's entries is counted again in 64-key ranges and that band is cut on the host).  For every chunk the workgroup builds in LDS a hash table of the
// band's keys whose slots carry the 16 row values (zero when absent) and 16 presence bytes;
// then each column streams its keys of that chunk (LPC lanes per column, coalesced), probes
// the table and accumulates 16 dot products and 16 counts in registers.  Keys match by
// integer equality, so counts are exact; chunk sums are added with compensation and the LPC
// lanes of a column combine in a fixed butterfly, so results do not depend on scheduling.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "common.hpp"
#include "queue.hpp"

namespace rk {
namespace {

constexpr int RB = 16;          // rows per band
constexpr int SP_THREADS = 1024;
constexpr int UMAX = 1632;      // row entries per chunk: 80 B of LDS each (16 values + 16 presence
                                // bytes); with the 32 KiB hash table 163,344 of 163,840 bytes
constexpr int SR = 4;           // column entries per lane per streaming pass
constexpr int HBITS = 12;
constexpr int HSIZE = 1 << HBITS;
constexpr uint32_t EMPTY = 0xFFFFFFFFu;
// Chunk bounds are kept in units of 2^ulog keys, ulog = min(wlog, FINE_LOG): a range of 64
// keys holds at most 16 x 64 = 1024 entries of a band (keys are unique per item), less than
// UMAX, so a micro-chunk wider than 64 keys that holds more than UMAX entries of a band can
// always be cut at 64-key granularity.
constexpr int FINE_LOG = 6;
constexpr int OVF_MAX = 1 << 16;  // overflowing (band, micro-chunk) pairs handled per prepare

enum { FLAG_UNSORTED = 1, FLAG_RANGE = 2, FLAG_OVERFLOW = 4 };

__device__ __forceinline__ uint32_t hslot(uint32_t key) { return (key * 2654435761u) >> (32 - HBITS); }

// Validate, pack to u32, FP64 norm.  One workgroup per item.
__global__ __launch_bounds__(256) void k_sp_validate(const int64_t *__restrict__ keys, const float *__restrict__ vals,
                                                     const int64_t *__restrict__ off, int n,
                                                     uint32_t *__restrict__ k32, float *__restrict__ inv_norm,
                                                     unsigned *__restrict__ flags, unsigned *__restrict__ maxkey)
{
    const int i = blockIdx.x;
    const int64_t b = off[i], e = off[i + 1];
    double ss = 0.0;
    unsigned bad = 0, mx = 0;
    for (int64_t p = b + threadIdx.x; p < e; p += 256) {
        const int64_t k = keys[p];
        if (k < 0 || k >= 0xFFFFFFFFll) bad |= FLAG_RANGE;  // 0xFFFFFFFF marks an empty hash slot
        if (p > b && keys[p - 1] >= k) bad |= FLAG_UNSORTED;
        k32[p] = (uint32_t)k;
        mx = max(mx, (unsigned)(k & 0xFFFFFFFFll));
        const double v = vals[p];
        ss += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) {
        ss += __shfl_xor(ss, o);
        bad |= __shfl_xor(bad, o);
        mx = max(mx, (unsigned)__shfl_xor((int)mx, o));
    }
    __shared__ double red[4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w] = ss;
        if (bad) atomicOr(flags, bad);
        atomicMax(maxkey, mx);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = (red[0] + red[1]) + (red[2] + red[3]);
        inv_norm[i] = t > 0 ? (float)(1.0 / sqrt(t)) : __builtin_nanf("");
    }
}

// Histogram of every band's keys over micro-chunks of width 2^wlog.
__global__ __launch_bounds__(256) void k_sp_hist(const uint32_t *__restrict__ k32, const int64_t *__restrict__ off,
                                                 const int *__restrict__ perm, int n, int wlog, int64_t nmc,
                                                 unsigned *__restrict__ hist)
{
    const int s = blockIdx.x;  // sorted position
    const int i = perm[s];
    unsigned *h = hist + (int64_t)(s / RB) * nmc;
    for (int64_t p = off[i] + threadIdx.x; p < off[i + 1]; p += 256) atomicAdd(h + (k32[p] >> wlog), 1u);
}

// Greedy cut of each band's micro-chunks into chunks of at most UMAX entries: a chunk is
// closed before the micro-chunk that would overflow it.  Pass 0 counts chunks per band,
// pass 1 writes their starting micro-chunk.  One workgroup per band stages the counts in
// LDS; one wave runs the greedy scan 64 counts at a time: a prefix sum over the lanes finds
// the next overflowing lane with one ballot, so a window costs one step plus one per cut.
// Pass 0 also appends every (band, micro-chunk) holding more than UMAX entries of the band
// to `ovf` (count in ovf_n); those bands are cut on the host at 64-key granularity, and pass
// 1 skips them (host_cut[band] != 0).  Bounds are written in units of 2^shift micro-chunk
// widths' fractions: micro-chunk m starts at unit m << shift.
__global__ __launch_bounds__(256) void k_sp_cut(const unsigned *__restrict__ hist, int64_t nmc, int pass, int shift,
                                                int *__restrict__ nchunks, const int64_t *__restrict__ cstart,
                                                int *__restrict__ bounds, unsigned *__restrict__ flags,
                                                int2 *__restrict__ ovf, unsigned *__restrict__ ovf_n,
                                                const int *__restrict__ host_cut)
{
    const int band = blockIdx.x;
    if (pass && host_cut && host_cut[band]) return;
    const unsigned *h = hist + (int64_t)band * nmc;
    __shared__ unsigned buf[4096];
    const int lane = threadIdx.x & 63;
    unsigned acc = 0;  // fill of the open chunk (wave-uniform)
    int cnt = 0;
    int *out = pass ? bounds + cstart[band] : nullptr;
    if (pass && threadIdx.x == 0) out[0] = 0;
    for (int64_t m0 = 0; m0 < nmc; m0 += 4096) {
        __syncthreads();
        for (int k = threadIdx.x; k < 4096; k += 256) buf[k] = m0 + k < nmc ? h[m0 + k] : 0u;
        __syncthreads();
        if (threadIdx.x >= 64) continue;
        const int lim = (int)min<int64_t>(4096, nmc - m0);
        for (int b = 0; b < lim; b += 64) {
            const unsigned c = b + lane < lim ? buf[b + lane] : 0u;
            if (!pass && c > (unsigned)UMAX) {
                const unsigned slot = atomicAdd(ovf_n, 1u);
                if (slot < (unsigned)OVF_MAX) ovf[slot] = make_int2(band, (int)(m0 + b + lane));
            }
            if (__ballot(c > (unsigned)UMAX) && lane == 0) atomicOr(flags, (unsigned)FLAG_OVERFLOW);
            int start = 0;
            for (;;) {
                const unsigned v = lane >= start ? c : 0u;
                unsigned sum = v;  // inclusive prefix over the lanes
                for (int o = 1; o < 64; o <<= 1) {
                    const unsigned t = __shfl_up(sum, o);
                    if (lane >= o) sum += t;
                }
                const bool cut = lane >= start && acc + sum > (unsigned)UMAX && acc + sum - v > 0u;
                const uint64_t m = __ballot(cut);
                if (m == 0) {
                    acc += __shfl(sum, 63);
                    break;
                }
                const int i = __ffsll((unsigned long long)m) - 1;
                ++cnt;
                if (pass && lane == 0) out[cnt] = (int)((m0 + b + i) << shift);
                acc = 0;
                start = i;
            }
        }
    }
    if (threadIdx.x == 0) {
        ++cnt;  // the last (possibly empty) chunk
        if (pass)
            out[cnt] = (int)(nmc << shift);
        else
            nchunks[band] = cnt;
    }
}

// Counts of a band's entries in each 64-key range of an overflowing micro-chunk: one
// workgroup per listed (band, micro-chunk), wave w scans the keys of the band's row w that
// fall in the micro-chunk (found by binary search in the row's ascending keys).
__global__ __launch_bounds__(1024) void k_sp_fine(const uint32_t *__restrict__ k32, const int64_t *__restrict__ off,
                                                  const int *__restrict__ perm, int n, int wlog,
                                                  const int2 *__restrict__ ovf, unsigned *__restrict__ fine)
{
    const int2 pr = ovf[blockIdx.x];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = pr.x * RB + w;
    if (r >= n) return;
    const int i = perm[r];
    const uint64_t lo = (uint64_t)pr.y << wlog, hi = lo + ((uint64_t)1 << wlog);
    int64_t a = off[i], e = off[i + 1];
    while (a < e) {  // first entry with key >= lo (wave-uniform search)
        const int64_t mid = a + ((e - a) >> 1);
        if ((uint64_t)k32[mid] < lo) a = mid + 1; else e = mid;
    }
    unsigned *f = fine + (int64_t)blockIdx.x * ((int64_t)1 << (wlog - FINE_LOG));
    for (int64_t p = a + lane; p < off[i + 1]; p += 64) {
        const uint64_t k = k32[p];
        if (k >= hi) break;
        atomicAdd(f + ((k - lo) >> FINE_LOG), 1u);
    }
}

template <int LPC>
__global__ __launch_bounds__(SP_THREADS, 1) void k_sparse(const uint32_t *__restrict__ k32, const float *__restrict__ vals,
                                                         const int64_t *__restrict__ off, const int *__restrict__ perm,
                                                         const float *__restrict__ inv_norm, int n, int ulog,
                                                         const int64_t *__restrict__ cshift,
                                                         const int *__restrict__ bounds, QueueArgs q,
                                                         float *__restrict__ out, uint32_t *__restrict__ counts)
{
    // hash slot = key (low 32 bits) | union index (high 32 bits): one 8-byte read per probe
    __shared__ uint64_t htab[HSIZE];
    __shared__ __align__(16) float uval[UMAX * RB];       // row values per union entry
    __shared__ __align__(16) uint32_t upres[UMAX * RB / 4];  // presence bytes per union entry
    __shared__ int s_item, s_ucount;

    constexpr int CB = SP_THREADS / LPC;  // columns per block
    static_assert(LPC == 4 || LPC == 8, "4 or 8 lanes per column");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int sub = lane & (LPC - 1);        // lane within the column group
    const int col = tid / LPC;               // column within the block
    const uint64_t gmask = ((1ull << LPC) - 1) << (lane & ~(LPC - 1));

    // the work item and this wave's row are wave-uniform: keep them in scalar registers
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    auto uni64 = [](int64_t v) {
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
        return (int64_t)(((uint64_t)hi << 32) | lo);
    };
    int prev = -1;
    for (;;) {
        const int it = __builtin_amdgcn_readfirstlane(queue_pop_wg(q, &s_item, prev));
        if (it < 0) break;
        const int4 w = q.items[it];
        const int band = __builtin_amdgcn_readfirstlane(w.x), cblk = __builtin_amdgcn_readfirstlane(w.y);
        const int r0 = band * RB, c0 = cblk * CB;
        // this wave stages row r0 + wave (16 waves, 16 rows)
        const int srow = r0 + wv;
        const bool row_ok = srow < n;
        const int irow = row_ok ? __builtin_amdgcn_readfirstlane(perm[srow]) : 0;
        int64_t rpos = row_ok ? uni64(off[irow]) : 0;
        const int64_t rend = row_ok ? uni64(off[irow + 1]) : 0;
        // this lane group's column
        const int scol = c0 + col;
        const bool col_ok = scol < n;
        const int icol = col_ok ? perm[scol] : 0;
        int64_t cpos = col_ok ? off[icol] : 0;
        const int64_t cend = col_ok ? off[icol + 1] : 0;

        float dot[RB], comp[RB];
        uint32_t cnt[RB];
#pragma unroll
        for (int t = 0; t < RB; ++t) {
            dot[t] = 0.f;
            comp[t] = 0.f;
            cnt[t] = 0;
        }
        // band b's nch + 1 chunk boundaries (micro-chunk indices) start at cshift[b]
        const int nch = (int)(cshift[band + 1] - cshift[band]) - 1;
        const int *bnd = bounds + cshift[band];
        int prev_u = UMAX;
        for (int ch = 0; ch < nch; ++ch) {
            const uint64_t K1 = (uint64_t)bnd[ch + 1] << ulog;
            // 1. clear the table
            for (int k = tid; k < HSIZE; k += SP_THREADS) htab[k] = ~0ull;
            for (int k = tid; k < prev_u * RB / 4; k += SP_THREADS) {
                upres[k] = 0u;
                *(float4 *)&uval[4 * k] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
            if (tid == 0) s_ucount = 0;
            __syncthreads();
            // 2a. insert the band's keys of this chunk (SR entries per lane per pass, all
            // loads of a pass independent).  The first pass also loads the values and keeps
            // both for 2b, which then needs no second trip to memory when the row's entries
            // of the chunk fit in one pass (the common case).
            uint32_t rk0[SR];
            float rv0[SR];
#pragma unroll
            for (int r = 0; r < SR; ++r) {
                const int64_t p = rpos + r * 64 + lane;
                const bool ok = p < rend;
                rk0[r] = ok ? k32[p] : EMPTY;
                rv0[r] = ok ? vals[p] : 0.f;
            }
            int64_t rp = rpos;
            bool one_pass = true;
            for (int pass = 0;; ++pass) {
                uint32_t kk[SR];
#pragma unroll
                for (int r = 0; r < SR; ++r) {
                    const int64_t p = rp + r * 64 + lane;
                    kk[r] = pass == 0 ? rk0[r] : p < rend ? k32[p] : EMPTY;
                }
                int nin = 0;
#pragma unroll
                for (int r = 0; r < SR; ++r) {
                    const bool in = kk[r] != EMPTY && (uint64_t)kk[r] < K1;
                    if (in) {
                        const uint32_t key = kk[r];
                        uint32_t h = hslot(key);
                        while (true) {
                            const unsigned long long old =
                                atomicCAS((unsigned long long *)&htab[h], ~0ull, (unsigned long long)key | (~0ull << 32));
                            if (old == ~0ull) {  // claimed: the union index goes in the high half
                                ((uint32_t *)&htab[h])[1] = (uint32_t)atomicAdd(&s_ucount, 1);
                                break;
                            }
                            if ((uint32_t)old == key) break;
                            h = (h + 1) & (HSIZE - 1);
                        }
                    }
                    nin += __popcll(__ballot(in));
                }
                rp += nin;
                if (nin < SR * 64) break;
                one_pass = false;
            }
            __syncthreads();
            // 2b. scatter the row values and presence bytes
            for (int pass = 0;; ++pass) {
                uint32_t kk[SR];
                float vv[SR];
#pragma unroll
                for (int r = 0; r < SR; ++r) {
                    const int64_t p = rpos + r * 64 + lane;
                    const bool ok = p < rend;
                    if (pass == 0 && one_pass) {
                        kk[r] = rk0[r];
                        vv[r] = rv0[r];
                    } else {
                        kk[r] = ok ? k32[p] : EMPTY;
                        vv[r] = ok ? vals[p] : 0.f;
                    }
                }
                int nin = 0;
#pragma unroll
                for (int r = 0; r < SR; ++r) {
                    const bool in = kk[r] != EMPTY && (uint64_t)kk[r] < K1;
                    if (in) {
                        const uint32_t key = kk[r];
                        uint32_t h = hslot(key);
                        uint64_t t;
                        while ((uint32_t)(t = htab[h]) != key) h = (h + 1) & (HSIZE - 1);
                        const int u = (int)(t >> 32);
                        uval[u * RB + ((((wave >> 2) + u) & 3) << 2) + (wave & 3)] = vv[r];
                        atomicOr(&upres[u * (RB / 4) + (wave >> 2)], 1u << (8 * (wave & 3)));
                    }
                    nin += __popcll(__ballot(in));
                }
                rpos += nin;
                if (nin < SR * 64) break;
            }
            __syncthreads();
            prev_u = min(s_ucount, UMAX);
            // 3. stream this column's keys of the chunk and probe.  Each pass loads SR keys
            // (and values) per lane, SR*LPC consecutive entries per column, with no
            // dependence between the loads, so one memory latency covers SR*LPC entries.
            float cd[RB];
#pragma unroll
            for (int t = 0; t < RB; ++t) cd[t] = 0.f;
            uint32_t pk[RB / 4] = {0u, 0u, 0u, 0u};
            int since = 0;
            while (true) {
                uint32_t kk[SR];
                float vv[SR];
#pragma unroll
                for (int r = 0; r < SR; ++r) {
                    const int64_t p = cpos + r * LPC + sub;
                    const bool ok = p < cend;
                    kk[r] = ok ? k32[p] : EMPTY;
                    vv[r] = ok ? vals[p] : 0.f;
                }
                int nin = 0;
#pragma unroll
                for (int r = 0; r < SR; ++r) {
                    const bool in = kk[r] != EMPTY && (uint64_t)kk[r] < K1;
                    if (in) {
                        const uint32_t key = kk[r];
                        const float vj = vv[r];
                        uint32_t h = hslot(key);
                        uint64_t t;
                        while ((uint32_t)(t = htab[h]) != key && (uint32_t)t != EMPTY) h = (h + 1) & (HSIZE - 1);
                        if ((uint32_t)t == key) {
                            const int u = (int)(t >> 32);
                            const float4 *uv = (const float4 *)&uval[u * RB];
#pragma unroll
                            for (int qd = 0; qd < RB / 4; ++qd) {
                                const float4 v4 = uv[(qd + u) & 3];  // rows 4 qd .. 4 qd + 3 (swizzled)
                                cd[4 * qd] = fmaf(v4.x, vj, cd[4 * qd]);
                                cd[4 * qd + 1] = fmaf(v4.y, vj, cd[4 * qd + 1]);
                                cd[4 * qd + 2] = fmaf(v4.z, vj, cd[4 * qd + 2]);
                                cd[4 * qd + 3] = fmaf(v4.w, vj, cd[4 * qd + 3]);
                            }
                            const uint4 pr = *(const uint4 *)&upres[u * (RB / 4)];
                            pk[0] += pr.x;
                            pk[1] += pr.y;
                            pk[2] += pr.z;
                            pk[3] += pr.w;
                            if (++since == 255) {  // unpack before a byte counter can wrap
#pragma unroll
                                for (int t = 0; t < RB; ++t) cnt[t] += (pk[t >> 2] >> (8 * (t & 3))) & 0xFFu;
                                pk[0] = pk[1] = pk[2] = pk[3] = 0u;
                                since = 0;
                            }
                        }
                    }
                    nin += __popcll(__ballot(in) & gmask);
                }
                cpos += nin;
                if (nin < SR * LPC) break;
            }

#pragma unroll
            for (int t = 0; t < RB; ++t) {
                cnt[t] += (pk[t >> 2] >> (8 * (t & 3))) & 0xFFu;
                // compensated add of the chunk sum
                const float y = cd[t] - comp[t];
                const float s = dot[t] + y;
                comp[t] = (s - dot[t]) - y;
                dot[t] = s;
            }
            __syncthreads();
        }
        // combine the LPC lanes of each column (fixed butterfly) and write
#pragma unroll
        for (int t = 0; t < RB; ++t) {
#pragma unroll
            for (int o = 1; o < LPC; o <<= 1) {
                dot[t] += __shfl_xor(dot[t], o);
                cnt[t] += __shfl_xor(cnt[t], o);
            }
        }
        if (col_ok) {
#pragma unroll
            for (int t = 0; t < RB; ++t) {
                if (t / (RB / LPC) != sub) continue;  // lane sub writes rows RB/LPC * sub ..
                const int srow2 = r0 + t;
                if (srow2 >= n || srow2 >= scol) continue;
                const int a = perm[srow2], b = icol;
                const int64_t i = min(a, b), j = max(a, b);
                const int64_t idx = i * n - i * (i + 1) / 2 + (j - i - 1);
                out[idx] = dot[t] * inv_norm[a] * inv_norm[b];
                if (counts) counts[idx] = cnt[t];
            }
        }
    }
}

}  // namespace

rocket_status sp_prepare(rocket_ctx *ctx, const rocket_items *it, int64_t n, hipStream_t s)
{
    SpState &sp = ctx->sp;
    sp.valid = false;
    if (n > 0 && (!it->offsets || !it->keys || !it->vals)) return fail(ctx, ROCKET_E_INVALID, "offsets/keys/vals NULL");
    if (n >= (1 << 30)) return fail(ctx, ROCKET_E_INVALID, "n too large");
    sp.n = n;
    sp.offsets = it->offsets;
    sp.keys = it->keys;
    sp.vals = it->vals;
    sp.h_offsets.assign((size_t)n + 1, 0);
    if (n > 0) {
        RK_HIP(hipMemcpyAsync(sp.h_offsets.data(), it->offsets, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s));
        RK_HIP(hipStreamSynchronize(s));
    }
    if (sp.h_offsets[0] != 0) return fail(ctx, ROCKET_E_INVALID, "offsets[0] != 0");
    for (int64_t i = 0; i < n; ++i)
        if (sp.h_offsets[i + 1] < sp.h_offsets[i]) return fail(ctx, ROCKET_E_INVALID, "offsets decrease");
    sp.total = sp.h_offsets[n];
    if (n < 2) {
        sp.tiles = 0;
        sp.valid = true;
        return ROCKET_OK;
    }
    // size sort
    sp.perm.resize(n);
    std::iota(sp.perm.begin(), sp.perm.end(), 0);
    std::stable_sort(sp.perm.begin(), sp.perm.end(), [&](int a, int b) {
        return sp.h_offsets[a + 1] - sp.h_offsets[a] > sp.h_offsets[b + 1] - sp.h_offsets[b];
    });
    // 4 lanes per column (256-column work items, half as many band-table builds) once that
    // still leaves at least 8 work items per CU, else 8 lanes (128-column work items)
    const int64_t nbands = (n + RB - 1) / RB;
    const int64_t wide_items = nbands * ((n + 255) / 256) / 2 + nbands;
    sp.lpc = ctx->opt[ROCKET_OPT_SP_LANES] ? (int)ctx->opt[ROCKET_OPT_SP_LANES]
             : wide_items >= 8 * (int64_t)ctx->num_cu ? 4
                                                       : 8;
    const int64_t CB = SP_THREADS / sp.lpc;
    const int64_t nblk = (n + CB - 1) / CB;
    // device buffers: u32 keys; meta = flags (2 words) | inverse norms | sorted-position -> item
    void *kp = nullptr, *meta = nullptr;
    RK_TRY(ws_get(ctx, WS_SP_KEYS, sizeof(uint32_t) * (size_t)std::max<int64_t>(sp.total, 1), &kp));
    RK_TRY(ws_get(ctx, WS_SP_META, 256 + (sizeof(float) + sizeof(int)) * (size_t)n, &meta));
    unsigned *flags = (unsigned *)meta;  // [0] error flags, [1] max key
    float *inv_norm = (float *)((char *)meta + 256);
    int *perm = (int *)(inv_norm + n);
    RK_HIP(hipMemsetAsync(flags, 0, 8, s));
    RK_HIP(hipMemcpyAsync(perm, sp.perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_sp_validate, dim3((unsigned)n), dim3(256), 0, s, it->keys, it->vals, it->offsets, (int)n,
                       (uint32_t *)kp, inv_norm, flags, flags + 1);
    RK_HIP(hipGetLastError());
    unsigned hf[2] = {0, 0};
    RK_HIP(hipMemcpyAsync(hf, flags, 8, hipMemcpyDeviceToHost, s));
    RK_HIP(hipStreamSynchronize(s));
    if (hf[0] & FLAG_RANGE) return fail(ctx, ROCKET_E_KEYRANGE, "a key is outside [0, 2^32 - 1)");
    if (hf[0] & FLAG_UNSORTED) return fail(ctx, ROCKET_E_UNSORTED, "keys of an item are not strictly ascending");
    // micro-chunk width 2^wlog: at most 2^20 micro-chunks and a histogram of at most 4 GiB
    const uint64_t maxkey = hf[1];
    int wlog = 0;
    while (((maxkey >> wlog) + 1) > (uint64_t)(1 << 20)) ++wlog;
    while ((uint64_t)nbands * ((maxkey >> wlog) + 1) * 4 > ((uint64_t)4 << 30)) ++wlog;
    while (ctx->opt[ROCKET_OPT_SP_CHUNK] > ((int64_t)1 << wlog)) ++wlog;  // caller's lower bound
    // keys are u32, so a shift by wlog must stay below 32 (set_option caps the width at 2^31)
    if (wlog > 31) return fail(ctx, ROCKET_E_INVALID, "sparse micro-chunk width above 2^31");
    const int64_t nmc = (int64_t)(maxkey >> wlog) + 1;
    const int ulog = std::min(wlog, FINE_LOG), shift = wlog - ulog;  // bounds in units of 2^ulog keys
    // WS_SP_CHUNKS: histogram [nbands][nmc] | chunk counts [nbands] | overflow count (+pad) |
    // overflow list [OVF_MAX] (band, micro-chunk)
    const size_t hist_bytes = sizeof(unsigned) * (size_t)(nbands * nmc);
    const size_t list_off = hist_bytes + sizeof(int) * (size_t)(nbands + 2);
    void *hp = nullptr;
    RK_TRY(ws_get(ctx, WS_SP_CHUNKS, list_off + sizeof(int2) * OVF_MAX, &hp));
    unsigned *hist = (unsigned *)hp;
    int *nchunks = (int *)(hist + nbands * nmc);
    unsigned *ovf_n = (unsigned *)(nchunks + nbands);
    int2 *ovf = (int2 *)((char *)hp + list_off);
    RK_HIP(hipMemsetAsync(hist, 0, list_off, s));
    hipLaunchKernelGGL(k_sp_hist, dim3((unsigned)n), dim3(256), 0, s, (const uint32_t *)kp, it->offsets,
                       (const int *)perm, (int)n, wlog, nmc, hist);
    RK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sp_cut, dim3((unsigned)nbands), dim3(256), 0, s, (const unsigned *)hist, nmc, 0, shift,
                       nchunks, (const int64_t *)nullptr, (int *)nullptr, flags, ovf, ovf_n, (const int *)nullptr);
    RK_HIP(hipGetLastError());
    std::vector<int> hn(nbands);
    unsigned novf = 0;
    RK_HIP(hipMemcpyAsync(hn.data(), nchunks, sizeof(int) * nbands, hipMemcpyDeviceToHost, s));
    RK_HIP(hipMemcpyAsync(&novf, ovf_n, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    RK_HIP(hipStreamSynchronize(s));
    // Bands with a micro-chunk holding more than UMAX of their entries are cut on the host at
    // 64-key granularity from a finer histogram of just those micro-chunks.
    std::vector<int> host_cut(nbands, 0);
    std::vector<std::vector<int>> hb(nbands);  // host-cut bounds (units), per band
    if (novf > 0) {
        if (novf > (unsigned)OVF_MAX)
            return fail(ctx, ROCKET_E_UNSUPPORTED,
                        "more than " + std::to_string(OVF_MAX) + " micro-chunks hold more than " +
                            std::to_string(UMAX) + " entries of one 16-item band");
        const int64_t nb = (int64_t)1 << shift;  // 64-key ranges per micro-chunk
        if ((int64_t)novf * nb * 4 > ((int64_t)1 << 30))
            return fail(ctx, ROCKET_E_UNSUPPORTED, "dense key ranges too wide for the fine histogram (1 GiB)");
        std::vector<int2> lst(novf);
        RK_HIP(hipMemcpyAsync(lst.data(), ovf, sizeof(int2) * novf, hipMemcpyDeviceToHost, s));
        RK_HIP(hipStreamSynchronize(s));
        std::sort(lst.begin(), lst.end(), [](int2 a, int2 b) { return a.x != b.x ? a.x < b.x : a.y < b.y; });
        void *fp = nullptr;
        RK_TRY(ws_get(ctx, WS_SP_FINE, (size_t)(novf * nb * 4), &fp));
        RK_HIP(hipMemcpyAsync(ovf, lst.data(), sizeof(int2) * novf, hipMemcpyHostToDevice, s));
        RK_HIP(hipMemsetAsync(fp, 0, (size_t)(novf * nb * 4), s));
        hipLaunchKernelGGL(k_sp_fine, dim3(novf), dim3(1024), 0, s, (const uint32_t *)kp, it->offsets,
                           (const int *)perm, (int)n, wlog, (const int2 *)ovf, (unsigned *)fp);
        RK_HIP(hipGetLastError());
        std::vector<unsigned> fine((size_t)(novf * nb)), row((size_t)nmc);
        RK_HIP(hipMemcpyAsync(fine.data(), fp, sizeof(unsigned) * fine.size(), hipMemcpyDeviceToHost, s));
        RK_HIP(hipStreamSynchronize(s));
        for (size_t q = 0; q < lst.size();) {
            const int b = lst[q].x;
            RK_HIP(hipMemcpy(row.data(), hist + (int64_t)b * nmc, sizeof(unsigned) * nmc, hipMemcpyDeviceToHost));
            // greedy: close a chunk before the unit whose entries would take it past UMAX
            std::vector<int> &bd = hb[b];
            bd.assign(1, 0);
            uint64_t acc = 0;
            auto take = [&](uint64_t c, int64_t unit) {
                if (acc + c > (uint64_t)UMAX && acc > 0) {
                    bd.push_back((int)unit);
                    acc = 0;
                }
                acc += c;
            };
            for (int64_t m = 0; m < nmc; ++m) {
                if (q < lst.size() && lst[q].x == b && lst[q].y == m) {
                    for (int64_t f = 0; f < nb; ++f) take(fine[q * nb + f], (m << shift) + f);
                    ++q;
                } else {
                    take(row[m], m << shift);
                }
            }
            bd.push_back((int)(nmc << shift));
            hn[b] = (int)bd.size() - 1;
            host_cut[b] = 1;
        }
    }
    // band b's nch_b + 1 boundaries live at cshift[b] = sum_{c<b} (nch_c + 1); the host-cut
    // flags follow cshift in the same buffer
    std::vector<int64_t> cshift(nbands + 1, 0);
    for (int64_t b = 0; b < nbands; ++b) cshift[b + 1] = cshift[b] + hn[b] + 1;
    void *csp = nullptr, *bp = nullptr;
    RK_TRY(ws_get(ctx, WS_SP_CSHIFT, sizeof(int64_t) * (size_t)(nbands + 1) + sizeof(int) * (size_t)nbands, &csp));
    RK_TRY(ws_get(ctx, WS_SP_BOUNDS, sizeof(int) * (size_t)cshift[nbands], &bp));
    int *dcut = (int *)((int64_t *)csp + nbands + 1);
    RK_HIP(hipMemcpyAsync(csp, cshift.data(), sizeof(int64_t) * (nbands + 1), hipMemcpyHostToDevice, s));
    RK_HIP(hipMemcpyAsync(dcut, host_cut.data(), sizeof(int) * nbands, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_sp_cut, dim3((unsigned)nbands), dim3(256), 0, s, (const unsigned *)hist, nmc, 1, shift,
                       nchunks, (const int64_t *)csp, (int *)bp, flags, ovf, ovf_n, (const int *)dcut);
    RK_HIP(hipGetLastError());
    for (int64_t b = 0; b < nbands; ++b)
        if (host_cut[b])
            RK_HIP(hipMemcpyAsync((int *)bp + cshift[b], hb[b].data(), sizeof(int) * hb[b].size(),
                                  hipMemcpyHostToDevice, s));
    RK_HIP(hipStreamSynchronize(s));  // the staging vectors go out of scope
    sp.wlog = wlog;
    sp.ulog = ulog;
    sp.cshift = (const int64_t *)csp;
    sp.bounds = (const int *)bp;
    sp.inv_norm = inv_norm;
    sp.dperm = perm;
    sp.k32 = (const uint32_t *)kp;
    sp.nchunks_total = cshift[nbands] - nbands;
    // tiles: (band, column block) with at least one pair a < b; cost = streamed entries
    std::vector<int64_t> bnnz(nblk, 0), rnnz(nbands, 0);
    for (int64_t s2 = 0; s2 < n; ++s2) {
        const int64_t c = sp.h_offsets[sp.perm[s2] + 1] - sp.h_offsets[sp.perm[s2]];
        bnnz[s2 / CB] += c;
        rnnz[s2 / RB] += c;
    }
    std::vector<int4> raw;
    std::vector<double> cost;
    for (int64_t b = 0; b < nbands; ++b)
        for (int64_t c = 0; c < nblk; ++c) {
            const int64_t rlo = b * RB, chi = std::min<int64_t>(n, (c + 1) * CB) - 1;
            if (rlo >= chi) continue;  // no pair a < b
            raw.push_back(make_int4((int)b, (int)c, 0, (int)raw.size()));
            cost.push_back((double)bnnz[c] + (double)rnnz[b] + 2048.0 * hn[b]);
        }
    plan_lpt(raw, cost, MAX_SEG, ctx->h_items, ctx->h_seg);
    if (ctx->opt[ROCKET_OPT_QUEUE_ORDER] == 1) shuffle_items(ctx->h_items, ctx->h_seg, (uint64_t)ctx->opt[ROCKET_OPT_SEED]);
    if (ctx->opt[ROCKET_OPT_QUEUE_ORDER] == 2) single_segment(ctx->h_seg, (int64_t)ctx->h_items.size());
    sp.tiles = (int64_t)ctx->h_items.size();
    if (sp.tiles) RK_TRY(upload_queue(ctx, s, &sp.qa));
    ctx->queue_owner = QOWN_SP;
    ctx->stats.tiles = sp.tiles;
    ctx->stats.work_items = sp.tiles;
    ctx->stats.tile = RB;
    ctx->stats.kchunk = sp.nchunks_total;
    ctx->stats.variant = sp.lpc;
    sp.valid = true;
    return ROCKET_OK;
}

rocket_status sp_compare(rocket_ctx *ctx, float *out, uint32_t *counts, hipStream_t s)
{
    SpState &sp = ctx->sp;
    if (!sp.valid) return fail(ctx, ROCKET_E_STATE, "sparse set not prepared");
    if (sp.n < 2 || sp.tiles == 0) return ROCKET_OK;
    if (ctx->queue_owner != QOWN_SP) return fail(ctx, ROCKET_E_STATE, "queue was replanned by another prepare");
    RK_TRY(reset_queue(ctx, s, sp.qa));
    const void *kern = sp.lpc == 4 ? (const void *)&k_sparse<4> : (const void *)&k_sparse<8>;
    const int grid = auto_grid(ctx, kern, SP_THREADS, 0, sp.tiles);
    ctx->stats.grid = grid;
    RK_TRY(timing_begin(ctx, s));
    if (sp.lpc == 4)
        hipLaunchKernelGGL(k_sparse<4>, dim3(grid), dim3(SP_THREADS), 0, s, sp.k32, sp.vals, sp.offsets, sp.dperm,
                           sp.inv_norm, (int)sp.n, sp.ulog, sp.cshift, sp.bounds, sp.qa, out, counts);
    else
        hipLaunchKernelGGL(k_sparse<8>, dim3(grid), dim3(SP_THREADS), 0, s, sp.k32, sp.vals, sp.offsets, sp.dperm,
                           sp.inv_norm, (int)sp.n, sp.ulog, sp.cshift, sp.bounds, sp.qa, out, counts);
    RK_HIP(hipGetLastError());
    RK_TRY(timing_end(ctx, s));
    return ROCKET_OK;
}

}  // namespace rk
