// Composition vectors of protein K-strings on the GPU (Section V-B pre-process), the
// K-string composition approach of Qi, Wang and Hao:
//   f(s) = n(s) / N_K over all windows of K residues inside one protein,
//   f0(s) = f(s_1..s_{K-1}) f(s_2..s_K) / f(s_2..s_{K-1}),   a(s) = (f(s) - f0(s)) / f0(s),
// one entry per K-string that occurs, keyed by its base-20 code, keys ascending.
//
// Species are processed in groups.  Per species the counts of K-, (K-1)- and (K-2)-strings
// are dense arrays over the code space (20^K u32; 256 MB at K = 6).  The K array is filled
// with atomics, one thread per window start; the shorter arrays get atomics only for the
// windows at a protein end and are then folded from the longer ones (a (K-1)-string's count
// is the sum over the 20 K-strings that extend it, plus its protein-end windows), the K ->
// K-1 fold also counting the non-zero codes of every 1024-code chunk.  A scan of the chunk
// counts gives every chunk its output base; an emit pass streams the dense K
// array chunk by chunk (one wave per chunk), ranks the non-zero codes with a wave prefix
// sum (so keys come out ascending), writes key and a(s) (FP64, rounded once to f32) and
// writes zeros back, so the K array is clean for the next group.
#include <algorithm>
#include <vector>

#include "common.hpp"

namespace rk {
namespace {

constexpr int CV_ALPHA = 20;
constexpr int CV_CHLOG = 10;  // 1024 codes per chunk
constexpr int CV_CH = 1 << CV_CHLOG;
constexpr int CV_GROUP_MAX = 64;  // species per group (one grid row each)

__host__ __device__ inline int64_t ipow20(int k)
{
    int64_t v = 1;
    for (int i = 0; i < k; ++i) v *= CV_ALPHA;
    return v;
}

__global__ void k_cv_zero(uint32_t *__restrict__ p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Base-20 code of the window of k residues starting at p (all < 20), else -1.
__device__ inline int64_t window_code(const uint8_t *__restrict__ res, int64_t p, int64_t end, int k)
{
    if (p + k > end) return -1;
    int64_t c = 0;
    for (int t = 0; t < k; ++t) {
        const int r = res[p + t];
        if (r >= CV_ALPHA) return -1;
        c = c * CV_ALPHA + r;
    }
    return c;
}

// grid (x, group size): blockIdx.y = species s0 + y, threads stride over its window starts.
// tot[3*y + {0,1,2}] accumulate N_K, N_{K-1}, N_{K-2}.
__global__ __launch_bounds__(256) void k_cv_count(const uint8_t *__restrict__ res, const int64_t *__restrict__ off,
                                                  int64_t s0, int K, uint32_t *__restrict__ cK,
                                                  uint32_t *__restrict__ c1, uint32_t *__restrict__ c2,
                                                  unsigned long long *__restrict__ tot)
{
    const int y = blockIdx.y;
    const int64_t b = off[s0 + y], e = off[s0 + y + 1];
    const int64_t szK = ipow20(K), sz1 = szK / CV_ALPHA, sz2 = sz1 / CV_ALPHA;
    uint32_t *cKy = cK + y * szK, *c1y = c1 + y * sz1, *c2y = c2 + y * sz2;
    unsigned nk = 0, n1 = 0, n2 = 0;
    for (int64_t p = b + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < e; p += (int64_t)gridDim.x * blockDim.x) {
        // Only K-windows are counted here; a shorter window that extends to a valid longer
        // one is counted when the (K-1)- and (K-2)-string arrays are folded from the longer
        // counts, so only windows at a protein end need their own atomic.
        const int64_t w2 = window_code(res, p, e, K - 2);
        if (w2 < 0) continue;  // a shorter window is a prefix of the longer ones
        ++n2;
        const int r1 = p + K - 1 <= e ? res[p + K - 2] : CV_ALPHA;
        if (r1 >= CV_ALPHA) {
            atomicAdd(c2y + w2, 1u);
            continue;
        }
        const int64_t w1 = w2 * CV_ALPHA + r1;
        ++n1;
        const int rK = p + K <= e ? res[p + K - 1] : CV_ALPHA;
        if (rK >= CV_ALPHA) {
            atomicAdd(c1y + w1, 1u);
            continue;
        }
        atomicAdd(cKy + w1 * CV_ALPHA + rK, 1u);
        ++nk;
    }
    // wave sums, one atomic per wave and total
    for (int o = 32; o > 0; o >>= 1) {
        nk += __shfl_xor(nk, o);
        n1 += __shfl_xor(n1, o);
        n2 += __shfl_xor(n2, o);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(tot + 3 * y, (unsigned long long)nk);
        atomicAdd(tot + 3 * y + 1, (unsigned long long)n1);
        atomicAdd(tot + 3 * y + 2, (unsigned long long)n2);
    }
}

// K -> K-1 fold and the occupancy of the K array's chunks in one pass over it.  One wave per
// block of 5120 K-codes (five 1024-code chunks = the 20 extensions of 256 (K-1)-codes).
// Lane l reads 16-byte vectors j * 64 + l, j < 20, so every load is one contiguous 1 KB run;
// vector j lies in chunk j / 4 of the block, so the non-zero counts per chunk are register
// sums reduced across the wave.  The vector sums go to LDS, where lane l adds up the five
// vectors of (K-1)-codes l, l + 64, l + 128 and l + 192.  grid (blocks / 4, group size).
constexpr int CV_FOLD_W = 256;  // (K-1)-codes per block
__global__ __launch_bounds__(256) void k_cv_fold_k(const uint32_t *__restrict__ cK, uint32_t *__restrict__ c1,
                                                   uint32_t *__restrict__ chunk_cnt, int64_t sz1, int64_t nchunks)
{
    constexpr int NV = CV_FOLD_W * CV_ALPHA / 4;  // 16-byte vectors per block (1280)
    constexpr int NJ = NV / 64;                   // per lane (20)
    constexpr int NCB = NJ / 4;                   // chunks per block (5)
    static_assert(NV % 64 == 0 && NJ % 4 == 0 && 4 * 4 * 64 == CV_CH, "four vectors of each lane per chunk");
    __shared__ uint32_t vsum[4][NV];
    const int y = blockIdx.y, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t blk = (int64_t)blockIdx.x * 4 + wave;
    const int64_t w0 = blk * CV_FOLD_W;
    if (w0 >= sz1) return;
    const int64_t nvalid = std::min<int64_t>(CV_FOLD_W, sz1 - w0) * (CV_ALPHA / 4);  // vectors of this block
    const uint4 *cl = (const uint4 *)(cK + (y * sz1 + w0) * CV_ALPHA);
    unsigned nz[NCB];
#pragma unroll
    for (int c = 0; c < NCB; ++c) nz[c] = 0u;
    uint4 v[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int e = j * 64 + lane;
        v[j] = e < nvalid ? cl[e] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        nz[j / 4] += (v[j].x != 0u) + (v[j].y != 0u) + (v[j].z != 0u) + (v[j].w != 0u);
        vsum[wave][j * 64 + lane] = v[j].x + v[j].y + v[j].z + v[j].w;
    }
#pragma unroll
    for (int c = 0; c < NCB; ++c)
        for (int o = 32; o > 0; o >>= 1) nz[c] += __shfl_xor(nz[c], o);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint32_t *cs = c1 + y * sz1;
#pragma unroll
    for (int q = 0; q < CV_FOLD_W / 64; ++q) {
        const int wl = q * 64 + lane;  // (K-1)-code within the block: vectors 5 wl .. 5 wl + 4
        if (w0 + wl < sz1) {
            const uint32_t *p = &vsum[wave][5 * wl];
            cs[w0 + wl] += p[0] + p[1] + p[2] + p[3] + p[4];
        }
    }
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
        const int64_t ch = blk * NCB + c;
        if (lane == 0 && ch < nchunks) chunk_cnt[y * nchunks + ch] = nz[c];
    }
}

// c_short[w] += sum_a c_long[20 w + a]: every window of the longer length starts with a
// valid window of the shorter one.  grid (x, group size), one thread per shorter string.
__global__ __launch_bounds__(256) void k_cv_fold(const uint32_t *__restrict__ c_long, uint32_t *__restrict__ c_short,
                                                 int64_t n_short)
{
    const int y = blockIdx.y;
    const uint32_t *cl = c_long + y * n_short * CV_ALPHA;
    uint32_t *cs = c_short + y * n_short;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < n_short; w += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t *q = cl + w * CV_ALPHA;  // 80 bytes, 16-byte aligned
        uint32_t t = 0;
#pragma unroll
        for (int a = 0; a < CV_ALPHA; a += 4) {
            const uint4 v = *(const uint4 *)(q + a);
            t += v.x + v.y + v.z + v.w;
        }
        cs[w] += t;
    }
}

// One workgroup per species of the group: exclusive scan of its chunk counts in place,
// total into nnz[y].
__global__ __launch_bounds__(1024) void k_cv_scan(uint32_t *__restrict__ chunk_cnt, int64_t nchunks,
                                                  int64_t *__restrict__ nnz)
{
    __shared__ int64_t part[1024];
    uint32_t *c = chunk_cnt + blockIdx.x * nchunks;
    const int64_t per = (nchunks + 1023) / 1024;
    const int64_t a = threadIdx.x * per, z = std::min<int64_t>(nchunks, a + per);
    int64_t s = 0;
    for (int64_t i = a; i < z; ++i) s += c[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive Hillis-Steele scan of the thread sums
        const int64_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
    for (int64_t i = a; i < z; ++i) {
        const uint32_t v = c[i];
        c[i] = (uint32_t)run;
        run += v;
    }
    if (threadIdx.x == 1023) nnz[blockIdx.x] = part[1023];
}

// Output offsets of the group's species, in order (one thread; the group is small).
__global__ void k_cv_base(const int64_t *__restrict__ nnz, int G, int64_t s0, int64_t *__restrict__ cv_off)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (s0 == 0) cv_off[0] = 0;
    int64_t run = cv_off[s0];
    for (int y = 0; y < G; ++y) {
        run += nnz[y];
        cv_off[s0 + y + 1] = run;
    }
}

// grid (chunks / 4, group size), 256 threads: one wave per 1024-code chunk, 16 codes per lane
// (four 16-byte loads); a wave prefix sum ranks the non-zero codes (so no workgroup barrier)
// and places them, in code order, in the wave's LDS list; the lanes then take the list's
// entries one each, so the lookups and stores of all of them are in flight together.
__global__ __launch_bounds__(256) void k_cv_emit(uint32_t *__restrict__ cK, const uint32_t *__restrict__ c1,
                                                 const uint32_t *__restrict__ c2,
                                                 const uint32_t *__restrict__ chunk_base, int64_t nchunks,
                                                 const unsigned long long *__restrict__ tot,
                                                 const int64_t *__restrict__ cv_off, int64_t s0, int K,
                                                 int64_t *__restrict__ keys, float *__restrict__ vals,
                                                 int64_t capacity, int *__restrict__ overflow)
{
    __shared__ uint16_t lcode[4][CV_CH];  // per wave: offset of the code in the chunk
    __shared__ uint32_t lcnt[4][CV_CH];   // and its count
    const int y = blockIdx.y;
    const int wave = threadIdx.x >> 6;
    const int64_t chunk = (int64_t)blockIdx.x * 4 + wave;
    if (chunk >= nchunks) return;
    const int lane = threadIdx.x & 63;
    const int64_t szK = ipow20(K), sz1 = szK / CV_ALPHA, sz2 = sz1 / CV_ALPHA;
    uint32_t *cKy = cK + y * szK;
    const uint32_t *c1y = c1 + y * sz1, *c2y = c2 + y * sz2;
    const int64_t code0 = (chunk << CV_CHLOG) + 16 * lane;
    uint32_t v[16];
    if (code0 + 15 < szK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 u = *(const uint4 *)(cKy + code0 + 4 * q);
            v[4 * q] = u.x;
            v[4 * q + 1] = u.y;
            v[4 * q + 2] = u.z;
            v[4 * q + 3] = u.w;
        }
    } else {
#pragma unroll
        for (int t = 0; t < 16; ++t) v[t] = code0 + t < szK ? cKy[code0 + t] : 0u;
    }
    int mine = 0;
#pragma unroll
    for (int t = 0; t < 16; ++t) mine += v[t] != 0u;
    int incl = mine;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    const int total = __shfl(incl, 63);
    if (total == 0) return;
    int slot = incl - mine;
#pragma unroll
    for (int t = 0; t < 16; ++t)
        if (v[t] != 0u) {
            lcode[wave][slot] = (uint16_t)(16 * lane + t);
            lcnt[wave][slot] = v[t];
            ++slot;
        }
    // the list is written and read by this wave only: a wave-wide LDS fence suffices
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double NK = (double)tot[3 * y], N1 = (double)tot[3 * y + 1], N2 = (double)tot[3 * y + 2];
    const int64_t base = cv_off[s0 + y] + chunk_base[y * nchunks + chunk];
    for (int e = lane; e < total; e += 64) {
        const int64_t code = (chunk << CV_CHLOG) + lcode[wave][e];
        const uint32_t cnt = lcnt[wave][e];
        const int64_t pos = base + e;
        if (pos >= capacity) {
            *overflow = 1;
        } else {
            const int64_t pre = code / CV_ALPHA, suf = code % sz1, mid = pre % sz2;
            const double f = (double)cnt / NK;
            const double f0 = ((double)c1y[pre] / N1) * ((double)c1y[suf] / N1) / ((double)c2y[mid] / N2);
            keys[pos] = code;
            vals[pos] = (float)((f - f0) / f0);
        }
        cKy[code] = 0u;  // leave the K array clean for the next group
    }
}

}  // namespace

rocket_status cv_build(rocket_ctx *ctx, const uint8_t *res, const int64_t *offsets, int64_t n, int K,
                       int64_t *cv_off, int64_t *keys, float *vals, int64_t capacity, hipStream_t s)
{
    if (n < 0) return fail(ctx, ROCKET_E_INVALID, "n < 0");
    if (K < 3 || K > 6) return fail(ctx, ROCKET_E_UNSUPPORTED, "K must be 3..6");
    if (!cv_off || (n > 0 && (!offsets || !res))) return fail(ctx, ROCKET_E_INVALID, "NULL pointer");
    if (capacity < 0) return fail(ctx, ROCKET_E_INVALID, "capacity < 0");
    std::vector<int64_t> h_off((size_t)n + 1, 0);
    if (n > 0) {
        RK_HIP(hipMemcpyAsync(h_off.data(), offsets, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s));
        RK_HIP(hipStreamSynchronize(s));
    }
    if (h_off[0] != 0) return fail(ctx, ROCKET_E_INVALID, "offsets[0] != 0");
    for (int64_t i = 0; i < n; ++i)
        if (h_off[i + 1] < h_off[i]) return fail(ctx, ROCKET_E_INVALID, "offsets decrease");
    if (capacity > 0 && (!keys || !vals)) return fail(ctx, ROCKET_E_INVALID, "keys or vals is NULL");
    ctx->stats.cache_loads = 0;
    if (n == 0) {
        const int64_t zero = 0;
        RK_HIP(hipMemcpyAsync(cv_off, &zero, sizeof(int64_t), hipMemcpyHostToDevice, s));
        RK_HIP(hipStreamSynchronize(s));
        return ROCKET_OK;
    }
    const int64_t szK = ipow20(K), sz1 = szK / CV_ALPHA, sz2 = sz1 / CV_ALPHA;
    const int64_t nchunks = (szK + CV_CH - 1) / CV_CH;
    const int64_t per_species = 4 * (szK + sz1 + sz2 + nchunks) + 8 * 4;
    // Species per group: as many as fit, up to 64 (more species per launch keep more of the
    // chip busy: at K = 6 every step from 1 to 63 species per group measured faster), within
    // a quarter of the free device memory and half the workspace cap, with the species spread
    // evenly over the groups.
    size_t free_b = 0, total_b = 0;
    RK_HIP(hipMemGetInfo(&free_b, &total_b));
    int64_t budget = (int64_t)(free_b / 4) + (int64_t)ctx->ws[WS_CV_K].bytes + (int64_t)ctx->ws[WS_CV_AUX].bytes;
    if (ctx->opt[ROCKET_OPT_WORKSPACE_CAP] > 0) budget = std::min<int64_t>(budget, ctx->opt[ROCKET_OPT_WORKSPACE_CAP] / 2);
    const int64_t gmax = std::max<int64_t>(1, std::min<int64_t>({n, (int64_t)CV_GROUP_MAX, budget / per_species}));
    const int64_t ngroups = (n + gmax - 1) / gmax;
    const int64_t G = (n + ngroups - 1) / ngroups;
    CvState &cs = ctx->cv;
    void *pK = nullptr, *p1 = nullptr, *p2 = nullptr, *pch = nullptr, *ptot = nullptr, *pnnz = nullptr,
         *pflag = nullptr;
    const bool fresh = !cs.clean || cs.K != K || cs.G < G || ctx->ws[WS_CV_K].ptr == nullptr;
    RK_TRY(ws_get(ctx, WS_CV_K, (size_t)(4 * G * szK), &pK));
    RK_TRY(ws_get(ctx, WS_CV_AUX, (size_t)(4 * G * (sz1 + sz2 + nchunks) + 8 * 4 * G + 64), &p1));
    p2 = (char *)p1 + 4 * G * sz1;
    pch = (char *)p2 + 4 * G * sz2;
    ptot = (char *)pch + 4 * G * nchunks;  // 3 x u64 per species, then nnz, then the flag
    ptot = (void *)(((uintptr_t)ptot + 7) & ~(uintptr_t)7);
    pnnz = (char *)ptot + 8 * 3 * G;
    pflag = (char *)pnnz + 8 * G;
    cs.clean = false;
    if (fresh) {
        hipLaunchKernelGGL(k_cv_zero, dim3(4096), dim3(256), 0, s, (uint32_t *)pK, G * szK);
        RK_HIP(hipGetLastError());
    }
    cs.K = K;
    cs.G = G;
    hipLaunchKernelGGL(k_cv_zero, dim3(1), dim3(64), 0, s, (uint32_t *)pflag, (int64_t)1);
    RK_TRY(timing_begin(ctx, s));
    for (int64_t s0 = 0; s0 < n; s0 += G) {
        const int g = (int)std::min<int64_t>(G, n - s0);
        int64_t longest = 0;
        for (int y = 0; y < g; ++y) longest = std::max(longest, h_off[s0 + y + 1] - h_off[s0 + y]);
        // clear the small count arrays, chunk counts and totals (the K array is kept clean)
        const int64_t aux_words = (int64_t)g * (sz1 + sz2 + nchunks);
        hipLaunchKernelGGL(k_cv_zero, dim3((unsigned)std::min<int64_t>(4096, (aux_words + 255) / 256)), dim3(256), 0,
                           s, (uint32_t *)p1, (int64_t)G * (sz1 + sz2 + nchunks));
        hipLaunchKernelGGL(k_cv_zero, dim3(1), dim3(256), 0, s, (uint32_t *)ptot, (int64_t)(2 * 3 * G));
        if (longest > 0) {
            const unsigned bx = (unsigned)std::min<int64_t>(2048, (longest + 255) / 256);
            hipLaunchKernelGGL(k_cv_count, dim3(bx, g), dim3(256), 0, s, res, offsets, s0, K, (uint32_t *)pK,
                               (uint32_t *)p1, (uint32_t *)p2, (unsigned long long *)ptot);
        }
        const int64_t fblocks = (sz1 + CV_FOLD_W - 1) / CV_FOLD_W;
        hipLaunchKernelGGL(k_cv_fold_k, dim3((unsigned)((fblocks + 3) / 4), g), dim3(256), 0, s, (const uint32_t *)pK,
                           (uint32_t *)p1, (uint32_t *)pch, sz1, nchunks);
        hipLaunchKernelGGL(k_cv_fold, dim3((unsigned)std::min<int64_t>(4096, (sz2 + 255) / 256), g), dim3(256), 0, s,
                           (const uint32_t *)p1, (uint32_t *)p2, sz2);
        hipLaunchKernelGGL(k_cv_scan, dim3(g), dim3(1024), 0, s, (uint32_t *)pch, nchunks, (int64_t *)pnnz);
        hipLaunchKernelGGL(k_cv_base, dim3(1), dim3(64), 0, s, (const int64_t *)pnnz, g, s0, cv_off);
        hipLaunchKernelGGL(k_cv_emit, dim3((unsigned)((nchunks + 3) / 4), g), dim3(256), 0, s, (uint32_t *)pK,
                           (const uint32_t *)p1, (const uint32_t *)p2, (const uint32_t *)pch, nchunks,
                           (const unsigned long long *)ptot, (const int64_t *)cv_off, s0, K, keys, vals, capacity,
                           (int *)pflag);
        RK_HIP(hipGetLastError());
    }
    RK_TRY(timing_end(ctx, s));
    int flag = 0;
    RK_HIP(hipMemcpyAsync(&flag, pflag, sizeof(int), hipMemcpyDeviceToHost, s));
    RK_HIP(hipStreamSynchronize(s));
    cs.clean = true;  // every emitted code was written back to zero
    ctx->stats.n = n;
    ctx->stats.pairs = 0;
    if (flag) return fail(ctx, ROCKET_E_INVALID, "capacity smaller than the total number of CV entries");
    return ROCKET_OK;
}

}  // namespace rk
