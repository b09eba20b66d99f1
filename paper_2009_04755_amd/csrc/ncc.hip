// Normalised cross-correlation of dense items (Section V-A compare kernel) on gfx950.
//
// rho_ij = <a_i - mu_i, a_j - mu_j> / (s_i s_j), s = centred L2 norm.  Stages:
//   k_ncc_stats   per item: mean and centred norm, FP64 (one pass with a shift)
//   k_ncc_split   per item: centred values in FP32, split into bf16 planes (or kept FP32),
//                 stored block-major, then by 16-deep K slice, then by component: rows are
//                 grouped in blocks of T (the tile edge) and element (r, k) of component c
//                 of block b sits at element ((b * nkt + k/16) * NC + c) * T * 16 + (r%T) * 16
//                 + k%16, so one K slice of a block (all components) is one contiguous run
//                 and a block is one contiguous region.  The out-of-core path's device
//                 cache slots have exactly this block layout.
//   k_ncc_gram    persistent: pops (tile, K chunk) items, stages both row blocks of every
//                 16-deep K slice in LDS (three stages, copies two slices ahead) and
//                 accumulates the tile's Gram block with MFMA, FP32 accumulation; writes
//                 one partial tile per item
//   k_ncc_finish  per output pair: fixed-order FP64 sum of the K-chunk partials, rescale by
//                 1/(s_i s_j) in FP64, rounded once, scatter to the packed upper triangle
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "queue.hpp"

namespace rk {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int SCH_FP32 = ROCKET_NCC_FP32, SCH_X3 = ROCKET_NCC_BF16X3, SCH_X6 = ROCKET_NCC_BF16X6;

template <int SCH>
struct Scheme;
template <>
struct Scheme<SCH_FP32> {
    static constexpr int NC = 1, ES = 4;
};
template <>
struct Scheme<SCH_X3> {
    static constexpr int NC = 2, ES = 2;
};
template <>
struct Scheme<SCH_X6> {
    static constexpr int NC = 3, ES = 2;
};

__device__ __forceinline__ uint32_t bf16_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_val(uint32_t h) { return __uint_as_float(h << 16); }

// ------------------------------------------------------------------------------------------
// Per-item statistics.  Sums of (x - K) and (x - K)^2 in FP64 with K = the item's first
// value; mean = K + S1/d, centred sum of squares = S2 - S1^2/d.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ncc_stats(const float *__restrict__ X, int64_t ld, int64_t d,
                                                   double *__restrict__ mu, float *__restrict__ inv_s)
{
    const int64_t row = blockIdx.x;
    const float *a = X + row * ld;
    const double K = (double)a[0];
    double s1a = 0, s2a = 0, s1b = 0, s2b = 0;
    const bool vec = ((ld & 3) == 0) && ((((uintptr_t)X) & 15) == 0);
    int64_t k_tail = 0;
    if (vec) {
        const float4 *a4 = (const float4 *)a;
        const int64_t d4 = d >> 2;
        int64_t k = threadIdx.x;
        for (; k + 256 < d4; k += 512) {
            const float4 u = a4[k], v = a4[k + 256];
            double t;
            t = (double)u.x - K; s1a += t; s2a += t * t;
            t = (double)u.y - K; s1a += t; s2a += t * t;
            t = (double)u.z - K; s1a += t; s2a += t * t;
            t = (double)u.w - K; s1a += t; s2a += t * t;
            t = (double)v.x - K; s1b += t; s2b += t * t;
            t = (double)v.y - K; s1b += t; s2b += t * t;
            t = (double)v.z - K; s1b += t; s2b += t * t;
            t = (double)v.w - K; s1b += t; s2b += t * t;
        }
        for (; k < d4; k += 256) {
            const float4 u = a4[k];
            double t;
            t = (double)u.x - K; s1a += t; s2a += t * t;
            t = (double)u.y - K; s1a += t; s2a += t * t;
            t = (double)u.z - K; s1a += t; s2a += t * t;
            t = (double)u.w - K; s1a += t; s2a += t * t;
        }
        k_tail = d4 << 2;
    }
    for (int64_t k = k_tail + threadIdx.x; k < d; k += 256) {
        const double t = (double)a[k] - K;
        s1a += t;
        s2a += t * t;
    }
    double s1 = s1a + s1b, s2 = s2a + s2b;
    for (int o = 32; o > 0; o >>= 1) {
        s1 += __shfl_xor(s1, o);
        s2 += __shfl_xor(s2, o);
    }
    __shared__ double r1[4], r2[4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        r1[w] = s1;
        r2[w] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s1 = (r1[0] + r1[1]) + (r1[2] + r1[3]);
        s2 = (r2[0] + r2[1]) + (r2[2] + r2[3]);
        const double dd = (double)d;
        double ss = s2 - s1 * s1 / dd;
        if (ss < 0) ss = 0;
        mu[row] = K + s1 / dd;
        inv_s[row] = ss > 0 ? (float)(1.0 / sqrt(ss)) : __builtin_nanf("");
    }
}

// ------------------------------------------------------------------------------------------
// Centre and split.  Workgroup = tile of 16 rows x 256 values (16 K slices).  Each wave reads
// 4 rows of the tile with 1 KiB coalesced loads (lane = four consecutive values), centres
// them in FP64 and stores them to LDS; then thread (row, slice) reads its 16 values back
// (padded rows: conflict-free 16-byte reads), splits them and writes 32-byte pieces per
// plane, consecutive threads writing consecutive rows of one slice.  Rows >= n (up to
// rows_pad) and values >= d become zeros.  grid = (ceil(nkt / 16), rows_pad / 16).
// ------------------------------------------------------------------------------------------
template <int SCH>
__global__ __launch_bounds__(256) void k_ncc_split(const float *__restrict__ X, int64_t ld, int64_t d, int64_t n,
                                                   const double *__restrict__ mu, int64_t rows_pad, int64_t nkt,
                                                   int64_t T, char *__restrict__ planes)
{
    // 16 rows x 256 values: 16.6 KB of LDS, so up to eight workgroups (32 waves) share a CU
    constexpr int TR = 16, TK = 256, LS = TK + 4;  // LDS row stride 1040 bytes
    constexpr int SPT = (TK / 16) * TR / 256;       // slices per thread in the write phase
    __shared__ __align__(16) float tile[TR * LS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.y * TR, k0 = (int64_t)blockIdx.x * TK;
    const bool vec = ((ld & 3) == 0) && ((((uintptr_t)X) & 15) == 0);
    for (int i = 0; i < TR / 4; ++i) {
        const int row = wave * (TR / 4) + i;
        const int64_t r = r0 + row, k = k0 + 4 * lane;
        float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r < n) {
            const double m = mu[r];
            const float *a = X + r * ld + k;
            if (vec && k + 4 <= d) {
                const float4 v = *(const float4 *)a;
                c = make_float4((float)((double)v.x - m), (float)((double)v.y - m), (float)((double)v.z - m),
                                (float)((double)v.w - m));
            } else {
                if (k < d) c.x = (float)((double)a[0] - m);
                if (k + 1 < d) c.y = (float)((double)a[1] - m);
                if (k + 2 < d) c.z = (float)((double)a[2] - m);
                if (k + 3 < d) c.w = (float)((double)a[3] - m);
            }
        }
        *(float4 *)&tile[row * LS + 4 * lane] = c;
    }
    __syncthreads();
    const int row = threadIdx.x % TR, sg = threadIdx.x / TR;  // slices sg*SPT .. sg*SPT + SPT - 1
    static_assert(SPT >= 1 && (TK / 16) % SPT == 0, "whole slices per thread");
    const int64_t r = r0 + row;
    if (r >= rows_pad) return;
    const int64_t blk = r / T, rr = r - blk * T;
    constexpr int NC = Scheme<SCH>::NC;
    const int64_t plane_bytes = T * 16 * Scheme<SCH>::ES;  // one component of one K slice of a block
    char *pb = planes + blk * nkt * NC * plane_bytes;
#pragma unroll
    for (int sl = 0; sl < SPT; ++sl) {
        const int ktl = sg * SPT + sl;
        const int64_t kt = (int64_t)blockIdx.x * (TK / 16) + ktl;
        if (kt >= nkt) break;
        float x[16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 v = *(const float4 *)&tile[row * LS + ktl * 16 + 4 * q];
            x[4 * q] = v.x;
            x[4 * q + 1] = v.y;
            x[4 * q + 2] = v.z;
            x[4 * q + 3] = v.w;
        }
        const int64_t dst = (kt * NC * T + rr) * 16;
        if constexpr (SCH == SCH_FP32) {
            float4 *p = (float4 *)((float *)pb + dst);
#pragma unroll
            for (int q = 0; q < 4; ++q) p[q] = make_float4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
        } else {
            uint32_t hw[8], mw[8], lw[8];
#pragma unroll
            for (int e = 0; e < 16; e += 2) {
                uint32_t h2[2], m2[2], l2[2];
#pragma unroll
                for (int f = 0; f < 2; ++f) {
                    h2[f] = bf16_rne(x[e + f]);
                    const float r1 = x[e + f] - bf16_val(h2[f]);
                    m2[f] = bf16_rne(r1);
                    const float r2 = r1 - bf16_val(m2[f]);
                    l2[f] = bf16_rne(r2);
                }
                hw[e / 2] = h2[0] | (h2[1] << 16);
                mw[e / 2] = m2[0] | (m2[1] << 16);
                lw[e / 2] = l2[0] | (l2[1] << 16);
            }
            uint4 *p0 = (uint4 *)((uint16_t *)pb + dst);
            p0[0] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
            p0[1] = make_uint4(hw[4], hw[5], hw[6], hw[7]);
            uint4 *p1 = (uint4 *)((uint16_t *)(pb + plane_bytes) + dst);
            p1[0] = make_uint4(mw[0], mw[1], mw[2], mw[3]);
            p1[1] = make_uint4(mw[4], mw[5], mw[6], mw[7]);
            if constexpr (SCH == SCH_X6) {
                uint4 *p2 = (uint4 *)((uint16_t *)(pb + 2 * plane_bytes) + dst);
                p2[0] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
                p2[1] = make_uint4(lw[4], lw[5], lw[6], lw[7]);
            }
        }
    }
}

// LDS segment swizzles (16-byte segments within a row of one K slice), chosen so that
// the 16-byte fragment reads of 16 consecutive lanes hit distinct banks.
template <int SEGS>
__device__ __forceinline__ int swz(int row)
{
    if constexpr (SEGS == 2)
        return ((row >> 2) ^ (row >> 3)) & 1;
    else
        return ((row >> 1) ^ (row >> 3)) & 3;
}

// Wait until at most N vector-memory operations of this wave are outstanding (gfx9
// s_waitcnt encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at max).
template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

typedef __attribute__((address_space(3))) void *lds_ptr_t;
typedef __attribute__((address_space(1))) void *gbl_ptr_t;

// ------------------------------------------------------------------------------------------
// Persistent Gram kernel.  NWV = 4 waves (2 x 2, one per SIMD) or 8 waves (2 x 4, two per
// SIMD) over a BM x BN output block; each wave owns (BM/2) x (BN/(NWV/2)) made of 32x32 MFMA
// blocks (with 8 waves on a 256 tile, two 32-column blocks four apart, so that a diagonal
// tile's blocks above the diagonal spread evenly over the SIMDs and the rest are skipped).
// One stage = a
// 16-deep K slice of all NC operand planes for both row blocks (A = BM rows of block bi,
// B = BN rows of block bj), copied HBM -> LDS with global_load_lds (no register staging)
// two slices ahead through three LDS buffers, so a copy has two slices of matrix work to
// land.
//   bf16:  v_mfma_f32_32x32x16_bf16, lane l holds row l%32, k = 8*(l/32) .. +8
//   fp32:  v_mfma_f32_32x32x2_f32 x 8 per stage; step s feeds k = s (lanes 0-31) and
//          k = 8 + s (lanes 32-63), the same permutation for both operands
// Output block layout (both): acc[r] of lane l is row 8*(r/4) + 4*(l/32) + r%4, col l%32.
// ------------------------------------------------------------------------------------------
template <int BM, int BN, int SCH, int NWV>
__global__ __launch_bounds__(64 * NWV, 1) void k_ncc_gram(const char *__restrict__ planes, int kt_per_chunk, int nkt,
                                                     int nchunks, QueueArgs q, float *__restrict__ partial)
{
    constexpr int NC = Scheme<SCH>::NC, ES = Scheme<SCH>::ES;
    constexpr int ROWB = 16 * ES;
    constexpr int SEGS = ROWB / 16;
    constexpr int TA = BM * ROWB, TB = BN * ROWB;  // bytes of one component, side A / side B
    constexpr int CSB = TA + TB;                     // bytes of one component, both sides
    constexpr int STAGEB = NC * CSB;
    constexpr int BLOCKS = STAGEB / 1024;            // 1 KiB wave-copies per stage
    constexpr int BPW = BLOCKS / NWV;                // per wave
    constexpr int ROWS_PER_BLOCK = 1024 / ROWB;
    constexpr int HALVES = BM / BN;
    // NWV = 4: 2 x 2 waves, one per SIMD; NWV = 8: 2 x 4 waves, two per SIMD, so one wave's
    // waits (LDS reads, barrier, copy completion) are covered by the other's MFMAs
    constexpr int WAVES_N = NWV / 2;
    constexpr int WM = BM / 2, WN = BN / WAVES_N;
    constexpr int MA = WM / 32, MBN = WN / 32;
    // products (A component, B component): h*h, h*m, m*h [, h*l, l*h, m*m]
    constexpr int NP = SCH == SCH_X6 ? 6 : SCH == SCH_X3 ? 3 : 0;
    constexpr int PA[6] = {0, 0, 1, 0, 2, 1};
    constexpr int PB[6] = {0, 1, 0, 2, 0, 1};
    static_assert(TA % 1024 == 0 && TB % 1024 == 0, "tile sides must be whole 1 KiB blocks");
    static_assert(BLOCKS % NWV == 0, "every wave issues the same number of copies");
    static_assert(NWV == 4 || NWV == 8, "4 or 8 waves");

    // three separately declared stage buffers: slice s is read from one while the copies of
    // slices s+1 and s+2 land in the others (the compiler can tell them apart and does not
    // serialise a copy with the fragment reads of another buffer)
    __shared__ __align__(1024) char lds0[STAGEB];
    __shared__ __align__(1024) char lds1[STAGEB];
    __shared__ __align__(1024) char lds2[STAGEB];
    __shared__ int s_item;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;
    // Column blocks of a wave.  With 8 waves on a 256 tile, wave (wm, wn) owns the 32-column
    // blocks g and g + 4 (g = wn for wm = 0, 3 - wn for wm = 1) with its four 32-row blocks.
    // On a diagonal tile (bi == bj) the 36 blocks on or above the diagonal then fall 9 to each
    // SIMD (waves w and w + 4 share one), and the MFMAs of the 28 blocks below it are skipped;
    // a kept block's MFMA sequence does not depend on which wave runs it.
    constexpr bool IL = NWV == 8 && BM == 256 && BN == 256;
    const int g = IL ? (wm == 0 ? wn : WAVES_N - 1 - wn) : 0;
    auto colblk = [&](int n) { return IL ? g + WAVES_N * n : wn * MBN + n; };
    const int h = lane >> 5;
    const int lrow = lane / SEGS, pseg = lane % SEGS;

    int prev = -1;
    for (;;) {
        const int it = __builtin_amdgcn_readfirstlane(queue_pop_wg(q, &s_item, prev));
        if (it < 0) break;
        const int4 w = q.items[it];
        // slot = tile * HALVES + half; all work-item fields are wave-uniform
        const int bi = __builtin_amdgcn_readfirstlane(w.x), bj = __builtin_amdgcn_readfirstlane(w.y);
        const int kc = __builtin_amdgcn_readfirstlane(w.z), slot = __builtin_amdgcn_readfirstlane(w.w);
        const int kt0 = kc * kt_per_chunk;
        const int kt1 = min(kt0 + kt_per_chunk, nkt);
        // bit m * MBN + n: block (m, n) of this wave lies on or above the diagonal
        unsigned live = 0;
#pragma unroll
        for (int m = 0; m < MA; ++m)
#pragma unroll
            for (int n = 0; n < MBN; ++n)
                if (wm * MA + m <= colblk(n)) live |= 1u << (m * MBN + n);
        live = __builtin_amdgcn_readfirstlane(live);
        const bool diag = IL && bi == bj;

        f32x16 acc[MA][MBN];
#pragma unroll
        for (int m = 0; m < MA; ++m)
#pragma unroll
            for (int n = 0; n < MBN; ++n)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[m][n][r] = 0.f;

        // block-major operands: slice kt, component c, row r of block b at
        // planes + ((b*nkt + kt)*NC + c)*BM*ROWB + r*ROWB
        const char *baseA = planes + (int64_t)bi * nkt * (NC * BM * ROWB);
        const char *baseB = planes + (int64_t)bj * nkt * (NC * BM * ROWB) + (int64_t)(slot % HALVES) * BN * ROWB;

        // Copy of K slice kt into dstbuf: this wave moves 1 KiB blocks wv, wv+4, ...; the
        // block's source base is wave-uniform (scalar registers), the lane adds its own
        // 32-bit offset (row within the block, swizzled 16-byte segment).
        auto issue = [&](int kt, char *dstbuf) {
#pragma unroll
            for (int c = 0; c < BPW; ++c) {
                const int b = wv + NWV * c;
                const int comp = (b * 1024) / CSB;
                const int inb = b * 1024 - comp * CSB;  // byte offset inside the component
                const int side = inb >= TA;
                const int rb = (side ? inb - TA : inb) / ROWB;
                const int row = rb + lrow;
                const int loff = lrow * ROWB + ((pseg ^ swz<SEGS>(row)) * 16);
                const char *sbase = (side ? baseB : baseA) + (int64_t)kt * (NC * BM * ROWB) + (comp * BM + rb) * ROWB;
                __builtin_amdgcn_global_load_lds((gbl_ptr_t)(sbase + loff), (lds_ptr_t)(dstbuf + b * 1024), 16, 0, 0);
            }
        };
        // one 16-deep K slice from `base`; the copy of slice kt + 2 into `nbuf` starts first.
        // DG: a diagonal tile, whose blocks below the diagonal get no MFMAs.
        auto stage = [&](auto dg, int kt, const char *base, char *nbuf) {
            constexpr bool DG = decltype(dg)::value;
            const bool ahead2 = kt + 2 < kt1;
            if (ahead2) issue(kt + 2, nbuf);
            if constexpr (SCH == SCH_FP32) {
                float fa[MA][8], fb[MBN][8];
#pragma unroll
                for (int m = 0; m < MA; ++m) {
                    const int ra = wm * WM + m * 32 + (lane & 31);
                    const char *pa = base + ra * ROWB;
                    const float4 a0 = *(const float4 *)(pa + (((2 * h) ^ swz<SEGS>(ra)) * 16));
                    const float4 a1 = *(const float4 *)(pa + (((2 * h + 1) ^ swz<SEGS>(ra)) * 16));
                    fa[m][0] = a0.x; fa[m][1] = a0.y; fa[m][2] = a0.z; fa[m][3] = a0.w;
                    fa[m][4] = a1.x; fa[m][5] = a1.y; fa[m][6] = a1.z; fa[m][7] = a1.w;
                }
#pragma unroll
                for (int n = 0; n < MBN; ++n) {
                    const int rb = colblk(n) * 32 + (lane & 31);
                    const char *pb = base + TA + rb * ROWB;
                    const float4 b0 = *(const float4 *)(pb + (((2 * h) ^ swz<SEGS>(rb)) * 16));
                    const float4 b1 = *(const float4 *)(pb + (((2 * h + 1) ^ swz<SEGS>(rb)) * 16));
                    fb[n][0] = b0.x; fb[n][1] = b0.y; fb[n][2] = b0.z; fb[n][3] = b0.w;
                    fb[n][4] = b1.x; fb[n][5] = b1.y; fb[n][6] = b1.z; fb[n][7] = b1.w;
                }
#pragma unroll
                for (int ss = 0; ss < 8; ++ss)
#pragma unroll
                    for (int m = 0; m < MA; ++m)
#pragma unroll
                        for (int n = 0; n < MBN; ++n)
                            if (!DG || ((live >> (m * MBN + n)) & 1u))
                                acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[m][ss], fb[n][ss], acc[m][n], 0,
                                                                                0, 0);
            } else {
                bf16x8 fb[NC][MBN];
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int n = 0; n < MBN; ++n) {
                        const int rb = colblk(n) * 32 + (lane & 31);
                        fb[c][n] = *(const bf16x8 *)(base + c * CSB + TA + rb * ROWB + ((h ^ swz<SEGS>(rb)) * 16));
                    }
                // products grouped by the A component: h*(h, m[, l]), m*(h[, m]), [l*h]
#pragma unroll
                for (int ca = 0; ca < NC; ++ca) {
                    bf16x8 fa[MA];
#pragma unroll
                    for (int m = 0; m < MA; ++m) {
                        const int ra = wm * WM + m * 32 + (lane & 31);
                        fa[m] = *(const bf16x8 *)(base + ca * CSB + ra * ROWB + ((h ^ swz<SEGS>(ra)) * 16));
                    }
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        if (PA[p] != ca) continue;
#pragma unroll
                        for (int m = 0; m < MA; ++m)
#pragma unroll
                            for (int n = 0; n < MBN; ++n)
                                if (!DG || ((live >> (m * MBN + n)) & 1u))
                                    acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[m], fb[PB[p]][n], acc[m][n],
                                                                                        0, 0, 0);
                    }
                }
            }
            // every MFMA of this slice stays ahead of the wait; the wait needs only the copy
            // of slice kt + 1 (issued one slice earlier), the copy of kt + 2 may stay in flight
            __builtin_amdgcn_sched_barrier(0);
            if (ahead2)
                wait_vmcnt<BPW>();
            else
                wait_vmcnt<0>();
            __syncthreads();
        };

        if constexpr (SCH == SCH_FP32 || NWV == 8) {
            issue(kt0, lds0);
            if (kt0 + 1 < kt1) {
                issue(kt0 + 1, lds1);
                wait_vmcnt<BPW>();
            } else {
                wait_vmcnt<0>();
            }
            __syncthreads();
            auto kloop = [&](auto dg) {
                for (int kt = kt0; kt < kt1; kt += 3) {
                    stage(dg, kt, lds0, lds2);
                    if (kt + 1 < kt1) stage(dg, kt + 1, lds1, lds0);
                    if (kt + 2 < kt1) stage(dg, kt + 2, lds2, lds1);
                }
            };
            if (IL && diag)
                kloop(std::true_type{});
            else
                kloop(std::false_type{});
        } else {
            // Split-phase pipeline.  The B fragments and the h fragments of A for slice s are
            // already in registers when slice s starts; its m (and l) fragments of A are read
            // at the start and used in the second half.  Between the halves every wave waits
            // for its copy of slice s+1, one barrier publishes all copies, and the B and h
            // fragments of s+1 are read while the second half of the MFMAs of s runs.
            bf16x8 fbA[NC][MBN], faA[MA], fbB[NC][MBN], faB[MA];
            auto frag_a = [&](bf16x8 (&fa)[MA], const char *base, int c) {
#pragma unroll
                for (int m = 0; m < MA; ++m) {
                    const int ra = wm * WM + m * 32 + (lane & 31);
                    fa[m] = *(const bf16x8 *)(base + c * CSB + ra * ROWB + ((h ^ swz<SEGS>(ra)) * 16));
                }
            };
            auto frag_b = [&](bf16x8 (&fb)[NC][MBN], const char *base) {
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int n = 0; n < MBN; ++n) {
                        const int rb = wn * WN + n * 32 + (lane & 31);
                        fb[c][n] = *(const bf16x8 *)(base + c * CSB + TA + rb * ROWB + ((h ^ swz<SEGS>(rb)) * 16));
                    }
            };
            auto mfma_row = [&](const bf16x8 (&fa)[MA], const bf16x8 (&fbc)[MBN]) {
#pragma unroll
                for (int m = 0; m < MA; ++m)
#pragma unroll
                    for (int n = 0; n < MBN; ++n)
                        acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[m], fbc[n], acc[m][n], 0, 0, 0);
            };
            auto pstage = [&](int kt, const char *cur, const char *nxt, char *dma, bf16x8 (&fbc)[NC][MBN],
                              bf16x8 (&fa0c)[MA], bf16x8 (&fbn)[NC][MBN], bf16x8 (&fa0n)[MA]) {
                bf16x8 fa1[MA], fa2[MA];
                frag_a(fa1, cur, 1);
                if constexpr (NC == 3) frag_a(fa2, cur, 2);
                const bool ahead1 = kt + 1 < kt1, ahead2 = kt + 2 < kt1;
                if (ahead2) issue(kt + 2, dma);
                // first half: h x (h, m[, l])
                mfma_row(fa0c, fbc[0]);
                mfma_row(fa0c, fbc[1]);
                if constexpr (NC == 3) mfma_row(fa0c, fbc[2]);
                if (ahead1) {
                    __builtin_amdgcn_sched_barrier(0);
                    if (ahead2)
                        wait_vmcnt<BPW>();
                    else
                        wait_vmcnt<0>();
                    __syncthreads();
                    frag_b(fbn, nxt);
                    frag_a(fa0n, nxt, 0);
                }
                // second half: m x (h[, m]) [, l x h]
                mfma_row(fa1, fbc[0]);
                if constexpr (NC == 3) {
                    mfma_row(fa1, fbc[1]);
                    mfma_row(fa2, fbc[0]);
                }
            };
            issue(kt0, lds0);
            if (kt0 + 1 < kt1) {
                issue(kt0 + 1, lds1);
                wait_vmcnt<BPW>();
            } else {
                wait_vmcnt<0>();
            }
            __syncthreads();
            frag_b(fbA, lds0);
            frag_a(faA, lds0, 0);
            for (int kt = kt0; kt < kt1; kt += 6) {
                pstage(kt, lds0, lds1, lds2, fbA, faA, fbB, faB);
                if (kt + 1 < kt1) pstage(kt + 1, lds1, lds2, lds0, fbB, faB, fbA, faA);
                if (kt + 2 < kt1) pstage(kt + 2, lds2, lds0, lds1, fbA, faA, fbB, faB);
                if (kt + 3 < kt1) pstage(kt + 3, lds0, lds1, lds2, fbB, faB, fbA, faA);
                if (kt + 4 < kt1) pstage(kt + 4, lds1, lds2, lds0, fbA, faA, fbB, faB);
                if (kt + 5 < kt1) pstage(kt + 5, lds2, lds0, lds1, fbB, faB, fbA, faA);
            }
        }

        // partial block as float4 [BM/4][BN]: element (r4, c) holds rows 4 r4 .. 4 r4 + 3 of
        // column c, which is what acc[m][n][4q .. 4q+3] of a lane is (two 512-byte runs per
        // store instruction)
        // the block and wave part of the address is wave-uniform (scalar registers), the lane
        // adds a 32-bit offset, so no per-store address is kept in vector registers
        const int wmu = __builtin_amdgcn_readfirstlane(wm);
        const int cb0 = __builtin_amdgcn_readfirstlane(colblk(0));  // column block n is cb0 + CBSTEP * n
        constexpr int CBSTEP = IL ? WAVES_N : 1;
        char *ubase = (char *)partial + (((int64_t)slot * nchunks + kc) * (int64_t)BM * BN) * 4 +
                      ((int64_t)(wmu * WM / 4) * BN + cb0 * 32) * 16;
        const int loff = (h * BN + (lane & 31)) * 16;
#pragma unroll
        for (int m = 0; m < MA; ++m)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq)
#pragma unroll
                for (int n = 0; n < MBN; ++n) {
                    char *ub = ubase + ((m * 8 + 2 * qq) * BN + n * CBSTEP * 32) * 16;
                    *(float4 *)(ub + loff) =
                        make_float4(acc[m][n][4 * qq], acc[m][n][4 * qq + 1], acc[m][n][4 * qq + 2], acc[m][n][4 * qq + 3]);
                }
    }
}

// ------------------------------------------------------------------------------------------
// Epilogue: out[idx(i,j)] = (sum_c partial_c[i][j]) * inv_s[i] * inv_s[j], chunks summed in
// ascending order.  One thread per float4 of the partial layout (four rows of one column),
// so partial reads are 16-byte coalesced and output writes are runs along j.
// ------------------------------------------------------------------------------------------
template <int BM, int BN>
__global__ __launch_bounds__(256) void k_ncc_finish(const float *__restrict__ partial, const int2 *__restrict__ tiles,
                                                    int nchunks, int64_t n, const float *__restrict__ inv_s,
                                                    float *__restrict__ out)
{
    constexpr int BPB = BM * BN / 4 / 256;  // workgroups per output block
    constexpr int HALVES = BM / BN;
    const int64_t slot = blockIdx.x / BPB;
    const int t = (int)(blockIdx.x % BPB) * 256 + threadIdx.x;  // float4 index in the block
    const int row0 = (t / BN) * 4, col = t % BN;
    const int2 tl = tiles[slot / HALVES];
    const int64_t j = (int64_t)tl.y * BM + (slot % HALVES) * BN + col;
    const int64_t i0 = (int64_t)tl.x * BM + row0;
    if (j >= n || i0 >= j) return;
    const float4 *p = (const float4 *)(partial + slot * nchunks * (int64_t)BM * BN) + t;
    // fixed order, in FP64: a long K (thousands of chunks) would otherwise add the FP32
    // rounding of every running sum to the result
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int k = 0; k < nchunks; ++k) {
        const float4 v = p[(int64_t)k * (BM * BN / 4)];
        s0 += v.x;
        s1 += v.y;
        s2 += v.z;
        s3 += v.w;
    }
    const double vals[4] = {s0, s1, s2, s3};
    const double sj = inv_s[j];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t i = i0 + e;
        if (i < j) out[i * n - i * (i + 1) / 2 + (j - i - 1)] = (float)(vals[e] * (double)inv_s[i] * sj);
    }
}

template <int BM>
constexpr int bn_of()
{
    return BM;
}

template <int BM, int SCH>
const void *gram_ptr(int nwv)
{
    if constexpr (BM >= 128)
        if (nwv == 8) return (const void *)&k_ncc_gram<BM, bn_of<BM>(), SCH, 8>;
    return (const void *)&k_ncc_gram<BM, bn_of<BM>(), SCH, 4>;
}

template <int SCH>
const void *gram_ptr_bm(int bm, int nwv)
{
    return bm == 64 ? gram_ptr<64, SCH>(nwv) : bm == 128 ? gram_ptr<128, SCH>(nwv) : gram_ptr<256, SCH>(nwv);
}

const void *gram_kernel(int bm, int sch, int nwv)
{
    return sch == SCH_FP32 ? gram_ptr_bm<SCH_FP32>(bm, nwv) : sch == SCH_X3 ? gram_ptr_bm<SCH_X3>(bm, nwv)
                                                                            : gram_ptr_bm<SCH_X6>(bm, nwv);
}

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

int nc_of(int sch) { return sch == SCH_X6 ? 3 : sch == SCH_X3 ? 2 : 1; }
int es_of(int sch) { return sch == SCH_FP32 ? 4 : 2; }

// Statistics workspace: FP64 means [n], then the f32 inverse norms [n] at the next 256-byte
// boundary.
size_t inv_s_offset(int64_t n) { return ((size_t)n * 8 + 255) & ~(size_t)255; }
size_t stats_bytes(int64_t n) { return inv_s_offset(n) + (size_t)n * 4; }

}  // namespace

static int ncc_tile(rocket_ctx *ctx, int64_t n)
{
    const int bm = (int)ctx->opt[ROCKET_OPT_NCC_TILE];
    return bm ? bm : n >= 1536 ? 256 : n >= 384 ? 128 : 64;
}

// Waves per Gram workgroup: 8 (two per SIMD) for tiles of 128 and 256, else 4.
static int ncc_waves(rocket_ctx *ctx, int bm)
{
    const int w = (int)ctx->opt[ROCKET_OPT_NCC_WAVES];
    if (bm < 128) return 4;
    return w ? w : 8;
}

// Split-K chunk length: enough chunks for ~2048 work items, within [256, 2048] elements.
// BF16x6: the accumulation inside the matrix cores loses accuracy with the chunk length, and
// relative to the dot product's error scale the loss grows with the item length (measured
// pass metric, median ~2.2e-6 sqrt((chunk / 2048) (d / 2^20))); chunk x d is kept at most
// 2^32, which leaves 2048 at d = 2^20 and gives 416 at 3648 x 2736 (max 4.8e-6 at 512 there,
// 9.8e-6 at 2048).
static int64_t ncc_kchunk(rocket_ctx *ctx, int64_t d_pad, int64_t tiles, int scheme)
{
    int64_t kc = ctx->opt[ROCKET_OPT_NCC_KCHUNK];
    if (!kc) {
        const int64_t want_chunks = std::max<int64_t>(1, (2048 + tiles - 1) / std::max<int64_t>(tiles, 1));
        kc = round_up((d_pad + want_chunks - 1) / want_chunks, 16);
        int64_t kmax = 2048;
        if (scheme == SCH_X6) kmax = std::min<int64_t>(kmax, ((int64_t)1 << 32) / std::max<int64_t>(d_pad, 1) / 16 * 16);
        kc = std::max<int64_t>(256, std::min<int64_t>(kc, kmax));
    }
    return std::min<int64_t>(kc, d_pad);
}

// Upload the work queue of the whole leaf list (every tile x K chunk, chunk-major in per-XCD
// segments, or reordered by ROCKET_OPT_QUEUE_ORDER) and the tile list of the epilogue.
static rocket_status ncc_upload_plan(rocket_ctx *ctx, hipStream_t s)
{
    NccState &pc = ctx->ncc;
    const int64_t order = ctx->opt[ROCKET_OPT_QUEUE_ORDER], seed = ctx->opt[ROCKET_OPT_SEED],
                  ledger = queue_flags(ctx);
    plan_chunked(pc.h_tiles, pc.nchunks, MAX_SEG, ctx->h_items, ctx->h_seg, 1);
    if (order == 1) shuffle_items(ctx->h_items, ctx->h_seg, (uint64_t)seed);
    if (order == 2) single_segment(ctx->h_seg, (int64_t)ctx->h_items.size());
    RK_TRY(upload_queue(ctx, s, &pc.qa));
    void *tl = nullptr;
    RK_TRY(ws_get(ctx, WS_NCC_TILES, sizeof(int2) * pc.h_tiles.size(), &tl));
    RK_HIP(hipMemcpyAsync(tl, pc.h_tiles.data(), sizeof(int2) * pc.h_tiles.size(), hipMemcpyHostToDevice, s));
    RK_HIP(hipStreamSynchronize(s));
    ctx->queue_owner = QOWN_NCC;
    pc.queue_batched = false;
    pc.pc_nchunks = pc.nchunks;
    pc.pc_order = order;
    pc.pc_seed = seed;
    pc.pc_ledger = ledger;
    return ROCKET_OK;
}

// Tiles per Gram launch so that the split-K partials (nchunks x T^2 floats per tile) fit the
// workspace: within ROCKET_OPT_WORKSPACE_CAP next to everything else the context holds, in
// the allocation-free arena what is left of it, otherwise half of the free device memory.
// All tiles (one launch) when they fit; 0 when not even one tile does.
static int64_t ncc_batch_tiles(rocket_ctx *ctx, const NccState &st)
{
    const int64_t tile_partial = (int64_t)st.nchunks * st.tile * st.tile * 4;
    const int64_t full = st.tiles * tile_partial;
    const int64_t cur = (int64_t)ctx->ws[WS_NCC_PARTIAL].bytes;
    const int64_t cap = ctx->opt[ROCKET_OPT_WORKSPACE_CAP];
    int64_t budget;
    if (ctx->arena) {
        budget = (int64_t)(ctx->arena_cap - ctx->arena_used) - (64 << 10);  // room for the batch segment table
    } else if (cap > 0) {
        // everything else the context holds, and up to 2 MiB of rounding for the partials
        // and 2 MiB for the batch segment table
        budget = cap - (ws_total(ctx) - cur) - ((int64_t)4 << 20);
    } else {
        if (cur >= full) return st.tiles;
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            return st.tiles;
        }
        budget = ((int64_t)fr + cur) / 2;
    }
    if (full <= budget) return st.tiles;
    return std::max<int64_t>(0, budget / tile_partial);
}

rocket_status ncc_prepare(rocket_ctx *ctx, const rocket_items *it, int64_t n, int scheme, hipStream_t s)
{
    if (n > 0 && !it->dense) return fail(ctx, ROCKET_E_INVALID, "dense is NULL");
    if (it->dim < 1) return fail(ctx, ROCKET_E_INVALID, "dim < 1");
    if (it->ld < it->dim) return fail(ctx, ROCKET_E_INVALID, "ld < dim");
    if (n > (int64_t)1 << 24) return fail(ctx, ROCKET_E_INVALID, "n too large");
    NccState &st = ctx->ncc;
    st.n = n;
    st.dim = it->dim;
    st.ld = it->ld;
    st.src = it->dense;
    st.scheme = scheme;
    const int bm = ncc_tile(ctx, n);
    st.tile = bm;
    st.waves = ncc_waves(ctx, bm);
    st.n_pad = round_up(std::max<int64_t>(n, 1), bm);
    st.d_pad = round_up(it->dim, 16);
    st.nkt = (int)(st.d_pad / 16);

    NccState &pc = st;
    if (ctx->queue_owner != QOWN_NCC) pc.pc_nchunks = -1;
    if (pc.pc_n != n || pc.pc_tile != bm) {
        plan_leaves(n, bm, pc.h_tiles);
        pc.pc_n = n;
        pc.pc_tile = bm;
        pc.pc_nchunks = -1;
    }
    st.tiles = (int64_t)pc.h_tiles.size();
    const int64_t kc = ncc_kchunk(ctx, st.d_pad, st.tiles, scheme);
    st.kt_per_chunk = (int)(kc / 16);
    st.nchunks = (int)((st.nkt + st.kt_per_chunk - 1) / st.kt_per_chunk);
    const int halves = 1;  // column slices per tile (the kernels use square blocks)
    st.items = st.tiles * halves * st.nchunks;
    ctx->stats.tiles = st.tiles;
    ctx->stats.work_items = st.items;
    ctx->stats.tile = bm;
    ctx->stats.kchunk = kc;
    ctx->stats.variant = scheme;
    if (st.items > INT32_MAX / 2) return fail(ctx, ROCKET_E_INVALID, "too many work items");

    const int64_t order = ctx->opt[ROCKET_OPT_QUEUE_ORDER], seed = ctx->opt[ROCKET_OPT_SEED],
                  ledger = queue_flags(ctx);
    if (st.tiles > 0 &&
        (pc.pc_nchunks != st.nchunks || pc.pc_order != order || pc.pc_seed != seed || pc.pc_ledger != ledger))
        RK_TRY(ncc_upload_plan(ctx, s));
    if (n == 0) return ROCKET_OK;

    void *stats = nullptr, *planes = nullptr;
    RK_TRY(ws_get(ctx, WS_NCC_STATS, stats_bytes(n), &stats));
    const int64_t plane_bytes = st.n_pad * st.d_pad * es_of(scheme);
    RK_TRY(ws_get(ctx, WS_NCC_PLANES, (size_t)(plane_bytes * nc_of(scheme)), &planes));
    double *mu = (double *)stats;
    float *inv_s = (float *)((char *)stats + inv_s_offset(n));
    hipLaunchKernelGGL(k_ncc_stats, dim3((unsigned)n), dim3(256), 0, s, it->dense, it->ld, it->dim, mu, inv_s);
    RK_HIP(hipGetLastError());
    const dim3 g((unsigned)((st.nkt + 15) / 16), (unsigned)((st.n_pad + 15) / 16));
    if (scheme == SCH_FP32)
        hipLaunchKernelGGL(k_ncc_split<SCH_FP32>, g, dim3(256), 0, s, it->dense, it->ld, it->dim, n, mu, st.n_pad,
                           (int64_t)st.nkt, (int64_t)bm, (char *)planes);
    else if (scheme == SCH_X3)
        hipLaunchKernelGGL(k_ncc_split<SCH_X3>, g, dim3(256), 0, s, it->dense, it->ld, it->dim, n, mu, st.n_pad,
                           (int64_t)st.nkt, (int64_t)bm, (char *)planes);
    else
        hipLaunchKernelGGL(k_ncc_split<SCH_X6>, g, dim3(256), 0, s, it->dense, it->ld, it->dim, n, mu, st.n_pad,
                           (int64_t)st.nkt, (int64_t)bm, (char *)planes);
    RK_HIP(hipGetLastError());
    return ROCKET_OK;
}

template <int BM, int SCH>
static void launch_gram(int grid, hipStream_t s, const char *planes, const NccState &st, const QueueArgs &qa,
                        float *partial)
{
    if constexpr (BM >= 128)
        if (st.waves == 8) {
            hipLaunchKernelGGL((k_ncc_gram<BM, bn_of<BM>(), SCH, 8>), dim3(grid), dim3(512), 0, s, planes,
                               st.kt_per_chunk, st.nkt, st.nchunks, qa, partial);
            return;
        }
    hipLaunchKernelGGL((k_ncc_gram<BM, bn_of<BM>(), SCH, 4>), dim3(grid), dim3(256), 0, s, planes, st.kt_per_chunk,
                       st.nkt, st.nchunks, qa, partial);
}

template <int SCH>
static void launch_gram_bm(int grid, hipStream_t s, const char *planes, const NccState &st, const QueueArgs &qa,
                           float *partial)
{
    if (st.tile == 64)
        launch_gram<64, SCH>(grid, s, planes, st, qa, partial);
    else if (st.tile == 128)
        launch_gram<128, SCH>(grid, s, planes, st, qa, partial);
    else
        launch_gram<256, SCH>(grid, s, planes, st, qa, partial);
}

static void launch_gram_any(int grid, hipStream_t s, const char *planes, const NccState &st, const QueueArgs &qa,
                            float *partial)
{
    if (st.scheme == SCH_FP32)
        launch_gram_bm<SCH_FP32>(grid, s, planes, st, qa, partial);
    else if (st.scheme == SCH_X3)
        launch_gram_bm<SCH_X3>(grid, s, planes, st, qa, partial);
    else
        launch_gram_bm<SCH_X6>(grid, s, planes, st, qa, partial);
}

static void launch_finish(hipStream_t s, const NccState &st, int64_t ntiles, const float *partial, const int2 *tiles,
                          const float *inv_s, float *out)
{
    const int bm = st.tile;
    const int64_t blocks = ntiles * (int64_t)bm * bm / 1024;  // every slice of every tile
    if (bm == 64)
        hipLaunchKernelGGL((k_ncc_finish<64, 64>), dim3((unsigned)blocks), dim3(256), 0, s, partial, tiles,
                           st.nchunks, st.n, inv_s, out);
    else if (bm == 128)
        hipLaunchKernelGGL((k_ncc_finish<128, 128>), dim3((unsigned)blocks), dim3(256), 0, s, partial, tiles,
                           st.nchunks, st.n, inv_s, out);
    else
        hipLaunchKernelGGL((k_ncc_finish<256, 256>), dim3((unsigned)blocks), dim3(256), 0, s, partial, tiles,
                           st.nchunks, st.n, inv_s, out);
}

rocket_status ncc_compare(rocket_ctx *ctx, float *out, hipStream_t s)
{
    NccState &st = ctx->ncc;
    if (st.n < 2 || st.tiles == 0) return ROCKET_OK;
    if (ctx->queue_owner != QOWN_NCC) return fail(ctx, ROCKET_E_STATE, "queue was replanned by another prepare");
    const int bm = st.tile;
    const int64_t tile_partial = (int64_t)st.nchunks * bm * bm * 4;
    const int64_t tb = ncc_batch_tiles(ctx, st);
    if (tb < 1) return fail(ctx, ROCKET_E_OOM, "workspace cap leaves no room for one tile's split-K partials");
    const char *planes = (const char *)ctx->ws[WS_NCC_PLANES].ptr;
    const float *inv_s = (const float *)((char *)ctx->ws[WS_NCC_STATS].ptr + inv_s_offset(st.n));
    const int2 *tiles = (const int2 *)ctx->ws[WS_NCC_TILES].ptr;
    void *partial = nullptr;
    if (tb >= st.tiles) {
        // one launch over every tile
        if (st.queue_batched) RK_TRY(ncc_upload_plan(ctx, s));
        RK_TRY(ws_get(ctx, WS_NCC_PARTIAL, (size_t)(st.tiles * tile_partial), &partial));
        RK_TRY(reset_queue(ctx, s, st.qa));
        const int grid = auto_grid(ctx, gram_kernel(bm, st.scheme, st.waves), 64 * st.waves, 0, st.items);
        ctx->stats.grid = grid;
        RK_TRY(timing_begin(ctx, s));
        launch_gram_any(grid, s, planes, st, st.qa, (float *)partial);
        RK_HIP(hipGetLastError());
        RK_TRY(timing_end(ctx, s));
        launch_finish(s, st, st.tiles, (const float *)partial, tiles, inv_s, out);
        RK_HIP(hipGetLastError());
        return ROCKET_OK;
    }
    // Batches of tb consecutive leaves (D&C order), each one Gram launch over its tiles' K
    // chunks (chunk-major in per-XCD segments, work items naming the tile's slot in the
    // batch) plus the epilogue, so the partials of one batch are all that is held.  Every
    // (tile, chunk) item and the epilogue's summation order are those of the single launch,
    // so the output is the same bit for bit.  The queue order options apply to single
    // launches only.
    RK_TRY(ws_get(ctx, WS_NCC_PARTIAL, (size_t)(tb * tile_partial), &partial));
    std::vector<int4> all_items, bi;
    std::vector<int> all_segs, bs;
    std::vector<int64_t> item0;
    all_items.reserve((size_t)st.items);
    for (int64_t t0 = 0; t0 < st.tiles; t0 += tb) {
        const std::vector<int2> sub(st.h_tiles.begin() + t0, st.h_tiles.begin() + std::min<int64_t>(st.tiles, t0 + tb));
        plan_chunked(sub, st.nchunks, MAX_SEG, bi, bs, 1);
        item0.push_back((int64_t)all_items.size());  // segment bounds stay relative to this
        all_items.insert(all_items.end(), bi.begin(), bi.end());
        all_segs.insert(all_segs.end(), bs.begin(), bs.end());
    }
    void *items = nullptr, *segs = nullptr;
    RK_TRY(ws_get(ctx, WS_QUEUE_ITEMS, sizeof(int4) * all_items.size(), &items));
    RK_TRY(ws_get(ctx, WS_QUEUE_SEGS, sizeof(int) * all_segs.size(), &segs));
    RK_HIP(hipMemcpyAsync(items, all_items.data(), sizeof(int4) * all_items.size(), hipMemcpyHostToDevice, s));
    RK_HIP(hipMemcpyAsync(segs, all_segs.data(), sizeof(int) * all_segs.size(), hipMemcpyHostToDevice, s));
    RK_HIP(hipStreamSynchronize(s));  // the host vectors are local
    st.queue_batched = true;          // the device queue no longer holds the prepared plan
    QueueArgs qa = st.qa;
    qa.items = (const int4 *)items;
    qa.seg = (const int *)segs;
    qa.nseg = MAX_SEG;
    RK_TRY(reset_queue(ctx, s, qa));  // heads, and the ledger of every item once
    int *ledger = qa.ledger;
    RK_TRY(timing_begin(ctx, s));
    for (size_t b = 0; b < item0.size(); ++b) {
        const int64_t t0 = (int64_t)b * tb, nt = std::min<int64_t>(tb, st.tiles - t0);
        const int64_t nit = (b + 1 < item0.size() ? item0[b + 1] : (int64_t)all_items.size()) - item0[b];
        QueueArgs qb = qa;
        qb.items = (const int4 *)items + item0[b];
        qb.seg = (const int *)segs + b * (MAX_SEG + 1);
        qb.ledger = ledger ? ledger + item0[b] : nullptr;
        qb.trace = qa.trace ? qa.trace + 3 * item0[b] : nullptr;
        if (b > 0) {
            QueueArgs qh = qb;
            qh.ledger = nullptr;  // heads only: the ledger and trace were cleared once for all batches
            qh.trace = nullptr;
            RK_TRY(reset_queue(ctx, s, qh));
        }
        const int grid = auto_grid(ctx, gram_kernel(bm, st.scheme, st.waves), 64 * st.waves, 0, nit);
        ctx->stats.grid = grid;
        launch_gram_any(grid, s, planes, st, qb, (float *)partial);
        RK_HIP(hipGetLastError());
        launch_finish(s, st, nt, (const float *)partial, tiles + t0, inv_s, out);
        RK_HIP(hipGetLastError());
    }
    RK_TRY(timing_end(ctx, s));
    return ROCKET_OK;
}

// ------------------------------------------------------------------------------------------
// Out-of-core all pairs (Section IV-A: a device cache of fixed-size slots, least recently
// used slot evicted on a miss, refilled from the next level, here the caller's host array).
// The cached unit is a block of `tile` items in split form (the GPU pre-process stage of the
// items); jobs are the divide-and-conquer leaf tiles in visiting order, which is what gives
// the cache its hits.  The host plans the whole schedule first: the LRU decisions fix a
// sequence of block loads and tile batches; a batch is cut where a load must evict a slot
// that the batch still reads.  On the device, loads run as host-to-device copies on a copy
// stream into two raw staging buffers, and stats + split on the caller's stream write the
// slot; each batch is one persistent Gram launch over its tiles' K chunks (items name slots,
// not blocks) plus the epilogue.  Copies run ahead of compute by up to two blocks.  Kernels,
// chunking and summation order are those of the in-core path, so results are identical.
// ------------------------------------------------------------------------------------------
namespace {

struct OocBatch {
    int64_t item0, nitems, tile0, ntiles;
};

struct OocOp {
    int batch;  // >= 0: run that batch; -1: load `block` into `slot`
    int block, slot;
};

}  // namespace

rocket_status ncc_allpairs_host(rocket_ctx *ctx, const float *host, int64_t n, int64_t dim, int64_t ld, int scheme,
                                float *out, hipStream_t s)
{
    if (n < 0) return fail(ctx, ROCKET_E_INVALID, "n < 0");
    if (n > 0 && !host) return fail(ctx, ROCKET_E_INVALID, "host items pointer is NULL");
    if (dim < 1) return fail(ctx, ROCKET_E_INVALID, "dim < 1");
    if (ld < dim) return fail(ctx, ROCKET_E_INVALID, "ld < dim");
    if (n > (int64_t)1 << 24) return fail(ctx, ROCKET_E_INVALID, "n too large");
    if (n >= 2 && !out) return fail(ctx, ROCKET_E_INVALID, "out is NULL");
    NccState &st = ctx->ncc;
    // the plane workspace now holds cache slots and the queue holds this schedule
    st.pc_n = -1;
    ctx->queue_owner = QOWN_NONE;
    st.n = n;
    st.dim = dim;
    st.ld = ld;
    st.src = nullptr;
    st.scheme = scheme;
    const int T = ncc_tile(ctx, n);
    st.tile = T;
    st.waves = ncc_waves(ctx, T);
    st.n_pad = round_up(std::max<int64_t>(n, 1), T);
    st.d_pad = round_up(dim, 16);
    st.nkt = (int)(st.d_pad / 16);
    std::vector<int2> leaves;
    plan_leaves(n, T, leaves);
    st.tiles = (int64_t)leaves.size();
    const int64_t kc = ncc_kchunk(ctx, st.d_pad, st.tiles, scheme);
    st.kt_per_chunk = (int)(kc / 16);
    st.nchunks = (int)((st.nkt + st.kt_per_chunk - 1) / st.kt_per_chunk);
    st.items = st.tiles * st.nchunks;
    ctx->stats.tiles = st.tiles;
    ctx->stats.work_items = st.items;
    ctx->stats.tile = T;
    ctx->stats.kchunk = kc;
    ctx->stats.variant = scheme;
    ctx->stats.cache_slots = 0;
    ctx->stats.cache_loads = 0;
    if (st.items > INT32_MAX / 2) return fail(ctx, ROCKET_E_INVALID, "too many work items");
    if (n < 2) return ROCKET_OK;

    const int64_t nb = (n + T - 1) / T;
    int64_t S = ctx->opt[ROCKET_OPT_CACHE_SLOTS] ? ctx->opt[ROCKET_OPT_CACHE_SLOTS] : nb;
    S = std::min<int64_t>(S, nb);
    if (nb >= 2 && S < 2) return fail(ctx, ROCKET_E_INVALID, "the device cache needs at least 2 slots");
    const int64_t rowb = 16 * es_of(scheme);
    const int64_t comp_bytes = (int64_t)st.nkt * T * rowb;
    const int64_t slot_bytes = nc_of(scheme) * comp_bytes;
    const int64_t tile_partial = (int64_t)st.nchunks * T * T * 4;
    const int64_t max_batch = std::max<int64_t>(1, std::min<int64_t>(64, ((int64_t)2 << 30) / tile_partial));

    // --- schedule: LRU over the slots, visiting the leaves in order --------------------------
    std::vector<int64_t> holder(S, -1), last(S, -1), where(nb, -1);
    std::vector<char> in_batch(S, 0);
    std::vector<OocOp> ops;
    std::vector<OocBatch> batches;
    std::vector<int2> bt_slots, bt_tiles;  // open batch: slot pairs, block pairs
    std::vector<int2> all_tiles;           // every batch's block pairs, batch after batch
    std::vector<int4> all_items;
    std::vector<int> all_segs;
    std::vector<int4> bi_items;
    std::vector<int> bi_seg;
    int64_t clock = 0, loads = 0;
    auto close_batch = [&]() {
        if (bt_slots.empty()) return;
        plan_chunked(bt_slots, st.nchunks, MAX_SEG, bi_items, bi_seg, 1);
        OocBatch b;
        b.item0 = (int64_t)all_items.size();
        b.nitems = (int64_t)bi_items.size();
        b.tile0 = (int64_t)all_tiles.size();
        b.ntiles = (int64_t)bt_tiles.size();
        all_items.insert(all_items.end(), bi_items.begin(), bi_items.end());
        all_segs.insert(all_segs.end(), bi_seg.begin(), bi_seg.end());
        all_tiles.insert(all_tiles.end(), bt_tiles.begin(), bt_tiles.end());
        ops.push_back({(int)batches.size(), -1, -1});
        batches.push_back(b);
        bt_slots.clear();
        bt_tiles.clear();
        std::fill(in_batch.begin(), in_batch.end(), 0);
    };
    for (const int2 &lf : leaves) {
        const int need[2] = {lf.x, lf.y};
        const int nneed = lf.x == lf.y ? 1 : 2;
        for (int q = 0; q < nneed; ++q) {
            const int b = need[q];
            ++clock;
            if (where[b] >= 0) {
                last[where[b]] = clock;
                continue;
            }
            const int64_t keep = nneed == 2 ? where[need[1 - q]] : -1;
            int64_t v = -1;
            for (int64_t k = 0; k < S && v < 0; ++k)
                if (holder[k] < 0) v = k;
            if (v < 0)
                for (int64_t k = 0; k < S; ++k)
                    if (k != keep && (v < 0 || last[k] < last[v])) v = k;
            if (in_batch[v]) close_batch();  // the open batch still reads the victim
            if (holder[v] >= 0) where[holder[v]] = -1;
            holder[v] = b;
            where[b] = v;
            last[v] = clock;
            ops.push_back({-1, b, (int)v});
            ++loads;
        }
        bt_slots.push_back(make_int2((int)where[lf.x], (int)where[lf.y]));
        bt_tiles.push_back(lf);
        in_batch[where[lf.x]] = in_batch[where[lf.y]] = 1;
        if ((int64_t)bt_slots.size() >= max_batch) close_batch();
    }
    close_batch();
    ctx->stats.cache_slots = S;
    ctx->stats.cache_loads = loads;

    // --- device buffers ------------------------------------------------------------------
    void *slots = nullptr, *stage = nullptr, *stats = nullptr, *partial = nullptr, *tiles = nullptr, *items = nullptr,
         *segs = nullptr, *heads = nullptr;
    const int64_t stage_bytes = (int64_t)T * ld * 4;
    RK_TRY(ws_get(ctx, WS_NCC_PLANES, (size_t)(S * slot_bytes), &slots));
    RK_TRY(ws_get(ctx, WS_OOC_STAGE, (size_t)(2 * stage_bytes), &stage));
    RK_TRY(ws_get(ctx, WS_NCC_STATS, stats_bytes(n), &stats));
    int64_t maxb = 0;
    for (const OocBatch &b : batches) maxb = std::max(maxb, b.ntiles);
    RK_TRY(ws_get(ctx, WS_NCC_PARTIAL, (size_t)(maxb * tile_partial), &partial));
    RK_TRY(ws_get(ctx, WS_NCC_TILES, sizeof(int2) * all_tiles.size(), &tiles));
    RK_TRY(ws_get(ctx, WS_QUEUE_ITEMS, sizeof(int4) * all_items.size(), &items));
    RK_TRY(ws_get(ctx, WS_QUEUE_SEGS, sizeof(int) * all_segs.size(), &segs));
    RK_TRY(ws_get(ctx, WS_QUEUE_HEADS, sizeof(int) * HEAD_STRIDE * MAX_SEG, &heads));
    RK_HIP(hipMemcpyAsync(tiles, all_tiles.data(), sizeof(int2) * all_tiles.size(), hipMemcpyHostToDevice, s));
    RK_HIP(hipMemcpyAsync(items, all_items.data(), sizeof(int4) * all_items.size(), hipMemcpyHostToDevice, s));
    RK_HIP(hipMemcpyAsync(segs, all_segs.data(), sizeof(int) * all_segs.size(), hipMemcpyHostToDevice, s));
    RK_HIP(hipStreamSynchronize(s));  // the schedule vectors are local
    OocState &oc = ctx->ooc;
    if (!oc.copy) {
        RK_HIP(hipStreamCreateWithFlags(&oc.copy, hipStreamNonBlocking));
        RK_HIP(hipEventCreateWithFlags(&oc.start, hipEventDisableTiming));
        for (int k = 0; k < 2; ++k) {
            RK_HIP(hipEventCreateWithFlags(&oc.copied[k], hipEventDisableTiming));
            RK_HIP(hipEventCreateWithFlags(&oc.freed[k], hipEventDisableTiming));
        }
    }
    double *mu = (double *)stats;
    float *inv_s = (float *)((char *)stats + inv_s_offset(n));
    const dim3 sg((unsigned)((st.nkt + 15) / 16), (unsigned)((T + 15) / 16));

    // --- enqueue -------------------------------------------------------------------------
    RK_HIP(hipEventRecord(oc.start, s));  // staging buffers are free once earlier work on s is done
    RK_HIP(hipStreamWaitEvent(oc.copy, oc.start, 0));
    RK_TRY(timing_begin(ctx, s));
    int64_t m = 0;
    for (const OocOp &op : ops) {
        if (op.batch < 0) {
            const int k = (int)(m & 1);
            const int64_t r0 = (int64_t)op.block * T, rows = std::min<int64_t>(T, n - r0);
            float *buf = (float *)((char *)stage + k * stage_bytes);
            if (m >= 2) RK_HIP(hipStreamWaitEvent(oc.copy, oc.freed[k], 0));
            RK_HIP(hipMemcpyAsync(buf, host + r0 * ld, (size_t)(rows * ld * 4), hipMemcpyHostToDevice, oc.copy));
            RK_HIP(hipEventRecord(oc.copied[k], oc.copy));
            RK_HIP(hipStreamWaitEvent(s, oc.copied[k], 0));
            hipLaunchKernelGGL(k_ncc_stats, dim3((unsigned)rows), dim3(256), 0, s, buf, ld, dim, mu + r0, inv_s + r0);
            char *dst = (char *)slots + op.slot * slot_bytes;
            if (scheme == SCH_FP32)
                hipLaunchKernelGGL(k_ncc_split<SCH_FP32>, sg, dim3(256), 0, s, buf, ld, dim, rows, mu + r0, (int64_t)T,
                                   (int64_t)st.nkt, (int64_t)T, dst);
            else if (scheme == SCH_X3)
                hipLaunchKernelGGL(k_ncc_split<SCH_X3>, sg, dim3(256), 0, s, buf, ld, dim, rows, mu + r0, (int64_t)T,
                                   (int64_t)st.nkt, (int64_t)T, dst);
            else
                hipLaunchKernelGGL(k_ncc_split<SCH_X6>, sg, dim3(256), 0, s, buf, ld, dim, rows, mu + r0, (int64_t)T,
                                   (int64_t)st.nkt, (int64_t)T, dst);
            RK_HIP(hipGetLastError());
            RK_HIP(hipEventRecord(oc.freed[k], s));
            ++m;
        } else {
            const OocBatch &b = batches[op.batch];
            QueueArgs qa;
            qa.items = (const int4 *)items + b.item0;
            qa.heads = (int *)heads;
            qa.seg = (const int *)segs + (int64_t)op.batch * (MAX_SEG + 1);
            qa.ledger = nullptr;
            qa.nseg = MAX_SEG;
            RK_TRY(reset_queue(ctx, s, qa));
            const int grid = auto_grid(ctx, gram_kernel(T, scheme, st.waves), 64 * st.waves, 0, b.nitems);
            ctx->stats.grid = grid;
            launch_gram_any(grid, s, (const char *)slots, st, qa, (float *)partial);
            RK_HIP(hipGetLastError());
            launch_finish(s, st, b.ntiles, (const float *)partial, (const int2 *)tiles + b.tile0, inv_s, out);
            RK_HIP(hipGetLastError());
        }
    }
    RK_TRY(timing_end(ctx, s));
    return ROCKET_OK;
}

}  // namespace rk
