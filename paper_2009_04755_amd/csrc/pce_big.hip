// PCE over all cyclic shifts for images larger than one LDS tile (Section V-A's PCE variant
// of the pattern comparison at the size of the forensics patterns): H x W items, H and W
// powers of two in [256, 2048].  The quantities are those of the in-LDS path:
//   C(s) = sum_x a(x + s) b(x),  s* = argmax C,  PCE = C(s*)^2 (HW - |N|) / sum_{s not in N} C(s)^2.
//
// Prepare (per item): FP64 mean and norm, then the 2-D FFT of the centred unit-norm image as
// row FFTs (length W, only columns 0 .. W/2 kept: the input is real) followed by column FFTs
// (length H) in place; spectra are H x (W/2 + 1) complex f32, row-major.
//
// Compare: pairs are visited tile by tile (T x T items, divide-and-conquer leaves), two at a
// time: P = conj(F_a) F_b + i conj(F_c) F_d is the spectrum of H W (C_1 + i C_2), both C real.
// A batch of such pair-pairs runs as three kernels with the transform staged in HBM:
//   row pass     per pair-pair and row pair {k, H - k}: build both rows of P over all W
//                columns from the four half spectra (Hermitian mirror for columns > W/2) and
//                transform them along the row;
//   column pass  per pair-pair and block of columns: transform along the columns, keep the
//                block's peak (largest value, smallest shift index r W + c on ties) and its
//                FP64 energy per channel, and leave H W C in place;
//   final        per pair-pair: the overall peak and energy, the energy of the (2h+1)^2 cells
//                around each peak, and the PCE of both pairs.
// The FFTs are radix-2 Stockham transforms in LDS (natural order in and out, twiddles
// W_N^m computed in FP64 and rounded once).
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace rk {
namespace {

constexpr int PB_THREADS = 256;
constexpr int PB_T = 8;           // items per block of the pair tiles
constexpr int PB_LDS_CPLX = 8192;  // complex values per LDS buffer of the column passes (64 KB + padding)
constexpr int64_t PB_STAGE_BYTES = (int64_t)128 << 20;  // default staging of one batch of transforms

__device__ __forceinline__ float2 pb_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 pb_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 pb_mul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
// conj(a) b
__device__ __forceinline__ float2 pb_cjmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.x, b.y, -(a.y * b.x)));
}

// W_N^m = exp(-2 pi i m / N), m < N/2, FP64 rounded once
__global__ void k_pb_twiddles(float2 *tw, int N)
{
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < N / 2; m += gridDim.x * blockDim.x) {
        double s, c;
        sincospi(-2.0 * m / N, &s, &c);
        tw[m] = make_float2((float)c, (float)s);
    }
}

// M independent N-point forward DFTs of x (vector v at x + v ld), radix-2 Stockham between
// x and y (same layout); returns the buffer that holds the result (natural order).
__device__ float2 *pb_fft(float2 *x, float2 *y, int N, int logN, int M, int ld, const float2 *__restrict__ tw)
{
    const int half = N >> 1;
    for (int s = 0; s < logN; ++s) {
        const int Ns = 1 << s;
        for (int t = threadIdx.x; t < M * half; t += PB_THREADS) {
            const int v = t / half, j = t - v * half;
            const int k = j & (Ns - 1);
            const float2 *xv = x + v * ld;
            const float2 a = xv[j];
            const float2 b = pb_mul(xv[j + half], tw[k * (half >> s)]);  // W_(2 Ns)^k
            float2 *yv = y + v * ld + ((j - k) << 1) + k;
            yv[0] = pb_add(a, b);
            yv[Ns] = pb_sub(a, b);
        }
        __syncthreads();
        float2 *t = x;
        x = y;
        y = t;
    }
    return x;
}

// Per item: FP64 mean and inverse norm of the centred values; live = non-zero variance.
__global__ __launch_bounds__(PB_THREADS) void k_pb_stats(const float *__restrict__ X, int64_t ld, int64_t d,
                                                         double2 *__restrict__ st, int *__restrict__ live)
{
    const float *x = X + (int64_t)blockIdx.x * ld;
    __shared__ double red[PB_THREADS / 64];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < d; i += PB_THREADS) s += (double)x[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    const double mean = ((red[0] + red[1]) + (red[2] + red[3])) / (double)d;
    __syncthreads();
    double q = 0.0;
    for (int64_t i = threadIdx.x; i < d; i += PB_THREADS) {
        const double c = (double)x[i] - mean;
        q = fma(c, c, q);
    }
    for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double ss = (red[0] + red[1]) + (red[2] + red[3]);
        st[blockIdx.x] = make_double2(mean, ss > 0.0 ? 1.0 / sqrt(ss) : 0.0);  // a constant item: zero spectrum
        live[blockIdx.x] = ss > 0.0;
    }
}

// Prepare, rows: grid (H, items).  Row r of item i, centred and scaled (FP64, rounded once),
// transformed along the row; columns 0 .. W/2 go to F.
__global__ __launch_bounds__(PB_THREADS) void k_pb_prep_rows(const float *__restrict__ X, int64_t ld, int W, int logW,
                                                             int64_t i0, const double2 *__restrict__ st,
                                                             const float2 *__restrict__ twW, float2 *__restrict__ F,
                                                             int H)
{
    extern __shared__ float2 pb_sm[];
    const int64_t i = i0 + blockIdx.y;
    const int r = blockIdx.x;
    const double2 ms = st[i];
    const float *x = X + i * ld + (int64_t)r * W;
    float2 *a = pb_sm, *b = pb_sm + W;
    for (int c = threadIdx.x; c < W; c += PB_THREADS) a[c] = make_float2((float)(((double)x[c] - ms.x) * ms.y), 0.f);
    __syncthreads();
    const float2 *o = pb_fft(a, b, W, logW, 1, W, twW);
    const int WH = W / 2 + 1;
    float2 *f = F + i * (int64_t)H * WH + (int64_t)r * WH;
    for (int c = threadIdx.x; c < WH; c += PB_THREADS) f[c] = o[c];
}

// Column FFTs in place over F (H x WH, row-major): grid (ceil(WH / CB), items); CB columns per
// workgroup, staged column by column in LDS with a padded stride of H + 1.
__global__ __launch_bounds__(PB_THREADS) void k_pb_prep_cols(float2 *__restrict__ F, int H, int logH, int WH, int CB,
                                                             int64_t i0, const float2 *__restrict__ twH)
{
    extern __shared__ float2 pb_sm[];
    float2 *f = F + (i0 + blockIdx.y) * (int64_t)H * WH;
    const int c0 = blockIdx.x * CB, nc = min(CB, WH - c0);
    const int ld = H + 1;
    float2 *a = pb_sm, *b = pb_sm + CB * ld;
    for (int t = threadIdx.x; t < nc * H; t += PB_THREADS) {
        const int r = t / nc, c = t - r * nc;  // consecutive threads: consecutive columns of a row
        a[c * ld + r] = f[(int64_t)r * WH + c0 + c];
    }
    __syncthreads();
    const float2 *o = pb_fft(a, b, H, logH, nc, ld, twH);
    for (int t = threadIdx.x; t < nc * H; t += PB_THREADS) {
        const int r = t / nc, c = t - r * nc;
        f[(int64_t)r * WH + c0 + c] = o[c * ld + r];
    }
}

// Row pass: grid (H/2 + 1, pair-pairs of the batch).  pp[q] = (a, b, c, d): the pairs (a, b) and
// (c, d) (c < 0: no second pair).  Builds rows k and H - k of P and transforms them.
__global__ __launch_bounds__(PB_THREADS) void k_pb_rowpass(const float2 *__restrict__ F, const int4 *__restrict__ pp,
                                                           int H, int W, int logW, const float2 *__restrict__ twW,
                                                           float2 *__restrict__ Q)
{
    extern __shared__ float2 pb_sm[];
    const int4 p = pp[blockIdx.y];
    const int k = blockIdx.x, k2 = (H - k) % H;
    const int nr = k2 == k ? 1 : 2;  // rows 0 and H/2 mirror onto themselves
    const int WH = W / 2 + 1;
    const int64_t NH = (int64_t)H * WH;
    const float2 *fa = F + p.x * NH, *fb = F + p.y * NH;
    const bool two = p.z >= 0;
    const float2 *fc = F + (two ? p.z : p.x) * NH, *fd = F + (two ? p.w : p.y) * NH;
    float2 *x = pb_sm, *y = pb_sm + 2 * W;  // two rows, then their scratch
    // Z1 = conj(A) B and Z2 = conj(C) D at rows k and k2, columns 0 .. W/2; P = Z1 + i Z2 there,
    // and P(row, W - c) = conj(Z1(mirror row, c)) + i conj(Z2(mirror row, c)) for 0 < c < W/2
    for (int t = threadIdx.x; t < 2 * WH; t += PB_THREADS) {
        const int which = t / WH, c = t - which * WH;
        const int row = which ? k2 : k, other = which;  // the row this element feeds directly
        const int64_t e = (int64_t)row * WH + c;
        const float2 z1 = pb_cjmul(fa[e], fb[e]);
        const float2 z2 = two ? pb_cjmul(fc[e], fd[e]) : make_float2(0.f, 0.f);
        if (which == 0 || nr == 2) x[other * W + c] = make_float2(z1.x - z2.y, z1.y + z2.x);
        // its mirror feeds the other row (or this row, when it mirrors onto itself)
        if (c > 0 && c < W / 2) {
            const int dst = nr == 2 ? 1 - which : 0;
            if (which == 0 || nr == 2) x[dst * W + (W - c)] = make_float2(z1.x + z2.y, z2.x - z1.y);
        }
    }
    __syncthreads();
    const float2 *o = pb_fft(x, y, W, logW, nr, W, twW);
    float2 *q = Q + (int64_t)blockIdx.y * H * W;
    for (int t = threadIdx.x; t < nr * W; t += PB_THREADS) {
        const int which = t / W, c = t - which * W;
        q[(int64_t)(which ? k2 : k) * W + c] = o[t];
    }
}

struct PbStat {
    float v0, v1;
    int i0, i1;
    double e0, e1;
};

// Column pass: grid (W / CB, pair-pairs).  Transforms CB columns of Q along the columns, writes
// the result back and the block's peak and energy per channel.
__global__ __launch_bounds__(PB_THREADS) void k_pb_colpass(float2 *__restrict__ Q, int H, int logH, int W, int CB,
                                                           const float2 *__restrict__ twH, PbStat *__restrict__ S)
{
    extern __shared__ float2 pb_sm[];
    float2 *q = Q + (int64_t)blockIdx.y * H * W;
    const int c0 = blockIdx.x * CB;
    const int ld = H + 1;
    float2 *a = pb_sm, *b = pb_sm + CB * ld;
    for (int t = threadIdx.x; t < CB * H; t += PB_THREADS) {
        const int r = t / CB, c = t - r * CB;
        a[c * ld + r] = q[(int64_t)r * W + c0 + c];
    }
    __syncthreads();
    const float2 *o = pb_fft(a, b, H, logH, CB, ld, twH);
    float best0 = -INFINITY, best1 = -INFINITY;
    int bi0 = 0x7fffffff, bi1 = 0x7fffffff;
    double e0 = 0.0, e1 = 0.0;
    for (int t = threadIdx.x; t < CB * H; t += PB_THREADS) {
        const int r = t / CB, c = t - r * CB;
        const float2 v = o[c * ld + r];
        q[(int64_t)r * W + c0 + c] = v;
        const int idx = r * W + c0 + c;
        if (v.x > best0 || (v.x == best0 && idx < bi0)) {
            best0 = v.x;
            bi0 = idx;
        }
        if (v.y > best1 || (v.y == best1 && idx < bi1)) {
            best1 = v.y;
            bi1 = idx;
        }
        e0 = fma((double)v.x, (double)v.x, e0);
        e1 = fma((double)v.y, (double)v.y, e1);
    }
    for (int off = 32; off > 0; off >>= 1) {
        const float ov0 = __shfl_xor(best0, off), ov1 = __shfl_xor(best1, off);
        const int oi0 = __shfl_xor(bi0, off), oi1 = __shfl_xor(bi1, off);
        if (ov0 > best0 || (ov0 == best0 && oi0 < bi0)) {
            best0 = ov0;
            bi0 = oi0;
        }
        if (ov1 > best1 || (ov1 == best1 && oi1 < bi1)) {
            best1 = ov1;
            bi1 = oi1;
        }
        e0 += __shfl_xor(e0, off);
        e1 += __shfl_xor(e1, off);
    }
    __shared__ PbStat red[PB_THREADS / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = PbStat{best0, best1, bi0, bi1, e0, e1};
    __syncthreads();
    if (threadIdx.x == 0) {
        PbStat r = red[0];
        for (int w = 1; w < PB_THREADS / 64; ++w) {
            const PbStat &u = red[w];
            if (u.v0 > r.v0 || (u.v0 == r.v0 && u.i0 < r.i0)) {
                r.v0 = u.v0;
                r.i0 = u.i0;
            }
            if (u.v1 > r.v1 || (u.v1 == r.v1 && u.i1 < r.i1)) {
                r.v1 = u.v1;
                r.i1 = u.i1;
            }
            r.e0 += u.e0;
            r.e1 += u.e1;
        }
        S[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = r;
    }
}

// Final: grid (pair-pairs), one workgroup each: the blocks' peaks and energies (in block
// order), the energy of the (2h+1)^2 cyclic neighbourhood of each peak, PCE.
__global__ __launch_bounds__(PB_THREADS) void k_pb_final(const float2 *__restrict__ Q, const PbStat *__restrict__ S,
                                                         int nblk, const int4 *__restrict__ pp, const int *__restrict__ live,
                                                         int H, int W, int h, int64_t n, float *__restrict__ out,
                                                         uint32_t *__restrict__ peak_out)
{
    const int4 p = pp[blockIdx.x];
    const PbStat *s = S + (int64_t)blockIdx.x * nblk;
    __shared__ PbStat tot;
    if (threadIdx.x == 0) {
        PbStat r = s[0];
        for (int b = 1; b < nblk; ++b) {
            const PbStat &u = s[b];
            if (u.v0 > r.v0 || (u.v0 == r.v0 && u.i0 < r.i0)) {
                r.v0 = u.v0;
                r.i0 = u.i0;
            }
            if (u.v1 > r.v1 || (u.v1 == r.v1 && u.i1 < r.i1)) {
                r.v1 = u.v1;
                r.i1 = u.i1;
            }
            r.e0 += u.e0;
            r.e1 += u.e1;
        }
        tot = r;
    }
    __syncthreads();
    const float2 *q = Q + (int64_t)blockIdx.x * H * W;
    const int sh = min(2 * h + 1, H), sw = min(2 * h + 1, W);
    const int cells = sh * sw;
    __shared__ double red[2][PB_THREADS / 64];
    double in0 = 0.0, in1 = 0.0;
    const int r0 = tot.i0 / W, c0 = tot.i0 % W, r1 = tot.i1 / W, c1 = tot.i1 % W;
    for (int t = threadIdx.x; t < cells; t += PB_THREADS) {
        const int dr = t / sw - min(h, (sh - 1) / 2), dc = t % sw - min(h, (sw - 1) / 2);
        const double x0 = q[(int64_t)((r0 + dr + H) % H) * W + (c0 + dc + W) % W].x;
        const double x1 = q[(int64_t)((r1 + dr + H) % H) * W + (c1 + dc + W) % W].y;
        in0 = fma(x0, x0, in0);
        in1 = fma(x1, x1, in1);
    }
    for (int o = 32; o > 0; o >>= 1) {
        in0 += __shfl_xor(in0, o);
        in1 += __shfl_xor(in1, o);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = in0;
        red[1][threadIdx.x >> 6] = in1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int ch = threadIdx.x;
        if (ch == 1 && p.z < 0) return;
        double inside = 0.0;
        for (int w = 0; w < PB_THREADS / 64; ++w) inside += red[ch][w];
        const double total = ch ? tot.e1 : tot.e0, pv = ch ? tot.v1 : tot.v0;
        const int pk = ch ? tot.i1 : tot.i0;
        const double rest = total - inside;
        const double num = pv * pv * (double)((int64_t)H * W - cells);
        const int64_t i = ch ? p.z : p.x, j = ch ? p.w : p.y;
        const int64_t pidx = i * n - i * (i + 1) / 2 + (j - i - 1);
        const bool ok = live[i] && live[j] && rest > 0.0;
        out[pidx] = ok ? (float)(num / rest) : __builtin_nanf("");
        if (peak_out) peak_out[pidx] = ok ? (uint32_t)pk : 0u;
    }
}

int log2_exact(int64_t v)
{
    int l = 0;
    while (((int64_t)1 << l) < v) ++l;
    return ((int64_t)1 << l) == v ? l : -1;
}

// columns per workgroup of the column passes: CB (H + 1) complex values per LDS buffer
int cols_per_block(int H, int ncols) { return std::min(ncols, std::max(1, PB_LDS_CPLX / H)); }

size_t col_lds(int H, int CB) { return 2 * (size_t)CB * (H + 1) * sizeof(float2); }

struct PbLayout {
    size_t spec, stats, live, tw;
};

PbLayout layout(int64_t n, int H, int W)
{
    const int64_t m = std::max<int64_t>(n, 1);
    PbLayout l;
    l.spec = (size_t)m * H * (W / 2 + 1) * sizeof(float2);
    l.stats = (size_t)m * sizeof(double2);
    l.live = ((size_t)m * sizeof(int) + 255) & ~(size_t)255;
    l.tw = (size_t)(H / 2 + W / 2) * sizeof(float2);
    return l;
}

rocket_status set_lds(rocket_ctx *ctx, const void *k, size_t bytes)
{
    RK_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return ROCKET_OK;
}

}  // namespace

bool pce_big_shape(int64_t H, int64_t W)
{
    const int lh = log2_exact(H), lw = log2_exact(W);
    return lh >= 4 && lh <= 11 && lw >= 4 && lw <= 11;
}

rocket_status pce_big_prepare(rocket_ctx *ctx, const rocket_items *it, int64_t n, int H, int W, hipStream_t s)
{
    PceState &p = ctx->pce;
    const int WH = W / 2 + 1;
    const PbLayout l = layout(n, H, W);
    void *buf = nullptr;
    RK_TRY(ws_get(ctx, WS_PCE_SPEC, l.spec + l.stats + l.live + l.tw, &buf));
    float2 *F = (float2 *)buf;
    double2 *st = (double2 *)((char *)buf + l.spec);
    int *live = (int *)((char *)st + l.stats);
    float2 *twH = (float2 *)((char *)live + l.live), *twW = twH + H / 2;
    hipLaunchKernelGGL(k_pb_twiddles, dim3(8), dim3(256), 0, s, twH, H);
    hipLaunchKernelGGL(k_pb_twiddles, dim3(8), dim3(256), 0, s, twW, W);
    RK_HIP(hipGetLastError());
    if (n > 0) {
        hipLaunchKernelGGL(k_pb_stats, dim3((unsigned)n), dim3(PB_THREADS), 0, s, it->dense, it->ld, it->dim, st, live);
        RK_HIP(hipGetLastError());
        const int logH = log2_exact(H), logW = log2_exact(W);
        const int CB = cols_per_block(H, WH);
        const size_t rl = 2 * (size_t)W * sizeof(float2), cl = col_lds(H, CB);
        RK_TRY(set_lds(ctx, (const void *)&k_pb_prep_rows, rl));
        RK_TRY(set_lds(ctx, (const void *)&k_pb_prep_cols, cl));
        for (int64_t i0 = 0; i0 < n; i0 += 65535) {
            const unsigned ni = (unsigned)std::min<int64_t>(65535, n - i0);
            hipLaunchKernelGGL(k_pb_prep_rows, dim3((unsigned)H, ni), dim3(PB_THREADS), rl, s, it->dense, it->ld, W, logW,
                               i0, st, twW, F, H);
            hipLaunchKernelGGL(k_pb_prep_cols, dim3((unsigned)((WH + CB - 1) / CB), ni), dim3(PB_THREADS), cl, s, F, H,
                               logH, WH, CB, i0, twH);
            RK_HIP(hipGetLastError());
        }
    }
    // pairs tile by tile (divide-and-conquer leaves of PB_T items), two per pair-pair
    std::vector<int2> tiles;
    plan_leaves(n, PB_T, tiles);
    std::vector<int4> &pp = p.h_pp;
    pp.clear();
    int pend_i = -1, pend_j = -1;
    for (const int2 &t : tiles) {
        const int i0 = t.x * PB_T, i1 = (int)std::min<int64_t>(n, i0 + PB_T);
        const int j0 = t.y * PB_T, j1 = (int)std::min<int64_t>(n, j0 + PB_T);
        for (int i = i0; i < i1; ++i)
            for (int j = std::max(j0, i + 1); j < j1; ++j) {
                if (pend_i < 0) {
                    pend_i = i;
                    pend_j = j;
                } else {
                    pp.push_back(make_int4(pend_i, pend_j, i, j));
                    pend_i = -1;
                }
            }
    }
    if (pend_i >= 0) pp.push_back(make_int4(pend_i, pend_j, -1, -1));
    if (!pp.empty()) {
        void *ppd = nullptr;
        RK_TRY(ws_get(ctx, WS_QUEUE_ITEMS, sizeof(int4) * pp.size(), &ppd));
        RK_HIP(hipMemcpyAsync(ppd, pp.data(), sizeof(int4) * pp.size(), hipMemcpyHostToDevice, s));
        RK_HIP(hipStreamSynchronize(s));  // pp is host staging reused by the next prepare
        ctx->queue_owner = QOWN_PCE;
    }
    p.tiles = (int64_t)tiles.size();
    ctx->stats.tiles = p.tiles;
    ctx->stats.work_items = (int64_t)pp.size();
    ctx->stats.tile = PB_T;
    ctx->stats.kchunk = 0;
    ctx->stats.variant = (int64_t)H * 10000 + W;
    return ROCKET_OK;
}

rocket_status pce_big_compare(rocket_ctx *ctx, float *out, uint32_t *peak, int h, hipStream_t s)
{
    PceState &p = ctx->pce;
    const int H = p.H, W = p.W;
    const int64_t n = p.n, npp = (int64_t)p.h_pp.size();
    if (npp == 0) return ROCKET_OK;
    if (ctx->queue_owner != QOWN_PCE) return fail(ctx, ROCKET_E_STATE, "queue was replanned by another prepare");
    const PbLayout l = layout(n, H, W);
    const float2 *F = (const float2 *)ctx->ws[WS_PCE_SPEC].ptr;
    const int *live = (const int *)((const char *)F + l.spec + l.stats);
    const float2 *twH = (const float2 *)((const char *)live + l.live), *twW = twH + H / 2;
    const int CB = cols_per_block(H, W);
    const int nblk = W / CB;
    // batch of pair-pairs: one staged H x W complex transform and nblk block stats each
    const int64_t per = (int64_t)H * W * (int64_t)sizeof(float2) + nblk * (int64_t)sizeof(PbStat);
    int64_t budget = ctx->opt[ROCKET_OPT_PCE_BATCH] > 0 ? ctx->opt[ROCKET_OPT_PCE_BATCH] * per : PB_STAGE_BYTES;
    const int64_t held = (int64_t)ctx->ws[WS_PCE_STAGE].bytes;
    if (ctx->arena)  // a slot that grows takes a new piece of the arena
        budget = std::min<int64_t>(budget, std::max<int64_t>(held, (int64_t)(ctx->arena_cap - ctx->arena_used)) - 256);
    else if (ctx->opt[ROCKET_OPT_WORKSPACE_CAP] > 0)  // allocations are rounded up to 2 MiB
        budget = std::min<int64_t>(budget, ctx->opt[ROCKET_OPT_WORKSPACE_CAP] - ws_total(ctx) + held - ((int64_t)2 << 20));
    const int64_t B = std::min<int64_t>({npp, 65535, budget / per});
    if (B < 1) return fail(ctx, ROCKET_E_OOM, "workspace cap leaves no room for one staged PCE transform");
    void *stage = nullptr;
    RK_TRY(ws_get(ctx, WS_PCE_STAGE, (size_t)(B * per), &stage));
    float2 *Q = (float2 *)stage;
    PbStat *S = (PbStat *)((char *)stage + B * (int64_t)H * W * sizeof(float2));
    const int4 *pp = (const int4 *)ctx->ws[WS_QUEUE_ITEMS].ptr;
    const int logH = log2_exact(H), logW = log2_exact(W);
    const size_t rl = 4 * (size_t)W * sizeof(float2), cl = col_lds(H, CB);
    RK_TRY(set_lds(ctx, (const void *)&k_pb_rowpass, rl));
    RK_TRY(set_lds(ctx, (const void *)&k_pb_colpass, cl));
    ctx->stats.grid = B;
    RK_TRY(timing_begin(ctx, s));
    for (int64_t q0 = 0; q0 < npp; q0 += B) {
        const unsigned nb = (unsigned)std::min<int64_t>(B, npp - q0);
        hipLaunchKernelGGL(k_pb_rowpass, dim3((unsigned)(H / 2 + 1), nb), dim3(PB_THREADS), rl, s, F, pp + q0, H, W, logW,
                           twW, Q);
        hipLaunchKernelGGL(k_pb_colpass, dim3((unsigned)nblk, nb), dim3(PB_THREADS), cl, s, Q, H, logH, W, CB, twH, S);
        hipLaunchKernelGGL(k_pb_final, dim3(nb), dim3(PB_THREADS), 0, s, (const float2 *)Q, (const PbStat *)S, nblk,
                           pp + q0, live, H, W, h, n, out, peak);
        RK_HIP(hipGetLastError());
    }
    RK_TRY(timing_end(ctx, s));
    return ROCKET_OK;
}

}  // namespace rk
