// PCE over all cyclic shifts for images larger than one LDS tile (Section V-A's PCE variant
// of the pattern comparison at the size of the forensics patterns): H x W items, H and W
// powers of two in [16, 2048].  The quantities are those of the in-LDS path:
//   C(s) = sum_x a(x + s) b(x),  s* = argmax C,  PCE = C(s*)^2 (HW - |N|) / sum_{s not in N} C(s)^2.
//
// Prepare (per item): FP64 mean and norm, then the 2-D FFT of the centred unit-norm image as
// row FFTs (length W, only columns 0 .. W/2 kept: the input is real) followed by column FFTs
// (length H) in place; spectra are H x (W/2 + 1) complex f32, row-major.
//
// Compare: pairs are visited tile by tile (T x T items, divide-and-conquer leaves), two at a
// time: P = conj(F_a) F_b + i conj(F_c) F_d is the spectrum of H W (C_1 + i C_2), both C real.
// A batch of such pair-pairs runs as three kernels with the transform staged in HBM:
//   row pass     per pair-pair and group of mirror row pairs {q, H - q}: build those rows of P
//                over all W columns from the four half spectra (Hermitian mirror for columns
//                > W/2) and transform them along the row;
//   column pass  per pair-pair and block of columns: transform along the columns and keep
//                only the block's peak (largest value, smallest shift index r W + c on ties)
//                and its FP64 energy per channel (H W C is not written back);
//   final        per pair-pair and channel: the overall peak and energy, the 2h+1 columns
//                around the peak transformed again (by the same code, so to the same values)
//                for the energy of the (2h+1)^2 cells around it, and the PCE.
// The staged transform of a pair-pair is stored as W/CB blocks of H x CB values (CB columns
// per column-pass workgroup), so that each column-pass workgroup reads one contiguous piece.
// Every FFT kernel works on one tile of 8K complex values in LDS with 512 threads: radix-16
// Stockham passes in registers (natural order in and out; pass twiddles computed in FP64 and
// rounded once), one padding slot per 16 values against bank conflicts.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace rk {
namespace {

constexpr int PB_THREADS = 256;     // per-item statistics kernel
constexpr int PB_NT = 512;          // FFT kernels (all others): one tile of PB_TILE complex values
constexpr int PB_EPT = 16;          // per workgroup, 16 per thread per pass (two workgroups per CU)
constexpr int PB_TILE = PB_NT * PB_EPT;
constexpr int PB_T = 8;             // items per block of the pair tiles
constexpr int64_t PB_STAGE_BYTES = (int64_t)512 << 20;  // default staging of one batch of transforms

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

// W_16^m = exp(-2 pi i m / 16), 0 < m < 8, m != 4 (FP64 literals rounded once)
__device__ __forceinline__ constexpr float2 pb_w16(int m)
{
    return m == 1   ? float2{0.92387953251128674f, -0.38268343236508977f}
           : m == 2 ? float2{0.70710678118654752f, -0.70710678118654752f}
           : m == 3 ? float2{0.38268343236508977f, -0.92387953251128674f}
           : m == 5 ? float2{-0.38268343236508977f, -0.92387953251128674f}
           : m == 6 ? float2{-0.70710678118654752f, -0.70710678118654752f}
                    : float2{-0.92387953251128674f, -0.38268343236508977f};
}

// R-point DFT of a[] in registers, natural order in and out (radix-2 Stockham steps with
// compile-time twiddles; W^0 and W^4 = -i are applied exactly).
template <int R>
__device__ __forceinline__ void pb_dft(float2 (&a)[R])
{
#pragma unroll
    for (int Ns = 1; Ns < R; Ns <<= 1) {
        float2 y[R];
#pragma unroll
        for (int j = 0; j < R / 2; ++j) {
            const int k = j & (Ns - 1);
            const int m = k * 8 / Ns;  // W_(2 Ns)^k = W_16^m
            float2 b = a[j + R / 2];
            if (m == 4)
                b = make_float2(b.y, -b.x);
            else if (m != 0)
                b = pb_mul(b, pb_w16(m));
            const int d = ((j - k) << 1) + k;
            y[d] = pb_add(a[j], b);
            y[d + Ns] = pb_sub(a[j], b);
        }
#pragma unroll
        for (int j = 0; j < R; ++j) a[j] = y[j];
    }
}

// Workgroup barrier that orders LDS accesses only: global loads in flight (a prefetch of the
// next work item) stay in flight across it.
__device__ __forceinline__ void pb_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS address of element e of a vector: one padding slot after every 16 values, so that the
// strided writes of the first pass and the column staging spread over the banks.
__device__ __forceinline__ int pb_pad(int e) { return e + (e >> 4); }

// Vector stride of M vectors of N values in LDS (odd, so that neighbouring vectors start
// in different banks).
__host__ __device__ __forceinline__ int pb_ld(int N) { return N + N / 16 + 1; }

// Unit u of a pass over M vectors, N/R = 2^logQ units per vector: vector v and index j.  Row
// kernels put consecutive units on consecutive j of one vector; column kernels (VF) put them
// on consecutive vectors (columns), so that their global loads and stores coalesce.
template <bool VF>
__device__ __forceinline__ void pb_unit(int u, int M, int logQ, int &v, int &j)
{
    if (VF) {
        v = u % M;
        j = u / M;
    } else {
        v = u >> logQ;
        j = u & ((1 << logQ) - 1);
    }
}

// Element access of M vectors held in LDS in the padded layout with stride ld.
struct PbLds {
    float2 *x;
    int ld;
    __device__ __forceinline__ float2 operator()(int v, int e) const { return x[v * ld + pb_pad(e)]; }
    __device__ __forceinline__ void operator()(int v, int e, float2 val) const { x[v * ld + pb_pad(e)] = val; }
};

// One radix-R pass of a Stockham FFT over M vectors of N = 2^logN values: unit (v, j),
// j < N/R, takes the R values j + r N/R of vector v from src, applies W_(R Ns)^(r k)
// (k = j mod Ns, from tw[(r - 1) Ns + k]), transforms them and hands value s to dst at
// (j - k) R + k + s Ns.  Every load of the workgroup finishes before its first store, so src
// and dst may be the same memory; a pass that stores to LDS ends with a barrier.
template <int R, int LR, bool VF, bool DST_LDS, class Src, class Dst>
__device__ __forceinline__ void pb_pass(int logN, int M, int logNs, const float2 *tw, const Src &src,
                                        const Dst &dst)
{
    constexpr int UPT = PB_EPT / R;
    const int logQ = logN - LR, Ns = 1 << logNs;
    const int units = M << logQ;
    float2 a[UPT][R];
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
        const int u = threadIdx.x + i * PB_NT;
        if (u < units) {
            int v, j;
            pb_unit<VF>(u, M, logQ, v, j);
            const int k = j & (Ns - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) a[i][r] = src(v, j + (r << logQ));
            if (logNs > 0) {
#pragma unroll
                for (int r = 1; r < R; ++r) a[i][r] = pb_mul(a[i][r], tw[((r - 1) << logNs) + k]);
            }
            pb_dft<R>(a[i]);
        }
    }
    pb_barrier();
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
        const int u = threadIdx.x + i * PB_NT;
        if (u < units) {
            int v, j;
            pb_unit<VF>(u, M, logQ, v, j);
            const int k = j & (Ns - 1);
            const int base = ((j - k) << LR) + k;
#pragma unroll
            for (int s = 0; s < R; ++s) dst(v, base + (s << logNs), a[i][s]);
        }
    }
    if (DST_LDS) pb_barrier();
}

// The passes after the first of a forward DFT of M vectors of N = 2^logN values (N >= 32):
// radix-16 passes through lds, then the last pass (radix 2, 4, 8 or 16) from lds to dst.
// tw points at the second pass's twiddles.
template <bool VF, class Dst>
__device__ __forceinline__ void pb_fft_rest(int logN, int M, const float2 *tw, const PbLds &lds, const Dst &dst)
{
    int logNs = 4;
    for (; logN - logNs > 4; logNs += 4) {
        pb_pass<16, 4, VF, true>(logN, M, logNs, tw, lds, lds);
        tw += 15 << logNs;
    }
    switch (logN - logNs) {
    case 1: pb_pass<2, 1, VF, false>(logN, M, logNs, tw, lds, dst); break;
    case 2: pb_pass<4, 2, VF, false>(logN, M, logNs, tw, lds, dst); break;
    case 3: pb_pass<8, 3, VF, false>(logN, M, logNs, tw, lds, dst); break;
    default: pb_pass<16, 4, VF, false>(logN, M, logNs, tw, lds, dst); break;
    }
}

// Forward DFT of M vectors of N = 2^logN values (N >= 16): radix-16 passes, then one radix-2,
// -4 or -8 pass for the rest.  The first pass reads src(v, e), the last hands every result to
// dst(v, e, value) (natural order); the passes between go through lds (M padded vectors of
// stride ld).  tw holds the passes' twiddles one after another, (R - 1) Ns values each.
// VF1 / VF: unit order of the first pass / of the others (VF: consecutive vectors).
template <bool VF1, bool VF, class Src, class Dst>
__device__ void pb_fft(int logN, int M, const float2 *tw, const PbLds &lds, const Src &src, const Dst &dst)
{
    if (logN == 4) {
        pb_pass<16, 4, VF1, false>(logN, M, 0, tw, src, dst);
        return;
    }
    pb_pass<16, 4, VF1, true>(logN, M, 0, tw, src, lds);
    pb_fft_rest<VF>(logN, M, tw + 15, lds, dst);
}

// The passes' twiddles W_(R Ns)^(r k) for an N-point transform, FP64 rounded once.
__global__ void k_pb_twiddles(float2 *tw, int logN)
{
    int logNs = 0;
    const int npass = (logN + 3) / 4;
    for (int p = 0; p < npass; ++p) {
        const int LR = p < logN / 4 ? 4 : (logN & 3), R = 1 << LR, Ns = 1 << logNs;
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < (R - 1) * Ns; e += gridDim.x * blockDim.x) {
            const int r = e / Ns + 1, k = e % Ns;
            double sn, cs;
            sincospi(-2.0 * r * k / ((double)R * Ns), &sn, &cs);
            tw[e] = make_float2((float)cs, (float)sn);
        }
        tw += (R - 1) * Ns;
        logNs += LR;
    }
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

// Prepare, rows: grid (H / RB, items), RB = min(H, PB_TILE / W) rows per workgroup.  The rows,
// centred and scaled (FP64, rounded once), transformed along the row; columns 0 .. W/2 go to F.
__global__ __launch_bounds__(PB_NT) void k_pb_prep_rows(const float *__restrict__ X, int64_t ld, int H, int W, int logW,
                                                        int RB, int64_t i0, const double2 *__restrict__ st,
                                                        const float2 *__restrict__ twW, float2 *__restrict__ F)
{
    extern __shared__ float2 pb_sm[];
    const int64_t i = i0 + blockIdx.y;
    const int r0 = blockIdx.x * RB, WH = W / 2 + 1;
    const double2 ms = st[i];
    const float *x = X + i * ld + (int64_t)r0 * W;
    float2 *f = F + i * (int64_t)H * WH + (int64_t)r0 * WH;
    auto src = [&](int v, int e) { return make_float2((float)(((double)x[v * W + e] - ms.x) * ms.y), 0.f); };
    auto dst = [&](int v, int e, float2 val) {
        if (e <= W / 2) f[v * WH + e] = val;
    };
    pb_fft<false, false>(logW, RB, twW, PbLds{pb_sm, pb_ld(W)}, src, dst);
}

// Column FFTs in place over F (H x WH, row-major): grid (ceil(WH / CB), items), CB = PB_TILE / H
// columns per workgroup (fewer in the last).
__global__ __launch_bounds__(PB_NT) void k_pb_prep_cols(float2 *__restrict__ F, int H, int logH, int WH, int CB,
                                                        int64_t i0, const float2 *__restrict__ twH)
{
    extern __shared__ float2 pb_sm[];
    float2 *f = F + (i0 + blockIdx.y) * (int64_t)H * WH + blockIdx.x * CB;
    const int nc = min(CB, WH - (int)blockIdx.x * CB);
    auto src = [&](int v, int e) { return f[(int64_t)e * WH + v]; };
    auto dst = [&](int v, int e, float2 val) { f[(int64_t)e * WH + v] = val; };
    pb_fft<true, true>(logH, nc, twH, PbLds{pb_sm, pb_ld(H)}, src, dst);
}

// Rows of the pair-pair spectrum P = conj(F_a) F_b + i conj(F_c) F_d come in mirror pairs:
// row pair q = 0 holds rows 0 and H/2 (each its own mirror), q > 0 rows q and H - q.
__device__ __forceinline__ int pb_row(int q, int slot, int H) { return q == 0 ? (slot ? H / 2 : 0) : (slot ? H - q : q); }

// Row pass: grid (H / (2 KP), pair-pairs of the batch), KP = min(H/2, PB_TILE / (2 W)) row pairs
// per workgroup.  Q holds each pair-pair's transform as W / CB blocks of H x CB values.  pp[q] = (a, b, c, d): the pairs (a, b) and (c, d) (c < 0: no second pair).
// Column c <= W/2 of a row comes from the half spectra at that row; column W - c (0 < c < W/2)
// is conj(Z1) + i conj(Z2) taken at the mirror row, column c.  Rows are transformed and
// written to Q.
__global__ __launch_bounds__(PB_NT) void k_pb_rowpass(const float2 *__restrict__ F, const int4 *__restrict__ pp, int H,
                                                      int W, int logW, int KP, int logCB,
                                                      const float2 *__restrict__ twW, float2 *__restrict__ Q)
{
    extern __shared__ float2 pb_sm[];
    const int4 p = pp[blockIdx.y];
    const int q0 = blockIdx.x * KP, lw = pb_ld(W), WH = W / 2 + 1, hw = W / 2;
    const int64_t NH = (int64_t)H * WH;
    const bool two = p.z >= 0;
    const float2 *fa = F + p.x * NH, *fb = F + p.y * NH;
    const float2 *fc = F + (two ? p.z : p.x) * NH, *fd = F + (two ? p.w : p.y) * NH;
    const bool same_a = p.z == p.x;  // consecutive pairs of a tile row share their first item
    // columns 0 .. W/2 - 1 of every row and their mirrors (at most PB_TILE / 2 elements: all
    // loads of a thread are issued before the first LDS store), then column W/2
    constexpr int G = PB_EPT / 2;
    const int nmain = 2 * KP * hw;
    float2 va[G], vb[G], vc[G], vd[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int t = threadIdx.x + g * PB_NT;
        if (t < nmain) {
            const int v = t >> (logW - 1), c = t & (hw - 1);
            const int64_t e = (int64_t)pb_row(q0 + (v >> 1), v & 1, H) * WH + c;
            va[g] = fa[e];
            vb[g] = fb[e];
            vc[g] = same_a ? va[g] : fc[e];
            vd[g] = fd[e];
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int t = threadIdx.x + g * PB_NT;
        if (t < nmain) {
            const int v = t >> (logW - 1), c = t & (hw - 1), q = q0 + (v >> 1);
            const float2 z1 = pb_cjmul(va[g], vb[g]);
            const float2 z2 = two ? pb_cjmul(vc[g], vd[g]) : make_float2(0.f, 0.f);
            pb_sm[v * lw + pb_pad(c)] = make_float2(z1.x - z2.y, z1.y + z2.x);
            if (c > 0) {
                const int mv = q == 0 ? v : (v ^ 1);
                pb_sm[mv * lw + pb_pad(W - c)] = make_float2(z1.x + z2.y, z2.x - z1.y);
            }
        }
    }
    if (threadIdx.x < 2 * KP) {  // column W/2 is its own mirror
        const int v = threadIdx.x;
        const int64_t e = (int64_t)pb_row(q0 + (v >> 1), v & 1, H) * WH + hw;
        const float2 z1 = pb_cjmul(fa[e], fb[e]);
        const float2 z2 = two ? pb_cjmul(fc[e], fd[e]) : make_float2(0.f, 0.f);
        pb_sm[v * lw + pb_pad(hw)] = make_float2(z1.x - z2.y, z1.y + z2.x);
    }
    __syncthreads();
    float2 *q = Q + (int64_t)blockIdx.y * H * W;
    const PbLds lds{pb_sm, lw};
    const int cbm = (1 << logCB) - 1;
    auto dst = [&](int v, int e, float2 val) {
        q[((int64_t)(e >> logCB) * H + pb_row(q0 + (v >> 1), v & 1, H)) * (cbm + 1) + (e & cbm)] = val;
    };
    pb_fft<false, false>(logW, 2 * KP, twW, lds, lds, dst);
}

struct PbStat {
    float v0, v1;  // largest value per channel
    int i0, i1;    // its shift index r W + c (the smallest on ties)
    double e0, e1; // energy per channel
};

__device__ __forceinline__ void pb_merge(PbStat &r, float v0, float v1, int i0, int i1, double e0, double e1)
{
    if (v0 > r.v0 || (v0 == r.v0 && i0 < r.i0)) {
        r.v0 = v0;
        r.i0 = i0;
    }
    if (v1 > r.v1 || (v1 == r.v1 && i1 < r.i1)) {
        r.v1 = v1;
        r.i1 = i1;
    }
    r.e0 += e0;
    r.e1 += e1;
}

// Workgroup reduction of per-thread statistics (the merge is order-independent for the
// peaks; the energies are summed in a fixed tree).  The result is valid in thread 0.
template <int NT>
__device__ __forceinline__ PbStat pb_reduce(PbStat r)
{
    for (int off = 32; off > 0; off >>= 1)
        pb_merge(r, __shfl_xor(r.v0, off), __shfl_xor(r.v1, off), __shfl_xor(r.i0, off), __shfl_xor(r.i1, off),
                 __shfl_xor(r.e0, off), __shfl_xor(r.e1, off));
    __shared__ PbStat red[NT / 64];
    pb_barrier();  // the previous reduction's reads of red are done
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
    pb_barrier();
    if (threadIdx.x == 0)
        for (int w = 1; w < NT / 64; ++w) pb_merge(r, red[w].v0, red[w].v1, red[w].i0, red[w].i1, red[w].e0, red[w].e1);
    return r;
}

// Energy of the (2h+1)^2 cells around the peak (r0, c0) of channel ch: the 2h+1 columns
// around c0 of the row-pass output q are transformed again, CF at a time, by the same code
// as in the column pass (so to the same values).  Valid in thread 0.
__device__ double pb_inside(const float2 *__restrict__ q, int H, int logH, int W, int logCB, int h, int CF, int r0,
                            int c0, int ch, const float2 *__restrict__ twH, const PbLds &lds)
{
    const int cbm = (1 << logCB) - 1;
    const int side = 2 * h + 1;
    double inside = 0.0;
    for (int k0 = 0; k0 < side; k0 += CF) {
        const int m = min(CF, side - k0), cs = c0 - h + k0 + W;
        auto src = [&](int v, int e) {
            const int c = (cs + v) & (W - 1);
            return q[((int64_t)(c >> logCB) * H + e) * (cbm + 1) + (c & cbm)];
        };
        auto dst = [&](int v, int e, float2 val) {
            if (((e - r0 + h + H) & (H - 1)) < side) {
                const double x = ch ? val.y : val.x;
                inside = fma(x, x, inside);
            }
        };
        pb_fft<true, false>(logH, m, twH, lds, src, dst);
    }
    for (int o = 32; o > 0; o >>= 1) inside += __shfl_xor(inside, o);
    __shared__ double red[PB_NT / 64];
    pb_barrier();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = inside;
    pb_barrier();
    if (threadIdx.x == 0)
        for (int w = 1; w < PB_NT / 64; ++w) inside += red[w];
    return inside;
}

// Column pass: grid (W / CB, pair-pairs), CB = min(W, PB_TILE / H) columns per workgroup.
// Transforms the columns of the row-pass output (left as it is) and writes the workgroup's
// peak (largest value, smallest shift index on ties) and FP64 energy per channel to S.
__global__ __launch_bounds__(PB_NT) void k_pb_colpass(const float2 *__restrict__ Q, int H, int logH, int W, int CB,
                                                      const float2 *__restrict__ twH, PbStat *__restrict__ S)
{
    extern __shared__ float2 pb_sm[];
    const float2 *q = Q + (int64_t)blockIdx.y * H * W;
    const int c0 = blockIdx.x * CB;
    PbStat st{-INFINITY, -INFINITY, 0x7fffffff, 0x7fffffff, 0.0, 0.0};
    const float2 *qb = q + (int64_t)blockIdx.x * H * CB;  // the block's columns: H x CB values in a row
    auto src = [&](int v, int e) { return qb[e * CB + v]; };
    auto dst = [&](int v, int e, float2 val) {
        const int idx = e * W + c0 + v;
        pb_merge(st, val.x, val.y, idx, idx, (double)val.x * val.x, (double)val.y * val.y);
    };
    pb_fft<true, false>(logH, CB, twH, PbLds{pb_sm, pb_ld(H)}, src, dst);
    st = pb_reduce<PB_NT>(st);
    if (threadIdx.x == 0) S[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = st;
}

// Final: grid (2 channels, pair-pairs).  The blocks' peaks and energies give the channel's
// peak s* and total energy; with the energy of the (2h+1)^2 cells around s*, the PCE.
__global__ __launch_bounds__(PB_NT) void k_pb_final(const float2 *__restrict__ Q, const PbStat *__restrict__ S, int nblk,
                                                    const int4 *__restrict__ pp, const int *__restrict__ live, int H,
                                                    int logH, int W, int logCB, int h, int CF, const float2 *__restrict__ twH,
                                                    int64_t n, float *__restrict__ out, uint32_t *__restrict__ peak_out)
{
    extern __shared__ float2 pb_sm[];
    const int ch = blockIdx.x;
    const int4 p = pp[blockIdx.y];
    if (ch == 1 && p.z < 0) return;  // a single pair: no second channel (uniform over the workgroup)
    const PbStat *s = S + (int64_t)blockIdx.y * nblk;
    PbStat r{-INFINITY, -INFINITY, 0x7fffffff, 0x7fffffff, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += PB_NT) pb_merge(r, s[b].v0, s[b].v1, s[b].i0, s[b].i1, s[b].e0, s[b].e1);
    r = pb_reduce<PB_NT>(r);
    __shared__ PbStat tot;
    if (threadIdx.x == 0) tot = r;
    pb_barrier();
    const int pk = ch ? tot.i1 : tot.i0;
    const bool found = pk != 0x7fffffff;  // false only for NaN surfaces
    const double inside = pb_inside(Q + (int64_t)blockIdx.y * H * W, H, logH, W, logCB, h, CF, found ? pk / W : 0,
                                    found ? pk % W : 0, ch, twH, PbLds{pb_sm, pb_ld(H)});
    if (threadIdx.x == 0) {
        const double pv = ch ? tot.v1 : tot.v0, rest = (ch ? tot.e1 : tot.e0) - inside;
        const double num = pv * pv * (double)((int64_t)H * W - (int64_t)(2 * h + 1) * (2 * h + 1));
        const int64_t i = ch ? p.z : p.x, j = ch ? p.w : p.y;
        const int64_t pidx = i * n - i * (i + 1) / 2 + (j - i - 1);
        const bool ok = found && live[i] && live[j] && rest > 0.0;
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

// LDS bytes of a workgroup holding M padded vectors of N complex values
size_t tile_lds(int M, int N) { return (size_t)M * pb_ld(N) * sizeof(float2); }

struct PbLayout {
    size_t spec, stats, live, tw;
};

// spectra | per item (mean, 1/norm) | live flags | twiddles of the H- and W-point transforms
PbLayout layout(int64_t n, int H, int W)
{
    const int64_t m = std::max<int64_t>(n, 1);
    PbLayout l;
    l.spec = (size_t)m * H * (W / 2 + 1) * sizeof(float2);
    l.stats = (size_t)m * sizeof(double2);
    l.live = ((size_t)m * sizeof(int) + 255) & ~(size_t)255;
    l.tw = (size_t)(H + W) * sizeof(float2);
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
    ctx->trace_valid = false;  // batched launches, no persistent queue to trace
    void *buf = nullptr;
    RK_TRY(ws_get(ctx, WS_PCE_SPEC, l.spec + l.stats + l.live + l.tw, &buf));
    float2 *F = (float2 *)buf;
    double2 *st = (double2 *)((char *)buf + l.spec);
    int *live = (int *)((char *)st + l.stats);
    float2 *twH = (float2 *)((char *)live + l.live), *twW = twH + H;
    const int logH = log2_exact(H), logW = log2_exact(W);
    hipLaunchKernelGGL(k_pb_twiddles, dim3(8), dim3(256), 0, s, twH, logH);
    hipLaunchKernelGGL(k_pb_twiddles, dim3(8), dim3(256), 0, s, twW, logW);
    RK_HIP(hipGetLastError());
    if (n > 0) {
        hipLaunchKernelGGL(k_pb_stats, dim3((unsigned)n), dim3(PB_THREADS), 0, s, it->dense, it->ld, it->dim, st, live);
        RK_HIP(hipGetLastError());
        const int RB = std::min(H, PB_TILE / W);         // rows per workgroup
        const int CB = PB_TILE / H;  // columns per workgroup (WH is not a power of two)
        const size_t rl = tile_lds(RB, W), cl = tile_lds(CB, H);
        RK_TRY(set_lds(ctx, (const void *)&k_pb_prep_rows, rl));
        RK_TRY(set_lds(ctx, (const void *)&k_pb_prep_cols, cl));
        for (int64_t i0 = 0; i0 < n; i0 += 65535) {
            const unsigned ni = (unsigned)std::min<int64_t>(65535, n - i0);
            hipLaunchKernelGGL(k_pb_prep_rows, dim3((unsigned)(H / RB), ni), dim3(PB_NT), rl, s, it->dense, it->ld, H, W,
                               logW, RB, i0, st, twW, F);
            hipLaunchKernelGGL(k_pb_prep_cols, dim3((unsigned)((WH + CB - 1) / CB), ni), dim3(PB_NT), cl, s, F, H, logH,
                               WH, CB, i0, twH);
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
    const float2 *twH = (const float2 *)((const char *)live + l.live), *twW = twH + H;
    // columns per column-pass workgroup; the staged transform is stored column block by column
    // block ([W / CB][H][CB]), so that each column-pass workgroup reads one contiguous piece
    const int CB = std::min(W, PB_TILE / H), logCB = log2_exact(CB);
    const int KP = std::min(H / 2, PB_TILE / (2 * W));                 // row pairs per row-pass workgroup
    const int nblk = W / CB;
    // batch of pair-pairs: one staged H x W complex transform and nblk block statistics each
    const int64_t per = (int64_t)H * W * (int64_t)sizeof(float2) + nblk * (int64_t)sizeof(PbStat);
    // default: as many transforms as 512 MiB holds (64 of 1024 x 1024), plus their statistics
    int64_t budget = (ctx->opt[ROCKET_OPT_PCE_BATCH] > 0 ? ctx->opt[ROCKET_OPT_PCE_BATCH]
                                                          : std::max<int64_t>(1, PB_STAGE_BYTES / ((int64_t)H * W * 8))) *
                     per;
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
    const size_t rl = tile_lds(2 * KP, W), cl = tile_lds(CB, H);
    RK_TRY(set_lds(ctx, (const void *)&k_pb_rowpass, rl));
    RK_TRY(set_lds(ctx, (const void *)&k_pb_colpass, cl));
    const int CF = std::min(2 * h + 1, PB_TILE / H);  // neighbourhood columns transformed at a time
    const size_t fl = tile_lds(CF, H);
    RK_TRY(set_lds(ctx, (const void *)&k_pb_final, fl));
    ctx->stats.grid = B;
    RK_TRY(timing_begin(ctx, s));
    for (int64_t q0 = 0; q0 < npp; q0 += B) {
        const unsigned nb = (unsigned)std::min<int64_t>(B, npp - q0);
        hipLaunchKernelGGL(k_pb_rowpass, dim3((unsigned)(H / (2 * KP)), nb), dim3(PB_NT), rl, s, F, pp + q0, H, W, logW, KP,
                           logCB, twW, Q);
        hipLaunchKernelGGL(k_pb_colpass, dim3((unsigned)nblk, nb), dim3(PB_NT), cl, s, (const float2 *)Q, H, logH, W, CB,
                           twH, S);
        hipLaunchKernelGGL(k_pb_final, dim3(2, nb), dim3(PB_NT), fl, s, (const float2 *)Q, (const PbStat *)S, nblk, pp + q0,
                           live, H, logH, W, logCB, h, CF, twH, n, out, peak);
        RK_HIP(hipGetLastError());
    }
    RK_TRY(timing_end(ctx, s));
    return ROCKET_OK;
}

}  // namespace rk
