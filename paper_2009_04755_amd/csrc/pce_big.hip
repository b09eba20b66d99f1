// PCE over all cyclic shifts for images larger than one LDS tile (Section V-A's PCE variant
// of the pattern comparison at the size of the forensics patterns): H x W items, H and W in
// [16, 4096] (a side that is not a power of two by Bluestein's chirp convolution).  The
// quantities are those of the in-LDS path:
//   C(s) = sum_x a(x + s) b(x),  s* = argmax C,  PCE = C(s*)^2 (HW - |N|) / sum_{s not in N} C(s)^2.
//
// Prepare (per item): FP64 mean and norm, then the 2-D DFT of the centred unit-norm image as
// row DFTs (length W, only columns 0 .. W/2 kept: the input is real) followed by column DFTs
// (length H) in place; spectra are H x (W/2 + 1) complex f32, row-major.
//
// Compare: pairs are visited tile by tile (T x T items, divide-and-conquer leaves), two at a
// time: P = conj(F_a) F_b + i conj(F_c) F_d is the spectrum of H W (C_1 + i C_2), both C real.
// A batch of such pair-pairs runs as four kernels with the transform staged in HBM:
//   row pass     per pair-pair and group of mirror row pairs {q, H - q} (row 0 alone for odd
//                H): build those rows of P over all W columns from the four half spectra
//                (Hermitian mirror for columns > W/2) and transform them along the row;
//   column pass  per pair-pair and group of columns: transform along the columns and keep
//                only the group's peak (largest value, smallest shift index r W + c on ties)
//                and its FP64 energy per channel (H W C is not written back);
//   peak         per pair-pair, channel and group of the 2h+1 columns around the peak: the
//                overall peak and energy, and those columns transformed again (by the same
//                code, so to the same values) for their energy inside the (2h+1)^2 cells
//                around the peak;
//   pce          per pair-pair and channel: the neighbourhood energy summed, and the PCE.
// With two staging buffers the row pass of batch b + 1 (caller's stream) runs beside the other
// three kernels of batch b (a second stream of the context), ordered by events.
// The staged transform of a pair-pair is stored as ceil(W/CB) blocks of H x CB values, so
// that the column-pass workgroups of a block read one contiguous piece.  Every FFT kernel
// works on one tile of 8K complex values in LDS with 512 threads (two workgroups per CU; the
// column pass takes 4K values with 256 threads where a column fits, four per CU, and rows of
// 8K-point transforms run one per workgroup): radix-16 Stockham passes in registers
// (natural order in and out; pass twiddles computed in FP64 and rounded once), one padding
// slot per 16 values against bank conflicts.  An axis of N values, N not a power of two, is
// an M-point FFT, its product with the chirp filter's spectrum and an inverse M-point FFT in
// the same tile (M the power of two >= 2N - 1), N <= 4096 so that M <= 8192.
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

// Workgroup coordinates in an XCD-aware order.  Workgroups go to the 8 XCDs (each with its
// own L2) round-robin by linear id, so neighbours in the grid run on different XCDs; when
// neighbouring workgroups read parts of the same cache lines (columns narrower than a line)
// every XCD would fetch each line.  Renumbered, XCD k takes the k-th eighth of the grid in
// order (the remainder of a grid not divisible by 8 keeps its place).
__device__ __forceinline__ void pb_xcd_order(bool on, int &x, int &y)
{
    x = blockIdx.x;
    y = blockIdx.y;
    if (!on) return;
    const int64_t total = (int64_t)gridDim.x * gridDim.y, lin = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (lin >= total / 8 * 8) return;
    const int64_t l = (lin & 7) * (total / 8) + (lin >> 3);
    y = (int)(l / gridDim.x);
    x = (int)(l - (int64_t)y * gridDim.x);
}

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
template <int R, int LR, bool VF, bool DST_LDS, int NT, class Src, class Dst>
__device__ __forceinline__ void pb_pass(int logN, int M, int logNs, const float2 *tw, const Src &src,
                                        const Dst &dst)
{
    constexpr int UPT = PB_EPT / R;
    const int logQ = logN - LR, Ns = 1 << logNs;
    const int units = M << logQ;
    float2 a[UPT][R];
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
        const int u = threadIdx.x + i * NT;
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
        const int u = threadIdx.x + i * NT;
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
template <bool VF, int NT, class Dst>
__device__ __forceinline__ void pb_fft_rest(int logN, int M, const float2 *tw, const PbLds &lds, const Dst &dst)
{
    int logNs = 4;
    for (; logN - logNs > 4; logNs += 4) {
        pb_pass<16, 4, VF, true, NT>(logN, M, logNs, tw, lds, lds);
        tw += 15 << logNs;
    }
    switch (logN - logNs) {
    case 1: pb_pass<2, 1, VF, false, NT>(logN, M, logNs, tw, lds, dst); break;
    case 2: pb_pass<4, 2, VF, false, NT>(logN, M, logNs, tw, lds, dst); break;
    case 3: pb_pass<8, 3, VF, false, NT>(logN, M, logNs, tw, lds, dst); break;
    default: pb_pass<16, 4, VF, false, NT>(logN, M, logNs, tw, lds, dst); break;
    }
}

// Forward DFT of M vectors of N = 2^logN values (N >= 16): radix-16 passes, then one radix-2,
// -4 or -8 pass for the rest.  The first pass reads src(v, e), the last hands every result to
// dst(v, e, value) (natural order); the passes between go through lds (M padded vectors of
// stride ld).  tw holds the passes' twiddles one after another, (R - 1) Ns values each.
// VF1 / VF: unit order of the first pass / of the others (VF: consecutive vectors); NT
// threads, at most NT * PB_EPT values.
template <bool VF1, bool VF, int NT, class Src, class Dst>
__device__ void pb_fft(int logN, int M, const float2 *tw, const PbLds &lds, const Src &src, const Dst &dst)
{
    if (logN == 4) {
        pb_pass<16, 4, VF1, false, NT>(logN, M, 0, tw, src, dst);
        return;
    }
    pb_pass<16, 4, VF1, true, NT>(logN, M, 0, tw, src, lds);
    pb_fft_rest<VF, NT>(logN, M, tw + 15, lds, dst);
}

// One axis of the 2-D transform: an N-point DFT.  When N is a power of two it is one FFT
// (M = N).  Otherwise Bluestein's chirp convolution: with w_n = exp(-i pi n^2 / N),
// X_k = w_k sum_n (x_n w_n) conj(w_(k-n)), a convolution that one circular convolution of
// length M >= 2N - 1 (a power of two) holds: X = w . IFFT_M(FFT_M(x w) . B) on k < N, with
// B = FFT_M(b), b_m = conj(w_|m|) for |m| < N (indices mod M) and 0 between.
struct PbDim {
    int N, M, logM;
    const float2 *tw;     // twiddles of the M-point FFT
    const float2 *chirp;  // w_n, n < N (Bluestein only)
    const float2 *filt;   // B (Bluestein only)
};

// The N-point DFT of nv vectors: src(v, e) for e < N, results to dst(v, e, X_e) for e < N.
// BLUE (a compile-time choice, so that the power-of-two kernels keep their registers): by
// Bluestein, the vectors occupying M values each in lds; the inverse FFT is the forward FFT
// of the conjugate, conjugated and scaled by 1/M (exact: M is a power of two).
template <bool BLUE, bool VF1, bool VF, int NT, class Src, class Dst>
__device__ void pb_dft(const PbDim &d, int nv, const PbLds &lds, const Src &src, const Dst &dst)
{
    if constexpr (!BLUE) {
        pb_fft<VF1, VF, NT>(d.logM, nv, d.tw, lds, src, dst);
    } else {
        const float2 *w = d.chirp, *B = d.filt;
        const int N = d.N;
        auto src1 = [&](int v, int e) { return e < N ? pb_mul(src(v, e), w[e]) : make_float2(0.f, 0.f); };
        auto dst1 = [&](int v, int e, float2 val) {
            const float2 z = pb_mul(val, B[e]);
            lds(v, e, make_float2(z.x, -z.y));
        };
        pb_fft<VF1, VF, NT>(d.logM, nv, d.tw, lds, src1, dst1);
        pb_barrier();
        const float inv = 1.f / (float)d.M;
        auto dst2 = [&](int v, int e, float2 val) {
            if (e < N) dst(v, e, pb_mul(make_float2(val.x * inv, -val.y * inv), w[e]));
        };
        pb_fft<VF, VF, NT>(d.logM, nv, d.tw, lds, lds, dst2);
    }
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

// Bluestein tables of an N-point DFT computed with M-point FFTs, FP64 rounded once: the chirp
// w_n = exp(-i pi n^2 / N) (angles reduced exactly: n^2 mod 2N) and the filter spectrum
// B_k = sum_m b_m exp(-2 pi i m k / M) over the 2N - 1 non-zero b_m.  Grid (M): one wave per
// k, lane l summing m = l, l + 64, ..., then a fixed shuffle tree; workgroup 0 also writes w.
__global__ __launch_bounds__(64) void k_pb_chirp(int N, int M, float2 *__restrict__ chirp, float2 *__restrict__ filt)
{
    const int k = blockIdx.x;
    if (k == 0)
        for (int n = threadIdx.x; n < N; n += 64) {
            double sn, cs;
            sincospi(-(double)(((int64_t)n * n) % (2 * N)) / N, &sn, &cs);
            chirp[n] = make_float2((float)cs, (float)sn);
        }
    double re = 0.0, im = 0.0;
    for (int m = threadIdx.x; m < N; m += 64) {  // b_m = exp(i pi m^2 / N) at m and at M - m
        const double a = (double)(((int64_t)m * m) % (2 * N)) / N, t = 2.0 * (double)(((int64_t)m * k) % M) / M;
        double sn, cs;
        sincospi(a - t, &sn, &cs);
        re += cs;
        im += sn;
        if (m > 0) {
            sincospi(a + t, &sn, &cs);
            re += cs;
            im += sn;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o);
        im += __shfl_xor(im, o);
    }
    if (threadIdx.x == 0) filt[k] = make_float2((float)re, (float)im);
}

// Per-item statistics, FP64, in three launches so that a large item is read by many
// workgroups: grid (items, nb) with chunk b of an item holding values [d b / nb, d (b+1) / nb).
// Every sum has a fixed order (per thread four interleaved accumulators, a fixed tree over the
// workgroup, the chunks in order), so the result does not depend on the schedule.
__device__ __forceinline__ double pb_chunk_sum(const float *__restrict__ x, int64_t lo, int64_t hi, double mean,
                                               bool centred)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t i = lo + threadIdx.x;
    for (; i + 3 * PB_THREADS < hi; i += 4 * PB_THREADS) {
        const double a = x[i], b = x[i + PB_THREADS], c = x[i + 2 * PB_THREADS], e = x[i + 3 * PB_THREADS];
        if (centred) {
            s0 = fma(a - mean, a - mean, s0);
            s1 = fma(b - mean, b - mean, s1);
            s2 = fma(c - mean, c - mean, s2);
            s3 = fma(e - mean, e - mean, s3);
        } else {
            s0 += a;
            s1 += b;
            s2 += c;
            s3 += e;
        }
    }
    for (; i < hi; i += PB_THREADS) {
        const double a = x[i];
        s0 = centred ? fma(a - mean, a - mean, s0) : s0 + a;
    }
    double r = (s0 + s1) + (s2 + s3);
    for (int o = 32; o > 0; o >>= 1) r += __shfl_xor(r, o);
    __shared__ double red[PB_THREADS / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// The item's mean from its nb chunk sums (the same arithmetic wherever it is needed).
__device__ __forceinline__ double pb_mean(const double *__restrict__ part, int nb, int64_t d)
{
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[b];
    return s / (double)d;
}

// Pass 1: chunk sums of the values to part[item][b].
__global__ __launch_bounds__(PB_THREADS) void k_pb_sum(const float *__restrict__ X, int64_t ld, int64_t d,
                                                       double *__restrict__ part)
{
    const int nb = gridDim.y, b = blockIdx.y;
    const double r = pb_chunk_sum(X + (int64_t)blockIdx.x * ld, d * b / nb, d * (b + 1) / nb, 0.0, false);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * nb + b] = r;
}

// Pass 2: chunk sums of the squared centred values to part2[item][b].
__global__ __launch_bounds__(PB_THREADS) void k_pb_sumsq(const float *__restrict__ X, int64_t ld, int64_t d,
                                                         const double *__restrict__ part, double *__restrict__ part2)
{
    const int nb = gridDim.y, b = blockIdx.y;
    __shared__ double mean;
    if (threadIdx.x == 0) mean = pb_mean(part + (int64_t)blockIdx.x * nb, nb, d);
    __syncthreads();
    const double r = pb_chunk_sum(X + (int64_t)blockIdx.x * ld, d * b / nb, d * (b + 1) / nb, mean, true);
    if (threadIdx.x == 0) part2[(int64_t)blockIdx.x * nb + b] = r;
}

// Pass 3, one thread per item: (mean, 1 / norm of the centred values) and live = non-zero
// variance (a constant item gets a zero spectrum).
__global__ void k_pb_stats(const double *__restrict__ part, const double *__restrict__ part2, int nb, int64_t n,
                           int64_t d, double2 *__restrict__ st, int *__restrict__ live)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ss = 0.0;
    for (int b = 0; b < nb; ++b) ss += part2[i * nb + b];
    st[i] = make_double2(pb_mean(part + i * nb, nb, d), ss > 0.0 ? 1.0 / sqrt(ss) : 0.0);
    live[i] = ss > 0.0;
}

// Prepare, rows: grid (ceil(H / RB), items), RB rows per workgroup (the last may hold fewer).
// The rows, centred and scaled (FP64, rounded once), transformed along the row; columns
// 0 .. W/2 go to F.
template <bool BLUE>
__global__ __launch_bounds__(PB_NT) void k_pb_prep_rows(const float *__restrict__ X, int64_t ld, int H, int W, int RB,
                                                        int64_t i0, const double2 *__restrict__ st, PbDim dW,
                                                        float2 *__restrict__ F)
{
    extern __shared__ float2 pb_sm[];
    const int64_t i = i0 + blockIdx.y;
    const int r0 = blockIdx.x * RB, nr = min(RB, H - r0), WH = W / 2 + 1;
    const double2 ms = st[i];
    const float *x = X + i * ld + (int64_t)r0 * W;
    float2 *f = F + i * (int64_t)H * WH + (int64_t)r0 * WH;
    auto src = [&](int v, int e) { return make_float2((float)(((double)x[v * W + e] - ms.x) * ms.y), 0.f); };
    auto dst = [&](int v, int e, float2 val) {
        if (e <= W / 2) f[v * WH + e] = val;
    };
    pb_dft<BLUE, false, false, PB_NT>(dW, nr, PbLds{pb_sm, pb_ld(dW.M)}, src, dst);
}

// Column transforms in place over F (H x WH, row-major): grid (ceil(WH / CB), items), CB columns
// per workgroup (fewer in the last).
template <bool BLUE>
__global__ __launch_bounds__(PB_NT) void k_pb_prep_cols(float2 *__restrict__ F, int H, int WH, int CB, int64_t i0,
                                                        PbDim dH)
{
    extern __shared__ float2 pb_sm[];
    int bx, by;
    pb_xcd_order(CB < 8, bx, by);  // fewer than 8 columns: rows of 64 bytes shared by workgroups
    float2 *f = F + (i0 + by) * (int64_t)H * WH + bx * CB;
    const int nc = min(CB, WH - bx * CB);
    auto src = [&](int v, int e) { return f[(int64_t)e * WH + v]; };
    auto dst = [&](int v, int e, float2 val) { f[(int64_t)e * WH + v] = val; };
    pb_dft<BLUE, true, true, PB_NT>(dH, nc, PbLds{pb_sm, pb_ld(dH.M)}, src, dst);
}

// Rows of the pair-pair spectrum P = conj(F_a) F_b + i conj(F_c) F_d come in mirror pairs:
// row pair q = 0 holds rows 0 and H/2 (each its own mirror; for odd H row 0 alone, slot 1
// empty), q > 0 rows q and H - q; (H + 1) / 2 row pairs in all.
__device__ __forceinline__ int pb_row(int q, int slot, int H) { return q == 0 ? (slot ? H / 2 : 0) : (slot ? H - q : q); }
__device__ __forceinline__ bool pb_empty(int q, int slot, int H) { return q == 0 && slot && (H & 1); }

// Row pass: grid (ceil((H + 1) / 2 / KP), pair-pairs of the batch), KP mirror row pairs per
// workgroup (the last may hold fewer).  pp[q] = (a, b, c, d): the pairs (a, b) and (c, d)
// (c < 0: no second pair).  Column c <= W/2 of a row comes from the half spectra at that row;
// column W - c (0 < c, W - c > W/2) is conj(Z1) + i conj(Z2) taken at the mirror row, column
// c.  Rows are transformed and written to Q, which holds each pair-pair's transform as
// ceil(W / CB) blocks of H x CB values (CB = 2^logCB).  lhc = log2 of hc = (W + 1) / 2, or -1
// if hc is not a power of two.
template <bool BLUE>
__global__ __launch_bounds__(PB_NT) void k_pb_rowpass(const float2 *__restrict__ F, const int4 *__restrict__ pp, int H,
                                                   int W, int lhc, int KP, int logCB, PbDim dW, float2 *__restrict__ Q)
{
    extern __shared__ float2 pb_sm[];
    const int4 p = pp[blockIdx.y];
    const int q0 = blockIdx.x * KP, nq = min(KP, (H + 1) / 2 - q0), lw = pb_ld(dW.M), WH = W / 2 + 1, hw = W / 2;
    const int hc = (W + 1) / 2;  // columns 0 .. hc - 1 with their mirrors (odd W: all but none)
    const int64_t NH = (int64_t)H * WH;
    const bool two = p.z >= 0;
    const float2 *fa = F + p.x * NH, *fb = F + p.y * NH;
    const float2 *fc = F + (two ? p.z : p.x) * NH, *fd = F + (two ? p.w : p.y) * NH;
    const bool same_a = p.z == p.x;  // consecutive pairs of a tile row share their first item
    // columns 0 .. hc - 1 of every row and their mirrors (at most PB_TILE / 2 elements: all
    // loads of a thread are issued before the first LDS store), then for even W column W/2
    constexpr int G = PB_EPT / 2;
    const int nmain = 2 * nq * hc;
    auto split = [&](int t, int &v, int &c) {
        if (lhc >= 0) {
            v = t >> lhc;
            c = t & (hc - 1);
        } else {
            v = t / hc;
            c = t - v * hc;
        }
    };
    float2 va[G], vb[G], vc[G], vd[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int t = threadIdx.x + g * PB_NT;
        if (t < nmain) {
            int v, c;
            split(t, v, c);
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
            int v, c;
            split(t, v, c);
            const int q = q0 + (v >> 1);
            const float2 z1 = pb_cjmul(va[g], vb[g]);
            const float2 z2 = two ? pb_cjmul(vc[g], vd[g]) : make_float2(0.f, 0.f);
            pb_sm[v * lw + pb_pad(c)] = make_float2(z1.x - z2.y, z1.y + z2.x);
            if (c > 0) {
                const int mv = q == 0 ? v : (v ^ 1);
                pb_sm[mv * lw + pb_pad(W - c)] = make_float2(z1.x + z2.y, z2.x - z1.y);
            }
        }
    }
    if (!(W & 1) && (int)threadIdx.x < 2 * nq) {  // even W: column W/2 is its own mirror
        const int v = threadIdx.x;
        const int64_t e = (int64_t)pb_row(q0 + (v >> 1), v & 1, H) * WH + hw;
        const float2 z1 = pb_cjmul(fa[e], fb[e]);
        const float2 z2 = two ? pb_cjmul(fc[e], fd[e]) : make_float2(0.f, 0.f);
        pb_sm[v * lw + pb_pad(hw)] = make_float2(z1.x - z2.y, z1.y + z2.x);
    }
    __syncthreads();
    float2 *q = Q + (int64_t)blockIdx.y * H * (((W + (1 << logCB) - 1) >> logCB) << logCB);
    const PbLds lds{pb_sm, lw};
    const int cbm = (1 << logCB) - 1;
    auto dst = [&](int v, int e, float2 val) {
        if (!pb_empty(q0 + (v >> 1), v & 1, H))
            q[((int64_t)(e >> logCB) * H + pb_row(q0 + (v >> 1), v & 1, H)) * (cbm + 1) + (e & cbm)] = val;
    };
    pb_dft<BLUE, false, false, PB_NT>(dW, 2 * nq, lds, lds, dst);
}

// Row pass for rows of 8K-point transforms: grid (H, pair-pairs), one row per workgroup of
// PB_NT threads and one LDS vector (two workgroups per CU).  Row r takes columns 0 .. W/2 from
// the half spectra at row r and columns W - c from its mirror row (as in k_pb_rowpass); the
// two workgroups of a mirror pair are neighbours in the XCD-aware order, so the second
// reads the shared spectra rows from the same L2.  Workgroup b takes slot b of the row pairs
// in order (for odd H, row pair 0 holds row 0 only, and b > 0 counts from slot 2).
template <bool BLUE>
__global__ __launch_bounds__(PB_NT) void k_pb_rowpass_one(const float2 *__restrict__ F, const int4 *__restrict__ pp,
                                                          int H, int W, int logCB, PbDim dW, float2 *__restrict__ Q)
{
    extern __shared__ float2 pb_sm[];
    int bx, by;
    pb_xcd_order(true, bx, by);
    const int4 p = pp[by];
    const int b2 = (H & 1) && bx > 0 ? bx + 1 : bx;
    const int q0 = b2 >> 1, slot = b2 & 1, WH = W / 2 + 1, hw = W / 2, hc = (W + 1) / 2;
    const int r = pb_row(q0, slot, H), rm = pb_row(q0, q0 ? slot ^ 1 : slot, H);  // rows 0, H/2: own mirrors
    const int64_t NH = (int64_t)H * WH;
    const bool two = p.z >= 0;
    const float2 *fa = F + p.x * NH, *fb = F + p.y * NH;
    const float2 *fc = F + (two ? p.z : p.x) * NH, *fd = F + (two ? p.w : p.y) * NH;
    // column c of row r is z1 + i z2 at (r, c); column W - c is conj(z1) + i conj(z2) at (rm, c)
    constexpr int G = 4096 / 2 / PB_NT;  // columns 0 .. hc - 1 per thread (W <= 4096)
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int c = threadIdx.x + g * PB_NT;
        if (c < hc) {
            const int64_t e = (int64_t)r * WH + c, em = (int64_t)rm * WH + c;
            const float2 u1 = pb_cjmul(fa[e], fb[e]), m1 = pb_cjmul(fa[em], fb[em]);
            const float2 u2 = two ? pb_cjmul(fc[e], fd[e]) : make_float2(0.f, 0.f);
            const float2 m2 = two ? pb_cjmul(fc[em], fd[em]) : make_float2(0.f, 0.f);
            pb_sm[pb_pad(c)] = make_float2(u1.x - u2.y, u1.y + u2.x);
            if (c > 0) pb_sm[pb_pad(W - c)] = make_float2(m1.x + m2.y, m2.x - m1.y);
        }
    }
    if (!(W & 1) && threadIdx.x == 0) {  // even W: column W/2 is its own mirror
        const int64_t e = (int64_t)r * WH + hw;
        const float2 z1 = pb_cjmul(fa[e], fb[e]);
        const float2 z2 = two ? pb_cjmul(fc[e], fd[e]) : make_float2(0.f, 0.f);
        pb_sm[pb_pad(hw)] = make_float2(z1.x - z2.y, z1.y + z2.x);
    }
    pb_barrier();
    const int CB = 1 << logCB, cbm = CB - 1;
    float2 *qo = Q + (int64_t)by * H * ((W + CB - 1) / CB * CB);
    auto dst = [&](int v, int e, float2 x) { qo[((int64_t)(e >> logCB) * H + r) * CB + (e & cbm)] = x; };
    pb_dft<BLUE, false, false, PB_NT>(dW, 1, PbLds{pb_sm, pb_ld(dW.M)}, PbLds{pb_sm, pb_ld(dW.M)}, dst);
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

// Energy of the cells of the (2h+1)^2 neighbourhood of the peak (r0, c0) of channel ch in
// columns k0 .. k0 + m - 1 of it (at most one LDS tile): those columns of the row-pass output
// q are transformed again by the same code as in the column pass (so to the same values).
// Valid in thread 0.
template <bool BLUE>
__device__ double pb_inside(const float2 *__restrict__ q, int H, int W, int logCB, int h, int k0, int m, int r0,
                            int c0, int ch, const PbDim &dH, const PbLds &lds)
{
    const int cbm = (1 << logCB) - 1;
    const int side = 2 * h + 1;
    double inside = 0.0;
    const int cs = c0 - h + k0 + W;
    auto src = [&](int v, int e) {
        const int c = (cs + v) % W;
        return q[((int64_t)(c >> logCB) * H + e) * (cbm + 1) + (c & cbm)];
    };
    auto dst = [&](int v, int e, float2 val) {
        if ((e - r0 + h + H) % H < side) {
            const double x = ch ? val.y : val.x;
            inside = fma(x, x, inside);
        }
    };
    pb_dft<BLUE, true, false, PB_NT>(dH, m, lds, src, dst);
    for (int o = 32; o > 0; o >>= 1) inside += __shfl_xor(inside, o);
    __shared__ double red[PB_NT / 64];
    pb_barrier();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = inside;
    pb_barrier();
    if (threadIdx.x == 0)
        for (int w = 1; w < PB_NT / 64; ++w) inside += red[w];
    return inside;
}

// Column pass: grid (ceil(W / CBS), pair-pairs): the workgroup's CBS columns (fewer in the
// last) are transformed from the row-pass output (left as it is), and the workgroup's peak
// (largest value, smallest shift index on ties) and FP64 energy per channel go to S.  CBS
// divides the block width CB, or one workgroup covers all W columns.
template <int NT, bool BLUE>
__global__ __launch_bounds__(NT) void k_pb_colpass(const float2 *__restrict__ Q, int H, int W, int logCB, int CBS,
                                                      PbDim dH, PbStat *__restrict__ S)
{
    extern __shared__ float2 pb_sm[];
    const int CB = 1 << logCB, Wp = ((W + CB - 1) >> logCB) << logCB;
    int bx, by;
    pb_xcd_order(CBS < CB, bx, by);  // the workgroups of one block share its cache lines
    const int c0 = bx * CBS, nc = min(CBS, W - c0);
    const float2 *qb = Q + (int64_t)by * H * Wp + (int64_t)(c0 >> logCB) * H * CB + (c0 & (CB - 1));
    PbStat st{-INFINITY, -INFINITY, 0x7fffffff, 0x7fffffff, 0.0, 0.0};
    auto src = [&](int v, int e) { return qb[e * CB + v]; };
    auto dst = [&](int v, int e, float2 val) {
        const int idx = e * W + c0 + v;
        pb_merge(st, val.x, val.y, idx, idx, (double)val.x * val.x, (double)val.y * val.y);
    };
    pb_dft<BLUE, true, false, NT>(dH, nc, PbLds{pb_sm, pb_ld(dH.M)}, src, dst);
    st = pb_reduce<NT>(st);
    if (threadIdx.x == 0) S[(int64_t)by * gridDim.x + bx] = st;
}

// Peak and neighbourhood: grid (2 G, pair-pairs), workgroup (channel, group g of CF of the
// 2h+1 columns around the peak).  Each workgroup merges the blocks' statistics into the
// channel's peak s* and total energy (the same in every workgroup), transforms its columns
// again and writes their energy inside the (2h+1)^2 neighbourhood to E; group 0 also writes
// the channel's totals to T.
template <bool BLUE>
__global__ __launch_bounds__(PB_NT) void k_pb_peak(const float2 *__restrict__ Q, const PbStat *__restrict__ S, int nblk,
                                                   const int4 *__restrict__ pp, int H, int W, int logCB, int h, int CF,
                                                   PbDim dH, PbStat *__restrict__ T, double *__restrict__ E)
{
    extern __shared__ float2 pb_sm[];
    const int ch = blockIdx.x & 1, g = blockIdx.x >> 1, G = gridDim.x >> 1;
    const int4 p = pp[blockIdx.y];
    if (ch == 1 && p.z < 0) return;  // a single pair: no second channel (uniform over the workgroup)
    const PbStat *s = S + (int64_t)blockIdx.y * nblk;
    PbStat r{-INFINITY, -INFINITY, 0x7fffffff, 0x7fffffff, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += PB_NT) pb_merge(r, s[b].v0, s[b].v1, s[b].i0, s[b].i1, s[b].e0, s[b].e1);
    r = pb_reduce<PB_NT>(r);
    __shared__ int pk;
    if (threadIdx.x == 0) pk = ch ? r.i1 : r.i0;
    pb_barrier();
    const bool found = pk != 0x7fffffff;  // false only for NaN surfaces
    const int CB = 1 << logCB, Wp = ((W + CB - 1) >> logCB) << logCB;
    const int k0 = g * CF;
    const double inside = pb_inside<BLUE>(Q + (int64_t)blockIdx.y * H * Wp, H, W, logCB, h, k0,
                                          min(CF, 2 * h + 1 - k0), found ? pk / W : 0, found ? pk % W : 0, ch, dH,
                                          PbLds{pb_sm, pb_ld(dH.M)});
    if (threadIdx.x == 0) {
        E[((int64_t)blockIdx.y * 2 + ch) * G + g] = inside;
        if (g == 0) T[(int64_t)blockIdx.y * 2 + ch] = r;
    }
}

// PCE per pair: one thread per (pair-pair, channel) of the batch, the neighbourhood energy
// summed over the G groups in order.
__global__ void k_pb_pce(const PbStat *__restrict__ T, const double *__restrict__ E, int G, int nb,
                         const int4 *__restrict__ pp, const int *__restrict__ live, int H, int W, int h, int64_t n,
                         float *__restrict__ out, uint32_t *__restrict__ peak_out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x, q = t >> 1, ch = t & 1;
    if (q >= nb) return;
    const int4 p = pp[q];
    if (ch == 1 && p.z < 0) return;
    const PbStat r = T[t];
    double inside = 0.0;
    for (int g = 0; g < G; ++g) inside += E[(int64_t)t * G + g];
    const int pk = ch ? r.i1 : r.i0;
    const double pv = ch ? r.v1 : r.v0, rest = (ch ? r.e1 : r.e0) - inside;
    const double num = pv * pv * (double)((int64_t)H * W - (int64_t)(2 * h + 1) * (2 * h + 1));
    const int64_t i = ch ? p.z : p.x, j = ch ? p.w : p.y;
    const int64_t pidx = i * n - i * (i + 1) / 2 + (j - i - 1);
    const bool ok = pk != 0x7fffffff && live[i] && live[j] && rest > 0.0;
    out[pidx] = ok ? (float)(num / rest) : __builtin_nanf("");
    if (peak_out) peak_out[pidx] = ok ? (uint32_t)pk : 0u;
}

int log2_exact(int64_t v)
{
    int l = 0;
    while (((int64_t)1 << l) < v) ++l;
    return ((int64_t)1 << l) == v ? l : -1;
}

// LDS bytes of a workgroup holding M padded vectors of N complex values
size_t tile_lds(int M, int N) { return (size_t)M * pb_ld(N) * sizeof(float2); }

// FFT length of an N-point axis: N itself for powers of two, else the Bluestein length
int fft_len(int N)
{
    if (log2_exact(N) >= 0) return N;
    int M = 1;
    while (M < 2 * N - 1) M *= 2;
    return M;
}

struct PbLayout {
    size_t spec, stats, live, tab, part;
    int MH, MW, nb;
};

// spectra | per item (mean, 1/norm) | live flags | per axis (H, then W): FFT twiddles (M),
// Bluestein chirp (N) and filter spectrum (M) | the statistics' chunk sums (two per chunk)
PbLayout layout(int64_t n, int H, int W)
{
    const int64_t m = std::max<int64_t>(n, 1);
    PbLayout l;
    l.MH = fft_len(H);
    l.MW = fft_len(W);
    // chunks of at least 16K values per item, at most 64, and at least 2048 workgroups where
    // the item count allows it
    const int64_t d = (int64_t)H * W;
    l.nb = (int)std::max<int64_t>(1, std::min<int64_t>({64, d / 16384, (2048 + m - 1) / m}));
    l.part = (size_t)m * l.nb * 2 * sizeof(double);
    l.spec = (size_t)m * H * (W / 2 + 1) * sizeof(float2);
    l.stats = (size_t)m * sizeof(double2);
    l.live = ((size_t)m * sizeof(int) + 255) & ~(size_t)255;
    l.tab = (size_t)(2 * l.MH + H + 2 * l.MW + W) * sizeof(float2);
    return l;
}

// the axis descriptors over the tables at tab (see layout)
void axes(const PbLayout &l, int H, int W, float2 *tab, PbDim &dH, PbDim &dW)
{
    dH = PbDim{H, l.MH, log2_exact(l.MH), tab, tab + l.MH, tab + l.MH + H};
    float2 *t = tab + 2 * l.MH + H;
    dW = PbDim{W, l.MW, log2_exact(l.MW), t, t + l.MW, t + l.MW + W};
}

rocket_status set_lds(rocket_ctx *ctx, const void *k, size_t bytes)
{
    RK_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return ROCKET_OK;
}

}  // namespace

bool pce_big_shape(int64_t H, int64_t W)
{
    // sides in [16, 4096] (FFT lengths up to 8192: one LDS tile)
    return H >= 16 && W >= 16 && H <= 4096 && W <= 4096;
}

rocket_status pce_big_prepare(rocket_ctx *ctx, const rocket_items *it, int64_t n, int H, int W, hipStream_t s)
{
    PceState &p = ctx->pce;
    if (!ctx->arena && !p.side) {  // the compare's second stream and its events, made here and not under a capture
        for (hipEvent_t *e : {&p.fork, &p.join, &p.staged[0], &p.staged[1], &p.consumed[0], &p.consumed[1]})
            if (!*e) RK_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
        RK_HIP(hipStreamCreateWithFlags(&p.side, hipStreamNonBlocking));  // last: a set stream means all events exist
    }
    const int WH = W / 2 + 1;
    const PbLayout l = layout(n, H, W);
    ctx->trace_valid = false;  // batched launches, no persistent queue to trace
    void *buf = nullptr;
    RK_TRY(ws_get(ctx, WS_PCE_SPEC, l.spec + l.stats + l.live + l.tab + l.part, &buf));
    float2 *F = (float2 *)buf;
    double2 *st = (double2 *)((char *)buf + l.spec);
    int *live = (int *)((char *)st + l.stats);
    PbDim dH, dW;
    axes(l, H, W, (float2 *)((char *)live + l.live), dH, dW);
    for (const PbDim *d : {&dH, &dW}) {
        hipLaunchKernelGGL(k_pb_twiddles, dim3(8), dim3(256), 0, s, (float2 *)d->tw, d->logM);
        if (d->M != d->N)
            hipLaunchKernelGGL(k_pb_chirp, dim3((unsigned)d->M), dim3(64), 0, s, d->N, d->M, (float2 *)d->chirp,
                               (float2 *)d->filt);
        RK_HIP(hipGetLastError());
    }
    if (n > 0) {
        double *part = (double *)((char *)live + l.live + l.tab), *part2 = part + n * l.nb;
        hipLaunchKernelGGL(k_pb_sum, dim3((unsigned)n, (unsigned)l.nb), dim3(PB_THREADS), 0, s, it->dense, it->ld,
                           it->dim, part);
        hipLaunchKernelGGL(k_pb_sumsq, dim3((unsigned)n, (unsigned)l.nb), dim3(PB_THREADS), 0, s, it->dense, it->ld,
                           it->dim, (const double *)part, part2);
        hipLaunchKernelGGL(k_pb_stats, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const double *)part,
                           (const double *)part2, l.nb, n, it->dim, st, live);
        RK_HIP(hipGetLastError());
        const int RB = std::min(H, PB_TILE / l.MW);  // rows per workgroup
        const int CB = PB_TILE / l.MH;               // columns per workgroup
        const size_t rl = tile_lds(RB, l.MW), cl = tile_lds(CB, l.MH);
        // Bluestein instantiations per axis (a side that is not a power of two)
        const auto kr = l.MW != W ? &k_pb_prep_rows<true> : &k_pb_prep_rows<false>;
        const auto kc = l.MH != H ? &k_pb_prep_cols<true> : &k_pb_prep_cols<false>;
        RK_TRY(set_lds(ctx, (const void *)kr, rl));
        RK_TRY(set_lds(ctx, (const void *)kc, cl));
        for (int64_t i0 = 0; i0 < n; i0 += 65535) {
            const unsigned ni = (unsigned)std::min<int64_t>(65535, n - i0);
            hipLaunchKernelGGL(kr, dim3((unsigned)((H + RB - 1) / RB), ni), dim3(PB_NT), rl, s, it->dense,
                               it->ld, H, W, RB, i0, st, dW, F);
            hipLaunchKernelGGL(kc, dim3((unsigned)((WH + CB - 1) / CB), ni), dim3(PB_NT), cl, s, F, H, WH,
                               CB, i0, dH);
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
    PbDim dH, dW;
    axes(l, H, W, (float2 *)((const char *)live + l.live), dH, dW);
    // column-pass workgroups: CBS columns each (one LDS tile; 256 threads over 4K values where
    // a column fits, four workgroups per CU).  The staged transform is stored column block by
    // column block ([ceil(W / CB)][H][CB], CB a power of two >= CBS, at least 8 where W allows,
    // so that the row pass stores runs of 64 bytes or more), so that the workgroups of one
    // block read one contiguous piece
    const int CNT = l.MH <= PB_TILE / 2 ? PB_NT / 2 : PB_NT;
    const int CBS = std::min(W, CNT * PB_EPT / l.MH);
    int CB = 1;
    while (CB < std::min(W, std::max(CBS, 8))) CB *= 2;
    const int logCB = log2_exact(CB), Wp = (W + CB - 1) / CB * CB;
    const int nblk = (W + CBS - 1) / CBS;  // column-pass workgroups (and statistics) per transform
    // row-pass workgroups: KP mirror row pairs, 2 KP vectors of MW values; rows of 8K-point
    // transforms one per workgroup (k_pb_rowpass_one)
    const bool wide = 2 * l.MW > PB_TILE;
    const int NQ = (H + 1) / 2;  // row pairs (odd H: the first holds row 0 alone)
    const int KP = wide ? 1 : std::max(1, std::min(NQ, PB_TILE / (2 * l.MW)));
    const int lhc = log2_exact((W + 1) / 2);
    // neighbourhood columns transformed again per workgroup, G groups of them
    const int CF = std::min(2 * h + 1, PB_TILE / l.MH), G = (2 * h + CF) / CF;
    // batch of pair-pairs: one staged H x Wp complex transform, nblk block statistics, and per
    // channel the totals and G neighbourhood energies each
    const int64_t per = (int64_t)H * Wp * (int64_t)sizeof(float2) + (nblk + 2) * (int64_t)sizeof(PbStat) +
                        2 * G * (int64_t)sizeof(double);
    // Two staging buffers where the workspace allows two batches and the library may create a
    // stream (not in the allocation-free arena): the row pass of batch b + 1 (caller's stream)
    // then runs while the column, peak and PCE kernels of batch b run on a second stream.
    // Batch: ROCKET_OPT_PCE_BATCH pair-pairs, else as many as 512 MiB holds (64 of 1024 x 1024,
    // so 1 GiB of staging with two buffers).
    int64_t room = INT64_MAX;  // transforms the workspace cap (or the arena) leaves room for
    const int64_t held = (int64_t)ctx->ws[WS_PCE_STAGE].bytes;
    if (ctx->arena)  // a slot that grows takes a new piece of the arena
        room = (std::max<int64_t>(held, (int64_t)(ctx->arena_cap - ctx->arena_used)) - 256) / per;
    else if (ctx->opt[ROCKET_OPT_WORKSPACE_CAP] > 0)  // allocations are rounded up to 2 MiB
        room = (ctx->opt[ROCKET_OPT_WORKSPACE_CAP] - ws_total(ctx) + held - ((int64_t)2 << 20)) / per;
    if (room < 1) return fail(ctx, ROCKET_E_OOM, "workspace cap leaves no room for one staged PCE transform");
    const int64_t fill = std::max<int64_t>(1, PB_STAGE_BYTES / ((int64_t)H * Wp * 8));
    const int64_t want = ctx->opt[ROCKET_OPT_PCE_BATCH] > 0 ? ctx->opt[ROCKET_OPT_PCE_BATCH] : fill;
    const int64_t B1 = std::min<int64_t>({npp, 65535, want, room});  // batch with one buffer
    const bool two = !ctx->arena && p.side && room >= 2 && npp > B1;  // more than one batch to overlap
    const int64_t B = two ? std::min<int64_t>(B1, room / 2) : B1;
    void *stage = nullptr;
    RK_TRY(ws_get(ctx, WS_PCE_STAGE, (size_t)((two ? 2 : 1) * B * per), &stage));
    const int4 *pp = (const int4 *)ctx->ws[WS_QUEUE_ITEMS].ptr;
    const size_t rl = tile_lds(wide ? 1 : 2 * KP, l.MW), cl = tile_lds(CBS, l.MH);
    // Bluestein instantiations per axis; 8K-point rows occur only with Bluestein (W <= 4096)
    const bool bw = l.MW != W, bh = l.MH != H;
    const auto kr = bw ? &k_pb_rowpass<true> : &k_pb_rowpass<false>;
    const auto kw = &k_pb_rowpass_one<true>;
    const auto kc = CNT < PB_NT ? (bh ? &k_pb_colpass<PB_NT / 2, true> : &k_pb_colpass<PB_NT / 2, false>)
                                : (bh ? &k_pb_colpass<PB_NT, true> : &k_pb_colpass<PB_NT, false>);
    const auto kf = bh ? &k_pb_peak<true> : &k_pb_peak<false>;
    RK_TRY(set_lds(ctx, wide ? (const void *)kw : (const void *)kr, rl));
    RK_TRY(set_lds(ctx, (const void *)kc, cl));
    const size_t fl = tile_lds(CF, l.MH);
    RK_TRY(set_lds(ctx, (const void *)kf, fl));
    const hipStream_t cs = two ? p.side : s;  // stream of the column, peak and PCE kernels
    ctx->stats.grid = B;
    RK_TRY(timing_begin(ctx, s));
    if (two) {  // the second stream starts after everything queued on the caller's stream
        RK_HIP(hipEventRecord(p.fork, s));
        RK_HIP(hipStreamWaitEvent(cs, p.fork, 0));
    }
    const unsigned rgrid = (unsigned)((NQ + KP - 1) / KP);
    int64_t b = 0;
    for (int64_t q0 = 0; q0 < npp; q0 += B, ++b) {
        const unsigned nb = (unsigned)std::min<int64_t>(B, npp - q0);
        const int k = two ? (int)(b & 1) : 0;
        char *buf = (char *)stage + k * B * per;  // buffer k: Q [B][H][Wp] | S [B][nblk] | T [B][2] | E [B][2][G]
        float2 *Q = (float2 *)buf;
        PbStat *S = (PbStat *)(buf + B * (int64_t)H * Wp * sizeof(float2));
        PbStat *T = S + B * nblk;
        double *E = (double *)(T + 2 * B);
        if (two && b >= 2) RK_HIP(hipStreamWaitEvent(s, p.consumed[k], 0));  // batch b - 2 is done with buffer k
        if (wide)
            hipLaunchKernelGGL(kw, dim3(H, nb), dim3(PB_NT), rl, s, F, pp + q0, H, W, logCB, dW, Q);
        else
            hipLaunchKernelGGL(kr, dim3(rgrid, nb), dim3(PB_NT), rl, s, F, pp + q0, H, W, lhc, KP, logCB, dW, Q);
        if (two) {
            RK_HIP(hipEventRecord(p.staged[k], s));
            RK_HIP(hipStreamWaitEvent(cs, p.staged[k], 0));
        }
        hipLaunchKernelGGL(kc, dim3((unsigned)nblk, nb), dim3(CNT), cl, cs, (const float2 *)Q, H, W, logCB, CBS,
                           dH, S);
        hipLaunchKernelGGL(kf, dim3(2 * G, nb), dim3(PB_NT), fl, cs, (const float2 *)Q, (const PbStat *)S, nblk,
                           pp + q0, H, W, logCB, h, CF, dH, T, E);
        hipLaunchKernelGGL(k_pb_pce, dim3((2 * nb + 255) / 256), dim3(256), 0, cs, (const PbStat *)T, (const double *)E,
                           G, (int)nb, pp + q0, live, H, W, h, n, out, peak);
        RK_HIP(hipGetLastError());
        if (two) RK_HIP(hipEventRecord(p.consumed[k], cs));
    }
    if (two) {  // the caller's stream continues after the second stream's last kernel
        RK_HIP(hipEventRecord(p.join, cs));
        RK_HIP(hipStreamWaitEvent(s, p.join, 0));
    }
    RK_TRY(timing_end(ctx, s));
    return ROCKET_OK;
}

}  // namespace rk
