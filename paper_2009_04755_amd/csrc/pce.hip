// Peak-to-correlation energy (PCE) over all cyclic shifts: the forensics application's PCE
// variant of the pattern comparison (Section V-A; the application's stage table names PCE).
//
//   C(s) = sum_x a(x + s) b(x)   (mean-removed L x L items, indices mod L)
//   s*   = argmax_s C(s),  PCE = C(s*)^2 (L^2 - |N|) / sum_{s not in N} C(s)^2,
//   N    = the (2h+1) x (2h+1) cyclic neighbourhood of s*.
//
// Prepare (l's GPU stage): one workgroup per item removes the mean and scales to unit norm
// (FP64; PCE does not depend on either) and transforms the item with a 2-D FFT in LDS;
// spectra F are stored in natural order, complex f32, columns 0 .. L/2 only (the rest is
// the conjugate mirror).
// Compare: a persistent kernel pulls tiles of T x T item pairs from the work queue (the
// spectra of a tile's 2T items stay in L2); per two pairs one workgroup forms
// conj(F_a) F_b + i conj(F_c) F_d in LDS and transforms it forward: the real part is L^2 times
// the first pair's C(s), the imaginary part the second's (both are real).  Per pair it finds
// the peak and the energy outside its neighbourhood and writes PCE and the peak shift.
//
// The L-point FFTs are four-step L = N1 x N2 transforms: N1-point DFTs in registers
// (radix-2, decimation in frequency), twiddles W_L^(n2 k1) from an LDS table, N2-point
// DFTs in registers.  Each task writes back to the positions it read, so a step needs no
// barrier between its reads and writes; the price is that position p of a transformed
// vector holds frequency k(p) = p / N2 + N1 (p % N2), which prepare undoes when it stores
// the spectra and the statistics undo when they name the peak.
#include <cmath>

#include "common.hpp"
#include "queue.hpp"

namespace rk {
namespace {

constexpr int PCE_THREADS = 256;  // prepare
constexpr int PCE_CMP_THREADS = 512;  // compare: two waves per SIMD hide LDS and L2 latency
constexpr int PCE_T = 8;  // items per block of the tile grid

// cos(pi m / 8) and sin(pi m / 8), m = 0..15
constexpr float kCos16[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f, 0.0f,
                              -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f, -1.0f,
                              -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f, 0.0f,
                              0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
constexpr float kSin16[16] = {0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f, 1.0f,
                              0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f, 0.0f,
                              -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f, -1.0f,
                              -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f};

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}

// d * W_16^m, W_16 = exp(-2 pi i / 16); m is a constant once the DFT loops are unrolled
__device__ __forceinline__ float2 tw16(float2 d, int m)
{
    if (m == 0) return d;
    if (m == 4) return make_float2(d.y, -d.x);
    if (m == 8) return make_float2(-d.x, -d.y);
    if (m == 12) return make_float2(-d.y, d.x);
    const float c = kCos16[m], s = kSin16[m];
    return make_float2(fmaf(d.x, c, d.y * s), fmaf(d.y, c, -(d.x * s)));
}

// In-register N-point forward DFT (N = 2, 4, 8, 16), radix-2 decimation in frequency;
// the output is bit-reversed: X[k] ends in x[rev(k)].
template <int N>
__device__ __forceinline__ void dft_dif(float2 (&x)[N])
{
#pragma unroll
    for (int span = N / 2; span >= 1; span >>= 1)
#pragma unroll
        for (int st = 0; st < N; st += 2 * span)
#pragma unroll
            for (int j = 0; j < span; ++j) {
                const float2 a = x[st + j], b = x[st + j + span];
                x[st + j] = cadd(a, b);
                x[st + j + span] = tw16(csub(a, b), (16 / (2 * span)) * j);
            }
}

template <int N>
__device__ __forceinline__ constexpr int bitrev(int k)
{
    int r = 0;
    for (int b = 1; b < N; b <<= 1) {
        r = (r << 1) | (k & 1);
        k >>= 1;
    }
    return r;
}

// One 2-D forward FFT of the L x L complex array at `a` (row stride RS = L + 1) in place.
// `tw` holds W_L^m, m = 0..L-1.  Position (pr, pc) ends holding frequency (k(pr), k(pc)).
template <int L, int N1, int N2, int NT>
__device__ void fft2d(float2 *a, const float2 *tw)
{
    constexpr int RS = L + 1;
#pragma unroll 1
    for (int dim = 0; dim < 2; ++dim) {
        // rows: vector v at v*RS, element stride 1; columns: vector v at v, stride RS
        const int vstride = dim == 0 ? RS : 1, estride = dim == 0 ? 1 : RS;
        // step A: for every (v, n2): N1-point DFT over n1 of x[N2 n1 + n2], twiddle W_L^(n2 k1)
        // tasks of a thread are unrolled so the LDS reads of all of them are in flight together
#pragma unroll
        for (int it = 0; it < (L * N2 + NT - 1) / NT; ++it) {
            const int id = it * NT + threadIdx.x;
            if (id >= L * N2) break;
            const int v = id % L, n2 = id / L;
            float2 *p = a + v * vstride + n2 * estride;
            float2 x[N1];
#pragma unroll
            for (int n1 = 0; n1 < N1; ++n1) x[n1] = p[n1 * N2 * estride];
            dft_dif<N1>(x);
#pragma unroll
            for (int k1 = 0; k1 < N1; ++k1) p[k1 * N2 * estride] = cmul(x[bitrev<N1>(k1)], tw[n2 * k1]);
        }
        __syncthreads();
        // step B: for every (v, k1): N2-point DFT over n2 of y[N2 k1 + n2], written back in place
#pragma unroll
        for (int it = 0; it < (L * N1 + NT - 1) / NT; ++it) {
            const int id = it * NT + threadIdx.x;
            if (id >= L * N1) break;
            const int v = id % L, k1 = id / L;
            float2 *p = a + v * vstride + k1 * N2 * estride;
            float2 x[N2];
#pragma unroll
            for (int n2 = 0; n2 < N2; ++n2) x[n2] = p[n2 * estride];
            dft_dif<N2>(x);
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) p[k2 * estride] = x[bitrev<N2>(k2)];
        }
        __syncthreads();
    }
}

template <int L>
__device__ void fill_twiddles(float2 *tw)
{
    for (int m = threadIdx.x; m < L; m += blockDim.x) {
        double s, c;
        sincospi(-2.0 * m / L, &s, &c);
        tw[m] = make_float2((float)c, (float)s);
    }
}

// frequency held at position p of a transformed vector, and the position of frequency k
template <int N1, int N2>
__device__ __forceinline__ int freq_of(int p)
{
    return p / N2 + N1 * (p % N2);
}
template <int N1, int N2>
__device__ __forceinline__ int pos_of(int k)
{
    return N2 * (k % N1) + k / N1;
}

// Prepare: grid = n items.  X: f32 [n][ld], item = L*L values row-major.  F: [n][L*L] float2.
template <int L, int N1, int N2>
__global__ __launch_bounds__(PCE_THREADS) void k_pce_prepare(const float *__restrict__ X, int64_t ld,
                                                             float2 *__restrict__ F, int *__restrict__ live)
{
    constexpr int RS = L + 1;
    extern __shared__ float2 sm[];
    float2 *a = sm, *tw = sm + L * RS;
    __shared__ double red[PCE_THREADS / 64];
    const float *x = X + (int64_t)blockIdx.x * ld;
    fill_twiddles<L>(tw);
    double s = 0.0;
    for (int i = threadIdx.x; i < L * L; i += PCE_THREADS) s += (double)x[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    const double mean = ((red[0] + red[1]) + (red[2] + red[3])) / (double)(L * L);
    __syncthreads();
    // unit norm: correlation scale is the same for every pair (two pairs share one FFT)
    double q = 0.0;
    for (int i = threadIdx.x; i < L * L; i += PCE_THREADS) {
        const double c = (double)x[i] - mean;
        q = fma(c, c, q);
    }
    for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
    __syncthreads();
    const double ss = (red[0] + red[1]) + (red[2] + red[3]);
    const double inv = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;  // a constant item gets a zero spectrum
    if (threadIdx.x == 0) live[blockIdx.x] = ss > 0.0;
    for (int i = threadIdx.x; i < L * L; i += PCE_THREADS)
        a[(i / L) * RS + i % L] = make_float2((float)(((double)x[i] - mean) * inv), 0.f);
    __syncthreads();
    fft2d<L, N1, N2, PCE_THREADS>(a, tw);
    // real input: F(-k) = conj F(k), so only columns kc = 0 .. L/2 are stored
    constexpr int LH = L / 2 + 1;
    float2 *f = F + (int64_t)blockIdx.x * L * LH;
    for (int i = threadIdx.x; i < L * LH; i += PCE_THREADS)
        f[i] = a[pos_of<N1, N2>(i / LH) * RS + pos_of<N1, N2>(i % LH)];
}

// Compare: persistent; work item = tile (bi, bj) of PCE_T-item blocks, bi <= bj.  The
// tile's pairs are taken two at a time: C1 and C2 are real, so one forward FFT of
// conj(Z1) + i conj(Z2) gives L^2 C1 in the real and L^2 C2 in the imaginary part.
template <int L, int N1, int N2>
__global__ __launch_bounds__(PCE_CMP_THREADS, 1) void k_pce(const float2 *__restrict__ F, const int *__restrict__ live,
                                                            int n, int h, QueueArgs q, float *__restrict__ out,
                                                            uint32_t *__restrict__ peak_out)
{
    constexpr int RS = L + 1;
    constexpr int NV = L * L;
    constexpr int NT = PCE_CMP_THREADS, NW = NT / 64;
    static_assert(NT == 512 && NT % L == 0, "two channels of 256 threads; whole rows per pass");
    extern __shared__ float2 sm[];
    float2 *a = sm, *tw = sm + L * RS;
    __shared__ float s_val[2][NW];
    __shared__ int s_idx[2][NW];
    __shared__ double s_sum[2][NW];
    __shared__ double s_in[NW];
    __shared__ int s_item;
    fill_twiddles<L>(tw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nb_side = 2 * h + 1 < L ? 2 * h + 1 : L;
    int prev = -1;
    for (;;) {
        const int it = queue_pop_wg(q, &s_item, prev);
        if (it < 0) break;
        const int4 w = q.items[it];
        const int i0 = w.x * PCE_T, i1 = min(n, i0 + PCE_T), j0 = w.y * PCE_T, j1 = min(n, j0 + PCE_T);
        // pairs of the tile in row-major order, i < j
        int pi[2], pj[2];
        int ci = i0, cj = max(j0, i0 + 1);
        auto next_pair = [&](int &oi, int &oj) -> bool {
            while (ci < i1 && cj >= j1) {
                ++ci;
                cj = max(j0, ci + 1);
            }
            if (ci >= i1) return false;
            oi = ci;
            oj = cj++;
            return true;
        };
        // next two pairs of the tile (fewer at its end): their count
        auto take = [&](int (&qi)[2], int (&qj)[2]) {
            int m = 0;
            if (next_pair(qi[0], qj[0])) ++m;
            if (m == 1 && next_pair(qi[1], qj[1])) ++m;
            return m;
        };
        // conj(Z) = conj(F_a) F_b for each pair; the second is packed as the imaginary part.
        // Both are Hermitian (real items), so the half spectrum gives every column: column
        // L - kc of row L - kr holds conj of column kc of row kr for each pair.  The spectra
        // come from L2/HBM in two rounds of LB elements per thread; the first round of the
        // next two pairs is loaded before this pair's transform, so it lands meanwhile.
        constexpr int LH = L / 2 + 1, NH = L * LH;  // stored half spectrum per item
        constexpr int LB = (NH + 2 * NT - 1) / (2 * NT);
        auto load = [&](int e0, const int (&qi)[2], const int (&qj)[2], int m, float2 (&u)[LB], float2 (&v)[LB],
                        float2 (&u2)[LB], float2 (&v2)[LB]) {
            const float2 *fa0 = F + (int64_t)qi[0] * NH, *fb0 = F + (int64_t)qj[0] * NH;
            const float2 *fa1 = F + (int64_t)qi[m - 1] * NH, *fb1 = F + (int64_t)qj[m - 1] * NH;
            const bool two = m == 2;
#pragma unroll
            for (int b = 0; b < LB; ++b) {
                const int e = e0 + b * NT + threadIdx.x;
                const bool ok = e < NH;
                u[b] = ok ? fa0[e] : make_float2(0.f, 0.f);
                v[b] = ok ? fb0[e] : make_float2(0.f, 0.f);
                u2[b] = ok && two ? fa1[e] : make_float2(0.f, 0.f);
                v2[b] = ok && two ? fb1[e] : make_float2(0.f, 0.f);
            }
        };
        auto product = [&](int e0, const float2 (&u)[LB], const float2 (&v)[LB], const float2 (&u2)[LB],
                           const float2 (&v2)[LB]) {
#pragma unroll
            for (int b = 0; b < LB; ++b) {
                const int e = e0 + b * NT + threadIdx.x;
                if (e >= NH) break;
                const int kr = e / LH, kc = e % LH;
                const float2 z = make_float2(fmaf(u[b].x, v[b].x, u[b].y * v[b].y),
                                             fmaf(u[b].x, v[b].y, -(u[b].y * v[b].x)));
                const float2 z2 = make_float2(fmaf(u2[b].x, v2[b].x, u2[b].y * v2[b].y),
                                              fmaf(u2[b].x, v2[b].y, -(u2[b].y * v2[b].x)));
                a[kr * RS + kc] = make_float2(z.x - z2.y, z.y + z2.x);  // z + i z2
                if (kc > 0 && kc < L / 2)  // conj(z) + i conj(z2) at the mirrored frequency
                    a[((L - kr) % L) * RS + (L - kc)] = make_float2(z.x + z2.y, z2.x - z.y);
            }
        };
        float2 p0[LB], p1[LB], p2[LB], p3[LB];  // first round of the current two pairs
        int np = take(pi, pj);
        if (np) load(0, pi, pj, np, p0, p1, p2, p3);
        while (np) {
            product(0, p0, p1, p2, p3);
#pragma unroll 1
            for (int e0 = LB * NT; e0 < NH; e0 += LB * NT) {
                float2 u[LB], v[LB], u2[LB], v2[LB];
                load(e0, pi, pj, np, u, v, u2, v2);
                product(e0, u, v, u2, v2);
            }
            int ni[2], nj[2];
            const int nnp = take(ni, nj);
            if (nnp) load(0, ni, nj, nnp, p0, p1, p2, p3);
            __syncthreads();
            fft2d<L, N1, N2, NT>(a, tw);
            // one pass: peak per channel (largest value, smallest shift index on ties) and the
            // total energy (FP64).  Thread = one column position, every (NT / L)-th row.
            float best[2] = {-INFINITY, -INFINITY};
            int bidx[2] = {0x7fffffff, 0x7fffffff};
            double en[2] = {0.0, 0.0};
            {
                constexpr int RSTEP = NT / L;
                const int pc = threadIdx.x % L, kc = freq_of<N1, N2>(pc);
                for (int pr = threadIdx.x / L; pr < L; pr += RSTEP) {
                    const float2 v = a[pr * RS + pc];
                    const int k = freq_of<N1, N2>(pr) * L + kc;
                    if (v.x > best[0] || (v.x == best[0] && k < bidx[0])) {
                        best[0] = v.x;
                        bidx[0] = k;
                    }
                    if (v.y > best[1] || (v.y == best[1] && k < bidx[1])) {
                        best[1] = v.y;
                        bidx[1] = k;
                    }
                    en[0] = fma((double)v.x, (double)v.x, en[0]);
                    en[1] = fma((double)v.y, (double)v.y, en[1]);
                }
            }
#pragma unroll
            for (int ch = 0; ch < 2; ++ch) {
                for (int o = 32; o > 0; o >>= 1) {
                    const float ov = __shfl_xor(best[ch], o);
                    const int oi = __shfl_xor(bidx[ch], o);
                    if (ov > best[ch] || (ov == best[ch] && oi < bidx[ch])) {
                        best[ch] = ov;
                        bidx[ch] = oi;
                    }
                    en[ch] += __shfl_xor(en[ch], o);
                }
                if (lane == 0) {
                    s_val[ch][wave] = best[ch];
                    s_idx[ch][wave] = bidx[ch];
                    s_sum[ch][wave] = en[ch];
                }
            }
            __syncthreads();
            float pv[2];
            int pk[2];
#pragma unroll
            for (int ch = 0; ch < 2; ++ch) {
                pv[ch] = s_val[ch][0];
                pk[ch] = s_idx[ch][0];
                for (int ww = 1; ww < NW; ++ww)
                    if (s_val[ch][ww] > pv[ch] || (s_val[ch][ww] == pv[ch] && s_idx[ch][ww] < pk[ch])) {
                        pv[ch] = s_val[ch][ww];
                        pk[ch] = s_idx[ch][ww];
                    }
            }
            // energy inside the cyclic neighbourhood of each peak: one thread per shift of it
            {
                const int side = nb_side, cells = side * side;
                const int ch = threadIdx.x >= 256 ? 1 : 0, c = threadIdx.x & 255;
                double inside = 0.0;
                const int r0 = pk[ch] / L, c0 = pk[ch] % L;
                for (int cc = c; cc < cells; cc += 256) {
                    const int kr = (r0 + cc / side - h + L) % L, kc = (c0 + cc % side - h + L) % L;
                    const float2 v = a[pos_of<N1, N2>(kr) * RS + pos_of<N1, N2>(kc)];
                    const double x = (double)(ch ? v.y : v.x);
                    inside = fma(x, x, inside);
                }
                for (int o = 32; o > 0; o >>= 1) inside += __shfl_xor(inside, o);
                if (lane == 0) s_in[wave] = inside;
            }
            __syncthreads();
            if (threadIdx.x < np) {
                const int ch = threadIdx.x;
                double total = 0.0, inside = 0.0;
                for (int ww = 0; ww < NW; ++ww) total += s_sum[ch][ww];
                for (int ww = ch * (NW / 2); ww < (ch + 1) * (NW / 2); ++ww) inside += s_in[ww];
                // FP64 sums of FP32 squares: the difference keeps ~1e-16 of the total
                const double rest = total - inside;
                const double num = (double)pv[ch] * (double)pv[ch] * (double)(NV - nb_side * nb_side);
                const int i = pi[ch], j = pj[ch];
                const int64_t pidx = (int64_t)i * n - (int64_t)i * (i + 1) / 2 + (j - i - 1);
                // a zero-variance item has no correlation: its channel holds only the other
                // channel's rounding, so it is reported as NaN with peak 0
                const bool ok = live[i] && live[j] && rest > 0.0;
                out[pidx] = ok ? (float)(num / rest) : __builtin_nanf("");
                if (peak_out) peak_out[pidx] = ok ? (uint32_t)pk[ch] : 0u;
            }
            __syncthreads();  // LDS is refilled by the next pairs
            pi[0] = ni[0];
            pi[1] = ni[1];
            pj[0] = nj[0];
            pj[1] = nj[1];
            np = nnp;
        }
    }
}

template <int L>
struct PceShape;
template <>
struct PceShape<32> {
    static constexpr int N1 = 8, N2 = 4;
};
template <>
struct PceShape<64> {
    static constexpr int N1 = 8, N2 = 8;
};
template <>
struct PceShape<128> {
    static constexpr int N1 = 16, N2 = 8;
};

template <int L>
size_t pce_lds() { return (size_t)(L * (L + 1) + L) * sizeof(float2); }

template <int L>
const void *pce_kernel() { return (const void *)&k_pce<L, PceShape<L>::N1, PceShape<L>::N2>; }

int side_of(int64_t dim)
{
    for (int L : {32, 64, 128})
        if ((int64_t)L * L == dim) return L;
    return 0;
}

}  // namespace

rocket_status pce_prepare(rocket_ctx *ctx, const rocket_items *it, int64_t n, hipStream_t s)
{
    PceState &p = ctx->pce;
    p.valid = false;
    if (n > 0 && !it->dense) return fail(ctx, ROCKET_E_INVALID, "dense is NULL");
    if (it->ld < it->dim) return fail(ctx, ROCKET_E_INVALID, "ld < dim");
    if (n >= (1 << 30)) return fail(ctx, ROCKET_E_INVALID, "n too large");
    const int64_t wopt = ctx->opt[ROCKET_OPT_PCE_WIDTH];
    const int L = wopt ? (wopt * wopt == it->dim ? side_of(it->dim) : 0) : side_of(it->dim);
    p.n = n;
    p.L = L;
    p.big = false;
    if (!L) {
        // H x W with W = ROCKET_OPT_PCE_WIDTH (square if 0): the staged multi-pass path
        int64_t W = wopt;
        if (!W) {
            W = (int64_t)std::llround(std::sqrt((double)it->dim));
            if (W * W != it->dim) W = 0;
        }
        const int64_t H = W > 0 && it->dim % W == 0 ? it->dim / W : 0;
        if (!H || !pce_big_shape(H, W))
            return fail(ctx, ROCKET_E_UNSUPPORTED,
                        "PCE items must be L x L with L = 32, 64 or 128, or H x W (W = ROCKET_OPT_PCE_WIDTH, square "
                        "if 0) with H and W in [16, 4096]");
        p.big = true;
        p.H = (int)H;
        p.W = (int)W;
        RK_TRY(pce_big_prepare(ctx, it, n, p.H, p.W, s));
        p.valid = true;
        return ROCKET_OK;
    }
    void *spec = nullptr;
    const size_t spec_bytes = (size_t)std::max<int64_t>(n, 1) * L * (L / 2 + 1) * sizeof(float2);
    RK_TRY(ws_get(ctx, WS_PCE_SPEC, spec_bytes + sizeof(int) * (size_t)std::max<int64_t>(n, 1), &spec));
    int *live = (int *)((char *)spec + spec_bytes);  // per item: non-zero variance
    if (n > 0) {
        const size_t lds = L == 32 ? pce_lds<32>() : L == 64 ? pce_lds<64>() : pce_lds<128>();
        const void *kp = L == 32   ? (const void *)&k_pce_prepare<32, 8, 4>
                         : L == 64 ? (const void *)&k_pce_prepare<64, 8, 8>
                                   : (const void *)&k_pce_prepare<128, 16, 8>;
        RK_HIP(hipFuncSetAttribute(kp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        if (L == 32)
            hipLaunchKernelGGL((k_pce_prepare<32, 8, 4>), dim3((unsigned)n), dim3(PCE_THREADS), lds, s, it->dense,
                               it->ld, (float2 *)spec, live);
        else if (L == 64)
            hipLaunchKernelGGL((k_pce_prepare<64, 8, 8>), dim3((unsigned)n), dim3(PCE_THREADS), lds, s, it->dense,
                               it->ld, (float2 *)spec, live);
        else
            hipLaunchKernelGGL((k_pce_prepare<128, 16, 8>), dim3((unsigned)n), dim3(PCE_THREADS), lds, s, it->dense,
                               it->ld, (float2 *)spec, live);
        RK_HIP(hipGetLastError());
    }
    std::vector<int2> tiles;
    plan_leaves(n, PCE_T, tiles);
    p.tiles = (int64_t)tiles.size();
    if (p.tiles > 0) {
        plan_chunked(tiles, 1, MAX_SEG, ctx->h_items, ctx->h_seg, 1);
        const int64_t order = ctx->opt[ROCKET_OPT_QUEUE_ORDER];
        if (order == 1) shuffle_items(ctx->h_items, ctx->h_seg, (uint64_t)ctx->opt[ROCKET_OPT_SEED]);
        if (order == 2) single_segment(ctx->h_seg, (int64_t)ctx->h_items.size());
        RK_TRY(upload_queue(ctx, s, &p.qa));
        ctx->queue_owner = QOWN_PCE;
    }
    ctx->stats.tiles = p.tiles;
    ctx->stats.work_items = p.tiles;
    ctx->stats.tile = PCE_T;
    ctx->stats.kchunk = 0;
    ctx->stats.variant = L;
    p.valid = true;
    return ROCKET_OK;
}

rocket_status pce_compare(rocket_ctx *ctx, float *out, uint32_t *peak, hipStream_t s)
{
    PceState &p = ctx->pce;
    if (!p.valid) return fail(ctx, ROCKET_E_STATE, "PCE set not prepared");
    const int h = ctx->opt[ROCKET_OPT_PCE_RADIUS] ? (int)ctx->opt[ROCKET_OPT_PCE_RADIUS] : 5;
    if (2 * h + 1 > (p.big ? std::min(p.H, p.W) : p.L))  // h < min(H, W) / 2: the neighbourhood does not wrap
        return fail(ctx, ROCKET_E_INVALID, "PCE neighbourhood radius must be < min(H, W)/2");
    if (p.n < 2 || p.tiles == 0) return ROCKET_OK;
    if (p.big) return pce_big_compare(ctx, out, peak, h, s);
    if (ctx->queue_owner != QOWN_PCE) return fail(ctx, ROCKET_E_STATE, "queue was replanned by another prepare");
    const int L = p.L;
    const size_t lds = L == 32 ? pce_lds<32>() : L == 64 ? pce_lds<64>() : pce_lds<128>();
    const void *kp = L == 32 ? pce_kernel<32>() : L == 64 ? pce_kernel<64>() : pce_kernel<128>();
    RK_HIP(hipFuncSetAttribute(kp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int grid = auto_grid(ctx, kp, PCE_CMP_THREADS, lds, p.tiles);
    ctx->stats.grid = grid;
    RK_TRY(reset_queue(ctx, s, p.qa));
    const float2 *F = (const float2 *)ctx->ws[WS_PCE_SPEC].ptr;
    const int *live = (const int *)((const char *)F + (size_t)p.n * L * (L / 2 + 1) * sizeof(float2));
    RK_TRY(timing_begin(ctx, s));
    if (L == 32)
        hipLaunchKernelGGL((k_pce<32, 8, 4>), dim3(grid), dim3(PCE_CMP_THREADS), lds, s, F, live, (int)p.n, h, p.qa, out,
                           peak);
    else if (L == 64)
        hipLaunchKernelGGL((k_pce<64, 8, 8>), dim3(grid), dim3(PCE_CMP_THREADS), lds, s, F, live, (int)p.n, h, p.qa, out,
                           peak);
    else
        hipLaunchKernelGGL((k_pce<128, 16, 8>), dim3(grid), dim3(PCE_CMP_THREADS), lds, s, F, live, (int)p.n, h, p.qa, out,
                           peak);
    RK_HIP(hipGetLastError());
    RK_TRY(timing_end(ctx, s));
    return ROCKET_OK;
}

}  // namespace rk
