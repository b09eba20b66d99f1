// Gaussian-overlap registration cost between 2-D point clouds (Section V-C compare kernel)
// and its adjoint with respect to a rigid transform, on gfx950.
//
//   C_ij = sum_k sum_l w_kl,  w_kl = exp(-|y'_l - x_k|^2 / (4 sigma^2)),
//   x = points of cloud i, y = points of cloud j, y' = y (cost) or R(theta)(y - c_j) + c_j + t (adjoint).
//   dC/dt     = -(1/(2 sigma^2)) sum_kl w_kl (y'_l - x_k)
//   dC/dtheta = -(1/(2 sigma^2)) sum_l < sum_k w_kl (y'_l - x_k), J R(theta)(y_l - c_j) >
//
// The same kernel evaluates the two per-localisation-uncertainty scores of Section V-C, where
// point k carries its own standard deviation s_k (v = s_k^2 + t_l^2, D = |x_k - y_l|^2):
//   GMM L2 cross term   sum_kl exp(-D / (2 v)) / (2 pi v)
//   Bhattacharya        sum_kl (2 s_k t_l / v) exp(-D / (4 v))
// and their adjoint (isotropic points rotate onto themselves): d term / d y' = -(2 a / v) term u,
// a = 1/2 (L2) or 1/4 (Bhattacharya).
// Prepare stores s~ = s sqrt(2 ln 2) (L2) or s sqrt(4 ln 2) (Bhattacharya) per packed point,
// so that with r = 1 / (s~_k^2 + t~_l^2) a term is exp2(-D r) r (L2, times ln2/pi per pair) or
// exp2(-D r) s~_k r t~_l (Bhattacharya, times 2 per pair): one reciprocal and one exp2 per term.
//
// Clouds have uneven sizes.  Prepare sorts them by size (largest first) and packs them
// contiguously, so that a tile of T x T sorted clouds holds pairs of similar cost; tiles are
// queued largest estimated cost first (sum of N_a N_b) and dealt to per-XCD segments.  One
// persistent workgroup per CU stages the two cloud blocks of its tile in LDS and gives each
// pair to one wavefront: lanes own points of cloud j (S lanes x R registers per chunk, 64/S
// phases, each over a contiguous run of the points of cloud i), every lane keeps FP32 partial sums, and the wavefront
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
constexpr int GMM_MAX_BLOCK_PTS = 6800;   // with one f32 deviation per point (81.6 KB)
constexpr float GMM_SIG_MIN = 1e-18f, GMM_SIG_MAX = 1e18f;
constexpr int FULL_MAX_BLOCK_PTS = 3300;  // with a float4 shape per point (24 B): 158 KB for two blocks

// Cloud score modes (OvlState::mode): the fixed-sigma overlap, the two per-point-sigma
// scores, and the two scores for points with a full 2 x 2 covariance (or isotropic
// deviations packed as s^2 I), the latter with or without the rigid-transform adjoint.
constexpr int MODE_OVERLAP = OVL_OVERLAP, MODE_GMM_L2 = OVL_GMM_L2, MODE_GMM_BH = OVL_GMM_BH,
              MODE_FULL_L2 = OVL_FULL_L2, MODE_FULL_BH = OVL_FULL_BH;

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Gather sorted clouds into one packed array: cloud s of the sorted order owns packed
// points coff[s] .. coff[s+1]-1.
__global__ void k_ovl_zero(int *flag) { flag[threadIdx.x] = 0; }

// With per-point deviations (sig != nullptr) also pack s~ = s * sscale and raise *flag when a
// deviation lies outside [GMM_SIG_MIN, GMM_SIG_MAX] (or is NaN).
__global__ void k_ovl_pack(const float2 *__restrict__ xy, const int64_t *__restrict__ offsets,
                           const int *__restrict__ perm, const int *__restrict__ coff, float2 *__restrict__ packed, int n,
                           const float *__restrict__ sig, double sscale, float *__restrict__ psig, int *__restrict__ flag)
{
    for (int s = blockIdx.x; s < n; s += gridDim.x) {
        const int64_t src = offsets[perm[s]];
        const int dst = coff[s], cnt = coff[s + 1] - coff[s];
        for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
            packed[dst + k] = xy[src + k];
            if (sig) {
                const float v = sig[src + k];
                if (!(v >= GMM_SIG_MIN && v <= GMM_SIG_MAX)) *flag = 1;
                psig[dst + k] = (float)((double)v * sscale);
            }
        }
    }
}

// Shape of every packed point for the full-covariance scores: (c_xx, c_xy, c_yy, (det C)^(1/4))
// from cov (3 floats per point) or, when cov is NULL, from sig as s^2 I.  Raises *flag when a
// covariance is not symmetric positive definite with entries and determinant in
// [1e-36, 1e36] (so that sums, determinants and their reciprocal square roots stay finite
// and normal in FP32).
__global__ void k_ovl_pack_shape(const int64_t *__restrict__ offsets, const int *__restrict__ perm,
                                 const int *__restrict__ coff, int n, const float *__restrict__ cov,
                                 const float *__restrict__ sig, float4 *__restrict__ shape, int *__restrict__ flag)
{
    for (int s = blockIdx.x; s < n; s += gridDim.x) {
        const int64_t src = offsets[perm[s]];
        const int dst = coff[s], cnt = coff[s + 1] - coff[s];
        for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
            double a, b, c;
            if (cov) {
                a = cov[3 * (src + k)];
                b = cov[3 * (src + k) + 1];
                c = cov[3 * (src + k) + 2];
            } else {
                const double v = sig[src + k];
                a = c = v * v;
                b = 0.0;
            }
            const double det = a * c - b * b;
            if (!(a >= 1e-36 && a <= 1e36 && c >= 1e-36 && c <= 1e36 && det >= 1e-36 && det <= 1e36)) *flag = 1;
            shape[dst + k] = make_float4((float)a, (float)b, (float)c, (float)sqrt(sqrt(det > 0 ? det : 0.0)));
        }
    }
}

// MODE_OVERLAP: cexp = log2(e) / (4 sigma^2), cpost unused.  GMM modes: psig holds the packed
// scaled deviations, LDS holds them behind the points at float offset sig_at, cpost is the
// per-pair factor.
template <int MODE, bool GRAD, int S, int R>
__global__ __launch_bounds__(OVL_THREADS, 1) void k_overlap(const float2 *__restrict__ pts, const int *__restrict__ coff,
                                                            const int *__restrict__ perm, int n, int T, float cexp,
                                                            QueueArgs q, float *__restrict__ out,
                                                            const float *__restrict__ cen,
                                                            const float *__restrict__ params, float *__restrict__ grad,
                                                            float gscale, const float *__restrict__ psig, int sig_at,
                                                            float cpost)
{
    constexpr bool GMM = MODE != MODE_OVERLAP;
    constexpr int P = 64 / S;  // phases over the points of cloud i
    constexpr int CH = S * R;  // points of cloud j per chunk
    extern __shared__ float2 lds_pts[];
    float *lds_sig = reinterpret_cast<float *>(lds_pts) + sig_at;
    __shared__ int s_item;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int slot = lane % S, phase = lane / S;

    int prev = -1;
    for (;;) {
        const int it = queue_pop_wg(q, &s_item, prev);
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
        if constexpr (GMM) {
            for (int k = tid; k < nI; k += OVL_THREADS) lds_sig[k] = psig[pI0 + k];
            for (int k = tid; k < nJ; k += OVL_THREADS) lds_sig[nI + k] = psig[pJ0 + k];
        }
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
                float yx[R], yy[R], lx[R], ly[R], vx[R], vy[R], tt[R], tq[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int l = c0 + r * S + slot;
                    if (l < Nj) {
                        const float2 y = lds_pts[base_j + l];
                        if constexpr (GMM) {
                            tq[r] = lds_sig[base_j + l];
                            tt[r] = tq[r] * tq[r];
                        }
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
                        tt[r] = 1.f;
                        tq[r] = 0.f;
                    }
                }
                // this lane's phase covers a contiguous run of cloud i's points, four per step
                float sc[R][2], sx[R][2], sy[R][2];
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int e = 0; e < 2; ++e) sc[r][e] = sx[r][e] = sy[r][e] = 0.f;
                auto term = [&](const float2 x, const float s, int r, int e) {
                    float ux = yx[r] - x.x, uy = yy[r] - x.y;
                    if constexpr (GRAD) {
                        ux += lx[r];
                        uy += ly[r];
                    }
                    const float d2 = fmaf(uy, uy, ux * ux);
                    if constexpr (GMM) {
                        const float rv = __builtin_amdgcn_rcpf(fmaf(s, s, tt[r]));
                        const float wkl = __builtin_amdgcn_exp2f(-(d2 * rv));
                        const float f = wkl * (MODE == MODE_GMM_L2 ? rv : s * rv);
                        sc[r][e] += f;
                        if constexpr (GRAD) {
                            // d term / d y' = -2 ln2 rv u term (the scaled deviations fold in the
                            // 1/(2v) or 1/(4v) of the exponent); the constant is applied per pair
                            const float fr = f * rv;
                            sx[r][e] = fmaf(fr, ux, sx[r][e]);
                            sy[r][e] = fmaf(fr, uy, sy[r][e]);
                        }
                    } else {
                        const float wkl = __builtin_amdgcn_exp2f(-(d2 * cexp));
                        sc[r][e] += wkl;
                        if constexpr (GRAD) {
                            sx[r][e] = fmaf(wkl, ux, sx[r][e]);
                            sy[r][e] = fmaf(wkl, uy, sy[r][e]);
                        }
                    }
                };
                const int per = (Ni + P - 1) / P;
                const int k0 = min(Ni, phase * per), k1 = min(Ni, k0 + per);
                const float2 *xs = lds_pts + base_i;
                const float *ss = lds_sig + base_i;
                int k = k0;
                for (; k + 4 <= k1; k += 4) {
                    const float2 x0 = xs[k], x1 = xs[k + 1], x2 = xs[k + 2], x3 = xs[k + 3];
                    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
                    if constexpr (GMM) {
                        s0 = ss[k];
                        s1 = ss[k + 1];
                        s2 = ss[k + 2];
                        s3 = ss[k + 3];
                    }
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        term(x0, s0, r, 0);
                        term(x1, s1, r, 1);
                        term(x2, s2, r, 0);
                        term(x3, s3, r, 1);
                    }
                }
                for (; k < k1; ++k) {
                    const float2 x0 = xs[k];
                    const float s0 = GMM ? ss[k] : 0.f;
#pragma unroll
                    for (int r = 0; r < R; ++r) term(x0, s0, r, 0);
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    sc[r][0] += sc[r][1];
                    sx[r][0] += sx[r][1];
                    sy[r][0] += sy[r][1];
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float fl = MODE == MODE_GMM_BH ? tq[r] : 1.f;  // the point of cloud j's factor
                    accC = fmaf(sc[r][0], fl, accC);
                    if constexpr (GRAD) {
                        accX = fmaf(sx[r][0], fl, accX);
                        accY = fmaf(sy[r][0], fl, accY);
                        accT = fmaf(vx[r] * fl, sx[r][0], fmaf(vy[r] * fl, sy[r][0], accT));
                    }
                }
            }
            const float C = wave_sum(accC);
            if constexpr (GRAD) {
                const float GX = wave_sum(accX), GY = wave_sum(accY), GT = wave_sum(accT);
                if (lane == 0) {
                    out[pidx] = GMM ? C * cpost : C;
                    if (grad) {
                        grad[3 * pidx] = gscale * GT;
                        grad[3 * pidx + 1] = gscale * GX;
                        grad[3 * pidx + 2] = gscale * GY;
                    }
                }
            } else if constexpr (GMM) {
                if (lane == 0) out[pidx] = C * cpost;
            } else {
                if (lane == 0) out[pidx] = C;
            }
        }
        __syncthreads();  // LDS is restaged for the next tile
    }
}

// Full-covariance scores.  Point k of cloud i: x_k, S_k; point l of cloud j: y_l, T_l, moved
// (GRAD) to y'_l = R(y_l - c_j) + c_j + t with T'_l = R T_l R^T.  V = S_k + T'_l, d = y'_l - x_k:
//   L2 (BH = false): w = exp2(-log2(e)/2 d^T V^-1 d) / sqrt(det V)            (x 1/(2 pi) per pair)
//   BH (BH = true):  w = exp2(-log2(e)/4 d^T V^-1 d) rho_k rho_l / sqrt(det V) (x 2 per pair)
// with rho = (det S)^(1/4); one reciprocal square root, one reciprocal and one exp2 per term.  The adjoint
// (a = 1/2 or 1/4, u = V^-1 d, g_l = J R(y_l - c_j), W_l = J T'_l - T'_l J):
//   dC/dt     = -2a sum w u
//   dC/dtheta = sum w (-2a g^T u + a u^T W u - tr(V^-1 W) / 2)
// Each lane keeps, per point l of its own, the sums over k of w, w u, w u u^T and the two
// pieces w (v_xx - v_yy) / det V and w v_xy / det V of the trace term, and contracts them
// with g_l and W_l once the k loop ends.  Lanes own points of cloud j, loop over a
// contiguous run of cloud i's points, and the wavefront reduces with a fixed butterfly.
template <bool BH, bool GRAD>
__global__ __launch_bounds__(OVL_THREADS, 1) void k_gmm_full(const float2 *__restrict__ pts,
                                                             const float4 *__restrict__ shape,
                                                             const int *__restrict__ coff, const int *__restrict__ perm,
                                                             int n, int T, QueueArgs q, float *__restrict__ out,
                                                             const float *__restrict__ cen,
                                                             const float *__restrict__ params,
                                                             float *__restrict__ grad, int shape_at, float cpost)
{
    // lanes per chunk of cloud j, points of cloud j per lane (more for the cost, whose terms
    // need fewer registers, so each staged point of cloud i serves more independent terms)
    constexpr int S = 16, R = GRAD ? 2 : 4;
    constexpr int P = 64 / S, CH = S * R;
    constexpr float A = BH ? 0.25f : 0.5f;
    constexpr float AL2E = A * 1.4426950408889634f;  // a log2(e)
    extern __shared__ float2 lds_pts[];
    float4 *lds_shape = reinterpret_cast<float4 *>(reinterpret_cast<float *>(lds_pts) + shape_at);
    __shared__ int s_item;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int slot = lane % S, phase = lane / S;

    int prev = -1;
    for (;;) {
        const int it = queue_pop_wg(q, &s_item, prev);
        if (it < 0) break;
        const int4 w = q.items[it];
        const int bI = w.x, bJ = w.y;
        const int a0 = bI * T, a1 = min(n, a0 + T), b0 = bJ * T, b1 = min(n, b0 + T);
        const bool diag = bI == bJ;
        const int pI0 = coff[a0], pI1 = coff[a1];
        const int pJ0 = coff[b0], pJ1 = coff[b1];
        const int nI = pI1 - pI0, nJ = diag ? 0 : pJ1 - pJ0;
        for (int k = tid; k < nI; k += OVL_THREADS) {
            lds_pts[k] = pts[pI0 + k];
            lds_shape[k] = shape[pI0 + k];
        }
        for (int k = tid; k < nJ; k += OVL_THREADS) {
            lds_pts[nI + k] = pts[pJ0 + k];
            lds_shape[nI + k] = shape[pJ0 + k];
        }
        __syncthreads();

        const int na = a1 - a0, nb = b1 - b0;
        for (int p = wave; p < na * nb; p += OVL_WAVES) {
            const int a = a0 + p / nb, b = b0 + p % nb;
            if (a >= b) continue;
            const int ia = perm[a], ib = perm[b];
            const int oi = min(ia, ib), oj = max(ia, ib);
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
                // this lane's points of cloud j: moved point (hi + lo), moved covariance, rho
                float yx[R], yy[R], lx[R], ly[R], r00[R], r01[R], r11[R], rl[R], gx_[R], gy_[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int l = c0 + r * S + slot;
                    if (l < Nj) {
                        const float2 y = lds_pts[base_j + l];
                        const float4 tq = lds_shape[base_j + l];
                        rl[r] = BH ? tq.w : 1.f;  // this point's factor on its sums
                        if constexpr (GRAD) {
                            const double rx = (double)y.x - cx, ry = (double)y.y - cy;
                            const double ox = dct * rx - dst * ry, oy = dst * rx + dct * ry;
                            const double px = ox + cx + tx, py = oy + cy + ty;
                            yx[r] = (float)px;
                            yy[r] = (float)py;
                            lx[r] = (float)(px - (double)yx[r]);
                            ly[r] = (float)(py - (double)yy[r]);
                            gx_[r] = (float)(-oy);
                            gy_[r] = (float)ox;
                            // T' = R T R^T in FP64, rounded once
                            const double m00 = dct * tq.x - dst * tq.y, m01 = dct * tq.y - dst * tq.z;
                            const double m10 = dst * tq.x + dct * tq.y, m11 = dst * tq.y + dct * tq.z;
                            r00[r] = (float)(m00 * dct - m01 * dst);
                            r01[r] = (float)(m00 * dst + m01 * dct);
                            r11[r] = (float)(m10 * dst + m11 * dct);
                        } else {
                            yx[r] = y.x;
                            yy[r] = y.y;
                            lx[r] = ly[r] = 0.f;
                            gx_[r] = gy_[r] = 0.f;
                            r00[r] = tq.x;
                            r01[r] = tq.y;
                            r11[r] = tq.z;
                        }
                    } else {
                        // no point: finite placeholder values, and a factor of 0 on its sums
                        yx[r] = yy[r] = 0.f;
                        lx[r] = ly[r] = 0.f;
                        gx_[r] = gy_[r] = 0.f;
                        r00[r] = r11[r] = 1.f;
                        r01[r] = 0.f;
                        rl[r] = 0.f;
                    }
                }
                float sc[R], sx[R], sy[R], sxx[R], syy[R], sxy[R], t1[R], t2[R];
#pragma unroll
                for (int r = 0; r < R; ++r) sc[r] = sx[r] = sy[r] = sxx[r] = syy[r] = sxy[r] = t1[r] = t2[r] = 0.f;
                const int per = (Ni + P - 1) / P;
                const int k0 = min(Ni, phase * per), k1 = min(Ni, k0 + per);
                const float2 *xs = lds_pts + base_i;
                const float4 *ss = lds_shape + base_i;
                // cost: two points of cloud i per step, both LDS reads issued before any term
                auto term = [&](const float2 x, const float4 sk) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const float v00 = sk.x + r00[r], v01 = sk.y + r01[r], v11 = sk.z + r11[r];
                        const float det = fmaf(v00, v11, -(v01 * v01));
                        const float rs = __builtin_amdgcn_rsqf(det);
                        const float idet = __builtin_amdgcn_rcpf(det);  // 1 ulp, not rs^2's ~3
                        const float dx = (yx[r] - x.x) + lx[r], dy = (yy[r] - x.y) + ly[r];
                        const float hx = fmaf(v11, dx, -(v01 * dy)), hy = fmaf(v00, dy, -(v01 * dx));  // adj(V) d
                        const float qf = fmaf(hx, dx, hy * dy) * idet;                              // d^T V^-1 d
                        float wt = __builtin_amdgcn_exp2f(-(qf * AL2E)) * rs;
                        if constexpr (BH) wt *= sk.w;
                        sc[r] += wt;
                        if constexpr (GRAD) {
                            const float ux = hx * idet, uy = hy * idet;
                            const float fu = wt * ux, fv = wt * uy;
                            sx[r] += fu;
                            sy[r] += fv;
                            sxx[r] = fmaf(fu, ux, sxx[r]);
                            syy[r] = fmaf(fv, uy, syy[r]);
                            sxy[r] = fmaf(fu, uy, sxy[r]);
                            const float wi = wt * idet;
                            t1[r] = fmaf(wi, v00 - v11, t1[r]);
                            t2[r] = fmaf(wi, v01, t2[r]);
                        }
                    }
                };
                int k = k0;
                if constexpr (!GRAD) {
                    for (; k + 2 <= k1; k += 2) {
                        const float2 x0 = xs[k], x1 = xs[k + 1];
                        const float4 s0 = ss[k], s1 = ss[k + 1];
                        term(x0, s0);
                        term(x1, s1);
                    }
                }
                for (; k < k1; ++k) term(xs[k], ss[k]);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float f = rl[r];
                    accC = fmaf(sc[r], f, accC);
                    if constexpr (GRAD) {
                        accX = fmaf(sx[r], f, accX);
                        accY = fmaf(sy[r], f, accY);
                        // u^T W u = -2 T'01 (u_x^2 - u_y^2) + 2 (T'00 - T'11) u_x u_y;
                        // tr(V^-1 W) = (2 T'01 (v00 - v11) - 2 (T'00 - T'11) v01) / det V
                        const float uwu = fmaf(-2.f * r01[r], sxx[r] - syy[r], 2.f * (r00[r] - r11[r]) * sxy[r]);
                        const float tr = fmaf(2.f * r01[r], t1[r], -2.f * (r00[r] - r11[r]) * t2[r]);
                        const float gu = fmaf(gx_[r], sx[r], gy_[r] * sy[r]);
                        const float th = fmaf(-2.f * A, gu, fmaf(A, uwu, -0.5f * tr));
                        accT = fmaf(th, f, accT);
                    }
                }
            }
            const float C = wave_sum(accC);
            if constexpr (GRAD) {
                const float GX = wave_sum(accX), GY = wave_sum(accY), GT = wave_sum(accT);
                if (lane == 0) {
                    out[pidx] = C * cpost;
                    if (grad) {
                        grad[3 * pidx] = GT * cpost;
                        grad[3 * pidx + 1] = (-2.f * A) * GX * cpost;
                        grad[3 * pidx + 2] = (-2.f * A) * GY * cpost;
                    }
                }
            } else {
                if (lane == 0) out[pidx] = C * cpost;
            }
        }
        __syncthreads();  // LDS is restaged for the next tile
    }
}

template <int MODE, bool GRAD>
const void *ovl_kernel_m(int variant)
{
    switch (variant) {
    case 1: return (const void *)&k_overlap<MODE, GRAD, 64, 1>;
    case 2: return (const void *)&k_overlap<MODE, GRAD, 32, 2>;
    case 4: return (const void *)&k_overlap<MODE, GRAD, 16, 4>;
    default: return (const void *)&k_overlap<MODE, GRAD, 16, 2>;
    }
}

const void *ovl_kernel(int mode, bool grad, int variant)
{
    if (mode == MODE_FULL_L2) return grad ? (const void *)&k_gmm_full<false, true> : (const void *)&k_gmm_full<false, false>;
    if (mode == MODE_FULL_BH) return grad ? (const void *)&k_gmm_full<true, true> : (const void *)&k_gmm_full<true, false>;
    switch (mode) {
    case MODE_GMM_L2: return grad ? ovl_kernel_m<MODE_GMM_L2, true>(variant) : ovl_kernel_m<MODE_GMM_L2, false>(variant);
    case MODE_GMM_BH: return grad ? ovl_kernel_m<MODE_GMM_BH, true>(variant) : ovl_kernel_m<MODE_GMM_BH, false>(variant);
    default: return grad ? ovl_kernel_m<MODE_OVERLAP, true>(variant) : ovl_kernel_m<MODE_OVERLAP, false>(variant);
    }
}

struct OvlLaunch {
    const float2 *pts;
    const int *coff, *perm;
    int n, T;
    float cexp;
    QueueArgs qa;
    float *out;
    const float *cen, *params;
    float *grad;
    float gscale;
    const float *psig;
    int sig_at;
    float cpost;
};

template <int MODE, bool GRAD, int S, int R>
void launch_one(int grid, size_t lds, hipStream_t s, const OvlLaunch &a)
{
    hipLaunchKernelGGL((k_overlap<MODE, GRAD, S, R>), dim3(grid), dim3(OVL_THREADS), lds, s, a.pts, a.coff, a.perm,
                       a.n, a.T, a.cexp, a.qa, a.out, a.cen, a.params, a.grad, a.gscale, a.psig, a.sig_at, a.cpost);
}

template <int MODE, bool GRAD>
void launch_m(int variant, int grid, size_t lds, hipStream_t s, const OvlLaunch &a)
{
    switch (variant) {
    case 1: launch_one<MODE, GRAD, 64, 1>(grid, lds, s, a); break;
    case 2: launch_one<MODE, GRAD, 32, 2>(grid, lds, s, a); break;
    case 4: launch_one<MODE, GRAD, 16, 4>(grid, lds, s, a); break;
    default: launch_one<MODE, GRAD, 16, 2>(grid, lds, s, a); break;
    }
}

template <bool BH, bool GRAD>
void launch_full(int grid, size_t lds, hipStream_t s, const OvlLaunch &a)
{
    hipLaunchKernelGGL((k_gmm_full<BH, GRAD>), dim3(grid), dim3(OVL_THREADS), lds, s, a.pts, (const float4 *)a.psig,
                       a.coff, a.perm, a.n, a.T, a.qa, a.out, a.cen, a.params, a.grad, a.sig_at, a.cpost);
}

void launch_ovl(int mode, bool grad, int variant, int grid, size_t lds, hipStream_t s, const OvlLaunch &a)
{
    if (mode == MODE_FULL_L2) return grad ? launch_full<false, true>(grid, lds, s, a) : launch_full<false, false>(grid, lds, s, a);
    if (mode == MODE_FULL_BH) return grad ? launch_full<true, true>(grid, lds, s, a) : launch_full<true, false>(grid, lds, s, a);
    switch (mode) {
    case MODE_GMM_L2:
        grad ? launch_m<MODE_GMM_L2, true>(variant, grid, lds, s, a) : launch_m<MODE_GMM_L2, false>(variant, grid, lds, s, a);
        break;
    case MODE_GMM_BH:
        grad ? launch_m<MODE_GMM_BH, true>(variant, grid, lds, s, a) : launch_m<MODE_GMM_BH, false>(variant, grid, lds, s, a);
        break;
    default:
        grad ? launch_m<MODE_OVERLAP, true>(variant, grid, lds, s, a) : launch_m<MODE_OVERLAP, false>(variant, grid, lds, s, a);
        break;
    }
}

struct OvlDev {
    float2 *pts;
    float *sig;
    int *coff, *perm;
};

OvlDev dev_ptrs(rocket_ctx *ctx, int64_t n)
{
    OvlDev d;
    d.pts = (float2 *)ctx->ws[WS_OVL_PACK].ptr;
    d.sig = (float *)ctx->ws[WS_OVL_SIG].ptr;
    d.coff = (int *)ctx->ws[WS_OVL_META].ptr;
    d.perm = d.coff + ((n + 1 + 63) / 64) * 64;
    return d;
}

bool full_mode(int mode) { return mode == MODE_FULL_L2 || mode == MODE_FULL_BH; }

int max_block_pts(int mode)
{
    return mode == MODE_OVERLAP ? OVL_MAX_BLOCK_PTS : full_mode(mode) ? FULL_MAX_BLOCK_PTS : GMM_MAX_BLOCK_PTS;
}

// Two staged blocks of points, then (per-point-sigma and full-covariance scores) their
// deviations or shapes in the same order.
size_t ovl_lds_bytes(int mode, int64_t mx)
{
    const size_t per = sizeof(float2) + (mode == MODE_OVERLAP ? 0 : full_mode(mode) ? sizeof(float4) : sizeof(float));
    return (size_t)2 * mx * per + 16;
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

// Default 8 clouds per block: the two staged blocks then take ~51 KB of LDS (~77 KB with
// per-point deviations), so two or three workgroups share a CU and hide each other's LDS and
// queue latency (measured ~25 % faster than 16 on 2048 clouds of 50..400 points).  With a
// full covariance per point (24 bytes) 4 clouds per block (measured on the same clouds: cost
// 64 / 79 / 74 ms and adjoint 97 / 116 / 104 ms at 4 / 3 / 8 clouds per block).
static int ovl_block(rocket_ctx *ctx)
{
    if (ctx->opt[ROCKET_OPT_OVL_BLOCK]) return (int)ctx->opt[ROCKET_OPT_OVL_BLOCK];
    return ctx->ovl.mode == MODE_FULL_L2 || ctx->ovl.mode == MODE_FULL_BH ? 4 : 8;
}
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
        if (mx <= max_block_pts(o.mode) || T == 1) break;
        T = std::max(1, T / 2);
    }
    if (mx > max_block_pts(o.mode)) return fail(ctx, ROCKET_E_UNSUPPORTED, "a single cloud exceeds the LDS capacity");
    o.block = T;
    o.max_block_pts = mx;
    o.tiles = (int64_t)ctx->h_items.size();
    if (o.tiles > 0) RK_TRY(upload_queue(ctx, s, &o.qa));
    ctx->queue_owner = QOWN_OVL;
    o.pc_block = ovl_block(ctx);
    o.pc_order = ctx->opt[ROCKET_OPT_QUEUE_ORDER];
    o.pc_seed = ctx->opt[ROCKET_OPT_SEED];
    o.pc_ledger = queue_flags(ctx);
    return ROCKET_OK;
}

rocket_status ovl_prepare(rocket_ctx *ctx, const rocket_items *it, int64_t n, int mode, hipStream_t s)
{
    OvlState &o = ctx->ovl;
    o.valid = false;
    o.grad_ready = false;
    if (n > 0 && (!it->offsets || !it->xy)) return fail(ctx, ROCKET_E_INVALID, "offsets or xy is NULL");
    if (mode == MODE_OVERLAP && (!(it->sigma > 0.0) || !std::isfinite(it->sigma)))
        return fail(ctx, ROCKET_E_INVALID, "sigma must be > 0");
    if (mode != MODE_OVERLAP && n > 0 && !it->point_sigma && !(full_mode(mode) && it->point_cov))
        return fail(ctx, ROCKET_E_INVALID, "point_sigma is NULL");
    o.mode = mode;
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
    void *mp = nullptr, *pp = nullptr, *sp = nullptr, *fp = nullptr;
    RK_TRY(ws_get(ctx, WS_OVL_META, sizeof(int) * meta.size(), &mp));
    RK_TRY(ws_get(ctx, WS_OVL_PACK, sizeof(float2) * (size_t)std::max<int64_t>(o.total, 1), &pp));
    const bool gmm = mode != MODE_OVERLAP, full = full_mode(mode);
    if (gmm) {
        RK_TRY(ws_get(ctx, WS_OVL_SIG, (full ? sizeof(float4) : sizeof(float)) * (size_t)std::max<int64_t>(o.total, 1),
                      &sp));
        RK_TRY(ws_get(ctx, WS_FLAGS, 256, &fp));
        hipLaunchKernelGGL(k_ovl_zero, dim3(1), dim3(64), 0, s, (int *)fp);
        RK_HIP(hipGetLastError());
    }
    RK_HIP(hipMemcpyAsync(mp, meta.data(), sizeof(int) * meta.size(), hipMemcpyHostToDevice, s));
    if (n > 0) {
        const OvlDev d = dev_ptrs(ctx, n);
        const unsigned pg = (unsigned)std::min<int64_t>(n, 65535);
        // s~^2 = 2 ln2 s^2 (L2) or 4 ln2 s^2 (Bhattacharya): see the kernel's header comment
        const double sscale = std::sqrt((mode == MODE_GMM_L2 ? 2.0 : 4.0) * 0.69314718055994530942);
        const bool psig = gmm && !full;
        hipLaunchKernelGGL(k_ovl_pack, dim3(pg), dim3(256), 0, s, (const float2 *)it->xy, it->offsets, d.perm, d.coff,
                           d.pts, (int)n, psig ? it->point_sigma : nullptr, sscale, psig ? d.sig : nullptr, (int *)fp);
        RK_HIP(hipGetLastError());
        if (full) {
            hipLaunchKernelGGL(k_ovl_pack_shape, dim3(pg), dim3(256), 0, s, it->offsets, (const int *)d.perm,
                               (const int *)d.coff, (int)n, it->point_cov, it->point_cov ? nullptr : it->point_sigma,
                               (float4 *)d.sig, (int *)fp);
            RK_HIP(hipGetLastError());
        }
    }
    int flag = 0;
    if (gmm) RK_HIP(hipMemcpyAsync(&flag, fp, sizeof(int), hipMemcpyDeviceToHost, s));
    RK_HIP(hipStreamSynchronize(s));  // meta staging vector goes out of scope
    if (flag && full)
        return fail(ctx, ROCKET_E_INVALID, "a point covariance is not positive definite within [1e-36, 1e36]");
    if (flag) return fail(ctx, ROCKET_E_INVALID, "point_sigma outside [1e-18, 1e18]");
    RK_TRY(ovl_replan(ctx, s));
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
    const size_t lds = ovl_lds_bytes(o.mode, o.max_block_pts);
    const bool g = params != nullptr;
    const void *kern = ovl_kernel(o.mode, g, variant);
    const int grid = auto_grid(ctx, kern, OVL_THREADS, lds, o.tiles);
    ctx->stats.grid = grid;
    ctx->stats.variant = variant;
    RK_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    RK_TRY(reset_queue(ctx, s, o.qa));
    OvlLaunch a;
    a.pts = d.pts;
    a.coff = d.coff;
    a.perm = d.perm;
    a.n = (int)o.n;
    a.T = o.block;
    a.cexp = o.mode == MODE_OVERLAP ? (float)(1.4426950408889634 / (4.0 * o.sigma * o.sigma)) : 0.f;
    a.qa = o.qa;
    a.out = out;
    a.cen = g ? cen : nullptr;
    a.params = g ? params : nullptr;
    a.grad = g ? grad : nullptr;
    a.gscale = o.mode == MODE_OVERLAP ? (float)(-1.0 / (2.0 * o.sigma * o.sigma)) : 0.f;  // per-point sigma: below
    a.psig = o.mode == MODE_OVERLAP ? nullptr : d.sig;
    a.sig_at = (int)(2 * 2 * o.max_block_pts);  // floats: behind 2 blocks of float2 points
    // per-pair factor: ln2 / pi (per-point-sigma L2), 1 / (2 pi) (full-covariance L2), 2 (Bhattacharya)
    a.cpost = o.mode == MODE_GMM_L2    ? (float)(0.69314718055994530942 / 3.14159265358979323846)
              : o.mode == MODE_FULL_L2 ? (float)(1.0 / (2.0 * 3.14159265358979323846))
              : (o.mode == MODE_GMM_BH || o.mode == MODE_FULL_BH) ? 2.f
                                                                   : 1.f;
    if (o.mode == MODE_GMM_L2 || o.mode == MODE_GMM_BH) a.gscale = (float)(-2.0 * 0.69314718055994530942) * a.cpost;
    RK_TRY(timing_begin(ctx, s));
    launch_ovl(o.mode, g, variant, grid, lds, s, a);
    RK_HIP(hipGetLastError());
    RK_TRY(timing_end(ctx, s));
    return ROCKET_OK;
}

rocket_status ovl_replan_public(rocket_ctx *ctx, hipStream_t s)
{
    RK_TRY(ovl_replan(ctx, s));
    ctx->stats.tiles = ctx->ovl.tiles;
    ctx->stats.work_items = ctx->ovl.tiles;
    ctx->stats.tile = ctx->ovl.block;
    ctx->stats.variant = ovl_variant(ctx);
    return ROCKET_OK;
}

rocket_status ovl_compare(rocket_ctx *ctx, float *out, const float *cen, const float *params, float *grad,
                          hipStream_t s)
{
    OvlState &o = ctx->ovl;
    if (!o.valid) return fail(ctx, ROCKET_E_STATE, "overlap set not prepared");
    if (o.n < 2 || o.tiles == 0) return ROCKET_OK;
    if (ctx->queue_owner != QOWN_OVL || o.pc_block != ovl_block(ctx) || o.pc_order != ctx->opt[ROCKET_OPT_QUEUE_ORDER] ||
        o.pc_seed != ctx->opt[ROCKET_OPT_SEED] || o.pc_ledger != queue_flags(ctx))
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
    const int blocks[] = {4, 8, 16};
    float best = 1e30f;
    int best_b = 8, best_v = 3;
    rocket_status st = ROCKET_OK;
    for (int b : blocks) {
        ctx->opt[ROCKET_OPT_OVL_BLOCK] = b;
        if ((st = ovl_replan(ctx, s)) != ROCKET_OK) break;
        if (o.block != b) continue;  // block did not fit in LDS
        for (int v = 1; v <= 4; ++v) {
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
