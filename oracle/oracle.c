/*
 * FP64 reference ("oracle") for the all-pairs hot path.  TEST INFRASTRUCTURE ONLY:
 * it exists to check the GPU library, shares no code with it, and only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may call it.
 *
 * The all-pairs problem computes f(l(i), l(j)) for every 1 <= i < j <= n
 * (Section III).  The paper treats each application's compare kernel as a black
 * box (Section V), so each function below is the plain textbook definition of the
 * pair function the application names, evaluated in double precision over the
 * exact f32/int64 values the GPU consumes, one pair at a time:
 *
 *   ncc      Section V-A: normalised cross-correlation of two noise patterns,
 *            read as zero-lag Pearson correlation.
 *   overlap  Section V-C: the transform-dependent cross term of the L2 distance
 *            between two Gaussian mixtures, sum_k sum_l exp(-|x_k-y_l|^2/(4 s^2)).
 *   grad     Section V-C: the registration optimiser's gradient of that term with
 *            respect to a rigid transform (theta, tx, ty) of the second cloud,
 *            rotating about its centroid.
 *   sparse   Section V-B: cosine similarity of two sparse composition vectors,
 *            with the exact size of the key intersection.
 *
 * Pairs are passed as explicit lists (pi[p], pj[p]); the packed upper-triangle
 * index of (i,j), i<j, is i*n - i*(i+1)/2 + (j-i-1).  Loops over pairs are
 * OpenMP-parallel; within a pair everything is a plain sequential FP64 loop.
 * Built with gcc -O2 and no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

int64_t oracle_packed_index(int64_t i, int64_t j, int64_t n)
{
    /* rows 0..i-1 of the strict upper triangle hold (n-1) + (n-2) + ... + (n-i) pairs */
    int64_t before = 0;
    for (int64_t r = 0; r < i; ++r) before += n - 1 - r;
    return before + (j - i - 1);
}

/* ---------------------------------------------------------------------------------------
 * NCC: rho_ij = sum_k (a_k - mu_a)(b_k - mu_b) / sqrt(sum_k (a_k-mu_a)^2 * sum_k (b_k-mu_b)^2)
 * ------------------------------------------------------------------------------------- */

/* Per-item mean and sum of squared deviations (two passes, FP64). */
void oracle_ncc_stats(const float *X, int64_t n, int64_t d, int64_t ld, double *mu, double *ss)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        const float *a = X + i * ld;
        double s = 0.0;
        for (int64_t k = 0; k < d; ++k) s += (double)a[k];
        double m = s / (double)d;
        double q = 0.0;
        for (int64_t k = 0; k < d; ++k) {
            double c = (double)a[k] - m;
            q += c * c;
        }
        mu[i] = m;
        ss[i] = q;
    }
}

/* rho for each listed pair, plus the error scale tau = sqrt(sum_k ahat_k^2 bhat_k^2) of
 * the dot product of the two centred, unit-norm vectors.  A zero-variance item gives NaN. */
void oracle_ncc_pairs(const float *X, int64_t d, int64_t ld, const double *mu, const double *ss,
                      const int64_t *pi, const int64_t *pj, int64_t np, double *rho, double *tau)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < np; ++p) {
        const int64_t i = pi[p], j = pj[p];
        const float *a = X + i * ld;
        const float *b = X + j * ld;
        const double ma = mu[i], mb = mu[j];
        const double na = sqrt(ss[i]), nb = sqrt(ss[j]);
        double cross = 0.0, t2 = 0.0;
        for (int64_t k = 0; k < d; ++k) {
            double ca = (double)a[k] - ma;
            double cb = (double)b[k] - mb;
            cross += ca * cb;
            double ha = ca / na, hb = cb / nb;
            t2 += ha * ha * hb * hb;
        }
        if (ss[i] > 0.0 && ss[j] > 0.0) {
            rho[p] = cross / sqrt(ss[i] * ss[j]);
            if (tau) tau[p] = sqrt(t2);
        } else {
            rho[p] = NAN;
            if (tau) tau[p] = NAN;
        }
    }
}

/* ---------------------------------------------------------------------------------------
 * Gaussian overlap: C_ij = sum_k sum_l exp(-|x_k - y_l|^2 / (4 sigma^2)),
 * x = points of cloud i, y = points of cloud j (interleaved f32 xy, offsets per cloud).
 * kappa_ij = sum |e_kl| w_kl / sum w_kl is the cost-weighted mean |exponent|; it sets
 * how much FP32 rounding of the exponent a GPU result may legitimately carry.
 * ------------------------------------------------------------------------------------- */
void oracle_overlap_pairs(const float *xy, const int64_t *off, double sigma, const int64_t *pi,
                          const int64_t *pj, int64_t np, double *cost, double *kappa)
{
    const double inv4s2 = 1.0 / (4.0 * sigma * sigma);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < np; ++p) {
        const int64_t i = pi[p], j = pj[p];
        double c = 0.0, ce = 0.0;
        for (int64_t k = off[i]; k < off[i + 1]; ++k) {
            const double xk = xy[2 * k], yk = xy[2 * k + 1];
            for (int64_t l = off[j]; l < off[j + 1]; ++l) {
                const double dx = xk - (double)xy[2 * l];
                const double dy = yk - (double)xy[2 * l + 1];
                const double e = (dx * dx + dy * dy) * inv4s2;
                const double w = exp(-e);
                c += w;
                ce += e * w;
            }
        }
        cost[p] = c;
        if (kappa) kappa[p] = c > 0.0 ? ce / c : 0.0;
    }
}

/* ---------------------------------------------------------------------------------------
 * Gaussian mixtures with a per-localisation uncertainty (Section V-C names the GMM L2
 * distance and the Bhattacharya distance as the two particle scores).  Point k of cloud i
 * is the isotropic component N(x_k, s_k^2 I), point l of cloud j is N(y_l, t_l^2 I);
 * v = s_k^2 + t_l^2, D = |x_k - y_l|^2.
 *   mode 0 (L2 cross term):  sum_kl  integral N(z; x_k, s_k^2) N(z; y_l, t_l^2) dz
 *                          = sum_kl  exp(-D / (2 v)) / (2 pi v)
 *   mode 1 (Bhattacharya):   sum_kl  integral sqrt(N(z; x_k, s_k^2) N(z; y_l, t_l^2)) dz
 *                          = sum_kl  (2 s_k t_l / v) exp(-D / (4 v))
 * ------------------------------------------------------------------------------------- */
void oracle_gmm_pairs(const float *xy, const float *sig, const int64_t *off, int mode, const int64_t *pi,
                      const int64_t *pj, int64_t np, double *cost, double *kappa)
{
    const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < np; ++p) {
        const int64_t i = pi[p], j = pj[p];
        double c = 0.0, ce = 0.0;
        for (int64_t k = off[i]; k < off[i + 1]; ++k) {
            const double xk = xy[2 * k], yk = xy[2 * k + 1], sk = sig[k];
            for (int64_t l = off[j]; l < off[j + 1]; ++l) {
                const double dx = xk - (double)xy[2 * l];
                const double dy = yk - (double)xy[2 * l + 1];
                const double tl = sig[l];
                const double v = sk * sk + tl * tl;
                const double D = dx * dx + dy * dy;
                double e, w;
                if (mode == 0) {
                    e = D / (2.0 * v);
                    w = exp(-e) / (two_pi * v);
                } else {
                    e = D / (4.0 * v);
                    w = (2.0 * sk * tl / v) * exp(-e);
                }
                c += w;
                ce += e * w;
            }
        }
        cost[p] = c;
        /* cost-weighted mean exponent, as for the plain overlap */
        if (kappa) kappa[p] = c > 0.0 ? ce / c : 0.0;
    }
}

/* ---------------------------------------------------------------------------------------
 * Registration gradient.  For pair p = (i, j) and transform q = (theta, tx, ty):
 *   y'_l = R(theta) (y_l - c_j) + c_j + t,   u_kl = y'_l - x_k,
 *   w_kl = exp(-|u_kl|^2 / (4 sigma^2)),     C = sum w_kl,
 *   dC/dt     = -(1/(2 sigma^2)) sum w_kl u_kl
 *   dC/dtheta = -(1/(2 sigma^2)) sum w_kl <u_kl, dR/dtheta (y_l - c_j)>
 * (dR/dtheta (y - c) = J R(theta)(y - c) with J the 90-degree rotation.)
 * tau[p][m] = sqrt(sum_kl (d term_kl / d q_m)^2) * max(1, kappa/50) is the error floor
 * for a signed sum of that many FP32 terms.  Params are double so finite differences
 * can step them exactly.
 * ------------------------------------------------------------------------------------- */
void oracle_overlap_grad_pairs(const float *xy, const int64_t *off, const float *cen, double sigma,
                               const int64_t *pi, const int64_t *pj, const double *params, int64_t np,
                               double *cost, double *grad, double *tau, double *kappa)
{
    const double inv4s2 = 1.0 / (4.0 * sigma * sigma);
    const double g = 2.0 * inv4s2; /* 1/(2 sigma^2) */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < np; ++p) {
        const int64_t i = pi[p], j = pj[p];
        const double th = params[3 * p], tx = params[3 * p + 1], ty = params[3 * p + 2];
        const double ct = cos(th), st = sin(th);
        const double cx = cen[2 * j], cy = cen[2 * j + 1];
        double c = 0.0, ce = 0.0, gth = 0.0, gx = 0.0, gy = 0.0;
        double q0 = 0.0, q1 = 0.0, q2 = 0.0;
        for (int64_t l = off[j]; l < off[j + 1]; ++l) {
            const double rx = (double)xy[2 * l] - cx, ry = (double)xy[2 * l + 1] - cy;
            const double ox = ct * rx - st * ry, oy = st * rx + ct * ry; /* R (y - c) */
            const double vx = -oy, vy = ox;                              /* dR/dtheta (y - c) */
            const double yx = ox + cx + tx, yy = oy + cy + ty;
            for (int64_t k = off[i]; k < off[i + 1]; ++k) {
                const double ux = yx - (double)xy[2 * k];
                const double uy = yy - (double)xy[2 * k + 1];
                const double e = (ux * ux + uy * uy) * inv4s2;
                const double w = exp(-e);
                const double dth = -g * w * (ux * vx + uy * vy);
                const double dx = -g * w * ux, dy = -g * w * uy;
                c += w;
                ce += e * w;
                gth += dth;
                gx += dx;
                gy += dy;
                q0 += dth * dth;
                q1 += dx * dx;
                q2 += dy * dy;
            }
        }
        cost[p] = c;
        grad[3 * p] = gth;
        grad[3 * p + 1] = gx;
        grad[3 * p + 2] = gy;
        const double kap = c > 0.0 ? ce / c : 0.0;
        if (kappa) kappa[p] = kap;
        if (tau) {
            const double f = kap > 50.0 ? kap / 50.0 : 1.0;
            tau[3 * p] = sqrt(q0) * f;
            tau[3 * p + 1] = sqrt(q1) * f;
            tau[3 * p + 2] = sqrt(q2) * f;
        }
    }
}

/* ---------------------------------------------------------------------------------------
 * Per-localisation-uncertainty scores with a full covariance per point, and their gradient
 * with respect to a rigid transform of the second cloud.  Point k of cloud i is the
 * Gaussian N(x_k, S_k); point l of cloud j is N(y_l, T_l).  Moving cloud j by
 * q = (theta, tx, ty) about its centroid c_j moves a point to y'_l = R(y_l - c_j) + c_j + t
 * and turns its covariance into T'_l = R T_l R^T.  With V = S_k + T'_l and d = y'_l - x_k:
 *   mode 0 (GMM L2 cross term):  w = exp(-d^T V^-1 d / 2) / (2 pi sqrt(det V)),
 *                                 the integral of N(z; x_k, S_k) N(z; y'_l, T'_l) over z;
 *   mode 1 (Bhattacharya):        w = 2 (det S_k det T_l)^(1/4) / sqrt(det V) exp(-d^T V^-1 d / 4),
 *                                 the integral of sqrt(N(z; x_k, S_k) N(z; y'_l, T'_l)).
 * cost = sum_kl w.  Covariances come from cov (3 floats per point: xx, xy, yy) or, when cov
 * is NULL, from sig (isotropic s^2 I).  params (double [np][3]) may be NULL: identity.
 * Gradient (grad may be NULL), with a = 1/2 (L2) or 1/4 (Bhattacharya), g = dd/dtheta =
 * J (y'_l - c_j - t) and W = dV/dtheta = J T'_l - T'_l J (J the 90-degree rotation):
 *   dw/dt     = -2 a w V^-1 d
 *   dw/dtheta = w (-a (2 g^T V^-1 d - d^T V^-1 W V^-1 d) - tr(V^-1 W) / 2).
 * kappa = cost-weighted mean of the exponent a d^T V^-1 d; tau[p][m] =
 * sqrt(sum_kl (dw/dq_m)^2) max(1, kappa/50), as for the fixed-sigma overlap.
 * ------------------------------------------------------------------------------------- */
void oracle_gmm_grad_pairs(const float *xy, const float *sig, const float *cov, const int64_t *off, const float *cen,
                           int mode, const int64_t *pi, const int64_t *pj, const double *params, int64_t np,
                           double *cost, double *grad, double *tau, double *kappa)
{
    const double two_pi = 6.283185307179586476925286766559;
    const double a = mode == 0 ? 0.5 : 0.25;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < np; ++p) {
        const int64_t i = pi[p], j = pj[p];
        const double th = params ? params[3 * p] : 0.0;
        const double tx = params ? params[3 * p + 1] : 0.0, ty = params ? params[3 * p + 2] : 0.0;
        const double ct = cos(th), st = sin(th);
        const double cx = cen ? (double)cen[2 * j] : 0.0, cy = cen ? (double)cen[2 * j + 1] : 0.0;
        double c = 0.0, ce = 0.0, gth = 0.0, gx = 0.0, gy = 0.0, q0 = 0.0, q1 = 0.0, q2 = 0.0;
        for (int64_t l = off[j]; l < off[j + 1]; ++l) {
            /* moved point and covariance of cloud j */
            const double rx = (double)xy[2 * l] - cx, ry = (double)xy[2 * l + 1] - cy;
            const double ox = ct * rx - st * ry, oy = st * rx + ct * ry;
            const double yx = ox + cx + tx, yy = oy + cy + ty;
            const double gvx = -oy, gvy = ox; /* J R (y - c) */
            double t00, t01, t11;
            if (cov) {
                t00 = cov[3 * l];
                t01 = cov[3 * l + 1];
                t11 = cov[3 * l + 2];
            } else {
                t00 = t11 = (double)sig[l] * (double)sig[l];
                t01 = 0.0;
            }
            const double detT = t00 * t11 - t01 * t01;
            /* T' = R T R^T */
            const double m00 = ct * t00 - st * t01, m01 = ct * t01 - st * t11; /* (R T) row 0 */
            const double m10 = st * t00 + ct * t01, m11 = st * t01 + ct * t11; /* (R T) row 1 */
            const double r00 = m00 * ct - m01 * st, r01 = m00 * st + m01 * ct;
            const double r11 = m10 * st + m11 * ct;
            /* W = J T' - T' J for J = [[0, -1], [1, 0]] */
            const double w00 = -2.0 * r01, w01 = r00 - r11, w11 = 2.0 * r01;
            for (int64_t k = off[i]; k < off[i + 1]; ++k) {
                double s00, s01, s11;
                if (cov) {
                    s00 = cov[3 * k];
                    s01 = cov[3 * k + 1];
                    s11 = cov[3 * k + 2];
                } else {
                    s00 = s11 = (double)sig[k] * (double)sig[k];
                    s01 = 0.0;
                }
                const double detS = s00 * s11 - s01 * s01;
                const double v00 = s00 + r00, v01 = s01 + r01, v11 = s11 + r11;
                const double det = v00 * v11 - v01 * v01;
                /* inverse of V */
                const double i00 = v11 / det, i01 = -v01 / det, i11 = v00 / det;
                const double dx = yx - (double)xy[2 * k], dy = yy - (double)xy[2 * k + 1];
                const double ux = i00 * dx + i01 * dy, uy = i01 * dx + i11 * dy; /* V^-1 d */
                const double qf = dx * ux + dy * uy;
                const double e = a * qf;
                double w;
                if (mode == 0)
                    w = exp(-e) / (two_pi * sqrt(det));
                else
                    w = 2.0 * pow(detS * detT, 0.25) / sqrt(det) * exp(-e);
                c += w;
                ce += e * w;
                if (grad || tau) {
                    /* V^-1 W V^-1 d and tr(V^-1 W) */
                    const double wux = w00 * ux + w01 * uy, wuy = w01 * ux + w11 * uy;
                    const double quad = ux * wux + uy * wuy; /* d^T V^-1 W V^-1 d */
                    const double tr = i00 * w00 + 2.0 * i01 * w01 + i11 * w11;
                    const double dth = w * (-a * (2.0 * (gvx * ux + gvy * uy) - quad) - 0.5 * tr);
                    const double dtx = -2.0 * a * w * ux, dty = -2.0 * a * w * uy;
                    gth += dth;
                    gx += dtx;
                    gy += dty;
                    q0 += dth * dth;
                    q1 += dtx * dtx;
                    q2 += dty * dty;
                }
            }
        }
        cost[p] = c;
        const double kap = c > 0.0 ? ce / c : 0.0;
        if (kappa) kappa[p] = kap;
        if (grad) {
            grad[3 * p] = gth;
            grad[3 * p + 1] = gx;
            grad[3 * p + 2] = gy;
        }
        if (tau) {
            const double f = kap > 50.0 ? kap / 50.0 : 1.0;
            tau[3 * p] = sqrt(q0) * f;
            tau[3 * p + 1] = sqrt(q1) * f;
            tau[3 * p + 2] = sqrt(q2) * f;
        }
    }
}

/* ---------------------------------------------------------------------------------------
 * Sparse cosine.  Each item is a list of strictly ascending int64 keys with f32 values.
 * count = |K_i intersect K_j| by a two-pointer merge; dot = sum over shared keys of
 * v_i * v_j; cos = dot / (|v_i|_2 |v_j|_2) with the norms over all entries of each item;
 * keysum = wrapping 64-bit sum of the shared keys (an exactness witness);
 * tau = sqrt(sum over shared keys of (v_i v_j)^2) / (|v_i|_2 |v_j|_2), the error scale of
 * the dot product when every product carries one unit rounding (signed values, such as
 * background-corrected composition vectors, can cancel to a cosine near 0; for values of
 * one sign tau <= |cos|).
 * ------------------------------------------------------------------------------------- */
void oracle_sparse_pairs(const int64_t *keys, const float *vals, const int64_t *off, const int64_t *pi,
                         const int64_t *pj, int64_t np, double *cosv, int64_t *count, uint64_t *keysum,
                         double *tau)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < np; ++p) {
        const int64_t i = pi[p], j = pj[p];
        int64_t a = off[i], ae = off[i + 1], b = off[j], be = off[j + 1];
        double ni = 0.0, nj = 0.0;
        for (int64_t k = a; k < ae; ++k) ni += (double)vals[k] * (double)vals[k];
        for (int64_t k = b; k < be; ++k) nj += (double)vals[k] * (double)vals[k];
        double dot = 0.0, sq = 0.0;
        int64_t m = 0;
        uint64_t ks = 0;
        while (a < ae && b < be) {
            if (keys[a] < keys[b]) {
                ++a;
            } else if (keys[b] < keys[a]) {
                ++b;
            } else {
                const double pr = (double)vals[a] * (double)vals[b];
                dot += pr;
                sq += pr * pr;
                ++m;
                ks += (uint64_t)keys[a];
                ++a;
                ++b;
            }
        }
        cosv[p] = dot / (sqrt(ni) * sqrt(nj));
        if (tau) tau[p] = sqrt(sq) / (sqrt(ni) * sqrt(nj));
        if (count) count[p] = m;
        if (keysum) keysum[p] = ks;
    }
}

/* Number of OpenMP threads the pair loops use (reported beside CPU timings). */
int oracle_num_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}
