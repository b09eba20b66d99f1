// Host driver for the sanitizer build (AddressSanitizer + UndefinedBehaviorSanitizer) of the
// FP64 oracle (oracle/oracle.c) and the native tile planner (csrc/plan.cpp): every entry
// point on small random inputs, including empty items, single points and n = 0 .. 40 for the
// planner, with the planner's exact-coverage invariant checked.  Exits 0 and prints "ok"
// when nothing was reported; the sanitizers abort on the first finding.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <set>
#include <vector>

extern "C" {
int64_t oracle_packed_index(int64_t i, int64_t j, int64_t n);
void oracle_ncc_stats(const float *X, int64_t n, int64_t d, int64_t ld, double *mu, double *ss);
void oracle_ncc_pairs(const float *X, int64_t d, int64_t ld, const double *mu, const double *ss, const int64_t *pi,
                      const int64_t *pj, int64_t np, double *rho, double *tau);
void oracle_overlap_pairs(const float *xy, const int64_t *off, double sigma, const int64_t *pi, const int64_t *pj,
                          int64_t np, double *cost, double *kappa);
void oracle_gmm_pairs(const float *xy, const float *sig, const int64_t *off, int mode, const int64_t *pi,
                      const int64_t *pj, int64_t np, double *cost, double *kappa);
void oracle_overlap_grad_pairs(const float *xy, const int64_t *off, const float *cen, double sigma, const int64_t *pi,
                               const int64_t *pj, const double *params, int64_t np, double *cost, double *grad,
                               double *tau, double *kappa);
void oracle_gmm_grad_pairs(const float *xy, const float *sig, const float *cov, const int64_t *off, const float *cen,
                           int mode, const int64_t *pi, const int64_t *pj, const double *params, int64_t np,
                           double *cost, double *grad, double *tau, double *kappa);
void oracle_sparse_pairs(const int64_t *keys, const float *vals, const int64_t *off, const int64_t *pi,
                         const int64_t *pj, int64_t np, double *cosv, int64_t *count, uint64_t *keysum, double *tau);
}

namespace rk {
void plan_leaves(int64_t n, int64_t T, std::vector<int2> &out);
void plan_chunked(const std::vector<int2> &tiles, int nchunks, int nseg, std::vector<int4> &items,
                  std::vector<int> &seg, int halves);
void plan_lpt(const std::vector<int4> &items_in, const std::vector<double> &cost, int nseg, std::vector<int4> &items,
              std::vector<int> &seg);
void shuffle_items(std::vector<int4> &items, std::vector<int> &seg, uint64_t seed);
void single_segment(std::vector<int> &seg, int64_t nitems);
}  // namespace rk

static int fails = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++fails;                                                    \
        }                                                               \
    } while (0)

int main()
{
    std::mt19937_64 g(20090475);
    std::normal_distribution<float> nd(0.f, 1.f);
    std::uniform_real_distribution<float> ud(0.f, 1.f);
    const int64_t n = 7;
    std::vector<int64_t> pi, pj;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            pi.push_back(i);
            pj.push_back(j);
            CHECK(oracle_packed_index(i, j, n) == (int64_t)pi.size() - 1);
        }
    const int64_t np = (int64_t)pi.size();
    std::vector<double> a(np), b(np), grad(3 * np), tau3(3 * np), params(3 * np);
    for (auto &p : params) p = 0.2 * (ud(g) - 0.5);

    // NCC: rows padded to ld, one constant item
    const int64_t d = 37, ld = 40;
    std::vector<float> X(n * ld, -7.f);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = 0; k < d; ++k) X[i * ld + k] = i == 3 ? 2.f : nd(g);
    std::vector<double> mu(n), ss(n);
    oracle_ncc_stats(X.data(), n, d, ld, mu.data(), ss.data());
    oracle_ncc_pairs(X.data(), d, ld, mu.data(), ss.data(), pi.data(), pj.data(), np, a.data(), b.data());
    for (int64_t p = 0; p < np; ++p) CHECK(pi[p] == 3 || pj[p] == 3 ? std::isnan(a[p]) : std::fabs(a[p]) <= 1.0 + 1e-12);

    // clouds: sizes 0, 1 and a few points; sigma per point and full covariances
    const int64_t sizes[n] = {0, 1, 5, 3, 8, 2, 6};
    std::vector<int64_t> off(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + sizes[i];
    const int64_t m = off[n];
    std::vector<float> xy(2 * m), sig(m), cov(3 * m), cen(2 * n);
    for (auto &v : xy) v = ud(g);
    for (int64_t k = 0; k < m; ++k) {
        sig[k] = 0.01f + 0.02f * ud(g);
        const float s0 = 0.01f + 0.02f * ud(g), s1 = 0.01f + 0.02f * ud(g), r = 0.5f * (ud(g) - 0.5f);
        cov[3 * k] = s0 * s0;
        cov[3 * k + 1] = r * s0 * s1;
        cov[3 * k + 2] = s1 * s1;
    }
    for (int64_t i = 0; i < n; ++i) {
        double sx = 0, sy = 0;
        for (int64_t k = off[i]; k < off[i + 1]; ++k) {
            sx += xy[2 * k];
            sy += xy[2 * k + 1];
        }
        cen[2 * i] = sizes[i] ? (float)(sx / sizes[i]) : 0.f;
        cen[2 * i + 1] = sizes[i] ? (float)(sy / sizes[i]) : 0.f;
    }
    oracle_overlap_pairs(xy.data(), off.data(), 0.02, pi.data(), pj.data(), np, a.data(), b.data());
    for (int64_t p = 0; p < np; ++p) CHECK(a[p] >= 0.0);
    for (int mode = 0; mode < 2; ++mode) {
        oracle_gmm_pairs(xy.data(), sig.data(), off.data(), mode, pi.data(), pj.data(), np, a.data(), b.data());
        oracle_gmm_grad_pairs(xy.data(), sig.data(), nullptr, off.data(), cen.data(), mode, pi.data(), pj.data(),
                              params.data(), np, a.data(), grad.data(), tau3.data(), b.data());
        oracle_gmm_grad_pairs(xy.data(), nullptr, cov.data(), off.data(), cen.data(), mode, pi.data(), pj.data(),
                              params.data(), np, a.data(), grad.data(), tau3.data(), b.data());
        oracle_gmm_grad_pairs(xy.data(), nullptr, cov.data(), off.data(), nullptr, mode, pi.data(), pj.data(),
                              nullptr, np, a.data(), grad.data(), tau3.data(), b.data());
    }
    oracle_overlap_grad_pairs(xy.data(), off.data(), cen.data(), 0.02, pi.data(), pj.data(), params.data(), np,
                              a.data(), grad.data(), tau3.data(), b.data());

    // sparse: ascending keys, an empty item, a shared run of keys
    std::vector<int64_t> soff(n + 1, 0), keys;
    std::vector<float> vals;
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = (int64_t)(g() % 5);
        const int64_t cnt = i == 2 ? 0 : 1 + (int64_t)(g() % 30);
        for (int64_t e = 0; e < cnt; ++e) {
            k += 1 + (int64_t)(g() % 4);
            keys.push_back(k);
            vals.push_back(nd(g));
        }
        soff[i + 1] = (int64_t)keys.size();
    }
    std::vector<int64_t> count(np);
    std::vector<uint64_t> ksum(np);
    oracle_sparse_pairs(keys.data(), vals.data(), soff.data(), pi.data(), pj.data(), np, a.data(), count.data(),
                        ksum.data(), b.data());
    for (int64_t p = 0; p < np; ++p) CHECK(count[p] >= 0 && count[p] <= keys.size());

    // planner: every pair i < j of n items in exactly one leaf tile, for several tile sizes
    for (int64_t nn = 0; nn <= 40; ++nn)
        for (int64_t T : {1, 3, 8}) {
            std::vector<int2> leaves;
            rk::plan_leaves(nn, T, leaves);
            std::set<std::pair<int64_t, int64_t>> seen;
            for (const int2 &t : leaves)
                for (int64_t i = t.x * T; i < std::min(nn, (int64_t)(t.x + 1) * T); ++i)
                    for (int64_t j = std::max(i + 1, (int64_t)t.y * T); j < std::min(nn, (int64_t)(t.y + 1) * T); ++j)
                        CHECK(seen.insert({i, j}).second);
            CHECK((int64_t)seen.size() == nn * (nn - 1) / 2);
            std::vector<int4> items, lpt;
            std::vector<int> seg, lseg;
            rk::plan_chunked(leaves, 3, 8, items, seg, 2);
            CHECK(items.size() == leaves.size() * 3 * 2 && seg.size() == 9 && seg.back() == (int)items.size());
            std::vector<double> cost(items.size());
            for (auto &c : cost) c = ud(g);
            rk::plan_lpt(items, cost, 8, lpt, lseg);
            CHECK(lpt.size() == items.size() && lseg.back() == (int)lpt.size());
            rk::shuffle_items(items, seg, 7 + (uint64_t)nn);
            CHECK(seg.size() == 2 && seg.back() == (int)items.size());
            rk::single_segment(lseg, (int64_t)lpt.size());
        }
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}
