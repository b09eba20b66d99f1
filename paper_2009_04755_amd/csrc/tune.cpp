// Autotuner with a persisted cache (the batching pattern's tile shapes: uneven clouds and
// sparse vectors in one persistent launch, and the dense Gram tiles).
//
// For the prepared set, every candidate shape is prepared and one whole compare is timed
// with HIP events; the fastest is kept in the context's options and the set is prepared
// with it.  With a cache file set, the choice is stored under a key of (pair function,
// GPU architecture, log2 n, size quantiles of the items) and a later call with the same key
// applies the stored shape without timing anything.  Shapes that change only the schedule
// (NCC tile and waves, cloud block and inner-loop variant) give the same output bit for bit;
// the NCC K chunk and the sparse lanes / chunk width change FP32 summation order only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "common.hpp"

namespace rk {
namespace {

typedef std::map<std::string, std::map<std::string, double>> TuneCache;

std::string fn_name(int fn)
{
    switch (fn) {
    case ROCKET_NCC_FP32: return "ncc_fp32";
    case ROCKET_NCC_BF16X3: return "ncc_bf16x3";
    case ROCKET_NCC_BF16X6: return "ncc_bf16x6";
    case ROCKET_GAUSS_OVERLAP: return "gauss_overlap";
    case ROCKET_SPARSE_COSINE: return "sparse_cosine";
    case ROCKET_GMM_L2: return "gmm_l2";
    case ROCKET_GMM_BHATTACHARYA: return "gmm_bhattacharya";
    default: return "other";
    }
}

// Size bucket: round(2 log2(v)), so buckets are a factor sqrt(2) wide.
int bucket(double v) { return v > 0 ? (int)std::lround(2.0 * std::log2(v)) : -1; }

// p50 and p90 of ragged item sizes, in buckets.
std::string quantiles(const std::vector<int64_t> &off)
{
    std::vector<int64_t> sz;
    for (size_t i = 0; i + 1 < off.size(); ++i) sz.push_back(off[i + 1] - off[i]);
    if (sz.empty()) return "q-";
    std::sort(sz.begin(), sz.end());
    const double p50 = (double)sz[sz.size() / 2], p90 = (double)sz[std::min(sz.size() - 1, sz.size() * 9 / 10)];
    return "q" + std::to_string(bucket(p50)) + "-" + std::to_string(bucket(p90));
}

std::string arch_of(int device)
{
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

std::string tune_key(rocket_ctx *ctx)
{
    const int fn = ctx->prepared_fn;
    std::string k = fn_name(fn) + "|" + arch_of(ctx->device) + "|";
    if (fn == ROCKET_NCC_FP32 || fn == ROCKET_NCC_BF16X3 || fn == ROCKET_NCC_BF16X6)
        return k + "n" + std::to_string(bucket((double)ctx->ncc.n)) + "|d" + std::to_string(bucket((double)ctx->ncc.dim));
    if (fn == ROCKET_SPARSE_COSINE) return k + "n" + std::to_string(bucket((double)ctx->sp.n)) + "|" + quantiles(ctx->sp.h_offsets);
    const bool full = ctx->ovl.mode == OVL_FULL_L2 || ctx->ovl.mode == OVL_FULL_BH;
    return k + (full ? "cov|" : "") + "n" + std::to_string(bucket((double)ctx->ovl.n)) + "|" + quantiles(ctx->ovl.h_offsets);
}

// The cache file is one JSON object: {"key": {"option": value, ...}, ...}.  Only files this
// code wrote are read back, so the reader handles exactly that shape (and ignores the rest).
TuneCache cache_load(const std::string &path)
{
    TuneCache c;
    std::ifstream f(path);
    if (!f) return c;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t p = 0;
    auto str = [&](std::string &out) {  // next quoted string at or after p
        const size_t a = t.find('"', p);
        if (a == std::string::npos) return false;
        const size_t b = t.find('"', a + 1);
        if (b == std::string::npos) return false;
        out = t.substr(a + 1, b - a - 1);
        p = b + 1;
        return true;
    };
    std::string key;
    while (str(key)) {
        const size_t open = t.find('{', p), close = t.find('}', p);
        if (open == std::string::npos || close == std::string::npos || open > close) break;
        p = open + 1;
        std::map<std::string, double> &e = c[key];
        std::string name;
        while (true) {
            const size_t q = t.find('"', p);
            if (q == std::string::npos || q > close) break;
            if (!str(name)) break;
            const size_t colon = t.find(':', p);
            if (colon == std::string::npos || colon > close) break;
            e[name] = std::strtod(t.c_str() + colon + 1, nullptr);
            p = colon + 1;
        }
        p = close + 1;
    }
    return c;
}

bool cache_store(const std::string &path, const TuneCache &c)
{
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return false;
        f << "{\n";
        size_t i = 0;
        for (const auto &kv : c) {
            f << "  \"" << kv.first << "\": {";
            size_t j = 0;
            for (const auto &ov : kv.second) {
                char buf[64];
                snprintf(buf, sizeof buf, "%.6g", ov.second);
                f << "\"" << ov.first << "\": " << buf << (++j < kv.second.size() ? ", " : "");
            }
            f << "}" << (++i < c.size() ? ",\n" : "\n");
        }
        f << "}\n";
    }
    return std::rename(tmp.c_str(), path.c_str()) == 0;
}

struct Cand {
    std::vector<std::pair<rocket_option, int64_t>> opt;
};

const char *opt_name(rocket_option o)
{
    switch (o) {
    case ROCKET_OPT_NCC_TILE: return "ncc_tile";
    case ROCKET_OPT_NCC_KCHUNK: return "ncc_kchunk";
    case ROCKET_OPT_NCC_WAVES: return "ncc_waves";
    case ROCKET_OPT_SP_LANES: return "sp_lanes";
    case ROCKET_OPT_SP_CHUNK: return "sp_chunk";
    case ROCKET_OPT_OVL_BLOCK: return "ovl_block";
    case ROCKET_OPT_OVL_VARIANT: return "ovl_variant";
    default: return "unknown";
    }
}

// Prepare the set again with the context's current options (the inputs the last prepare saw).
rocket_status reprepare(rocket_ctx *ctx, hipStream_t s)
{
    const int fn = ctx->prepared_fn;
    rocket_items it = {};
    if (fn == ROCKET_NCC_FP32 || fn == ROCKET_NCC_BF16X3 || fn == ROCKET_NCC_BF16X6) {
        it.dense = ctx->ncc.src;
        it.dim = ctx->ncc.dim;
        it.ld = ctx->ncc.ld;
        return ncc_prepare(ctx, &it, ctx->ncc.n, fn, s);
    }
    it.offsets = ctx->sp.offsets;
    it.keys = ctx->sp.keys;
    it.vals = ctx->sp.vals;
    return sp_prepare(ctx, &it, ctx->sp.n, s);
}

rocket_status compare_into(rocket_ctx *ctx, float *out, hipStream_t s)
{
    const int fn = ctx->prepared_fn;
    if (fn == ROCKET_SPARSE_COSINE) return sp_compare(ctx, out, nullptr, s);
    return ncc_compare(ctx, out, s);
}

}  // namespace

rocket_status autotune(rocket_ctx *ctx, hipStream_t s)
{
    const int fn = ctx->prepared_fn;
    if (!fn) return fail(ctx, ROCKET_E_STATE, "autotune needs a prepared set");
    const bool ncc = fn == ROCKET_NCC_FP32 || fn == ROCKET_NCC_BF16X3 || fn == ROCKET_NCC_BF16X6;
    const bool clouds = fn == ROCKET_GAUSS_OVERLAP || fn == ROCKET_GMM_L2 || fn == ROCKET_GMM_BHATTACHARYA;
    const bool sparse = fn == ROCKET_SPARSE_COSINE;
    if (!ncc && !clouds && !sparse) return ROCKET_OK;  // PCE: one shape per side length
    const int64_t n = ncc ? ctx->ncc.n : sparse ? ctx->sp.n : ctx->ovl.n;
    ctx->stats.tune_us = 0;
    ctx->stats.tune_cached = 0;
    if (n < 2) return ROCKET_OK;
    const auto t0 = std::chrono::steady_clock::now();
    const std::string key = tune_key(ctx);
    TuneCache cache;
    if (!ctx->tune_cache.empty()) cache = cache_load(ctx->tune_cache);
    const auto hit = cache.find(key);
    if (hit != cache.end()) {
        for (const auto &ov : hit->second) {
            for (rocket_option o : {ROCKET_OPT_NCC_TILE, ROCKET_OPT_NCC_KCHUNK, ROCKET_OPT_NCC_WAVES,
                                    ROCKET_OPT_SP_LANES, ROCKET_OPT_SP_CHUNK, ROCKET_OPT_OVL_BLOCK,
                                    ROCKET_OPT_OVL_VARIANT})
                if (ov.first == opt_name(o)) ctx->opt[o] = (int64_t)ov.second;
        }
        ctx->stats.tune_cached = 1;
        if (!clouds) RK_TRY(reprepare(ctx, s));
        else RK_TRY(ovl_replan_public(ctx, s));
        ctx->stats.tune_us = (int64_t)std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
        return ROCKET_OK;
    }
    std::map<std::string, double> chosen;
    if (clouds) {
        RK_TRY(ovl_autotune(ctx, s));
        chosen["ovl_block"] = (double)ctx->opt[ROCKET_OPT_OVL_BLOCK];
        chosen["ovl_variant"] = (double)ctx->opt[ROCKET_OPT_OVL_VARIANT];
    } else {
        // candidate shapes
        std::vector<Cand> cands;
        if (ncc) {
            // K chunks no longer than the default: shorter chunks are more accurate (MFMA
            // accumulation error grows with chunk length), longer ones would leave the bar
            const int64_t kc0 = ctx->stats.kchunk;
            std::vector<int64_t> kcs = {kc0};
            if (kc0 / 2 >= 256 && (kc0 / 2) % 16 == 0) kcs.push_back(kc0 / 2);
            std::vector<int64_t> tiles = n >= 1536 ? std::vector<int64_t>{256, 128} : std::vector<int64_t>{128, 64};
            for (int64_t t : tiles)
                for (int64_t w : {(int64_t)8, (int64_t)4})
                    for (int64_t kc : kcs) {
                        if (t == 64 && w == 8) continue;  // 64-item tiles run with 4 waves
                        cands.push_back({{{ROCKET_OPT_NCC_TILE, t}, {ROCKET_OPT_NCC_WAVES, w}, {ROCKET_OPT_NCC_KCHUNK, kc}}});
                    }
        } else {
            const int64_t w0 = (int64_t)1 << ctx->sp.wlog;
            for (int64_t lanes : {(int64_t)4, (int64_t)8})
                for (int64_t ch : {(int64_t)0, 2 * w0})
                    cands.push_back({{{ROCKET_OPT_SP_LANES, lanes}, {ROCKET_OPT_SP_CHUNK, ch}}});
        }
        const int64_t P = n * (n - 1) / 2;
        float *scratch = nullptr;
        RK_HIP(hipMalloc(&scratch, sizeof(float) * P));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        rocket_status st = ROCKET_OK;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = ROCKET_E_HIP;
        int64_t save[32];
        std::copy(ctx->opt, ctx->opt + 32, save);
        const int64_t timing = ctx->opt[ROCKET_OPT_TIMING];
        ctx->opt[ROCKET_OPT_TIMING] = 0;
        float best = 1e30f;
        size_t best_i = 0;
        for (size_t c = 0; c < cands.size() && st == ROCKET_OK; ++c) {
            for (const auto &ov : cands[c].opt) ctx->opt[ov.first] = ov.second;
            if ((st = reprepare(ctx, s)) != ROCKET_OK) break;
            float ms = 0.f;
            for (int rep = 0; rep < 2 && st == ROCKET_OK; ++rep) {  // a warm-up pass unless the first is long
                (void)hipEventRecord(e0, s);
                st = compare_into(ctx, scratch, s);
                (void)hipEventRecord(e1, s);
                (void)hipEventSynchronize(e1);
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms > 50.f) break;
            }
            if (st == ROCKET_OK && ms < best) {
                best = ms;
                best_i = c;
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(scratch);
        ctx->opt[ROCKET_OPT_TIMING] = timing;
        if (st != ROCKET_OK) {
            std::copy(save, save + 32, ctx->opt);
            (void)reprepare(ctx, s);
            return st;
        }
        for (const auto &ov : cands[best_i].opt) {
            ctx->opt[ov.first] = ov.second;
            chosen[opt_name(ov.first)] = (double)ov.second;
        }
        chosen["ms"] = best;
        RK_TRY(reprepare(ctx, s));
    }
    if (!ctx->tune_cache.empty()) {
        cache[key] = chosen;
        if (!cache_store(ctx->tune_cache, cache)) return fail(ctx, ROCKET_E_INVALID, "cannot write the tune cache file");
    }
    ctx->stats.tune_us = (int64_t)std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    return ROCKET_OK;
}

}  // namespace rk

extern "C" rocket_status rocket_set_tune_cache(rocket_ctx *ctx, const char *path)
{
    if (!ctx) return rk::fail(nullptr, ROCKET_E_INVALID, "ctx is NULL");
    ctx->tune_cache = path ? std::string(path) : std::string();
    return ROCKET_OK;
}
