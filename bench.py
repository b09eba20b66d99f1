#!/usr/bin/env python3
"""All-pairs benchmark on one MI355X.

Workload: normalised cross-correlation of every pair of 4096 dense noise patterns of
1,048,576 float32 values (64 N(0,1) sources, item = 0.02 * source + N(0,1), zero-mean and
unit-norm), computed with the BF16 three-way split on the matrix cores (six bf16 products,
FP32 accumulation).  One step = the whole hot path for one batch: per-item FP64 statistics
and split (prepare), the persistent tile kernel over the divide-and-conquer queue, and the
split-K epilogue into the packed upper triangle (8,386,560 results).

Prints ONE JSON line.  ``value`` is pairs/s; ``roofline`` is the Gram kernel's algorithmic
2*d flop per pair against the bf16 dense MFMA peak (``traffic``: the HBM bytes of the
committed counter file when its kernel-source hash matches); ``cpu_baseline`` times the
FP64 oracle on a bounded sample of the same workload on this host.  Extra fields report the
plain FP32 and two-term split paths at the same shape, the same workload through the
out-of-core device cache, the NCC of 256 x 4096 and of 1024 patterns of 3648 x 2736 values
(the forensics images' size), the Gaussian-overlap, GMM and registration-gradient costs over
2048 point clouds (also with a full covariance per point, and the registration on each GMM
score), the sparse cosine of 8192 k-mer vectors, the PCE of 1024 images of 128 x 128 (one
LDS tile per pair), of 256 images of 1024 x 1024 and of 32 of 3648 x 2736 (transforms staged
in HBM), and the
composition-vector construction of 128 proteomes, each with its own roofline and, where
cheap enough, the oracle on a sample.  ``--only`` runs one of those workloads alone (for
profiling).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pairs/sec + % roofline per pair fn; BF16-split vs FP32 on same GPU at ≤1e-5 err"
PEAK_BF16 = 2500.0      # TFLOP/s, dense bf16 MFMA
PEAK_FP32_MFMA = 157.3  # TFLOP/s
PEAK_HBM = 8000.0       # GB/s
# VALU issue peak: the published FP32 vector peak (157.3 TFLOP/s = 256 CU x 128 FMA lanes x
# 2.4 GHz x 2 flop) as lane-instruction slots/s; a transcendental (exp2, rcp) takes 4 slots
VALU_LANE_OPS = 157.3e12 / 2
PEAK_FP32_VALU = 157.3  # TFLOP/s, the same peak as FMA flops
COUNTERS_FILE = os.path.join(ROOT, "profiles", "ncc_gram_bf16x6_4096x1048576_counters.txt")


def _gram_source(text):
    """The parts of the NCC source that decide the Gram kernel's memory traffic: the kernel
    itself (from its template line to the epilogue's header) and the host functions that
    pick its tile, K chunk and waves."""
    a = text.index("template <int BM, int BN, int SCH, int NWV>\n__global__")
    b = text.index("// Epilogue:", a)
    parts = [text[a:b]]
    for fn in ("static int ncc_tile(", "static int ncc_waves(", "static int64_t ncc_kchunk("):
        c = text.index(fn)
        parts.append(text[c:text.index("\n}\n", c) + 3])
    return "".join(parts)


def _src_hash(*names):
    """Hash of the Gram kernel's traffic-deciding source (ncc.hip) and of the other named
    sources whole."""
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2009_04755_amd", "csrc", n)) as f:
            t = f.read()
        h.update((_gram_source(t) if n == "ncc.hip" else t).encode())
    return h.hexdigest()[:16]


def _traffic_from_profile():
    """HBM bytes per gram launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source; else None."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    vals = {}
    with open(COUNTERS_FILE) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != _src_hash("ncc.hip", "queue.hpp"):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _dist(e, bar=1e-5):
    """max, median, p99, p99.99 and the count above ``bar`` of a per-result error array."""
    import numpy as np
    e = np.asarray(e, dtype=np.float64).ravel()
    if e.size == 0:
        return {"n": 0}
    q = np.quantile(e, [0.5, 0.99, 0.9999], method="higher")  # order statistics (no interpolation)
    f = lambda x: float(x) if np.isfinite(x) else str(float(x))  # strict JSON has no inf / nan
    return {"n": int(e.size), "max": f(e.max()), "p50": f(q[0]), "p99": f(q[1]), "p99_99": f(q[2]),
            "over_1e-5": int((e > bar).sum())}


def _errors(got, ref, floor=None, scale=None):
    """Per-result error report: the pure relative error |g - r| / |r| and the pass metric
    (|g - r| / max(|r|, floor), or |g - r| / scale when the bar has its own scale), each as
    a distribution; ``floor_active_frac`` is the share of results whose bar is set by the
    floor rather than by |r|."""
    import numpy as np
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    diff = np.abs(got - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        pure = np.where(ref != 0, diff / np.abs(ref), np.where(diff == 0, 0.0, np.inf))
    rep = {"pure_rel": _dist(pure)}
    if scale is not None:
        rep["pass_metric"] = _dist(diff / scale)
        rep["floor_active_frac"] = float(np.mean(scale > np.abs(ref) * (1 + 1e-12)))
    elif floor is not None:
        rep["pass_metric"] = _dist(diff / np.maximum(np.abs(ref), floor))
        rep["floor_active_frac"] = float(np.mean(floor > np.abs(ref)))
    return rep


def _host_info():
    """CPUs this process may run on and the CPU model (for the oracle timings)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"affinity_cpus": len(os.sched_getaffinity(0)), "cpu_model": model}


def _trace_summary(tr, grid):
    """Load balance of one traced persistent launch: span from the first start to the last
    end, the fraction of grid x span that workgroups spent in work items, per-XCD busy
    fractions (workgroup b on XCD b mod 8), and the tail after the first workgroup ran dry."""
    import numpy as np
    ran = tr[tr["workgroup"] >= 0]
    span = float(ran["end_ns"].max() - ran["start_ns"].min())
    busy = float(np.sum(ran["end_ns"] - ran["start_ns"]))
    last = np.array([ran["end_ns"][ran["workgroup"] == w].max() for w in np.unique(ran["workgroup"])])
    xcd = ran["workgroup"] % 8
    per_xcd = [float(np.sum((ran["end_ns"] - ran["start_ns"])[xcd == x])) / (span * grid / 8) for x in range(8)]
    return {"items": int(tr.size), "items_run": int(ran.size), "workgroups": int(grid), "span_ms": span * 1e-6,
            "busy_frac": busy / (span * grid), "busy_frac_per_xcd": per_xcd,
            "tail_ms": float(last.max() - last.min()) * 1e-6,
            "item_ms_p50_p99": [float(np.percentile(ran["end_ns"] - ran["start_ns"], q)) * 1e-6 for q in (50, 99)]}


def _ensure_built():
    from paper_2009_04755_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2009_04755_amd import build
        build.build()


def _time_fn(ctx, x, fn, out, steps, warmup):
    import torch
    for _ in range(warmup):
        ctx.allpairs(x, fn, out=out)
    torch.cuda.synchronize()
    kern = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.allpairs(x, fn, out=out)
        kern.append(ctx.stats()["kernel_ns"] * 1e-9)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, sum(kern) / len(kern)


def ncc_sample(n, T, seed=7):
    """Pairs checked against the oracle at full size: all pairs of 64 rows (the first and
    last row of every 256-item tile block among them, so tile edges are covered) plus 64
    random pairs in every output tile (drawn among 12 random rows per block)."""
    import numpy as np
    g = np.random.default_rng(seed)
    nb = (n + T - 1) // T
    edges = sorted({r for b in range(nb) for r in (b * T, min(n, (b + 1) * T) - 1)})
    rest = np.setdiff1d(np.arange(n), edges)
    rows64 = np.sort(np.concatenate([edges, g.choice(rest, 64 - len(edges), replace=False)]))[:64]
    iu = np.triu_indices(64, 1)
    pi, pj = [rows64[iu[0]]], [rows64[iu[1]]]
    per_block = [np.sort(g.choice(np.arange(b * T, min(n, (b + 1) * T)), 12, replace=False)) for b in range(nb)]
    for bi in range(nb):
        for bj in range(bi, nb):
            A, B = np.meshgrid(per_block[bi], per_block[bj], indexing="ij")
            a, b = A.ravel(), B.ravel()
            keep = a < b
            a, b = a[keep], b[keep]
            sel = g.choice(a.size, min(64, a.size), replace=False)
            pi.append(a[sel])
            pj.append(b[sel])
    pi, pj = np.concatenate(pi).astype(np.int64), np.concatenate(pj).astype(np.int64)
    _, first = np.unique(pi * n + pj, return_index=True)  # each pair once, in sampling order
    first = np.sort(first)
    return pi[first], pj[first]


def cpu_baseline(X, out, n, T, min_s=10.0):
    """FP64 oracle on the sampled pairs of the full-size workload (timed on every host
    thread it uses: FP64 item statistics + pair loop, rows already in host memory), and
    the per-result error report of the GPU output on the same pairs."""
    import numpy as np
    import oracle

    pi, pj = ncc_sample(n, T)
    rows = np.unique(np.concatenate([pi, pj]))
    Xh = X[torch_index(rows, X.device)].cpu().numpy()
    li, lj = np.searchsorted(rows, pi), np.searchsorted(rows, pj)
    reps = 0
    t0 = time.perf_counter()
    while True:
        rho, tau = oracle.ncc(Xh, li, lj)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= min_s or reps >= 20:
            break
    idx = pi * n - pi * (pi + 1) // 2 + (pj - pi - 1)
    got = out.cpu().numpy()[idx]
    rep = _errors(got, rho, floor=tau)
    rep["pairs"] = int(pi.size)
    rep["sample"] = "all pairs of 64 rows incl. the first and last row of each tile block, plus 64 pairs per output tile"
    base = {"value": pi.size * reps / dt, "unit": "pairs/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "%d pairs over %d of the 4096 patterns (1,048,576 values each): all pairs of 64 rows and 64 "
                      "pairs per output tile, %d pass(es); FP64 stats + pair loop, rows already in host memory"
                      % (pi.size, rows.size, reps)}
    base.update(_host_info())
    return base, rep


def torch_index(rows, device):
    import torch
    return torch.from_numpy(rows).to(device)


def ncc_small(ctx, with_cpu=True):
    """The 256 x 4096 NCC workload (8 sources, item = 0.05 source[i mod 8] + noise, zero-mean
    unit-norm), FP32 and BF16x6, all 32,640 pairs checked against the oracle."""
    import numpy as np
    import torch
    import oracle
    from paper_2009_04755_amd import synth

    n, d = 256, 4096
    X, _ = synth.dense_patterns(n, d, 8, 0.05, config=0)
    Xd = torch.from_numpy(X).cuda()
    P = n * (n - 1) // 2
    out = torch.empty(P, device="cuda")
    pi, pj = oracle.all_pairs(n)
    t0 = time.perf_counter()
    rho, tau = oracle.ncc(X, pi, pj)
    dto = time.perf_counter() - t0
    res = {"workload": "NCC all pairs of 256 patterns x 4096 f32 values (8 sources, amp 0.05)", "pairs": P}
    # the library's default shape for this size (64-item tiles, 256-element K chunks): the
    # context may hold the shape the autotuner chose for the 4096 x 2^20 headline
    keep = {k: ctx.get(k) for k in ("ncc_tile", "ncc_waves", "ncc_kchunk")}
    ctx.set(**{k: 0 for k in keep})
    for fn, peak, ops in (("ncc_fp32", PEAK_FP32_MFMA, 1), ("ncc_bf16x6", PEAK_BF16, 6)):
        dt, kern = _time_fn(ctx, Xd, fn, out, 20, 3)
        st = ctx.stats()
        flop = 2.0 * d * P
        res[fn] = {"pairs_per_s": 20 * P / dt, "ms_per_step": dt / 20 * 1e3, "kernel_ms": kern * 1e3,
                   "roofline": {"bound": "mfma", "achieved": flop / kern / 1e12, "peak": peak, "unit": "TFLOP/s",
                                "frac": flop / kern / 1e12 / peak},
                   "tile": st["tile"], "kchunk": st["kchunk"], "work_items": st["work_items"],
                   "errors": _errors(out.cpu().numpy(), rho, floor=tau)}
    ctx.set(**keep)
    if with_cpu:
        base = {"value": P / dto, "unit": "pairs/s", "cores": oracle.num_threads(), "kind": "oracle",
                "sample": "all 32,640 pairs (FP64 stats + pair loop)"}
        base.update(_host_info())
        res["cpu_baseline"] = base
    return res


def forensics_ncc(ctx, with_cpu=True):
    """NCC (BF16x6) of all pairs of 1024 synthetic patterns at the size of the forensics data
    set's images, 3648 x 2736 = 9,980,928 values each (Section V-A), with the library's
    default shape for this size."""
    import numpy as np
    import torch
    import oracle
    from paper_2009_04755_amd import synth

    n, d = 1024, 3648 * 2736
    X, _ = synth.dense_patterns_device(n, d, 64, 0.02, seed=3, device="cuda")
    P = n * (n - 1) // 2
    out = torch.empty(P, device="cuda")
    keep = {k: ctx.get(k) for k in ("ncc_tile", "ncc_waves", "ncc_kchunk")}
    ctx.set(**{k: 0 for k in keep})
    dt, kern = _time_fn(ctx, X, "ncc_bf16x6", out, 3, 1)
    st = ctx.stats()
    ctx.set(**keep)
    flop = 2.0 * d * P
    res = {"workload": "NCC all pairs of 1024 patterns x 3648 x 2736 f32 values (64 sources, amp 0.02), BF16x6",
           "pairs_per_s": 3 * P / dt, "ms_per_step": dt / 3 * 1e3, "kernel_ms": kern * 1e3,
           "us_per_pair": dt / 3 / P * 1e6, "tile": st["tile"], "kchunk": st["kchunk"],
           "work_items": st["work_items"],
           "roofline": {"bound": "mfma", "achieved": flop / kern / 1e12, "peak": PEAK_BF16, "unit": "TFLOP/s",
                        "frac": flop / kern / 1e12 / PEAK_BF16},
           "paper_context": "1.1 ms per pair for the same comparison on a TitanX (Maxwell) GPU (another machine)"}
    if with_cpu:
        # 32 random pairs against the oracle (FP64), timed on the host cores
        g = np.random.default_rng(11)
        pi = g.integers(0, n, 48)
        pj = g.integers(0, n, 48)
        keepp = pi != pj
        pi, pj = np.minimum(pi, pj)[keepp][:32], np.maximum(pi, pj)[keepp][:32]
        rows = np.unique(np.concatenate([pi, pj]))
        Xs = X[torch.from_numpy(rows).cuda()].cpu().numpy()
        loc = {r: k for k, r in enumerate(rows.tolist())}
        li = np.array([loc[a] for a in pi.tolist()])
        lj = np.array([loc[b] for b in pj.tolist()])
        t0 = time.perf_counter()
        rho, tau = oracle.ncc(Xs, li, lj)
        dto = time.perf_counter() - t0
        idx = pi * n - pi * (pi + 1) // 2 + (pj - pi - 1)
        res["errors"] = _errors(out.cpu().numpy()[idx], rho, floor=tau)
        res["cpu_baseline"] = dict({"value": len(li) / dto, "unit": "pairs/s", "cores": oracle.num_threads(),
                                    "kind": "oracle", "sample": "%d random pairs (FP64 stats + dot)" % len(li)},
                                   **_host_info())
    del X, out
    torch.cuda.empty_cache()
    return res


PEAK_PCIE = 64.0  # GB/s per direction, PCIe 5.0 x16


def out_of_core(ctx, X, ref):
    """Same NCC workload with the items in pinned host memory and a device cache of 8 and
    of 16 slots (256 items each); `ref` holds the in-core result."""
    import torch
    n, d = X.shape
    Xh = torch.empty((n, d), dtype=torch.float32, pin_memory=True)
    Xh.copy_(X)
    P = n * (n - 1) // 2
    res = {"workload": "4096 x 1,048,576 f32 in pinned host memory, BF16x6, LRU device cache of 256-item slots"}
    for slots in (8, 16):
        ctx.set(cache_slots=slots)
        got = ctx.allpairs_host(Xh, "ncc_bf16x6")  # warm-up (allocates the cache)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        got = ctx.allpairs_host(Xh, "ncc_bf16x6", out=got)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = ctx.stats()
        nb = (n + st["tile"] - 1) // st["tile"]
        h2d = st["cache_loads"] * st["tile"] * d * 4
        res["slots_%d" % slots] = {"pairs_per_s": P / dt, "ms": dt * 1e3, "loads": st["cache_loads"],
                                   "reload_factor": st["cache_loads"] / nb, "h2d_bytes": h2d,
                                   "h2d_GBps": h2d / dt / 1e9, "pcie_frac": h2d / dt / 1e9 / PEAK_PCIE,
                                   "identical_to_in_core": bool(torch.equal(got, ref))}
    ctx.set(cache_slots=0)
    del Xh
    return res


# Process pool for the numpy oracles (numpy's FFT and sorting hold the interpreter lock, so
# threads do not scale): fresh interpreters that never touch the GPU, one per host CPU of
# this process (at most 16), each handed the data it needs once.
_POOL_DATA = {}


def _pool_init(data):
    _POOL_DATA.update(data)


def _pool_size():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _pce_job(job):
    """Oracle PCE of pairs (i, j): the oracle's own peak and PCE, and the oracle PCE at the
    GPU's peak g with whether C(g) is within 1e-5 RMS of the maximum."""
    import numpy as np
    import oracle.pce as opce
    X, L = _POOL_DATA["X"], _POOL_DATA["L"]
    out = []
    for i, j, g in job:
        C = opce.correlation(X[i].reshape(L, L), X[j].reshape(L, L))
        own, pk = opce.pce_of_surface(C, 5)
        at_g, _ = opce.pce_of_surface(C, 5, peak=g)
        out.append((own, pk, at_g, bool(C.flat[g] >= C.max() - 1e-5 * np.sqrt(np.mean(C * C)))))
    return out


def _pce_big_job(job):
    """Oracle PCE of H x W pairs (i, j) with the GPU's peak g: own PCE and peak, PCE at g, and
    whether C(g) is within 1e-5 RMS of the maximum."""
    import numpy as np
    import oracle.pce as opce
    X, H, W = _POOL_DATA["X"], _POOL_DATA["H"], _POOL_DATA["W"]
    out = []
    for i, j, g in job:
        C = opce.correlation(X[i].reshape(H, W), X[j].reshape(H, W))
        own, pk = opce.pce_of_surface(C, 5)
        at_g, _ = opce.pce_of_surface(C, 5, peak=g)
        out.append((own, pk, at_g, bool(C.flat[g] >= C.max() - 1e-5 * np.sqrt(np.mean(C * C)))))
    return out


def _cv_job(s):
    import oracle.cv as ocv
    res, off, K = _POOL_DATA["res"], _POOL_DATA["off"], _POOL_DATA["K"]
    return ocv.composition_vector(res[off[s]:off[s + 1]], K)


def _run_pool(fn, jobs, data):
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(_pool_size(), initializer=_pool_init, initargs=(data,)) as pool:
        pool.map(fn, jobs[:_pool_size()])  # warm every worker (imports) outside the timing
        t0 = time.perf_counter()
        r = pool.map(fn, jobs)
        return r, time.perf_counter() - t0


def cv_pipeline(ctx, with_cpu=True):
    """Composition vectors of 128 synthetic proteomes (~0.84 M residues each, K = 6) on the
    GPU, then the sparse cosine of all their pairs."""
    import numpy as np
    import torch
    from paper_2009_04755_amd import synth

    n, K = 128, 6
    res, off = synth.proteomes(n, config=5, salt=100)
    r = torch.from_numpy(res).cuda()
    o = torch.from_numpy(off).cuda()
    S = ctx.cv_build(r, o, K)  # warm-up: allocates and zeroes the count arrays
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = ctx.cv_build(r, o, K)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern = ctx.stats()["kernel_ns"] * 1e-9
    entries = int(S.offsets[-1].item())
    streamed = n * 4 * 20 ** K  # the emit pass reads every species' dense K-string counts once
    res_ = {"workload": "128 synthetic proteomes (4000-family pool, p_keep 0.7), %d residues, K = 6" % off[-1],
            "species_per_s": n / dt, "residues_per_s": off[-1] / dt, "ms": dt * 1e3, "device_ms": kern * 1e3,
            "entries": entries, "entries_per_species": entries / n,
            "roofline": {"bound": "hbm", "achieved": streamed / kern / 1e9, "peak": PEAK_HBM, "unit": "GB/s",
                         "frac": streamed / kern / 1e9 / PEAK_HBM,
                         "model": "4 * 20^K bytes of dense counts streamed per species"}}
    out = torch.empty(n * (n - 1) // 2, device="cuda")
    # the library's default sparse shape for this set (the context may hold the one tuned for
    # the 8192-item sparse workload)
    keep = {k: ctx.get(k) for k in ("sp_lanes", "sp_chunk")}
    ctx.set(**{k: 0 for k in keep})
    ctx.allpairs(S, "sparse_cosine", out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.allpairs(S, "sparse_cosine", out=out)
    torch.cuda.synchronize()
    res_["cosine_all_pairs"] = {"pairs": n * (n - 1) // 2, "ms": (time.perf_counter() - t0) * 1e3}
    ctx.set(**keep)
    if with_cpu:
        # oracle composition vectors of the first 24 species (one process per host CPU),
        # checked against the GPU's, then the oracle cosine of their 276 pairs against the
        # GPU cosine of the same pairs in the 128-species run (signed values: floored bar)
        import oracle
        m = 24
        cvs, dto = _run_pool(_cv_job, list(range(m)), {"res": res[: off[m]], "off": off[: m + 1], "K": K})
        goff = S.offsets.cpu().numpy()
        gk, gv = S.keys.cpu().numpy(), S.vals.cpu().numpy()
        keys_exact = all(np.array_equal(gk[goff[s_]:goff[s_ + 1]], cvs[s_][0]) for s_ in range(m))
        vref = np.concatenate([c[1] for c in cvs])
        vgot = gv[: goff[m]]
        co = np.zeros(m + 1, dtype=np.int64)
        co[1:] = np.cumsum([c[0].size for c in cvs])
        ck = np.concatenate([c[0] for c in cvs])
        pi, pj = oracle.all_pairs(m)
        ref, rcnt, _, tau = oracle.sparse_cosine(co, ck, vref.astype(np.float32), pi, pj, with_tau=True)
        idx = pi * n - pi * (pi + 1) // 2 + (pj - pi - 1)
        res_["errors"] = {"keys_bit_exact": bool(keys_exact),
                          "values_f32_ulps_max": float(np.max(np.abs(vgot.astype(np.float64) - vref) /
                                                              np.spacing(np.abs(vref).astype(np.float32)))),
                          "cosine": _errors(out.cpu().numpy()[idx], ref, floor=tau)}
        res_["cpu_baseline"] = dict({"value": m / dto, "unit": "species/s", "cores": _pool_size(), "kind": "oracle",
                                     "sample": "the first 24 of the 128 proteomes (numpy, one process per CPU)"},
                                    **_host_info())
    return res_


PEAK_LDS = 256 * 128 * 2.4e9 / 1e9  # GB/s: 128 bytes per clock per CU


def pce_pair_fn(ctx, with_cpu=True):
    """PCE over all shifts for 1024 noise images of 128 x 128 (523,776 pairs)."""
    import numpy as np
    import torch
    from paper_2009_04755_amd import synth

    n, L = 1024, 128
    X, _, _ = synth.noise_images(n, L, nsrc=16, amp=0.3, config=6, salt=0)
    Xd = torch.from_numpy(X).cuda()
    P = n * (n - 1) // 2
    out = torch.empty(P, device="cuda")
    dt, kern = _time_fn(ctx, Xd, "pce", out, 3, 1)
    # LDS bytes per pair of the in-LDS design, per FFT shared by two pairs: product tile
    # written, four FFT steps read and write the L x L complex tile, one statistics pass
    lds_bytes = (1 + 8 + 1) * L * L * 8 / 2
    res = {"workload": "1024 noise images 128 x 128 (16 sources, amp 0.3, 25 % shifted crops), h = 5",
           "pairs_per_s": 3 * P / dt, "kernel_ms": kern * 1e3,
           "roofline": {"bound": "lds", "achieved": P * lds_bytes / kern / 1e9, "peak": PEAK_LDS, "unit": "GB/s",
                        "frac": P * lds_bytes / kern / 1e9 / PEAK_LDS,
                        "model": "10 L^2 complex f32 LDS passes per FFT, one FFT per two pairs"}}
    if with_cpu:
        # all pairs among 64 random images, oracle on one process per host CPU; the GPU's
        # PCE is compared at the GPU's peak where that peak is a valid one (its correlation
        # within 1e-5 RMS of the maximum), and peak agreement is reported
        import oracle
        g = np.random.default_rng(8)
        rows = np.sort(g.choice(n, 64, replace=False))
        li, lj = oracle.all_pairs(64)
        pi, pj = rows[li], rows[lj]
        idx = pi * n - pi * (pi + 1) // 2 + (pj - pi - 1)
        got, pk = ctx.allpairs(Xd, "pce", counts=True)
        got, pk = got.cpu().numpy()[idx], pk.cpu().numpy()[idx].astype(np.int64)
        jobs = [list(zip(li[a:a + 32].tolist(), lj[a:a + 32].tolist(), pk[a:a + 32].tolist()))
                for a in range(0, li.size, 32)]
        r, dto = _run_pool(_pce_job, jobs, {"X": X[rows], "L": L})
        r = [t for part in r for t in part]
        own = np.array([t[0] for t in r])
        at_g = np.array([t[2] for t in r])
        valid = np.array([t[3] for t in r])
        res["errors"] = {"peak_agrees_frac": float(np.mean(np.array([t[1] for t in r]) == pk)),
                         "gpu_peak_valid_frac": float(np.mean(valid)),
                         "pce_at_gpu_peak": _errors(got[valid], at_g[valid])}
        res["cpu_baseline"] = dict({"value": li.size / dto, "unit": "pairs/s", "cores": _pool_size(),
                                    "kind": "oracle", "sample": "all 2016 pairs of 64 random images (numpy FFT, "
                                                                "FP64, one process per CPU)"}, **_host_info())
        del own
    return res


def _fft_len(N):
    """FFT length of an N-point axis of the staged PCE: N for a power of two, else the
    Bluestein length (the power of two >= 2N - 1), and the number of FFTs per DFT."""
    if N & (N - 1) == 0:
        return N, 1
    M = 1
    while M < 2 * N - 1:
        M *= 2
    return M, 2


def pce_big_pair_fn(ctx, with_cpu=True, n=256, H=1024, W=1024, nsrc=16, sample=128):
    """PCE over all shifts for n noise images of H x W (default: 256 of 1024 x 1024, 32,640
    pairs): the staged multi-pass path, in its default batches of two-pair transforms."""
    import numpy as np
    import torch
    from paper_2009_04755_amd import synth

    X, _, _ = synth.noise_images(n, (H, W), nsrc=nsrc, amp=0.3, config=6, salt=1 if H == W == 1024 else H + W)
    Xd = torch.from_numpy(X).cuda()
    P = n * (n - 1) // 2
    out = torch.empty(P, device="cuda")
    ctx.set(pce_width=W)
    dt, kern = _time_fn(ctx, Xd, "pce", out, 3, 1)
    st = ctx.stats()
    npp = (P + 1) // 2
    # bytes per two-pair transform the design has to move: the four half spectra read, the
    # staged H x W complex transform written by the row pass and read by the column pass
    spec = H * (W // 2 + 1) * 8
    per_pp = 4 * spec + 2 * H * W * 8
    # nominal FFT flops per two-pair transform (5 M log2 M per M-point FFT): H row DFTs and
    # W column DFTs, each one FFT, or two of the Bluestein length
    (MW, kw), (MH, kh) = _fft_len(W), _fft_len(H)
    flops_pp = 5 * (H * kw * MW * np.log2(MW) + W * kh * MH * np.log2(MH))
    pct = "%d %%" % round(100 * 0.25) if H == W == 1024 else "25 %"
    res = {"workload": "%d noise images %d x %d (%d sources, amp 0.3, %s shifted crops), h = 5" % (n, H, W, nsrc, pct),
           "pairs_per_s": 3 * P / dt, "kernel_ms": kern * 1e3, "batch_pair_pairs": st["grid"],
           "roofline": {"bound": "hbm", "achieved": npp * per_pp / kern / 1e9, "peak": PEAK_HBM, "unit": "GB/s",
                        "frac": npp * per_pp / kern / 1e9 / PEAK_HBM, "bytes_per_pair_pair": per_pp,
                        "model": "4 half spectra read + staged H x W complex transform written and read once, "
                                 "per two-pair transform (row pass, column pass, peak and PCE kernels together)"},
           "fft_flop_rate": {"achieved": npp * flops_pp / kern / 1e12, "unit": "TFLOP/s", "peak": PEAK_FP32_VALU,
                             "frac": npp * flops_pp / kern / 1e12 / PEAK_FP32_VALU, "flops_per_pair_pair": flops_pp,
                             "model": "5 M log2 M per M-point FFT; an axis that is not a power of two costs two "
                                      "FFTs of the Bluestein length M >= 2N - 1"}}
    if H != W or H & (H - 1):
        res["fft_lengths"] = {"rows": int(MW), "columns": int(MH)}
    if with_cpu:
        # random pairs, oracle (numpy FFT, FP64) on one process per host CPU; PCE compared at
        # the GPU's peak where that peak is a valid one
        g = np.random.default_rng(9)
        pi = g.integers(0, n, sample + sample // 4)
        pj = g.integers(0, n, sample + sample // 4)
        keep = pi != pj
        pi, pj = np.minimum(pi, pj)[keep][:sample], np.maximum(pi, pj)[keep][:sample]
        idx = pi * n - pi * (pi + 1) // 2 + (pj - pi - 1)
        got, pk = ctx.allpairs(Xd, "pce", counts=True)
        got, pk = got.cpu().numpy()[idx], pk.cpu().numpy()[idx].astype(np.int64)
        rows = np.unique(np.concatenate([pi, pj]))
        loc = {r: k for k, r in enumerate(rows)}
        li = [loc[a] for a in pi.tolist()]
        lj = [loc[b] for b in pj.tolist()]
        per_job = max(1, min(8, len(li) // _pool_size()))
        jobs = [list(zip(li[a:a + per_job], lj[a:a + per_job], pk[a:a + per_job].tolist()))
                for a in range(0, len(li), per_job)]
        r, dto = _run_pool(_pce_big_job, jobs, {"X": X[rows], "H": H, "W": W})
        r = [t for part in r for t in part]
        at_g = np.array([t[2] for t in r])
        valid = np.array([t[3] for t in r])
        res["errors"] = {"peak_agrees_frac": float(np.mean(np.array([t[1] for t in r]) == pk)),
                         "gpu_peak_valid_frac": float(np.mean(valid)),
                         "pce_at_gpu_peak": _errors(got[valid], at_g[valid])}
        res["cpu_baseline"] = dict({"value": len(li) / dto, "unit": "pairs/s", "cores": _pool_size(),
                                    "kind": "oracle", "sample": "%d random pairs of the %d images (numpy FFT, "
                                                                "FP64, one process per CPU)" % (len(li), n)},
                                   **_host_info())
    ctx.set(pce_width=0)
    del Xd
    torch.cuda.empty_cache()
    return res


def valu_probe():
    """Measured issue rates behind the VALU rooflines: FP32 FMA, v_exp_f32 and v_rcp_f32 in
    independent chains (rocket_probe_valu), against the lane-slot peak used as denominator."""
    from paper_2009_04755_amd import probe_valu
    r = probe_valu(0)
    r.update({"lane_slot_peak": VALU_LANE_OPS, "fma_frac_of_peak": r["fma_per_s"] / VALU_LANE_OPS,
              "exp2_frac_of_quarter_peak": r["exp2_per_s"] / (VALU_LANE_OPS / 4),
              "rcp_frac_of_quarter_peak": r["rcp_per_s"] / (VALU_LANE_OPS / 4),
              "exp2_cost_in_fma": r["fma_per_s"] / r["exp2_per_s"], "rcp_cost_in_fma": r["fma_per_s"] / r["rcp_per_s"]})
    return r


def other_pair_fns(ctx, with_cpu=True, autotune=True):
    """Gaussian overlap (2048 uneven clouds), the two per-point-sigma scores and the
    20-step registration, one entry each."""
    import numpy as np
    import torch
    from paper_2009_04755_amd import Clouds, register, synth

    res = {}
    off, xy = synth.point_clouds(2048, config=2)
    cl = Clouds(torch.from_numpy(off).cuda(), torch.from_numpy(xy).cuda(), 0.02)
    P = 2048 * 2047 // 2
    out = torch.empty(P, device="cuda")
    ctx.set(ovl_variant=0, ovl_block=0)
    tune = None
    if autotune:  # untimed setup: clouds per block x inner-loop variant
        ctx.prepare(cl, "gauss_overlap")
        tune = ctx.autotune()
    dt, kern = _time_fn(ctx, cl, "gauss_overlap", out, 5, 1)
    cnt = np.diff(off).astype(np.float64)
    terms = (cnt.sum() ** 2 - (cnt ** 2).sum()) / 2
    # per term: 2 sub, mul, fma, mul, add (VALU) + exp (transcendental, counted as 4 slots)
    peak_terms = VALU_LANE_OPS / 10.0
    res["gauss_overlap"] = {"workload": "2048 clouds, 50..400 points, sigma 0.02", "pairs_per_s": 5 * P / dt,
                            "kernel_ms": kern * 1e3, "terms_per_s": terms / kern,
                            "roofline": {"bound": "alu", "achieved": terms / kern, "peak": peak_terms,
                                         "unit": "terms/s", "frac": terms / kern / peak_terms}}
    if tune is not None:
        res["gauss_overlap"]["autotune"] = dict(tune, candidates="block {4, 8, 16} x variant 1..4")
    ctx.set(ovl_variant=0, ovl_block=0)  # the other scores run with their defaults
    if with_cpu:
        import oracle
        g = np.random.default_rng(5)
        pi = g.integers(0, 2047, 3000)
        pj = np.minimum(2047, pi + 1 + g.integers(0, 2047, 3000) % (2047 - pi))
        t0 = time.perf_counter()
        ref, kap = oracle.overlap(off, xy, pi, pj, 0.02)
        dto = time.perf_counter() - t0
        res["gauss_overlap"]["cpu_baseline"] = dict(
            {"value": pi.size / dto, "unit": "pairs/s", "cores": oracle.num_threads(), "kind": "oracle",
             "sample": "3000 random pairs of the 2048 clouds"}, **_host_info())
        # bar: |g - r| <= 1e-5 (r max(1, kappa/50) + 1e5 N_i N_j 2^-126), reported as |g - r| / (...)
        nn = cnt[pi] * cnt[pj]
        got = out.cpu().numpy()[pi * 2048 - pi * (pi + 1) // 2 + (pj - pi - 1)]
        res["gauss_overlap"]["errors"] = _errors(got, ref, scale=ref * np.maximum(1, kap / 50) + 1e5 * nn * 2.0 ** -126)
        res["gauss_overlap"]["errors"]["kappa_over_50_frac"] = float(np.mean(kap > 50))
    # per-localisation-uncertainty scores on the same clouds, sigma_k ~ U[0.01, 0.03]
    sig = synth.point_sigmas(off)
    clg = Clouds(cl.offsets, cl.xy, 0.02, torch.from_numpy(sig).cuda())
    for fn, mode, slots in (("gmm_l2", "l2", 15.0), ("gmm_bhattacharya", "bhattacharya", 16.0)):
        # per term: 2 sub, mul, fma, fma, mul, fma (+ one mul for Bhattacharya) VALU, rcp + exp2 (4 slots each)
        dtg, kg = _time_fn(ctx, clg, fn, out, 5, 1)
        peak_g = VALU_LANE_OPS / slots
        res[fn] = {"workload": "2048 clouds, 50..400 points, per-point sigma U[0.01, 0.03]",
                   "pairs_per_s": 5 * P / dtg, "kernel_ms": kg * 1e3, "terms_per_s": terms / kg,
                   "roofline": {"bound": "alu", "achieved": terms / kg, "peak": peak_g, "unit": "terms/s",
                                "frac": terms / kg / peak_g}}
        if with_cpu:
            import oracle
            g = np.random.default_rng(6)
            pi = g.integers(0, 2047, 2000)
            pj = np.minimum(2047, pi + 1 + g.integers(0, 2047, 2000) % (2047 - pi))
            t0 = time.perf_counter()
            ref, kap = oracle.gmm(off, xy, sig, pi, pj, mode, with_kappa=True)
            dto = time.perf_counter() - t0
            res[fn]["cpu_baseline"] = dict(
                {"value": pi.size / dto, "unit": "pairs/s", "cores": oracle.num_threads(), "kind": "oracle",
                 "sample": "2000 random pairs of the 2048 clouds"}, **_host_info())
            nn = cnt[pi] * cnt[pj]
            pre = max(1.0, 1.0 / (2 * np.pi * float(sig.min()) ** 2))
            got = out.cpu().numpy()[pi * 2048 - pi * (pi + 1) // 2 + (pj - pi - 1)]
            res[fn]["errors"] = _errors(got, ref, scale=ref * np.maximum(1, kap / 50) + 1e5 * nn * pre * 2.0 ** -126)
            res[fn]["errors"]["kappa_over_50_frac"] = float(np.mean(kap > 50))
    # full covariance per localisation (uncertainty ellipses, semi-axes U[0.01, 0.03]); VALU
    # slots per term counted in the kernels' compiled inner loops (3 transcendentals at 4)
    cov = synth.point_covs(off)
    clc = Clouds(cl.offsets, cl.xy, 0.02, point_cov=torch.from_numpy(cov).cuda())
    g = np.random.default_rng(12)
    sel = np.sort(g.choice(P, 1000, replace=False))
    iu = np.triu_indices(2048, 1)
    spi, spj = iu[0][sel].astype(np.int64), iu[1][sel].astype(np.int64)
    for fn, mode, slots in (("gmm_l2", "l2", 30.6), ("gmm_bhattacharya", "bhattacharya", 31.6)):
        dtg, kg = _time_fn(ctx, clc, fn, out, 3, 1)
        peak_g = VALU_LANE_OPS / slots
        rec = {"workload": "2048 clouds, 50..400 points, full covariance per point (semi-axes U[0.01, 0.03])",
               "pairs_per_s": 3 * P / dtg, "kernel_ms": kg * 1e3, "terms_per_s": terms / kg,
               "roofline": {"bound": "alu", "achieved": terms / kg, "peak": peak_g, "unit": "terms/s",
                            "frac": terms / kg / peak_g, "valu_slots_per_term": slots}}
        if with_cpu:
            import oracle
            t0 = time.perf_counter()
            ref, _, _, kap = oracle.gmm_grad(off, xy, spi, spj, mode, cov=cov)
            dto = time.perf_counter() - t0
            nn = cnt[spi] * cnt[spj]
            pre = max(1.0, 1.0 / (2 * np.pi * 2 * 0.01 ** 2)) if mode == "l2" else 2.0
            rec["errors"] = _errors(out.cpu().numpy()[sel], ref,
                                    scale=ref * np.maximum(1, kap / 50) + 1e5 * nn * pre * 2.0 ** -126)
            rec["errors"]["kappa_over_50_frac"] = float(np.mean(kap > 50))
            rec["cpu_baseline"] = dict({"value": sel.size / dto, "unit": "pairs/s", "cores": oracle.num_threads(),
                                        "kind": "oracle", "sample": "1000 random pairs of the 2048 clouds"},
                                       **_host_info())
        res[fn + "_full_cov"] = rec
    cen = torch.from_numpy(synth.cloud_centroids(off, xy)).cuda()
    p0 = torch.from_numpy(synth.rigid_starts(P, config=3)).cuda()
    # registration on each GMM score with full covariances: 20 GD steps of the adjoint kernel;
    # the step is scaled by the score's largest term (1 / (4 pi s^2) at s = 0.02 for L2) so the
    # three registrations move their transforms by comparable amounts
    for fn, mode, slots, lr in (("gmm_l2", "l2", 47.0, 0.01 * 4 * np.pi * 0.02 ** 2),
                                ("gmm_bhattacharya", "bhattacharya", 48.0, 0.01)):
        register(clc, cen, p0, steps=1, ctx=ctx, fn=fn, lr=lr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pf = register(clc, cen, p0, steps=20, ctx=ctx, fn=fn, lr=lr)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kern = ctx.stats()["kernel_ns"] * 1e-9
        peak_g = VALU_LANE_OPS / slots
        rec = {"workload": "same clouds with full covariances, adjoint of (theta, tx, ty) of the %s score, 20 GD "
                           "steps" % mode,
               "pair_steps_per_s": 20 * P / dt, "kernel_ms": kern * 1e3,
               "roofline": {"bound": "alu", "achieved": terms / kern, "peak": peak_g, "unit": "terms/s",
                            "frac": terms / kern / peak_g, "valu_slots_per_term": slots}}
        if with_cpu:
            import oracle
            cost, grad = ctx.cost_grad(clc, cen, pf.contiguous(), fn=fn)
            prm = pf.cpu().numpy()[sel].astype(np.float64)
            rc, rg, tau, kap = oracle.gmm_grad(off, xy, spi, spj, mode, cov=cov, centroids=cen.cpu().numpy(),
                                               params=prm)
            nn = cnt[spi] * cnt[spj]
            pre = max(1.0, 1.0 / (2 * np.pi * 2 * 0.01 ** 2)) if mode == "l2" else 2.0
            sl = nn * pre * 2.0 ** -126
            rec["errors"] = {
                "cost": _errors(cost.cpu().numpy()[sel], rc, scale=rc * np.maximum(1, kap / 50) + 1e5 * sl),
                "grad": _errors(grad.cpu().numpy()[sel], rg, floor=tau + 1e5 * (sl * 1e4)[:, None]),
                "kappa_over_50_frac": float(np.mean(kap > 50)), "at": "final iterate of the 20 GPU steps, 1000 pairs"}
        res["registration_%s_full_cov_20_steps" % fn] = rec
    register(cl, cen, p0, steps=1, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pf = register(cl, cen, p0, steps=20, ctx=ctx)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern = ctx.stats()["kernel_ns"] * 1e-9
    peak_g = VALU_LANE_OPS / 14.0  # 8 VALU + 2 hi/lo adds + exp (4 slots) per term
    res["overlap_grad_20_steps"] = {"workload": "same clouds, adjoint of (theta, tx, ty), 20 GD steps",
                                    "pair_steps_per_s": 20 * P / dt, "kernel_ms": kern * 1e3,
                                    "roofline": {"bound": "alu", "achieved": terms / kern, "peak": peak_g,
                                                 "unit": "terms/s", "frac": terms / kern / peak_g}}
    if with_cpu:
        # cost and adjoint at the GPU's final iterate, 4096 sampled pairs, against the oracle
        import oracle
        cost, grad = ctx.overlap_cost_grad(cl, cen, pf.contiguous())
        g = np.random.default_rng(9)
        idx = np.sort(g.choice(P, 4096, replace=False))
        iu = np.triu_indices(2048, 1)
        pi, pj = iu[0][idx].astype(np.int64), iu[1][idx].astype(np.int64)
        prm = pf.cpu().numpy()[idx].astype(np.float64)
        t0 = time.perf_counter()
        rc, rg, tau, kap = oracle.overlap_grad(off, xy, cen.cpu().numpy(), pi, pj, prm, 0.02)
        dto = time.perf_counter() - t0
        nn = cnt[pi] * cnt[pj]
        gc = cost.cpu().numpy()[idx]
        gg = grad.cpu().numpy()[idx]
        res["overlap_grad_20_steps"]["errors"] = {
            "cost": _errors(gc, rc, scale=rc * np.maximum(1, kap / 50) + 1e5 * nn * 2.0 ** -126),
            "grad": _errors(gg, rg, floor=tau + 1e5 * (nn * 2.0 ** -126 * 2500.0)[:, None]),
            "kappa_over_50_frac": float(np.mean(kap > 50)), "at": "final iterate of the 20 GPU steps"}
        res["overlap_grad_20_steps"]["cpu_baseline"] = dict(
            {"value": pi.size / dto, "unit": "pair-evaluations/s", "cores": oracle.num_threads(), "kind": "oracle",
             "sample": "cost + gradient of 4096 random pairs at one parameter set"}, **_host_info())
    return res


def sparse_pair_fn(ctx, with_cpu=True, autotune=True):
    """Sparse cosine over 8192 composition-vector-like items (about 1.56e9 entries)."""
    import numpy as np
    import torch
    from paper_2009_04755_amd import SparseSet, synth

    off, keys, vals = synth.sparse_vectors_device(8192, seed=0, device="cuda")
    S = SparseSet(off, keys, vals)
    n = 8192
    P = n * (n - 1) // 2
    out = torch.empty(P, device="cuda")
    ctx.prepare(S, "sparse_cosine")
    tune = ctx.autotune() if autotune else None  # untimed setup: lanes x chunk width
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.compare(out=out)
    kern = ctx.stats()["kernel_ns"] * 1e-9
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # streamed bytes: every (16-item band, CB-item column block) work item reads the u32 keys
    # and f32 values of its 16 rows and CB columns once; CB = 1024 / (lanes per column)
    cb = 1024 // ctx.stats()["variant"]
    nnz = np.sort(np.diff(off.cpu().numpy()))[::-1].astype(np.float64)
    band = np.add.reduceat(nnz, np.arange(0, n, 16))
    blk = np.add.reduceat(nnz, np.arange(0, n, cb))
    byts = 0.0
    for b in range(band.size):
        for c in range(blk.size):
            if b * 16 < min(n, (c + 1) * cb) - 1:
                byts += 8.0 * (band[b] + blk[c])
    # the reference model: a row tile of T = 16 items per band, columns streamed once per
    # band, (n / 2T) * 8 * sum(nnz) bytes
    ref_bytes = n / (2 * 16) * 8.0 * nnz.sum()
    res = {"workload": "8192 sparse vectors over 20^6 keys, lognormal nnz (mean 2e5), Zipf(1.1) keys",
           "entries": int(nnz.sum()), "pairs_per_s": P / dt, "kernel_ms": kern * 1e3,
           "roofline": {"bound": "hbm", "achieved": ref_bytes / kern / 1e9, "peak": PEAK_HBM, "unit": "GB/s",
                        "frac": ref_bytes / kern / 1e9 / PEAK_HBM, "algorithmic_bytes_per_launch": ref_bytes,
                        "model": "(n / 2T) * 8 * sum(nnz), T = 16 rows per band",
                        "streaming_model_bytes": byts, "streaming_model_frac": byts / kern / 1e9 / PEAK_HBM}}
    if tune is not None:
        res["autotune"] = dict(tune, candidates="lanes {4, 8} x micro-chunk width {automatic, twice that}")
    if with_cpu:
        import oracle
        m = 24  # all pairs among the first 24 items
        offh = off.cpu().numpy()
        e = int(offh[m])
        kh, vh = keys[:e].cpu().numpy(), vals[:e].cpu().numpy()
        pi, pj = oracle.all_pairs(m)
        t0 = time.perf_counter()
        ref, rcnt, _, tau = oracle.sparse_cosine(offh[: m + 1], kh, vh, pi, pj, with_tau=True)
        dto = time.perf_counter() - t0
        res["cpu_baseline"] = dict({"value": pi.size / dto, "unit": "pairs/s", "cores": oracle.num_threads(),
                                    "kind": "oracle", "sample": "all 276 pairs among the first 24 items"},
                                   **_host_info())
        # the first 24 items in the caller's order: their pairs' results
        idx = pi * n - pi * (pi + 1) // 2 + (pj - pi - 1)
        res["errors"] = _errors(out.cpu().numpy()[idx], ref, floor=tau)
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the FP32 and two-term split comparison runs")
    ap.add_argument("--no-autotune", action="store_true", help="skip the autotuner in the untimed setup")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM counter scaling)")
    ap.add_argument("--only", choices=["clouds", "sparse", "cv", "pce", "pce_big", "pce_camera", "ooc", "small",
                                             "valu", "forensics"],
                    help="run only this secondary workload (for profiling it) and print its record; "
                         "clouds = overlap, GMM L2 / Bhattacharya and the registration gradient; "
                         "small = the 256 x 4096 NCC workload; forensics = NCC of 1024 patterns of "
                         "3648 x 2736 values")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: there is no multi-GPU path (requested %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    _ensure_built()
    from paper_2009_04755_amd import Context, synth

    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    n, d = 4096, 1 << 20
    P = n * (n - 1) // 2
    if args.only and args.only != "ooc":
        ctx = Context(0)
        ctx.set(timing=1)
        cpu = not args.no_cpu_baseline
        tune = not args.no_autotune
        run = {"clouds": lambda: other_pair_fns(ctx, cpu, tune), "sparse": lambda: sparse_pair_fn(ctx, cpu, tune),
               "cv": lambda: cv_pipeline(ctx, cpu), "pce": lambda: pce_pair_fn(ctx, cpu),
               "pce_big": lambda: pce_big_pair_fn(ctx, cpu), "valu": valu_probe,
               "pce_camera": lambda: pce_big_pair_fn(ctx, cpu, n=32, H=3648, W=2736, nsrc=4, sample=16),
               "small": lambda: ncc_small(ctx, cpu), "forensics": lambda: forensics_ncc(ctx, cpu)}[args.only]
        print(json.dumps({"only": args.only, "record": run()}))
        sys.stdout.flush()
        return
    X, _ = synth.dense_patterns_device(n, d, 64, 0.02, seed=1, device="cuda")
    ctx = Context(0)
    ctx.set(timing=1)
    out = torch.empty(P, dtype=torch.float32, device="cuda")
    if args.only == "ooc":
        ctx.allpairs(X, "ncc_bf16x6", out=out)
        torch.cuda.synchronize()
        print(json.dumps({"only": args.only, "record": out_of_core(ctx, X, out)}))
        sys.stdout.flush()
        return

    # untimed setup: the autotuner picks the Gram tile shape for this set (cache in a
    # temporary file, so a second tuning call would reuse it)
    import tempfile
    tune_cache = os.path.join(tempfile.mkdtemp(prefix="rocket_tune_"), "tune.json")
    ctx.set_tune_cache(tune_cache)
    ctx.prepare(X, "ncc_bf16x6")
    tune = ctx.autotune() if not args.no_autotune else None
    dt, kern = _time_fn(ctx, X, "ncc_bf16x6", out, args.steps, args.warmup)
    st = ctx.stats()
    value = P * args.steps / dt
    flop = 2.0 * d * P
    achieved = flop / kern / 1e12
    # issued MFMA flops: 32x32 output blocks x 16-deep slices x 6 products; the 256-tile kernel
    # skips the 28 blocks below the diagonal of each of the n/256 diagonal tiles
    T = st["tile"]
    blocks = st["tiles"] * (T // 32) ** 2 - (28 * ((n + T - 1) // T) if T == 256 else 0)
    issued = 6 * 2.0 * 32 * 32 * ((d + 15) // 16 * 16) * blocks
    waves = ctx.get("ncc_waves") or 8
    # the committed counter file was taken with the default shape (256-item tiles, 8 waves, 2048 K chunks)
    traffic = _traffic_from_profile() if (T, waves, st["kchunk"]) == (256, 8, 2048) else None
    rec = {
        "metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic (seeded, generated on the device)",
        "config": {"workload": "NCC all pairs of 4096 patterns x 1,048,576 f32 values, BF16 3-way split "
                               "(6 bf16 MFMA products, FP32 accumulation)",
                   "n": n, "d": d, "pairs": P, "pair_fn": "ncc_bf16x6", "tile": st["tile"],
                   "kchunk": st["kchunk"], "work_items": st["work_items"], "grid": st["grid"]},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16, "traffic": traffic,
                     "kernel": "k_ncc_gram<%d, %d, bf16x6, %d waves>" % (T, T, waves), "kernel_ms": kern * 1e3,
                     "algorithmic_flop_per_launch": flop, "issued_mfma_flop_per_launch": issued,
                     "issued_frac": issued / kern / 1e12 / PEAK_BF16},
    }
    for fn, peak in (() if args.no_variants else (("ncc_fp32", PEAK_FP32_MFMA), ("ncc_bf16x3", PEAK_BF16))):
        dt2, kern2 = _time_fn(ctx, X, fn, out, 3, 1)
        rec[fn] = {"pairs_per_s": 3 * P / dt2, "ms_per_step": dt2 / 3 * 1e3, "kernel_ms": kern2 * 1e3,
                   "frac_of_own_peak": flop / kern2 / 1e12 / peak}
    if "ncc_fp32" in rec:
        rec["bf16x6_speedup_vs_fp32"] = value / rec["ncc_fp32"]["pairs_per_s"]
    # leave the BF16x6 result in `out` for the parity sample, from one untimed step with the
    # per-tile trace on (the queue's load balance)
    ctx.set(trace=1)
    ctx.allpairs(X, "ncc_bf16x6", out=out)
    torch.cuda.synchronize()
    rec["queue_trace"] = _trace_summary(ctx.trace(), ctx.stats()["grid"])
    ctx.set(trace=0)
    if tune is not None:
        rec["autotune"] = dict(tune, candidates="tile {256, 128} x waves {8, 4} x K chunk {2048, 1024}")
    if traffic is not None:
        # HBM bytes moved by one Gram launch over the bytes of the f32 data set
        rec["roofline"]["R_HBM"] = traffic / (4.0 * n * d)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"], rec["errors"] = cpu_baseline(X, out, n, T)
    if not args.no_extras:
        rec["ncc_small"] = ncc_small(ctx, not args.no_cpu_baseline)
        rec["ncc_out_of_core"] = out_of_core(ctx, X, out)
        del X
        torch.cuda.empty_cache()
        rec["ncc_forensics_size"] = forensics_ncc(ctx, not args.no_cpu_baseline)
        rec["valu_probe"] = valu_probe()
        rec["pair_fns"] = other_pair_fns(ctx, not args.no_cpu_baseline, not args.no_autotune)
        rec["pair_fns"]["sparse_cosine"] = sparse_pair_fn(ctx, not args.no_cpu_baseline, not args.no_autotune)
        rec["cv_build"] = cv_pipeline(ctx, not args.no_cpu_baseline)
        rec["pair_fns"]["pce"] = pce_pair_fn(ctx, not args.no_cpu_baseline)
        rec["pair_fns"]["pce_1024"] = pce_big_pair_fn(ctx, not args.no_cpu_baseline)
        # the image size of the forensics data set (Section V-A): both sides by Bluestein
        # (8192-point FFTs)
        rec["pair_fns"]["pce_3648x2736"] = pce_big_pair_fn(ctx, not args.no_cpu_baseline, n=32, H=3648, W=2736,
                                                           nsrc=4, sample=16)
    print(json.dumps(rec))
    sys.stdout.flush()


if __name__ == "__main__":
    main()
