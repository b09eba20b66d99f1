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
out-of-core device cache, the Gaussian-overlap, GMM and registration-gradient costs over
2048 point clouds, the sparse cosine of 8192 k-mer vectors, the PCE of 1024 images and the
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
COUNTERS_FILE = os.path.join(ROOT, "profiles", "ncc_gram_bf16x6_4096x1048576_counters.txt")


def _src_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2009_04755_amd", "csrc", n), "rb") as f:
            h.update(f.read())
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


def cpu_baseline(X, out, n, budget_s=15.0):
    """FP64 oracle on pairs among the first rows of the workload; also a parity sample."""
    import numpy as np
    import oracle

    rows = 24
    Xh = X[:rows].cpu().numpy()
    pi, pj = oracle.all_pairs(rows)
    t0 = time.perf_counter()
    oracle.ncc(Xh, pi[:8], pj[:8])
    est = (time.perf_counter() - t0) / 8
    m = int(max(8, min(pi.size, budget_s / max(est, 1e-6))))
    reps = 1
    while m * reps * est < budget_s * 0.5 and reps < 8:
        reps += 1
    t0 = time.perf_counter()
    for _ in range(reps):
        rho, tau = oracle.ncc(Xh, pi[:m], pj[:m])
    dt = time.perf_counter() - t0
    idx = pi[:m] * n - pi[:m] * (pi[:m] + 1) // 2 + (pj[:m] - pi[:m] - 1)
    got = out.cpu().numpy()[idx]
    err = np.abs(got - rho) / np.maximum(np.abs(rho), tau)
    return ({"value": m * reps / dt, "unit": "pairs/s", "cores": oracle.num_threads(), "kind": "oracle",
             "sample": "%d pairs among the first %d of the 4096 patterns (1,048,576 values each), %d pass(es); "
                       "FP64 stats + pair loop, data already in host memory" % (m, rows, reps)},
            {"pairs": int(m), "max_floored_rel_err": float(err.max())})


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
    if with_cpu:
        import oracle.cv as ocv
        t0 = time.perf_counter()
        for s in range(2):
            ocv.composition_vector(res[off[s]:off[s + 1]], K)
        dto = time.perf_counter() - t0
        res_["cpu_baseline"] = {"value": 2 / dto, "unit": "species/s", "cores": 1, "kind": "oracle",
                                "sample": "2 of the 128 proteomes (numpy, one thread)"}
    out = torch.empty(n * (n - 1) // 2, device="cuda")
    ctx.allpairs(S, "sparse_cosine", out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.allpairs(S, "sparse_cosine", out=out)
    torch.cuda.synchronize()
    res_["cosine_all_pairs"] = {"pairs": n * (n - 1) // 2, "ms": (time.perf_counter() - t0) * 1e3}
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
        import oracle.pce as opce
        g = np.random.default_rng(8)
        t0 = time.perf_counter()
        m = 0
        while time.perf_counter() - t0 < 5.0:
            i, j = sorted(g.choice(n, 2, replace=False))
            opce.pce(X[i].reshape(L, L), X[j].reshape(L, L))
            m += 1
        dto = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": m / dto, "unit": "pairs/s", "cores": 1, "kind": "oracle",
                               "sample": "%d random pairs (numpy FFT, FP64)" % m}
    return res


def other_pair_fns(ctx, with_cpu=True):
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
    dt, kern = _time_fn(ctx, cl, "gauss_overlap", out, 5, 1)
    cnt = np.diff(off).astype(np.float64)
    terms = (cnt.sum() ** 2 - (cnt ** 2).sum()) / 2
    # per term: 2 sub, mul, fma, mul, add (VALU) + exp (transcendental, counted as 4 slots)
    peak_terms = VALU_LANE_OPS / 10.0
    res["gauss_overlap"] = {"workload": "2048 clouds, 50..400 points, sigma 0.02", "pairs_per_s": 5 * P / dt,
                            "kernel_ms": kern * 1e3, "terms_per_s": terms / kern,
                            "roofline": {"bound": "alu", "achieved": terms / kern, "peak": peak_terms,
                                         "unit": "terms/s", "frac": terms / kern / peak_terms}}
    if with_cpu:
        import oracle
        g = np.random.default_rng(5)
        pi = g.integers(0, 2047, 3000)
        pj = np.minimum(2047, pi + 1 + g.integers(0, 2047, 3000) % (2047 - pi))
        t0 = time.perf_counter()
        oracle.overlap(off, xy, pi, pj, 0.02)
        dto = time.perf_counter() - t0
        res["gauss_overlap"]["cpu_baseline"] = {"value": pi.size / dto, "unit": "pairs/s", "cores": oracle.num_threads(),
                                                "kind": "oracle", "sample": "3000 random pairs of the 2048 clouds"}
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
            oracle.gmm(off, xy, sig, pi, pj, mode)
            dto = time.perf_counter() - t0
            res[fn]["cpu_baseline"] = {"value": pi.size / dto, "unit": "pairs/s", "cores": oracle.num_threads(),
                                       "kind": "oracle", "sample": "2000 random pairs of the 2048 clouds"}
    cen = torch.from_numpy(synth.cloud_centroids(off, xy)).cuda()
    p0 = torch.from_numpy(synth.rigid_starts(P, config=3)).cuda()
    register(cl, cen, p0, steps=1, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    register(cl, cen, p0, steps=20, ctx=ctx)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern = ctx.stats()["kernel_ns"] * 1e-9
    peak_g = VALU_LANE_OPS / 14.0  # 8 VALU + 2 hi/lo adds + exp (4 slots) per term
    res["overlap_grad_20_steps"] = {"workload": "same clouds, adjoint of (theta, tx, ty), 20 GD steps",
                                    "pair_steps_per_s": 20 * P / dt, "kernel_ms": kern * 1e3,
                                    "roofline": {"bound": "alu", "achieved": terms / kern, "peak": peak_g,
                                                 "unit": "terms/s", "frac": terms / kern / peak_g}}
    return res


def sparse_pair_fn(ctx, with_cpu=True):
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
    res = {"workload": "8192 sparse vectors over 20^6 keys, lognormal nnz (mean 2e5), Zipf(1.1) keys",
           "entries": int(nnz.sum()), "pairs_per_s": P / dt, "kernel_ms": kern * 1e3,
           "roofline": {"bound": "hbm", "achieved": byts / kern / 1e9, "peak": PEAK_HBM, "unit": "GB/s",
                        "frac": byts / kern / 1e9 / PEAK_HBM, "algorithmic_bytes_per_launch": byts}}
    if with_cpu:
        import oracle
        m = 24  # all pairs among the first 24 items
        offh = off.cpu().numpy()
        e = int(offh[m])
        kh, vh = keys[:e].cpu().numpy(), vals[:e].cpu().numpy()
        pi, pj = oracle.all_pairs(m)
        t0 = time.perf_counter()
        oracle.sparse_cosine(offh[: m + 1], kh, vh, pi, pj)
        dto = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": pi.size / dto, "unit": "pairs/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": "all 276 pairs among the first 24 items"}
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the FP32 and two-term split comparison runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM counter scaling)")
    ap.add_argument("--only", choices=["clouds", "sparse", "cv", "pce", "ooc"],
                    help="run only this secondary workload (for profiling it) and print its record; "
                         "clouds = overlap, GMM L2 / Bhattacharya and the registration gradient")
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
        run = {"clouds": lambda: other_pair_fns(ctx, cpu), "sparse": lambda: sparse_pair_fn(ctx, cpu),
               "cv": lambda: cv_pipeline(ctx, cpu), "pce": lambda: pce_pair_fn(ctx, cpu)}[args.only]
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
    traffic = _traffic_from_profile()
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
                     "kernel": "k_ncc_gram<256, 256, bf16x6, 8 waves>", "kernel_ms": kern * 1e3,
                     "algorithmic_flop_per_launch": flop, "issued_mfma_flop_per_launch": issued,
                     "issued_frac": issued / kern / 1e12 / PEAK_BF16},
    }
    for fn, peak in (() if args.no_variants else (("ncc_fp32", PEAK_FP32_MFMA), ("ncc_bf16x3", PEAK_BF16))):
        dt2, kern2 = _time_fn(ctx, X, fn, out, 3, 1)
        rec[fn] = {"pairs_per_s": 3 * P / dt2, "ms_per_step": dt2 / 3 * 1e3, "kernel_ms": kern2 * 1e3,
                   "frac_of_own_peak": flop / kern2 / 1e12 / peak}
    if "ncc_fp32" in rec:
        rec["bf16x6_speedup_vs_fp32"] = value / rec["ncc_fp32"]["pairs_per_s"]
    # leave the BF16x6 result in `out` for the parity sample
    ctx.allpairs(X, "ncc_bf16x6", out=out)
    torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        rec["cpu_baseline"], rec["parity_sample"] = cpu_baseline(X, out, n)
    if not args.no_extras:
        rec["ncc_out_of_core"] = out_of_core(ctx, X, out)
        del X
        torch.cuda.empty_cache()
        rec["pair_fns"] = other_pair_fns(ctx, not args.no_cpu_baseline)
        rec["pair_fns"]["sparse_cosine"] = sparse_pair_fn(ctx, not args.no_cpu_baseline)
        rec["cv_build"] = cv_pipeline(ctx, not args.no_cpu_baseline)
        rec["pair_fns"]["pce"] = pce_pair_fn(ctx, not args.no_cpu_baseline)
    print(json.dumps(rec))
    sys.stdout.flush()


if __name__ == "__main__":
    main()
