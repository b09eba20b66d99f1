"""GPU parity of the sparse cosine against the FP64 oracle.

Intersection sizes must be bit-exact.  Cosines: |g - r| <= 1e-5 max(|r|, tau), tau the
oracle's error scale of the dot product; for the non-negative frequencies here tau <= r,
so this is the plain 1e-5 relative bar.  A pair with no shared key must give exactly 0.
"""
import numpy as np
import pytest

import oracle
from paper_2009_04755_amd import synth

from gpu_util import announce, device_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    device_or_skip()
    from paper_2009_04755_amd import Context
    return Context(0)


def _dev(off, keys, vals):
    import torch
    from paper_2009_04755_amd import SparseSet
    return SparseSet(torch.from_numpy(off).cuda(), torch.from_numpy(keys).cuda(), torch.from_numpy(vals).cuda())


def _check(got, cnt, off, keys, vals, pi, pj):
    ref, rcnt, _, tau = oracle.sparse_cosine(off, keys, vals, pi, pj, with_tau=True)
    assert np.array_equal(cnt.astype(np.int64), rcnt), np.nonzero(cnt != rcnt)[0][:5]
    zero = rcnt == 0
    nanref = np.isnan(ref)
    assert np.all(np.isnan(got[nanref]))
    ok = ~nanref
    assert np.all(got[ok & zero] == 0.0)
    # floored bar |g - r| <= 1e-5 max(|r|, tau): the plain relative bar for values of one
    # sign (tau <= |r| there), the dot product's error scale where signed values cancel
    err = np.abs(got[ok] - ref[ok]) / np.maximum(np.abs(ref[ok]), np.maximum(tau[ok], 1e-300))
    err[zero[ok]] = 0
    assert err.max() <= 1e-5, err.max()
    return err.max()


@pytest.mark.parametrize("n,nnz_mean,nnz_max,key_space", [
    (2, 50, 200, 1000), (17, 300, 2000, 5000), (40, 500, 3000, 20 ** 4), (130, 800, 5000, 20 ** 4),
    (300, 2000, 20000, 20 ** 6),
])
@pytest.mark.parametrize("lanes", [4, 8])
def test_all_pairs_small(ctx, n, nnz_mean, nnz_max, key_space, lanes):
    announce("sparse all pairs n=%d nnz~%d keys<%d lanes=%d" % (n, nnz_mean, key_space, lanes))
    off, keys, vals = synth.sparse_vectors(n, key_space=key_space, nnz_mean=nnz_mean, nnz_min=1, nnz_max=nnz_max,
                                           config=4, salt=n)
    ctx.set(queue_order=0, sp_lanes=lanes)
    got, cnt = ctx.allpairs(_dev(off, keys, vals), "sparse_cosine", counts=True)
    ctx.set(sp_lanes=0)
    pi, pj = oracle.all_pairs(n)
    _check(got.cpu().numpy(), cnt.cpu().numpy(), off, keys, vals, pi, pj)


def test_edge_items(ctx):
    announce("sparse edge items")
    items = [
        ([], []),                                    # empty: zero norm -> NaN
        ([0, 5, 9, 2 ** 32 - 2], [0.5, 0.25, 0.125, 2.0]),
        ([0, 5, 9, 2 ** 32 - 2], [0.5, 0.25, 0.125, 2.0]),  # duplicate: cos 1, count 4
        ([1, 6, 10], [1.0, 2.0, 3.0]),               # disjoint from the above
        ([5], [0.0]),                                # zero norm, but shares key 5
        ([9, 10, 11, 12, 13], [1.0, 1.0, 1.0, 1.0, 1.0]),
    ]
    off = np.zeros(len(items) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(k) for k, _ in items])
    keys = np.concatenate([np.asarray(k, dtype=np.int64) for k, _ in items])
    vals = np.concatenate([np.asarray(v, dtype=np.float32) for _, v in items])
    got, cnt = ctx.allpairs(_dev(off, keys, vals), "sparse_cosine", counts=True)
    got, cnt = got.cpu().numpy(), cnt.cpu().numpy()
    n = len(items)
    pi, pj = oracle.all_pairs(n)
    _check(got, cnt, off, keys, vals, pi, pj)
    from paper_2009_04755_amd import pair_index
    assert cnt[pair_index(1, 2, n)] == 4 and abs(got[pair_index(1, 2, n)] - 1.0) < 1e-6
    assert cnt[pair_index(1, 4, n)] == 1 and np.isnan(got[pair_index(1, 4, n)])


def test_workload_shaped_sampled_and_deterministic(ctx):
    # 600 items over 20^6 keys, lognormal nnz (mean 20,000, clipped to [2,000, 100,000]), Zipf(1.1)
    import torch
    announce("sparse n=600 workload-shaped sampled + determinism")
    off, keys, vals = synth.sparse_vectors(600, nnz_mean=20_000, nnz_min=2_000, nnz_max=100_000, config=4, salt=77)
    S = _dev(off, keys, vals)
    ctx.set(queue_order=0, ledger=1)
    a, ca = ctx.allpairs(S, "sparse_cosine", counts=True)
    assert np.all(ctx.ledger() == 1)
    ctx.set(queue_order=1, seed=5, ledger=0)
    b, cb = ctx.allpairs(S, "sparse_cosine", counts=True)
    ctx.set(queue_order=0, seed=0)
    assert torch.equal(a, b) and torch.equal(ca, cb)
    g = np.random.default_rng(1)
    i = g.integers(0, 600, 4000)
    j = g.integers(0, 600, 4000)
    pi, pj = np.minimum(i, j), np.maximum(i, j)
    keep = pi < pj
    pi, pj = pi[keep], pj[keep]
    idx = pi * 600 - pi * (pi + 1) // 2 + (pj - pi - 1)
    err = _check(a.cpu().numpy()[idx], ca.cpu().numpy()[idx], off, keys, vals, pi, pj)
    announce("max rel err %.2e" % err)


def test_lanes_and_chunk_width_options(ctx):
    # 4 or 8 lanes per column and a coarser micro-chunk grid change the work split and the
    # summation order, never the intersections
    import torch
    announce("sparse lanes 4/8 x chunk width auto/2^14")
    off, keys, vals = synth.sparse_vectors(300, nnz_mean=6_000, nnz_min=500, nnz_max=40_000, config=4, salt=21)
    S = _dev(off, keys, vals)
    pi, pj = oracle.all_pairs(300)
    sel = np.arange(0, pi.size, 7)
    counts = []
    for lanes in (4, 8):
        for width in (0, 1 << 14):
            ctx.set(sp_lanes=lanes, sp_chunk=width)
            got, cnt = ctx.allpairs(S, "sparse_cosine", counts=True)
            assert ctx.stats()["variant"] == lanes
            counts.append(cnt)
            _check(got.cpu().numpy()[sel], cnt.cpu().numpy()[sel], off, keys, vals, pi[sel], pj[sel])
    ctx.set(sp_lanes=0, sp_chunk=0)
    assert all(torch.equal(counts[0], c) for c in counts[1:])


def test_device_generator_is_reproducible_across_processes():
    # the seeded device generator gives the same bytes in a fresh process (its Zipf CDF is
    # a sequential host sum, so no parallel scan can move a draw)
    import subprocess
    import sys
    import torch
    device_or_skip()
    announce("sparse device generator: same bytes in a child process")
    code = ("import sys; sys.path.insert(0, %r); import torch; from paper_2009_04755_amd import synth; "
            "o, k, v = synth.sparse_vectors_device(48, nnz_mean=3000, nnz_min=500, nnz_max=20000, seed=3); "
            "print(synth.sha256(o.cpu().numpy(), k.cpu().numpy(), v.cpu().numpy()))")
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    child = subprocess.run([sys.executable, "-c", code % root], capture_output=True, text=True, timeout=300)
    assert child.returncode == 0, child.stderr[-2000:]
    o, k, v = synth.sparse_vectors_device(48, nnz_mean=3000, nnz_min=500, nnz_max=20000, seed=3)
    torch.cuda.synchronize()
    assert child.stdout.strip().splitlines()[-1] == synth.sha256(o.cpu().numpy(), k.cpu().numpy(), v.cpu().numpy())


def test_option_validation(ctx):
    from paper_2009_04755_amd._lib import RocketError, E_INVALID
    announce("sparse option validation")
    for name, bad in (("sp_lanes", 2), ("sp_lanes", 16), ("sp_chunk", 3), ("sp_chunk", 1000), ("sp_chunk", 1 << 32), ("sp_chunk", 1 << 40)):
        with pytest.raises(RocketError) as e:
            ctx.set(**{name: bad})
        assert e.value.status == E_INVALID


@pytest.mark.parametrize("lanes", [4, 8])
@pytest.mark.parametrize("base,span,n", [(3 << 30, 4096, 16), (2 ** 32 - 70000, 8192, 40), (1 << 31, 1500, 33)])
def test_dense_key_ranges(ctx, base, span, n, lanes):
    # keys near the top of the u32 range force wide micro-chunks (2^12 keys); every item
    # holds `span` consecutive keys from `base` (shifted by item, so blocks overlap partly)
    # plus random keys, so one micro-chunk holds far more than one chunk's capacity of a
    # band's entries and must be cut at 64-key granularity
    announce("sparse dense key ranges base=%d span=%d n=%d lanes=%d" % (base, span, n, lanes))
    g = np.random.default_rng(span + n)
    ks, vs = [], []
    for i in range(n):
        dense = base + 17 * i + np.arange(span, dtype=np.int64)
        extra = g.integers(0, 2 ** 32 - 1, g.integers(50, 400))
        k = np.unique(np.concatenate([dense, extra]))
        k = k[k < 2 ** 32 - 1]
        ks.append(k)
        vs.append((g.random(k.size) - 0.3).astype(np.float32))  # signed values
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum([k.size for k in ks])
    keys, vals = np.concatenate(ks), np.concatenate(vs)
    ctx.set(queue_order=0, sp_lanes=lanes)
    got, cnt = ctx.allpairs(_dev(off, keys, vals), "sparse_cosine", counts=True)
    st = ctx.stats()
    ctx.set(sp_lanes=0)
    pi, pj = oracle.all_pairs(n)
    _check(got.cpu().numpy(), cnt.cpu().numpy(), off, keys, vals, pi, pj)
    # the dense block alone needs several chunks per band
    assert st["kchunk"] >= (n + 15) // 16 * (16 * span // 1632)


def test_errors(ctx):
    from paper_2009_04755_amd._lib import RocketError, E_KEYRANGE, E_UNSORTED
    announce("sparse errors")
    off = np.array([0, 3, 5], dtype=np.int64)
    vals = np.ones(5, dtype=np.float32)
    with pytest.raises(RocketError) as e:
        ctx.allpairs(_dev(off, np.array([1, 3, 3, 0, 1], dtype=np.int64), vals), "sparse_cosine")
    assert e.value.status == E_UNSORTED
    with pytest.raises(RocketError) as e:
        ctx.allpairs(_dev(off, np.array([1, 3, 2 ** 32 - 1, 0, 1], dtype=np.int64), vals), "sparse_cosine")
    assert e.value.status == E_KEYRANGE
    with pytest.raises(RocketError) as e:
        ctx.allpairs(_dev(off, np.array([-1, 3, 4, 0, 1], dtype=np.int64), vals), "sparse_cosine")
    assert e.value.status == E_KEYRANGE


@pytest.mark.timeout(900)
def test_full_scale_sampled():
    """8192 items over 20^6 keys (lognormal nnz, mean 200,000, clipped to [20,000, 1,000,000];
    Zipf(1.1) keys; about 1.56e9 entries), all 33,550,336 pairs in one persistent launch;
    2,000 pairs among 150 sampled items against the FP64 oracle (exact counts, cosine
    within 1e-5)."""
    import torch
    device_or_skip()
    from paper_2009_04755_amd import Context, SparseSet
    announce("sparse full scale n=8192 (device generator), sampled parity")
    off, keys, vals = synth.sparse_vectors_device(8192, seed=0, device="cuda")
    S = SparseSet(off, keys, vals)
    ctx = Context(0)
    got, cnt = ctx.allpairs(S, "sparse_cosine", counts=True)
    torch.cuda.synchronize()
    g = np.random.default_rng(9)
    pool = g.choice(8192, 150, replace=False)  # keeps the host copy to ~350 MB
    i = pool[g.integers(0, 150, 2200)]
    j = pool[g.integers(0, 150, 2200)]
    pi, pj = np.minimum(i, j), np.maximum(i, j)
    keep = pi < pj
    pi, pj = pi[keep][:2000], pj[keep][:2000]
    need = np.unique(np.concatenate([pi, pj]))
    offh = off.cpu().numpy()
    # copy only the sampled items to the host
    parts_k, parts_v, sub_off = [], [], [0]
    for it in need:
        a, b = int(offh[it]), int(offh[it + 1])
        parts_k.append(keys[a:b].cpu().numpy())
        parts_v.append(vals[a:b].cpu().numpy())
        sub_off.append(sub_off[-1] + (b - a))
    remap = {int(r): k for k, r in enumerate(need)}
    sk, sv, so = np.concatenate(parts_k), np.concatenate(parts_v), np.array(sub_off, dtype=np.int64)
    idx = torch.from_numpy(pi * 8192 - pi * (pi + 1) // 2 + (pj - pi - 1)).cuda()
    gv = got[idx].cpu().numpy()
    gc = cnt[idx].cpu().numpy()
    err = _check(gv, gc, so, sk, sv, np.array([remap[int(v)] for v in pi]), np.array([remap[int(v)] for v in pj]))
    announce("max rel err %.2e, mean count %.0f" % (err, gc.mean()))
    ctx.close()


def test_without_counts_same_cosines():
    # the counts are optional: without them the kernel skips the presence sums only, so the
    # cosines are identical bit for bit
    import torch
    from paper_2009_04755_amd import Context, SparseSet
    device_or_skip()
    announce("sparse cosine with and without counts, n=300")
    off, keys, vals = synth.sparse_vectors(300, key_space=20 ** 6, nnz_mean=3000, nnz_min=300, nnz_max=20000,
                                           config=4, salt=41)
    S = SparseSet(torch.from_numpy(off).cuda(), torch.from_numpy(keys).cuda(), torch.from_numpy(vals).cuda())
    for lanes in (4, 8):
        c = Context(0).set(sp_lanes=lanes)
        with_counts, cnt = c.allpairs(S, "sparse_cosine", counts=True)
        without = c.allpairs(S, "sparse_cosine")
        assert torch.equal(with_counts, without), lanes
        c.close()
