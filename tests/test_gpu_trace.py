"""Per-tile trace (ROCKET_OPT_TRACE, the timeline of Section IV-C's profiling): every work
item ran once, in one workgroup of the persistent grid, the items of a workgroup do not
overlap in time, and tracing leaves the output bit for bit unchanged."""
import numpy as np
import pytest

from paper_2009_04755_amd import synth

from gpu_util import announce, device_or_skip

pytestmark = pytest.mark.gpu


def _ctx(**opts):
    device_or_skip()
    from paper_2009_04755_amd import Context
    return Context(0).set(**opts)


def _check(tr, grid):
    assert tr.size > 0
    assert np.all(tr["workgroup"] >= 0) and np.all(tr["workgroup"] < grid)
    assert np.all(tr["start_ns"] >= 0) and np.all(tr["end_ns"] >= tr["start_ns"])
    assert tr["start_ns"].min() == 0
    for w in np.unique(tr["workgroup"]):
        t = np.sort(tr[tr["workgroup"] == w], order="start_ns")
        assert np.all(t["end_ns"][:-1] <= t["start_ns"][1:]), w  # one item at a time


def _run(x, fn, counts=False, **opts):
    ref_ctx = _ctx(**opts)
    ref = ref_ctx.allpairs(x, fn, counts=counts)
    ref_ctx.close()
    c = _ctx(trace=1, **opts)
    got = c.allpairs(x, fn, counts=counts)
    tr, grid = c.trace(), c.stats()["grid"]
    c.close()
    return ref, got, tr, grid


def test_ncc_trace():
    import torch
    announce("trace ncc_bf16x6 n=700 d=5000")
    X, _ = synth.dense_patterns(700, 5000, 8, 0.05, config=0, salt=31)
    ref, got, tr, grid = _run(torch.from_numpy(X).cuda(), "ncc_bf16x6")
    assert torch.equal(ref, got)
    _check(tr, grid)
    # every (tile, chunk) of the plan appears once
    keys = set(zip(tr["tile_i"].tolist(), tr["tile_j"].tolist(), tr["chunk"].tolist()))
    assert len(keys) == tr.size


def test_ncc_batched_trace():
    # a workspace cap splits the Gram launches into batches of leaf tiles: one record per
    # item across all batches
    import torch
    announce("trace ncc batched n=700 d=5000")
    X, _ = synth.dense_patterns(700, 5000, 8, 0.05, config=0, salt=32)
    Xd = torch.from_numpy(X).cuda()
    c0 = _ctx()
    ref = c0.allpairs(Xd, "ncc_bf16x6")
    c0.close()
    c = _ctx(trace=1)
    c.prepare(Xd, "ncc_bf16x6")
    st = c.stats()
    T, nchunks = st["tile"], st["work_items"] // st["tiles"]
    # room for what prepare allocated, the 4 MiB margin and two tiles' partials per launch
    c.set(workspace_cap=st["workspace_bytes"] + (4 << 20) + 2 * nchunks * T * T * 4 + (2 << 20) - 1)
    got = c.compare()
    tr = c.trace()
    c.close()
    assert torch.equal(ref, got)
    assert tr.size == st["work_items"]
    assert np.all(tr["workgroup"] >= 0) and np.all(tr["end_ns"] >= tr["start_ns"])
    keys = set(zip(tr["tile_i"].tolist(), tr["tile_j"].tolist(), tr["chunk"].tolist()))
    assert len(keys) == tr.size


def test_overlap_sparse_pce_traces():
    import torch
    from paper_2009_04755_amd import Clouds, SparseSet
    announce("trace overlap / sparse / pce")
    off, xy = synth.point_clouds(300, config=2, salt=33)
    cl = Clouds(torch.from_numpy(off).cuda(), torch.from_numpy(xy).cuda(), 0.02)
    ref, got, tr, grid = _run(cl, "gauss_overlap")
    assert torch.equal(ref, got)
    _check(tr, grid)
    off, keys, vals = synth.sparse_vectors(150, key_space=20 ** 6, nnz_mean=2000, nnz_min=200, nnz_max=8000,
                                           config=4, salt=34)
    S = SparseSet(torch.from_numpy(off).cuda(), torch.from_numpy(keys).cuda(), torch.from_numpy(vals).cuda())
    ref, got, tr, grid = _run(S, "sparse_cosine", counts=True)
    assert torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])
    _check(tr, grid)
    X, _, _ = synth.noise_images(40, 32, nsrc=3, amp=0.4, config=6, salt=35)
    ref, got, tr, grid = _run(torch.from_numpy(X).cuda(), "pce")
    assert torch.equal(ref, got)
    _check(tr, grid)


def test_no_trace_without_a_queue():
    import torch
    from paper_2009_04755_amd._lib import RocketError, E_STATE
    announce("trace staged pce")
    X, _, _ = synth.noise_images(4, (16, 64), nsrc=2, amp=0.4, config=6, salt=36)
    c = _ctx(trace=1, pce_width=64)
    c.allpairs(torch.from_numpy(X).cuda(), "pce")
    with pytest.raises(RocketError) as e:
        c.trace()
    assert e.value.status == E_STATE
    c.close()
