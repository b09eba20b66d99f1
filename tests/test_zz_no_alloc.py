"""The allocation-free entry point (rocket_allpairs_noalloc) against rocket_allpairs_ex.

Both run the same kernels; the allocation-free one takes its workspace from the library's
static per-device scratch array.  Each case makes two calls in a row, the second with a
smaller input, so the second call runs on scratch that still holds the first call's data.
Outputs must equal those of rocket_allpairs_ex (default options, fresh context) bit for
bit, and the dense and sparse cases are also held to the oracle's bar.  A problem whose
workspace exceeds the scratch array must be refused without touching the output.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2009_04755_amd import synth

from gpu_util import announce, device_or_skip

pytestmark = pytest.mark.gpu


def _call_ex(fn, x, with_counts=False):
    """Reference: rocket_allpairs_ex on a fresh context with default options."""
    import torch
    from paper_2009_04755_amd import Context, _lib, api
    code = _lib.FN_BY_NAME[fn]
    ctx = Context(0)
    it, n = ctx._items(x, code)
    P = n * (n - 1) // 2
    out = torch.full((P,), -7.0, device="cuda")
    cnt = torch.full((P,), -7, dtype=torch.int32, device="cuda") if with_counts else None
    _lib.check(_lib.load().rocket_allpairs_ex(ctx.handle, ctypes.byref(it), n, code, api._ptr(out), api._ptr(cnt),
                                              api._stream()), ctx.handle)
    torch.cuda.synchronize()
    ctx.close()
    return out.cpu().numpy(), (cnt.cpu().numpy() if with_counts else None)


def _call_noalloc(fn, x, with_counts=False):
    """rocket_allpairs_noalloc through the C ABI (outputs allocated here, by the caller)."""
    import torch
    from paper_2009_04755_amd import _lib, api
    code = _lib.FN_BY_NAME[fn]
    it, n = api._items_struct(x, code, 0)
    P = n * (n - 1) // 2
    out = torch.full((P,), -9.0, device="cuda")
    cnt = torch.full((P,), -9, dtype=torch.int32, device="cuda") if with_counts else None
    st = _lib.load().rocket_allpairs_noalloc(ctypes.byref(it), n, code, api._ptr(out), api._ptr(cnt), api._stream())
    _lib.check(st)
    torch.cuda.synchronize()
    return out.cpu().numpy(), (cnt.cpu().numpy() if with_counts else None)


@pytest.mark.parametrize("fn", ["ncc_bf16x6", "ncc_fp32"])
def test_ncc_two_calls(fn):
    import torch
    device_or_skip()
    for n, d in ((200, 3000), (70, 1000)):
        announce("noalloc %s n=%d d=%d" % (fn, n, d))
        X, _ = synth.dense_patterns(n, d, 8, 0.05, config=0, salt=n + d)
        Xd = torch.from_numpy(X).cuda()
        got, _ = _call_noalloc(fn, Xd)
        ref, _ = _call_ex(fn, Xd)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
        pi, pj = oracle.all_pairs(n)
        rho, tau = oracle.ncc(X, pi, pj)
        assert np.max(np.abs(got - rho) / np.maximum(np.abs(rho), tau)) <= 1e-5


def test_overlap_two_calls():
    import torch
    device_or_skip()
    from paper_2009_04755_amd import Clouds
    for n in (300, 60):
        announce("noalloc gauss_overlap n=%d" % n)
        off, xy = synth.point_clouds(n, nmin=20, nmax=200, config=2, salt=n)
        cl = Clouds(torch.from_numpy(off).cuda(), torch.from_numpy(xy).cuda(), 0.02)
        got, _ = _call_noalloc("gauss_overlap", cl)
        ref, _ = _call_ex("gauss_overlap", cl)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
        pi, pj = oracle.all_pairs(n)
        r, kap = oracle.overlap(off, xy, pi, pj, 0.02)
        nn = np.diff(off)[pi] * np.diff(off)[pj]
        assert np.all(np.abs(got - r) <= 1e-5 * r * np.maximum(1, kap / 50) + nn * 2.0 ** -126)


def test_sparse_two_calls():
    import torch
    device_or_skip()
    from paper_2009_04755_amd import SparseSet
    for n in (40, 12):
        announce("noalloc sparse_cosine n=%d" % n)
        off, keys, vals = synth.sparse_vectors(n, key_space=20 ** 4, nnz_mean=600, nnz_min=5, nnz_max=4000, salt=n)
        S = SparseSet(torch.from_numpy(off).cuda(), torch.from_numpy(keys).cuda(), torch.from_numpy(vals).cuda())
        got, cnt = _call_noalloc("sparse_cosine", S, with_counts=True)
        ref, rcnt = _call_ex("sparse_cosine", S, with_counts=True)
        assert np.array_equal(cnt, rcnt)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
        pi, pj = oracle.all_pairs(n)
        oc, ocnt, _ = oracle.sparse_cosine(off, keys, vals, pi, pj)
        assert np.array_equal(cnt.astype(np.int64), ocnt)
        assert np.all(np.abs(got - oc) <= 1e-5 * np.abs(oc))


def test_gmm_and_pce_two_calls():
    import torch
    device_or_skip()
    from paper_2009_04755_amd import Clouds
    for n in (120, 30):
        announce("noalloc gmm_l2 n=%d" % n)
        off, xy = synth.point_clouds(n, nmin=10, nmax=150, config=2, salt=n + 1)
        sig = synth.point_sigmas(off, salt=n)
        cl = Clouds(torch.from_numpy(off).cuda(), torch.from_numpy(xy).cuda(), 0.02, torch.from_numpy(sig).cuda())
        got, _ = _call_noalloc("gmm_l2", cl)
        ref, _ = _call_ex("gmm_l2", cl)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    # 256 x 256 takes the staged path: at n = 40 its transforms run in batches bounded by
    # what is left of the scratch array (the reference runs them in one batch); 96 x 96, 48 x 48
    # and 45 x 45 (odd sides) take it with Bluestein transforms
    for n, L in ((40, 64), (12, 32), (40, 256), (12, 256), (20, 96), (8, 48), (6, 45)):
        announce("noalloc pce n=%d L=%d" % (n, L))
        X, _, _ = synth.noise_images(n, L, nsrc=4, amp=0.4, salt=n)
        Xd = torch.from_numpy(X).cuda()
        got, pk = _call_noalloc("pce", Xd, with_counts=True)
        ref, rpk = _call_ex("pce", Xd, with_counts=True)
        assert np.array_equal(pk, rpk)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_too_large_is_refused():
    import torch
    device_or_skip()
    from paper_2009_04755_amd import _lib, allpairs_noalloc
    announce("noalloc refusal: 2048 x 8192 NCC needs more than the scratch array")
    n, d = 2048, 8192  # bf16x6 planes alone: 2048 * 8192 * 6 bytes = 96 MiB > 64 MiB
    X = torch.randn(n, d, device="cuda")
    out = torch.full((n * (n - 1) // 2,), 3.0, device="cuda")
    with pytest.raises(_lib.RocketError) as e:
        allpairs_noalloc(X, "ncc_bf16x6", out)
    assert e.value.status == _lib.E_OOM and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out == 3.0).all())
    # the entry point stays usable after a refusal
    X, _ = synth.dense_patterns(50, 500, 4, 0.1, config=0, salt=3)
    Xd = torch.from_numpy(X).cuda()
    got = allpairs_noalloc(Xd, "ncc_bf16x6", torch.empty(50 * 49 // 2, device="cuda")).cpu().numpy()
    ref, _ = _call_ex("ncc_bf16x6", Xd)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
