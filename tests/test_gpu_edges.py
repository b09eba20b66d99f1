"""Empty and single-item sets for every pair function, and the default-context entry point."""
import numpy as np
import pytest

import oracle
from paper_2009_04755_amd import synth

from gpu_util import announce, device_or_skip

pytestmark = pytest.mark.gpu


def _sets(n):
    import torch
    from paper_2009_04755_amd import Clouds, SparseSet
    dense = torch.zeros((n, 1024), device="cuda") + torch.arange(1024, device="cuda").float()
    off = torch.arange(n + 1, dtype=torch.int64, device="cuda") * 3
    xy = torch.rand(int(off[-1]) * 2, device="cuda")
    clouds = Clouds(off, xy, 0.02, torch.full((int(off[-1]),), 0.02, device="cuda"))
    keys = torch.arange(int(off[-1]), dtype=torch.int64, device="cuda")
    sp = SparseSet(off, keys, torch.ones(int(off[-1]), device="cuda"))
    return {"ncc_fp32": dense, "ncc_bf16x3": dense, "ncc_bf16x6": dense, "pce": dense, "gauss_overlap": clouds,
            "gmm_l2": clouds, "gmm_bhattacharya": clouds, "sparse_cosine": sp}


@pytest.mark.parametrize("n", [0, 1])
def test_no_pairs(n):
    device_or_skip()
    from paper_2009_04755_amd import Context
    announce("edges n=%d" % n)
    ctx = Context(0)
    for fn, x in _sets(n).items():
        out = ctx.allpairs(x, fn)
        assert out.numel() == 0, fn
    ctx.close()


def test_default_context_entry_point():
    import torch
    device_or_skip()
    from paper_2009_04755_amd import SparseSet, allpairs
    announce("default context allpairs")
    X, _ = synth.dense_patterns(40, 777, 4, 0.1, config=0, salt=5)
    got = allpairs(torch.from_numpy(X).cuda(), "ncc_bf16x6").cpu().numpy()
    pi, pj = oracle.all_pairs(40)
    rho, tau = oracle.ncc(X, pi, pj)
    assert np.max(np.abs(got - rho) / np.maximum(np.abs(rho), tau)) <= 1e-5
    off, keys, vals = synth.sparse_vectors(12, key_space=5000, nnz_mean=200, nnz_min=5, nnz_max=900, salt=6)
    S = SparseSet(torch.from_numpy(off).cuda(), torch.from_numpy(keys).cuda(), torch.from_numpy(vals).cuda())
    got, cnt = allpairs(S, "sparse_cosine", counts=True)
    pi, pj = oracle.all_pairs(12)
    ref, rcnt, _ = oracle.sparse_cosine(off, keys, vals, pi, pj)
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64), rcnt)


def test_c_abi_allpairs_synchronous_call():
    # rocket_allpairs: default context on the current device, synchronises before returning
    import ctypes
    import torch
    device_or_skip()
    from paper_2009_04755_amd import _lib
    announce("rocket_allpairs C entry")
    X, _ = synth.dense_patterns(33, 500, 4, 0.1, config=0, salt=7)
    Xd = torch.from_numpy(X).cuda()
    out = torch.empty(33 * 32 // 2, device="cuda")
    it = _lib.Items()
    it.dense = Xd.data_ptr()
    it.dim = 500
    it.ld = 500
    st = _lib.load().rocket_allpairs(ctypes.byref(it), 33, _lib.NCC_FP32, ctypes.c_void_p(out.data_ptr()))
    assert st == _lib.OK
    pi, pj = oracle.all_pairs(33)
    rho, tau = oracle.ncc(X, pi, pj)
    assert np.max(np.abs(out.cpu().numpy() - rho) / np.maximum(np.abs(rho), tau)) <= 1e-5
