"""Out-of-core NCC (items in host memory, fixed-size device cache; Section IV-A).

The host path runs the in-core kernels on cache slots with the same chunking and summation
order, so its output must equal the in-core output bit for bit; the number of block loads
must equal the reference LRU simulation over the divide-and-conquer leaf order
(``oracle.plan.lru_loads``); sampled pairs are also checked against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
from oracle import plan
from paper_2009_04755_amd import synth

from gpu_util import announce, device_or_skip, floored_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    device_or_skip()
    from paper_2009_04755_amd import Context
    return Context(0)


def _pinned(X):
    import torch
    h = torch.empty(X.shape, dtype=torch.float32, pin_memory=True)
    h.copy_(torch.from_numpy(X))
    return h


def _blocks(n, T):
    return (n + T - 1) // T


@pytest.mark.parametrize("n,d,tile,kchunk,slots", [
    (700, 5000, 0, 0, 2), (700, 5000, 0, 0, 3), (700, 5000, 0, 0, 0), (300, 3001, 64, 256, 2),
    (300, 3001, 64, 256, 4), (130, 777, 128, 0, 2), (2, 33, 0, 0, 0),
])
@pytest.mark.parametrize("fn", ["ncc_fp32", "ncc_bf16x3", "ncc_bf16x6"])
def test_identical_to_in_core_and_lru_loads(ctx, n, d, tile, kchunk, slots, fn):
    import torch
    announce("ooc n=%d d=%d tile=%d kchunk=%d slots=%d %s" % (n, d, tile, kchunk, slots, fn))
    g = np.random.default_rng(n + d)
    X = (g.standard_normal((n, d)) * g.uniform(0.5, 2, (n, 1)) + g.uniform(-1, 1, (n, 1))).astype(np.float32)
    ctx.set(ncc_tile=tile, ncc_kchunk=kchunk, queue_order=0, ledger=0, cache_slots=slots)
    ref = ctx.allpairs(torch.from_numpy(X).cuda(), fn)
    got = ctx.allpairs_host(_pinned(X), fn)
    torch.cuda.synchronize()
    st = ctx.stats()
    T = st["tile"]
    nb = _blocks(n, T)
    S = min(slots or nb, nb)
    assert st["cache_slots"] == S
    assert st["cache_loads"] == plan.lru_loads(n, T, S)[0]
    assert torch.equal(got, ref), (got - ref).abs().max().item()
    sel = np.arange(0, n * (n - 1) // 2, 37)
    pi, pj = oracle.all_pairs(n)
    rho, tau = oracle.ncc(X, pi[sel], pj[sel])
    tol = 1e-4 if fn == "ncc_bf16x3" else 1e-5
    assert floored_rel(got.cpu().numpy()[sel], rho, tau).max() <= tol
    ctx.set(ncc_tile=0, ncc_kchunk=0, cache_slots=0)


def test_prepared_set_is_dropped_and_in_core_still_works(ctx):
    import torch
    from paper_2009_04755_amd._lib import RocketError, E_STATE
    announce("ooc then in-core on one context")
    g = np.random.default_rng(5)
    X = g.standard_normal((200, 1000)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    ctx.prepare(Xd, "ncc_bf16x6")
    ctx.set(cache_slots=2)
    a = ctx.allpairs_host(_pinned(X), "ncc_bf16x6")
    with pytest.raises(RocketError) as e:
        ctx.compare()
    assert e.value.status == E_STATE
    b = ctx.allpairs(Xd, "ncc_bf16x6")
    assert torch.equal(a, b)
    ctx.set(cache_slots=0)


def test_errors(ctx):
    import torch
    from paper_2009_04755_amd import _lib
    from paper_2009_04755_amd._lib import RocketError, E_INVALID, E_UNSUPPORTED
    announce("ooc errors")
    X = _pinned(np.ones((600, 64), dtype=np.float32))
    with pytest.raises(RocketError) as e:
        ctx.allpairs_host(X, "gauss_overlap")
    assert e.value.status == E_UNSUPPORTED
    ctx.set(cache_slots=1)
    with pytest.raises(RocketError) as e:
        ctx.allpairs_host(X, "ncc_fp32")
    assert e.value.status == E_INVALID
    ctx.set(cache_slots=0)
    L = _lib.load()
    out = torch.empty(10, device="cuda")
    st = L.rocket_allpairs_host(ctx.handle, X.data_ptr(), 5, 64, 32, 1, out.data_ptr(), None)  # ld < dim
    assert st == E_INVALID
    one = ctx.allpairs_host(_pinned(np.ones((1, 8), dtype=np.float32)), "ncc_fp32")
    assert one.numel() == 0


@pytest.mark.timeout(900)
def test_full_scale_host_resident():
    """4096 x 1,048,576 f32 (16 GiB) in pinned host memory, 8 device slots of 256 items
    (half the set): every one of the 8,386,560 outputs equals the in-core result."""
    import torch
    device_or_skip()
    from paper_2009_04755_amd import Context
    announce("ooc full scale 4096 x 2^20, 8 slots")
    X, _ = synth.dense_patterns_device(4096, 1 << 20, 64, 0.02, seed=1, device="cuda")
    c = Context(0)
    ref = c.allpairs(X, "ncc_bf16x6")
    torch.cuda.synchronize()
    Xh = torch.empty(X.shape, dtype=torch.float32, pin_memory=True)
    Xh.copy_(X)
    del X
    torch.cuda.empty_cache()
    c.set(cache_slots=8)
    got = c.allpairs_host(Xh, "ncc_bf16x6")
    torch.cuda.synchronize()
    st = c.stats()
    announce("loads %d (reference %d)" % (st["cache_loads"], plan.lru_loads(4096, 256, 8)[0]))
    assert st["cache_loads"] == plan.lru_loads(4096, 256, 8)[0]
    assert torch.equal(got, ref)
    c.close()
