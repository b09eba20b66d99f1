"""GPU parity of the NCC path (prepare + persistent Gram + epilogue) against the FP64 oracle.

Pass metric (FP32 and BF16X6): |g - r| <= 1e-5 * max(|r|, tau), tau the FP64 error scale
of the dot product of the two centred unit vectors.  BF16X3 (two-term split) is held
to 1e-4 only: dropping the h*l, l*h and m*m products leaves ~2^-17 per product.
"""
import numpy as np
import pytest

import oracle
from paper_2009_04755_amd import synth

from gpu_util import announce, device_or_skip, floored_rel

pytestmark = pytest.mark.gpu

TOL = {"ncc_fp32": 1e-5, "ncc_bf16x6": 1e-5, "ncc_bf16x3": 1e-4}


def _run(ctx, X, fn):
    import torch
    out = ctx.allpairs(torch.from_numpy(X).cuda(), fn)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.fixture(scope="module")
def ctx():
    device_or_skip()
    from paper_2009_04755_amd import Context
    return Context(0)


@pytest.mark.parametrize("fn", ["ncc_fp32", "ncc_bf16x3", "ncc_bf16x6"])
def test_small_workload_all_pairs(ctx, fn):
    # 256 items x 4096 values, 8 sources, amplitude 0.05: all 32,640 pairs
    announce("ncc all pairs n=256 d=4096 " + fn)
    X, _ = synth.dense_patterns(256, 4096, 8, 0.05, assign="mod", config=0)
    ctx.set(ncc_tile=0, ncc_kchunk=0, queue_order=0)
    got = _run(ctx, X, fn)
    pi, pj = oracle.all_pairs(256)
    rho, tau = oracle.ncc(X, pi, pj)
    err = floored_rel(got, rho, tau)
    assert np.all(np.isfinite(got))
    assert err.max() <= TOL[fn], (fn, err.max(), np.mean(err > 1e-5))


@pytest.mark.parametrize("n,d,tile,kchunk", [
    (2, 1, 64, 0), (3, 15, 64, 0), (17, 16, 64, 0), (65, 17, 64, 16), (130, 100, 128, 32), (300, 1000, 256, 256),
    (257, 513, 64, 64), (129, 4096, 128, 0),
])
@pytest.mark.parametrize("fn", ["ncc_fp32", "ncc_bf16x6"])
def test_ragged_shapes(ctx, n, d, tile, kchunk, fn):
    announce("ncc ragged n=%d d=%d tile=%d kchunk=%d %s" % (n, d, tile, kchunk, fn))
    g = np.random.default_rng(n * 1000 + d)
    X = (g.standard_normal((n, d)) * g.uniform(0.5, 3, (n, 1)) + g.uniform(-2, 2, (n, 1))).astype(np.float32)
    if d == 1:
        X[:, 0] = np.arange(n)  # one value per item: every item has zero variance
    ctx.set(ncc_tile=tile, ncc_kchunk=kchunk)
    got = _run(ctx, X, fn)
    pi, pj = oracle.all_pairs(n)
    rho, tau = oracle.ncc(X, pi, pj)
    if d == 1:
        assert np.all(np.isnan(got))
        return
    err = floored_rel(got, rho, tau)
    assert err.max() <= TOL[fn], err.max()
    st = ctx.stats()
    assert st["pairs"] == n * (n - 1) // 2 and st["tile"] == tile


def test_strided_rows_duplicates_and_constant_item(ctx):
    import torch
    announce("ncc strided/duplicate/constant")
    g = np.random.default_rng(3)
    base = g.standard_normal((40, 300)).astype(np.float32)
    base[7] = base[3] * 2.5 + 1.0  # affine copy: rho = 1
    base[11] = 4.0                 # constant item: NaN in all its pairs
    full = torch.zeros((40, 320), dtype=torch.float32)
    full[:, :300] = torch.from_numpy(base)
    x = full.cuda()[:, :300]       # ld = 320 > dim = 300
    ctx.set(ncc_tile=64, ncc_kchunk=0)
    got = ctx.allpairs(x, "ncc_bf16x6").cpu().numpy()
    from paper_2009_04755_amd import pair_index
    assert abs(got[pair_index(3, 7, 40)] - 1.0) < 1e-5
    bad = [pair_index(min(i, 11), max(i, 11), 40) for i in range(40) if i != 11]
    assert np.all(np.isnan(got[bad]))
    pi, pj = oracle.all_pairs(40)
    rho, tau = oracle.ncc(base, pi, pj)
    ok = ~np.isnan(rho)
    assert np.all(floored_rel(got[ok], rho[ok], tau[ok]) <= 1e-5)


def test_deterministic_across_queue_orders_and_exactly_once(ctx):
    import torch
    announce("ncc determinism + ledger")
    X, _ = synth.dense_patterns(300, 2048, 8, 0.05, config=0, salt=5)
    x = torch.from_numpy(X).cuda()
    ctx.set(ncc_tile=64, ncc_kchunk=256, ledger=1, queue_order=0)
    a = ctx.allpairs(x, "ncc_bf16x6").cpu().numpy()
    led = ctx.ledger()
    assert led.size == ctx.stats()["work_items"] and np.all(led == 1)
    b = ctx.allpairs(x, "ncc_bf16x6").cpu().numpy()
    ctx.set(queue_order=1, seed=1234)
    c = ctx.allpairs(x, "ncc_bf16x6").cpu().numpy()
    assert np.all(ctx.ledger() == 1)
    ctx.set(queue_order=2, grid=3)
    d = ctx.allpairs(x, "ncc_bf16x6").cpu().numpy()
    ctx.set(queue_order=0, ledger=0, seed=0, grid=0)
    assert a.tobytes() == b.tobytes() == c.tobytes() == d.tobytes()


def test_degenerate_and_errors(ctx):
    import torch
    from paper_2009_04755_amd._lib import RocketError, E_INVALID, E_STATE
    announce("ncc degenerate + errors")
    for n in (0, 1):
        out = ctx.allpairs(torch.zeros((n, 8), device="cuda"), "ncc_fp32")
        assert out.numel() == 0
    fresh = type(ctx)(0)
    with pytest.raises(RocketError) as e:
        fresh.compare()
    assert e.value.status == E_STATE
    with pytest.raises(RocketError) as e:
        fresh.set(ncc_tile=96)
    assert e.value.status == E_INVALID
    fresh.close()


@pytest.mark.timeout(900)
def test_full_scale_sampled():
    """4096 items x 1,048,576 values (16 GiB), the benchmark's launch configuration;
    all pairs among ~48 rows spanning several tiles plus ~2,000 pairs among 128 random rows."""
    import torch
    device_or_skip()
    from paper_2009_04755_amd import Context
    announce("ncc full scale n=4096 d=1048576 bf16x6 + fp32 (sampled)")
    n, d = 4096, 1 << 20
    X, _ = synth.dense_patterns_device(n, d, 64, 0.02, seed=1, device="cuda")
    ctx = Context(0)
    g = np.random.default_rng(7)
    rows = np.unique(np.concatenate([np.arange(0, 16), np.arange(250, 262), np.arange(4080, 4096),
                                     g.integers(0, n, 4)]))
    ii, jj = np.triu_indices(rows.size, 1)
    pool = g.choice(n, 128, replace=False)
    a = pool[g.integers(0, 128, 2000)]
    b = pool[g.integers(0, 128, 2000)]
    pi = np.concatenate([rows[ii], np.minimum(a, b)])
    pj = np.concatenate([rows[jj], np.maximum(a, b)])
    keep = pi < pj
    pi, pj = pi[keep], pj[keep]
    need = np.unique(np.concatenate([pi, pj]))
    Xh = X[torch.from_numpy(need).cuda()].cpu().numpy()
    remap = {int(r): k for k, r in enumerate(need)}
    rho, tau = oracle.ncc(Xh, np.array([remap[int(v)] for v in pi]), np.array([remap[int(v)] for v in pj]))
    idx = torch.from_numpy(pi * n - pi * (pi + 1) // 2 + (pj - pi - 1)).cuda()
    for fn in ("ncc_bf16x6", "ncc_fp32"):
        out = ctx.allpairs(X, fn)
        got = out[idx].cpu().numpy()
        err = floored_rel(got, rho, tau)
        announce("%s max floored rel err %.3e" % (fn, err.max()))
        assert err.max() <= 1e-5, (fn, err.max())
        del out
    ctx.close()
    del X
    torch.cuda.empty_cache()


@pytest.mark.parametrize("fn", ["ncc_fp32", "ncc_bf16x3", "ncc_bf16x6"])
@pytest.mark.parametrize("tile", [128, 256])
def test_four_and_eight_wave_gram_agree(ctx, fn, tile):
    # both workgroup shapes issue the same MFMA sequence per output: results are identical
    import torch
    announce("ncc waves 4 vs 8 tile=%d %s" % (tile, fn))
    g = np.random.default_rng(tile)
    X = torch.from_numpy(g.standard_normal((tile * 3 + 5, 3000)).astype(np.float32)).cuda()
    ctx.set(ncc_tile=tile, ncc_waves=4)
    a = ctx.allpairs(X, fn)
    # 8 waves on a 256 tile skip the blocks below the diagonal of diagonal tiles; every
    # item is still popped exactly once
    ctx.set(ncc_waves=8, ledger=1)
    b = ctx.allpairs(X, fn)
    led = ctx.ledger()
    ctx.set(ncc_tile=0, ncc_waves=0, ledger=0)
    assert led.size == ctx.stats()["work_items"] and np.all(led == 1)
    assert torch.equal(a, b)
    n = X.shape[0]
    pi, pj = oracle.all_pairs(n)
    sel = np.arange(0, pi.size, 53)
    rho, tau = oracle.ncc(X.cpu().numpy(), pi[sel], pj[sel])
    assert floored_rel(b.cpu().numpy()[sel], rho, tau).max() <= TOL[fn]
