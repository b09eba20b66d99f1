"""Workspace bounds: the NCC compare batches its tiles when the split-K partials do not fit
the workspace cap (same output bit for bit, every work item popped once), and every pair
function refuses a cap it cannot work within with ROCKET_E_OOM, leaving the context usable.
"""
import numpy as np
import pytest

import oracle
from paper_2009_04755_amd import synth

from gpu_util import announce, device_or_skip, floored_rel

pytestmark = pytest.mark.gpu
MiB = 1 << 20


def _fresh():
    device_or_skip()
    from paper_2009_04755_amd import Context
    return Context(0)


@pytest.mark.parametrize("fn", ["ncc_bf16x6", "ncc_fp32"])
@pytest.mark.parametrize("tiles_per_batch", [1, 3])
def test_capped_ncc_batches_match_uncapped(fn, tiles_per_batch):
    import torch
    announce("ncc workspace cap: %s, ~%d tiles per launch" % (fn, tiles_per_batch))
    n, d = 700, 5000  # tile 128: 21 leaf tiles
    X, _ = synth.dense_patterns(n, d, 8, 0.05, config=0, salt=tiles_per_batch)
    Xd = torch.from_numpy(X).cuda()
    ref_ctx = _fresh()
    ref = ref_ctx.allpairs(Xd, fn).cpu().numpy()
    ref_ctx.close()

    ctx = _fresh()
    ctx.set(ledger=1)
    ctx.prepare(Xd, fn)
    st = ctx.stats()
    T, nchunks = st["tile"], st["work_items"] // st["tiles"]
    tile_partial = nchunks * T * T * 4
    assert st["tiles"] == 21 and nchunks > 1
    # room for everything prepare allocated, the documented margin and the chosen tiles
    ctx.set(workspace_cap=st["workspace_bytes"] + 4 * MiB + tiles_per_batch * tile_partial + 2 * MiB - 1)
    out = ctx.compare()
    got = out.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    assert ctx.stats()["workspace_bytes"] <= ctx.get("workspace_cap")
    # every (tile, chunk) item ran exactly once over all batches
    led = ctx.ledger()
    assert led.size == 21 * nchunks and np.all(led == 1)
    # a second compare on the same preparation, then back to one launch: still identical
    got2 = ctx.compare().cpu().numpy()
    assert np.array_equal(got2.view(np.uint32), ref.view(np.uint32))
    ctx.set(workspace_cap=0)
    got3 = ctx.compare().cpu().numpy()
    assert np.array_equal(got3.view(np.uint32), ref.view(np.uint32))
    pi, pj = oracle.all_pairs(n)
    rho, tau = oracle.ncc(X, pi, pj)
    assert floored_rel(got, rho, tau).max() <= 1e-5
    ctx.close()


def test_cap_below_one_tile_is_refused():
    import torch
    from paper_2009_04755_amd import _lib
    announce("ncc workspace cap: no room for one tile's partials")
    X, _ = synth.dense_patterns(300, 3000, 4, 0.1, config=0, salt=2)
    Xd = torch.from_numpy(X).cuda()
    ctx = _fresh()
    ctx.prepare(Xd, "ncc_bf16x6")
    ctx.set(workspace_cap=ctx.stats()["workspace_bytes"] + MiB)
    with pytest.raises(_lib.RocketError) as e:
        ctx.compare()
    assert e.value.status == _lib.E_OOM and "partials" in str(e.value)
    ctx.set(workspace_cap=0)
    got = ctx.allpairs(Xd, "ncc_bf16x6").cpu().numpy()
    pi, pj = oracle.all_pairs(300)
    rho, tau = oracle.ncc(X, pi, pj)
    assert floored_rel(got, rho, tau).max() <= 1e-5
    ctx.close()


def test_tiny_cap_refuses_every_pair_function():
    import torch
    from paper_2009_04755_amd import Clouds, SparseSet, _lib
    announce("workspace cap of 1 MiB: every pair function refuses with E_OOM")
    X, _ = synth.dense_patterns(100, 20000, 4, 0.1, config=0, salt=3)      # planes alone ~12 MiB
    off, xy = synth.point_clouds(1500, nmin=200, nmax=400, config=2, salt=3)  # packed points ~3.6 MB
    sig = synth.point_sigmas(off, salt=3)
    so, sk, sv = synth.sparse_vectors(40, key_space=20 ** 6, nnz_mean=20000, nnz_min=5000, nnz_max=50000, salt=3)
    Xp, _, _ = synth.noise_images(200, 128, nsrc=4, amp=0.3, salt=3)        # spectra ~13 MiB
    cl = Clouds(torch.from_numpy(off).cuda(), torch.from_numpy(xy).cuda(), 0.02, torch.from_numpy(sig).cuda())
    sets = {"ncc_bf16x6": torch.from_numpy(X).cuda(), "gauss_overlap": cl, "gmm_l2": cl,
            "sparse_cosine": SparseSet(torch.from_numpy(so).cuda(), torch.from_numpy(sk).cuda(),
                                       torch.from_numpy(sv).cuda()),
            "pce": torch.from_numpy(Xp).cuda()}
    for fn, x in sets.items():
        ctx = _fresh()
        ctx.set(workspace_cap=MiB)
        with pytest.raises(_lib.RocketError) as e:
            ctx.allpairs(x, fn)
        assert e.value.status == _lib.E_OOM, (fn, e.value.status)
        assert ctx.stats()["workspace_bytes"] <= MiB
        ctx.set(workspace_cap=0)
        out = ctx.allpairs(x, fn)  # the context stays usable
        torch.cuda.synchronize()
        assert bool(torch.isfinite(out).any()), fn
        ctx.close()
