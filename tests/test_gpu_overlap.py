"""GPU parity of the Gaussian-overlap cost and its adjoint against the FP64 oracle.

Cost pass metric: |g - r| <= 1e-5 * r * max(1, kappa/50) + N_i N_j 2^-126, kappa the
cost-weighted mean |exponent| (FP32 rounding of an exponent of size E moves a term by
~3u E).  Gradient: |g - r| <= 1e-5 * max(|r|, tau) + slack, tau the RMS-type floor of a
signed sum of FP32 terms (oracle).
"""
import numpy as np
import pytest

import oracle
from paper_2009_04755_amd import synth

from gpu_util import announce, device_or_skip

pytestmark = pytest.mark.gpu
SIG = 0.02
TINY = 2.0 ** -126


def _cost_ok(got, ref, kappa, nn):
    slack = nn * TINY
    lim = 1e-5 * ref * np.maximum(1.0, kappa / 50.0) + slack
    return np.abs(got - ref) <= lim


@pytest.fixture(scope="module")
def ctx():
    device_or_skip()
    from paper_2009_04755_amd import Context
    return Context(0)


def _clouds_dev(off, xy):
    import torch
    from paper_2009_04755_amd import Clouds
    return Clouds(torch.from_numpy(off).cuda(), torch.from_numpy(xy).cuda(), SIG)


def _mixed_set():
    # uneven clouds incl. empty, single-point and identical clouds
    off, xy = synth.point_clouds(30, nmin=1, nmax=90, config=2, salt=21)
    pts = xy.reshape(-1, 2)
    clouds = [pts[off[i]:off[i + 1]] for i in range(30)]
    clouds[4] = pts[:0]
    clouds[9] = clouds[8].copy()
    clouds.append(np.array([[0.5, 0.5]], dtype=np.float32))
    o = np.zeros(len(clouds) + 1, dtype=np.int64)
    o[1:] = np.cumsum([len(c) for c in clouds])
    return o, np.concatenate(clouds).astype(np.float32).reshape(-1)


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
@pytest.mark.parametrize("block", [4, 16])
def test_cost_small_mixed(ctx, variant, block):
    announce("overlap mixed n=31 variant=%d block=%d" % (variant, block))
    off, xy = _mixed_set()
    n = off.size - 1
    ctx.set(ovl_variant=variant, ovl_block=block, queue_order=0)
    got = ctx.allpairs(_clouds_dev(off, xy), "gauss_overlap").cpu().numpy()
    pi, pj = oracle.all_pairs(n)
    ref, kap = oracle.overlap(off, xy, pi, pj, SIG)
    nn = np.diff(off)[pi] * np.diff(off)[pj]
    ok = _cost_ok(got, ref, kap, nn)
    assert ok.all(), np.abs(got - ref)[~ok][:5]


def test_cost_workload_subset_all_pairs(ctx):
    # 256 clouds of the workload recipe (50..400 points), every pair
    announce("overlap n=256 all pairs")
    off, xy = synth.point_clouds(256, config=2)
    ctx.set(ovl_variant=0, ovl_block=0)
    got = ctx.allpairs(_clouds_dev(off, xy), "gauss_overlap").cpu().numpy()
    pi, pj = oracle.all_pairs(256)
    ref, kap = oracle.overlap(off, xy, pi, pj, SIG)
    nn = np.diff(off)[pi] * np.diff(off)[pj]
    ok = _cost_ok(got, ref, kap, nn)
    rel = np.abs(got - ref) / np.maximum(ref, 1e-300)
    announce("pure rel err p50 %.2e max(ok pairs) %.2e, kappa>50: %.3f" % (
        np.median(rel[ref > 0]), rel[ok & (ref > 1e-30)].max(), np.mean(kap > 50)))
    assert ok.all()


def test_cost_full_scale_sampled_and_deterministic(ctx):
    # 2048 clouds, 2,096,128 pairs in one persistent launch; 3,000 sampled pairs vs FP64
    import torch
    announce("overlap full n=2048 sampled + determinism")
    off, xy = synth.point_clouds(2048, config=2)
    cl = _clouds_dev(off, xy)
    ctx.set(ovl_variant=0, ovl_block=0, queue_order=0, ledger=1)
    a = ctx.allpairs(cl, "gauss_overlap")
    led = ctx.ledger()
    assert np.all(led == 1)
    ctx.set(queue_order=1, seed=99, ledger=0)
    b = ctx.allpairs(cl, "gauss_overlap")
    ctx.set(queue_order=0, seed=0)
    assert torch.equal(a, b)
    g = np.random.default_rng(11)
    i = g.integers(0, 2048, 3000)
    j = g.integers(0, 2048, 3000)
    pi, pj = np.minimum(i, j), np.maximum(i, j)
    keep = pi < pj
    pi, pj = pi[keep], pj[keep]
    ref, kap = oracle.overlap(off, xy, pi, pj, SIG)
    idx = pi * 2048 - pi * (pi + 1) // 2 + (pj - pi - 1)
    got = a.cpu().numpy()[idx]
    nn = np.diff(off)[pi] * np.diff(off)[pj]
    assert _cost_ok(got, ref, kap, nn).all()


def test_autotune_picks_valid_shape(ctx):
    announce("overlap autotune n=512")
    off, xy = synth.point_clouds(512, config=2, salt=3)
    cl = _clouds_dev(off, xy)
    ctx.set(ovl_variant=0, ovl_block=0)
    ctx.prepare(cl, "gauss_overlap")
    choice = ctx.autotune()
    assert choice["ovl_block"] in (4, 8, 16) and choice["ovl_variant"] in (1, 2, 3, 4)
    got = ctx.compare().cpu().numpy()
    pi, pj = oracle.all_pairs(512)
    sel = np.arange(0, pi.size, 97)
    ref, kap = oracle.overlap(off, xy, pi[sel], pj[sel], SIG)
    nn = np.diff(off)[pi[sel]] * np.diff(off)[pj[sel]]
    assert _cost_ok(got[sel], ref, kap, nn).all()
    ctx.set(ovl_variant=0, ovl_block=0)


def test_errors(ctx):
    import torch
    from paper_2009_04755_amd import Clouds
    from paper_2009_04755_amd._lib import RocketError, E_INVALID
    announce("overlap errors")
    off = torch.tensor([0, 3, 2], dtype=torch.int64, device="cuda")
    xy = torch.zeros(6, device="cuda")
    with pytest.raises(RocketError) as e:
        ctx.allpairs(Clouds(off, xy, SIG), "gauss_overlap")
    assert e.value.status == E_INVALID
    with pytest.raises(RocketError) as e:
        ctx.allpairs(Clouds(torch.tensor([0, 1, 2], device="cuda"), xy[:4], 0.0), "gauss_overlap")
    assert e.value.status == E_INVALID
