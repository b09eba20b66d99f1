"""The autotuner: tuned shapes give the default shape's output (bit for bit where only the
schedule changes, within the oracle's bar where the summation order changes), the choice is
written to the cache file, and a second context with the same cache applies it without
timing."""
import json

import numpy as np
import pytest

import oracle
from paper_2009_04755_amd import synth

from gpu_util import announce, device_or_skip, floored_rel

pytestmark = pytest.mark.gpu


def _ctx():
    device_or_skip()
    from paper_2009_04755_amd import Context
    return Context(0)


def test_ncc_tuning_and_cache(tmp_path):
    import torch
    announce("autotune ncc_bf16x6 n=700 d=5000")
    X, _ = synth.dense_patterns(700, 5000, 8, 0.05, config=0, salt=21)
    Xd = torch.from_numpy(X).cuda()
    c0 = _ctx()
    ref = c0.allpairs(Xd, "ncc_bf16x6").cpu().numpy()
    kc0 = c0.stats()["kchunk"]
    c0.close()
    cache = str(tmp_path / "tune.json")
    c1 = _ctx()
    c1.set_tune_cache(cache)
    c1.prepare(Xd, "ncc_bf16x6")
    ch = c1.autotune()
    assert not ch["cached"] and ch["tune_ms"] > 0
    assert ch["ncc_tile"] in (64, 128) and ch["ncc_waves"] in (4, 8) and ch["ncc_kchunk"] in (kc0, kc0 // 2)
    got = c1.compare().cpu().numpy()
    if ch["ncc_kchunk"] == kc0:  # tile and waves change only the schedule
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    pi, pj = oracle.all_pairs(700)
    rho, tau = oracle.ncc(X, pi, pj)
    assert floored_rel(got, rho, tau).max() <= 1e-5
    data = json.load(open(cache))
    assert len(data) == 1 and list(data.values())[0]["ncc_tile"] == ch["ncc_tile"]
    # a second context: the cached shape, nothing timed, the same output
    c2 = _ctx()
    c2.set_tune_cache(cache)
    c2.prepare(Xd, "ncc_bf16x6")
    ch2 = c2.autotune()
    assert ch2["cached"] and all(ch2[k] == ch[k] for k in ("ncc_tile", "ncc_waves", "ncc_kchunk"))
    got2 = c2.compare().cpu().numpy()
    assert np.array_equal(got2.view(np.uint32), got.view(np.uint32))
    c1.close()
    c2.close()


def test_sparse_tuning_and_cache(tmp_path):
    import torch
    from paper_2009_04755_amd import SparseSet
    announce("autotune sparse_cosine n=200")
    off, keys, vals = synth.sparse_vectors(200, key_space=20 ** 6, nnz_mean=3000, nnz_min=300, nnz_max=20000,
                                           config=4, salt=22)
    S = SparseSet(torch.from_numpy(off).cuda(), torch.from_numpy(keys).cuda(), torch.from_numpy(vals).cuda())
    cache = str(tmp_path / "tune.json")
    c1 = _ctx()
    c1.set_tune_cache(cache)
    c1.set(autotune=1)  # tune at the end of prepare
    got, cnt = c1.allpairs(S, "sparse_cosine", counts=True)
    st = c1.stats()
    assert st["tune_us"] > 0 and st["tune_cached"] == 0
    ch = {k: c1.get(k) for k in ("sp_lanes", "sp_chunk")}
    assert ch["sp_lanes"] in (4, 8)
    pi, pj = oracle.all_pairs(200)
    ref, rcnt, _, tau = oracle.sparse_cosine(off, keys, vals, pi, pj, with_tau=True)
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64), rcnt)
    g = got.cpu().numpy()
    ok = rcnt > 0
    assert np.all(np.abs(g[ok] - ref[ok]) <= 1e-5 * np.maximum(np.abs(ref[ok]), tau[ok]))
    c2 = _ctx()
    c2.set_tune_cache(cache)
    c2.set(autotune=1)
    got2, cnt2 = c2.allpairs(S, "sparse_cosine", counts=True)
    assert c2.stats()["tune_cached"] == 1
    assert all(c2.get(k) == v for k, v in ch.items())
    assert torch.equal(got, got2) and torch.equal(cnt, cnt2)
    c1.close()
    c2.close()


def test_cloud_tuning_is_schedule_only_and_cached(tmp_path):
    import torch
    from paper_2009_04755_amd import Clouds
    announce("autotune gauss_overlap n=300")
    off, xy = synth.point_clouds(300, config=2, salt=23)
    cl = Clouds(torch.from_numpy(off).cuda(), torch.from_numpy(xy).cuda(), 0.02)
    c0 = _ctx()
    ref = c0.allpairs(cl, "gauss_overlap")
    c0.close()
    cache = str(tmp_path / "tune.json")
    c1 = _ctx()
    c1.set_tune_cache(cache)
    c1.prepare(cl, "gauss_overlap")
    ch = c1.autotune()
    got = c1.compare()
    # the chosen block and variant change the schedule; each pair's sums are per lane
    # layout, so the variant may change the summation order: within the overlap bar
    pi, pj = oracle.all_pairs(300)
    sel = np.arange(0, pi.size, 31)
    r, kap = oracle.overlap(off, xy, pi[sel], pj[sel], 0.02)
    nn = np.diff(off)[pi[sel]] * np.diff(off)[pj[sel]]
    g = got.cpu().numpy()[sel]
    assert np.all(np.abs(g - r) <= 1e-5 * r * np.maximum(1, kap / 50) + nn * 2.0 ** -126)
    if ch["ovl_variant"] == 3:  # the default inner loop: only the block (schedule) differs
        assert torch.equal(got, ref)
    c2 = _ctx()
    c2.set_tune_cache(cache)
    c2.prepare(cl, "gauss_overlap")
    ch2 = c2.autotune()
    assert ch2["cached"] and ch2["ovl_block"] == ch["ovl_block"] and ch2["ovl_variant"] == ch["ovl_variant"]
    assert torch.equal(c2.compare(), got)
    c1.close()
    c2.close()
