"""GPU PCE of images larger than one LDS tile (forensics PCE variant, Section V-A) against
the FP64 oracle: H x W items with sides in [16, 4096] (a side that is not a power of two by
Bluestein's chirp convolution; odd sides pair their rows and columns without a middle one),
pair transforms staged in HBM.

Pass metric as for the in-LDS sizes: |g - r| <= 1e-5 * r, with r the oracle's PCE at the
GPU's peak shift; that peak must be the oracle's argmax, or (where the two largest
correlations are closer than FP32 can resolve) within 1e-5 RMS of the maximum.
"""
import numpy as np
import pytest

from oracle import pce
from paper_2009_04755_amd import synth

from gpu_util import announce, device_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    device_or_skip()
    from paper_2009_04755_amd import Context
    c = Context(0)
    yield c
    c.close()


def _run(ctx, X, W, **opts):
    import torch
    ctx.set(pce_width=W, **opts)
    try:
        v, pk = ctx.allpairs(torch.from_numpy(X).cuda(), "pce", counts=True)
        torch.cuda.synchronize()
    finally:
        ctx.set(pce_width=0, **{k: 0 for k in opts})
    return v.cpu().numpy(), pk.cpu().numpy().astype(np.int64)


def _check(got, gpk, X, H, W, pairs, h=5):
    n = X.shape[0]
    worst = 0.0
    for i, j in pairs:
        idx = i * n - i * (i + 1) // 2 + (j - i - 1)
        C = pce.correlation(X[i].reshape(H, W), X[j].reshape(H, W))
        ref, rpk = pce.pce_of_surface(C, h)
        if np.isnan(ref):
            assert np.isnan(got[idx]), (i, j)
            continue
        if gpk[idx] != rpk:
            rms = np.sqrt(np.mean(C * C))
            assert C.flat[gpk[idx]] >= C.max() - 1e-5 * rms, (i, j, gpk[idx], rpk)
            ref, _ = pce.pce_of_surface(C, h, peak=gpk[idx])
        err = abs(float(got[idx]) - ref) / ref
        worst = max(worst, err)
        assert err <= 1e-5, (i, j, got[idx], ref)
    return worst


@pytest.mark.parametrize("H,W", [(16, 64), (64, 16), (256, 512), (512, 256), (2048, 16)])
def test_all_pairs_rectangular(ctx, H, W):
    n = 11  # 55 pairs: 27 two-pair transforms and one single pair
    announce("pce staged all pairs n=%d %dx%d" % (n, H, W))
    X, _, _ = synth.noise_images(n, (H, W), nsrc=3, amp=0.3, config=6, salt=H + 3 * W)
    got, gpk = _run(ctx, X, W)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    announce("max rel err %.2e" % _check(got, gpk, X, H, W, pairs, h=min(5, min(H, W) // 2 - 1)))


def test_all_pairs_1024(ctx):
    n = 7
    announce("pce staged all pairs n=%d 1024x1024" % n)
    X, c, sh = synth.noise_images(n, 1024, nsrc=2, amp=0.3, p_shift=0.5, config=6, salt=1024)
    got, gpk = _run(ctx, X, 0)  # square: the width option may stay 0
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    announce("max rel err %.2e" % _check(got, gpk, X, 1024, 1024, pairs))
    for i, j in pairs:
        if c[i] == c[j]:  # same source: the peak is the relative shift of the two crops
            idx = i * n - i * (i + 1) // 2 + (j - i - 1)
            assert gpk[idx] == ((sh[i, 0] - sh[j, 0]) % 1024) * 1024 + (sh[i, 1] - sh[j, 1]) % 1024


@pytest.mark.parametrize("L", [16, 2048, 4096])
def test_smallest_and_largest_square(ctx, L):
    # the size limits of the staged path: 16 x 16 (one radix-16 pass per axis) and 4096 x 4096
    # (2^24 values per item), with 2048 x 2048 between
    n = {16: 12, 2048: 3, 4096: 2}[L]
    announce("pce staged all pairs n=%d %dx%d" % (n, L, L))
    # one source, strong enough that the true shift beats the noise maxima at 256 shifts
    X, c, sh = synth.noise_images(n, L, nsrc=1, amp=2.0 if L == 16 else 0.5, p_shift=0.7, config=6, salt=L + 7)
    got, gpk = _run(ctx, X, 0)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    announce("max rel err %.2e" % _check(got, gpk, X, L, L, pairs))
    for i, j in pairs:  # one source: the peak is the relative shift of the two crops
        idx = i * n - i * (i + 1) // 2 + (j - i - 1)
        assert gpk[idx] == ((sh[i, 0] - sh[j, 0]) % L) * L + (sh[i, 1] - sh[j, 1]) % L


def _check_shifts(gpk, c, sh, H, W):
    n = len(c)
    for i in range(n):
        for j in range(i + 1, n):
            if c[i] == c[j]:  # same source: the peak is the relative shift of the two crops
                idx = i * n - i * (i + 1) // 2 + (j - i - 1)
                assert gpk[idx] == ((sh[i, 0] - sh[j, 0]) % H) * W + (sh[i, 1] - sh[j, 1]) % W, (i, j)


@pytest.mark.parametrize("H,W", [(48, 80), (96, 40), (100, 64), (64, 100), (18, 30), (1000, 16)])
def test_all_pairs_not_powers_of_two(ctx, H, W):
    # one side or both not a power of two: Bluestein along those axes (FFT lengths 64 .. 2048)
    n = 11
    announce("pce staged bluestein all pairs n=%d %dx%d" % (n, H, W))
    X, c, sh = synth.noise_images(n, (H, W), nsrc=3, amp=1.0, p_shift=0.7, config=6, salt=H + 5 * W)
    got, gpk = _run(ctx, X, W)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    announce("max rel err %.2e" % _check(got, gpk, X, H, W, pairs))
    _check_shifts(gpk, c, sh, H, W)


@pytest.mark.parametrize("H,W", [(17, 33), (45, 64), (64, 45), (31, 31), (99, 101)])
def test_all_pairs_odd_sides(ctx, H, W):
    # odd sides: row 0 (and no row H/2) pairs with itself, column W/2 does not exist
    n = 9
    announce("pce staged odd sides all pairs n=%d %dx%d" % (n, H, W))
    X, c, sh = synth.noise_images(n, (H, W), nsrc=2, amp=1.0, p_shift=0.7, config=6, salt=7 * H + W)
    got, gpk = _run(ctx, X, W)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    announce("max rel err %.2e" % _check(got, gpk, X, H, W, pairs, h=min(5, min(H, W) // 2 - 1)))
    _check_shifts(gpk, c, sh, H, W)


@pytest.mark.parametrize("H,W", [(2050, 16), (16, 4094), (4096, 16), (4095, 16), (16, 4095), (3001, 2001)])
def test_longest_axes(ctx, H, W):
    # 8192-point transforms: Bluestein columns one per column-pass workgroup (2050, 4095), Bluestein
    # rows one per row-pass workgroup (4094, 4095), the longest power-of-two side (4096), and an odd
    # camera-like size
    n = 3 if H * W > 10 ** 6 else 6
    announce("pce staged all pairs n=%d %dx%d" % (n, H, W))
    X, c, sh = synth.noise_images(n, (H, W), nsrc=2, amp=1.0, p_shift=0.7, config=6, salt=H + 9 * W)
    got, gpk = _run(ctx, X, W)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    announce("max rel err %.2e" % _check(got, gpk, X, H, W, pairs))
    _check_shifts(gpk, c, sh, H, W)


def test_camera_sensor_size(ctx):
    # 3648 x 2736, the image size of the forensics data set (Section V-A): both axes by
    # Bluestein with 8192-point FFTs
    H, W, n = 3648, 2736, 3
    announce("pce staged bluestein n=%d %dx%d" % (n, H, W))
    X, c, sh = synth.noise_images(n, (H, W), nsrc=1, amp=0.3, p_shift=1.0, config=6, salt=3648)
    got, gpk = _run(ctx, X, W)
    pairs = [(0, 1), (0, 2), (1, 2)]
    announce("max rel err %.2e" % _check(got, gpk, X, H, W, pairs))
    _check_shifts(gpk, c, sh, H, W)


@pytest.mark.parametrize("H,W", [(32, 64), (48, 40)])
def test_one_and_two_items(ctx, H, W):
    # one item: no pairs (prepare runs, compare has nothing to do); two items: one pair-pair
    # holding a single pair (no second channel)
    import torch
    announce("pce staged n=1 and n=2 %dx%d" % (H, W))
    X, _, _ = synth.noise_images(2, (H, W), nsrc=1, amp=1.0, p_shift=1.0, config=6, salt=H * W)
    ctx.set(pce_width=W)
    try:
        v1 = ctx.allpairs(torch.from_numpy(X[:1]).cuda(), "pce")
        torch.cuda.synchronize()
        assert v1.numel() == 0
    finally:
        ctx.set(pce_width=0)
    got, gpk = _run(ctx, X, W)
    assert got.shape == (1,)
    _check(got, gpk, X, H, W, [(0, 1)])


def test_shifted_copies_and_constant_item(ctx):
    announce("pce staged shifted copies 256x1024")
    H, W = 256, 1024
    g = np.random.default_rng(11)
    base = g.standard_normal((H, W)).astype(np.float32)
    shifts = [(0, 0), (5, 900), (255, 1), (128, 512), (17, 0)]
    X = np.stack([np.roll(base, s, axis=(0, 1)).reshape(-1) for s in shifts] + [np.full(H * W, -2.0, np.float32)])
    got, gpk = _run(ctx, X, W)
    n = X.shape[0]
    for i in range(5):
        for j in range(i + 1, 5):
            idx = i * n - i * (i + 1) // 2 + (j - i - 1)
            assert gpk[idx] == ((shifts[i][0] - shifts[j][0]) % H) * W + (shifts[i][1] - shifts[j][1]) % W
        assert np.isnan(got[i * n - i * (i + 1) // 2 + (5 - i - 1)])
    _check(got, gpk, X, H, W, [(i, j) for i in range(n) for j in range(i + 1, n)])


def test_batches_change_only_the_schedule(ctx):
    # the pair-pairs are the same whatever the batch size; each is computed by the same
    # kernels in the same order, so the output is identical bit for bit
    import torch
    announce("pce staged batches 128x256 n=13")
    X, _, _ = synth.noise_images(13, (128, 256), nsrc=3, amp=0.3, config=6, salt=5)
    ref, rpk = _run(ctx, X, 256)
    for b in (1, 7):
        got, gpk = _run(ctx, X, 256, pce_batch=b)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)) and np.array_equal(gpk, rpk)
    # a capped workspace bounds the batch the same way: room for k staged transforms of
    # 128 x 256 complex f32 and their block statistics (a few hundred bytes each, counted
    # here as 4 KiB; allocations are rounded to 2 MiB) gives two staging buffers of k // 2
    # transforms (the row pass of one batch overlapping the column pass of the other), room
    # for one a single buffer, and room for less than one transform fails with E_OOM
    from paper_2009_04755_amd import Context
    from paper_2009_04755_amd._lib import RocketError, E_OOM
    Xd = torch.from_numpy(X).cuda()
    per = 128 * 256 * 8 + 4096
    for k, ok in ((5, True), (1, True), (0, False)):
        c2 = Context(0).set(pce_width=256)
        c2.prepare(Xd, "pce")
        base = c2.stats()["workspace_bytes"]
        c2.set(workspace_cap=base + (2 << 20) + (k * per if ok else 128 * 256 * 8 - 1))
        if ok:
            got, gpk = c2.compare(counts=True)
            assert np.array_equal(got.cpu().numpy().view(np.uint32), ref.view(np.uint32))
            assert c2.stats()["grid"] == (k // 2 if k >= 2 else k)
        else:
            with pytest.raises(RocketError) as e:
                c2.compare()
            assert e.value.status == E_OOM
        c2.close()


@pytest.mark.parametrize("H,W", [(64, 128), (45, 64)])
def test_radius_option(ctx, H, W):
    # the smallest radius and the largest allowed one (h < min(H, W) / 2), also with an odd
    # side taken by Bluestein
    announce("pce staged radius %dx%d" % (H, W))
    X, _, _ = synth.noise_images(6, (H, W), nsrc=2, amp=0.4, config=6, salt=8 + H)
    pairs = [(i, j) for i in range(6) for j in range(i + 1, 6)]
    for h in (1, (min(H, W) - 1) // 2):
        got, gpk = _run(ctx, X, W, pce_radius=h)
        _check(got, gpk, X, H, W, pairs, h=h)


def test_errors(ctx):
    import torch
    from paper_2009_04755_amd._lib import RocketError, E_INVALID, E_UNSUPPORTED
    announce("pce staged errors")
    bad = [(1000, 64), (4097 * 16, 16), (16 * 4097, 4097), (8 * 64, 64), (64 * 15, 15), (15 * 15, 0)]
    for dim, w in bad:  # width not dividing, a side above 4096 or below 16
        ctx.set(pce_width=w)
        try:
            with pytest.raises(RocketError) as e:
                ctx.allpairs(torch.zeros((3, dim), device="cuda"), "pce")
            assert e.value.status == E_UNSUPPORTED, (dim, w)
        finally:
            ctx.set(pce_width=0)
    for dim, w, h in ((16 * 64, 64, 8), (45 * 64, 64, 23)):  # h < min(H, W) / 2: below 8, at most 22
        ctx.set(pce_width=w, pce_radius=h)
        try:
            with pytest.raises(RocketError) as e:
                ctx.allpairs(torch.zeros((3, dim), device="cuda"), "pce")
            assert e.value.status == E_INVALID
        finally:
            ctx.set(pce_width=0, pce_radius=0)


def test_workload_sampled(ctx):
    # the benchmark's staged workload and launch configuration: 256 noise images of 1024 x 1024
    # (32,640 pairs, default batches of 64 two-pair transforms), sampled pairs against the oracle
    announce("pce staged n=256 1024x1024 sampled")
    n = 256
    X, c, sh = synth.noise_images(n, 1024, nsrc=16, amp=0.3, config=6, salt=1)
    got, gpk = _run(ctx, X, 0)
    g = np.random.default_rng(6)
    i = g.integers(0, n, 40)
    j = g.integers(0, n, 40)
    pairs = sorted({(min(a, b), max(a, b)) for a, b in zip(i, j) if a != b})[:30]
    pairs += [(0, 1), (n - 2, n - 1), (0, n - 1)]
    announce("max rel err %.2e" % _check(got, gpk, X, 1024, 1024, pairs))
    assert np.all(np.isfinite(got)) and np.all(got > 0)
