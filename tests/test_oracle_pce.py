"""Pins for the PCE oracle (forensics variant of Section V-A)."""
import numpy as np
import pytest

from oracle import pce


def test_fft_correlation_matches_explicit_sum():
    g = np.random.default_rng(0)
    a = g.standard_normal((8, 8))
    b = g.standard_normal((8, 8))
    A, B = a - a.mean(), b - b.mean()
    C = np.zeros((8, 8))
    for sr in range(8):
        for sc in range(8):
            C[sr, sc] = sum(A[(r + sr) % 8, (c + sc) % 8] * B[r, c] for r in range(8) for c in range(8))
    np.testing.assert_allclose(pce.correlation(a, b), C, rtol=0, atol=1e-12)


@pytest.mark.parametrize("shift", [(0, 0), (3, 5), (7, 1)])
def test_peak_is_the_shift_between_copies(shift):
    g = np.random.default_rng(1)
    b = g.standard_normal((16, 16))
    a = np.roll(b, shift, axis=(0, 1))  # a(x) = b(x - shift)
    v, p = pce.pce(a, b)
    assert p == shift[0] * 16 + shift[1]
    v0, p0 = pce.pce(b, b)
    assert p0 == 0 and abs(v - v0) <= 1e-9 * v0  # shifting a copy does not change the score


@pytest.mark.parametrize("L,k,h", [(16, 1, 1), (32, 3, 5), (64, 5, 5)])
def test_cosine_wave_closed_form(L, k, h):
    # a = b = cos(2 pi k c / L): C(s) = (L^2/2) cos(2 pi k s_c / L), independent of s_r, so
    # PCE = (L^2 - (2h+1)^2) / (L^2/2 - (2h+1) S),  S = sum_{|t|<=h} cos^2(2 pi k t / L)
    c = np.arange(L)
    a = np.tile(np.cos(2 * np.pi * k * c / L), (L, 1))
    v, _ = pce.pce(a, a, h)
    S = sum(np.cos(2 * np.pi * k * t / L) ** 2 for t in range(-h, h + 1))
    want = (L * L - (2 * h + 1) ** 2) / (L * L / 2 - (2 * h + 1) * S)
    assert abs(v - want) <= 1e-9 * want


def test_scale_invariance_and_constant_item():
    g = np.random.default_rng(2)
    a = g.standard_normal((16, 16))
    b = g.standard_normal((16, 16))
    v1, p1 = pce.pce(a, b)
    v2, p2 = pce.pce(4.0 * a + 3.0, 0.5 * b - 1.0)  # positive scale and offset
    assert p1 == p2 and abs(v1 - v2) <= 1e-9 * v1
    v3, _ = pce.pce(np.full((16, 16), 2.0), b)
    assert np.isnan(v3)


def test_neighbourhood_wraps_around():
    # a peak at the corner: the excluded neighbourhood spans all four corners
    C = np.zeros((16, 16))
    C[0, 0] = 10.0
    C[15, 15] = 3.0   # inside the cyclic 3x3 neighbourhood of (0, 0): excluded
    C[8, 8] = 1.0     # outside
    v, p = pce.pce_of_surface(C, h=1)
    assert p == 0 and abs(v - 100.0 * (256 - 9) / 1.0) < 1e-9


def test_rectangular_correlation_matches_explicit_sum():
    # H != W catches a transposed axis or a modulus taken over the wrong side
    g = np.random.default_rng(3)
    a = g.standard_normal((4, 6))
    b = g.standard_normal((4, 6))
    A, B = a - a.mean(), b - b.mean()
    C = np.zeros((4, 6))
    for sr in range(4):
        for sc in range(6):
            C[sr, sc] = sum(A[(r + sr) % 4, (c + sc) % 6] * B[r, c] for r in range(4) for c in range(6))
    np.testing.assert_allclose(pce.correlation(a, b), C, rtol=0, atol=1e-12)


def test_odd_shape_correlation_matches_explicit_sum():
    # odd sides: no self-mirror middle row or column in the spectrum; the cyclic sum is the same
    g = np.random.default_rng(5)
    a = g.standard_normal((5, 7))
    b = g.standard_normal((5, 7))
    A, B = a - a.mean(), b - b.mean()
    C = np.zeros((5, 7))
    for sr in range(5):
        for sc in range(7):
            C[sr, sc] = sum(A[(r + sr) % 5, (c + sc) % 7] * B[r, c] for r in range(5) for c in range(7))
    np.testing.assert_allclose(pce.correlation(a, b), C, rtol=0, atol=1e-12)


def test_neighbourhood_spanning_an_odd_side():
    # 9 x 11 with h = 4: 2h + 1 = 9 rows, so the neighbourhood of (4, 5) holds every row and
    # columns 1 .. 9; PCE = 10^2 (99 - 81) / (energy outside) with only C[0, 0] outside
    C = np.zeros((9, 11))
    C[4, 5] = 10.0
    C[8, 9] = 3.0   # row distance 4, column distance 4: inside, excluded
    C[0, 0] = 2.0   # column distance 5: outside
    v, p = pce.pce_of_surface(C, h=4)
    assert p == 4 * 11 + 5 and abs(v - 100.0 * 18 / 4.0) < 1e-9


@pytest.mark.parametrize("H,W", [(256, 512), (1024, 1024), (96, 40)])
def test_large_correlation_matches_explicit_sums_at_sampled_shifts(H, W):
    g = np.random.default_rng(H + W)
    a = g.standard_normal((H, W))
    b = 0.3 * np.roll(a, (17, W - 5), axis=(0, 1)) + g.standard_normal((H, W))
    C = pce.correlation(a, b)
    A, B = a - a.mean(), b - b.mean()
    shifts = [(0, 0), (H - 17, 5), (H - 1, W - 1), (1, 0), (0, 1)] + \
        [tuple(s) for s in np.stack([g.integers(0, H, 15), g.integers(0, W, 15)], axis=1)]
    scale = np.sqrt(np.sum(A * A) * np.sum(B * B))
    for sr, sc in shifts:
        want = np.sum(np.roll(A, (-sr, -sc), axis=(0, 1)) * B)  # sum_x a(x + s) b(x)
        assert abs(C[sr, sc] - want) <= 1e-12 * scale, (sr, sc)
    # b holds a copy of a shifted by (17, -5): a(x) ~ b(x - s*) at s* = (-17, 5)
    assert int(np.argmax(C)) == (H - 17) * W + 5


@pytest.mark.parametrize("H,W,k,h,axis", [(16, 32, 3, 2, 1), (32, 16, 3, 2, 1), (64, 16, 5, 3, 0), (48, 80, 7, 3, 1),
                                           (36, 20, 4, 2, 0)])
def test_rectangular_cosine_wave_closed_form(H, W, k, h, axis):
    # a = b = cos(2 pi k t / n) along one axis of n values: C(s) = (H W / 2) cos(2 pi k s_axis / n),
    # PCE = (H W - (2h+1)^2) / (H W / 2 - (2h+1) S),  S = sum_{|t|<=h} cos^2(2 pi k t / n)
    n = (H, W)[axis]
    wave = np.cos(2 * np.pi * k * np.arange(n) / n)
    a = np.tile(wave, (H, 1)) if axis == 1 else np.tile(wave[:, None], (1, W))
    v, p = pce.pce(a, a, h)
    S = sum(np.cos(2 * np.pi * k * t / n) ** 2 for t in range(-h, h + 1))
    want = (H * W - (2 * h + 1) ** 2) / (H * W / 2 - (2 * h + 1) * S)
    assert p == 0 and abs(v - want) <= 1e-9 * want
