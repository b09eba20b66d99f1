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
