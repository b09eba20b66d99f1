"""Pins for the per-localisation-uncertainty mixture scores (Section V-C: GMM L2 distance and
Bhattacharya distance between particles)."""
import numpy as np
from scipy.integrate import simpson

import oracle
from paper_2009_04755_amd import synth


def _clouds(*clouds):
    off = np.zeros(len(clouds) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(c) for c in clouds])
    xy = np.concatenate([np.asarray(c, dtype=np.float32).reshape(-1, 2) for c in clouds]).reshape(-1)
    return off, xy


def _grid(P, smax):
    lo = P.min(axis=0) - 9 * smax
    hi = P.max(axis=0) + 9 * smax
    h = smax / 12
    gx = np.linspace(lo[0], hi[0], int(np.ceil((hi[0] - lo[0]) / h)) | 1)
    gy = np.linspace(lo[1], hi[1], int(np.ceil((hi[1] - lo[1]) / h)) | 1)
    return gx, gy, np.meshgrid(gx, gy, indexing="ij")


def _normal(Z, p, s):
    return np.exp(-((Z[0] - p[0]) ** 2 + (Z[1] - p[1]) ** 2) / (2 * s * s)) / (2 * np.pi * s * s)


def test_l2_cross_term_is_integral_of_mixture_product():
    g = np.random.default_rng(1)
    X = 0.5 + 0.02 * g.standard_normal((3, 2))
    Y = 0.5 + 0.02 * g.standard_normal((2, 2))
    off, xy = _clouds(X, Y)
    P = xy.astype(np.float64).reshape(-1, 2)
    sig = np.array([0.01, 0.02, 0.015, 0.025, 0.012], dtype=np.float32)
    gx, gy, Z = _grid(P, 0.025)
    fx = sum(_normal(Z, P[k], float(sig[k])) for k in range(3))
    fy = sum(_normal(Z, P[3 + l], float(sig[3 + l])) for l in range(2))
    ref = simpson(simpson(fx * fy, x=gy, axis=1), x=gx)
    got = oracle.gmm(off, xy, sig, [0], [1], "l2")[0]
    assert abs(got - ref) <= 1e-9 * ref


def test_bhattacharya_coefficient_of_single_components():
    for (a, b, s, t) in [((0.5, 0.5), (0.52, 0.49), 0.01, 0.02), ((0.1, 0.2), (0.1, 0.2), 0.015, 0.015)]:
        off, xy = _clouds([a], [b])
        sig = np.array([s, t], dtype=np.float32)
        P = xy.astype(np.float64).reshape(-1, 2)
        gx, gy, Z = _grid(P, max(s, t))
        f = np.sqrt(_normal(Z, P[0], float(sig[0])) * _normal(Z, P[1], float(sig[1])))
        ref = simpson(simpson(f, x=gy, axis=1), x=gx)
        got = oracle.gmm(off, xy, sig, [0], [1], "bhattacharya")[0]
        assert abs(got - ref) <= 1e-8 * ref
    # identical components: coefficient exactly 1
    off, xy = _clouds([[0.3, 0.4]], [[0.3, 0.4]])
    assert abs(oracle.gmm(off, xy, np.array([0.02, 0.02], np.float32), [0], [1], "bhattacharya")[0] - 1) < 1e-15


def test_equal_sigmas_reduce_to_the_plain_overlap():
    # s = t = sigma: L2 term = exp(-D/(4 sigma^2)) / (4 pi sigma^2); Bhattacharya term = exp(-D/(8 sigma^2))
    off, xy = synth.point_clouds(6, nmin=5, nmax=40, config=2, salt=3)
    s = np.float32(0.02)
    sig = np.full(int(off[-1]), s, dtype=np.float32)
    pi, pj = oracle.all_pairs(6)
    s64 = float(s)
    base, _ = oracle.overlap(off, xy, pi, pj, s64)
    l2 = oracle.gmm(off, xy, sig, pi, pj, "l2")
    np.testing.assert_allclose(l2 * 4 * np.pi * s64 ** 2, base, rtol=1e-12)
    wide, _ = oracle.overlap(off, xy, pi, pj, np.sqrt(2.0) * s64)
    bh = oracle.gmm(off, xy, sig, pi, pj, "bhattacharya")
    np.testing.assert_allclose(bh, wide, rtol=1e-12)


def test_symmetry():
    off, xy = synth.point_clouds(5, nmin=5, nmax=30, config=2, salt=4)
    sig = synth.point_sigmas(off, salt=4)
    pi, pj = oracle.all_pairs(5)
    for mode in ("l2", "bhattacharya"):
        np.testing.assert_allclose(oracle.gmm(off, xy, sig, pi, pj, mode), oracle.gmm(off, xy, sig, pj, pi, mode),
                                   rtol=1e-13)


def test_kappa_of_a_single_term_is_its_exponent():
    off, xy = _clouds([[0.1, 0.2]], [[0.13, 0.16]])
    sig = np.array([0.01, 0.02], dtype=np.float32)
    P = xy.astype(np.float64).reshape(-1, 2)
    D = float(((P[0] - P[1]) ** 2).sum())
    v = float(sig[0]) ** 2 + float(sig[1]) ** 2
    for mode, e in (("l2", D / (2 * v)), ("bhattacharya", D / (4 * v))):
        c, k = oracle.gmm(off, xy, sig, [0], [1], mode, with_kappa=True)
        assert abs(k[0] - e) <= 1e-12 * e
