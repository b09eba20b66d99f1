"""Pins for the full-covariance particle scores and their registration gradient (Section V-C:
GMM L2 distance and Bhattacharya distance between particles whose localisations carry an
uncertainty; the registration optimiser moves one particle rigidly)."""
import numpy as np
from scipy.integrate import simpson

import oracle

SQ = 0.015625  # 2^-6: the same value in f32 and f64


def _clouds(*clouds):
    off = np.zeros(len(clouds) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(c) for c in clouds])
    xy = np.concatenate([np.asarray(c, dtype=np.float32).reshape(-1, 2) for c in clouds]).reshape(-1)
    return off, xy


def _spd(g, scale):
    """A random symmetric positive definite 2 x 2 covariance, eigenvalues in scale * [0.3, 1]."""
    th = g.uniform(0, np.pi)
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    C = R @ np.diag(scale ** 2 * g.uniform(0.3, 1.0, 2)) @ R.T
    return np.array([C[0, 0], C[0, 1], C[1, 1]], dtype=np.float32)


def _density(Z, mu, c):
    """Bivariate normal density with covariance [[c0, c1], [c1, c2]] on the grid Z."""
    c = c.astype(np.float64)
    det = c[0] * c[2] - c[1] * c[1]
    dx, dy = Z[0] - mu[0], Z[1] - mu[1]
    q = (c[2] * dx * dx - 2 * c[1] * dx * dy + c[0] * dy * dy) / det
    return np.exp(-q / 2) / (2 * np.pi * np.sqrt(det))


def _grid(P, smax, h_div=14):
    lo = P.min(axis=0) - 10 * smax
    hi = P.max(axis=0) + 10 * smax
    h = smax / h_div
    gx = np.linspace(lo[0], hi[0], int(np.ceil((hi[0] - lo[0]) / h)) | 1)
    gy = np.linspace(lo[1], hi[1], int(np.ceil((hi[1] - lo[1]) / h)) | 1)
    return gx, gy, np.meshgrid(gx, gy, indexing="ij")


def test_l2_cross_term_is_integral_of_full_covariance_mixture_product():
    g = np.random.default_rng(3)
    X = 0.5 + 0.02 * g.standard_normal((3, 2))
    Y = 0.5 + 0.02 * g.standard_normal((2, 2))
    off, xy = _clouds(X, Y)
    cov = np.stack([_spd(g, 0.02) for _ in range(5)])
    P = xy.astype(np.float64).reshape(-1, 2)
    gx, gy, Z = _grid(P, 0.02)
    fx = sum(_density(Z, P[k], cov[k]) for k in range(3))
    fy = sum(_density(Z, P[3 + l], cov[3 + l]) for l in range(2))
    ref = simpson(simpson(fx * fy, x=gy, axis=1), x=gx)
    got = oracle.gmm_grad(off, xy, [0], [1], "l2", cov=cov)[0][0]
    assert abs(got - ref) <= 1e-9 * ref


def test_bhattacharya_coefficient_of_full_covariance_components():
    g = np.random.default_rng(4)
    for a, b in [((0.5, 0.5), (0.52, 0.49)), ((0.1, 0.2), (0.1, 0.21))]:
        off, xy = _clouds([a], [b])
        cov = np.stack([_spd(g, 0.015), _spd(g, 0.025)])
        P = xy.astype(np.float64).reshape(-1, 2)
        gx, gy, Z = _grid(P, 0.025)
        f = np.sqrt(_density(Z, P[0], cov[0]) * _density(Z, P[1], cov[1]))
        ref = simpson(simpson(f, x=gy, axis=1), x=gx)
        got = oracle.gmm_grad(off, xy, [0], [1], "bhattacharya", cov=cov)[0][0]
        assert abs(got - ref) <= 1e-8 * ref
    # identical components: coefficient exactly 1
    off, xy = _clouds([[0.3, 0.4]], [[0.3, 0.4]])
    c = _spd(g, 0.02)
    assert abs(oracle.gmm_grad(off, xy, [0], [1], "bhattacharya", cov=np.stack([c, c]))[0][0] - 1) < 1e-14


def test_isotropic_covariances_reduce_to_the_per_point_sigma_scores():
    g = np.random.default_rng(5)
    off, xy = _clouds(0.5 + 0.03 * g.standard_normal((7, 2)), 0.5 + 0.03 * g.standard_normal((5, 2)),
                      0.5 + 0.03 * g.standard_normal((4, 2)))
    sig = g.uniform(0.01, 0.03, 16).astype(np.float32)
    cov = np.stack([sig.astype(np.float64) ** 2, np.zeros(16), sig.astype(np.float64) ** 2], axis=1).astype(np.float32)
    pi, pj = oracle.all_pairs(3)
    for mode in ("l2", "bhattacharya"):
        ref = oracle.gmm(off, xy, sig, pi, pj, mode)
        via_sig = oracle.gmm_grad(off, xy, pi, pj, mode, sig=sig)[0]
        assert np.allclose(via_sig, ref, rtol=1e-13, atol=0)
        # s^2 rounded to f32 moves the score by ~1e-7 relative: the same reduction within that
        via_cov = oracle.gmm_grad(off, xy, pi, pj, mode, cov=cov)[0]
        assert np.allclose(via_cov, ref, rtol=2e-6, atol=0)


def test_equal_fixed_sigma_l2_score_and_gradient_are_the_scaled_plain_overlap():
    # s_k = t_l = sigma: each L2 term is exp(-d^2 / (4 sigma^2)) / (4 pi sigma^2), so cost and
    # gradient are the fixed-sigma overlap's divided by 4 pi sigma^2 (a separately pinned oracle)
    g = np.random.default_rng(6)
    off, xy = _clouds(0.5 + 0.02 * g.standard_normal((9, 2)), 0.5 + 0.02 * g.standard_normal((6, 2)),
                      0.5 + 0.02 * g.standard_normal((5, 2)))
    n = 3
    cen = np.stack([xy.reshape(-1, 2)[off[c]:off[c + 1]].astype(np.float64).mean(axis=0) for c in range(n)]
                   ).astype(np.float32)
    pi, pj = oracle.all_pairs(n)
    prm = np.stack([g.uniform(-0.3, 0.3, pi.size), g.uniform(-0.01, 0.01, pi.size),
                    g.uniform(-0.01, 0.01, pi.size)], axis=1)
    sig = np.full(20, SQ, dtype=np.float32)
    c1, g1, _, _ = oracle.gmm_grad(off, xy, pi, pj, "l2", sig=sig, centroids=cen, params=prm)
    c0, g0, _, _ = oracle.overlap_grad(off, xy, cen, pi, pj, prm, SQ)
    s2 = SQ * SQ
    assert np.allclose(c1 * 4 * np.pi * s2, c0, rtol=1e-12, atol=0)
    assert np.allclose(g1 * 4 * np.pi * s2, g0, rtol=1e-10, atol=1e-13 * np.abs(g0).max())


def _quarter_turn(P, c):
    """Points rotated by +90 degrees about c (exact for dyadic coordinates)."""
    return np.stack([c[0] - (P[:, 1] - c[1]), c[1] + (P[:, 0] - c[0])], axis=1)


def test_transform_moves_points_and_rotates_covariances():
    # a quarter turn about the (dyadic) centroid plus a dyadic shift, applied by the oracle's
    # transform path, equals the identity path on the cloud moved beforehand: points rotated
    # and shifted, covariances [[a, b], [b, c]] -> [[c, -b], [-b, a]]
    g = np.random.default_rng(7)
    X = np.round((0.5 + 0.02 * g.standard_normal((5, 2))) * 2 ** 12) / 2 ** 12
    Y = np.round((0.5 + 0.02 * g.standard_normal((4, 2))) * 2 ** 12) / 2 ** 12
    cov = np.stack([_spd(g, 0.02) for _ in range(9)])
    c = np.array([0.5, 0.5])
    t = np.array([0.0078125, -0.00390625])
    Ym = _quarter_turn(Y, c) + t
    covm = cov.copy()
    covm[5:] = np.stack([cov[5:, 2], -cov[5:, 1], cov[5:, 0]], axis=1)
    off, xy = _clouds(X, Y)
    _, xym = _clouds(X, Ym)
    cen = np.array([[0.5, 0.5], [0.5, 0.5]], dtype=np.float32)
    for mode in ("l2", "bhattacharya"):
        moved = oracle.gmm_grad(off, xy, [0], [1], mode, cov=cov, centroids=cen,
                                params=np.array([[np.pi / 2, t[0], t[1]]]))[0][0]
        pre = oracle.gmm_grad(off, xym, [0], [1], mode, cov=covm)[0][0]
        assert abs(moved - pre) <= 1e-12 * pre


def test_joint_rigid_motion_leaves_the_scores_unchanged():
    g = np.random.default_rng(8)
    X = np.round((0.5 + 0.02 * g.standard_normal((6, 2))) * 2 ** 12) / 2 ** 12
    Y = np.round((0.5 + 0.02 * g.standard_normal((5, 2))) * 2 ** 12) / 2 ** 12
    cov = np.stack([_spd(g, 0.02) for _ in range(11)])
    c = np.array([0.25, 0.75])
    t = np.array([0.125, -0.0625])
    off, xy = _clouds(X, Y)
    _, xym = _clouds(_quarter_turn(X, c) + t, _quarter_turn(Y, c) + t)
    covm = np.stack([cov[:, 2], -cov[:, 1], cov[:, 0]], axis=1)
    for mode in ("l2", "bhattacharya"):
        a = oracle.gmm_grad(off, xy, [0], [1], mode, cov=cov)[0][0]
        b = oracle.gmm_grad(off, xym, [0], [1], mode, cov=covm)[0][0]
        assert abs(a - b) <= 1e-13 * a


def _cost(off, xy, cov, cen, mode, q):
    return oracle.gmm_grad(off, xy, [0], [1], mode, cov=cov, centroids=cen, params=np.array([q], dtype=np.float64))[0][0]


def _richardson(off, xy, cov, cen, mode, q, m, h):
    def cd(hh):
        e = np.zeros(3)
        e[m] = hh
        return (_cost(off, xy, cov, cen, mode, q + e) - _cost(off, xy, cov, cen, mode, q - e)) / (2 * hh)
    return (4 * cd(h / 2) - cd(h)) / 3


def test_gradient_matches_richardson_differences_of_the_cost():
    g = np.random.default_rng(9)
    X = 0.5 + 0.02 * g.standard_normal((6, 2))
    Y = 0.5 + 0.02 * g.standard_normal((5, 2))
    off, xy = _clouds(X, Y)
    cov = np.stack([_spd(g, 0.02) for _ in range(11)])
    cen = np.stack([X.mean(axis=0), Y.mean(axis=0)]).astype(np.float32)
    for mode in ("l2", "bhattacharya"):
        for q in ([0.0, 0.0, 0.0], [0.4, 0.01, -0.005], [-1.2, -0.02, 0.015]):
            q = np.array(q)
            _, gr, tau, _ = oracle.gmm_grad(off, xy, [0], [1], mode, cov=cov, centroids=cen, params=q[None])
            for m, h in ((0, 1e-3), (1, 1e-4), (2, 1e-4)):
                fd = _richardson(off, xy, cov, cen, mode, q, m, h)
                assert abs(gr[0, m] - fd) <= 1e-6 * max(abs(fd), tau[0, m]), (mode, q, m, gr[0, m], fd)


def test_error_floors_of_one_and_two_terms():
    # one term: kappa is its exponent and tau_m = |d term / d q_m| max(1, kappa/50); two terms
    # with their own gradients: kappa is the cost-weighted mean exponent and
    # tau_m = sqrt(g1^2 + g2^2) max(1, kappa/50) (a plain or absolute sum fails)
    g = np.random.default_rng(10)
    c1, c2, c3 = _spd(g, 0.02), _spd(g, 0.02), _spd(g, 0.02)
    x1, x2, y = np.array([0.5, 0.5]), np.array([0.47, 0.52]), np.array([0.51, 0.49])
    cen = np.array([[0.5, 0.5], [0.51, 0.49], [0.51, 0.49]], dtype=np.float32)
    q = np.array([[0.3, 0.004, -0.002]])
    for mode in ("l2", "bhattacharya"):
        parts = []
        for x, cx in ((x1, c1), (x2, c2)):
            off, xy = _clouds([x], [y])
            cost, gr, tau, kap = oracle.gmm_grad(off, xy, [0], [1], mode, cov=np.stack([cx, c3]),
                                                 centroids=cen[1:], params=q)
            fd = np.array([_richardson(off, xy, np.stack([cx, c3]), cen[1:], mode, q[0], m, h)
                           for m, h in ((0, 1e-3), (1, 1e-4), (2, 1e-4))])
            # kappa of one term is its exponent ln(prefactor / term), the prefactor being the
            # term's value at the same rotation with the two points on top of each other
            # (cloud j is one point at its centroid, so y' = y + t)
            q0 = np.array([[q[0, 0], x[0] - y[0], x[1] - y[1]]])
            pre = oracle.gmm_grad(off, xy, [0], [1], mode, cov=np.stack([cx, c3]), centroids=cen[1:], params=q0)[0][0]
            assert abs(kap[0] - np.log(pre / cost[0])) <= 1e-9 * kap[0]
            assert np.allclose(tau[0], np.abs(fd) * max(1.0, kap[0] / 50), rtol=1e-6)
            parts.append((cost[0], fd, kap[0]))
        off, xy = _clouds([x1, x2], [y])
        cost, gr, tau, kap = oracle.gmm_grad(off, xy, [0], [1], mode, cov=np.stack([c1, c2, c3]),
                                             centroids=cen[1:], params=q)
        assert abs(cost[0] - (parts[0][0] + parts[1][0])) <= 1e-14 * cost[0]
        kref = (parts[0][0] * parts[0][2] + parts[1][0] * parts[1][2]) / (parts[0][0] + parts[1][0])
        assert abs(kap[0] - kref) <= 1e-12 * kref
        tref = np.sqrt(parts[0][1] ** 2 + parts[1][1] ** 2) * max(1.0, kref / 50)
        assert np.allclose(tau[0], tref, rtol=1e-6)
