"""Pins for the FP64 registration-gradient reference (Section V-C optimiser)."""
import numpy as np

import oracle
from paper_2009_04755_amd import synth

SIG = 0.02


def _setup(salt=0, n=4, nmin=20, nmax=60):
    off, xy = synth.point_clouds(n, nmin=nmin, nmax=nmax, config=3, salt=salt)
    cen = synth.cloud_centroids(off, xy)
    return off, xy, cen


def _cost(off, xy, cen, pi, pj, params):
    c, _, _, _ = oracle.overlap_grad(off, xy, cen, pi, pj, params, SIG)
    return c


def test_cost_at_identity_matches_plain_overlap():
    off, xy, cen = _setup(1)
    pi, pj = oracle.all_pairs(4)
    c0, _ = oracle.overlap(off, xy, pi, pj, SIG)
    c1 = _cost(off, xy, cen, pi, pj, np.zeros((pi.size, 3)))
    np.testing.assert_allclose(c1, c0, rtol=1e-13)


def test_translation_moves_cloud_j():
    # translating y by t equals translating x by -t
    off, xy, cen = _setup(2, n=2)
    t = np.array([0.013, -0.021])
    P = xy.astype(np.float64).reshape(-1, 2)
    X = P[off[0]:off[1]] - t
    Y = P[off[1]:off[2]]
    off2 = np.array([0, len(X), len(X) + len(Y)], dtype=np.int64)
    xy2 = np.concatenate([X, Y]).astype(np.float32).reshape(-1)
    a = _cost(off, xy, cen, [0], [1], np.array([[0.0, t[0], t[1]]]))
    b, _ = oracle.overlap(off2, xy2, [0], [1], SIG)
    assert abs(a[0] - b[0]) <= 1e-5 * max(a[0], 1e-30)


def test_rotation_is_about_centroid_of_cloud_j():
    # rotating y about its centroid c by +90 degrees equals rotating x about c by -90 degrees;
    # dyadic coordinates keep both sides exact in f32
    g = np.random.default_rng(4)
    X = np.round(g.uniform(0.3, 0.7, (25, 2)) * 256) / 256
    Y = np.round(g.uniform(0.3, 0.7, (18, 2)) * 256) / 256
    c = np.array([0.5, 0.5])
    off = np.array([0, 25, 43], dtype=np.int64)
    xy = np.concatenate([X, Y]).astype(np.float32).reshape(-1)
    cen = np.array([[0.5, 0.5], [c[0], c[1]]], dtype=np.float32)
    a = _cost(off, xy, cen, [0], [1], np.array([[np.pi / 2, 0.0, 0.0]]))
    Xr = np.stack([(X - c)[:, 1], -(X - c)[:, 0]], axis=1) + c  # R(-90deg)(x - c) + c
    xy2 = np.concatenate([Xr, Y]).astype(np.float32).reshape(-1)
    b, _ = oracle.overlap(off, xy2, [0], [1], SIG)
    assert abs(a[0] - b[0]) <= 1e-12 * max(b[0], 1e-30)


def test_gradient_matches_richardson_finite_differences():
    off, xy, cen = _setup(5, n=5, nmin=30, nmax=80)
    pi, pj = oracle.all_pairs(5)
    g = np.random.default_rng(6)
    params = np.stack([g.uniform(-0.2, 0.2, pi.size), g.uniform(-0.03, 0.03, pi.size),
                       g.uniform(-0.03, 0.03, pi.size)], axis=1)
    _, grad, tau, _ = oracle.overlap_grad(off, xy, cen, pi, pj, params, SIG)
    h = 1e-3
    for m in range(3):
        e = np.zeros(3)
        e[m] = 1.0

        def fd(step):
            cp = _cost(off, xy, cen, pi, pj, params + step * e)
            cm = _cost(off, xy, cen, pi, pj, params - step * e)
            return (cp - cm) / (2 * step)

        gr = (4 * fd(h / 2) - fd(h)) / 3
        err = np.abs(grad[:, m] - gr)
        assert np.all(err <= 1e-5 * np.maximum(np.abs(gr), tau[:, m])), (m, err.max())


def test_zero_gradient_for_identical_clouds_at_identity():
    off, xy, _ = _setup(7, n=1, nmin=40, nmax=40)
    off2 = np.array([0, 40, 80], dtype=np.int64)
    xy2 = np.concatenate([xy, xy])
    cen = synth.cloud_centroids(off2, xy2)
    c, grad, tau, _ = oracle.overlap_grad(off2, xy2, cen, [0], [1], np.zeros((1, 3)), SIG)
    assert c[0] >= 40.0
    assert np.all(np.abs(grad[0]) <= 1e-12 * np.maximum(tau[0], 1.0))


# --- error floors tau_p and kappa of the gradient oracle ---------------------------------
# tau_p = sqrt(sum_kl (d term_kl / d q_p)^2) * max(1, kappa / 50) and kappa = cost-weighted
# mean exponent.  The pins below build them from per-term derivatives taken by Richardson
# central differences of single-term costs (not from the oracle's analytic gradient), so a
# wrong combination rule (a plain or absolute sum instead of the root of the squares, a
# missing kappa factor) fails.

def _moved(y, c, q):
    th, tx, ty = q
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    return R @ (y - c) + c + np.array([tx, ty])


def _term(x, y, c, q):
    u = _moved(y, c, q) - x
    return np.exp(-(u @ u) / (4 * SIG * SIG))


def _term_grad_fd(x, y, c, q, h=1e-5):
    g = np.zeros(3)
    for m in range(3):
        e = np.zeros(3)
        e[m] = 1.0

        def fd(s):
            return (_term(x, y, c, q + s * e) - _term(x, y, c, q - s * e)) / (2 * s)

        g[m] = (4 * fd(h / 2) - fd(h)) / 3
    return g


def _one_pair(X, Y, c):
    """Cloud 0 = X, cloud 1 = Y (f32-exact dyadic coordinates), centroid of cloud 1 = c."""
    off = np.array([0, len(X), len(X) + len(Y)], dtype=np.int64)
    xy = np.concatenate([X, Y]).astype(np.float32).reshape(-1)
    cen = np.array([[0.0, 0.0], c], dtype=np.float32)
    return off, xy, cen


def test_tau_and_kappa_of_a_single_term():
    x = np.array([0.5, 0.5])
    y = np.array([0.53125, 0.484375])  # dyadic: exact in f32
    c = np.array([0.5, 0.4375])        # rotation centre away from y, so d/dtheta != 0
    off, xy, cen = _one_pair([x], [y], c)
    for q in ([0.1, 0.01, -0.02], [-0.3, 0.0, 0.03], [0.0, 0.25, 0.1]):
        q = np.array(q)
        cost, grad, tau, kappa = oracle.overlap_grad(off, xy, cen, [0], [1], q[None, :], SIG)
        u = _moved(y, c, q) - x
        e = (u @ u) / (4 * SIG * SIG)
        assert abs(kappa[0] - e) <= 1e-12 * e
        gfd = _term_grad_fd(x, y, c, q)
        f = max(1.0, e / 50.0)
        for m in range(3):
            assert abs(tau[0, m] - abs(gfd[m]) * f) <= 1e-7 * abs(gfd[m]) * f + 1e-300, (q, m)
    # the last transform puts the term at exponent > 50, so the kappa factor is exercised
    assert e > 50.0


def test_tau_and_kappa_of_two_terms_with_opposite_slopes():
    # two points of cloud i on either side of the moved point: their t-derivatives have
    # opposite signs, so |g1 + g2|, |g1| + |g2| and sqrt(g1^2 + g2^2) all differ
    x1 = np.array([0.46875, 0.5])
    x2 = np.array([0.546875, 0.5078125])
    y = np.array([0.5, 0.5])
    c = np.array([0.5625, 0.4375])
    off, xy, cen = _one_pair([x1, x2], [y], c)
    q = np.array([0.05, 0.004, -0.003])
    cost, grad, tau, kappa = oracle.overlap_grad(off, xy, cen, [0], [1], q[None, :], SIG)
    w = np.array([_term(x1, y, c, q), _term(x2, y, c, q)])
    ex = np.array([(_moved(y, c, q) - xk) @ (_moved(y, c, q) - xk) / (4 * SIG * SIG) for xk in (x1, x2)])
    kap = (ex * w).sum() / w.sum()
    assert abs(kappa[0] - kap) <= 1e-12 * kap
    g1, g2 = _term_grad_fd(x1, y, c, q), _term_grad_fd(x2, y, c, q)
    assert g1[1] * g2[1] < 0  # opposite slopes in tx
    want = np.sqrt(g1 ** 2 + g2 ** 2) * max(1.0, kap / 50.0)
    np.testing.assert_allclose(tau[0], want, rtol=1e-7)
    # the gradient itself is the plain sum of the per-term derivatives
    np.testing.assert_allclose(grad[0], g1 + g2, rtol=1e-7, atol=1e-9 * np.abs(want).max())


def test_kappa_at_identity_equals_overlap_kappa():
    off, xy, cen = _setup(11, n=6, nmin=20, nmax=90)
    pi, pj = oracle.all_pairs(6)
    _, k0 = oracle.overlap(off, xy, pi, pj, SIG)
    _, _, _, k1 = oracle.overlap_grad(off, xy, cen, pi, pj, np.zeros((pi.size, 3)), SIG)
    np.testing.assert_allclose(k1, k0, rtol=1e-12, atol=0)
