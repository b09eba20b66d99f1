"""Pins for the FP64 sparse-cosine reference (Section V-B, composition-vector compare)."""
import numpy as np

import oracle
from paper_2009_04755_amd import synth


def _items(*items):
    off = np.zeros(len(items) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(k) for k, _ in items])
    keys = np.concatenate([np.asarray(k, dtype=np.int64) for k, _ in items])
    vals = np.concatenate([np.asarray(v, dtype=np.float32) for _, v in items])
    return off, keys, vals


def test_matches_set_and_dict_brute_force():
    off, keys, vals = synth.sparse_vectors(7, key_space=5000, nnz_mean=300, nnz_min=1, nnz_max=2000, config=4, salt=1)
    pi, pj = oracle.all_pairs(7)
    cosv, cnt, ks = oracle.sparse_cosine(off, keys, vals, pi, pj)
    for p in range(pi.size):
        a = dict(zip(keys[off[pi[p]]:off[pi[p] + 1]].tolist(), vals[off[pi[p]]:off[pi[p] + 1]].astype(float)))
        b = dict(zip(keys[off[pj[p]]:off[pj[p] + 1]].tolist(), vals[off[pj[p]]:off[pj[p] + 1]].astype(float)))
        shared = set(a) & set(b)
        assert cnt[p] == len(shared)
        assert int(ks[p]) == sum(shared) % 2 ** 64
        dot = sum(a[k] * b[k] for k in shared)
        ref = dot / (np.sqrt(sum(v * v for v in a.values())) * np.sqrt(sum(v * v for v in b.values())))
        assert abs(cosv[p] - ref) <= 1e-13


def test_duplicate_item_and_disjoint_items():
    off, keys, vals = _items(([1, 5, 9, 100], [0.1, 0.2, 0.3, 0.4]), ([1, 5, 9, 100], [0.1, 0.2, 0.3, 0.4]),
                             ([2, 6, 10], [1.0, 2.0, 3.0]))
    cosv, cnt, _ = oracle.sparse_cosine(off, keys, vals, [0, 0], [1, 2])
    assert abs(cosv[0] - 1.0) < 1e-15 and cnt[0] == 4
    assert cosv[1] == 0.0 and cnt[1] == 0


def test_symmetry_bounds_and_scale_invariance():
    off, keys, vals = synth.sparse_vectors(6, key_space=3000, nnz_mean=400, nnz_min=50, nnz_max=1500, config=4, salt=2)
    pi, pj = oracle.all_pairs(6)
    a, ca, _ = oracle.sparse_cosine(off, keys, vals, pi, pj)
    b, cb, _ = oracle.sparse_cosine(off, keys, vals, pj, pi)
    assert np.array_equal(ca, cb)
    np.testing.assert_allclose(a, b, rtol=1e-15)
    nnz = np.diff(off)
    assert np.all(ca <= np.minimum(nnz[pi], nnz[pj]))
    v3 = vals.copy()
    v3[off[0]:off[1]] *= 4.0  # exact power-of-two scale
    c, _, _ = oracle.sparse_cosine(off, keys, v3, pi, pj)
    assert np.array_equal(c, a)


def test_error_scale_special_cases():
    # one shared key: the cosine is a single product, so tau = |cos|
    off, keys, vals = _items(([3, 8, 20], [0.5, -0.25, 2.0]), ([8, 9], [-3.0, 1.0]))
    c, _, _, tau = oracle.sparse_cosine(off, keys, vals, [0], [1], with_tau=True)
    assert tau[0] == abs(c[0]) and c[0] > 0
    # m shared keys with equal products: Cauchy-Schwarz holds with equality, tau = cos / sqrt(m)
    off, keys, vals = _items(([1, 2, 3, 4], [1.0, 2.0, 4.0, 8.0]), ([1, 2, 3, 4], [8.0, 4.0, 2.0, 1.0]))
    c, _, _, tau = oracle.sparse_cosine(off, keys, vals, [0], [1], with_tau=True)
    assert abs(tau[0] - c[0] / 2.0) <= 1e-16 and abs(c[0] - 32.0 / 85.0) <= 1e-16
    # two products of opposite sign cancel: cos = 0 exactly while tau = sqrt(2) p / (|a||b|)
    off, keys, vals = _items(([5, 7], [1.0, 1.0]), ([5, 7], [0.5, -0.5]))
    c, _, _, tau = oracle.sparse_cosine(off, keys, vals, [0], [1], with_tau=True)
    assert c[0] == 0.0 and abs(tau[0] - np.sqrt(2) * 0.5 / (np.sqrt(2) * np.sqrt(0.5))) <= 1e-16
    # disjoint items: no products, tau = 0
    off, keys, vals = _items(([1], [1.0]), ([2], [1.0]))
    _, _, _, tau = oracle.sparse_cosine(off, keys, vals, [0], [1], with_tau=True)
    assert tau[0] == 0.0


def test_error_scale_bounds_for_one_sign():
    # for non-negative values tau lies in [cos / sqrt(m), cos]; a missed square root, a
    # dropped norm or a sum of |products| breaks one of the bounds on these inputs
    off, keys, vals = synth.sparse_vectors(8, key_space=4000, nnz_mean=500, nnz_min=20, nnz_max=1500, config=4, salt=3)
    pi, pj = oracle.all_pairs(8)
    c, m, _, tau = oracle.sparse_cosine(off, keys, vals, pi, pj, with_tau=True)
    ok = m > 1
    assert ok.sum() > 10
    assert np.all(tau[ok] <= c[ok] * (1 + 1e-12))
    assert np.all(tau[ok] >= c[ok] / np.sqrt(m[ok]) * (1 - 1e-12))
    assert np.all(tau[ok] < c[ok] * 0.999)  # strictly inside: more than one product contributes
