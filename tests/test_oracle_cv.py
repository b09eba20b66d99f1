"""Pins for the composition-vector oracle (Section V-B pre-process, Qi et al. K-string CV)."""
import os
from collections import Counter

import numpy as np
import pytest

from oracle import cv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_hand_worked_example():
    lines = [l.split() for l in open(os.path.join(GOLDEN, "cv_k3_hand.txt")) if l.strip() and l[0] != "#"]
    K = int(lines[0][1])
    res = np.array([int(v) for v in lines[1][1:]], dtype=np.uint8)
    want = [(int(a), float(b)) for a, b in lines[2:]]
    keys, vals = cv.composition_vector(res, K)
    assert list(keys) == [k for k, _ in want]
    np.testing.assert_allclose(vals, [v for _, v in want], rtol=0, atol=1e-15)


@pytest.mark.parametrize("m", [2, 3, 10, 1000])
def test_periodic_sequence_closed_form(m):
    # (AB)^m, K = 3: ABA and BAB each occur m-1 times and a = 1 / (4 m (m-1)) for both
    res = np.tile(np.array([0, 1], dtype=np.uint8), m)
    keys, vals = cv.composition_vector(res, 3)
    assert list(keys) == [0 * 400 + 1 * 20 + 0, 1 * 400 + 0 * 20 + 1]
    # a = f/f0 - 1 cancels: FP64 leaves ~1e-16 of f/f0 ~ 1 absolute
    np.testing.assert_allclose(vals, 1.0 / (4 * m * (m - 1)), rtol=1e-12, atol=1e-14)


def _brute(res, K):
    prots, cur = [], []
    for r in res:
        if r >= 20:
            prots.append(cur)
            cur = []
        else:
            cur.append(int(r))
    prots.append(cur)

    def count(k):
        c = Counter()
        for p in prots:
            for i in range(len(p) - k + 1):
                c[tuple(p[i:i + k])] += 1
        return c, sum(c.values())

    cK, NK = count(K)
    c1, N1 = count(K - 1)
    c2, N2 = count(K - 2)
    out = {}
    for s, n in cK.items():
        f = n / NK
        f0 = (c1[s[:-1]] / N1) * (c1[s[1:]] / N1) / (c2[s[1:-1]] / N2)
        code = 0
        for r in s:
            code = code * 20 + r
        out[code] = f / f0 - 1
    return out


@pytest.mark.parametrize("seed,K", [(0, 3), (1, 4), (2, 5), (3, 6)])
def test_brute_force_with_breaks(seed, K):
    g = np.random.default_rng(seed)
    res = g.integers(0, 6, 400).astype(np.uint8)  # small alphabet: many repeats
    res[g.integers(0, 400, 12)] = 255            # protein ends
    res[g.integers(0, 400, 3)] = 23              # non-standard residue codes also break
    keys, vals = cv.composition_vector(res, K)
    ref = _brute(res, K)
    assert list(keys) == sorted(ref)
    np.testing.assert_allclose(vals, [ref[k] for k in keys], rtol=1e-13, atol=1e-15)


def test_breaks_split_proteins_and_ragged_set():
    g = np.random.default_rng(4)
    a = g.integers(0, 20, 300).astype(np.uint8)
    b = g.integers(0, 20, 200).astype(np.uint8)
    joined = np.concatenate([a, [255], b])
    for k in (1, 2, 3):
        cj, nj, Nj = cv.kstring_counts(joined, k)
        ca, na, Na = cv.kstring_counts(a, k)
        cb, nb, Nb = cv.kstring_counts(b, k)
        assert Nj == Na + Nb == (300 - k + 1) + (200 - k + 1)
        tot = Counter(dict(zip(ca.tolist(), na.tolist()))) + Counter(dict(zip(cb.tolist(), nb.tolist())))
        assert dict(zip(cj.tolist(), nj.tolist())) == dict(tot)
    off = np.array([0, 300, 300, 500], dtype=np.int64)  # middle species is empty
    co, ck, cvv = cv.composition_vectors(np.concatenate([a, b]), off, 4)
    assert co[1] == co[2] and np.all(np.diff(ck[co[0]:co[1]]) > 0)
    k0, v0 = cv.composition_vector(a, 4)
    np.testing.assert_array_equal(ck[:co[1]], k0)
