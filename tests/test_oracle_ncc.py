"""Pins for the FP64 NCC reference (zero-lag Pearson correlation, Section V-A)."""
import numpy as np
import pytest

import oracle
from paper_2009_04755_amd import synth


def test_matches_numpy_corrcoef():
    g = np.random.default_rng(1)
    for n, d in [(2, 5), (5, 17), (8, 64)]:
        X = (g.standard_normal((n, d)) * g.uniform(0.1, 10, (n, 1)) + g.uniform(-5, 5, (n, 1))).astype(np.float32)
        pi, pj = oracle.all_pairs(n)
        rho, _ = oracle.ncc(X, pi, pj)
        ref = np.corrcoef(X.astype(np.float64))[pi, pj]
        np.testing.assert_allclose(rho, ref, rtol=0, atol=1e-12)


def test_self_correlation_is_one_and_bounded():
    X, _ = synth.dense_patterns(16, 300, 4, 0.5, config=0, salt=7)
    idx = np.arange(16)
    rho, _ = oracle.ncc(X, idx, idx)
    np.testing.assert_allclose(rho, 1.0, rtol=0, atol=1e-14)
    pi, pj = oracle.all_pairs(16)
    rho, _ = oracle.ncc(X, pi, pj)
    assert np.all(np.abs(rho) <= 1.0)


def test_symmetry():
    X, _ = synth.dense_patterns(12, 257, 3, 0.3, config=0, salt=3)
    pi, pj = oracle.all_pairs(12)
    a, ta = oracle.ncc(X, pi, pj)
    b, tb = oracle.ncc(X, pj, pi)
    assert np.array_equal(a, b)
    np.testing.assert_allclose(ta, tb, rtol=1e-14)


def test_affine_invariance_exact():
    # small-integer data: 3a+7 and -2a+1 are exact in f32, so rho must not move
    g = np.random.default_rng(5)
    A = g.integers(-50, 50, (4, 101)).astype(np.float32)
    B = np.concatenate([A, 3 * A[:1] + 7, -2 * A[:1] + 1]).astype(np.float32)
    r, _ = oracle.ncc(B, np.array([0, 4, 5]), np.array([1, 1, 1]))
    assert abs(r[0] - r[1]) < 1e-14
    assert abs(r[0] + r[2]) < 1e-14


def test_tau_of_balanced_sign_vectors():
    # +-1 vectors with zero mean: every centred, normalised entry is +-1/sqrt(d),
    # so tau = sqrt(sum 1/d^2) = 1/sqrt(d)
    d = 256
    g = np.random.default_rng(9)
    rows = []
    for _ in range(3):
        v = np.array([1.0] * (d // 2) + [-1.0] * (d // 2))
        g.shuffle(v)
        rows.append(v)
    X = np.array(rows, dtype=np.float32)
    _, tau = oracle.ncc(X, np.array([0, 0, 1]), np.array([1, 2, 2]))
    np.testing.assert_allclose(tau, 1.0 / np.sqrt(d), rtol=1e-14)


def test_zero_variance_gives_nan():
    X = np.ones((2, 10), dtype=np.float32)
    X[1] = np.arange(10)
    rho, _ = oracle.ncc(X, np.array([0]), np.array([1]))
    assert np.isnan(rho[0])


def test_generator_same_source_mean():
    # items amp*src[c] + N(0,1): same-source pairs correlate with mean amp^2/(1+amp^2),
    # cross-source pairs with mean 0 (4096-long patterns, 256 items, 8 sources)
    n, d, nsrc, amp = 256, 4096, 8, 0.05
    X, c = synth.dense_patterns(n, d, nsrc, amp, assign="mod", config=0)
    pi, pj = oracle.all_pairs(n)
    rho, _ = oracle.ncc(X, pi, pj)
    same = c[pi] == c[pj]
    expect = amp ** 2 / (1 + amp ** 2)
    se_same = rho[same].std() / np.sqrt(same.sum()) * 1.5
    se_cross = rho[~same].std() / np.sqrt((~same).sum()) * 1.5
    assert abs(rho[same].mean() - expect) < 5 * se_same
    assert abs(rho[~same].mean()) < 5 * se_cross
    # spread at the noise floor, 1/sqrt(d)
    assert 0.8 / np.sqrt(d) < rho[~same].std() < 1.2 / np.sqrt(d)
