"""Composition vectors of protein K-strings -- TEST INFRASTRUCTURE ONLY.

Section V-B builds each species' composition vector (CV) on the GPU from the frequency
of the length-K substrings of its protein sequences, following Qi, Wang and Hao (2004):

  f(s)   = n(s) / N_K, n(s) the number of occurrences of the K-string s over all proteins
           of the species, N_K the number of K-string positions (every window of K
           consecutive residues inside one protein);
  f0(s)  = f(s_1..s_{K-1}) f(s_2..s_K) / f(s_2..s_{K-1})   (order K-2 Markov prediction,
           the three frequencies normalised by N_{K-1}, N_{K-1}, N_{K-2});
  a(s)   = (f(s) - f0(s)) / f0(s).

The vector holds a(s) for every K-string s that occurs in the species (f(s) > 0, hence
f0(s) > 0), keyed by the base-20 code of s, keys ascending.  Residues are codes 0..19;
any other code (>= 20) ends a protein, so no window spans it.  FP64 throughout.
"""
from __future__ import annotations

import numpy as np

ALPHA = 20


def _windows(res: np.ndarray, k: int):
    """Base-20 codes of every window of k valid residues (no code >= 20 inside)."""
    res = np.asarray(res, dtype=np.int64)
    L = res.size
    if k <= 0 or L < k:
        return np.zeros(0, dtype=np.int64)
    bad = (res >= ALPHA).astype(np.int64)
    cb = np.concatenate([[0], np.cumsum(bad)])
    ok = (cb[k:] - cb[:-k]) == 0  # window starting at p holds no break
    code = np.zeros(L - k + 1, dtype=np.int64)
    for t in range(k):
        code = code * ALPHA + np.where(bad[t:L - k + 1 + t] == 1, 0, res[t:L - k + 1 + t])
    return code[ok]


def kstring_counts(res: np.ndarray, k: int):
    """(codes ascending, counts, number of positions N_k) of the k-strings of one species."""
    w = _windows(res, k)
    codes, counts = np.unique(w, return_counts=True)
    return codes, counts.astype(np.int64), int(w.size)


def composition_vector(res: np.ndarray, K: int):
    """(keys int64 ascending, a float64) of one species' composition vector."""
    if K < 3:
        raise ValueError("K >= 3")
    cK, nK, NK = kstring_counts(res, K)
    c1, n1, N1 = kstring_counts(res, K - 1)
    c2, n2, N2 = kstring_counts(res, K - 2)
    if cK.size == 0:
        return np.zeros(0, dtype=np.int64), np.zeros(0)
    pre = cK // ALPHA                    # s_1 .. s_{K-1}
    suf = cK % ALPHA ** (K - 1)          # s_2 .. s_K
    mid = (cK // ALPHA) % ALPHA ** (K - 2)  # s_2 .. s_{K-1}
    n_pre = n1[np.searchsorted(c1, pre)]
    n_suf = n1[np.searchsorted(c1, suf)]
    n_mid = n2[np.searchsorted(c2, mid)]
    f = nK / NK
    f0 = (n_pre / N1) * (n_suf / N1) / (n_mid / N2)
    return cK, (f - f0) / f0


def composition_vectors(residues: np.ndarray, offsets: np.ndarray, K: int):
    """CVs of every species (residues[offsets[s]:offsets[s+1]]) as one ragged set:
    (cv_offsets int64 [n+1], keys int64, values float64)."""
    keys, vals, off = [], [], [0]
    for s in range(offsets.size - 1):
        k, a = composition_vector(residues[offsets[s]:offsets[s + 1]], K)
        keys.append(k)
        vals.append(a)
        off.append(off[-1] + k.size)
    return (np.array(off, dtype=np.int64),
            np.concatenate(keys) if keys else np.zeros(0, np.int64),
            np.concatenate(vals) if vals else np.zeros(0))
