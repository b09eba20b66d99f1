"""Peak-to-correlation energy over all cyclic shifts -- TEST INFRASTRUCTURE ONLY.

The forensics application compares camera noise patterns; its PCE variant (Section V-A
names the comparison metric, the stage table names PCE) correlates two patterns over all
cyclic 2-D shifts and scores the sharpness of the highest peak:

  C(s)  = sum_x a(x + s) b(x)              (a, b: H x W items minus their means; row
                                            index mod H, column index mod W)
  s*    = argmax_s C(s)                     (first in row-major order on ties)
  PCE   = C(s*)^2 (H W - |N|) / sum_{s not in N} C(s)^2,

N the (2h+1) x (2h+1) cyclic neighbourhood of s* (h = 5 by default).  C is evaluated as
the inverse FFT of A conj(B) (numpy FFT, FP64).
"""
from __future__ import annotations

import numpy as np


def correlation(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """C[s] = sum_x a(x+s) b(x) over cyclic shifts, both items mean-removed, FP64."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    a = a - a.mean()
    b = b - b.mean()
    return np.real(np.fft.ifft2(np.fft.fft2(a) * np.conj(np.fft.fft2(b))))


def pce_of_surface(C: np.ndarray, h: int = 5, peak=None):
    """(pce, peak index) of a correlation surface; ``peak`` forces the peak location."""
    L0, L1 = C.shape
    p = int(np.argmax(C)) if peak is None else int(peak)
    r, c = divmod(p, L1)
    dr = np.minimum((np.arange(L0) - r) % L0, (r - np.arange(L0)) % L0)
    dc = np.minimum((np.arange(L1) - c) % L1, (c - np.arange(L1)) % L1)
    inside = (dr[:, None] <= h) & (dc[None, :] <= h)
    rest = float(np.sum(C[~inside] ** 2))
    num = float(C[r, c]) ** 2 * (C.size - int(inside.sum()))
    return (num / rest if rest > 0 else float("nan")), p


def pce(a: np.ndarray, b: np.ndarray, h: int = 5, peak=None):
    return pce_of_surface(correlation(a, b), h, peak)


def pce_pairs(X: np.ndarray, L, pi, pj, h: int = 5):
    """(pce float64 [np], peak int64 [np]) for the listed pairs of items X[k]: L x L values
    (L an int) or H x W values (L a pair (H, W)), row-major."""
    H, W = (L, L) if np.isscalar(L) else (int(L[0]), int(L[1]))
    X = np.asarray(X, dtype=np.float32)
    out = np.empty(len(pi))
    pk = np.empty(len(pi), dtype=np.int64)
    for t, (i, j) in enumerate(zip(pi, pj)):
        out[t], pk[t] = pce(X[i].reshape(H, W), X[j].reshape(H, W), h)
    return out, pk
