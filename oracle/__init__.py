"""FP64 CPU reference for the all-pairs hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2009_04755_amd``) and never imports it.  The arithmetic lives in
``oracle.c`` (plain C, FP64, OpenMP over pairs); this module compiles it with
gcc and wraps it with ctypes.  ``plan.py`` holds the reference for the
divide-and-conquer tile split.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc -O2 -fopenmp, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        L.oracle_packed_index.argtypes = [I64, I64, I64]
        L.oracle_packed_index.restype = I64
        L.oracle_ncc_stats.argtypes = [P, I64, I64, I64, P, P]
        L.oracle_ncc_pairs.argtypes = [P, I64, I64, P, P, P, P, I64, P, P]
        L.oracle_overlap_pairs.argtypes = [P, P, D, P, P, I64, P, P]
        L.oracle_overlap_grad_pairs.argtypes = [P, P, P, D, P, P, P, I64, P, P, P, P]
        L.oracle_sparse_pairs.argtypes = [P, P, P, P, P, I64, P, P, P, P]
        L.oracle_gmm_pairs.argtypes = [P, P, P, ctypes.c_int, P, P, I64, P, P]
        L.oracle_gmm_grad_pairs.argtypes = [P, P, P, P, P, ctypes.c_int, P, P, P, I64, P, P, P, P]
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def packed_index(i: int, j: int, n: int) -> int:
    return int(lib().oracle_packed_index(i, j, n))


def all_pairs(n: int):
    """Every (i, j) with 0 <= i < j < n, in packed upper-triangle order."""
    iu = np.triu_indices(n, k=1)
    return iu[0].astype(np.int64), iu[1].astype(np.int64)


def _pairs(pi, pj):
    pi = np.ascontiguousarray(pi, dtype=np.int64)
    pj = np.ascontiguousarray(pj, dtype=np.int64)
    assert pi.shape == pj.shape
    return pi, pj


def ncc(X: np.ndarray, pi, pj, d: int | None = None):
    """(rho f64[np], tau f64[np]) for the listed pairs of rows of ``X`` (f32 [n][ld])."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, ld = X.shape
    d = ld if d is None else d
    pi, pj = _pairs(pi, pj)
    rows = np.unique(np.concatenate([pi, pj])) if pi.size else np.zeros(0, np.int64)
    mu = np.zeros(n)
    ss = np.zeros(n)
    if rows.size:
        sub = np.ascontiguousarray(X[rows])
        m2 = np.empty(rows.size)
        s2 = np.empty(rows.size)
        lib().oracle_ncc_stats(_p(sub), rows.size, d, ld, _p(m2), _p(s2))
        mu[rows] = m2
        ss[rows] = s2
    rho = np.empty(pi.size)
    tau = np.empty(pi.size)
    lib().oracle_ncc_pairs(_p(X), d, ld, _p(mu), _p(ss), _p(pi), _p(pj), pi.size, _p(rho), _p(tau))
    return rho, tau


def overlap(offsets, xy, pi, pj, sigma: float = 0.02):
    """(cost f64[np], kappa f64[np]) of the Gaussian-overlap cost for the listed pairs."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    xy = np.ascontiguousarray(xy, dtype=np.float32)
    pi, pj = _pairs(pi, pj)
    cost = np.empty(pi.size)
    kappa = np.empty(pi.size)
    lib().oracle_overlap_pairs(_p(xy), _p(offsets), float(sigma), _p(pi), _p(pj), pi.size, _p(cost), _p(kappa))
    return cost, kappa


def overlap_grad(offsets, xy, centroids, pi, pj, params, sigma: float = 0.02):
    """(cost [np], grad [np][3], tau [np][3], kappa [np]) at transforms ``params`` [np][3]."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    xy = np.ascontiguousarray(xy, dtype=np.float32)
    cen = np.ascontiguousarray(centroids, dtype=np.float32)
    params = np.ascontiguousarray(params, dtype=np.float64)
    pi, pj = _pairs(pi, pj)
    assert params.shape == (pi.size, 3)
    cost = np.empty(pi.size)
    grad = np.empty((pi.size, 3))
    tau = np.empty((pi.size, 3))
    kappa = np.empty(pi.size)
    lib().oracle_overlap_grad_pairs(_p(xy), _p(offsets), _p(cen), float(sigma), _p(pi), _p(pj), _p(params),
                                    pi.size, _p(cost), _p(grad), _p(tau), _p(kappa))
    return cost, grad, tau, kappa


def gmm(offsets, xy, sig, pi, pj, mode: str = "l2", with_kappa: bool = False):
    """Per-localisation-uncertainty mixture score for the listed pairs: ``mode='l2'`` is the
    L2 cross term sum N(x_k - y_l; 0, (s_k^2 + t_l^2) I), ``'bhattacharya'`` the sum of the
    components' Bhattacharya coefficients.  With ``with_kappa`` also the cost-weighted mean
    exponent of each pair."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    xy = np.ascontiguousarray(xy, dtype=np.float32)
    sig = np.ascontiguousarray(sig, dtype=np.float32)
    pi, pj = _pairs(pi, pj)
    cost = np.empty(pi.size)
    kappa = np.empty(pi.size)
    lib().oracle_gmm_pairs(_p(xy), _p(sig), _p(offsets), {"l2": 0, "bhattacharya": 1}[mode], _p(pi), _p(pj),
                           pi.size, _p(cost), _p(kappa))
    return (cost, kappa) if with_kappa else cost


def gmm_grad(offsets, xy, pi, pj, mode: str = "l2", sig=None, cov=None, centroids=None, params=None):
    """Per-localisation-uncertainty score with a covariance per point (``cov`` f32 [total][3]:
    xx, xy, yy) or an isotropic deviation (``sig`` f32 [total]), for the listed pairs, with
    cloud j moved by ``params`` [np][3] = (theta, tx, ty) about ``centroids[j]`` (identity when
    None).  Returns (cost [np], grad [np][3], tau [np][3], kappa [np])."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    xy = np.ascontiguousarray(xy, dtype=np.float32)
    sig = None if sig is None else np.ascontiguousarray(sig, dtype=np.float32)
    cov = None if cov is None else np.ascontiguousarray(cov, dtype=np.float32).reshape(-1)
    assert (sig is None) != (cov is None)
    pi, pj = _pairs(pi, pj)
    cen = None if centroids is None else np.ascontiguousarray(centroids, dtype=np.float32)
    prm = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
    if prm is not None:
        assert prm.shape == (pi.size, 3) and cen is not None
    cost = np.empty(pi.size)
    grad = np.empty((pi.size, 3))
    tau = np.empty((pi.size, 3))
    kappa = np.empty(pi.size)
    lib().oracle_gmm_grad_pairs(_p(xy), _p(sig), _p(cov), _p(offsets), _p(cen), {"l2": 0, "bhattacharya": 1}[mode],
                                _p(pi), _p(pj), _p(prm), pi.size, _p(cost), _p(grad), _p(tau), _p(kappa))
    return cost, grad, tau, kappa


def sparse_cosine(offsets, keys, vals, pi, pj, with_tau: bool = False):
    """(cos f64[np], count int64[np], keysum uint64[np]) for the listed pairs; with
    ``with_tau`` also the error scale tau f64[np] of each cosine."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    keys = np.ascontiguousarray(keys, dtype=np.int64)
    vals = np.ascontiguousarray(vals, dtype=np.float32)
    pi, pj = _pairs(pi, pj)
    cosv = np.empty(pi.size)
    cnt = np.empty(pi.size, dtype=np.int64)
    ks = np.empty(pi.size, dtype=np.uint64)
    tau = np.empty(pi.size) if with_tau else None
    lib().oracle_sparse_pairs(_p(keys), _p(vals), _p(offsets), _p(pi), _p(pj), pi.size, _p(cosv), _p(cnt), _p(ks),
                              _p(tau))
    return (cosv, cnt, ks, tau) if with_tau else (cosv, cnt, ks)
