"""Seeded synthetic inputs for the three all-pairs workloads.

This module only draws random inputs.  It holds none of the pair-function
arithmetic: the FP64 checker and the GPU library both consume these arrays,
and neither imports the other.  Every stream comes from
``numpy.random.PCG64(SeedSequence([20090475, config, salt]))`` (or, for the
multi-GiB dense workload, from a seeded ``torch.Generator`` on the device), so
the same arguments always give the same bytes.

Workload shapes follow the three applications of the paper (Section V):
dense noise-pattern vectors (forensics, NCC), 2-D localisation point clouds
(microscopy, Gaussian-mixture registration cost) and sparse k-mer composition
vectors (bioinformatics, cosine of sparse vectors).  The datasets the paper
used are not available; these generators stand in for them.
"""
from __future__ import annotations

import hashlib

import numpy as np

SEED_BASE = 20090475


def rng(config: int, salt: int = 0) -> np.random.Generator:
    """The PCG64 stream for workload ``config`` (0..4) and an optional salt."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, int(config), int(salt)])))


def sha256(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


# --------------------------------------------------------------------------------------------
# Dense noise patterns (forensics stand-in)
# --------------------------------------------------------------------------------------------

def dense_patterns(n: int, d: int, nsrc: int, amp: float, assign: str = "mod", config: int = 0,
                   salt: int = 0, normalise: bool = True):
    """Items ``amp * source[c_i] + N(0,1)`` with ``nsrc`` shared N(0,1) sources.

    ``assign='mod'`` uses ``c_i = i mod nsrc``; ``'uniform'`` draws ``c_i`` uniformly.
    With ``normalise`` each row is then made zero-mean and unit-norm (FP64, stored f32),
    as the workload recipe states.  Returns ``(X f32[n][d], c int64[n])``.
    """
    g = rng(config, salt)
    src = g.standard_normal((nsrc, d))
    if assign == "mod":
        c = np.arange(n, dtype=np.int64) % nsrc
    elif assign == "uniform":
        c = g.integers(0, nsrc, n).astype(np.int64)
    else:
        raise ValueError(assign)
    X = amp * src[c] + g.standard_normal((n, d))
    if normalise:
        X -= X.mean(axis=1, keepdims=True)
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    return X.astype(np.float32), c


def dense_patterns_device(n: int, d: int, nsrc: int, amp: float, seed: int, device, rows_per_chunk: int = 128):
    """Device-side generator for multi-GiB dense workloads (same recipe, ``assign='uniform'``).

    Uses a seeded ``torch.Generator`` on ``device``; rows are drawn and normalised in
    chunks so that the FP64 temporaries stay small.  Returns ``(X f32[n][d] on device,
    c int64[n] on host)``.
    """
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(SEED_BASE * 1000 + int(seed))
    src = torch.randn((nsrc, d), generator=g, device=device, dtype=torch.float32)
    c = torch.randint(0, nsrc, (n,), generator=g, device=device)
    X = torch.empty((n, d), device=device, dtype=torch.float32)
    for r0 in range(0, n, rows_per_chunk):
        r1 = min(n, r0 + rows_per_chunk)
        noise = torch.randn((r1 - r0, d), generator=g, device=device, dtype=torch.float32)
        blk = amp * src[c[r0:r1]].to(torch.float64) + noise.to(torch.float64)
        blk -= blk.mean(dim=1, keepdim=True)
        blk /= torch.linalg.vector_norm(blk, dim=1, keepdim=True)
        X[r0:r1] = blk.to(torch.float32)
        del noise, blk
    return X, c.cpu().numpy()


# --------------------------------------------------------------------------------------------
# 2-D point clouds (localisation-microscopy stand-in)
# --------------------------------------------------------------------------------------------

def point_clouds(n: int, nmin: int = 50, nmax: int = 400, nsites: int = 40, p_keep: float = 0.7,
                 jitter: float = 0.01, config: int = 2, salt: int = 0):
    """Uneven 2-D clouds: repeated localisations of a shared random site template.

    A template of ``nsites`` sites is drawn once in the unit square.  Each cloud keeps
    every site with probability ``p_keep`` (redrawn if none survives), draws its point
    count uniformly in ``[nmin, nmax]``, places each point on a uniformly chosen kept
    site plus N(0, jitter^2) per coordinate, then rotates by U[0, 2pi) about (0.5, 0.5)
    and translates by U[-0.5, 0.5]^2.  Returns ``(offsets int64[n+1], xy f32[2*total])``
    with coordinates interleaved (x0, y0, x1, y1, ...).
    """
    g = rng(config, salt)
    sites = g.random((nsites, 2))
    counts = g.integers(nmin, nmax + 1, n).astype(np.int64)
    offsets = np.zeros(n + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    xy = np.empty((int(offsets[-1]), 2), dtype=np.float64)
    for i in range(n):
        keep = g.random(nsites) < p_keep
        while not keep.any():
            keep = g.random(nsites) < p_keep
        kept = sites[keep]
        pick = g.integers(0, kept.shape[0], counts[i])
        pts = kept[pick] + jitter * g.standard_normal((counts[i], 2))
        th = g.random() * 2.0 * np.pi
        t = g.random(2) - 0.5
        c, s = np.cos(th), np.sin(th)
        rel = pts - 0.5
        rot = np.stack([c * rel[:, 0] - s * rel[:, 1], s * rel[:, 0] + c * rel[:, 1]], axis=1)
        xy[offsets[i]:offsets[i + 1]] = rot + 0.5 + t
    return offsets, xy.astype(np.float32).reshape(-1)


def cloud_centroids(offsets: np.ndarray, xy: np.ndarray) -> np.ndarray:
    """Per-cloud centroid (FP64 mean, stored f32): the rotation centre handed to the
    registration gradient as an explicit input.  Empty clouds get (0, 0)."""
    n = offsets.shape[0] - 1
    pts = xy.reshape(-1, 2).astype(np.float64)
    out = np.zeros((n, 2), dtype=np.float64)
    for i in range(n):
        a, b = offsets[i], offsets[i + 1]
        if b > a:
            out[i] = pts[a:b].mean(axis=0)
    return out.astype(np.float32)


def point_sigmas(offsets: np.ndarray, lo: float = 0.01, hi: float = 0.03, config: int = 2, salt: int = 0):
    """Per-localisation uncertainty sigma_k ~ U[lo, hi] (f32), one per point."""
    g = rng(config, 500 + salt)
    return g.uniform(lo, hi, int(offsets[-1])).astype(np.float32)


def point_covs(offsets: np.ndarray, lo: float = 0.01, hi: float = 0.03, config: int = 2, salt: int = 0):
    """Per-localisation uncertainty ellipse as a full covariance (xx, xy, yy) per point (f32
    [total][3]): semi-axes ~ U[lo, hi] each, orientation ~ U[0, pi)."""
    g = rng(config, 700 + salt)
    m = int(offsets[-1])
    a, b = g.uniform(lo, hi, m), g.uniform(lo, hi, m)
    th = g.uniform(0.0, np.pi, m)
    c, s = np.cos(th), np.sin(th)
    xx = c * c * a * a + s * s * b * b
    yy = s * s * a * a + c * c * b * b
    xy = c * s * (a * a - b * b)
    return np.stack([xx, xy, yy], axis=1).astype(np.float32)


def rigid_starts(npairs: int, config: int = 3, salt: int = 0) -> np.ndarray:
    """Per-pair start transform (theta, tx, ty): theta ~ U[-pi, pi), t ~ U[-0.5, 0.5]^2."""
    g = rng(config, salt)
    p = np.empty((npairs, 3), dtype=np.float64)
    p[:, 0] = (g.random(npairs) * 2.0 - 1.0) * np.pi
    p[:, 1:] = g.random((npairs, 2)) - 0.5
    return p.astype(np.float32)


# --------------------------------------------------------------------------------------------
# Sparse k-mer composition vectors (bioinformatics stand-in)
# --------------------------------------------------------------------------------------------

def _zipf_ranks(g: np.random.Generator, a: float, rmax: int, size: int) -> np.ndarray:
    """Zipf(a) ranks truncated to [1, rmax] by rejection."""
    out = np.empty(0, dtype=np.int64)
    while out.size < size:
        r = g.zipf(a, size=max(1024, int((size - out.size) * 1.3)))
        r = r[r <= rmax]
        out = np.concatenate([out, r.astype(np.int64)])
    return out[:size]


def sparse_vectors(n: int, key_space: int = 20 ** 6, zipf_a: float = 1.1, nnz_mean: float = 200_000,
                   nnz_min: int = 20_000, nnz_max: int = 1_000_000, sigma_ln: float = 1.0,
                   config: int = 4, salt: int = 0):
    """Sparse frequency vectors over ``key_space`` int64 keys.

    nnz_i ~ LogNormal(ln(nnz_mean) - sigma_ln^2/2, sigma_ln) rounded and clipped to
    [nnz_min, nnz_max].  Zipf(``zipf_a``) ranks truncated to the key space are drawn
    until nnz_i distinct ranks have appeared; each rank r maps to key (a*r + b) mod
    key_space with a seeded multiplier coprime to the key space, so popular keys spread
    over the whole range.  A key's value is its draw count divided by the number of
    draws (FP64, stored f32), so each vector sums to 1.  Keys are strictly ascending per
    item.  Returns ``(offsets int64[n+1], keys int64[total], vals f32[total])``.
    """
    g = rng(config, salt)
    mu = np.log(nnz_mean) - 0.5 * sigma_ln ** 2
    nnz = np.clip(np.rint(g.lognormal(mu, sigma_ln, n)), nnz_min, nnz_max).astype(np.int64)
    nnz = np.minimum(nnz, key_space)
    while True:
        mult = int(g.integers(1, key_space))
        if np.gcd(mult, key_space) == 1:
            break
    add = int(g.integers(0, key_space))
    offsets = np.zeros(n + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(nnz)
    keys = np.empty(int(offsets[-1]), dtype=np.int64)
    vals = np.empty(int(offsets[-1]), dtype=np.float32)
    for i in range(n):
        want = int(nnz[i])
        draws = np.empty(0, dtype=np.int64)
        batch = max(4 * want, 4096)
        while True:
            draws = np.concatenate([draws, _zipf_ranks(g, zipf_a, key_space, batch)])
            uniq, first = np.unique(draws, return_index=True)
            if uniq.size >= want:
                cut = np.sort(first)[want - 1]
                draws = draws[: cut + 1]
                break
            batch *= 2
        ranks, cnt = np.unique(draws, return_counts=True)
        k = (mult * (ranks - 1) + add) % key_space
        order = np.argsort(k, kind="stable")
        a, b = offsets[i], offsets[i + 1]
        keys[a:b] = k[order]
        vals[a:b] = (cnt[order].astype(np.float64) / float(draws.size)).astype(np.float32)
    return offsets, keys, vals


def sparse_vectors_device(n: int, key_space: int = 20 ** 6, zipf_a: float = 1.1, nnz_mean: float = 200_000,
                          nnz_min: int = 20_000, nnz_max: int = 1_000_000, sigma_ln: float = 1.0, seed: int = 0,
                          device="cuda"):
    """Device-side version of :func:`sparse_vectors` for multi-GB sets (same recipe).

    nnz and the key bijection come from the host PCG64 stream; Zipf ranks are drawn on the
    device by inverse-CDF lookup in the truncated distribution's FP64 CDF (summed on the
    host), from a seeded ``torch.Generator``.  Returns device tensors ``(offsets int64[n+1], keys int64[total],
    vals f32[total])``.
    """
    import torch

    g = rng(4, 1000 + seed)
    mu = np.log(nnz_mean) - 0.5 * sigma_ln ** 2
    nnz = np.clip(np.rint(g.lognormal(mu, sigma_ln, n)), nnz_min, nnz_max).astype(np.int64)
    nnz = np.minimum(nnz, key_space)
    while True:
        mult = int(g.integers(1, key_space))
        if np.gcd(mult, key_space) == 1:
            break
    add = int(g.integers(0, key_space))
    tg = torch.Generator(device=device)
    tg.manual_seed(SEED_BASE * 1000 + 4000 + int(seed))
    # the truncated Zipf CDF by a sequential host sum (a parallel device scan need not give
    # the same last bits on every run, and a last-bit change moves a rare draw)
    c = np.cumsum(np.arange(1, key_space + 1, dtype=np.float64) ** -zipf_a)
    c /= c[-1]
    cdf = torch.from_numpy(c).to(device)
    del c
    offsets = np.zeros(n + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(nnz)
    keys = torch.empty(int(offsets[-1]), dtype=torch.int64, device=device)
    vals = torch.empty(int(offsets[-1]), dtype=torch.float32, device=device)
    for i in range(n):
        want = int(nnz[i])
        draws = torch.empty(0, dtype=torch.int64, device=device)
        batch = 6 * want + 4096
        while True:
            u = torch.rand(batch, generator=tg, device=device, dtype=torch.float64)
            r = torch.searchsorted(cdf, u).clamp_(max=key_space - 1)  # rank - 1
            draws = torch.cat([draws, r])
            uniq, inv = torch.unique(draws, return_inverse=True)
            if uniq.numel() >= want:
                pos = torch.arange(draws.numel(), device=device)
                first = torch.full((uniq.numel(),), draws.numel(), dtype=torch.int64, device=device)
                first.scatter_reduce_(0, inv, pos, reduce="amin")
                cut = int(torch.kthvalue(first, want).values)
                draws = draws[: cut + 1]
                break
            batch *= 2
        rk, cnt = torch.unique(draws, return_counts=True)
        k = (mult * rk + add) % key_space
        order = torch.argsort(k)
        a, b = int(offsets[i]), int(offsets[i + 1])
        keys[a:b] = k[order]
        vals[a:b] = (cnt[order].to(torch.float64) / float(draws.numel())).to(torch.float32)
    return torch.from_numpy(offsets).to(device), keys, vals


def proteomes(n: int, n_families: int = 4000, len_min: int = 100, len_max: int = 500, p_keep: float = 0.7,
              rate_min: float = 0.05, rate_max: float = 0.6, config: int = 5, salt: int = 0):
    """Synthetic proteomes standing in for bacterial reference proteomes.

    A pool of ``n_families`` ancestral proteins (lengths U{len_min..len_max}, residues
    drawn from a seeded background distribution over the 20 amino-acid codes 0..19) is
    shared by all species; species s keeps each family with probability ``p_keep`` and
    substitutes each residue with probability rate_s ~ U[rate_min, rate_max] by a fresh
    background draw.  Proteins are concatenated with the code 255 after each one.
    Returns (residues uint8, offsets int64 [n+1]) with species s at offsets[s]..offsets[s+1]-1.
    """
    g = rng(config, salt)
    bg = g.dirichlet(np.full(20, 8.0))
    lens = g.integers(len_min, len_max + 1, n_families)
    pool = g.choice(20, size=int(lens.sum()), p=bg).astype(np.uint8)
    starts = np.concatenate([[0], np.cumsum(lens)])
    parts, off = [], [0]
    for s in range(n):
        keep = np.nonzero(g.random(n_families) < p_keep)[0]
        rate = g.uniform(rate_min, rate_max)
        seq = []
        for f in keep:
            seq.append(pool[starts[f]:starts[f + 1]])
            seq.append(np.array([255], dtype=np.uint8))
        sp = np.concatenate(seq) if seq else np.zeros(0, np.uint8)
        mut = (g.random(sp.size) < rate) & (sp != 255)
        sp = sp.copy()
        sp[mut] = g.choice(20, size=int(mut.sum()), p=bg).astype(np.uint8)
        parts.append(sp)
        off.append(off[-1] + sp.size)
    return np.concatenate(parts) if parts else np.zeros(0, np.uint8), np.array(off, dtype=np.int64)


def noise_images(n: int, L, nsrc: int = 8, amp: float = 0.05, p_shift: float = 0.25, config: int = 6,
                 salt: int = 0):
    """Camera-noise-like images of L x L (L an int) or H x W (L a pair) values, flattened
    row-major (f32 [n][H*W]): item = amp * source[c] + N(0, 1) with c uniform over ``nsrc``
    N(0, 1) sources; with probability ``p_shift`` the source is cyclically shifted by a
    uniform (dy, dx) (a crop taken at another offset).
    Returns (images, source index, shift (dy, dx) per item)."""
    H, W = (L, L) if np.isscalar(L) else (int(L[0]), int(L[1]))
    g = rng(config, salt)
    src = g.standard_normal((nsrc, H, W))
    c = g.integers(0, nsrc, n)
    shifted = g.random(n) < p_shift
    sh = np.where(shifted[:, None], np.stack([g.integers(0, H, n), g.integers(0, W, n)], axis=1), 0) \
        if H != W else np.where(shifted[:, None], g.integers(0, H, (n, 2)), 0)
    X = np.empty((n, H * W), dtype=np.float32)
    for i in range(n):
        s = np.roll(src[c[i]], (int(sh[i, 0]), int(sh[i, 1])), axis=(0, 1))
        X[i] = (amp * s + g.standard_normal((H, W))).reshape(-1)
    return X, c, sh
