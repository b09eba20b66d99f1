"""Python binding over the C ABI: torch tensors in, torch tensors out.

PyTorch provides device memory, streams and autograd only; every step of the
all-pairs evaluation runs in the HIP library.  Work is enqueued on
``torch.cuda.current_stream()``.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib

NCC_FNS = ("ncc_fp32", "ncc_bf16x3", "ncc_bf16x6")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def num_pairs(n: int) -> int:
    return n * (n - 1) // 2


@dataclass
class Clouds:
    """Ragged 2-D point clouds: cloud i owns points offsets[i] .. offsets[i+1]-1 of xy.

    ``sigma`` is the common scale of ``gauss_overlap``; ``point_sigma`` the per-point
    standard deviation read by ``gmm_l2`` and ``gmm_bhattacharya``; ``point_cov`` a full
    covariance (xx, xy, yy) per point for the same two scores (used instead of
    ``point_sigma`` when given)."""
    offsets: torch.Tensor  # int64 [n+1], device
    xy: torch.Tensor       # float32 [2 * total] interleaved (x, y), device
    sigma: float = 0.02
    point_sigma: torch.Tensor | None = None  # float32 [total], device
    point_cov: torch.Tensor | None = None    # float32 [total][3] (or [3 * total]), device

    @property
    def n(self) -> int:
        return self.offsets.numel() - 1


@dataclass
class SparseSet:
    """Ragged sparse vectors: item i owns keys/vals offsets[i] .. offsets[i+1]-1."""
    offsets: torch.Tensor  # int64 [n+1], device
    keys: torch.Tensor     # int64 [total], strictly ascending per item, device
    vals: torch.Tensor     # float32 [total], device

    @property
    def n(self) -> int:
        return self.offsets.numel() - 1


def _check_dev(t, name: str, dtype, device: int, contiguous: bool = True):
    """Check that ``t`` can be handed to the C ABI as a device pointer on ``device``: a
    torch tensor of ``dtype`` on that device (and contiguous when the layout is packed).
    Raises before any pointer reaches the library."""
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor, got %s" % (name, type(t).__name__))
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor (got one on %s)" % (name, t.device))
    if t.device.index != device:
        raise ValueError("%s is on %s but the context is on cuda:%d" % (name, t.device, device))
    if contiguous and not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _items_struct(x, fn: int, device: int):
    """The rocket_items struct for ``x`` and its item count, after checking every tensor."""
    it = _lib.Items()
    if fn in (_lib.NCC_FP32, _lib.NCC_BF16X3, _lib.NCC_BF16X6, _lib.PCE):
        _check_dev(x, "items", torch.float32, device, contiguous=False)
        if x.dim() != 2 or (x.shape[0] > 1 and x.stride(1) != 1) or (x.shape[0] > 1 and x.stride(0) < x.shape[1]):
            raise ValueError("dense items must be a 2-D [n][d] tensor with unit column stride and rows "
                             "at least d apart")
        it.dense = x.data_ptr()
        it.dim = x.shape[1]
        it.ld = x.stride(0) if x.shape[0] > 1 else x.shape[1]
        return it, x.shape[0]
    if fn in (_lib.GAUSS_OVERLAP, _lib.GMM_L2, _lib.GMM_BHATTACHARYA):
        if not isinstance(x, Clouds):
            raise TypeError("point-cloud pair functions take a Clouds set")
        _check_dev(x.offsets, "offsets", torch.int64, device)
        _check_dev(x.xy, "xy", torch.float32, device)
        it.offsets = x.offsets.data_ptr()
        it.xy = x.xy.data_ptr()
        it.sigma = float(x.sigma)
        if fn != _lib.GAUSS_OVERLAP and x.point_sigma is not None:
            ps = _check_dev(x.point_sigma, "point_sigma", torch.float32, device)
            if ps.numel() * 2 != x.xy.numel():
                raise ValueError("point_sigma must hold one value per point")
            it.point_sigma = ps.data_ptr()
        if fn != _lib.GAUSS_OVERLAP and x.point_cov is not None:
            pc = _check_dev(x.point_cov, "point_cov", torch.float32, device)
            if pc.numel() * 2 != 3 * x.xy.numel():
                raise ValueError("point_cov must hold three values (xx, xy, yy) per point")
            it.point_cov = pc.data_ptr()
        return it, x.n
    if fn == _lib.SPARSE_COSINE:
        if not isinstance(x, SparseSet):
            raise TypeError("sparse_cosine takes a SparseSet")
        _check_dev(x.offsets, "offsets", torch.int64, device)
        _check_dev(x.keys, "keys", torch.int64, device)
        _check_dev(x.vals, "vals", torch.float32, device)
        if x.keys.numel() != x.vals.numel():
            raise ValueError("keys and vals must have the same length")
        it.offsets = x.offsets.data_ptr()
        it.keys = x.keys.data_ptr()
        it.vals = x.vals.data_ptr()
        return it, x.n
    raise ValueError(fn)


class Context:
    """One ``rocket_ctx``: workspace, plan cache and options on one device."""

    def __init__(self, device=None):
        L = _lib.load()
        dev = torch.cuda.current_device() if device is None else torch.device(device).index or 0
        self.device = dev
        h = ctypes.c_void_p()
        _lib.check(L.rocket_create(ctypes.byref(h), dev))
        self.handle = h
        self._n = 0

    def close(self):
        if self.handle:
            _lib.load().rocket_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set(self, **opts):
        L = _lib.load()
        for k, v in opts.items():
            _lib.check(L.rocket_set_option(self.handle, _lib.OPT[k], int(v)), self.handle)
        return self

    def get(self, name: str) -> int:
        v = ctypes.c_int64()
        _lib.check(_lib.load().rocket_get_option(self.handle, _lib.OPT[name], ctypes.byref(v)), self.handle)
        return v.value

    def stats(self) -> dict:
        s = _lib.Stats()
        _lib.check(_lib.load().rocket_get_stats(self.handle, ctypes.byref(s)), self.handle)
        return {name: getattr(s, name) for name, _ in _lib.Stats._fields_}

    def ledger(self):
        import numpy as np
        L = _lib.load()
        cnt = ctypes.c_int64()
        _lib.check(L.rocket_get_ledger(self.handle, None, 0, ctypes.byref(cnt)), self.handle)
        out = np.zeros(cnt.value, dtype=np.int32)
        _lib.check(L.rocket_get_ledger(self.handle, out.ctypes.data_as(ctypes.c_void_p), cnt.value,
                                       ctypes.byref(cnt)), self.handle)
        return out

    def trace(self):
        """Per-tile trace of the last compare (option ``trace`` set before prepare): a numpy
        structured array with tile_i, tile_j, chunk, workgroup, start_ns, end_ns per work item."""
        import numpy as np
        L = _lib.load()
        cnt = ctypes.c_int64()
        _lib.check(L.rocket_get_trace(self.handle, None, 0, ctypes.byref(cnt)), self.handle)
        dt = np.dtype([("tile_i", np.int32), ("tile_j", np.int32), ("chunk", np.int32), ("workgroup", np.int32),
                       ("start_ns", np.int64), ("end_ns", np.int64)])
        assert dt.itemsize == ctypes.sizeof(_lib.TraceRec)
        out = np.zeros(cnt.value, dtype=dt)
        _lib.check(L.rocket_get_trace(self.handle, out.ctypes.data_as(ctypes.c_void_p), cnt.value, ctypes.byref(cnt)),
                   self.handle)
        return out

    # -- items ----------------------------------------------------------------------------
    def _dev(self, t, name: str, dtype, contiguous: bool = True):
        return _check_dev(t, name, dtype, self.device, contiguous)

    def _items(self, x, fn: int):
        return _items_struct(x, fn, self.device)

    def prepare(self, x, fn: str):
        code = _lib.FN_BY_NAME[fn]
        it, n = self._items(x, code)
        self._keep = (x, it)
        _lib.check(_lib.load().rocket_prepare(self.handle, ctypes.byref(it), n, code, _stream()), self.handle)
        self._n = n
        self._fn = fn
        return self

    def compare(self, out=None, counts: bool = False):
        n = self._n
        P = num_pairs(n)
        dev = torch.device("cuda", self.device)
        if out is None:
            out = torch.empty(P, dtype=torch.float32, device=dev)
        cnt = torch.empty(P, dtype=torch.int32, device=dev) if counts else None
        _lib.check(_lib.load().rocket_compare(self.handle, _ptr(out), _ptr(cnt), _stream()), self.handle)
        return (out, cnt) if counts else out

    def allpairs(self, x, fn: str, out=None, counts: bool = False):
        self.prepare(x, fn)
        return self.compare(out=out, counts=counts)

    def allpairs_host(self, x, fn: str = "ncc_bf16x6", out=None):
        """All pairs of NCC items kept in host memory (float32 [n][d] CPU tensor, ideally
        pinned) through the device cache; ``set(cache_slots=S)`` bounds the cache."""
        code = _lib.FN_BY_NAME[fn]
        if not isinstance(x, torch.Tensor) or x.is_cuda or x.dtype != torch.float32 or x.dim() != 2:
            raise ValueError("host items must be a float32 [n][d] CPU tensor")
        if x.shape[0] > 1 and (x.stride(1) != 1 or x.stride(0) < x.shape[1]):
            raise ValueError("host items need unit column stride and rows at least d apart")
        n, d = x.shape
        ld = x.stride(0) if n > 1 else d
        if out is None:
            out = torch.empty(num_pairs(n), dtype=torch.float32, device=torch.device("cuda", self.device))
        self._keep = (x,)
        self._n = 0  # no prepared set remains
        _lib.check(_lib.load().rocket_allpairs_host(self.handle, ctypes.c_void_p(x.data_ptr()), n, d, ld, code,
                                                    _ptr(out), _stream()), self.handle)
        return out

    def cv_build(self, residues, offsets, K: int = 6):
        """Composition vectors of n species (uint8 residue codes on the device, int64
        offsets [n+1]) as a :class:`SparseSet` ready for ``sparse_cosine``."""
        self._dev(residues, "residues", torch.uint8)
        self._dev(offsets, "offsets", torch.int64)
        n = offsets.numel() - 1
        cap = max(int(residues.numel()), 1)
        dev = residues.device
        cv_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
        keys = torch.empty(cap, dtype=torch.int64, device=dev)
        vals = torch.empty(cap, dtype=torch.float32, device=dev)
        _lib.check(_lib.load().rocket_cv_build(self.handle, _ptr(residues), _ptr(offsets), n, K, _ptr(cv_off),
                                               _ptr(keys), _ptr(vals), cap, _stream()), self.handle)
        total = int(cv_off[-1].item()) if n > 0 else 0
        return SparseSet(cv_off, keys[:total], vals[:total])

    def autotune(self):
        """Tune the tile shape of the prepared set (cached when a cache file is set); returns
        the options it chose and the tuning time."""
        _lib.check(_lib.load().rocket_autotune(self.handle, _stream()), self.handle)
        names = {"ncc": ("ncc_tile", "ncc_waves", "ncc_kchunk"), "sparse_cosine": ("sp_lanes", "sp_chunk")}
        fn = getattr(self, "_fn", "")
        keys = names["ncc"] if fn.startswith("ncc") else names.get(fn, ("ovl_block", "ovl_variant"))
        st = self.stats()
        out = {k: self.get(k) for k in keys}
        out.update(tune_ms=st["tune_us"] / 1e3, cached=bool(st["tune_cached"]))
        return out

    def set_tune_cache(self, path: str | None):
        """Autotuner cache file (JSON); None disables it."""
        _lib.check(_lib.load().rocket_set_tune_cache(self.handle, path.encode() if path else None), self.handle)
        return self

    def cost_grad(self, clouds: Clouds, centroids, params, fn: str = "gauss_overlap", with_grad: bool = True,
                  reuse: bool = False):
        """Score of every pair with the second cloud moved by ``params`` [P, 3] = (theta, tx,
        ty) about its centroid, and the gradient with respect to ``params``, for
        ``gauss_overlap``, ``gmm_l2`` or ``gmm_bhattacharya`` (the latter two with the clouds'
        ``point_cov`` or ``point_sigma``; covariances rotate with the cloud).  ``reuse`` as
        for :meth:`overlap_cost_grad`."""
        if fn == "gauss_overlap":
            return self.overlap_cost_grad(clouds, centroids, params, with_grad=with_grad, reuse=reuse)
        code = _lib.FN_BY_NAME[fn]
        if code not in (_lib.GMM_L2, _lib.GMM_BHATTACHARYA):
            raise ValueError("cost gradients exist for gauss_overlap, gmm_l2 and gmm_bhattacharya")
        n = clouds.n
        P = num_pairs(n)
        it, _ = self._items(clouds, code)
        self._dev(params, "params", torch.float32)
        self._dev(centroids, "centroids", torch.float32)
        if tuple(params.shape) != (P, 3) or tuple(centroids.shape) != (n, 2):
            raise ValueError("params must be [P, 3] and centroids [n, 2]")
        tens = [clouds.offsets, clouds.xy, clouds.point_sigma, clouds.point_cov]
        key = (fn, n) + tuple((t.data_ptr(), t._version) if t is not None else None for t in tens)
        prev = getattr(self, "_grad_clouds", None)
        reuse = reuse and prev is not None and prev[0] is clouds and prev[1] == key
        cost = torch.empty(P, dtype=torch.float32, device=params.device)
        grad = torch.empty((P, 3), dtype=torch.float32, device=params.device) if with_grad else None
        _lib.check(_lib.load().rocket_cost_grad(self.handle, None if reuse else ctypes.byref(it), n, code,
                                                _ptr(centroids), _ptr(params), _ptr(cost), _ptr(grad), _stream()),
                   self.handle)
        self._grad_clouds = (clouds, key)
        return cost, grad

    def overlap_cost_grad(self, clouds: Clouds, centroids, params, with_grad: bool = True, reuse: bool = False):
        """Cost and gradient of every pair's rigid transform ``params`` [P, 3].

        With ``reuse=True`` the library reuses the clouds that the previous call on this
        context prepared, skipping the size sort and packing, provided ``clouds`` is the
        same object with the same, unmodified tensors (the context keeps a reference to
        it); otherwise the clouds are prepared again."""
        n = clouds.n
        P = num_pairs(n)
        it, _ = self._items(clouds, _lib.GAUSS_OVERLAP)
        self._dev(params, "params", torch.float32)
        self._dev(centroids, "centroids", torch.float32)
        if tuple(params.shape) != (P, 3) or tuple(centroids.shape) != (n, 2):
            raise ValueError("params must be [P, 3] and centroids [n, 2]")
        # reuse only what this context prepared from these very tensors, unmodified since
        key = ("gauss_overlap", clouds.offsets.data_ptr(), clouds.offsets._version, clouds.xy.data_ptr(),
               clouds.xy._version, float(clouds.sigma), n)
        prev = getattr(self, "_grad_clouds", None)
        reuse = reuse and prev is not None and prev[0] is clouds and prev[1] == key
        cost = torch.empty(P, dtype=torch.float32, device=params.device)
        grad = torch.empty((P, 3), dtype=torch.float32, device=params.device) if with_grad else None
        _lib.check(_lib.load().rocket_overlap_cost_grad(self.handle, None if reuse else ctypes.byref(it), n,
                                                        _ptr(centroids), _ptr(params), _ptr(cost), _ptr(grad),
                                                        _stream()), self.handle)
        self._grad_clouds = (clouds, key)
        return cost, grad


_default = {}


def default_context() -> Context:
    dev = torch.cuda.current_device()
    if dev not in _default:
        _default[dev] = Context(dev)
    return _default[dev]


def allpairs(x, fn: str, counts: bool = False, ctx: Context | None = None):
    """All n(n-1)/2 pair results in packed upper-triangle order (float32 on the device).

    ``x``: float32 [n][d] for the NCC functions, :class:`Clouds` for ``gauss_overlap``,
    ``gmm_l2`` and ``gmm_bhattacharya`` (the latter two read ``Clouds.point_sigma``),
    :class:`SparseSet` for ``sparse_cosine`` (``counts=True`` also returns the exact
    intersection sizes).
    """
    return (ctx or default_context()).allpairs(x, fn, counts=counts)


def allpairs_noalloc(x, fn: str, out, counts=None):
    """All pairs like :func:`allpairs`, through ``rocket_allpairs_noalloc``: the library
    takes every workspace buffer from its static per-device scratch array and allocates
    nothing.  The caller passes the outputs: ``out`` float32 [P] (and for
    ``sparse_cosine`` or ``pce`` optionally ``counts`` int32 [P]) on the current device.
    Problems whose workspace exceeds the scratch array raise :class:`RocketError`."""
    code = _lib.FN_BY_NAME[fn]
    dev = torch.cuda.current_device()
    it, n = _items_struct(x, code, dev)
    P = num_pairs(n)
    _check_dev(out, "out", torch.float32, dev)
    if out.numel() < P:
        raise ValueError("out must hold n(n-1)/2 = %d values" % P)
    if counts is not None:
        _check_dev(counts, "counts", torch.int32, dev)
        if counts.numel() < P:
            raise ValueError("counts must hold n(n-1)/2 = %d values" % P)
    _lib.check(_lib.load().rocket_allpairs_noalloc(ctypes.byref(it), n, code, _ptr(out), _ptr(counts), _stream()))
    return out


def probe_valu(device: int = 0) -> dict:
    """Issue rates (instructions/s over all lanes) of FP32 FMA, v_exp_f32 and v_rcp_f32 on
    ``device`` (rocket_probe_valu): the measured denominators of the VALU rooflines."""
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _lib.check(_lib.load().rocket_probe_valu(int(device), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), None)
    return {"fma_per_s": a.value, "exp2_per_s": b.value, "rcp_per_s": c.value}


def plan_tiles(n: int, T: int):
    """Host-only divide-and-conquer leaves (bi, bj) for n items and tile T."""
    import numpy as np
    L = _lib.load()
    m = L.rocket_plan_tiles(n, T, None, None, 0)
    if m < 0:
        raise ValueError("bad arguments")
    bi = np.zeros(max(m, 1), dtype=np.int32)
    bj = np.zeros(max(m, 1), dtype=np.int32)
    L.rocket_plan_tiles(n, T, bi.ctypes.data_as(ctypes.c_void_p), bj.ctypes.data_as(ctypes.c_void_p), m)
    return list(zip(bi[:m].tolist(), bj[:m].tolist()))


def pair_index(i: int, j: int, n: int) -> int:
    return int(_lib.load().rocket_pair_index(i, j, n))


class OverlapCost(torch.autograd.Function):
    """Per-pair particle score C(params) with the hand-written adjoint as its gradient.

    forward(params [P,3], clouds, centroids, rctx, reuse, fn) -> cost [P] for ``fn`` in
    gauss_overlap (default), gmm_l2, gmm_bhattacharya; backward(g [P]) -> g[:,None] * dC/dparams.
    """

    @staticmethod
    def forward(ctx_, params, clouds: Clouds, centroids, rctx: Context | None = None, reuse: bool = False,
                fn: str = "gauss_overlap"):
        rc = rctx or default_context()
        cost, grad = rc.cost_grad(clouds, centroids, params.detach().contiguous(), fn=fn, with_grad=True, reuse=reuse)
        ctx_.save_for_backward(grad)
        return cost

    @staticmethod
    def backward(ctx_, g):
        (grad,) = ctx_.saved_tensors
        return g[:, None] * grad, None, None, None, None, None


def register(clouds: Clouds, centroids, params0, steps: int = 20, lr: float = 0.01, ctx: Context | None = None,
             record: bool = False, fn: str = "gauss_overlap"):
    """Rigid registration of every pair by gradient descent on E = -C / (N_i N_j), C the
    pair's ``fn`` score (gauss_overlap, gmm_l2 or gmm_bhattacharya).

    Each step evaluates the cost and its adjoint once (one persistent launch) and moves
    params <- params - lr * dE/dparams.  Returns the final params (and, with ``record``,
    the list of iterates params_0 .. params_steps).
    """
    n = clouds.n
    counts = (clouds.offsets[1:] - clouds.offsets[:-1]).to(torch.float32)
    iu = torch.triu_indices(n, n, offset=1, device=params0.device)
    norm = (counts[iu[0]] * counts[iu[1]]).clamp_min(1.0)
    p = params0.detach().clone().contiguous().requires_grad_(True)
    hist = [p.detach().clone()] if record else None
    rc = ctx or default_context()
    for step in range(steps):
        # the clouds do not change during the descent: prepare them once, reuse afterwards
        cost = OverlapCost.apply(p, clouds, centroids, rc, step > 0, fn)
        energy = -(cost / norm).sum()
        (g,) = torch.autograd.grad(energy, p)
        with torch.no_grad():
            p -= lr * g
        if record:
            hist.append(p.detach().clone())
    out = p.detach()
    return (out, hist) if record else out
