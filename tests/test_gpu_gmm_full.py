"""GPU parity of the particle scores for localisations with a full covariance, and of the
registration adjoint of the GMM L2 and Bhattacharya scores (per-point sigma or full
covariance), against the FP64 oracle.

Cost bar: |g - r| <= 1e-5 r max(1, kappa/50) + slack (FP32 terms that underflow);
gradient bar: |g - r| <= 1e-5 max(|r|, tau) + slack, tau the oracle's error floor; against
Richardson-extrapolated central differences of the FP64 cost the bar is 1e-4.
"""
import numpy as np
import pytest

import oracle
from paper_2009_04755_amd import synth

from gpu_util import announce, device_or_skip

pytestmark = pytest.mark.gpu
MODES = {"gmm_l2": "l2", "gmm_bhattacharya": "bhattacharya"}


@pytest.fixture(scope="module")
def ctx():
    device_or_skip()
    from paper_2009_04755_amd import Context
    return Context(0)


def _setup(n, salt, nmin=1, nmax=150, kind="cov"):
    import torch
    from paper_2009_04755_amd import Clouds
    off, xy = synth.point_clouds(n, nmin=nmin, nmax=nmax, config=3, salt=salt)
    cen = synth.cloud_centroids(off, xy)
    shape = synth.point_covs(off, salt=salt) if kind == "cov" else synth.point_sigmas(off, salt=salt)
    cl = Clouds(torch.from_numpy(off).cuda(), torch.from_numpy(xy).cuda(), 0.02,
                point_sigma=None if kind == "cov" else torch.from_numpy(shape).cuda(),
                point_cov=torch.from_numpy(shape).cuda() if kind == "cov" else None)
    return off, xy, cen, shape, cl, torch.from_numpy(cen).cuda()


def _oracle(off, xy, shape, kind, pi, pj, mode, cen=None, params=None):
    kw = {"cov": shape} if kind == "cov" else {"sig": shape}
    return oracle.gmm_grad(off, xy, pi, pj, mode, centroids=cen, params=params, **kw)


def _slack(off, shape, kind, pi, pj, mode):
    # each FP32 term below ~2^-126 of its prefactor may flush to zero
    nn = (np.diff(off)[pi] * np.diff(off)[pj]).astype(np.float64)
    smin = float(np.sqrt(shape[:, 0].min())) if kind == "cov" else float(shape.min())
    pre = 1.0 / (2 * np.pi * 2 * smin * smin) if mode == "l2" else 2.0
    return nn * 2.0 ** -126 * max(pre, 1.0)


def _check_cost(got, ref, kap, slack):
    err = np.abs(got - ref) / (ref * np.maximum(1.0, kap / 50.0) + slack * 1e5)
    assert err.max() <= 1e-5, err.max()


@pytest.mark.parametrize("fn", list(MODES))
def test_full_covariance_scores_all_pairs(ctx, fn):
    announce("full-covariance %s all pairs n=48" % fn)
    off, xy, cen, cov, cl, _ = _setup(48, 1)
    got = ctx.allpairs(cl, fn).cpu().numpy()
    pi, pj = oracle.all_pairs(48)
    ref, _, _, kap = _oracle(off, xy, cov, "cov", pi, pj, MODES[fn])
    _check_cost(got, ref, kap, _slack(off, cov, "cov", pi, pj, MODES[fn]))
    # isotropic covariances through the full-covariance path agree with the sigma path's bar
    import torch
    from paper_2009_04755_amd import Clouds
    sig = synth.point_sigmas(off, salt=4)
    iso = np.stack([sig.astype(np.float64) ** 2, np.zeros(sig.size), sig.astype(np.float64) ** 2], 1).astype(np.float32)
    c2 = Clouds(cl.offsets, cl.xy, 0.02, point_cov=torch.from_numpy(iso).cuda())
    got2 = ctx.allpairs(c2, fn).cpu().numpy()
    ref2, _, _, kap2 = _oracle(off, xy, iso, "cov", pi, pj, MODES[fn])
    _check_cost(got2, ref2, kap2, _slack(off, iso, "cov", pi, pj, MODES[fn]))


def _check_grad(off, xy, cen, shape, kind, pi, pj, mode, params, cost, grad):
    rc, rg, tau, kap = _oracle(off, xy, shape, kind, pi, pj, mode, cen, params.astype(np.float64))
    sl = _slack(off, shape, kind, pi, pj, mode)
    _check_cost(cost, rc, kap, sl)
    # a flushed term sits where |u| = |V^-1 d| <~ 1e3 and |tr(V^-1 W)| <~ 1e4 for these deviations
    lim = 1e-5 * np.maximum(np.abs(rg), tau) + (sl * 1e4)[:, None]
    err = np.abs(grad - rg)
    assert np.all(err <= lim), (err / np.maximum(np.abs(rg), tau)).max()
    return rg, tau


@pytest.mark.parametrize("kind", ["cov", "sigma"])
@pytest.mark.parametrize("fn", list(MODES))
def test_adjoint_matches_oracle(ctx, fn, kind):
    import torch
    announce("gmm adjoint %s %s n=40" % (fn, kind))
    off, xy, cen, shape, cl, cen_d = _setup(40, 2, kind=kind)
    P = 40 * 39 // 2
    params = synth.rigid_starts(P, config=3, salt=5)
    params[::3] *= np.float32(0.02)  # near-identity transforms, where clouds overlap
    cost, grad = ctx.cost_grad(cl, cen_d, torch.from_numpy(params).cuda(), fn=fn)
    pi, pj = oracle.all_pairs(40)
    _check_grad(off, xy, cen, shape, kind, pi, pj, MODES[fn], params, cost.cpu().numpy(), grad.cpu().numpy())


@pytest.mark.parametrize("fn", list(MODES))
def test_adjoint_matches_richardson_fd(ctx, fn):
    import torch
    announce("gmm adjoint vs Richardson FD %s n=20" % fn)
    off, xy, cen, cov, cl, cen_d = _setup(20, 3, nmin=20, nmax=120)
    P = 20 * 19 // 2
    g = np.random.default_rng(7)
    params = np.stack([g.uniform(-0.3, 0.3, P), g.uniform(-0.03, 0.03, P), g.uniform(-0.03, 0.03, P)],
                      axis=1).astype(np.float32)
    _, grad = ctx.cost_grad(cl, cen_d, torch.from_numpy(params).cuda(), fn=fn)
    grad = grad.cpu().numpy()
    pi, pj = oracle.all_pairs(20)
    p64 = params.astype(np.float64)
    _, _, tau, _ = _oracle(off, xy, cov, "cov", pi, pj, MODES[fn], cen, p64)
    for m in range(3):
        e = np.zeros(3)
        e[m] = 1.0

        def fd(step):
            cp = _oracle(off, xy, cov, "cov", pi, pj, MODES[fn], cen, p64 + step * e)[0]
            cm = _oracle(off, xy, cov, "cov", pi, pj, MODES[fn], cen, p64 - step * e)[0]
            return (cp - cm) / (2 * step)

        h = 1e-3 if m == 0 else 2e-4
        gr = (4 * fd(h / 2) - fd(h)) / 3
        err = np.abs(grad[:, m] - gr) / np.maximum(np.abs(gr), tau[:, m])
        assert err.max() <= 1e-4, (m, err.max())


@pytest.mark.parametrize("fn", list(MODES))
def test_registration_20_steps_at_gpu_iterates(ctx, fn):
    """300 clouds with full covariances, every pair registered for 20 GD steps on the
    score; cost and adjoint checked against the oracle at the GPU's own iterates on 1,500
    sampled pairs."""
    import torch
    from paper_2009_04755_amd import register
    announce("gmm registration 20 steps %s n=300" % fn)
    off, xy, cen, cov, cl, cen_d = _setup(300, 6, nmin=50, nmax=400)
    P = 300 * 299 // 2
    p0 = torch.from_numpy(synth.rigid_starts(P, config=3, salt=8) * np.float32(0.2)).cuda()
    pfin, hist = register(cl, cen_d, p0, steps=20, lr=0.01, ctx=ctx, record=True, fn=fn)
    assert torch.isfinite(pfin).all()
    g = np.random.default_rng(11)
    sel = np.sort(g.choice(P, 1500, replace=False))
    pi_all, pj_all = np.triu_indices(300, 1)
    pi, pj = pi_all[sel], pj_all[sel]
    seld = torch.from_numpy(sel).cuda()
    for s in (0, 19):
        cost, grad = ctx.cost_grad(cl, cen_d, hist[s].contiguous(), fn=fn)
        _check_grad(off, xy, cen, cov, "cov", pi, pj, MODES[fn], hist[s][seld].cpu().numpy(),
                    cost[seld].cpu().numpy(), grad[seld].cpu().numpy())


def test_errors_and_reuse(ctx):
    import torch
    from paper_2009_04755_amd import Clouds, _lib
    announce("gmm full covariance errors and reuse")
    off, xy, cen, cov, cl, cen_d = _setup(12, 9)
    bad = cov.copy()
    bad[3, 1] = np.sqrt(bad[3, 0] * bad[3, 2]) * 1.5  # |c_xy| > sqrt(c_xx c_yy): not positive definite
    cb = Clouds(cl.offsets, cl.xy, 0.02, point_cov=torch.from_numpy(bad).cuda())
    with pytest.raises(_lib.RocketError) as e:
        ctx.allpairs(cb, "gmm_l2")
    assert e.value.status == _lib.E_INVALID
    P = 12 * 11 // 2
    params = torch.from_numpy(synth.rigid_starts(P, config=3, salt=2) * np.float32(0.05)).cuda()
    c1, g1 = ctx.cost_grad(cl, cen_d, params, fn="gmm_bhattacharya")
    c2, g2 = ctx.cost_grad(cl, cen_d, params, fn="gmm_bhattacharya", reuse=True)
    assert torch.equal(c1, c2) and torch.equal(g1, g2)
    # another score does not reuse the Bhattacharya preparation
    c3, _ = ctx.cost_grad(cl, cen_d, params, fn="gmm_l2", reuse=True)
    ref = _oracle(off, xy, cov, "cov", *oracle.all_pairs(12), "l2", cen, params.cpu().numpy().astype(np.float64))[0]
    assert np.all(np.abs(c3.cpu().numpy() - ref) <= 1e-4 * ref + 1e-30)
    with pytest.raises(ValueError):  # the binding refuses before any pointer reaches the library
        ctx.cost_grad(cl, cen_d, params, fn="sparse_cosine")
    # the C entry point refuses it too, and items = NULL for a score not prepared is a state error
    import ctypes
    from paper_2009_04755_amd import api
    it, n = api._items_struct(cl, _lib.GMM_L2, 0)
    L = _lib.load()
    args = (ctypes.c_void_p(cen_d.data_ptr()), ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(c3.data_ptr()),
            None, None)
    assert L.rocket_cost_grad(ctx.handle, ctypes.byref(it), n, _lib.SPARSE_COSINE, *args) == _lib.E_UNSUPPORTED
    ctx.allpairs(cl, "gauss_overlap")  # another prepare in between
    assert L.rocket_cost_grad(ctx.handle, None, n, _lib.GMM_L2, *args) == _lib.E_STATE
    torch.cuda.synchronize()
