"""GPU adjoint of the overlap cost w.r.t. (theta, tx, ty) and the 20-step registration.

Checked against the FP64 oracle gradient (|g - r| <= 1e-5 max(|r|, tau)) and against
Richardson-extrapolated central differences of the FP64 oracle cost at h = 1e-3 and 5e-4
(|g - g_R| <= 1e-4 max(|g_R|, tau)); plain h = 1e-3 central differences carry O(h^2/sigma^2)
truncation error of a few 1e-4 at sigma = 0.02.
"""
import numpy as np
import pytest

import oracle
from paper_2009_04755_amd import synth

from gpu_util import announce, device_or_skip

pytestmark = pytest.mark.gpu
SIG = 0.02
TINY = 2.0 ** -126


@pytest.fixture(scope="module")
def ctx():
    device_or_skip()
    from paper_2009_04755_amd import Context
    return Context(0)


def _setup(n, salt, nmin=50, nmax=400):
    import torch
    from paper_2009_04755_amd import Clouds
    off, xy = synth.point_clouds(n, nmin=nmin, nmax=nmax, config=3, salt=salt)
    cen = synth.cloud_centroids(off, xy)
    cl = Clouds(torch.from_numpy(off).cuda(), torch.from_numpy(xy).cuda(), SIG)
    return off, xy, cen, cl, torch.from_numpy(cen).cuda()


def _check_grad(off, xy, cen, pi, pj, params, cost, grad, tol=1e-5):
    rc, rg, tau, kap = oracle.overlap_grad(off, xy, cen, pi, pj, params.astype(np.float64), SIG)
    nn = (np.diff(off)[pi] * np.diff(off)[pj]).astype(np.float64)
    lim_c = 1e-5 * rc * np.maximum(1.0, kap / 50.0) + nn * TINY
    assert np.all(np.abs(cost - rc) <= lim_c), np.max(np.abs(cost - rc) / np.maximum(rc, 1e-300))
    slack = (nn * TINY * 2500.0)[:, None]
    lim_g = tol * np.maximum(np.abs(rg), tau) + slack
    err = np.abs(grad - rg)
    assert np.all(err <= lim_g), (err / np.maximum(np.abs(rg), tau)).max()
    return rg, tau


def test_adjoint_matches_oracle_small(ctx):
    import torch
    announce("grad n=48 random transforms")
    off, xy, cen, cl, cen_d = _setup(48, 1, nmin=1, nmax=120)
    P = 48 * 47 // 2
    params = synth.rigid_starts(P, config=3, salt=4)
    params[::7] *= 0.01  # some near-identity transforms, where clouds overlap
    cost, grad = ctx.overlap_cost_grad(cl, cen_d, torch.from_numpy(params).cuda())
    pi, pj = oracle.all_pairs(48)
    _check_grad(off, xy, cen, pi, pj, params, cost.cpu().numpy(), grad.cpu().numpy())


def test_adjoint_matches_richardson_fd(ctx):
    import torch
    announce("grad vs Richardson FD n=24")
    off, xy, cen, cl, cen_d = _setup(24, 2, nmin=20, nmax=150)
    P = 24 * 23 // 2
    g = np.random.default_rng(5)
    params = np.stack([g.uniform(-0.3, 0.3, P), g.uniform(-0.05, 0.05, P), g.uniform(-0.05, 0.05, P)],
                      axis=1).astype(np.float32)
    _, grad = ctx.overlap_cost_grad(cl, cen_d, torch.from_numpy(params).cuda())
    grad = grad.cpu().numpy()
    pi, pj = oracle.all_pairs(24)
    p64 = params.astype(np.float64)
    _, _, tau, _ = oracle.overlap_grad(off, xy, cen, pi, pj, p64, SIG)
    h = 1e-3
    for m in range(3):
        e = np.zeros(3)
        e[m] = 1.0

        def fd(step):
            cp, _, _, _ = oracle.overlap_grad(off, xy, cen, pi, pj, p64 + step * e, SIG)
            cm, _, _, _ = oracle.overlap_grad(off, xy, cen, pi, pj, p64 - step * e, SIG)
            return (cp - cm) / (2 * step)

        g1, g2 = fd(h), fd(h / 2)
        gr = (4 * g2 - g1) / 3
        err = np.abs(grad[:, m] - gr) / np.maximum(np.abs(gr), tau[:, m])
        announce("param %d: max err vs Richardson FD %.2e; raw h=1e-3 FD vs Richardson %.2e" % (
            m, err.max(), (np.abs(g1 - gr) / np.maximum(np.abs(gr), tau[:, m])).max()))
        assert err.max() <= 1e-4


def test_autograd_function_backward(ctx):
    import torch
    from paper_2009_04755_amd import OverlapCost
    announce("grad autograd.Function")
    off, xy, cen, cl, cen_d = _setup(16, 3)
    P = 16 * 15 // 2
    p = torch.from_numpy(synth.rigid_starts(P, config=3, salt=6) * 0.05).cuda().requires_grad_(True)
    w = torch.randn(P, device="cuda", dtype=torch.float32)
    c = OverlapCost.apply(p, cl, cen_d, ctx)
    (c * w).sum().backward()
    _, grad = ctx.overlap_cost_grad(cl, cen_d, p.detach().contiguous())
    assert torch.allclose(p.grad, w[:, None] * grad, rtol=1e-6, atol=0)


def test_registration_20_steps_full_scale_sampled(ctx):
    """2048 clouds, all 2,096,128 pairs registered for 20 GD steps; the adjoint is checked
    against the FP64 oracle at the GPU's own iterates on 2,000 sampled pairs."""
    import torch
    from paper_2009_04755_amd import register
    announce("grad registration 20 steps n=2048")
    off, xy, cen, cl, cen_d = _setup(2048, 0)
    P = 2048 * 2047 // 2
    p0 = torch.from_numpy(synth.rigid_starts(P, config=3)).cuda()
    pfin, hist = register(cl, cen_d, p0, steps=20, lr=0.01, ctx=ctx, record=True)
    assert torch.isfinite(pfin).all()
    g = np.random.default_rng(3)
    sel = np.sort(g.choice(P, 2000, replace=False))
    pi_all, pj_all = np.triu_indices(2048, 1)
    pi, pj = pi_all[sel], pj_all[sel]
    for s in (0, 10, 19):
        ps = hist[s][torch.from_numpy(sel).cuda()].contiguous()
        full = hist[s].contiguous()
        cost, grad = ctx.overlap_cost_grad(cl, cen_d, full)
        c = cost[torch.from_numpy(sel).cuda()].cpu().numpy()
        gr = grad[torch.from_numpy(sel).cuda()].cpu().numpy()
        _check_grad(off, xy, cen, pi, pj, ps.cpu().numpy(), c, gr)


def test_new_contents_at_same_address_are_prepared_again(ctx):
    """Clouds overwritten in place (same device addresses, same n) must not reuse the old
    preparation: the binding re-prepares when a tensor's version changed, and the C entry
    point only reuses when the caller passes clouds = NULL."""
    import ctypes
    import torch
    from paper_2009_04755_amd import Clouds, Context, _lib
    announce("grad: in-place change of the clouds at the same address")
    off, xy, cen, cl, cen_d = _setup(32, 8, nmin=10, nmax=80)
    off2, xy2 = synth.point_clouds(32, nmin=10, nmax=80, config=3, salt=9)
    xy2 = xy2[: xy.size] if xy2.size >= xy.size else np.resize(xy2, xy.size)
    P = 32 * 31 // 2
    params = torch.from_numpy(synth.rigid_starts(P, config=3, salt=10) * np.float32(0.02)).cuda()
    c1, g1 = ctx.overlap_cost_grad(cl, cen_d, params)
    c1r, g1r = ctx.overlap_cost_grad(cl, cen_d, params, reuse=True)  # unchanged: reused
    assert torch.equal(c1, c1r) and torch.equal(g1, g1r)
    ptr = cl.xy.data_ptr()
    cl.xy.copy_(torch.from_numpy(xy2.astype(np.float32)).cuda())
    assert cl.xy.data_ptr() == ptr
    c2, g2 = ctx.overlap_cost_grad(cl, cen_d, params, reuse=True)  # version changed: prepared again
    fresh = Context(0)
    c3, g3 = fresh.overlap_cost_grad(Clouds(cl.offsets, cl.xy.clone(), SIG), cen_d, params)
    assert torch.equal(c2, c3) and torch.equal(g2, g3)
    assert not torch.equal(c1, c2)
    # the C entry point: clouds = NULL without a matching earlier call is a state error
    L = _lib.load()
    st = L.rocket_overlap_cost_grad(fresh.handle, None, 31, ctypes.c_void_p(cen_d.data_ptr()),
                                    ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(c3.data_ptr()), None, None)
    assert st == _lib.E_STATE
    torch.cuda.synchronize()
    fresh.close()
