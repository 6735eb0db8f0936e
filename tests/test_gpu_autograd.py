"""The Sinkhorn divergence as a torch.autograd.Function (Sec. II-B, eq. 7, by automatic
differentiation): backward w.r.t. samples and reference weights against
the FP64 oracle gradient, against central differences of the converged oracle
objective, and composition with other torch operations."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _grads(ct, x, y, w, eps, iters):
    dev = torch.device("cuda")
    xt = torch.as_tensor(x, device=dev).requires_grad_(True)
    wt = torch.as_tensor(w, device=dev).requires_grad_(True)
    S = ct.sinkhorn_divergence(xt, torch.as_tensor(y, device=dev), wt, eps=eps, iters=iters)
    S.backward()
    torch.cuda.synchronize()
    return S.item(), xt.grad.cpu().numpy(), wt.grad.cpu().numpy()


def test_backward_matches_oracle_on_3d_workload(ct):
    cfg = W.CONFIGS["autograd_3d"]
    x, y, _w, _g = W.config_inputs(cfg, T=1024, M=4096)
    w = W.positive_weights(np.random.default_rng(2), 4096)
    S, gx, gw = _grads(ct, x, y, w, cfg.eps, cfg.iters)
    r = oracle.sinkhorn(x, y, w, eps=cfg.eps, iters=cfg.iters)
    e = (rel(gx, r.grad_x), rel(gw, r.grad_w), abs(S - r.value) / abs(r.value))
    print("3d T=1024 M=4096 K=300:", e)
    assert max(e) < 1e-5, e


def test_backward_matches_central_differences_at_convergence(ct):
    cfg = W.CONFIGS["autograd_3d"]
    x, y, _w, _g = W.config_inputs(cfg, T=96, M=256)
    w = np.random.default_rng(1).uniform(0.5, 2.0, 256).astype(np.float32)
    eps, h = cfg.eps, cfg.extra["fd_h"]
    S, gx, gw = _grads(ct, x, y, w, eps, 4000)

    def solve(xx, ww, init):
        r = oracle.sinkhorn(xx, y, ww, eps=eps, iters=50, init=init)
        while r.resid > 1e-13:
            r = oracle.sinkhorn(xx, y, ww, eps=eps, iters=50, init=(r.f, r.g, r.p, r.q))
        return r

    base = solve(x.astype(np.float64), w.astype(np.float64), None)
    assert rel(gx, base.grad_x) < 1e-5 and rel(gw, base.grad_w) < 1e-5
    init = (base.f, base.g, base.p, base.q)
    rng = np.random.default_rng(cfg.seed)
    xd, wd = x.astype(np.float64), w.astype(np.float64)
    for i, k in [(int(rng.integers(96)), int(rng.integers(3))) for _ in range(6)]:
        xp, xm = xd.copy(), xd.copy()
        xp[i, k] += h
        xm[i, k] -= h
        fd = (solve(xp, wd, init).value - solve(xm, wd, init).value) / (2 * h)
        assert abs(gx[i, k] - fd) <= 1e-5 * max(abs(fd), 1e-2 * np.abs(gx).max()), (i, k)
    for j in rng.choice(256, 6, replace=False):
        wp, wm = wd.copy(), wd.copy()
        wp[j] += h
        wm[j] -= h
        fd = (solve(xd, wp, init).value - solve(xd, wm, init).value) / (2 * h)
        assert abs(gw[j] - fd) <= 1e-5 * max(abs(fd), 1e-2 * np.abs(gw).max()), j


def test_composes_with_torch_and_scales_with_grad_output(ct):
    dev = torch.device("cuda")
    x, y, w, _g = W.config_inputs(W.CONFIGS["grad_2d"], T=500, M=900)
    xt = torch.as_tensor(x, device=dev).requires_grad_(True)
    yt = torch.as_tensor(y, device=dev)
    loss = 3.0 * ct.sinkhorn_divergence(xt, yt, None, eps=0.01, iters=30) + (xt ** 2).sum()
    loss.backward()
    out = ct.sinkhorn_grad(torch.as_tensor(x, device=dev), yt, None, eps=0.01, iters=30)
    expect = 3.0 * out.grad_x + 2.0 * torch.as_tensor(x, device=dev)
    assert torch.allclose(xt.grad, expect, rtol=1e-6, atol=1e-9)
    # weights that do not require grad are not differentiated
    wt = torch.as_tensor(w, device=dev)
    x2 = torch.as_tensor(x, device=dev).requires_grad_(True)
    ct.sinkhorn_divergence(x2, yt, wt, eps=0.01, iters=30).backward()
    assert wt.grad is None and x2.grad is not None


def test_cached_reference_potential_matches_recomputing_it(ct):
    """The reference self potential does not depend on the trajectory (eq. 6's
    OT(b, b)): computed once (reference_self_potential) and passed as ref_q, the
    value and both gradients match a call that iterates it, within float32
    rounding, and the FP64 oracle at 1e-5.  With one launch per sweep the key
    ranges of the cross sweeps do not depend on whether q is iterated, so dS/dx is
    bit-equal; the exchange solve (the automatic choice at this size) shares its
    waves between the g and q rows, so g is summed in another order when q is
    cached and dS/dx agrees to float32 rounding."""
    dev = torch.device("cuda")
    x, y, _w, _g = W.config_inputs(W.CONFIGS["roofline_2d"], T=1200, M=3001)
    w = np.random.default_rng(7).uniform(0.5, 1.5, len(y)).astype(np.float32)
    xt, yt, wt = (torch.as_tensor(a, device=dev) for a in (x, y, w))
    eps, K = 0.01, 60
    full = ct.sinkhorn_grad(xt, yt, wt, eps=eps, iters=K, value=True, grad_w=True)
    q = ct.reference_self_potential(yt, wt, eps=eps, iters=K)
    cached = ct.sinkhorn_grad(xt, yt, wt, eps=eps, iters=K, value=True, grad_w=True, ref_q=q)
    xr = xt.clone().requires_grad_(True)
    wr = wt.clone().requires_grad_(True)
    S = ct.sinkhorn_divergence(xr, yt, wr, eps=eps, iters=K, ref_q=q)
    S.backward()
    torch.cuda.synchronize()
    r = oracle.sinkhorn(x, y, w, eps=eps, iters=K)
    assert rel(q.cpu().numpy(), r.q) < 1e-6
    assert rel(cached.grad_x.cpu().numpy(), full.grad_x.cpu().numpy()) < 2e-6
    a = ct.sinkhorn_grad(xt, yt, wt, eps=eps, iters=K, fused=False)
    b = ct.sinkhorn_grad(xt, yt, wt, eps=eps, iters=K, ref_q=q, fused=False)
    assert torch.equal(a.grad_x, b.grad_x)                  # q does not enter dS/dx
    assert rel(cached.grad_w.cpu().numpy(), full.grad_w.cpu().numpy()) < 1e-6
    assert abs(cached.value.item() - full.value.item()) <= 1e-6 * abs(full.value.item())
    assert torch.equal(xr.grad, cached.grad_x) and torch.equal(wr.grad, cached.grad_w)
    assert abs(S.item() - r.value) / abs(r.value) < 1e-5
    assert rel(wr.grad.cpu().numpy(), r.grad_w) < 1e-5
