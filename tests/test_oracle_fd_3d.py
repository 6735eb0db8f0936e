"""Finite-difference pin of the oracle gradients on a reduced instance of the
3D differentiation workload (anisotropic 8-component mixture, eps = 0.01):
central differences (h = 1e-4) of the converged FP64 objective on random
coordinates of the samples and of the reference weights (Sec. II-B, eq. 7).
The central difference has an O(h^2) truncation error (third derivatives scale
like 1/eps^2), so agreement is required to 1e-5 relative, with the scale floored
at 1% of the largest gradient entry."""
import numpy as np
import pytest

import oracle
import workloads as W


def _solve(x, y, w, eps, init, tol=1e-13):
    r = oracle.sinkhorn(x, y, w, eps=eps, iters=50, init=init)
    while r.resid > tol:
        r = oracle.sinkhorn(x, y, w, eps=eps, iters=50, init=(r.f, r.g, r.p, r.q))
    return r


@pytest.mark.slow
def test_fd_on_reduced_3d_workload():
    cfg = W.CONFIGS["autograd_3d"]
    x, y, w, _g = W.config_inputs(cfg, T=96, M=256)
    x = x.astype(np.float64)
    y = y.astype(np.float64)
    w = np.random.default_rng(1).uniform(0.5, 2.0, len(y))
    eps, h = cfg.eps, cfg.extra["fd_h"]
    base = _solve(x, y, w, eps, None)
    init = (base.f, base.g, base.p, base.q)
    rng = np.random.default_rng(cfg.seed)
    coords = [(int(rng.integers(len(x))), int(rng.integers(3))) for _ in range(8)]
    for i, k in coords:
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        fd = (_solve(xp, y, w, eps, init).value - _solve(xm, y, w, eps, init).value) / (2 * h)
        scale = max(abs(fd), 1e-2 * np.abs(base.grad_x).max())
        assert abs(fd - base.grad_x[i, k]) <= 1e-5 * scale, (i, k, fd, base.grad_x[i, k])
    for j in rng.choice(len(y), 8, replace=False):
        wp, wm = w.copy(), w.copy()
        wp[j] += h
        wm[j] -= h
        fd = (_solve(x, y, wp, eps, init).value - _solve(x, y, wm, eps, init).value) / (2 * h)
        scale = max(abs(fd), 1e-2 * np.abs(base.grad_w).max())
        assert abs(fd - base.grad_w[j]) <= 1e-5 * scale, (j, fd, base.grad_w[j])
