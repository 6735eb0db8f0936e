"""Writes the stored oracle outputs used by tests/test_gpu_fullsize.py.

Calls only the FP64 oracle (oracle/) on the seeded workload generators
(workloads/); nothing here touches the GPU path.  Each fixture is one .npz
named after its workload, holding the oracle's grad_x, grad_w, value, the
gauge-comparable potentials and, for the Stein workloads, phi and h.

    python tests/golden/make_oracle_fixtures.py [name ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

# (fixture name, workload, T, M, iters); None = the workload's own size
SINKHORN = [
    ("planner_2d_full", "planner_2d", None, None, None),
    ("grad_2d_full", "grad_2d", None, None, None),
    ("autograd_3d_T4096_M16384", "autograd_3d", 4096, 16384, None),
    ("roofline_2d_T4096_M16384", "roofline_2d", 4096, 16384, None),
]
STEIN = [
    ("grad_2d_full_svgd", "grad_2d", None),
    ("roofline_2d_T16384_svgd", "roofline_2d", 16384),
]


def sinkhorn_fixture(name, cfg_name, T, M, iters):
    cfg = W.CONFIGS[cfg_name]
    x, y, w, _g = W.config_inputs(cfg, T=T, M=M)
    K = cfg.iters if iters is None else iters
    t0 = time.time()
    r = oracle.sinkhorn(x, y, w, eps=cfg.eps, iters=K)
    np.savez_compressed(os.path.join(HERE, name + ".npz"), workload=cfg_name, T=len(x), M=len(y),
                        eps=cfg.eps, iters=K, grad_x=r.grad_x, grad_w=r.grad_w, value=r.value,
                        f=r.f, g=r.g, p=r.p, q=r.q, f_plus=r.f_plus, g_plus=r.g_plus,
                        resid=r.resid)
    print(f"{name}: T={len(x)} M={len(y)} K={K} S={r.value:.6g} resid={r.resid:.2e} "
          f"({time.time() - t0:.0f} s)", flush=True)


def stein_fixture(name, cfg_name, T):
    cfg = W.CONFIGS[cfg_name]
    x, _y, _w, g = W.config_inputs(cfg, T=T, M=16)
    t0 = time.time()
    sc = oracle.gmm_score(x, g.weights, g.means, g.sigmas, g.floor)
    h = oracle.median_bandwidth(x)
    phi = oracle.svgd_phi(x, sc, h)
    np.savez_compressed(os.path.join(HERE, name + ".npz"), workload=cfg_name, T=len(x),
                        score=sc, h=h, phi=phi)
    print(f"{name}: T={len(x)} h={h:.6g} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    want = set(sys.argv[1:])
    for spec in STEIN:
        if not want or spec[0] in want:
            stein_fixture(*spec)
    for spec in SINKHORN:
        if not want or spec[0] in want:
            sinkhorn_fixture(*spec)
