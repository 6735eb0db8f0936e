"""Writes the stored oracle outputs used by tests/test_gpu_fullsize.py.

Calls only the FP64 oracle (oracle/) on the seeded workload generators
(workloads/); nothing here touches the GPU path.  Each fixture is one .npz
named after its workload, holding the oracle's grad_x, grad_w, value, the
gauge-comparable potentials and, for the Stein workloads, phi and h.

    python tests/golden/make_oracle_fixtures.py [name ...]

The large 2-D workload at full size (T = 65536, M = 262144, eps = 0.002,
K = 500; about 1.9e13 point pairs, hours on a few cores) is written without the
reference self problem (its M x M iterations would add 3.4e13 pairs), so it
holds the gradient and the cross and trajectory-self potentials but no value
or weight gradient.  Its iterations run in chunks whose state is kept in
CT_FIXTURE_CHECKPOINT (a directory, default the system's temporary one), so
an interrupted run resumes where it stopped; the chunks continue the same
iteration exactly (the oracle's warm start), so the result does not depend on
the chunking.  CT_FIXTURE_MAX_SECONDS stops such a run after the chunk that
passes that many seconds (the checkpoint stays for the next run), and
CT_FIXTURE_DIR writes the fixtures to another directory than this one.

The Stein fixture of the large workload takes the samples of its Sinkhorn
inputs (T = 65536) and the bandwidth from the pair-counting median (the sorted
median would list 2.1e9 distances).  The finite-difference fixture holds the
converged FP64 gradients of a 3-D instance (T = 2048, M = 8192) and central
differences of its converged objective on 64 sample coordinates and 64 weights.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
OUT = os.environ.get("CT_FIXTURE_DIR", HERE)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

# (fixture name, workload, T, M, iters); None = the workload's own size
SINKHORN = [
    ("planner_2d_full", "planner_2d", None, None, None),
    ("grad_2d_full", "grad_2d", None, None, None),
    ("autograd_3d_T4096_M16384", "autograd_3d", 4096, 16384, None),
    ("roofline_2d_T4096_M16384", "roofline_2d", 4096, 16384, None),
    ("autograd_3d_full", "autograd_3d", None, None, None),
]
# (fixture name, workload): full size, no reference self problem, chunked
SINKHORN_NOREF = [
    ("roofline_2d_full", "roofline_2d"),
]
# (fixture name, problems b of the ragged batch): their gradients only
BATCH = [
    ("batched_2d_sample16", list(range(0, 256, 16))),
]
# (fixture name, workload, T, M of the draw that fixes the samples): M = 16 draws the
# samples beside a 16-point reference; None takes the workload's own reference size,
# i.e. the very samples its Sinkhorn workload uses (bandwidth by pair counting)
# (fixture name, workload, T, M): central differences of the converged objective
FD = [
    ("fd_3d_T2048_M8192", "autograd_3d", 2048, 8192),
]
STEIN = [
    ("grad_2d_full_svgd", "grad_2d", None, 16),
    ("roofline_2d_T16384_svgd", "roofline_2d", 16384, 16),
    ("roofline_2d_full_svgd", "roofline_2d", None, None),
]


def sinkhorn_fixture(name, cfg_name, T, M, iters):
    cfg = W.CONFIGS[cfg_name]
    x, y, w, _g = W.config_inputs(cfg, T=T, M=M)
    K = cfg.iters if iters is None else iters
    t0 = time.time()
    r = oracle.sinkhorn(x, y, w, eps=cfg.eps, iters=K)
    np.savez_compressed(os.path.join(OUT, name + ".npz"), workload=cfg_name, T=len(x), M=len(y),
                        eps=cfg.eps, iters=K, grad_x=r.grad_x, grad_w=r.grad_w, value=r.value,
                        f=r.f, g=r.g, p=r.p, q=r.q, f_plus=r.f_plus, g_plus=r.g_plus,
                        resid=r.resid)
    print(f"{name}: T={len(x)} M={len(y)} K={K} S={r.value:.6g} resid={r.resid:.2e} "
          f"({time.time() - t0:.0f} s)", flush=True)


def sinkhorn_noref_fixture(name, cfg_name, chunk=25):
    import tempfile
    cfg = W.CONFIGS[cfg_name]
    x, y, w, _g = W.config_inputs(cfg)
    T, M, K = len(x), len(y), cfg.iters
    ck_dir = os.environ.get("CT_FIXTURE_CHECKPOINT", tempfile.gettempdir())
    ck = os.path.join(ck_dir, name + ".checkpoint.npz")
    f, g, p, done = np.zeros(T), np.zeros(M), np.zeros(T), 0
    if os.path.exists(ck):
        c = np.load(ck, allow_pickle=False)
        f, g, p, done = c["f"], c["g"], c["p"], int(c["done"])
        print(f"{name}: resuming after {done} iterations", flush=True)
    t0 = time.time()
    limit = float(os.environ.get("CT_FIXTURE_MAX_SECONDS", "inf"))
    zq = np.zeros(M)
    while done < K:
        if time.time() - t0 > limit:
            print(f"{name}: stopping after {done}/{K} iterations (time limit); checkpoint {ck}",
                  flush=True)
            return
        n = min(chunk, K - done)
        r = oracle.sinkhorn(x, y, w, eps=cfg.eps, iters=n, want_value=False, want_grad_w=False,
                            init=(f, g, p, zq))
        f, g, p, done = r.f, r.g, r.p, done + n
        np.savez(ck + ".tmp.npz", f=f, g=g, p=p, done=done)
        os.replace(ck + ".tmp.npz", ck)
        print(f"{name}: {done}/{K} iterations ({time.time() - t0:.0f} s)", flush=True)
    r = oracle.sinkhorn(x, y, w, eps=cfg.eps, iters=0, want_value=False, want_grad_w=False,
                        init=(f, g, p, zq))
    np.savez_compressed(os.path.join(OUT, name + ".npz"), workload=cfg_name, T=T, M=M,
                        eps=cfg.eps, iters=K, grad_x=r.grad_x, f=r.f, g=r.g, p=r.p,
                        f_plus=r.f_plus, p_plus=r.p_plus)
    print(f"{name}: T={T} M={M} K={K} ({time.time() - t0:.0f} s)", flush=True)


def batch_fixture(name, problems):
    cfg = W.CONFIGS["batched_2d"]
    probs = W.batch_inputs(cfg)
    t0 = time.time()
    Ts, Ms, grads = [], [], []
    for b in problems:
        x, y, w = probs[b]
        r = oracle.sinkhorn(x, y, w, eps=cfg.eps, iters=cfg.iters, want_value=False,
                            want_grad_w=False)
        Ts.append(len(x))
        Ms.append(len(y))
        grads.append(r.grad_x)
    np.savez_compressed(os.path.join(OUT, name + ".npz"), workload="batched_2d",
                        problems=np.array(problems), T=np.array(Ts), M=np.array(Ms),
                        eps=cfg.eps, iters=cfg.iters, grad_x=np.concatenate(grads))
    print(f"{name}: {len(problems)} problems ({time.time() - t0:.0f} s)", flush=True)


def _converged(x, y, w, eps, init, tol=1e-13):
    r = oracle.sinkhorn(x, y, w, eps=eps, iters=25, init=init)
    while r.resid > tol:
        r = oracle.sinkhorn(x, y, w, eps=eps, iters=25, init=(r.f, r.g, r.p, r.q))
    return r


def fd_fixture(name, cfg_name, T, M):
    """The converged FP64 gradients (column residual below 1e-13) and central
    differences of the converged objective (h from the workload, each side
    re-solved from the converged potentials) on the workload's number of seeded
    random coordinates of the samples and of the reference weights (weights drawn
    in [0.5, 2])."""
    cfg = W.CONFIGS[cfg_name]
    x, y, _w, _g = W.config_inputs(cfg, T=T, M=M)
    w = W.positive_weights(np.random.default_rng(1), M)
    xd, yd, wd = (a.astype(np.float64) for a in (x, y, w))
    eps, h, n = cfg.eps, cfg.extra["fd_h"], cfg.extra["fd_coords"]
    t0 = time.time()
    base = _converged(xd, yd, wd, eps, None)
    init = (base.f, base.g, base.p, base.q)
    rng = np.random.default_rng(cfg.seed + 7)
    xi = rng.choice(T * cfg.d, n, replace=False)
    wj = rng.choice(M, n, replace=False)
    fdx, fdw = np.empty(n), np.empty(n)
    for c, flat in enumerate(xi):
        i, k = divmod(int(flat), cfg.d)
        xp, xm = xd.copy(), xd.copy()
        xp[i, k] += h
        xm[i, k] -= h
        fdx[c] = (_converged(xp, yd, wd, eps, init).value -
                  _converged(xm, yd, wd, eps, init).value) / (2 * h)
    for c, j in enumerate(wj):
        wp, wm = wd.copy(), wd.copy()
        wp[j] += h
        wm[j] -= h
        fdw[c] = (_converged(xd, yd, wp, eps, init).value -
                  _converged(xd, yd, wm, eps, init).value) / (2 * h)
    np.savez_compressed(os.path.join(OUT, name + ".npz"), workload=cfg_name, T=T, M=M, eps=eps,
                        h=h, w=w, grad_x=base.grad_x, grad_w=base.grad_w, value=base.value,
                        resid=base.resid, x_coords=xi, w_coords=wj, fd_x=fdx, fd_w=fdw)
    print(f"{name}: T={T} M={M} {n}+{n} coordinates ({time.time() - t0:.0f} s)", flush=True)


def stein_fixture(name, cfg_name, T, M):
    cfg = W.CONFIGS[cfg_name]
    x, _y, _w, g = W.config_inputs(cfg, T=T, M=M)
    t0 = time.time()
    sc = oracle.gmm_score(x, g.weights, g.means, g.sigmas, g.floor)
    h = oracle.median_bandwidth(x) if M is not None else oracle.median_bandwidth_by_counting(x)
    phi = oracle.svgd_phi(x, sc, h)
    np.savez_compressed(os.path.join(OUT, name + ".npz"), workload=cfg_name, T=len(x),
                        M_draw=-1 if M is None else M, score=sc, h=h, phi=phi)
    print(f"{name}: T={len(x)} h={h:.6g} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    want = set(sys.argv[1:])
    for spec in STEIN:
        if not want or spec[0] in want:
            stein_fixture(*spec)
    for spec in SINKHORN:
        if not want or spec[0] in want:
            sinkhorn_fixture(*spec)
    for spec in FD:
        if not want or spec[0] in want:
            fd_fixture(*spec)
    for spec in BATCH:
        if not want or spec[0] in want:
            batch_fixture(*spec)
    for spec in SINKHORN_NOREF:
        if not want or spec[0] in want:
            sinkhorn_noref_fixture(*spec)
