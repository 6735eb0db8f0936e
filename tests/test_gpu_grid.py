"""GPU parity of the continuous-utility reference (a utility on a grid, Sec. II-A;
the score-only Stein flow, Sec. II-B) against the FP64 oracle: the grid score
(float64 on both sides, compared to 2e-6), the Stein flow on a caller's score,
the weighted grid samples (positions bit-exact, weights to float32 rounding),
the Sinkhorn flow on those samples, and one planner step toward a grid."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import rel
from test_gpu_sinkhorn import _compare, _run

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def _maps(n, seed, floor, lo=None, hi=None):
    u, lo, hi = W.utility_map(np.random.default_rng(seed), n, lo=lo, hi=hi)
    return u, lo, hi, float(np.float32(floor))


def _gpu_grid(ct, u, lo, hi, floor):
    return ct.UtilityGrid(torch.as_tensor(u, device="cuda"), [float(v) for v in lo],
                          [float(v) for v in hi], floor)


def _oracle_grid(u, lo, hi, floor):
    return oracle.grid.Grid(u.astype(np.float64), lo.astype(np.float64), hi.astype(np.float64),
                            floor)


def _points(rng, lo, hi, n_nodes, T):
    """Inside the box, beyond it on every side, and exactly on node positions."""
    d = len(lo)
    span = hi - lo
    inside = rng.uniform(lo, hi, (T, d))
    outside = rng.uniform(lo - 0.3 * span, hi + 0.3 * span, (T // 4, d))
    nodes = np.stack([lo[t] + rng.integers(0, n_nodes[t], T // 8) * (span[t] / (n_nodes[t] - 1))
                      for t in range(d)], axis=1)
    return np.concatenate([inside, outside, nodes]).astype(np.float32)


@pytest.mark.parametrize("n,floor,T", [((64, 48), 0.0, 3000), ((33, 129), 0.05, 5001),
                                       ((500, 487), 0.0, 65536), ((17, 12, 9), 0.0, 4000),
                                       ((8, 8, 8), 0.02, 1234)])
def test_grid_score_matches_oracle(ct, n, floor, T):
    d = len(n)
    u, lo, hi, fl = _maps(n, 100 + len(n) * 7 + n[0], floor,
                          lo=np.full(d, -1.5), hi=np.linspace(2.0, 3.0, d))
    x = _points(np.random.default_rng(n[0]), lo.astype(np.float64), hi.astype(np.float64), n, T)
    sc = ct.grid_score(torch.as_tensor(x, device="cuda"), _gpu_grid(ct, u, lo, hi, fl))
    torch.cuda.synchronize()
    got = sc.cpu().numpy()
    want = oracle.grid.score(_oracle_grid(u, lo, hi, fl), x.astype(np.float64))
    print(n, floor, T, "rel", rel(got, want), "zero rows", int(np.sum(np.all(want == 0, axis=1))))
    np.testing.assert_allclose(got, want, rtol=2e-6, atol=1e-9 * np.abs(want).max())


def test_grid_score_non_finite_rows_and_scale_invariance(ct):
    u, lo, hi, fl = _maps((20, 30), 5, 0.01)
    x = np.random.default_rng(5).uniform(0, 1, (300, 2)).astype(np.float32)
    x[7, 0] = np.nan
    x[11, 1] = np.inf
    dev = torch.device("cuda")
    a = ct.grid_score(torch.as_tensor(x, device=dev), _gpu_grid(ct, u, lo, hi, fl)).cpu().numpy()
    b = ct.grid_score(torch.as_tensor(x, device=dev),
                      _gpu_grid(ct, u * np.float32(8.0), lo, hi, fl * 8.0)).cpu().numpy()
    bad = ~np.isfinite(a).all(axis=1)
    assert list(np.flatnonzero(bad)) == [7, 11]
    np.testing.assert_array_equal(a[~bad], b[~bad])          # powers of two scale exactly


def test_svgd_score_entry_reproduces_the_mixture_flow(ct):
    x, _y, _w, g = W.config_inputs(W.CONFIGS["grad_2d"], T=3001, M=16)
    dev = torch.device("cuda")
    xt = torch.as_tensor(x, device=dev)
    for h in (None, 0.0123):
        phi, hu, sc = ct.svgd_grad(xt, ct.GMM.from_numpy(g, dev), h, return_score=True)
        phi2, hu2 = ct.svgd_grad_score(xt, sc, h)
        torch.cuda.synchronize()
        assert torch.equal(phi, phi2) and torch.equal(hu, hu2)


@pytest.mark.parametrize("d,n,T", [(2, (128, 96), 2048), (2, (40, 40), 777), (3, (24, 20, 16), 1500)])
def test_stein_flow_toward_a_grid_matches_oracle(ct, d, n, T):
    u, lo, hi, fl = _maps(n, 40 + d, 0.0)
    cfg = W.CONFIGS["grad_2d" if d == 2 else "autograd_3d"]
    x, _y, _w, _g = W.config_inputs(cfg, T=T, M=16)
    dev = torch.device("cuda")
    xt = torch.as_tensor(x, device=dev)
    sc = ct.grid_score(xt, _gpu_grid(ct, u, lo, hi, fl))
    phi, hu = ct.svgd_grad_score(xt, sc)
    torch.cuda.synchronize()
    og = _oracle_grid(u, lo, hi, fl)
    rsc = oracle.grid.score(og, x)
    rh = oracle.median_bandwidth(x)
    rphi = oracle.svgd_phi(x, rsc, rh)
    e = dict(score=rel(sc.cpu().numpy(), rsc), h=abs(float(hu.item()) - rh) / rh,
             phi=rel(phi.cpu().numpy(), rphi))
    print(d, n, T, e)
    assert e["score"] < 2e-6 and e["h"] < 1e-6 and e["phi"] < TOL, e


@pytest.mark.parametrize("n,floor", [((50, 40), 0.0), ((31, 17), 0.01), ((1100, 300), 0.0),
                                     ((12, 10, 9), 0.0), ((7, 5, 33), 0.003)])
def test_grid_samples_match_oracle(ct, n, floor):
    d = len(n)
    u, lo, hi, fl = _maps(n, 60 + n[0], floor, lo=np.full(d, 0.25), hi=np.full(d, 3.75))
    y, w = ct.grid_samples(_gpu_grid(ct, u, lo, hi, fl))
    torch.cuda.synchronize()
    ry, rw = oracle.grid.samples(_oracle_grid(u, lo, hi, fl))
    assert y.shape[0] == ry.shape[0], (y.shape, ry.shape)
    np.testing.assert_array_equal(y.cpu().numpy(), ry.astype(np.float32))
    np.testing.assert_allclose(w.cpu().numpy(), rw, rtol=1e-6)
    if floor == 0.0:
        assert y.shape[0] == int(np.count_nonzero(u))


def test_grid_samples_reject_invalid_utilities(ct):
    dev = torch.device("cuda")
    u, lo, hi, _ = _maps((9, 7), 3, 0.0)
    for bad in (-1.0, np.nan, np.inf):
        v = u.copy()
        v[2, 3] = bad
        with pytest.raises(ct.CtError, match="negative or non-finite"):
            ct.grid_samples(ct.UtilityGrid(torch.as_tensor(v, device=dev), list(lo), list(hi), 0.0))
    z = np.zeros_like(u)
    with pytest.raises(ct.CtError, match="zero on every node"):
        ct.grid_samples(ct.UtilityGrid(torch.as_tensor(z, device=dev), list(lo), list(hi), 0.0))
    y, w = ct.grid_samples(ct.UtilityGrid(torch.as_tensor(z, device=dev), list(lo), list(hi), 0.5))
    assert y.shape[0] == z.size                                  # a floor keeps every node
    ry, rw = oracle.grid.samples(_oracle_grid(z, lo, hi, float(np.float32(0.5))))
    np.testing.assert_allclose(w.cpu().numpy(), rw, rtol=1e-6)


@pytest.mark.parametrize("d,n,T,eps,iters", [(2, (64, 64), 1500, 0.01, 50), (3, (16, 14, 12), 900, 0.02, 30)])
def test_sinkhorn_flow_toward_grid_samples_matches_oracle(ct, d, n, T, eps, iters):
    u, lo, hi, fl = _maps(n, 80 + d, 0.0)
    y, w = ct.grid_samples(_gpu_grid(ct, u, lo, hi, fl))
    ry, rw = oracle.grid.samples(_oracle_grid(u, lo, hi, fl))
    cfg = W.CONFIGS["grad_2d" if d == 2 else "autograd_3d"]
    x, _y, _w, _g = W.config_inputs(cfg, T=T, M=16)
    g = _run(ct, x, y.cpu().numpy(), w.cpu().numpy(), eps, iters)
    r = oracle.sinkhorn(x, ry.astype(np.float32).astype(np.float64), rw, eps=eps, iters=iters)
    errs = _compare(g, r, T, ry.shape[0], rw)
    print(d, n, T, errs)


def test_planner_step_toward_a_grid_matches_oracle(ct):
    cfg = W.CONFIGS["roofline_2d"]
    e = cfg.extra
    T = 600
    rng = np.random.default_rng(cfg.seed + 3)
    u0 = np.stack([np.full(T, e["v0"]), rng.normal(size=T) * e["omega_std"]], axis=1)
    s0 = np.array(e["s0"])
    Q, R = np.eye(2), 0.01 * np.eye(2)
    u, lo, hi, fl = _maps((96, 80), 91, 0.01)
    u1, _s, hist = ct.plan("unicycle", s0, u0, e["dt"], Q, R, "svgd_grid", 1, 0.05,
                           grid=_gpu_grid(ct, u, lo, hi, fl))
    r_u1, _rs, r_obj, _ra, _rv = oracle.plan_step("unicycle", s0, u0, e["dt"], Q, R, "svgd_grid",
                                                 step=0.05, grid=_oracle_grid(u, lo, hi, fl))
    assert abs(hist[0] - r_obj) / abs(r_obj) < 1e-5
    assert rel(u1 - u0, r_u1 - u0) < 1e-5


def test_planner_step_toward_a_3d_grid_matches_oracle(ct):
    # the 3-D point mass (the aircraft's stand-in) steered by the Stein flow toward a 3-D map
    T = 400
    rng = np.random.default_rng(77)
    u0 = rng.normal(size=(T, 3)) * 0.1
    s0 = np.array([0.5, 0.5, 0.5, 0.0, 0.0, 0.0])
    Q, R = np.eye(3), 0.01 * np.eye(3)
    u, lo, hi, fl = _maps((20, 16, 12), 93, 0.02)
    u1, _s, hist = ct.plan("double_integrator", s0, u0, 0.05, Q, R, "svgd_grid", 1, 0.05,
                           grid=_gpu_grid(ct, u, lo, hi, fl))
    r_u1, _rs, r_obj, _ra, _rv = oracle.plan_step("double_integrator", s0, u0, 0.05, Q, R,
                                                 "svgd_grid", step=0.05,
                                                 grid=_oracle_grid(u, lo, hi, fl))
    assert abs(hist[0] - r_obj) / abs(r_obj) < 1e-5
    assert rel(u1 - u0, r_u1 - u0) < 1e-5


@pytest.mark.parametrize("n,floor", [((2, 2), 0.0), ((2, 2, 2), 1e-6), ((3, 2), 5.0)])
def test_grid_score_single_cells_and_box_faces(ct, n, floor):
    # the smallest grids (one cell per axis), points on every corner and face of the
    # box and just outside it, a vanishing and a dominant floor
    d = len(n)
    u, lo, hi, fl = _maps(n, 300 + d, floor)
    lo64, hi64 = lo.astype(np.float64), hi.astype(np.float64)
    corners = np.array([[lo64[t] if (k >> t) & 1 == 0 else hi64[t] for t in range(d)]
                        for k in range(1 << d)])
    mids = (lo64 + hi64) / 2
    faces = np.concatenate([np.where(np.eye(d, dtype=bool)[t], lo64, mids)[None] for t in range(d)] +
                           [np.where(np.eye(d, dtype=bool)[t], hi64, mids)[None] for t in range(d)])
    eps = (hi64 - lo64) * 1e-3
    outside = np.concatenate([corners - eps, corners + eps])
    inner = np.random.default_rng(d).uniform(lo64, hi64, (200, d))
    x = np.concatenate([corners, faces, outside, inner]).astype(np.float32)
    sc = ct.grid_score(torch.as_tensor(x, device="cuda"), _gpu_grid(ct, u, lo, hi, fl))
    torch.cuda.synchronize()
    want = oracle.grid.score(_oracle_grid(u, lo, hi, fl), x.astype(np.float64))
    np.testing.assert_allclose(sc.cpu().numpy(), want, rtol=2e-6, atol=1e-9 * max(1.0, np.abs(want).max()))
    y, w = ct.grid_samples(_gpu_grid(ct, u, lo, hi, fl))
    ry, rw = oracle.grid.samples(_oracle_grid(u, lo, hi, fl))
    np.testing.assert_array_equal(y.cpu().numpy(), ry.astype(np.float32))
    np.testing.assert_allclose(w.cpu().numpy(), rw, rtol=1e-6)
