"""Parity at the workloads' own sizes.

* Stored oracle outputs (tests/golden/*.npz, written by
  tests/golden/make_oracle_fixtures.py, which calls only the oracle) for the
  planner and 2D-gradient workloads at full size and reduced instances of the 3D
  and large 2D workloads: elementwise comparison, tolerance 1e-5.
* The large 2D workload (T=65536, M=262144, eps=0.002, K=500) at full size, in the
  launch configuration the benchmark uses: properties that hold at any size,
  evaluated in float64 on sampled rows from the kernel's own outputs: the final
  pass reproduces f+ = T_b(g) and the barycentric gradient from the returned
  potentials, the weight gradient is centred, the plan is nearly feasible; for the
  Stein flow, the bandwidth is a median of the pairwise distances and phi on
  sampled rows equals eq. 4 at that bandwidth."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from helpers import gauge, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-5


TABLE = os.path.join(os.path.dirname(GOLD), "..", "paper_2511_11514_amd", "tuning", "mi355x.txt")


@pytest.fixture
def stored_schedules(ct):
    """The stored MI355X schedule table (what the benchmark loads), for one test."""
    ct.tuning_load(os.path.normpath(TABLE))
    yield
    ct.tuning_clear()


def _fixture(name):
    path = os.path.join(GOLD, name + ".npz")
    if not os.path.exists(path):
        pytest.skip(f"fixture {name} not generated (tests/golden/make_oracle_fixtures.py)")
    return np.load(path, allow_pickle=False)


@pytest.mark.parametrize("expanded", [False, True], ids=["difference", "expanded"])
@pytest.mark.parametrize("name", ["planner_2d_full", "grad_2d_full", "autograd_3d_T4096_M16384",
                                  "roofline_2d_T4096_M16384", "autograd_3d_full"])
def test_sinkhorn_against_stored_oracle(ct, stored_schedules, name, expanded):
    """Each stored workload through the default execution (whose per-sweep launches
    use the expanded exponent), and through the per-sweep launches with the
    difference form (CT_DIFFERENCE), with the stored MI355X schedules (the launch
    configuration the benchmark times)."""
    F = _fixture(name)
    cfg = W.CONFIGS[str(F["workload"])]
    T, M, K = int(F["T"]), int(F["M"]), int(F["iters"])
    x, y, w, _g = W.config_inputs(cfg, T=T, M=M)
    dev = torch.device("cuda")
    t = lambda a: torch.as_tensor(a, device=dev)
    out = ct.sinkhorn_grad(t(x), t(y), t(w), eps=cfg.eps, iters=K, value=True, grad_w=True,
                           potentials=True, expanded=expanded,
                           fused=None if expanded else False)
    torch.cuda.synchronize()
    pot = out.pot.cpu().numpy()
    f1, g1 = gauge(pot[:T], pot[T:T + M], T, M)
    f2, g2 = gauge(F["f"], F["g"], T, M)
    e = dict(grad_x=rel(out.grad_x.cpu().numpy(), F["grad_x"]),
             grad_w=rel(out.grad_w.cpu().numpy(), F["grad_w"]),
             value=abs(out.value.item() - float(F["value"])) / abs(float(F["value"])),
             f=rel(f1, f2), g=rel(g1, g2),
             p=rel(pot[T + M:2 * T + M], F["p"]), q=rel(pot[2 * T + M:], F["q"]))
    if out.pot_plus is not None:
        # (f+, g+) carry the gauge of (f, g): shift them by the constant that fixes (f, g)
        pp = out.pot_plus.cpu().numpy().astype(np.float64)
        c1, c2 = f1[0] - pot[0], f2[0] - F["f"][0]
        e["f_plus"] = rel(pp[:T] + c1, F["f_plus"] + c2)
        e["g_plus"] = rel(pp[T:T + M] - c1, F["g_plus"] - c2)
    print(name, "expanded" if expanded else "", " ".join(f"{k}={v:.2e}" for k, v in e.items()))
    assert max(e.values()) < TOL, e


@pytest.mark.parametrize("name", ["grad_2d_full_svgd", "roofline_2d_T16384_svgd",
                                  "roofline_2d_full_svgd"])
def test_svgd_against_stored_oracle(ct, name):
    F = _fixture(name)
    cfg = W.CONFIGS[str(F["workload"])]
    m_draw = int(F["M_draw"]) if "M_draw" in F.files else 16
    x, _y, _w, g = W.config_inputs(cfg, T=int(F["T"]), M=None if m_draw < 0 else m_draw)
    dev = torch.device("cuda")
    phi, h, sc = ct.svgd_grad(torch.as_tensor(x, device=dev), ct.GMM.from_numpy(g, dev),
                              return_score=True)
    torch.cuda.synchronize()
    e = dict(phi=rel(phi.cpu().numpy(), F["phi"]), score=rel(sc.cpu().numpy(), F["score"]),
             h=abs(h.item() - float(F["h"])) / float(F["h"]))
    print(name, " ".join(f"{k}={v:.2e}" for k, v in e.items()))
    assert e["phi"] < TOL and e["score"] < TOL and e["h"] < 1e-6, e


def _lse_rows(xq, xk, logw, pot, eps, rows):
    """-eps log sum_j exp(logw_j + (pot_j - |xq_i - xk_j|^2)/eps) and the mean
    offset, in float64, for the sampled rows only."""
    out, bary = [], []
    for i in rows:
        z = logw + (pot - ((xk - xq[i]) ** 2).sum(1)) / eps
        m = z.max()
        e = np.exp(z - m)
        out.append(-eps * (m + np.log(e.sum())))
        bary.append((e[:, None] * (xk - xq[i])).sum(0) / e.sum())
    return np.array(out), np.array(bary)


def test_large_workload_properties(ct):
    cfg = W.CONFIGS["roofline_2d"]
    x, y, w, _g = W.config_inputs(cfg)
    T, M, eps = len(x), len(y), cfg.eps
    dev = torch.device("cuda")
    t = lambda a: torch.as_tensor(a, device=dev)
    ct.autotune_sinkhorn(T, M, 2, eps)
    out = ct.sinkhorn_grad(t(x), t(y), t(w), eps=eps, iters=cfg.iters, value=True, grad_w=True,
                           potentials=True, aux=True)
    torch.cuda.synchronize()
    pot = out.pot.cpu().numpy().astype(np.float64)
    pp = out.pot_plus.cpu().numpy().astype(np.float64)
    f, g, p = pot[:T], pot[T:T + M], pot[T + M:2 * T + M]
    xd, yd = x.astype(np.float64), y.astype(np.float64)
    rows = np.random.default_rng(cfg.seed).choice(T, 48, replace=False)
    logb = np.log(w / w.sum(dtype=np.float64))
    loga = np.full(T, -np.log(T))
    fp_ref, dy = _lse_rows(xd, yd, logb, g, eps, rows)
    pp_ref, ds = _lse_rows(xd, xd, loga, p, eps, rows)
    gx = out.grad_x.cpu().numpy()[rows]
    assert rel(pp[:T][rows], fp_ref) < TOL
    assert rel(pp[T + M:2 * T + M][rows], pp_ref) < TOL
    assert rel(gx, 2.0 / T * (ds - dy)) < TOL
    gw = out.grad_w.cpu().numpy().astype(np.float64)
    assert abs(w @ gw) < 1e-5 * np.abs(w).sum() * np.abs(gw).max()
    aux = out.aux.cpu().numpy()
    assert np.isfinite(out.value.item()) and aux[3] < 1e-2 and aux[5] == 0


def test_large_workload_svgd_properties(ct):
    cfg = W.CONFIGS["roofline_2d"]
    x, _y, _w, g = W.config_inputs(cfg, M=16)
    T = len(x)
    dev = torch.device("cuda")
    phi, h, sc = ct.svgd_grad(torch.as_tensor(x, device=dev), ct.GMM.from_numpy(g, dev),
                              return_score=True)
    torch.cuda.synchronize()
    h = h.item()
    med2 = h * np.log(T)                               # squared median distance
    npair = T * (T - 1) // 2
    lt, _ = oracle.pair_count(x, med2 * (1 - 2e-6))
    _, le = oracle.pair_count(x, med2 * (1 + 2e-6))
    assert lt <= npair // 2 and le >= (npair + 1) // 2
    rows = np.random.default_rng(cfg.seed).choice(T, 32, replace=False)
    xd = x.astype(np.float64)
    scd = sc.cpu().numpy().astype(np.float64)
    ref = []
    for i in rows:
        dd = xd[i] - xd
        k = np.exp(-(dd ** 2).sum(1) / h)
        ref.append((k[:, None] * (scd + (2.0 / h) * dd)).sum(0) / T)
    assert rel(phi.cpu().numpy()[rows], np.array(ref)) < TOL
    sref = oracle.gmm_score(x[rows], g.weights, g.means, g.sigmas, g.floor)
    assert rel(scd[rows], sref) < TOL


@pytest.mark.parametrize("expanded", [False, True], ids=["difference", "expanded"])
def test_large_workload_against_stored_oracle(ct, stored_schedules, expanded):
    """The large 2-D workload at full size (T = 65536, M = 262144, eps = 0.002,
    K = 500) in the benchmark's launch configuration (stored schedule table,
    autograd form, one stream, reference self potential computed once and passed
    in) against the stored
    FP64 oracle pass of the cross and trajectory-self solves: the gradient with
    respect to the samples, the gauge-fixed cross potentials, the self potential
    and the extrapolated ones."""
    F = _fixture("roofline_2d_full")
    cfg = W.CONFIGS["roofline_2d"]
    x, y, w, _g = W.config_inputs(cfg)
    T, M, K = len(x), len(y), cfg.iters
    assert (T, M, K) == (int(F["T"]), int(F["M"]), int(F["iters"]))
    dev = torch.device("cuda")
    xt, yt, wt = (torch.as_tensor(a, device=dev) for a in (x, y, w))
    q = ct.reference_self_potential(yt, wt, eps=cfg.eps, iters=K)
    xr = xt.clone().requires_grad_(True)
    S = ct.sinkhorn_divergence(xr, yt, wt, eps=cfg.eps, iters=K, one_stream=True, ref_q=q,
                               expanded=expanded)
    S.backward()
    out = ct.sinkhorn_grad(xt, yt, wt, eps=cfg.eps, iters=K, value=True, grad_w=True,
                           potentials=True, one_stream=True, ref_q=q, expanded=expanded)
    torch.cuda.synchronize()
    assert torch.equal(out.grad_x, xr.grad)
    pot = out.pot.cpu().numpy()
    pp = out.pot_plus.cpu().numpy()
    f1, g1 = gauge(pot[:T], pot[T:T + M], T, M)
    f2, g2 = gauge(F["f"], F["g"], T, M)
    c1, c2 = f1[0] - pot[0], f2[0] - F["f"][0]       # f+ carries the gauge of f
    e = dict(grad_x=rel(xr.grad.cpu().numpy(), F["grad_x"]), f=rel(f1, f2), g=rel(g1, g2),
             p=rel(pot[T + M:2 * T + M], F["p"]),
             f_plus=rel(pp[:T].astype(np.float64) + c1, F["f_plus"] + c2),
             p_plus=rel(pp[T + M:2 * T + M], F["p_plus"]))
    print("roofline_2d_full", "expanded" if expanded else "",
          " ".join(f"{k}={v:.2e}" for k, v in e.items()))
    assert max(e.values()) < TOL, e
    assert np.isfinite(S.item())


def test_batch_against_stored_oracle_sample(ct):
    """The full 256-problem ragged batch through the batched path (lockstep
    launches), eagerly and as a replayed graph: the gradients of 16 of its
    problems against their stored FP64 oracle passes."""
    F = _fixture("batched_2d_sample16")
    cfg = W.CONFIGS["batched_2d"]
    probs = W.batch_inputs(cfg)
    dev = torch.device("cuda")
    xs = [torch.as_tensor(p[0], device=dev) for p in probs]
    ys = [torch.as_tensor(p[1], device=dev) for p in probs]
    bs = ct.BatchedSinkhorn(xs, ys, None, eps=cfg.eps, iters=cfg.iters)
    bs.run()
    torch.cuda.synchronize()
    eager = bs.grad_x.clone()
    g = bs.capture()
    for _ in range(2):
        bs.grad_x.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(bs.grad_x, eager)
    gx = bs.split(eager, bs.T_off)
    off = np.concatenate([[0], np.cumsum(F["T"])])
    errs = []
    for i, b in enumerate(F["problems"]):
        b = int(b)
        assert (len(probs[b][0]), len(probs[b][1])) == (int(F["T"][i]), int(F["M"][i]))
        errs.append(rel(gx[b].cpu().numpy(), F["grad_x"][off[i]:off[i + 1]]))
    print("batched_2d sample of 16: max grad_x error %.2e, median %.2e" %
          (max(errs), float(np.median(errs))))
    assert max(errs) < TOL, errs


def test_backward_against_central_differences_of_converged_oracle(ct):
    """The autograd backward at convergence (3-D workload at T = 2048, M = 8192,
    eps = 0.01, weights in [0.5, 2]) against central differences (h = 1e-4) of the
    converged FP64 objective on 64 seeded sample coordinates and 64 weights,
    stored by the fixture script.  Per coordinate the GPU gradient must agree to
    1e-5 of max(|difference quotient|, 5 % of the largest gradient entry); the
    converged oracle gradient itself is checked norm-wise at 1e-5."""
    F = _fixture("fd_3d_T2048_M8192")
    cfg = W.CONFIGS["autograd_3d"]
    T, M = int(F["T"]), int(F["M"])
    x, y, _w, _g = W.config_inputs(cfg, T=T, M=M)
    w = F["w"].astype(np.float32)
    dev = torch.device("cuda")
    xt = torch.as_tensor(x, device=dev).requires_grad_(True)
    wt = torch.as_tensor(w, device=dev).requires_grad_(True)
    S = ct.sinkhorn_divergence(xt, torch.as_tensor(y, device=dev), wt, eps=cfg.eps, iters=3000)
    S.backward()
    torch.cuda.synchronize()
    gx = xt.grad.cpu().numpy().astype(np.float64)
    gw = wt.grad.cpu().numpy().astype(np.float64)
    ex, ew = rel(gx, F["grad_x"]), rel(gw, F["grad_w"])
    fx = gx.ravel()[F["x_coords"]]
    fw = gw[F["w_coords"]]
    sx = np.maximum(np.abs(F["fd_x"]), 0.05 * np.abs(gx).max())
    sw = np.maximum(np.abs(F["fd_w"]), 0.05 * np.abs(gw).max())
    cx, cw = np.abs(fx - F["fd_x"]) / sx, np.abs(fw - F["fd_w"]) / sw
    print("fd_3d: norm-wise grad_x %.2e grad_w %.2e; per coordinate vs FD: x max %.2e median "
          "%.2e, w max %.2e median %.2e" % (ex, ew, cx.max(), np.median(cx), cw.max(),
                                            np.median(cw)))
    assert ex < TOL and ew < TOL
    assert cx.max() < TOL and cw.max() < TOL, (cx.max(), cw.max())
