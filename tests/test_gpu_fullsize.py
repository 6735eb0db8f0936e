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


def _fixture(name):
    path = os.path.join(GOLD, name + ".npz")
    if not os.path.exists(path):
        pytest.skip(f"fixture {name} not generated (tests/golden/make_oracle_fixtures.py)")
    return np.load(path, allow_pickle=False)


@pytest.mark.parametrize("name", ["planner_2d_full", "grad_2d_full", "autograd_3d_T4096_M16384",
                                  "roofline_2d_T4096_M16384"])
def test_sinkhorn_against_stored_oracle(ct, name):
    F = _fixture(name)
    cfg = W.CONFIGS[str(F["workload"])]
    T, M, K = int(F["T"]), int(F["M"]), int(F["iters"])
    x, y, w, _g = W.config_inputs(cfg, T=T, M=M)
    dev = torch.device("cuda")
    t = lambda a: torch.as_tensor(a, device=dev)
    out = ct.sinkhorn_grad(t(x), t(y), t(w), eps=cfg.eps, iters=K, value=True, grad_w=True,
                           potentials=True)
    torch.cuda.synchronize()
    pot = out.pot.cpu().numpy()
    f1, g1 = gauge(pot[:T], pot[T:T + M], T, M)
    f2, g2 = gauge(F["f"], F["g"], T, M)
    e = dict(grad_x=rel(out.grad_x.cpu().numpy(), F["grad_x"]),
             grad_w=rel(out.grad_w.cpu().numpy(), F["grad_w"]),
             value=abs(out.value.item() - float(F["value"])) / abs(float(F["value"])),
             f=rel(f1, f2), g=rel(g1, g2),
             p=rel(pot[T + M:2 * T + M], F["p"]), q=rel(pot[2 * T + M:], F["q"]))
    print(name, " ".join(f"{k}={v:.2e}" for k, v in e.items()))
    assert max(e.values()) < TOL, e


@pytest.mark.parametrize("name", ["grad_2d_full_svgd", "roofline_2d_T16384_svgd"])
def test_svgd_against_stored_oracle(ct, name):
    F = _fixture(name)
    cfg = W.CONFIGS[str(F["workload"])]
    x, _y, _w, g = W.config_inputs(cfg, T=int(F["T"]), M=16)
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
