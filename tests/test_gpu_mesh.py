"""The exchange solve (CT_MESH: all K Sinkhorn iterations in one launch of
workgroups that each hold every point in LDS, own at most 64 rows of x and of
y, and pass their rows' new potentials to each other as versioned words instead
of meeting at grid barriers) against the FP64 oracle (Sec. II-B, eqs. 5-7) and
against the other executions.

Sizes cover two blocks, blocks without rows of one point set (T or M far below
the other), ragged row ranges, d = 2 and 3, the planner's short-horizon shapes
and the largest problems whose points fit in one workgroup's LDS; warm starts
with rescued rows, a cached reference potential, the safe (tracked-maximum)
mode and the give-up path (waits that no version satisfies, forced from the
host: every kernel still finishes, the outputs are NaN and the status query
reports CT_E_DEVICE)."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as W
from helpers import rel
from test_gpu_fused import TOL, _errs, _run

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d,T,M,eps,iters", [
    (2, 65, 70, 0.01, 30),
    (2, 129, 1, 0.01, 10),
    (2, 1, 200, 0.01, 10),
    (3, 100, 100, 0.01, 100),
    (2, 256, 512, 0.01, 100),
    (3, 300, 300, 0.01, 50),
    (3, 500, 430, 0.02, 40),
    (2, 700, 1500, 0.005, 40),
    (3, 1000, 1000, 0.01, 30),
])
def test_mesh_matches_oracle(ct, d, T, M, eps, iters):
    cfg = W.CONFIGS["grad_2d"] if d == 2 else W.CONFIGS["autograd_3d"]
    x, y, w, _g = W.config_inputs(cfg, T=T, M=M)
    print(f"exchange parity d={d} T={T} M={M} eps={eps} K={iters}", flush=True)
    g = _run(ct, x, y, w, eps, iters, fused="mesh")
    r = oracle.sinkhorn(x, y, w, eps=eps, iters=iters)
    e = _errs(g, r, T, M, w)
    print(" ".join(f"{k}={v:.2e}" for k, v in e.items()))
    assert max(e.values()) < TOL, e
    assert g["aux"][6] == 0.0


def test_mesh_agrees_with_other_executions_and_is_deterministic(ct):
    x, y, w, _g = W.config_inputs(W.CONFIGS["grad_2d"], T=600, M=900)
    w = W.positive_weights(np.random.default_rng(17), 900)
    a = _run(ct, x, y, w, 0.01, 60, fused="mesh")
    b = _run(ct, x, y, w, 0.01, 60, fused=False)
    c = _run(ct, x, y, w, 0.01, 60, fused="mesh")
    for k in ("grad_x", "grad_w"):
        assert rel(a[k], b[k]) < 2e-6, (k, rel(a[k], b[k]))
    for k in ("grad_x", "grad_w", "value", "pot"):
        assert np.array_equal(a[k], c[k]), k


def test_mesh_not_debiased_warm_start_rescue_and_safe_mode(ct):
    T, M = 200, 450
    x, y, _w, _g = W.config_inputs(W.CONFIGS["grad_2d"], T=T, M=M)
    w = W.positive_weights(np.random.default_rng(13), M)
    g = _run(ct, x, y, w, 0.01, 40, fused="mesh", debias=False)
    r = oracle.sinkhorn(x, y, w, eps=0.01, iters=40, debias=False)
    e = _errs(g, r, T, M, w, debias=False)
    assert max(e.values()) < TOL, ("not debiased", e)
    # a warm start far from the fixed point: the lagged shifts of the first
    # iteration are unusable and the rows are recomputed with a tracked maximum
    init = np.zeros(2 * T + 2 * M, dtype=np.float64)
    init[:T] = 3.0
    init[T:T + M] = -1.0
    init[T + M:2 * T + M] = -2.0
    g = _run(ct, x, y, w, 0.01, 20, fused="mesh", init=init)
    assert g["aux"][4] > 0, "rescue path was not exercised"
    r = oracle.sinkhorn(x, y, w, eps=0.01, iters=20,
                        init=(init[:T], init[T:T + M], init[T + M:2 * T + M], init[2 * T + M:]))
    e = _errs(g, r, T, M, w)
    assert max(e.values()) < TOL, ("rescue", e)
    g = _run(ct, x, y, w, 0.01, 30, fused="mesh", safe=True)
    r = oracle.sinkhorn(x, y, w, eps=0.01, iters=30)
    e = _errs(g, r, T, M, w)
    assert max(e.values()) < TOL, ("safe", e)


def test_mesh_cached_reference_and_planner(ct):
    cfg = W.CONFIGS["planner_2d"]
    x, y, w, _g = W.config_inputs(cfg)
    dev = torch.device("cuda")
    q = ct.reference_self_potential(torch.as_tensor(y, device=dev), torch.as_tensor(w, device=dev),
                                    eps=cfg.eps, iters=cfg.iters)
    g = _run(ct, x, y, w, cfg.eps, cfg.iters, fused="mesh", ref_q=q.cpu().numpy())
    full = _run(ct, x, y, w, cfg.eps, cfg.iters, fused=False)
    assert rel(g["grad_x"], full["grad_x"]) < TOL
    assert rel(g["grad_w"], full["grad_w"]) < TOL
    # one planner step through the exchange solve against the oracle planner
    e = cfg.extra
    u0 = np.random.default_rng(cfg.seed + 1).normal(size=(cfg.T, 2)) * e["u_std"]
    s0 = np.array(e["s0"])
    Q, R = np.eye(2), 0.01 * np.eye(2)
    u1, _s, hist = ct.plan("double_integrator", s0, u0, e["dt"], Q, R, "sinkhorn", 1, 0.5,
                           y=torch.as_tensor(y, device=dev), w=torch.as_tensor(w, device=dev),
                           eps=cfg.eps, iters=cfg.iters, fused="mesh")
    r_u1, _rs, r_obj, _ra, _rv = oracle.plan_step("double_integrator", s0, u0, e["dt"], Q, R,
                                                 "sinkhorn", step=0.5, y=y, w=w, eps=cfg.eps,
                                                 iters=cfg.iters)
    assert abs(hist[0] - r_obj) / abs(r_obj) < TOL
    assert rel(u1 - u0, r_u1 - u0) < TOL


def test_mesh_at_the_longest_sinkhorn_horizon(ct):
    """T = M = 2500 in 3-D (the longest horizon of the paper's Sinkhorn sweep), the
    reference self potential cached as the planner does: 40 workgroups, each with
    every point in LDS; against the per-sweep launches with the same cached
    potential, and the uncached 2-D case T = 1200, M = 2000 against the oracle."""
    dev = torch.device("cuda")
    cfg = W.CONFIGS["autograd_3d"]
    x, y, w, _g = W.config_inputs(cfg, T=2500, M=2500)
    q = ct.reference_self_potential(torch.as_tensor(y, device=dev), torch.as_tensor(w, device=dev),
                                    eps=0.01, iters=30)
    print("exchange T=M=2500 d=3 cached reference potential", flush=True)
    a = _run(ct, x, y, w, 0.01, 30, fused="mesh", ref_q=q.cpu().numpy())
    b = _run(ct, x, y, w, 0.01, 30, fused=False, ref_q=q.cpu().numpy())
    for k in ("grad_x", "grad_w"):
        assert rel(a[k], b[k]) < 2e-6, (k, rel(a[k], b[k]))
    cfg = W.CONFIGS["grad_2d"]
    x, y, w, _g = W.config_inputs(cfg, T=1200, M=2000)
    g = _run(ct, x, y, w, 0.01, 25, fused="mesh")
    r = oracle.sinkhorn(x, y, w, eps=0.01, iters=25)
    e = _errs(g, r, 1200, 2000, w)
    assert max(e.values()) < TOL, e


def test_mesh_rejects_problems_it_cannot_plan(ct):
    # one block's worth of rows: the one-workgroup solve's case
    x, y, w, _g = W.config_inputs(W.CONFIGS["grad_2d"], T=40, M=64)
    with pytest.raises(ct.CtError) as e:
        _run(ct, x, y, w, 0.01, 5, fused="mesh")
    assert e.value.code == -6
    # more points than one workgroup's LDS holds
    x, y, w, _g = W.config_inputs(W.CONFIGS["grad_2d"], T=3000, M=4000)
    with pytest.raises(ct.CtError) as e:
        _run(ct, x, y, w, 0.01, 5, fused="mesh")
    assert e.value.code == -6


def test_mesh_give_up_is_flagged(ct, monkeypatch):
    """Waits that no version satisfies, bounded at 16 polls: the first wait gives
    up, every later one passes at once, the kernel ends, grad_x, grad_w and the
    value are NaN and the status query returns CT_E_DEVICE.  The next call on the
    same workspace starts from cleared words and is valid again."""
    from paper_2511_11514_amd import _lib as L
    dev = torch.device("cuda")
    x, y, w, _g = W.config_inputs(W.CONFIGS["grad_2d"], T=300, M=500)
    xt, yt, wt = (torch.as_tensor(a, device=dev) for a in (x, y, w))
    T, M = len(x), len(y)
    o = L.SinkhornOpts(2, 20, 0.01, L.CT_DEBIAS | L.CT_VALUE | L.CT_GRAD_W | L.CT_MESH)
    nbytes = L.lib().ct_sinkhorn_workspace_size(T, M, ctypes.byref(o))
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    gx = torch.empty_like(xt)
    gw = torch.empty(M, dtype=torch.float32, device=dev)
    val = torch.empty(1, dtype=torch.float32, device=dev)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)

    def call():
        st = L.lib().ct_sinkhorn_grad(p(xt), T, p(yt), p(wt), M, ctypes.byref(o), p(gx), p(gw),
                                      p(val), None, None, None, p(ws), nbytes, stream)
        assert st == L.CT_OK, L.lib().ct_last_error()
        return L.lib().ct_status_sync(p(ws), ctypes.c_float(0.0), None, None, None, stream)

    monkeypatch.setenv("CT_MESH_WAIT_POLLS", "16")
    monkeypatch.setenv("CT_MESH_UNSATISFIABLE_WAITS", "1")
    print("exchange give-up path: T=300 M=500 K=20, unsatisfiable waits", flush=True)
    assert call() == L.CT_E_DEVICE
    assert torch.isnan(gx).all() and torch.isnan(gw).all() and torch.isnan(val).all()
    monkeypatch.delenv("CT_MESH_UNSATISFIABLE_WAITS")
    monkeypatch.delenv("CT_MESH_WAIT_POLLS")
    assert call() == L.CT_OK
    assert torch.isfinite(gx).all() and torch.isfinite(gw).all() and torch.isfinite(val).all()
