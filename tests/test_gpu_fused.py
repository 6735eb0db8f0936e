"""The fused solve (CT_FUSED: all K Sinkhorn iterations in one launch, grid-wide
barriers between half-iterations) against the FP64 oracle (Sec. II-B, eqs. 5-7)
and against the per-sweep launches (CT_UNFUSED).

Sizes cover one block (a single unit per half-iteration), many blocks with key
splits merged by arrival tickets, ragged tails, d = 2 and 3, the planner's
short-horizon shapes, warm starts, a cached reference potential and the safe
(tracked-maximum) mode.  The give-up path of the barrier is forced from the
host (waits that no arrival count satisfies, a small poll bound): every kernel
still finishes, the outputs are NaN and the status query reports CT_E_DEVICE."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import gauge, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def _run(ct, x, y, w, eps, iters, fused, debias=True, init=None, ref_q=None, safe=False):
    dev = torch.device("cuda")
    t = lambda a: torch.as_tensor(a, device=dev)
    out = ct.sinkhorn_grad(t(x), t(y), None if w is None else t(w), eps=eps, iters=iters,
                           debias=debias, value=True, grad_w=True, potentials=True, aux=True,
                           init=None if init is None else t(init.astype(np.float32)),
                           ref_q=None if ref_q is None else t(ref_q.astype(np.float32)),
                           safe=safe, fused=fused)
    torch.cuda.synchronize()
    return {k: (None if v is None else v.cpu().numpy()) for k, v in out.__dict__.items()}


def _errs(g, r, T, M, w, debias=True):
    b = None if w is None else np.asarray(w, np.float64) / np.sum(w, dtype=np.float64)
    e = dict(grad_x=rel(g["grad_x"], r.grad_x), grad_w=rel(g["grad_w"], r.grad_w),
             value=abs(float(g["value"][0]) - r.value) / max(abs(r.value), 1e-30))
    pot = g["pot"]
    f1, g1 = gauge(pot[:T], pot[T:T + M], T, M, b)
    f2, g2 = gauge(r.f, r.g, T, M, b)
    e["f"], e["g"] = rel(f1, f2), rel(g1, g2)
    if debias:
        e["p"] = rel(pot[T + M:2 * T + M], r.p)
        e["q"] = rel(pot[2 * T + M:], r.q)
    return e


@pytest.mark.parametrize("d,T,M,eps,iters", [
    (2, 1, 1, 0.01, 5),
    (2, 37, 53, 0.01, 30),
    (3, 100, 100, 0.01, 100),
    (2, 256, 512, 0.01, 100),
    (2, 700, 1500, 0.005, 60),
    (3, 1000, 1000, 0.01, 40),
    (3, 2500, 2500, 0.01, 20),
])
def test_fused_matches_oracle(ct, d, T, M, eps, iters):
    cfg = W.CONFIGS["grad_2d"] if d == 2 else W.CONFIGS["autograd_3d"]
    x, y, w, _g = W.config_inputs(cfg, T=T, M=M)
    print(f"fused parity d={d} T={T} M={M} eps={eps} K={iters}", flush=True)
    g = _run(ct, x, y, w, eps, iters, fused=True)
    r = oracle.sinkhorn(x, y, w, eps=eps, iters=iters)
    e = _errs(g, r, T, M, w)
    print(" ".join(f"{k}={v:.2e}" for k, v in e.items()))
    assert max(e.values()) < TOL, e
    assert g["aux"][6] == 0.0


def test_fused_and_unfused_agree(ct):
    """Same inputs through both executions: the split plans differ, so the sums
    are rounded in a different order; the results agree to float32 rounding."""
    x, y, w, _g = W.config_inputs(W.CONFIGS["grad_2d"], T=1200, M=3000)
    rng = np.random.default_rng(3)
    w = W.positive_weights(rng, 3000)
    a = _run(ct, x, y, w, 0.01, 50, fused=True)
    b = _run(ct, x, y, w, 0.01, 50, fused=False)
    for k in ("grad_x", "grad_w"):
        assert rel(a[k], b[k]) < 2e-6, (k, rel(a[k], b[k]))
    assert abs(a["value"][0] - b["value"][0]) <= 2e-6 * abs(b["value"][0])


def test_fused_is_deterministic(ct):
    x, y, w, _g = W.config_inputs(W.CONFIGS["grad_2d"], T=900, M=2100)
    a = _run(ct, x, y, w, 0.01, 40, fused=True)
    b = _run(ct, x, y, w, 0.01, 40, fused=True)
    for k in ("grad_x", "grad_w", "value", "pot"):
        assert np.array_equal(a[k], b[k]), k


def test_fused_not_debiased_weighted(ct):
    x, y, _w, _g = W.config_inputs(W.CONFIGS["grad_2d"], T=300, M=800)
    w = W.positive_weights(np.random.default_rng(11), 800)
    g = _run(ct, x, y, w, 0.01, 40, fused=True, debias=False)
    r = oracle.sinkhorn(x, y, w, eps=0.01, iters=40, debias=False)
    e = _errs(g, r, 300, 800, w, debias=False)
    assert max(e.values()) < TOL, e


def test_fused_warm_start_cached_reference_and_safe_mode(ct):
    cfg = W.CONFIGS["planner_2d"]
    x, y, w, _g = W.config_inputs(cfg)
    T, M = len(x), len(y)
    base = oracle.sinkhorn(x, y, w, eps=cfg.eps, iters=20)
    init = np.concatenate([base.f, base.g, base.p, base.q])
    g = _run(ct, x, y, w, cfg.eps, 30, fused=True, init=init)
    r = oracle.sinkhorn(x, y, w, eps=cfg.eps, iters=30, init=(base.f, base.g, base.p, base.q))
    e = _errs(g, r, T, M, w)
    assert max(e.values()) < TOL, ("warm", e)
    # reference potential cached (q computed once, not iterated in the call): the
    # same result as recomputing it, up to float32 rounding
    dev = torch.device("cuda")
    q = ct.reference_self_potential(torch.as_tensor(y, device=dev), torch.as_tensor(w, device=dev),
                                    eps=cfg.eps, iters=30)
    g = _run(ct, x, y, w, cfg.eps, 30, fused=True, ref_q=q.cpu().numpy())
    full = _run(ct, x, y, w, cfg.eps, 30, fused=True)
    assert rel(g["grad_x"], full["grad_x"]) < TOL
    assert rel(g["grad_w"], full["grad_w"]) < TOL
    g = _run(ct, x, y, w, cfg.eps, 30, fused=True, safe=True)
    r = oracle.sinkhorn(x, y, w, eps=cfg.eps, iters=30)
    e = _errs(g, r, T, M, w)
    assert max(e.values()) < TOL, ("safe", e)


def test_fused_barrier_give_up_is_flagged(ct, monkeypatch):
    """Waits that no arrival count satisfies, bounded at 16 polls: the first wait
    gives up, every later one passes at once, the kernel ends, grad_x, grad_w and
    the value are NaN and the status query returns CT_E_DEVICE.  The next call on
    the same workspace starts from cleared status words and is valid again."""
    import ctypes
    from paper_2511_11514_amd import _lib as L
    dev = torch.device("cuda")
    x, y, w, _g = W.config_inputs(W.CONFIGS["grad_2d"], T=2000, M=4000)
    xt, yt, wt = (torch.as_tensor(a, device=dev) for a in (x, y, w))
    T, M = len(x), len(y)
    o = L.SinkhornOpts(2, 20, 0.01, L.CT_DEBIAS | L.CT_VALUE | L.CT_GRAD_W | L.CT_FUSED)
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

    monkeypatch.setenv("CT_FUSED_WAIT_POLLS", "16")
    monkeypatch.setenv("CT_FUSED_UNSATISFIABLE_WAITS", "1")
    print("fused give-up path: T=2000 M=4000 K=20, unsatisfiable waits", flush=True)
    assert call() == L.CT_E_DEVICE
    assert torch.isnan(gx).all() and torch.isnan(gw).all() and torch.isnan(val).all()
    monkeypatch.delenv("CT_FUSED_UNSATISFIABLE_WAITS")
    monkeypatch.delenv("CT_FUSED_WAIT_POLLS")
    assert call() == L.CT_OK
    assert torch.isfinite(gx).all() and torch.isfinite(gw).all() and torch.isfinite(val).all()


# ---------------------------------------------------------------- one workgroup (CT_TINY)

@pytest.mark.parametrize("d,T,M,eps,iters", [
    (2, 1, 1, 0.01, 5),
    (2, 37, 53, 0.01, 30),
    (3, 100, 100, 0.01, 100),
    (2, 256, 512, 0.01, 100),
    (3, 300, 300, 0.01, 50),
    (2, 65, 1100, 0.005, 40),
    (3, 700, 600, 0.02, 20),
])
def test_one_workgroup_matches_oracle(ct, d, T, M, eps, iters):
    cfg = W.CONFIGS["grad_2d"] if d == 2 else W.CONFIGS["autograd_3d"]
    x, y, w, _g = W.config_inputs(cfg, T=T, M=M)
    print(f"one-workgroup parity d={d} T={T} M={M} eps={eps} K={iters}", flush=True)
    g = _run(ct, x, y, w, eps, iters, fused="tiny")
    r = oracle.sinkhorn(x, y, w, eps=eps, iters=iters)
    e = _errs(g, r, T, M, w)
    print(" ".join(f"{k}={v:.2e}" for k, v in e.items()))
    assert max(e.values()) < TOL, e


@pytest.mark.parametrize("rows_per_lane", [1, 2, 4])
@pytest.mark.parametrize("d,T,M", [(3, 150, 97), (2, 300, 260)])
def test_one_workgroup_every_rows_per_lane_matches_oracle(ct, monkeypatch, rows_per_lane, d, T, M):
    """Each plan shape of the one-workgroup solve (1, 2 or 4 query rows per lane,
    forced through the CT_TINY_R hook) on ragged sizes: row groups with a partial
    last group, key ranges with a short last range."""
    monkeypatch.setenv("CT_TINY_R", str(rows_per_lane))
    cfg = W.CONFIGS["grad_2d"] if d == 2 else W.CONFIGS["autograd_3d"]
    x, y, w, _g = W.config_inputs(cfg, T=T, M=M)
    w = W.positive_weights(np.random.default_rng(T + M), M)
    print(f"one-workgroup R={rows_per_lane} d={d} T={T} M={M}", flush=True)
    g = _run(ct, x, y, w, 0.01, 40, fused="tiny")
    r = oracle.sinkhorn(x, y, w, eps=0.01, iters=40)
    e = _errs(g, r, T, M, w)
    print(" ".join(f"{k}={v:.2e}" for k, v in e.items()))
    assert max(e.values()) < TOL, e


def test_one_workgroup_agrees_with_other_executions_and_is_deterministic(ct):
    x, y, w, _g = W.config_inputs(W.CONFIGS["grad_2d"], T=300, M=700)
    w = W.positive_weights(np.random.default_rng(5), 700)
    a = _run(ct, x, y, w, 0.01, 60, fused="tiny")
    b = _run(ct, x, y, w, 0.01, 60, fused=False)
    c = _run(ct, x, y, w, 0.01, 60, fused="tiny")
    for k in ("grad_x", "grad_w"):
        assert rel(a[k], b[k]) < 2e-6, (k, rel(a[k], b[k]))
    for k in ("grad_x", "grad_w", "value", "pot"):
        assert np.array_equal(a[k], c[k]), k


def test_one_workgroup_not_debiased_warm_start_rescue_and_safe_mode(ct):
    x, y, _w, _g = W.config_inputs(W.CONFIGS["grad_2d"], T=200, M=450)
    T, M = 200, 450
    w = W.positive_weights(np.random.default_rng(13), M)
    g = _run(ct, x, y, w, 0.01, 40, fused="tiny", debias=False)
    r = oracle.sinkhorn(x, y, w, eps=0.01, iters=40, debias=False)
    e = _errs(g, r, T, M, w, debias=False)
    assert max(e.values()) < TOL, ("not debiased", e)
    # a warm start far from the fixed point: every row's lagged shift is unusable in
    # the first iteration and the rows are recomputed with a tracked maximum
    init = np.zeros(2 * T + 2 * M, dtype=np.float64)
    init[:T] = 3.0
    init[T:T + M] = -1.0
    init[T + M:2 * T + M] = -2.0
    g = _run(ct, x, y, w, 0.01, 20, fused="tiny", init=init)
    assert g["aux"][4] > 0, "rescue path was not exercised"
    r = oracle.sinkhorn(x, y, w, eps=0.01, iters=20,
                        init=(init[:T], init[T:T + M], init[T + M:2 * T + M], init[2 * T + M:]))
    e = _errs(g, r, T, M, w)
    assert max(e.values()) < TOL, ("rescue", e)
    g = _run(ct, x, y, w, 0.01, 30, fused="tiny", safe=True)
    r = oracle.sinkhorn(x, y, w, eps=0.01, iters=30)
    e = _errs(g, r, T, M, w)
    assert max(e.values()) < TOL, ("safe", e)


def test_one_workgroup_cached_reference_and_planner(ct):
    cfg = W.CONFIGS["planner_2d"]
    x, y, w, _g = W.config_inputs(cfg)
    dev = torch.device("cuda")
    q = ct.reference_self_potential(torch.as_tensor(y, device=dev), torch.as_tensor(w, device=dev),
                                    eps=cfg.eps, iters=cfg.iters)
    g = _run(ct, x, y, w, cfg.eps, cfg.iters, fused="tiny", ref_q=q.cpu().numpy())
    full = _run(ct, x, y, w, cfg.eps, cfg.iters, fused=False)
    assert rel(g["grad_x"], full["grad_x"]) < TOL
    assert rel(g["grad_w"], full["grad_w"]) < TOL
    # one planner step through the one-workgroup solve against the oracle planner
    e = cfg.extra
    u0 = np.random.default_rng(cfg.seed + 1).normal(size=(cfg.T, 2)) * e["u_std"]
    s0 = np.array(e["s0"])
    Q, R = np.eye(2), 0.01 * np.eye(2)
    u1, _s, hist = ct.plan("double_integrator", s0, u0, e["dt"], Q, R, "sinkhorn", 1, 0.5,
                           y=torch.as_tensor(y, device=dev), w=torch.as_tensor(w, device=dev),
                           eps=cfg.eps, iters=cfg.iters, fused="tiny")
    r_u1, _rs, r_obj, _ra, _rv = oracle.plan_step("double_integrator", s0, u0, e["dt"], Q, R,
                                                 "sinkhorn", step=0.5, y=y, w=w, eps=cfg.eps,
                                                 iters=cfg.iters)
    assert abs(hist[0] - r_obj) / abs(r_obj) < TOL
    assert rel(u1 - u0, r_u1 - u0) < TOL


def test_one_workgroup_rejects_problems_beyond_its_lds(ct):
    x, y, w, _g = W.config_inputs(W.CONFIGS["grad_2d"], T=1000, M=3000)
    with pytest.raises(ct.CtError) as e:
        _run(ct, x, y, w, 0.01, 5, fused="tiny")
    assert e.value.code == -6
