"""Batched path (ct_sinkhorn_grad_batched), in its three executions — lockstep
launches over job tables (CT_UNFUSED), the persistent work-list kernel
(CT_PERSISTENT) and the exchange solve of every problem in one launch (CT_MESH,
the default where it applies) — against the FP64 oracle per problem and against
the per-problem path; graph capture and replay."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def _ragged(seed, B, tmax, mmax, d=2):
    rng = np.random.default_rng(seed)
    probs = []
    for b in range(B):
        T = int(rng.integers(1, tmax + 1)) if b % 3 else int(rng.integers(1, 4))
        M = int(rng.integers(1, mmax + 1))
        g = W.gmm_params(rng, int(rng.integers(2, 7)), d, 0.03, 0.12)
        probs.append((W.random_walk(rng, T, d), W.gmm_sample(rng, g, M), W.positive_weights(rng, M)))
    return probs


def _batch(ct, probs, eps, iters, **kw):
    dev = torch.device("cuda")
    t = lambda a: torch.as_tensor(a, device=dev)
    bs = ct.BatchedSinkhorn([t(p[0]) for p in probs], [t(p[1]) for p in probs],
                            [t(p[2]) for p in probs], eps=eps, iters=iters, value=True,
                            grad_w=True, **kw)
    return bs


MODES = [pytest.param("lockstep", id="lockstep"), pytest.param("persistent", id="persistent"),
         pytest.param("mesh", id="mesh")]
LARGE_MODES = MODES[:2]   # problems too large for the exchange solve


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("d", [2, 3])
def test_ragged_batch_matches_oracle(ct, d, mode):
    probs = _ragged(11 + d, 9, 700, 1500, d)
    eps, iters = 0.01, 25
    print(f"batched parity d={d} mode={mode}", flush=True)
    bs = _batch(ct, probs, eps, iters, mode=mode)
    bs.run()
    torch.cuda.synchronize()
    gx = bs.split(bs.grad_x.cpu().numpy(), bs.T_off)
    gw = bs.split(bs.grad_w.cpu().numpy(), bs.M_off)
    val = bs.value.cpu().numpy()
    assert np.isfinite(val).all()
    for b, (x, y, w) in enumerate(probs):
        r = oracle.sinkhorn(x, y, w, eps=eps, iters=iters)
        e = (rel(gx[b], r.grad_x), rel(gw[b], r.grad_w), abs(val[b] - r.value) / abs(r.value))
        assert max(e) < TOL, (b, len(x), len(y), e)


@pytest.mark.parametrize("mode", MODES)
def test_batched_equals_plain_and_graph_replay(ct, mode):
    probs = _ragged(21, 12, 700, 1200)
    eps, iters = 0.01, 30
    dev = torch.device("cuda")
    print(f"batched vs plain and graph replay mode={mode}", flush=True)
    bs = _batch(ct, probs, eps, iters, mode=mode)
    bs.run()
    torch.cuda.synchronize()
    ref_x = bs.grad_x.clone()
    ref_w = bs.grad_w.clone()
    ref_v = bs.value.clone()
    for b, (x, y, w) in enumerate(probs):
        out = ct.sinkhorn_grad(torch.as_tensor(x, device=dev), torch.as_tensor(y, device=dev),
                               torch.as_tensor(w, device=dev), eps=eps, iters=iters, value=True,
                               grad_w=True)
        gx = ref_x[bs.T_off[b]:bs.T_off[b + 1]]
        assert rel(gx.cpu().numpy(), out.grad_x.cpu().numpy()) < 2e-6
        assert abs(ref_v[b].item() - out.value.item()) <= 2e-6 * abs(out.value.item())
    # graph capture and replays, with eager work in between: each replay equals eager
    g = bs.capture()
    for rep in range(3):
        bs.grad_x.zero_()
        bs.value.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(bs.grad_x, ref_x), rep
        assert torch.equal(bs.grad_w, ref_w), rep
        assert torch.equal(bs.value, ref_v), rep
        _ = (torch.randn(1000, device=dev) ** 2).sum().item()


def test_unprepared_workspace_is_rejected(ct):
    import ctypes
    from paper_2511_11514_amd import _lib
    probs = _ragged(31, 3, 50, 80)
    bs = _batch(ct, probs, 0.05, 5)
    other = torch.empty_like(bs.ws)
    st = _lib.lib().ct_sinkhorn_grad_batched(bs.B, bs._to, bs._mo, ctypes.c_void_p(bs.x.data_ptr()),
                                             ctypes.c_void_p(bs.y.data_ptr()), None,
                                             ctypes.byref(bs.o),
                                             ctypes.c_void_p(bs.grad_x.data_ptr()), None, None,
                                             ctypes.c_void_p(other.data_ptr()), bs.nbytes, None)
    assert st == _lib.CT_E_ARG


@pytest.mark.parametrize("mode", LARGE_MODES)
def test_scaled_batch_workload_sampled(ct, mode):
    """The 256-problem batch shape at 1/8 of its sizes; four problems checked."""
    cfg = W.CONFIGS["batched_2d"]
    probs = W.batch_inputs(cfg, B=48, scale=0.125)
    bs = _batch(ct, probs, cfg.eps, 40, mode=mode)
    bs.run()
    torch.cuda.synchronize()
    gx = bs.split(bs.grad_x.cpu().numpy(), bs.T_off)
    val = bs.value.cpu().numpy()
    for b in (0, 7, 23, 47):
        x, y, w = probs[b]
        r = oracle.sinkhorn(x, y, w, eps=cfg.eps, iters=40)
        assert rel(gx[b], r.grad_x) < TOL and abs(val[b] - r.value) < TOL * abs(r.value)


def test_mode_mismatch_is_rejected(ct):
    """A workspace prepared for lockstep launches is not valid for the persistent
    kernel (the mode is part of what was prepared)."""
    import ctypes
    from paper_2511_11514_amd import _lib
    probs = _ragged(41, 3, 50, 80)
    bs = _batch(ct, probs, 0.05, 5, mode="lockstep")
    o = _lib.SinkhornOpts(bs.o.d, bs.o.iters, bs.o.eps,
                          (bs.o.flags & ~_lib.CT_UNFUSED) | _lib.CT_PERSISTENT)
    P = ctypes.c_void_p
    st = _lib.lib().ct_sinkhorn_grad_batched(bs.B, bs._to, bs._mo, P(bs.x.data_ptr()),
                                             P(bs.y.data_ptr()), P(bs.w.data_ptr()), ctypes.byref(o),
                                             P(bs.grad_x.data_ptr()), P(bs.grad_w.data_ptr()),
                                             P(bs.value.data_ptr()), P(bs.ws.data_ptr()), bs.nbytes,
                                             None)
    assert st == _lib.CT_E_ARG


@pytest.mark.parametrize("mode", [None, "lockstep"])
@pytest.mark.parametrize("iters,debias,safe", [(0, True, False), (1, True, False), (6, False, False),
                                               (6, True, True)])
def test_lockstep_edge_cases(ct, iters, debias, safe, mode):
    """Lockstep launches, and the default execution (the exchange solve at these
    sizes): no iteration, one (cold) iteration, the non-debiased and the
    tracked-maximum modes, on a batch with single-point and tiny problems."""
    probs = _ragged(51, 7, 300, 600)
    probs[0] = (probs[0][0][:1], probs[0][1][:1], probs[0][2][:1])
    eps = 0.02
    dev = torch.device("cuda")
    t = lambda a: torch.as_tensor(a, device=dev)
    bs = ct.BatchedSinkhorn([t(p[0]) for p in probs], [t(p[1]) for p in probs],
                            [t(p[2]) for p in probs], eps=eps, iters=iters, debias=debias,
                            value=True, grad_w=True, safe=safe, mode=mode)
    bs.run()
    torch.cuda.synchronize()
    gx = bs.split(bs.grad_x.cpu().numpy(), bs.T_off)
    gw = bs.split(bs.grad_w.cpu().numpy(), bs.M_off)
    val = bs.value.cpu().numpy()
    for b, (x, y, w) in enumerate(probs):
        r = oracle.sinkhorn(x, y, w, eps=eps, iters=iters, debias=debias)
        scale = max(np.abs(r.grad_x).max(), 1e-30)
        assert np.abs(gx[b] - r.grad_x).max() <= TOL * scale + 1e-7, b
        assert rel(gw[b], r.grad_w) < TOL or np.abs(gw[b] - r.grad_w).max() < 1e-6, b
        assert abs(val[b] - r.value) <= TOL * abs(r.value) + 1e-7, b


def test_expired_persistent_wait_flags_every_output(ct, monkeypatch):
    """The persistent kernel's dependency waits are bounded; when one expires (forced
    here from the host: a bound of zero polls, so every wait that is not satisfied
    at once gives up and the kernel still runs to its end), every gradient and
    value of the call is NaN; with the normal bound the same prepared batch gives
    the oracle's results again."""
    probs = _ragged(77, 3, 3000, 5000)
    eps, iters = 0.01, 8
    bs = _batch(ct, probs, eps, iters, mode="persistent")
    monkeypatch.setenv("CT_PERSISTENT_WAIT_POLLS", "0")
    bs.run()
    torch.cuda.synchronize()
    assert torch.isnan(bs.grad_x).all() and torch.isnan(bs.grad_w).all()
    assert torch.isnan(bs.value).all()
    monkeypatch.delenv("CT_PERSISTENT_WAIT_POLLS")
    bs.run()
    torch.cuda.synchronize()
    gx = bs.split(bs.grad_x, bs.T_off)
    for b, (x, y, w) in enumerate(probs):
        r = oracle.sinkhorn(x, y, w, eps=eps, iters=iters)
        assert rel(gx[b].cpu().numpy(), r.grad_x) < TOL


@pytest.mark.parametrize("mode", MODES)
def test_problems_far_from_coordinate_origin(ct, mode):
    """Each problem shifted far from the coordinate origin, by a different offset:
    the staging centres every problem on its own mean before the sqrt(kappa)
    prescale, so the batch matches the oracle at the same bar as near the origin."""
    probs = []
    for b, (x, y, w) in enumerate(_ragged(41, 6, 600, 1200)):
        shift = np.array([300.0 + 170.0 * b, -220.0 + 45.0 * b])
        probs.append(((x.astype(np.float64) + shift).astype(np.float32),
                      (y.astype(np.float64) + shift).astype(np.float32), w))
    eps, iters = 0.01, 25
    bs = _batch(ct, probs, eps, iters, mode=mode)
    bs.run()
    torch.cuda.synchronize()
    gx = bs.split(bs.grad_x.cpu().numpy(), bs.T_off)
    gw = bs.split(bs.grad_w.cpu().numpy(), bs.M_off)
    val = bs.value.cpu().numpy()
    for b, (x, y, w) in enumerate(probs):
        r = oracle.sinkhorn(x, y, w, eps=eps, iters=iters)
        e = (rel(gx[b], r.grad_x), rel(gw[b], r.grad_w), abs(val[b] - r.value) / abs(r.value))
        assert max(e) < TOL, (b, len(x), len(y), e)


def test_mesh_batch_give_up_flags_every_output(ct, monkeypatch):
    """The exchange solve's waits are bounded; with waits that no version
    satisfies (forced from the host when the batch is prepared, bounded at 16
    polls) every gradient and value of the call is NaN and every kernel finishes;
    a batch prepared without the hook gives the oracle's results."""
    probs = _ragged(83, 5, 400, 700)
    eps, iters = 0.01, 10
    monkeypatch.setenv("CT_MESH_WAIT_POLLS", "16")
    monkeypatch.setenv("CT_MESH_UNSATISFIABLE_WAITS", "1")
    bs = _batch(ct, probs, eps, iters, mode="mesh")
    monkeypatch.delenv("CT_MESH_UNSATISFIABLE_WAITS")
    monkeypatch.delenv("CT_MESH_WAIT_POLLS")
    print("batched exchange give-up path", flush=True)
    bs.run()
    torch.cuda.synchronize()
    assert torch.isnan(bs.grad_x).all() and torch.isnan(bs.grad_w).all()
    assert torch.isnan(bs.value).all()
    bs = _batch(ct, probs, eps, iters, mode="mesh")
    bs.run()
    torch.cuda.synchronize()
    gx = bs.split(bs.grad_x, bs.T_off)
    for b, (x, y, w) in enumerate(probs):
        r = oracle.sinkhorn(x, y, w, eps=eps, iters=iters)
        assert rel(gx[b].cpu().numpy(), r.grad_x) < TOL


def test_mesh_batch_rejects_problems_it_cannot_take(ct):
    """CT_MESH for a batch with a problem whose points do not fit in one
    workgroup's LDS (T = 3000, M = 4000)."""
    rng = np.random.default_rng(87)
    probs = _ragged(87, 3, 200, 300)
    g = W.gmm_params(rng, 3, 2, 0.03, 0.12)
    probs[1] = (W.random_walk(rng, 3000, 2), W.gmm_sample(rng, g, 4000), W.positive_weights(rng, 4000))
    with pytest.raises(ct.CtError) as e:
        _batch(ct, probs, 0.01, 5, mode="mesh")
    assert e.value.code == -6


def test_lockstep_difference_form_matches_oracle(ct):
    """The lockstep launches with the difference form (CT_DIFFERENCE; the default
    lagged sweeps use the expanded exponent) against the oracle."""
    probs = _ragged(29, 7, 900, 1600)
    eps, iters = 0.01, 25
    bs = _batch(ct, probs, eps, iters, expanded=False, mode="lockstep")
    bs.run()
    torch.cuda.synchronize()
    gx = bs.split(bs.grad_x.cpu().numpy(), bs.T_off)
    gw = bs.split(bs.grad_w.cpu().numpy(), bs.M_off)
    for b, (x, y, w) in enumerate(probs):
        r = oracle.sinkhorn(x, y, w, eps=eps, iters=iters)
        e = (rel(gx[b], r.grad_x), rel(gw[b], r.grad_w))
        assert max(e) < TOL, (b, len(x), len(y), e)
