"""GPU planner (ct_plan, Sec. II-C) against the oracle's outer loop.  Parity is
checked per outer step from identical controls (the end state of a multi-step
run is not unique, Sec. III-C), plus monotone decrease of S over the planner
workload's ten steps."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _c1():
    cfg = W.CONFIGS["planner_2d"]
    e = cfg.extra
    x, y, w, g = W.config_inputs(cfg)
    rng = np.random.default_rng(cfg.seed + 1)
    u0 = rng.normal(size=(cfg.T, 2)) * e["u_std"]
    return cfg, e, y, w, g, u0


def test_sinkhorn_plan_one_step_parity(ct):
    cfg, e, y, w, g, u0 = _c1()
    dev = torch.device("cuda")
    s0 = np.array(e["s0"])
    Q, R = np.eye(2), 0.01 * np.eye(2)
    u1, s, hist = ct.plan("double_integrator", s0, u0, e["dt"], Q, R, "sinkhorn", 1, 0.5,
                          y=torch.as_tensor(y, device=dev), w=torch.as_tensor(w, device=dev),
                          eps=cfg.eps, iters=cfg.iters)
    r_u1, r_s, r_obj, r_a, r_v = oracle.plan_step("double_integrator", s0, u0, e["dt"], Q, R,
                                                 "sinkhorn", step=0.5, y=y, w=w, eps=cfg.eps,
                                                 iters=cfg.iters)
    assert abs(hist[0] - r_obj) / abs(r_obj) < 1e-5
    assert rel(u1 - u0, r_u1 - u0) < 1e-5
    np.testing.assert_allclose(s, oracle.rollout("double_integrator", s0, u1, e["dt"]), rtol=1e-12)


def test_sinkhorn_plan_ten_steps_decrease(ct):
    cfg, e, y, w, g, u0 = _c1()
    dev = torch.device("cuda")
    s0 = np.array(e["s0"])
    Q, R = np.eye(2), 0.01 * np.eye(2)
    _u, _s, hist = ct.plan("double_integrator", s0, u0, e["dt"], Q, R, "sinkhorn", e["outer"], 0.5,
                           y=torch.as_tensor(y, device=dev), w=torch.as_tensor(w, device=dev),
                           eps=cfg.eps, iters=cfg.iters)
    _ru, _rs, rhist = oracle.plan("double_integrator", s0, u0, e["dt"], Q, R, "sinkhorn",
                                  e["outer"], step=0.5, y=y, w=w, eps=cfg.eps, iters=cfg.iters)
    assert np.all(np.diff(hist) < 0), hist
    assert hist[-1] < 0.05 * hist[0]
    np.testing.assert_allclose(hist, rhist, rtol=1e-3)


def test_svgd_unicycle_plan_one_step_parity(ct):
    cfg = W.CONFIGS["roofline_2d"]
    e = cfg.extra
    T = 700
    _x, _y, _w, g = W.config_inputs(cfg, T=T, M=16)
    rng = np.random.default_rng(cfg.seed + 1)
    u0 = np.stack([np.full(T, e["v0"]), rng.normal(size=T) * e["omega_std"]], axis=1)
    s0 = np.array(e["s0"])
    Q, R = np.eye(2), 0.01 * np.eye(2)
    dev = torch.device("cuda")
    u1, _s, hist = ct.plan("unicycle", s0, u0, e["dt"], Q, R, "svgd", 1, 0.5,
                           gmm=ct.GMM.from_numpy(g, dev))
    r_u1, _rs, r_obj, _ra, _rv = oracle.plan_step("unicycle", s0, u0, e["dt"], Q, R, "svgd",
                                                 step=0.5, gmm=g)
    assert abs(hist[0] - r_obj) / abs(r_obj) < 1e-5
    assert rel(u1 - u0, r_u1 - u0) < 1e-5


@pytest.mark.parametrize("name,T", [("sinkhorn_aircraft", 300), ("svgd_drive", 500)])
def test_horizon_sweep_workloads_one_step_parity(ct, name, T):
    """The horizon-sweep workloads (Stein flow with differential drive; Sinkhorn
    flow with the 3-D double integrator standing in for the aircraft): one outer
    step from identical controls matches the oracle's, and the GPU planner keeps
    decreasing its objective over the sweep's outer iterations."""
    c = W.HORIZON_SWEEPS[name]
    s0, u0, y, w, g = W.horizon_inputs(name, T)
    d = c["d"]
    Q, R = c["Q"] * np.eye(d), c["R"] * np.eye(u0.shape[1])
    dev = torch.device("cuda")
    kw = dict(gmm=ct.GMM.from_numpy(g, dev)) if c["flow"] == "svgd" else dict(
        y=torch.as_tensor(y, device=dev), w=torch.as_tensor(w, device=dev), eps=c["eps"],
        iters=c["iters"])
    okw = dict(gmm=g) if c["flow"] == "svgd" else dict(y=y, w=w, eps=c["eps"], iters=c["iters"])
    u1, _s, hist = ct.plan(c["dynamics"], s0, u0, c["dt"], Q, R, c["flow"], 1, c["step"], **kw)
    r_u1, _rs, r_obj, _ra, _rv = oracle.plan_step(c["dynamics"], s0, u0, c["dt"], Q, R, c["flow"],
                                                 step=c["step"], **okw)
    assert abs(hist[0] - r_obj) / abs(r_obj) < 1e-5
    assert rel(u1 - u0, r_u1 - u0) < 1e-5
    _u, s, hist = ct.plan(c["dynamics"], s0, u0, c["dt"], Q, R, c["flow"], c["outer"],
                          c["step"], **kw)
    if c["flow"] == "sinkhorn":
        assert np.all(np.diff(hist) < 0), hist
    else:
        # the Stein flow has no objective of its own: the samples' mean log-density
        # under the target mixture must rise
        s_init = oracle.rollout(c["dynamics"], s0, u0, c["dt"])
        lp = lambda st: oracle.gmm_logpdf(st[1:, :d], g.weights, g.means, g.sigmas, g.floor).mean()
        assert lp(s) > lp(s_init) + 5.0, (lp(s_init), lp(s))


def _ensemble_inputs(S, T):
    c = W.HORIZON_SWEEPS["sinkhorn_aircraft"]
    s0, _u0, y, w, g = W.horizon_inputs("sinkhorn_aircraft", T)
    rng = np.random.default_rng(123)
    U0 = rng.normal(size=(S, T, c["d"])) * c["u_std"] * (1.0 + np.arange(S))[:, None, None]
    Q, R = c["Q"] * np.eye(c["d"]), c["R"] * np.eye(c["d"])
    return c, s0, U0, y, w, Q, R


def test_plan_ensemble_matches_oracle_per_seed(ct):
    """Seed ensemble (ct_plan_ensemble): one outer step of every seed matches the
    oracle's step from that seed's controls, the reported values are the oracle's
    divergence of each final trajectory, and the best seed is their argmin."""
    S, T = 3, 200
    c, s0, U0, y, w, Q, R = _ensemble_inputs(S, T)
    dev = torch.device("cuda")
    U1, s, values, best = ct.plan_ensemble(c["dynamics"], s0, U0, c["dt"], Q, R, 1, c["step"],
                                           y=torch.as_tensor(y, device=dev),
                                           w=torch.as_tensor(w, device=dev), eps=c["eps"],
                                           iters=c["iters"])
    ref_vals = []
    for b in range(S):
        r_u1, _rs, _obj, _a, _v = oracle.plan_step(c["dynamics"], s0, U0[b], c["dt"], Q, R,
                                                  "sinkhorn", step=c["step"], y=y, w=w,
                                                  eps=c["eps"], iters=c["iters"])
        assert rel(U1[b] - U0[b], r_u1 - U0[b]) < 1e-5, b
        np.testing.assert_allclose(s[b], oracle.rollout(c["dynamics"], s0, U1[b], c["dt"]),
                                   rtol=1e-12, atol=1e-12)
        xf = s[b][1:, :c["d"]].astype(np.float32).astype(np.float64)
        ref_vals.append(oracle.sinkhorn(xf, y, w, eps=c["eps"], iters=c["iters"]).value)
    ref_vals = np.array(ref_vals)
    np.testing.assert_allclose(values, ref_vals, rtol=1e-5)
    assert best == int(np.argmin(ref_vals))


def test_plan_ensemble_equals_independent_plans(ct):
    """The lockstep ensemble follows the same trajectories as S independent
    planner runs (batched vs per-problem sweeps differ only in rounding)."""
    S, T, outer = 4, 300, 5
    c, s0, U0, y, w, Q, R = _ensemble_inputs(S, T)
    dev = torch.device("cuda")
    yt, wt = torch.as_tensor(y, device=dev), torch.as_tensor(w, device=dev)
    U, s, values, best = ct.plan_ensemble(c["dynamics"], s0, U0, c["dt"], Q, R, outer, c["step"],
                                          y=yt, w=wt, eps=c["eps"], iters=c["iters"])
    for b in range(S):
        ub, _sb, _h = ct.plan(c["dynamics"], s0, U0[b], c["dt"], Q, R, "sinkhorn", outer,
                              c["step"], y=yt, w=wt, eps=c["eps"], iters=c["iters"])
        assert rel(U[b] - U0[b], ub - U0[b]) < 1e-4, b
    assert np.all(np.isfinite(values)) and 0 <= best < S
    assert values[best] == values.min()


def test_plan_ensemble_is_deterministic(ct):
    """The seeds' host work runs on several threads; two identical calls return
    bit-identical controls, divergences and best seed."""
    S, T, outer = 6, 250, 3
    c, s0, U0, y, w, Q, R = _ensemble_inputs(S, T)
    dev = torch.device("cuda")
    yt, wt = torch.as_tensor(y, device=dev), torch.as_tensor(w, device=dev)
    runs = [ct.plan_ensemble(c["dynamics"], s0, U0, c["dt"], Q, R, outer, c["step"], y=yt, w=wt,
                             eps=c["eps"], iters=c["iters"]) for _ in range(2)]
    (U1, s1, v1, b1), (U2, s2, v2, b2) = runs
    np.testing.assert_array_equal(U1, U2)
    np.testing.assert_array_equal(s1, s2)
    np.testing.assert_array_equal(v1, v2)
    assert b1 == b2
