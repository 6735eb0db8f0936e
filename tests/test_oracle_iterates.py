"""Pins of the oracle's fixed-K iterates and of its dynamics rollout.

Every GPU parity test compares iterates after a fixed number K of Sinkhorn
iterations, which depend on the update scheme, so the scheme itself is pinned
here against textbook matrix scaling (Sec. II-B names the Sinkhorn algorithm;
the scaling form is Cuturi's): the cross problem's Gauss-Seidel sweeps are
Sinkhorn-Knopp's alternating row and column scalings started from v = b, and
the averaged self sweeps p <- (p + T_a(p))/2 are the symmetric scaling
u <- sqrt(u * a / (K u)) started from u = a.  Both loops run on the dense
kernel matrix in the scaling domain (no log-sum-exp), so they share nothing
with the oracle's streaming C loops.  Planted mistakes (a Jacobi cross update,
other dampings) are shown to fail these pins.

The Euler rollout of Sec. II-A (eq. 3 discretised) is pinned by closed forms:
the double integrator under constant acceleration, and the unicycle at
constant speed and turn rate (a straight line when the turn rate is zero)."""
import inspect
import sys
import types

import numpy as np
import pytest

import oracle

# the package re-exports the function under the module's name, so take the module itself
orc_sk = sys.modules["oracle.sinkhorn"]


def _problem(seed, T=6, M=9, d=2, eps=0.05):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, (T, d))
    y = rng.uniform(0.0, 1.0, (M, d))
    w = rng.uniform(0.5, 2.0, M)
    return x, y, w, eps


def _textbook(x, y, w, eps, K):
    """K Sinkhorn-Knopp iterations in the scaling domain, plus the self problems'
    symmetric scalings; returns the log-domain potentials they stand for."""
    T, M = len(x), len(y)
    a = np.full(T, 1.0 / T)
    b = w / w.sum()
    Kxy = np.exp(-((x[:, None] - y[None]) ** 2).sum(-1) / eps)
    Kxx = np.exp(-((x[:, None] - x[None]) ** 2).sum(-1) / eps)
    Kyy = np.exp(-((y[:, None] - y[None]) ** 2).sum(-1) / eps)
    v = b.copy()                       # g = 0
    u = a.copy()
    for _ in range(K):
        u = a / (Kxy @ v)              # row scaling from the current column scaling
        v = b / (Kxy.T @ u)            # column scaling from the new row scaling
    us, vs = a.copy(), b.copy()        # p = 0, q = 0
    for _ in range(K):
        us = np.sqrt(us * a / (Kxx @ us))
        vs = np.sqrt(vs * b / (Kyy @ vs))
    f, g = eps * np.log(u / a), eps * np.log(v / b)
    p, q = eps * np.log(us / a), eps * np.log(vs / b)
    # one extrapolation pass: the row-exact scalings of the final columns
    u_plus = a / (Kxy @ v)
    p_plus = -eps * np.log(Kxx @ us)
    q_plus = -eps * np.log(Kyy @ vs)
    v_plus = b / (Kxy.T @ u_plus)
    P = u_plus[:, None] * Kxy * v[None, :]          # cross plan (f+, g), rows sum to a
    Ps = (a * np.exp(p_plus / eps))[:, None] * Kxx * us[None, :]  # self plan (p+, p)
    Dy = (P / a[:, None]) @ y - x
    Ds = (Ps / a[:, None]) @ x - x
    return dict(f=f, g=g, p=p, q=q, f_plus=eps * np.log(u_plus / a),
                g_plus=eps * np.log(v_plus / b), p_plus=p_plus, q_plus=q_plus,
                grad_x=2.0 * a[:, None] * (Ds - Dy), P=P, Ps=Ps)


def _compare(r, ref, tol=1e-12):
    """Largest difference over the iterates, scaled by the potentials' size."""
    worst = 0.0
    for k in ("f", "g", "p", "q", "f_plus", "g_plus", "p_plus", "q_plus", "grad_x"):
        got, want = np.asarray(getattr(r, k)), ref[k]
        scale = max(1.0, np.abs(want).max())
        worst = max(worst, np.abs(got - want).max() / scale)
    return worst


@pytest.mark.parametrize("K", [1, 2, 5])
@pytest.mark.parametrize("seed", [40, 41])
def test_fixed_K_iterates_equal_textbook_scaling(K, seed):
    x, y, w, eps = _problem(seed)
    r = oracle.sinkhorn(x, y, w, eps=eps, iters=K)
    ref = _textbook(x, y, w, eps, K)
    assert r.resid > 1e-8                      # not converged: the scheme matters
    assert _compare(r, ref) < 1e-12, _compare(r, ref)
    # the rows of both plans sum to a exactly (the extrapolated potentials are row-exact)
    np.testing.assert_allclose(ref["P"].sum(1), 1.0 / len(x), rtol=1e-13)
    np.testing.assert_allclose(ref["Ps"].sum(1), 1.0 / len(x), rtol=1e-13)


def test_fixed_K_iterates_in_3d():
    x, y, w, eps = _problem(42, T=5, M=7, d=3, eps=0.08)
    for K in (1, 4):
        r = oracle.sinkhorn(x, y, w, eps=eps, iters=K)
        assert _compare(r, _textbook(x, y, w, eps, K)) < 1e-12


def _planted(old: str, new: str):
    """A copy of the oracle's Sinkhorn routine with one source line changed."""
    src = inspect.getsource(orc_sk)
    assert src.count(old) == 1, old
    src = src.replace(old, new).replace("from ._clib import", "from oracle._clib import")
    mod = types.ModuleType("planted_sinkhorn")
    sys.modules["planted_sinkhorn"] = mod        # dataclasses look their module up
    try:
        exec(compile(src, "planted_sinkhorn", "exec"), mod.__dict__)
    finally:
        del sys.modules["planted_sinkhorn"]
    return mod.sinkhorn


@pytest.mark.parametrize("old,new", [
    # Jacobi cross update: g from the previous f
    ("        f, _u = lse_update(x, y, logb, g, eps)          # f <- T_b(g)\n"
     "        g, _u = lse_update(y, x, loga, f, eps)          # g <- T_a(f)   (new f)\n",
     "        f_new, _u = lse_update(x, y, logb, g, eps)\n"
     "        g, _u = lse_update(y, x, loga, f, eps)\n"
     "        f = f_new\n"),
    # g updated before f
    ("        f, _u = lse_update(x, y, logb, g, eps)          # f <- T_b(g)\n"
     "        g, _u = lse_update(y, x, loga, f, eps)          # g <- T_a(f)   (new f)\n",
     "        g, _u = lse_update(y, x, loga, f, eps)\n"
     "        f, _u = lse_update(x, y, logb, g, eps)\n"),
    # self update damped by 0.6 instead of 1/2
    ("            p = 0.5 * (p + tp)", "            p = 0.4 * p + 0.6 * tp"),
    # reference self update undamped
    ("            q = 0.5 * (q + tq)", "            q = tq"),
])
def test_planted_scheme_mistakes_fail_the_textbook_pin(old, new):
    bad = _planted(old, new)
    x, y, w, eps = _problem(40)
    for K in (1, 2, 5):
        ref = _textbook(x, y, w, eps, K)
        good = oracle.sinkhorn(x, y, w, eps=eps, iters=K)
        assert _compare(good, ref) < 1e-12
    # the mistake shows at some K of the pinned set
    assert max(_compare(bad(x, y, w, eps=eps, iters=K), _textbook(x, y, w, eps, K))
               for K in (1, 2, 5)) > 1e-6


def test_planner_flow_is_twice_the_translation():
    """The planner's Sinkhorn flow is -dS/dx_i divided by the sample's mass a_i:
    when the reference is the trajectory translated by c (equal weights) it is
    2c at every sample, the per-unit-mass descent direction of S = |c|^2.  Pins
    the factor T between the library's gradient and the flow."""
    rng = np.random.default_rng(44)
    x = rng.uniform(0.2, 0.8, (8, 2))
    c = np.array([0.07, -0.04])
    flow, S = oracle.reference_flow("sinkhorn", x, y=x + c, eps=0.1, iters=6000)
    assert abs(S - c @ c) < 1e-9
    np.testing.assert_allclose(flow, np.tile(2.0 * c, (8, 1)), atol=1e-8)


@pytest.mark.parametrize("d", [2, 3])
def test_double_integrator_rollout_constant_acceleration(d):
    """Euler steps p <- p + dt v, v <- v + dt u under constant u give
    v_t = v_0 + t dt u and p_t = p_0 + t dt v_0 + dt^2 u t(t-1)/2."""
    rng = np.random.default_rng(45 + d)
    p0, v0, u = rng.normal(size=d), rng.normal(size=d), rng.normal(size=d)
    T, dt = 37, 0.05
    s = oracle.rollout("double_integrator", np.concatenate([p0, v0]), np.tile(u, (T, 1)), dt)
    t = np.arange(T + 1)[:, None]
    np.testing.assert_allclose(s[:, d:], v0 + t * dt * u, atol=1e-12)
    np.testing.assert_allclose(s[:, :d], p0 + t * dt * v0 + dt * dt * u * t * (t - 1) / 2,
                               atol=1e-12)


def test_unicycle_rollout_straight_line_and_constant_turn():
    """Zero turn rate: a straight line at speed v along the initial heading.
    Constant turn rate w: heading th_t = th_0 + t dt w and, by the sum of cosines
    (sines) of an arithmetic sequence,
    x_t = x_0 + dt v sin(t dt w / 2) / sin(dt w / 2) cos(th_0 + (t-1) dt w / 2)."""
    T, dt, v = 50, 0.01, 0.3
    s0 = np.array([0.5, 0.4, 0.7])
    s = oracle.rollout("unicycle", s0, np.tile([v, 0.0], (T, 1)), dt)
    t = np.arange(T + 1)
    np.testing.assert_allclose(s[:, 0], 0.5 + t * dt * v * np.cos(0.7), atol=1e-13)
    np.testing.assert_allclose(s[:, 1], 0.4 + t * dt * v * np.sin(0.7), atol=1e-13)
    np.testing.assert_allclose(s[:, 2], 0.7, atol=0)
    om = 2.5
    s = oracle.rollout("unicycle", s0, np.tile([v, om], (T, 1)), dt)
    b = dt * om
    ratio = np.where(t == 0, 0.0, np.sin(t * b / 2) / np.sin(b / 2))
    mid = 0.7 + (t - 1) * b / 2
    np.testing.assert_allclose(s[:, 2], 0.7 + t * b, atol=1e-13)
    np.testing.assert_allclose(s[:, 0], 0.5 + dt * v * ratio * np.cos(mid), atol=1e-13)
    np.testing.assert_allclose(s[:, 1], 0.4 + dt * v * ratio * np.sin(mid), atol=1e-13)
