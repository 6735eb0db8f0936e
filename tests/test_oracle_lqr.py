"""Pins of the FP64 linear-quadratic flow-matching oracle (Sec. II-C, eqs. 8-10):
the Riccati recursion against the dense least-squares definition and against
scipy's discrete algebraic Riccati solution, plus the planner's dynamics
Jacobians against central differences."""
import numpy as np
import pytest
from scipy.linalg import solve_discrete_are

import oracle


def _random_problem(rng, T, n, m):
    A = rng.normal(size=(T, n, n)) * 0.5
    B = rng.normal(size=(T, n, m))
    a = rng.normal(size=(T, n))
    Q = np.diag(rng.uniform(0.5, 2.0, n))
    Q[n - 1, n - 1] = 0.0                      # an unweighted component, as for velocities
    R = np.diag(rng.uniform(0.01, 0.1, m))
    return A, B, a, Q, R


@pytest.mark.parametrize("T,n,m", [(1, 2, 1), (7, 3, 2), (40, 4, 2)])
def test_riccati_equals_dense_least_squares(T, n, m):
    rng = np.random.default_rng(30 + T)
    A, B, a, Q, R = _random_problem(rng, T, n, m)
    dt = 0.05
    v1, z1 = oracle.lqr_track_dense(A, B, a, Q, R, dt)
    v2, z2 = oracle.lqr_track_riccati(A, B, a, Q, R, dt)
    np.testing.assert_allclose(v2, v1, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(z2, z1, rtol=1e-9, atol=1e-10)
    # the dense solution is the least-squares optimum: the gradient of the cost vanishes
    # along random perturbations (first order) and the cost increases (second order)
    def cost(v):
        z = np.zeros((T + 1, n))
        for t in range(T):
            z[t + 1] = z[t] + dt * A[t] @ z[t] + dt * B[t] @ v[t]
        e = a - z[1:]
        return dt * np.einsum("ti,ij,tj->", e, Q, e) + dt * np.einsum("ti,ij,tj->", v, R, v)
    c0 = cost(v1)
    for _ in range(3):
        dv = rng.normal(size=v1.shape) * 1e-3
        assert cost(v1 + dv) >= c0 - 1e-15


def test_zero_target_gives_zero_control():
    rng = np.random.default_rng(31)
    A, B, _a, Q, R = _random_problem(rng, 30, 3, 2)
    v, z = oracle.lqr_track_riccati(A, B, np.zeros((30, 3)), Q, R, 0.1)
    assert np.abs(v).max() == 0.0 and np.abs(z).max() == 0.0


def test_long_horizon_lti_riccati_reaches_dare():
    rng = np.random.default_rng(32)
    n, m, T, dt = 3, 2, 3000, 0.05
    A0 = rng.normal(size=(n, n)) * 0.3
    B0 = rng.normal(size=(n, m))
    Q = np.diag([1.0, 2.0, 0.5])
    R = np.diag([0.05, 0.1])
    A = np.repeat(A0[None], T, 0)
    B = np.repeat(B0[None], T, 0)
    _v, _z, Ps, _K = oracle.lqr_track_riccati(A, B, np.zeros((T, n)), Q, R, dt, return_gains=True)
    X = solve_discrete_are(np.eye(n) + dt * A0, dt * B0, dt * Q, dt * R)
    # the recursion's S_t = dt Q + P_{t+1} is the DARE iterate
    np.testing.assert_allclose(dt * Q + Ps[1], X, rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("kind,n,m", [("double_integrator", 4, 2), ("unicycle", 3, 2)])
def test_dynamics_jacobians_match_central_differences(kind, n, m):
    rng = np.random.default_rng(33)
    s = rng.normal(size=(5, n))
    u = rng.normal(size=(5, m))
    A, B = oracle.dynamics_jac(kind, s, u)
    h = 1e-6
    for k in range(n):
        e = np.zeros(n)
        e[k] = h
        fd = (oracle.dynamics_f(kind, s + e, u) - oracle.dynamics_f(kind, s - e, u)) / (2 * h)
        np.testing.assert_allclose(A[:, :, k], fd, atol=1e-8)
    for k in range(m):
        e = np.zeros(m)
        e[k] = h
        fd = (oracle.dynamics_f(kind, s, u + e) - oracle.dynamics_f(kind, s, u - e)) / (2 * h)
        np.testing.assert_allclose(B[:, :, k], fd, atol=1e-8)


def test_one_plan_step_reduces_sinkhorn_divergence():
    """A single outer step along the LQR-projected flow lowers S (first-order
    descent for a small step)."""
    import workloads as W
    cfg = W.CONFIGS["planner_2d"]
    rng = np.random.default_rng(cfg.seed)
    x, y, w, g = W.config_inputs(cfg, T=64, M=128)
    T = 64
    u0 = rng.normal(size=(T, 2)) * 0.1
    s0 = np.array([0.5, 0.5, 0.0, 0.0])
    Q = np.eye(2)
    R = 0.01 * np.eye(2)
    u1, s, obj0, a, v = oracle.plan_step("double_integrator", s0, u0, 0.05, Q, R, "sinkhorn",
                                         step=0.2, y=y, w=w, eps=0.01, iters=100)
    _u2, _s, obj1, _a, _v = oracle.plan_step("double_integrator", s0, u1, 0.05, Q, R, "sinkhorn",
                                             step=0.2, y=y, w=w, eps=0.01, iters=100)
    assert obj1 < obj0
