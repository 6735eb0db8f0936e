"""The outer planning loop (Sec. II-A eqs. 1-3 and Sec. II-C), float64 oracle.

Test infrastructure only.

One outer iteration from controls u:
  1. roll the dynamics forward with Euler steps: s_{t+1} = s_t + dt f(s_t, u_t);
  2. the trajectory samples are the positions of s_1..s_T (equal weights);
  3. reference flow at every sample (Sec. II-B, "reference flow on state
     trajectory"): for the Sinkhorn flow the per-unit-mass descent direction
     -T dS/dx_i; for the Stein flow phi_i of eq. 4;
  4. Jacobians A_t, B_t along (s_t, u_t) (eq. 8);
  5. linear-quadratic flow matching (eq. 9) with the flow as the target of the
     position block of z_{t+1};
  6. u <- u + step * v*.

Dynamics: a planar double integrator (state p, v; control acceleration) and a
unicycle / differential drive (state p_x, p_y, heading; control speed, turn
rate).
"""
from __future__ import annotations

import numpy as np

from .lqr import lqr_track_riccati
from .sinkhorn import sinkhorn
from .svgd import gmm_score, median_bandwidth, svgd_phi
from .grid import score as grid_score


def dynamics_f(kind: str, s: np.ndarray, u: np.ndarray) -> np.ndarray:
    if kind == "double_integrator":
        d = s.shape[-1] // 2
        return np.concatenate([s[..., d:], u], axis=-1)
    if kind == "unicycle":
        th = s[..., 2]
        return np.stack([u[..., 0] * np.cos(th), u[..., 0] * np.sin(th), u[..., 1]], axis=-1)
    raise ValueError(kind)


def dynamics_jac(kind: str, s: np.ndarray, u: np.ndarray):
    """(df/ds [T,n,n], df/du [T,n,m]) along the trajectory."""
    T = s.shape[0]
    if kind == "double_integrator":
        n = s.shape[1]
        d = n // 2
        A = np.zeros((T, n, n))
        B = np.zeros((T, n, d))
        for k in range(d):
            A[:, k, d + k] = 1.0
            B[:, d + k, k] = 1.0
        return A, B
    if kind == "unicycle":
        th = s[:, 2]
        v = u[:, 0]
        A = np.zeros((T, 3, 3))
        B = np.zeros((T, 3, 2))
        A[:, 0, 2] = -v * np.sin(th)
        A[:, 1, 2] = v * np.cos(th)
        B[:, 0, 0] = np.cos(th)
        B[:, 1, 0] = np.sin(th)
        B[:, 2, 1] = 1.0
        return A, B
    raise ValueError(kind)


def rollout(kind: str, s0, u, dt: float) -> np.ndarray:
    u = np.asarray(u, np.float64)
    T = u.shape[0]
    s = np.empty((T + 1, len(s0)))
    s[0] = s0
    for t in range(T):
        s[t + 1] = s[t] + dt * dynamics_f(kind, s[t], u[t])
    return s


def reference_flow(flow: str, x, y=None, w=None, gmm=None, eps=0.01, iters=100, h=None,
                   grid=None):
    """(flow [T,d], scalar): the per-sample reference flow and the objective
    reported for it (S for Sinkhorn, mean |phi| for Stein; "svgd_grid" is the
    Stein flow toward a utility grid, oracle.grid.Grid)."""
    T = x.shape[0]
    if flow == "sinkhorn":
        r = sinkhorn(x, y, w, eps=eps, iters=iters, want_value=True, want_grad_w=False)
        return -T * r.grad_x, r.value
    if flow == "svgd":
        sc = gmm_score(x, gmm.weights, gmm.means, gmm.sigmas, gmm.floor)
        hh = median_bandwidth(x) if (h is None or h <= 0) else h
        phi = svgd_phi(x, sc, hh)
        return phi, float(np.mean(np.linalg.norm(phi, axis=1)))
    if flow == "svgd_grid":
        sc = grid_score(grid, x)
        hh = median_bandwidth(x) if (h is None or h <= 0) else h
        phi = svgd_phi(x, sc, hh)
        return phi, float(np.mean(np.linalg.norm(phi, axis=1)))
    raise ValueError(flow)


def plan_step(kind, s0, u, dt, Q, R, flow, step=1.0, x_cast=np.float32, **flow_kw):
    """One outer iteration; returns (u_new, s, objective, flow, v).

    x_cast: the trajectory samples are rounded to this type before the flow is
    evaluated (the GPU path evaluates the flow on float32 samples)."""
    s = rollout(kind, s0, u, dt)
    d = Q.shape[0]
    x = s[1:, :d].astype(x_cast).astype(np.float64)
    a, obj = reference_flow(flow, x, **flow_kw)
    A, B = dynamics_jac(kind, s[:-1], u)
    n = s.shape[1]
    Qn = np.zeros((n, n))
    Qn[:d, :d] = Q
    target = np.zeros((len(u), n))
    target[:, :d] = a
    v, _z = lqr_track_riccati(A, B, target, Qn, R, dt)
    return u + step * v, s, obj, a, v


def plan(kind, s0, u, dt, Q, R, flow, outer, step=1.0, **flow_kw):
    hist = []
    for _ in range(outer):
        u, s, obj, _a, _v = plan_step(kind, s0, u, dt, Q, R, flow, step, **flow_kw)
        hist.append(obj)
    return u, rollout(kind, s0, u, dt), np.array(hist)
