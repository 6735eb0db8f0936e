"""Linear-quadratic flow matching (Sec. II-C, eqs. 8-10) in float64 (oracle).

Test infrastructure only.

Problem (eq. 9 discretised with forward Euler at the trajectory step dt):
  z_0 = 0,  z_{t+1} = (I + dt A_t) z_t + dt B_t v_t,             t = 0..T-1
  minimise  sum_{t=0}^{T-1} dt |a_t - z_{t+1}|^2_Q  +  dt |v_t|^2_R
where A_t, B_t are the Jacobians of the dynamics along the current trajectory
(eq. 8) and a_t is the reference flow at the state sample reached after step t.

Two independent solvers of the same problem:
* lqr_track_dense   - the plain definition: stack z = G v and solve the normal
                      equations of the least-squares problem (small T only);
* lqr_track_riccati - backward Riccati recursion with the affine tracking term,
                      then a forward rollout (the closed form the paper refers
                      to, in discrete time).
"""
from __future__ import annotations

import numpy as np


def _discrete(A, B, dt):
    T, n, _ = A.shape
    Ad = np.eye(n)[None] + dt * np.asarray(A, dtype=np.float64)
    Bd = dt * np.asarray(B, dtype=np.float64)
    return Ad, Bd


def lqr_track_dense(A, B, a, Q, R, dt):
    """Returns (v [T,m], z [T+1,n]) by dense least squares."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    a = np.asarray(a, np.float64)
    T, n, m = B.shape
    Ad, Bd = _discrete(A, B, dt)
    G = np.zeros((T * n, T * m))          # row block t: z_{t+1};  column block s: v_s
    for s in range(T):
        blk = Bd[s]                       # effect of v_s on z_{s+1}
        for t in range(s, T):
            G[t * n:(t + 1) * n, s * m:(s + 1) * m] = blk
            if t + 1 < T:
                blk = Ad[t + 1] @ blk
    Qb = np.kron(np.eye(T), dt * np.asarray(Q, np.float64))
    Rb = np.kron(np.eye(T), dt * np.asarray(R, np.float64))
    H = G.T @ Qb @ G + Rb
    rhs = G.T @ Qb @ a.reshape(-1)
    v = np.linalg.solve(H, rhs).reshape(T, m)
    z = np.zeros((T + 1, n))
    z[1:] = (G @ v.reshape(-1)).reshape(T, n)
    return v, z


def lqr_track_riccati(A, B, a, Q, R, dt, return_gains: bool = False):
    """Returns (v [T,m], z [T+1,n]) by the backward Riccati recursion.

    Value function V_t(z) = z'P_t z - 2 p_t'z + const, V_T = 0.  With
    S = dt Q + P_{t+1}, s = dt Q a_t + p_{t+1}, H = dt R + B'SB:
      v_t = -K_t z_t + k_t,  K_t = H^-1 B'SA,  k_t = H^-1 B's,
      P_t = A'SA - A'SB K_t,  p_t = A'(s - SB k_t).
    """
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    a = np.asarray(a, np.float64)
    T, n, m = B.shape
    Ad, Bd = _discrete(A, B, dt)
    Qd = dt * np.asarray(Q, np.float64)
    Rd = dt * np.asarray(R, np.float64)
    P = np.zeros((n, n))
    p = np.zeros(n)
    Ks = np.empty((T, m, n))
    ks = np.empty((T, m))
    Ps = np.empty((T + 1, n, n))
    Ps[T] = P
    for t in range(T - 1, -1, -1):
        S = Qd + P
        s = Qd @ a[t] + p
        At, Bt = Ad[t], Bd[t]
        H = Rd + Bt.T @ S @ Bt
        K = np.linalg.solve(H, Bt.T @ S @ At)
        k = np.linalg.solve(H, Bt.T @ s)
        P = At.T @ S @ At - At.T @ S @ Bt @ K
        P = 0.5 * (P + P.T)
        p = At.T @ (s - S @ Bt @ k)
        Ks[t], ks[t], Ps[t] = K, k, P
    z = np.zeros((T + 1, n))
    v = np.empty((T, m))
    for t in range(T):
        v[t] = -Ks[t] @ z[t] + ks[t]
        z[t + 1] = Ad[t] @ z[t] + Bd[t] @ v[t]
    if return_gains:
        return v, z, Ps, Ks
    return v, z
