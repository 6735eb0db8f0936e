"""Debiased Sinkhorn divergence and its gradients, in float64 (oracle).

Test infrastructure only.

Definitions (Sec. II-B):
* eq. 1 discretised at equal time steps: the trajectory is the point cloud
  x_1..x_T with equal mass a_i = 1/T;
* the reference is the point cloud y_1..y_M with masses b_j = w_j / sum(w);
* eq. 5 with the squared-norm cost C_ij = |x_i - y_j|^2 and the entropy taken
  relative to the product of the marginals, solved by the Sinkhorn algorithm
  in its log-domain (dual potential) form;
* eq. 6: S = OT(a,b) - OT(a,a)/2 - OT(b,b)/2;
* eq. 7: the flow is the gradient of S with respect to each x_i.

Readings where the paper is silent (each is a design decision listed with the
others in the design notes):
* marginals are probability vectors (a = 1/T, b = w/sum w);
* cross problem: Gauss-Seidel sweeps f <- T_b(g), then g <- T_a(f), from
  f = g = 0; self problems: averaged sweeps p <- (p + T_a(p))/2 from p = 0;
  the same fixed iteration count for all three;
* outputs are read off one final extrapolation pass, so that every transport
  plan used is exactly row-normalised:  f+ = T_b(g), p+ = T_a(p),
  g+ = T_a(f+), q+ = T_b(q);
* gradient (envelope theorem):  dS/dx_i = 2 a_i (D^s_i - D^y_i), where D^y_i is
  the plan-weighted mean of (y_j - x_i) under the cross plan and D^s_i that of
  (x_k - x_i) under the self plan;
* value: each OT term is its dual objective at its row-exact pair
  (f+, g), (p+, p), (q+, q);
* weight gradient through b = w / sum w:  G_j = g+_j - q+_j,
  dS/dw_j = (G_j - <b, G>) / sum w;
* without debiasing only the cross term is kept (S = OT(a,b)).

Here T_b(g)_i = -eps * log sum_j b_j exp((g_j - C_ij)/eps) and T_a likewise.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from ._clib import dptr, f64, lib


def lse_update(xq: np.ndarray, xk: np.ndarray, logw_k: np.ndarray, pot_k: np.ndarray,
               eps: float, want_bary: bool = False):
    """Soft-min update  out_i = -eps * log sum_j exp(logw_j + (pot_j - |xq_i - xk_j|^2)/eps).

    Returns (out [Nq], bary [Nq,d] or None) where bary_i is the mean of
    (xk_j - xq_i) under the normalised weights of that sum."""
    xq = f64(xq)
    xk = f64(xk)
    d = xq.shape[1]
    h = f64(logw_k + f64(pot_k) / eps)
    lse = np.empty(xq.shape[0])
    bary = np.empty((xq.shape[0], d)) if want_bary else None
    lib().orc_lse(d, xq.shape[0], dptr(xq), xk.shape[0], dptr(xk), dptr(h), float(eps),
                  dptr(lse), dptr(bary) if want_bary else None)
    return -eps * lse, bary


@dataclass
class SinkhornResult:
    grad_x: np.ndarray            # [T,d]   dS/dx
    grad_w: Optional[np.ndarray]  # [M]     dS/dw
    value: Optional[float]        # S
    f: np.ndarray                 # last iterates (cross, self, reference-self)
    g: np.ndarray
    p: Optional[np.ndarray]
    q: Optional[np.ndarray]
    f_plus: np.ndarray            # extrapolated potentials of the final pass
    g_plus: Optional[np.ndarray]
    p_plus: Optional[np.ndarray]
    q_plus: Optional[np.ndarray]
    bary_y: np.ndarray            # D^y  [T,d]
    bary_s: Optional[np.ndarray]  # D^s  [T,d]
    ot_ab: Optional[float]
    ot_aa: Optional[float]
    ot_bb: Optional[float]
    resid: Optional[float]        # column-marginal L1 error of the plan (f+, g)


def sinkhorn(x, y, w=None, eps: float = 0.01, iters: int = 100, debias: bool = True,
             want_value: bool = True, want_grad_w: bool = True,
             init=None) -> SinkhornResult:
    """Debiased Sinkhorn divergence between the trajectory samples x [T,d] and the
    weighted reference samples (y [M,d], w [M]); see the module docstring.

    init: optional (f, g, p, q) starting potentials (warm start); zeros otherwise.
    """
    x = f64(x)
    y = f64(y)
    T, d = x.shape
    M = y.shape[0]
    w = np.ones(M) if w is None else f64(w)
    wsum = w.sum()
    b = w / wsum
    loga = np.full(T, -np.log(T))
    logb = np.log(b)
    a = np.full(T, 1.0 / T)
    need_ref = debias and (want_value or want_grad_w)

    if init is None:
        f, g, p, q = np.zeros(T), np.zeros(M), np.zeros(T), np.zeros(M)
    else:
        f, g, p, q = (f64(v).copy() for v in init)

    for _ in range(iters):
        f, _u = lse_update(x, y, logb, g, eps)          # f <- T_b(g)
        g, _u = lse_update(y, x, loga, f, eps)          # g <- T_a(f)   (new f)
        if debias:
            tp, _u = lse_update(x, x, loga, p, eps)     # p <- (p + T_a(p)) / 2
            p = 0.5 * (p + tp)
        if need_ref:
            tq, _u = lse_update(y, y, logb, q, eps)     # q <- (q + T_b(q)) / 2
            q = 0.5 * (q + tq)

    f_plus, bary_y = lse_update(x, y, logb, g, eps, want_bary=True)
    p_plus = bary_s = None
    if debias:
        p_plus, bary_s = lse_update(x, x, loga, p, eps, want_bary=True)
        grad_x = 2.0 * a[:, None] * (bary_s - bary_y)
    else:
        grad_x = -2.0 * a[:, None] * bary_y

    g_plus = q_plus = None
    value = grad_w = ot_ab = ot_aa = ot_bb = resid = None
    if want_value or want_grad_w:
        g_plus, _u = lse_update(y, x, loga, f_plus, eps)
        if need_ref:
            q_plus, _u = lse_update(y, y, logb, q, eps)
        resid = float(np.sum(b * np.abs(np.exp((g - g_plus) / eps) - 1.0)))
        ot_ab = float(a @ f_plus + b @ g)
        if debias:
            ot_aa = float(a @ p_plus + a @ p)
            ot_bb = float(b @ q_plus + b @ q)
            value = ot_ab - 0.5 * ot_aa - 0.5 * ot_bb
            G = g_plus - q_plus
        else:
            value = ot_ab
            G = g_plus
        grad_w = (G - b @ G) / wsum
        if not want_value:
            value = None
        if not want_grad_w:
            grad_w = None

    return SinkhornResult(grad_x, grad_w, value, f, g, p if debias else None,
                          q if need_ref else None, f_plus, g_plus, p_plus, q_plus,
                          bary_y, bary_s, ot_ab, ot_aa, ot_bb, resid)


def gauge_fix(f: np.ndarray, g: np.ndarray, a: Optional[np.ndarray] = None,
              b: Optional[np.ndarray] = None):
    """Cross potentials are defined up to (f + c, g - c); return the pair with
    <a,f> = <b,g> so that two solutions can be compared entrywise."""
    a = np.full(len(f), 1.0 / len(f)) if a is None else a
    b = np.full(len(g), 1.0 / len(g)) if b is None else b
    c = 0.5 * (b @ g - a @ f)
    return f + c, g - c
