"""Continuous-utility references on a regular grid, in float64 (oracle).

Test infrastructure only.

The reference q may be given as a continuous utility function over the search
space rather than as samples (Sec. II-A).  The Stein flow needs only the score
grad log q, so the utility need not be normalised (Sec. II-B, properties of the
reference flows); the Sinkhorn flow needs samples, which a gridded utility gives
as weighted grid nodes (the flow's weights b_j, eq. 5).

Readings where the paper is silent (the utility's representation is not fixed):
* utility values u_j >= 0 sit on the nodes of a regular grid over the box
  [lo, hi]: n_t >= 2 nodes on axis t, node index j_t at lo_t + j_t (hi_t - lo_t) / (n_t - 1);
  axis 0 varies fastest in memory (j = j_0 + n_0 (j_1 + n_1 j_2));
* the density is proportional to U(x) + rho, with U the multilinear interpolant of
  the node values evaluated at x clamped into the box (so it is constant along an
  axis outside the box) and rho >= 0 an additive floor;
* cell of a point: c_t = min(floor(s_t), n_t - 2) with s_t = (x_t - lo_t)(n_t - 1) / (hi_t - lo_t)
  clamped into [0, n_t - 1]; a point on a face shared by two cells takes the upper
  cell (the last cell on the box's upper face);
* score = grad U / (U + rho), the gradient of the cell's multilinear piece; the
  component along an axis on which x lies outside the box is zero; where
  U + rho = 0 the score is zero;
* weighted grid samples: every node, with weight (u_j + rho) times its
  trapezoid-rule volume (halved once for each axis on which the node lies on the
  box face), normalised to sum 1; nodes of zero weight are dropped; order is node
  order.  The trapezoid rule integrates every cell's multilinear piece exactly, so
  the weights carry the exact mass of the interpolated density.
"""
from __future__ import annotations

from dataclasses import dataclass
import itertools

import numpy as np


@dataclass
class Grid:
    """u: node values, shape (n_1, n_0) for d = 2 or (n_2, n_1, n_0) for d = 3
    (C order, so axis 0 is the fastest); lo, hi: box corners [d]; floor: rho."""
    u: np.ndarray
    lo: np.ndarray
    hi: np.ndarray
    floor: float = 0.0

    @property
    def d(self) -> int:
        return self.u.ndim

    @property
    def n(self):
        """Nodes per axis, axis 0 first."""
        return tuple(reversed(self.u.shape))


def _cell(g: Grid, x: np.ndarray):
    """Cell index c [n,d], fraction f [n,d], inside-box mask [n,d] and the scale
    ds/dx [d] of every coordinate."""
    x = np.asarray(x, np.float64)
    lo = np.asarray(g.lo, np.float64)
    hi = np.asarray(g.hi, np.float64)
    n = np.array(g.n, np.float64)
    s = (x - lo) * (n - 1) / (hi - lo)
    inside = (x >= lo) & (x <= hi)
    s = np.clip(s, 0.0, n - 1)
    c = np.minimum(np.floor(s), n - 2).astype(np.int64)
    return c, s - c, inside, (n - 1) / (hi - lo)


def _node_value(g: Grid, idx: np.ndarray) -> np.ndarray:
    """u at integer node indices idx [n,d] (axis 0 first)."""
    return np.asarray(g.u, np.float64)[tuple(idx[:, t] for t in reversed(range(g.d)))]


def interp(g: Grid, x) -> np.ndarray:
    """U(x) + rho, [n]."""
    c, f, _, _ = _cell(g, x)
    val = np.zeros(c.shape[0])
    for bits in itertools.product((0, 1), repeat=g.d):
        wgt = np.ones(c.shape[0])
        for t, b in enumerate(bits):
            wgt *= f[:, t] if b else 1.0 - f[:, t]
        val += wgt * _node_value(g, c + np.array(bits))
    return val + g.floor


def score(g: Grid, x) -> np.ndarray:
    """grad log(U + rho) at every point, [n,d]."""
    c, f, inside, scale = _cell(g, x)
    npt, d = c.shape
    grad = np.zeros((npt, d))
    for bits in itertools.product((0, 1), repeat=d):
        u = _node_value(g, c + np.array(bits))
        for t in range(d):
            wgt = np.ones(npt) * (1.0 if bits[t] else -1.0)
            for s_ in range(d):
                if s_ != t:
                    wgt *= f[:, s_] if bits[s_] else 1.0 - f[:, s_]
            grad[:, t] += wgt * u
    grad *= scale[None, :] * inside
    den = interp(g, x)
    out = np.zeros_like(grad)
    pos = den > 0
    out[pos] = grad[pos] / den[pos, None]
    return out


def node_positions(g: Grid) -> np.ndarray:
    """Coordinates of every node in node order, [N,d]."""
    axes = [g.lo[t] + np.arange(g.n[t]) * ((g.hi[t] - g.lo[t]) / (g.n[t] - 1))
            for t in range(g.d)]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")      # slowest axis first
    return np.stack([m.ravel() for m in reversed(mesh)], axis=1)


def trapezoid_volume(g: Grid) -> np.ndarray:
    """Trapezoid-rule weight of every node in node order (cell volume times 1/2
    per axis on which the node lies on the box face), [N]."""
    per_axis = []
    for t in range(g.d):
        h = (g.hi[t] - g.lo[t]) / (g.n[t] - 1)
        v = np.full(g.n[t], h)
        v[0] *= 0.5
        v[-1] *= 0.5
        per_axis.append(v)
    vol = per_axis[g.d - 1]
    for t in reversed(range(g.d - 1)):
        vol = np.multiply.outer(vol, per_axis[t])             # slowest axis first
    return vol.ravel()


def samples(g: Grid):
    """(y [M,d], w [M]): the weighted grid samples defined above."""
    m = (np.asarray(g.u, np.float64).ravel() + g.floor) * trapezoid_volume(g)
    keep = m > 0
    return node_positions(g)[keep], m[keep] / np.sum(m[keep])
