"""Torch-facing wrappers of the C ABI (argument marshalling only).

Every function here checks dtypes/devices, allocates the outputs and the
workspace with torch, and calls the matching libct.so entry point on the
current torch stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch
from torch.autograd.function import once_differentiable

from . import _lib as L
from ._lib import check, lib


def version() -> str:
    return lib().ct_version().decode()


def _stream(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def _req(t: torch.Tensor, name: str, dev: Optional[torch.device] = None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32 (got {t.dtype})")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if dev is not None and t.device != dev:
        raise ValueError(f"{name} is on {t.device}, expected {dev}")
    return t.contiguous()


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _workspace(nbytes: int, dev: torch.device) -> torch.Tensor:
    if nbytes == 0:
        raise ValueError("invalid problem shape (workspace size 0)")
    return torch.empty(int(nbytes), dtype=torch.uint8, device=dev)


@dataclass
class SinkhornOut:
    grad_x: torch.Tensor
    grad_w: Optional[torch.Tensor]
    value: Optional[torch.Tensor]
    pot: Optional[torch.Tensor]        # [2T+2M] f, g, p, q (last iterates)
    pot_plus: Optional[torch.Tensor]   # [2T+2M] f+, g+, p+, q+
    aux: Optional[torch.Tensor]        # [8]


def _opts(d: int, eps: float, iters: int, flags: int) -> L.SinkhornOpts:
    return L.SinkhornOpts(int(d), int(iters), float(eps), int(flags))


def _fused_flag(fused) -> int:
    """None: the library's size rule; True: CT_FUSED; False: CT_UNFUSED; "tiny": CT_TINY;
    "mesh": CT_MESH."""
    if fused is None:
        return 0
    if isinstance(fused, str):
        if fused not in ("tiny", "mesh"):
            raise ValueError(f"fused must be None, True, False, 'tiny' or 'mesh' (got {fused!r})")
        return L.CT_TINY if fused == "tiny" else L.CT_MESH
    return L.CT_FUSED if fused else L.CT_UNFUSED


def sinkhorn_grad(x: torch.Tensor, y: torch.Tensor, w: Optional[torch.Tensor] = None, *,
                  eps: float, iters: int, debias: bool = True, value: bool = False,
                  grad_w: bool = False, init: Optional[torch.Tensor] = None,
                  ref_q: Optional[torch.Tensor] = None, safe: bool = False,
                  potentials: bool = False, aux: bool = False,
                  one_stream: bool = False, static_scratch: bool = False,
                  fused=None, expanded: bool = True) -> SinkhornOut:
    """Gradient of the (debiased) Sinkhorn divergence; see ct_sinkhorn_grad.

    x [T,d], y [M,d], w [M] or None: float32 GPU tensors.
    init: optional [2T+2M] starting potentials (f, g, p, q) -> CT_WARM_START.
    ref_q: optional [M] converged reference self potential -> CT_REF_CACHED.
    fused: True -> CT_FUSED (all iterations in one launch), "tiny" -> CT_TINY (all
    iterations in one workgroup), "mesh" -> CT_MESH (all iterations in one launch of
    workgroups that exchange potentials without grid barriers), False -> CT_UNFUSED,
    None -> the library's size rule.
    expanded: the lagged sweeps' exponent in the expanded form (default); False ->
    CT_DIFFERENCE (the difference form).
    static_scratch: call ct_sinkhorn_grad_static (the library's static device
    scratch instead of a workspace; only the outputs are allocated here).
    """
    dev = x.device
    x = _req(x, "x")
    y = _req(y, "y", dev)
    if w is not None:
        w = _req(w, "w", dev)
    T, d = x.shape
    M = y.shape[0]
    if y.shape[1] != d:
        raise ValueError("x and y must have the same dimension")
    flags = (L.CT_DEBIAS if debias else 0) | (L.CT_VALUE if value else 0) | \
        (L.CT_GRAD_W if grad_w else 0) | (L.CT_SAFE_LSE if safe else 0) | \
        (L.CT_ONE_STREAM if one_stream else 0) | _fused_flag(fused) | \
        (0 if expanded else L.CT_DIFFERENCE)
    pot = None
    if init is not None or ref_q is not None or potentials:
        pot = torch.zeros(2 * T + 2 * M, dtype=torch.float32, device=dev)
        if init is not None:
            pot.copy_(_req(init, "init", dev).reshape(-1))
            flags |= L.CT_WARM_START
        if ref_q is not None:
            pot[2 * T + M:].copy_(_req(ref_q, "ref_q", dev).reshape(-1))
            flags |= L.CT_REF_CACHED
    o = _opts(d, eps, iters, flags)
    gx = torch.empty_like(x)
    gw = torch.empty(M, dtype=torch.float32, device=dev) if grad_w else None
    val = torch.empty(1, dtype=torch.float32, device=dev) if value else None
    pp = torch.empty(2 * T + 2 * M, dtype=torch.float32, device=dev) if potentials else None
    ax = torch.empty(8, dtype=torch.float32, device=dev) if aux else None
    if static_scratch:
        st = lib().ct_sinkhorn_grad_static(_p(x), T, _p(y), _p(w), M, ctypes.byref(o), _p(gx),
                                           _p(gw), _p(val), _p(pot), _p(pp), _p(ax), _stream(dev))
        check("ct_sinkhorn_grad_static", st)
    else:
        nbytes = lib().ct_sinkhorn_workspace_size(T, M, ctypes.byref(o))
        ws = _workspace(nbytes, dev)
        st = lib().ct_sinkhorn_grad(_p(x), T, _p(y), _p(w), M, ctypes.byref(o), _p(gx), _p(gw),
                                    _p(val), _p(pot), _p(pp), _p(ax), _p(ws), nbytes, _stream(dev))
        check("ct_sinkhorn_grad", st)
    return SinkhornOut(gx, gw, val, pot if potentials else None, pp, ax)


def static_scratch_bytes() -> int:
    """Size of the device array that ct_sinkhorn_grad_static works in."""
    return int(lib().ct_sinkhorn_static_scratch_bytes())


class SinkhornDivergence(torch.autograd.Function):
    """S(x, (y, w)) as an autograd function (Sec. II-B, eq. 7, by automatic
    differentiation).  The forward pass computes S together with dS/dx and
    dS/dw (envelope theorem on the extrapolated potentials); the backward pass
    only scales them by the incoming gradient, so no second solve is needed."""

    @staticmethod
    def forward(ctx, x, y, w, eps: float, iters: int, debias: bool = True,
                one_stream: bool = False, ref_q: Optional[torch.Tensor] = None,
                expanded: bool = True):
        need_w = bool(w is not None and ctx.needs_input_grad[2])
        out = sinkhorn_grad(x.detach(), y.detach(), None if w is None else w.detach(), eps=eps,
                            iters=iters, debias=debias, value=True, grad_w=need_w,
                            one_stream=one_stream,
                            ref_q=None if ref_q is None else ref_q.detach(), expanded=expanded)
        ctx.save_for_backward(out.grad_x, out.grad_w if need_w else None)
        ctx.need_w = need_w
        return out.value.reshape(())

    @staticmethod
    @once_differentiable
    def backward(ctx, gS):
        gx, gw = ctx.saved_tensors
        return (gS * gx, None, (gS * gw if ctx.need_w else None), None, None, None, None, None,
                None)


def sinkhorn_divergence(x, y, w=None, *, eps: float, iters: int, debias: bool = True,
                        one_stream: bool = False, ref_q: Optional[torch.Tensor] = None,
                        expanded: bool = True):
    """S(x, (y, w)) with autograd (SinkhornDivergence).  ref_q: the reference self
    potential after the same `iters` averaged sweeps (reference_self_potential),
    which does not depend on x: passing it skips those sweeps (CT_REF_CACHED) and
    gives the result of recomputing it up to float32 rounding (the staged
    coordinates are centred on the mean of the points of the call that made q).
    expanded: as for sinkhorn_grad."""
    return SinkhornDivergence.apply(x, y, w, eps, iters, debias, one_stream, ref_q, expanded)


def reference_self_potential(y: torch.Tensor, w: Optional[torch.Tensor] = None, *, eps: float,
                             iters: int) -> torch.Tensor:
    """q after `iters` averaged sweeps q <- (q + T_b(q))/2 from zero: the reference
    self problem OT(b, b) of eq. 6, independent of the trajectory, for reuse across
    gradient calls with the same reference (ref_q).  Runs ct_sinkhorn_grad with a
    single trajectory sample, so the cross and trajectory-self work is negligible."""
    out = sinkhorn_grad(y[:1].contiguous(), y, w, eps=eps, iters=iters, value=True,
                        potentials=True)
    return out.pot[2 + y.shape[0]:].clone()   # pot = f[1], g[M], p[1], q[M]


@dataclass
class BatchedOut:
    grad_x: List[torch.Tensor]
    grad_w: Optional[List[torch.Tensor]]
    value: Optional[torch.Tensor]


def _batched_mode_flag(mode, persistent: bool) -> int:
    """None: the library's rule (the exchange solve when it applies, else lockstep
    launches); "lockstep" -> CT_UNFUSED; "persistent" (or persistent=True) ->
    CT_PERSISTENT; "mesh" -> CT_MESH."""
    if persistent:
        if mode not in (None, "persistent"):
            raise ValueError("persistent=True conflicts with mode=%r" % (mode,))
        return L.CT_PERSISTENT
    table = {None: 0, "lockstep": L.CT_UNFUSED, "persistent": L.CT_PERSISTENT, "mesh": L.CT_MESH}
    if mode not in table:
        raise ValueError(f"mode must be None, 'lockstep', 'persistent' or 'mesh' (got {mode!r})")
    return table[mode]


def sinkhorn_grad_batched(xs: Sequence[torch.Tensor], ys: Sequence[torch.Tensor],
                          ws: Optional[Sequence[torch.Tensor]] = None, *, eps: float, iters: int,
                          debias: bool = True, value: bool = False, grad_w: bool = False,
                          safe: bool = False, persistent: bool = False,
                          expanded: bool = True, mode: Optional[str] = None) -> BatchedOut:
    """Many independent problems (ragged T_b, M_b) in one batch: by default the
    exchange solve in one launch when every problem fits it, else lockstep
    launches over all of them; mode "lockstep", "persistent" (or persistent=True:
    one persistent work-list launch) or "mesh" forces one execution.  expanded: as
    for sinkhorn_grad (the lockstep launches' lagged sweeps)."""
    B = len(xs)
    if B < 1 or len(ys) != B or (ws is not None and len(ws) != B):
        raise ValueError("xs, ys (and ws) must be non-empty lists of equal length")
    dev = xs[0].device
    d = xs[0].shape[1]
    T_off = np.zeros(B + 1, dtype=np.int64)
    M_off = np.zeros(B + 1, dtype=np.int64)
    for b in range(B):
        T_off[b + 1] = T_off[b] + xs[b].shape[0]
        M_off[b + 1] = M_off[b] + ys[b].shape[0]
    x = _req(torch.cat([_req(t, "x", dev) for t in xs]), "x")
    y = _req(torch.cat([_req(t, "y", dev) for t in ys]), "y")
    w = None if ws is None else _req(torch.cat([_req(t, "w", dev) for t in ws]), "w")
    flags = (L.CT_DEBIAS if debias else 0) | (L.CT_VALUE if value else 0) | \
        (L.CT_GRAD_W if grad_w else 0) | (L.CT_SAFE_LSE if safe else 0) | \
        _batched_mode_flag(mode, persistent) | (0 if expanded else L.CT_DIFFERENCE)
    o = _opts(d, eps, iters, flags)
    to = T_off.ctypes.data_as(L.PI64)
    mo = M_off.ctypes.data_as(L.PI64)
    gx = torch.empty_like(x)
    gw = torch.empty(int(M_off[-1]), dtype=torch.float32, device=dev) if grad_w else None
    val = torch.empty(B, dtype=torch.float32, device=dev) if value else None
    nbytes = lib().ct_sinkhorn_batched_workspace_size(B, to, mo, ctypes.byref(o))
    wsb = _workspace(nbytes, dev)
    check("ct_sinkhorn_batched_prepare",
          lib().ct_sinkhorn_batched_prepare(B, to, mo, ctypes.byref(o), _p(wsb), nbytes, _stream(dev)))
    st = lib().ct_sinkhorn_grad_batched(B, to, mo, _p(x), _p(y), _p(w), ctypes.byref(o), _p(gx),
                                        _p(gw), _p(val), _p(wsb), nbytes, _stream(dev))
    check("ct_sinkhorn_grad_batched", st)
    gxs = [gx[T_off[b]:T_off[b + 1]] for b in range(B)]
    gws = None if gw is None else [gw[M_off[b]:M_off[b + 1]] for b in range(B)]
    return BatchedOut(gxs, gws, val)


class BatchedSinkhorn:
    """A prepared batch: fixed sizes, inputs copied into static buffers, outputs
    and workspace allocated once.  run() enqueues only kernels (no host sync), so
    it can be captured into a graph (capture()) and replayed."""

    def __init__(self, xs, ys, ws=None, *, eps: float, iters: int, debias: bool = True,
                 value: bool = False, grad_w: bool = False, safe: bool = False,
                 persistent: bool = False, expanded: bool = True, mode: Optional[str] = None):
        B = len(xs)
        if B < 1 or len(ys) != B or (ws is not None and len(ws) != B):
            raise ValueError("xs, ys (and ws) must be non-empty lists of equal length")
        self.dev = xs[0].device
        self.d = xs[0].shape[1]
        self.B = B
        self.T_off = np.zeros(B + 1, dtype=np.int64)
        self.M_off = np.zeros(B + 1, dtype=np.int64)
        for b in range(B):
            self.T_off[b + 1] = self.T_off[b] + xs[b].shape[0]
            self.M_off[b + 1] = self.M_off[b] + ys[b].shape[0]
        self.x = _req(torch.cat([_req(t, "x", self.dev) for t in xs]), "x")
        self.y = _req(torch.cat([_req(t, "y", self.dev) for t in ys]), "y")
        self.w = None if ws is None else _req(torch.cat([_req(t, "w", self.dev) for t in ws]), "w")
        flags = (L.CT_DEBIAS if debias else 0) | (L.CT_VALUE if value else 0) | \
            (L.CT_GRAD_W if grad_w else 0) | (L.CT_SAFE_LSE if safe else 0) | \
            _batched_mode_flag(mode, persistent) | (0 if expanded else L.CT_DIFFERENCE)
        self.o = _opts(self.d, eps, iters, flags)
        self._to = self.T_off.ctypes.data_as(L.PI64)
        self._mo = self.M_off.ctypes.data_as(L.PI64)
        self.grad_x = torch.empty_like(self.x)
        self.grad_w = torch.empty(int(self.M_off[-1]), dtype=torch.float32,
                                  device=self.dev) if grad_w else None
        self.value = torch.empty(B, dtype=torch.float32, device=self.dev) if value else None
        self.nbytes = lib().ct_sinkhorn_batched_workspace_size(B, self._to, self._mo,
                                                               ctypes.byref(self.o))
        self.ws = _workspace(self.nbytes, self.dev)
        check("ct_sinkhorn_batched_prepare",
              lib().ct_sinkhorn_batched_prepare(B, self._to, self._mo, ctypes.byref(self.o),
                                                _p(self.ws), self.nbytes, _stream(self.dev)))

    def run(self) -> None:
        st = lib().ct_sinkhorn_grad_batched(self.B, self._to, self._mo, _p(self.x), _p(self.y),
                                            _p(self.w), ctypes.byref(self.o), _p(self.grad_x),
                                            _p(self.grad_w), _p(self.value), _p(self.ws),
                                            self.nbytes, _stream(self.dev))
        check("ct_sinkhorn_grad_batched", st)

    def capture(self):
        """Capture run() into a torch CUDA (HIP) graph; replay with g.replay()."""
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        return g

    def split(self, t: torch.Tensor, off: np.ndarray):
        return [t[off[b]:off[b + 1]] for b in range(self.B)]


@dataclass
class GMM:
    """Gaussian mixture on the GPU: weights [K], means [K,d], sigmas [K,d], uniform floor."""
    weights: torch.Tensor
    means: torch.Tensor
    sigmas: torch.Tensor
    floor: float = 0.0

    @staticmethod
    def from_numpy(g, device) -> "GMM":
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=device)
        return GMM(t(g.weights), t(g.means), t(g.sigmas), float(g.floor))

    def desc(self) -> L.GMMDesc:
        return L.GMMDesc(int(self.weights.shape[0]), self.weights.data_ptr(),
                         self.means.data_ptr(), self.sigmas.data_ptr(), float(self.floor))


def svgd_grad(x: torch.Tensor, gmm: GMM, h: Optional[float] = None, *, return_score: bool = False):
    """Stein variational flow phi (eq. 4) with the RBF kernel and the mixture's
    score; h None/<=0 selects the median heuristic.  Returns (phi, h_used[, score])."""
    dev = x.device
    x = _req(x, "x")
    T, d = x.shape
    for name in ("weights", "means", "sigmas"):
        setattr(gmm, name, _req(getattr(gmm, name), name, dev))
    phi = torch.empty_like(x)
    score = torch.empty_like(x) if return_score else None
    hu = torch.empty(1, dtype=torch.float32, device=dev)
    nbytes = lib().ct_svgd_workspace_size(T, d)
    ws = _workspace(nbytes, dev)
    desc = gmm.desc()
    st = lib().ct_svgd_grad(_p(x), T, d, ctypes.byref(desc), float(h if h else 0.0), _p(phi),
                            _p(score), _p(hu), _p(ws), nbytes, _stream(dev))
    check("ct_svgd_grad", st)
    return (phi, hu, score) if return_score else (phi, hu)


def svgd_grad_score(x: torch.Tensor, score: torch.Tensor, h: Optional[float] = None):
    """Stein variational flow phi (eq. 4) for a score already on the GPU (any
    unnormalised target).  Returns (phi, h_used)."""
    dev = x.device
    x = _req(x, "x")
    score = _req(score, "score", dev)
    T, d = x.shape
    if tuple(score.shape) != (T, d):
        raise ValueError(f"score must have shape {(T, d)}, got {tuple(score.shape)}")
    phi = torch.empty_like(x)
    hu = torch.empty(1, dtype=torch.float32, device=dev)
    nbytes = lib().ct_svgd_workspace_size(T, d)
    ws = _workspace(nbytes, dev)
    st = lib().ct_svgd_grad_score(_p(x), T, d, _p(score), float(h if h else 0.0), _p(phi), _p(hu),
                                  _p(ws), nbytes, _stream(dev))
    check("ct_svgd_grad_score", st)
    return phi, hu


@dataclass
class UtilityGrid:
    """Utility map on a regular grid over the box [lo, hi] (a continuous-utility
    reference): u [n1, n0] (d = 2) or [n2, n1, n0] (d = 3) on the GPU, axis 0
    varying fastest; the density is proportional to its multilinear interpolant
    plus ``floor``."""
    u: torch.Tensor
    lo: Sequence[float]
    hi: Sequence[float]
    floor: float = 0.0

    @property
    def d(self) -> int:
        return self.u.dim()

    def desc(self) -> L.GridDesc:
        d = self.d
        if d not in (2, 3):
            raise ValueError("u must have 2 or 3 dimensions")
        if len(self.lo) != d or len(self.hi) != d:
            raise ValueError("lo and hi need one entry per axis")
        self.u = _req(self.u, "u")
        n = list(reversed(self.u.shape)) + [1] * (3 - d)
        pad = lambda v: [float(a) for a in v] + [0.0] * (3 - d)
        return L.GridDesc((ctypes.c_int32 * 3)(*n), (ctypes.c_float * 3)(*pad(self.lo)),
                          (ctypes.c_float * 3)(*pad(self.hi)), self.u.data_ptr(), float(self.floor))


def grid_score(x: torch.Tensor, grid: UtilityGrid) -> torch.Tensor:
    """grad log(U + floor) at every sample (the utility grid's score)."""
    x = _req(x, "x", grid.u.device)
    T, d = x.shape
    if d != grid.d:
        raise ValueError(f"x has d={d}, the grid d={grid.d}")
    desc = grid.desc()
    score = torch.empty_like(x)
    st = lib().ct_grid_score(_p(x), T, d, ctypes.byref(desc), _p(score), _stream(x.device))
    check("ct_grid_score", st)
    return score


def grid_samples(grid: UtilityGrid):
    """The utility's nodes as weighted reference samples for the Sinkhorn flow:
    (y [M,d], w [M]), trapezoid-rule weights normalised to 1, zero-weight nodes
    dropped.  Synchronous."""
    desc = grid.desc()
    d = grid.d
    dev = grid.u.device
    N = grid.u.numel()
    y = torch.empty((N, d), dtype=torch.float32, device=dev)
    w = torch.empty(N, dtype=torch.float32, device=dev)
    M = ctypes.c_int64(0)
    nbytes = lib().ct_grid_samples_workspace_size(ctypes.byref(desc), d)
    ws = _workspace(nbytes, dev)
    st = lib().ct_grid_samples(ctypes.byref(desc), d, _p(y), _p(w), ctypes.byref(M), _p(ws), nbytes,
                               _stream(dev))
    check("ct_grid_samples", st)
    return y[:M.value], w[:M.value]


def _dp(a: np.ndarray):
    return a.ctypes.data_as(L.PD)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def lqr_track(A, B, a, Q, R, dt: float):
    """Host FP64 tracking LQR (eqs. 9-10); returns (v [T,m], z [T+1,n])."""
    A, B, a, Q, R = (_f64(t) for t in (A, B, a, Q, R))
    T, n, m = B.shape
    v = np.empty((T, m))
    z = np.empty((T + 1, n))
    st = lib().ct_lqr_track(T, n, m, float(dt), _dp(A), _dp(B), _dp(a), _dp(Q), _dp(R), _dp(v), _dp(z))
    check("ct_lqr_track", st)
    return v, z


_DYN = {"double_integrator": L.CT_DYN_DOUBLE_INTEGRATOR, "unicycle": L.CT_DYN_UNICYCLE}
_FLOW = {"sinkhorn": L.CT_FLOW_SINKHORN, "svgd": L.CT_FLOW_SVGD, "svgd_grid": L.CT_FLOW_SVGD_GRID}


def plan(dynamics: str, s0, u, dt: float, Q, R, flow: str, outer: int, step: float = 1.0, *,
         y: Optional[torch.Tensor] = None, w: Optional[torch.Tensor] = None,
         gmm: Optional[GMM] = None, grid: Optional[UtilityGrid] = None, eps: float = 0.01,
         iters: int = 100, debias: bool = True, svgd_h: float = 0.0, device=None,
         fused=None):
    """Outer planning loop (ct_plan).  flow: "sinkhorn" (y, w), "svgd" (gmm) or
    "svgd_grid" (grid).  fused: as for sinkhorn_grad.  Returns (u [T,m],
    s [T+1,n], hist [outer])."""
    s0 = _f64(s0)
    u = _f64(u).copy()
    Q = _f64(Q)
    R = _f64(R)
    T, m = u.shape
    d = Q.shape[0]
    n = s0.shape[0]
    dev = torch.device(device) if device is not None else (
        y.device if y is not None else gmm.weights.device if gmm is not None else grid.u.device)
    prob = L.PlanProblem(_DYN[dynamics], d, T, float(dt), _dp(s0))
    sk = _opts(d, eps, iters, (L.CT_DEBIAS if debias else 0) | _fused_flag(fused))
    gdesc = grid.desc() if grid is not None else None
    opts = L.PlanOpts(_FLOW[flow], int(outer), float(step), _dp(Q), _dp(R), sk, float(svgd_h),
                      ctypes.pointer(gdesc) if gdesc is not None else None)
    M = 0
    if y is not None:
        y = _req(y, "y", dev)
        M = y.shape[0]
        if w is not None:
            w = _req(w, "w", dev)
    desc = None
    if gmm is not None:
        for name in ("weights", "means", "sigmas"):
            setattr(gmm, name, _req(getattr(gmm, name), name, dev))
        desc = gmm.desc()
    s = np.empty((T + 1, n))
    hist = np.empty(outer)
    nbytes = lib().ct_plan_workspace_size(ctypes.byref(prob), ctypes.byref(opts), M)
    ws = _workspace(nbytes, dev)
    st = lib().ct_plan(ctypes.byref(prob), ctypes.byref(opts), _p(y), _p(w), M,
                       ctypes.byref(desc) if desc is not None else None, _dp(u), _dp(s), _dp(hist),
                       _p(ws), nbytes, _stream(dev))
    check("ct_plan", st)
    return u, s, hist


def plan_ensemble(dynamics: str, s0, U, dt: float, Q, R, outer: int, step: float = 1.0, *,
                  y: torch.Tensor, w: Optional[torch.Tensor] = None, eps: float = 0.01,
                  iters: int = 100, debias: bool = True):
    """Seed ensemble of the Sinkhorn planner (ct_plan_ensemble): U [S,T,m] initial
    controls.  Returns (U [S,T,m], s [S,T+1,n], values [S], best)."""
    s0 = _f64(s0)
    U = np.ascontiguousarray(_f64(U)).copy()
    Q = _f64(Q)
    R = _f64(R)
    S, T, m = U.shape
    d = Q.shape[0]
    n = s0.shape[0]
    dev = y.device
    y = _req(y, "y", dev)
    M = y.shape[0]
    if w is not None:
        w = _req(w, "w", dev)
    prob = L.PlanProblem(_DYN[dynamics], d, T, float(dt), _dp(s0))
    sk = _opts(d, eps, iters, L.CT_DEBIAS if debias else 0)
    opts = L.PlanOpts(_FLOW["sinkhorn"], int(outer), float(step), _dp(Q), _dp(R), sk, 0.0)
    s = np.empty((S, T + 1, n))
    values = np.empty(S)
    best = ctypes.c_int32(-1)
    nbytes = lib().ct_plan_ensemble_workspace_size(ctypes.byref(prob), ctypes.byref(opts), S, M,
                                                   1 if w is not None else 0)
    ws = _workspace(nbytes, dev)
    st = lib().ct_plan_ensemble(ctypes.byref(prob), ctypes.byref(opts), S, _p(y), _p(w), M,
                                _dp(U), _dp(s), _dp(values), ctypes.byref(best), _p(ws), nbytes,
                                _stream(dev))
    check("ct_plan_ensemble", st)
    return U, s, values, int(best.value)


def autotune_sinkhorn(T: int, M: int, d: int, eps: float, device="cuda") -> None:
    """Time the candidate sweep schedules for this shape and record the best."""
    dev = torch.device(device)
    o = _opts(d, eps, 1, L.CT_DEBIAS | L.CT_VALUE | L.CT_GRAD_W)
    nbytes = lib().ct_sinkhorn_workspace_size(T, M, ctypes.byref(o))
    ws = _workspace(nbytes, dev)
    st = lib().ct_autotune_sinkhorn(T, M, ctypes.byref(o), _p(ws), nbytes, _stream(dev))
    check("ct_autotune_sinkhorn", st)


def probe_alu_rates(device="cuda") -> dict:
    """Measured issue rates of the instructions that bound the sweeps (see
    ct_probe_alu_rates): lanes per clock per CU of add, FMA and exp2, MFMA FP32
    FMAs per clock per CU, the MFMA/exp overlap ratio and the clock in Hz."""
    dev = torch.device(device)
    n = lib().ct_probe_workspace_size()
    ws = _workspace(n, dev)
    out = (ctypes.c_double * 6)()
    check("ct_probe_alu_rates", lib().ct_probe_alu_rates(out, _p(ws), n, _stream(dev)))
    keys = ("add", "fma", "exp", "mfma_f32", "mfma_exp_overlap", "clock_hz")
    return dict(zip(keys, list(out)))


def tuning_table():
    """Entries (d, qclass, kclass, R, WS, blocks_per_cu, sep, us)."""
    n = lib().ct_tuning_count()
    out = []
    buf = (ctypes.c_int32 * 8)()
    for i in range(n):
        check("ct_tuning_entry", lib().ct_tuning_entry(i, buf))
        out.append(tuple(buf))
    return out


def tuning_save(path: str) -> None:
    check("ct_tuning_save", lib().ct_tuning_save(path.encode()))


def tuning_load(path: str) -> None:
    check("ct_tuning_load", lib().ct_tuning_load(path.encode()))


def tuning_clear() -> None:
    lib().ct_tuning_clear()
