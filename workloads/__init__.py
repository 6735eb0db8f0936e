"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and arranges them into arrays; it holds
none of the method's arithmetic (no costs, potentials, scores or flows).  Both
the FP64 oracle and the HIP path read exactly the arrays produced here: every
generator works in float64 with numpy's PCG64 and rounds the result to float32
once, so the oracle (which widens the float32 values back to float64) and the
GPU see bit-identical inputs.

The shapes and distributions stand in for the paper's coverage workloads
(Sec. III; its reference maps and trajectories are not published):

* trajectory samples: a smooth, reflected random walk in the unit box, i.e. the
  time-equispaced states of a moving robot (Sec. II-A, eq. 1);
* reference samples: draws from a Gaussian mixture on the unit box, optionally
  mixed with a uniform floor (Sec. II-A: the target given as samples or as a
  density);
* utility maps: node values on a regular grid over the unit box, a sum of a few
  random bumps with a rectangular region of zero utility (an obstacle) (Sec. II-A:
  the target given as a continuous utility function).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "GMM", "gmm_params", "gmm_sample", "random_walk", "uniform_points",
    "positive_weights", "Config", "CONFIGS", "config_inputs", "batch_inputs",
    "HORIZON_SWEEPS", "horizon_inputs", "utility_map",
]


@dataclass
class GMM:
    """Gaussian-mixture description: weights [K], means [K,d], std-devs [K,d],
    and the mass of a uniform floor on [0,1]^d (0 = no floor).  All float32."""
    weights: np.ndarray
    means: np.ndarray
    sigmas: np.ndarray
    floor: float = 0.0

    @property
    def K(self) -> int:
        return int(self.weights.shape[0])

    @property
    def d(self) -> int:
        return int(self.means.shape[1])


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def gmm_params(rng: np.random.Generator, K: int, d: int, sigma_lo: float, sigma_hi: float,
               anisotropic: bool = False, floor: float = 0.0) -> GMM:
    """Mixture weights ~ Dirichlet(1_K), means ~ U[0.2,0.8]^d, standard deviations
    ~ U[sigma_lo, sigma_hi] (one per component, or one per axis if anisotropic)."""
    w = rng.dirichlet(np.ones(K))
    mu = rng.uniform(0.2, 0.8, size=(K, d))
    if anisotropic:
        sig = rng.uniform(sigma_lo, sigma_hi, size=(K, d))
    else:
        sig = np.repeat(rng.uniform(sigma_lo, sigma_hi, size=(K, 1)), d, axis=1)
    return GMM(_f32(w), _f32(mu), _f32(sig), float(np.float32(floor)))


def gmm_sample(rng: np.random.Generator, g: GMM, n: int) -> np.ndarray:
    """n draws from the mixture (with the uniform floor as one more component).
    Samples are not clipped to the box."""
    w = g.weights.astype(np.float64)
    w = w / w.sum() * (1.0 - g.floor)
    probs = np.concatenate([w, [g.floor]])
    comp = rng.choice(g.K + 1, size=n, p=probs / probs.sum())
    z = rng.standard_normal(size=(n, g.d))
    out = g.means.astype(np.float64)[np.minimum(comp, g.K - 1)] + \
        z * g.sigmas.astype(np.float64)[np.minimum(comp, g.K - 1)]
    uni = comp == g.K
    if uni.any():
        out[uni] = rng.uniform(0.0, 1.0, size=(int(uni.sum()), g.d))
    return _f32(out)


def random_walk(rng: np.random.Generator, T: int, d: int, momentum: float = 0.98,
                step: float = 0.002) -> np.ndarray:
    """Smooth random walk reflected into [0,1]^d: x0 ~ U[0.3,0.7]^d, v0 = 0,
    v <- momentum*v + step*N(0,I), x <- x + v (position and velocity reflected
    at the walls).  Returns the T positions after x0."""
    x = rng.uniform(0.3, 0.7, size=d)
    v = np.zeros(d)
    out = np.empty((T, d))
    noise = rng.standard_normal(size=(T, d))
    for t in range(T):
        v = momentum * v + step * noise[t]
        x = x + v
        lo = x < 0.0
        x[lo] = -x[lo]
        v[lo] = -v[lo]
        hi = x > 1.0
        x[hi] = 2.0 - x[hi]
        v[hi] = -v[hi]
        out[t] = x
    return _f32(out)


def uniform_points(rng: np.random.Generator, n: int, d: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    return _f32(rng.uniform(lo, hi, size=(n, d)))


def utility_map(rng: np.random.Generator, n, bumps: int = 5, obstacle: bool = True,
                lo=None, hi=None):
    """(u, lo, hi): a synthetic utility map on a grid of n = (n_0, ..., n_{d-1})
    nodes over the box [lo, hi] (default the unit box).  u has shape
    (n_{d-1}, ..., n_0) (axis 0 fastest in memory): the sum of `bumps` random
    isotropic bumps (amplitudes U[0.5, 2], centres U[0.15, 0.85] of the box, widths
    U[0.05, 0.2] of its extent), zeroed on a random axis-aligned box covering about
    a tenth of the area when `obstacle`.  float32."""
    d = len(n)
    lo = np.zeros(d) if lo is None else np.asarray(lo, np.float64)
    hi = np.ones(d) if hi is None else np.asarray(hi, np.float64)
    axes = [np.linspace(0.0, 1.0, k) for k in n]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")        # slowest axis first
    pts = np.stack(list(reversed(mesh)), axis=-1)              # [..., d], unit coordinates
    u = np.zeros(tuple(reversed(n)))
    for _ in range(bumps):
        a = rng.uniform(0.5, 2.0)
        c = rng.uniform(0.15, 0.85, d)
        s = rng.uniform(0.05, 0.2)
        u += a * np.exp(-np.sum((pts - c) ** 2, axis=-1) / (2.0 * s * s))
    if obstacle:
        side = 0.1 ** (1.0 / d)
        c0 = rng.uniform(0.1, 0.9 - side, d)
        inside = np.all((pts >= c0) & (pts <= c0 + side), axis=-1)
        u[inside] = 0.0
    return _f32(u), _f32(lo), _f32(hi)


def positive_weights(rng: np.random.Generator, n: int, lo: float = 0.5, hi: float = 2.0) -> np.ndarray:
    return _f32(rng.uniform(lo, hi, size=n))


@dataclass
class Config:
    """One benchmark/parity workload (sizes, distributions, solver settings)."""
    name: str
    d: int
    T: int
    M: int
    K_gmm: int
    sigma: tuple
    eps: float
    iters: int
    seed: int
    anisotropic: bool = False
    floor: float = 0.0
    trajectory: str = "walk"          # "walk" (random walk) or "uniform"
    extra: dict = field(default_factory=dict)


# The five workloads: planner-sized, the 2D gradient benchmark, the 3D
# differentiation case, the ragged batch, and the large roofline case.
CONFIGS = {
    "planner_2d": Config("planner_2d", 2, 256, 512, 3, (0.05, 0.15), 0.01, 100, 1000,
                         extra=dict(dynamics="double_integrator", dt=0.05, outer=10,
                                    s0=(0.5, 0.5, 0.0, 0.0), u_std=0.1, Q=1.0, R=0.01)),
    "grad_2d": Config("grad_2d", 2, 4096, 16384, 5, (0.03, 0.12), 0.005, 200, 2000),
    "autograd_3d": Config("autograd_3d", 3, 16384, 65536, 8, (0.02, 0.1), 0.01, 300, 3000,
                          anisotropic=True, extra=dict(fd_h=1e-4, fd_coords=64)),
    "batched_2d": Config("batched_2d", 2, 0, 0, 0, (0.03, 0.12), 0.01, 150, 4000,
                         extra=dict(B=256, T_range=(500, 8000), M_range=(1024, 32768),
                                    K_range=(2, 6))),
    "roofline_2d": Config("roofline_2d", 2, 65536, 262144, 16, (0.02, 0.08), 0.002, 500, 5000,
                          floor=0.1, extra=dict(dynamics="unicycle", dt=0.01, outer=20,
                                                s0=(0.5, 0.5, 0.0), v0=0.3, omega_std=0.5)),
}


# Planner time-versus-horizon sweeps (the shape of the paper's timing benchmark,
# Sec. III-A): the Stein flow with differential-drive (unicycle) dynamics over
# horizons 100..1000 step 100 and 2000..10000 step 1000, and the Sinkhorn flow
# over 100..500 step 100 and 1000..2500 step 500.  The paper's 3-D aircraft model
# is not given; a 3-D double integrator (point mass with acceleration control)
# stands in for it.  The Sinkhorn reference has as many samples as the horizon.
# Control steps: 0.5 (Sinkhorn) and 0.05 (Stein: its flow scales with the mixture
# score, ~1/sigma^2; steps of 0.1 and above diverge at some horizons of the sweep,
# 0.05 raised the samples' mean log-density at every horizon tried, 100..2000).
HORIZON_SWEEPS = {
    "svgd_drive": dict(flow="svgd", dynamics="unicycle", d=2,
                       horizons=list(range(100, 1001, 100)) + list(range(2000, 10001, 1000)),
                       K_gmm=4, sigma=(0.05, 0.12), floor=0.0, dt=0.01, s0=(0.5, 0.5, 0.0),
                       v0=0.3, omega_std=0.5, Q=1.0, R=0.01, step=0.05, outer=10, seed=6000),
    "sinkhorn_aircraft": dict(flow="sinkhorn", dynamics="double_integrator", d=3,
                              horizons=list(range(100, 501, 100)) + list(range(1000, 2501, 500)),
                              K_gmm=4, sigma=(0.05, 0.12), floor=0.0, dt=0.05,
                              s0=(0.5, 0.5, 0.5, 0.0, 0.0, 0.0), u_std=0.1, Q=1.0, R=0.01,
                              step=0.5, outer=10, eps=0.01, iters=100, seed=7000),
}


def horizon_inputs(name: str, T: int):
    """(s0 [n], u0 [T,m], y [M,d] or None, w [M] or None, gmm) for one horizon of a
    sweep; seeded per (sweep, T)."""
    c = HORIZON_SWEEPS[name]
    d = c["d"]
    rng = np.random.default_rng(c["seed"] + T)
    g = gmm_params(rng, c["K_gmm"], d, c["sigma"][0], c["sigma"][1], False, c["floor"])
    s0 = np.array(c["s0"], dtype=np.float64)
    if c["dynamics"] == "unicycle":
        u0 = np.stack([np.full(T, c["v0"]), rng.normal(size=T) * c["omega_std"]], axis=1)
    else:
        u0 = rng.normal(size=(T, d)) * c["u_std"]
    y = w = None
    if c["flow"] == "sinkhorn":
        y = gmm_sample(rng, g, T)
        w = np.ones(T, dtype=np.float32)
    return s0, u0, y, w, g


def config_inputs(cfg: Config, T: Optional[int] = None, M: Optional[int] = None):
    """(x [T,d], y [M,d], w [M], gmm) for a single-problem workload, optionally at
    reduced sizes (same seed and distributions)."""
    T = cfg.T if T is None else T
    M = cfg.M if M is None else M
    rng = np.random.default_rng(cfg.seed)
    g = gmm_params(rng, cfg.K_gmm, cfg.d, cfg.sigma[0], cfg.sigma[1], cfg.anisotropic, cfg.floor)
    y = gmm_sample(rng, g, M)
    if cfg.trajectory == "walk":
        x = random_walk(rng, T, cfg.d)
    else:
        x = uniform_points(rng, T, cfg.d)
    w = np.ones(M, dtype=np.float32)
    return x, y, w, g


def batch_inputs(cfg: Config, B: Optional[int] = None, scale: float = 1.0):
    """Ragged batch: list of (x_b, y_b, w_b) with T_b ~ U{T_range}, M_b ~ U{M_range}
    (optionally scaled down), each reference from its own GMM."""
    B = cfg.extra["B"] if B is None else B
    t_lo, t_hi = cfg.extra["T_range"]
    m_lo, m_hi = cfg.extra["M_range"]
    k_lo, k_hi = cfg.extra["K_range"]
    out = []
    for b in range(B):
        rng = np.random.default_rng(cfg.seed + b)
        T = max(1, int(round(rng.integers(t_lo, t_hi + 1) * scale)))
        M = max(1, int(round(rng.integers(m_lo, m_hi + 1) * scale)))
        K = int(rng.integers(k_lo, k_hi + 1))
        g = gmm_params(rng, K, cfg.d, cfg.sigma[0], cfg.sigma[1])
        y = gmm_sample(rng, g, M)
        x = random_walk(rng, T, cfg.d)
        out.append((x, y, np.ones(M, dtype=np.float32)))
    return out
