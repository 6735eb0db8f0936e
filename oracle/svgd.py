"""Stein variational flow (Sec. II-B, eq. 4) in float64 (oracle).

Test infrastructure only.

  g(s_i) = 1/n sum_j [ k(s_j, s_i) grad log q(s_j) + grad_{s_j} k(s_j, s_i) ]

with the radial basis kernel k(s, s') = exp(-|s - s'|^2 / h).  Since
grad_{s_j} k(s_j, s_i) = (2/h)(s_i - s_j) k(s_j, s_i), this is
  phi_i = 1/n sum_j k_ij [score_j + (2/h)(x_i - x_j)]   (the j = i term included).

Readings where the paper is silent:
* bandwidth by the median heuristic of the SVGD paper the method cites:
  h = med^2 / ln n, med = median of the n(n-1)/2 distances |x_i - x_j|, i < j
  (mean of the two middle values when that count is even); h = 1 when n = 1 or
  when the median distance is zero (all samples coincide);
* the reference q is a Gaussian mixture with diagonal covariances, optionally
  mixed with a uniform density of mass rho on [0,1]^d:
    q(x) = (1 - rho) sum_k pi_k N(x; mu_k, diag sigma_k^2) + rho 1[x in [0,1]^d];
  its score is sum_k r_k(x) (-(x - mu_k) / sigma_k^2) with r_k the posterior
  responsibility of component k (the uniform part has zero gradient).
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._clib import dptr, f64, lib


def _component_logs(x, weights, means, sigmas, floor):
    """log((1-rho) pi_k N_k(x)) for every component, plus the uniform component's
    log-mass (-inf outside the box or when rho = 0).  Shapes [n,K], [n]."""
    x = f64(x)
    mu = f64(means)
    sg = f64(sigmas)
    pi = f64(weights)
    diff = x[:, None, :] - mu[None, :, :]                       # [n,K,d]
    logn = -0.5 * np.sum(diff ** 2 / sg[None] ** 2 + np.log(2.0 * np.pi * sg[None] ** 2), axis=2)
    with np.errstate(divide="ignore"):
        logc = np.log((1.0 - floor) * pi)[None, :] + logn
        inside = np.all((x >= 0.0) & (x <= 1.0), axis=1)
        logu = np.where(inside & (floor > 0.0), np.log(floor) if floor > 0 else -np.inf, -np.inf)
    return logc, logu, diff, sg


def gmm_logpdf(x, weights, means, sigmas, floor: float = 0.0) -> np.ndarray:
    logc, logu, _, _ = _component_logs(x, weights, means, sigmas, floor)
    allv = np.concatenate([logc, logu[:, None]], axis=1)
    m = np.max(allv, axis=1, keepdims=True)
    return (m + np.log(np.sum(np.exp(allv - m), axis=1, keepdims=True)))[:, 0]


def gmm_score(x, weights, means, sigmas, floor: float = 0.0) -> np.ndarray:
    """grad log q(x) for the mixture above, [n,d]."""
    logc, logu, diff, sg = _component_logs(x, weights, means, sigmas, floor)
    allv = np.concatenate([logc, logu[:, None]], axis=1)
    m = np.max(allv, axis=1, keepdims=True)
    r = np.exp(allv - m)
    r = r / np.sum(r, axis=1, keepdims=True)                     # responsibilities
    rk = r[:, :-1]                                               # the uniform one has zero score
    return np.sum(rk[:, :, None] * (-diff / sg[None] ** 2), axis=1)


def median_bandwidth(x) -> float:
    """h = med^2 / ln n from the median pairwise distance (i < j)."""
    x = f64(x)
    n = x.shape[0]
    if n < 2:
        return 1.0
    iu = np.triu_indices(n, k=1)
    dist = np.sqrt(np.sum((x[iu[0]] - x[iu[1]]) ** 2, axis=1))
    npair = dist.shape[0]
    srt = np.partition(dist, [(npair - 1) // 2, npair // 2])
    med = 0.5 * (srt[(npair - 1) // 2] + srt[npair // 2])
    if med == 0.0:
        return 1.0
    return float(med * med / np.log(n))


def svgd_phi(x, score, h: float) -> np.ndarray:
    """phi_i = 1/n sum_j exp(-|x_i-x_j|^2/h) [score_j + (2/h)(x_i - x_j)], [n,d]."""
    x = f64(x)
    s = f64(score)
    phi = np.empty_like(x)
    lib().orc_svgd_phi(x.shape[1], x.shape[0], dptr(x), dptr(s), float(h), dptr(phi))
    return phi


def _kth_sqdist(x, k: int, lo_bits: int = -1) -> float:
    """The k-th smallest (0-based) squared distance |x_i - x_j|^2 over pairs i < j,
    found by bisection on the threshold with pair counts: non-negative doubles
    order like their bit patterns, so bisecting the pattern between one whose
    count of pairs at or below it is <= k and one whose count exceeds k ends on
    the exact value after at most 63 halvings."""
    hi = 0x7FF0000000000000                       # +inf: every pair is at or below it
    lo = lo_bits                                  # below every pair
    while hi - lo > 1:
        mid = (lo + hi) // 2
        v = float(np.array([mid], dtype=np.int64).view(np.float64)[0])
        if pair_count(x, v)[1] >= k + 1:
            hi = mid
        else:
            lo = mid
    return float(np.array([hi], dtype=np.int64).view(np.float64)[0])


def median_bandwidth_by_counting(x) -> float:
    """The median heuristic of median_bandwidth, with the two middle order
    statistics found by pair counting (no list of all n(n-1)/2 distances, so it
    runs at any n); the same value in exact arithmetic and, as both take the
    square root of the same double squared distance, in float64."""
    x = f64(x)
    n = x.shape[0]
    if n < 2:
        return 1.0
    npair = n * (n - 1) // 2
    k1, k2 = (npair - 1) // 2, npair // 2
    v1 = _kth_sqdist(x, k1)
    if k2 == k1 or pair_count(x, v1)[1] >= k2 + 1:
        v2 = v1
    else:
        v2 = _kth_sqdist(x, k2, lo_bits=int(np.array([v1]).view(np.int64)[0]))
    med = 0.5 * (np.sqrt(v1) + np.sqrt(v2))
    if med == 0.0:
        return 1.0
    return float(med * med / np.log(n))


def pair_count(x, thr_sq: float):
    """(#pairs i<j with |x_i-x_j|^2 < thr_sq, #pairs with <= thr_sq)."""
    x = f64(x)
    lt = ctypes.c_int64()
    le = ctypes.c_int64()
    lib().orc_pair_count(x.shape[1], x.shape[0], dptr(x), float(thr_sq),
                         ctypes.byref(lt), ctypes.byref(le))
    return lt.value, le.value
