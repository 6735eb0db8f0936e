"""Property-based pins of the FP64 oracle (hypothesis, derandomised): invariants
that hold for every input, checked over random small clouds at convergence.

* The debiased Sinkhorn divergence (Sec. II-B, eq. 6) is nonnegative, symmetric
  in its two uniform measures, unchanged by a common translation of both clouds
  and by a rescaling of the reference weights (which enter as b = w / sum w), so
  its weight gradient is orthogonal to w.
* The utility grid's multilinear interpolant is a convex combination of its
  cell's corners.
* The Riccati recursion equals the dense least-squares solution of the tracking
  problem (eqs. 9-10) for random stable systems.
"""
import numpy as np
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import oracle  # noqa: E402
from oracle import grid as G  # noqa: E402

SET = settings(max_examples=25, deadline=None, derandomize=True)


def _clouds(seed, T, M, d, spread):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, spread, (T, d))
    y = rng.uniform(0.0, spread, (M, d))
    w = rng.uniform(0.2, 2.0, M)
    return x, y, w


@SET
@given(seed=st.integers(0, 10**6), T=st.integers(1, 6), M=st.integers(1, 6), d=st.sampled_from([2, 3]),
       eps=st.floats(0.1, 1.0))
def test_divergence_nonnegative_and_invariant(seed, T, M, d, eps):
    x, y, w = _clouds(seed, T, M, d, 1.0)
    iters = 400
    r = oracle.sinkhorn(x, y, w, eps=eps, iters=iters)
    assert r.value >= -1e-10
    shift = np.random.default_rng(seed + 1).normal(size=d)
    r2 = oracle.sinkhorn(x + shift, y + shift, w, eps=eps, iters=iters)
    assert r2.value == pytest.approx(r.value, rel=1e-8, abs=1e-12)
    np.testing.assert_allclose(r2.grad_x, r.grad_x, rtol=1e-7, atol=1e-11)
    r3 = oracle.sinkhorn(x, y, 7.5 * w, eps=eps, iters=iters)
    assert r3.value == pytest.approx(r.value, rel=1e-10, abs=1e-14)
    assert abs(w @ r.grad_w) <= 1e-9 * max(1.0, np.abs(w).sum() * np.abs(r.grad_w).max())


@SET
@given(seed=st.integers(0, 10**6), T=st.integers(1, 6), M=st.integers(1, 6), d=st.sampled_from([2, 3]),
       eps=st.floats(0.1, 1.0))
def test_divergence_is_symmetric_for_uniform_measures(seed, T, M, d, eps):
    x, y, _w = _clouds(seed, T, M, d, 1.0)
    a = oracle.sinkhorn(x, y, None, eps=eps, iters=400)
    b = oracle.sinkhorn(y, x, None, eps=eps, iters=400)
    assert a.value == pytest.approx(b.value, rel=1e-8, abs=1e-12)


@SET
@given(seed=st.integers(0, 10**6), n0=st.integers(2, 7), n1=st.integers(2, 7),
       n2=st.integers(2, 5), three=st.booleans(), floor=st.floats(0.0, 0.5))
def test_grid_interpolant_is_a_convex_combination_of_corners(seed, n0, n1, n2, three, floor):
    rng = np.random.default_rng(seed)
    n = (n0, n1, n2) if three else (n0, n1)
    d = len(n)
    u = rng.uniform(0.0, 3.0, tuple(reversed(n)))
    lo = rng.uniform(-1.0, 1.0, d)
    hi = lo + rng.uniform(0.5, 2.0, d)
    g = G.Grid(u, lo, hi, floor)
    x = rng.uniform(lo, hi, (64, d))
    val = G.interp(g, x) - floor
    c = np.minimum(np.floor((x - lo) * (np.array(n) - 1) / (hi - lo)), np.array(n) - 2).astype(int)
    for k in range(len(x)):
        corners = [u[tuple(reversed(tuple(c[k] + np.array(bits))))]
                   for bits in np.ndindex(*([2] * d))]
        assert min(corners) - 1e-12 <= val[k] <= max(corners) + 1e-12


@SET
@given(seed=st.integers(0, 10**6), T=st.integers(1, 12), n=st.integers(1, 4), m=st.integers(1, 3))
def test_riccati_equals_dense_least_squares(seed, T, n, m):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(T, n, n)) * 0.3
    B = rng.normal(size=(T, n, m))
    a = rng.normal(size=(T, n))
    Q = np.diag(rng.uniform(0.5, 2.0, n))
    R = np.diag(rng.uniform(0.05, 1.0, m))
    dt = 0.1
    v1, z1 = oracle.lqr_track_dense(A, B, a, Q, R, dt)
    v2, z2 = oracle.lqr_track_riccati(A, B, a, Q, R, dt)
    np.testing.assert_allclose(v2, v1, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(z2, z1, rtol=1e-7, atol=1e-9)
