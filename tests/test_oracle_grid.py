"""Pins of the gridded-utility oracle (continuous-utility references, Sec. II-A,
and the score-only Stein flow, Sec. II-B) against closed forms, brute force and
independently written formulas."""
import itertools

import numpy as np
import pytest

from oracle import grid as G


def _box(d, rng):
    lo = rng.uniform(-2.0, 1.0, d)
    return lo, lo + rng.uniform(0.5, 3.0, d)


def _grid_u(n, rng, zero_frac=0.0):
    """Random node values with shape (n_{d-1}, ..., n_0)."""
    u = rng.uniform(0.2, 2.0, tuple(reversed(n)))
    if zero_frac:
        u[rng.uniform(size=u.shape) < zero_frac] = 0.0
    return u


@pytest.mark.parametrize("n", [(5, 7), (4, 6, 3)])
def test_separable_affine_utility_closed_form(n):
    # u(x) = prod_t (alpha_t + beta_t x_t) is multilinear, so the interpolant
    # reproduces it exactly and its score is beta_t / (alpha_t + beta_t x_t).
    rng = np.random.default_rng(11)
    d = len(n)
    lo, hi = _box(d, rng)
    beta = rng.uniform(-1.0, 1.0, d)
    alpha = 1.0 + np.abs(beta) * np.maximum(np.abs(lo), np.abs(hi)) + rng.uniform(0.1, 1.0, d)
    axes = [np.linspace(lo[t], hi[t], n[t]) for t in range(d)]
    fac = [alpha[t] + beta[t] * axes[t] for t in range(d)]
    u = fac[d - 1]
    for t in reversed(range(d - 1)):
        u = np.multiply.outer(u, fac[t])
    g = G.Grid(u, lo, hi, 0.0)
    x = rng.uniform(lo, hi, size=(400, d))
    want_val = np.prod(alpha + beta * x, axis=1)
    want_score = beta / (alpha + beta * x)
    np.testing.assert_allclose(G.interp(g, x), want_val, rtol=1e-12)
    np.testing.assert_allclose(G.score(g, x), want_score, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("n", [(4, 3), (3, 5, 2)])
def test_interpolant_hits_nodes_and_edge_midpoints(n):
    # A non-separable field on a non-square grid: any transposition of the
    # memory layout or of the node spacing moves these values.
    rng = np.random.default_rng(12)
    d = len(n)
    lo, hi = _box(d, rng)
    u = _grid_u(n, rng)
    g = G.Grid(u, lo, hi, 0.25)
    for j in itertools.product(*[range(k) for k in n]):
        p = np.array([lo[t] + j[t] * (hi[t] - lo[t]) / (n[t] - 1) for t in range(d)])
        assert G.interp(g, p[None])[0] == pytest.approx(u[tuple(reversed(j))] + 0.25, rel=1e-12)
        if j[0] + 1 < n[0]:
            q = p.copy()
            q[0] += 0.5 * (hi[0] - lo[0]) / (n[0] - 1)
            k = (j[0] + 1,) + tuple(j[1:])
            mid = 0.5 * (u[tuple(reversed(j))] + u[tuple(reversed(k))]) + 0.25
            assert G.interp(g, q[None])[0] == pytest.approx(mid, rel=1e-12)


@pytest.mark.parametrize("n", [(6, 5), (4, 5, 3)])
def test_score_is_gradient_of_log_interpolant(n):
    # Central differences of log(U + rho) at points kept away from cell faces.
    rng = np.random.default_rng(13)
    d = len(n)
    lo, hi = _box(d, rng)
    g = G.Grid(_grid_u(n, rng), lo, hi, 0.1)
    cells = np.array([rng.integers(0, k - 1, 200) for k in n]).T
    frac = rng.uniform(0.1, 0.9, (200, d))
    h = (hi - lo) / (np.array(n) - 1)
    x = lo + (cells + frac) * h
    step = 1e-6 * h
    fd = np.empty_like(x)
    for t in range(d):
        e = np.zeros(d)
        e[t] = step[t]
        fd[:, t] = (np.log(G.interp(g, x + e)) - np.log(G.interp(g, x - e))) / (2 * step[t])
    np.testing.assert_allclose(G.score(g, x), fd, rtol=1e-6, atol=1e-6)


def test_score_outside_box_and_zero_density():
    rng = np.random.default_rng(14)
    n = (5, 4)
    lo, hi = np.array([0.0, 0.0]), np.array([2.0, 1.0])
    u = _grid_u(n, rng)
    g = G.Grid(u, lo, hi, 0.0)
    inner = rng.uniform(lo, hi, (50, 2))
    out = inner.copy()
    out[:, 0] = hi[0] + rng.uniform(0.1, 5.0, 50)                  # beyond the upper x face
    clamped = out.copy()
    clamped[:, 0] = hi[0]
    s_out = G.score(g, out)
    s_cl = G.score(g, clamped)
    assert np.all(s_out[:, 0] == 0.0)                              # constant along x outside
    np.testing.assert_allclose(s_out[:, 1], s_cl[:, 1], rtol=1e-14)
    # a utility that vanishes on a whole cell, with no floor: zero score there
    z = np.zeros((4, 5))
    z[2:, 3:] = 1.0
    gz = G.Grid(z, lo, hi, 0.0)
    pts = rng.uniform([0.0, 0.0], [1.0, 0.33], (20, 2))             # cells far from the support
    assert np.all(G.score(gz, pts) == 0.0)


def test_score_ignores_normalisation():
    # the Stein flow needs only the score: scaling the utility and its floor together leaves it alone
    rng = np.random.default_rng(15)
    n = (4, 6, 3)
    lo, hi = _box(3, rng)
    u = _grid_u(n, rng, zero_frac=0.3)
    x = rng.uniform(lo - 0.2, hi + 0.2, (300, 3))
    a = G.score(G.Grid(u, lo, hi, 0.05), x)
    b = G.score(G.Grid(u * 37.5, lo, hi, 0.05 * 37.5), x)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("n", [(3, 4), (2, 3, 5)])
def test_samples_of_a_constant_utility(n):
    # closed form: weight of node j = prod_t c_t / (n_t - 1), c_t = 1/2 on a face, 1 inside
    rng = np.random.default_rng(16)
    d = len(n)
    lo, hi = _box(d, rng)
    g = G.Grid(np.full(tuple(reversed(n)), 3.0), lo, hi, 0.0)
    y, w = G.samples(g)
    assert y.shape == (int(np.prod(n)), d)
    k = 0
    for j in itertools.product(*[range(m) for m in reversed(n)]):
        j = tuple(reversed(j))                                     # axis 0 fastest
        want = np.prod([(0.5 if j[t] in (0, n[t] - 1) else 1.0) / (n[t] - 1) for t in range(d)])
        assert w[k] == pytest.approx(want, rel=1e-12)
        np.testing.assert_allclose(y[k], [lo[t] + j[t] * (hi[t] - lo[t]) / (n[t] - 1)
                                          for t in range(d)], rtol=1e-13, atol=1e-13)
        k += 1


@pytest.mark.parametrize("n", [(5, 4), (3, 4, 3)])
def test_sample_mass_is_the_interpolants_integral(n):
    # The integral of a multilinear cell piece is the cell volume times the mean
    # of its corners; summed over cells it must equal sum_j (u_j + rho) vol_j.
    rng = np.random.default_rng(17)
    d = len(n)
    lo, hi = _box(d, rng)
    u = _grid_u(n, rng, zero_frac=0.25)
    rho = 0.07
    g = G.Grid(u, lo, hi, rho)
    cell_vol = np.prod((hi - lo) / (np.array(n) - 1))
    exact = 0.0
    for c in itertools.product(*[range(m - 1) for m in n]):
        corners = [u[tuple(reversed(tuple(ci + b for ci, b in zip(c, bits))))]
                   for bits in itertools.product((0, 1), repeat=d)]
        exact += cell_vol * (np.mean(corners) + rho)
    mass = np.dot(u.ravel() + rho, G.trapezoid_volume(g))
    assert mass == pytest.approx(exact, rel=1e-12)
    assert exact == pytest.approx(np.prod(hi - lo) * np.mean(
        G.interp(g, rng.uniform(lo, hi, (200000, d)))), rel=2e-2)   # Monte Carlo sanity
    y, w = G.samples(g)
    assert w.sum() == pytest.approx(1.0, rel=1e-14)
    np.testing.assert_allclose(w, (u.ravel() + rho) * G.trapezoid_volume(g) / exact, rtol=1e-12)


def test_samples_drop_zero_nodes_in_node_order():
    rng = np.random.default_rng(18)
    n = (6, 5)
    lo, hi = np.array([-1.0, 0.5]), np.array([3.0, 2.5])
    u = _grid_u(n, rng, zero_frac=0.4)
    y, w = G.samples(G.Grid(u, lo, hi, 0.0))
    keep = [(j0, j1) for j1 in range(n[1]) for j0 in range(n[0]) if u[j1, j0] > 0]
    assert y.shape[0] == len(keep) == w.shape[0]
    for k, (j0, j1) in enumerate(keep):
        np.testing.assert_allclose(y[k], [lo[0] + j0 * 4.0 / 5, 0.5 + j1 * 2.0 / 4], atol=1e-14)
    assert np.all(w > 0)
