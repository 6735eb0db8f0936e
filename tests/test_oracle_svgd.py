"""Pins of the FP64 Stein-flow oracle (Sec. II-B, eq. 4): mixture density
against scipy, the score against the single-Gaussian closed form and central
differences, the median rule against numpy/scipy, and closed forms of eq. 4."""
import numpy as np
import pytest
from scipy.spatial.distance import pdist
from scipy.stats import multivariate_normal

import oracle
import workloads as W


def _gmm(rng, K, d, floor=0.0):
    return W.gmm_params(rng, K, d, 0.03, 0.12, anisotropic=True, floor=floor)


@pytest.mark.parametrize("floor", [0.0, 0.1])
def test_mixture_logpdf_matches_scipy(floor):
    rng = np.random.default_rng(20)
    g = _gmm(rng, 4, 2, floor)
    x = rng.uniform(-0.1, 1.1, size=(50, 2))
    dens = sum(float(g.weights[k]) * multivariate_normal(g.means[k].astype(float),
               np.diag(g.sigmas[k].astype(float) ** 2)).pdf(x) for k in range(4))
    dens = (1 - floor) * dens + floor * np.all((x >= 0) & (x <= 1), axis=1)
    np.testing.assert_allclose(oracle.gmm_logpdf(x, g.weights, g.means, g.sigmas, floor),
                               np.log(dens), rtol=1e-12, atol=1e-12)


def test_single_gaussian_score_is_closed_form():
    rng = np.random.default_rng(21)
    mu = np.array([[0.4, 0.6, 0.5]])
    sg = np.array([[0.05, 0.1, 0.07]])
    x = rng.uniform(0, 1, size=(40, 3))
    s = oracle.gmm_score(x, np.array([1.0]), mu, sg)
    np.testing.assert_allclose(s, -(x - mu) / sg ** 2, rtol=1e-14, atol=1e-12)


@pytest.mark.parametrize("floor,d", [(0.0, 2), (0.1, 2), (0.0, 3)])
def test_score_matches_central_differences(floor, d):
    rng = np.random.default_rng(22 + d)
    g = _gmm(rng, 5, d, floor)
    x = rng.uniform(0.05, 0.95, size=(30, d))
    s = oracle.gmm_score(x, g.weights, g.means, g.sigmas, floor)
    h = 1e-6
    for k in range(d):
        e = np.zeros(d)
        e[k] = h
        fd = (oracle.gmm_logpdf(x + e, g.weights, g.means, g.sigmas, floor)
              - oracle.gmm_logpdf(x - e, g.weights, g.means, g.sigmas, floor)) / (2 * h)
        np.testing.assert_allclose(s[:, k], fd, rtol=1e-5, atol=1e-3)


@pytest.mark.parametrize("n", [2, 3, 10, 11, 200])
def test_median_bandwidth(n):
    rng = np.random.default_rng(23 + n)
    x = rng.uniform(size=(n, 2))
    med = np.median(pdist(x))
    assert abs(oracle.median_bandwidth(x) - med * med / np.log(n)) < 1e-14
    npair = n * (n - 1) // 2
    lt, _ = oracle.pair_count(x, med * med * (1 - 1e-12))
    _, le = oracle.pair_count(x, med * med * (1 + 1e-12))
    assert lt <= npair // 2 and le >= (npair + 1) // 2
    assert oracle.median_bandwidth(x[:1]) == 1.0


@pytest.mark.parametrize("shape", [(4, 4), (3, 3, 2)])
def test_pair_count_on_lattice_ties_matches_brute_force(shape):
    """Integer lattice points tie exactly at every squared distance they share,
    so the strict and non-strict counts differ there; both against an explicit
    double loop over the pairs i < j."""
    x = np.array(list(np.ndindex(*shape)), dtype=np.float64)
    n = len(x)
    d2 = [float(((x[i] - x[j]) ** 2).sum()) for i in range(n) for j in range(i + 1, n)]
    for thr in (0.5, 1.0, 1.5, 2.0, 4.0, 5.0, 100.0):
        lt, le = oracle.pair_count(x, thr)
        assert lt == sum(v < thr for v in d2), thr
        assert le == sum(v <= thr for v in d2), thr
    assert oracle.pair_count(x, 1.0)[1] > oracle.pair_count(x, 1.0)[0]


def test_single_particle_phi_is_score():
    x = np.array([[0.3, 0.4]])
    s = np.array([[1.5, -2.0]])
    np.testing.assert_allclose(oracle.svgd_phi(x, s, 0.7), s, rtol=1e-15)


def test_two_particles_closed_form():
    x = np.array([[0.3, 0.4], [0.5, 0.45]])
    s = np.array([[1.5, -2.0], [0.25, 3.0]])
    h = 0.05
    k = np.exp(-np.sum((x[0] - x[1]) ** 2) / h)
    phi0 = 0.5 * (s[0] + k * s[1] + (2 / h) * (x[0] - x[1]) * k)
    phi1 = 0.5 * (s[1] + k * s[0] + (2 / h) * (x[1] - x[0]) * k)
    np.testing.assert_allclose(oracle.svgd_phi(x, s, h), np.stack([phi0, phi1]), rtol=1e-14)


def test_repulsion_is_antisymmetric_and_small_h_limit():
    rng = np.random.default_rng(24)
    x = rng.uniform(size=(40, 3))
    s = rng.normal(size=(40, 3))
    rep = oracle.svgd_phi(x, np.zeros_like(x), 0.2)
    assert np.abs(rep.sum(0)).max() < 1e-13
    # as h -> 0 only the self term survives: phi_i -> score_i / n
    np.testing.assert_allclose(oracle.svgd_phi(x, s, 1e-9), s / 40, rtol=1e-12)
    # attraction part is linear in the score
    full = oracle.svgd_phi(x, s, 0.2)
    att = oracle.svgd_phi(x, s, 0.2) - rep
    np.testing.assert_allclose(oracle.svgd_phi(x, 2 * s, 0.2), rep + 2 * att, atol=1e-13)
    assert np.isfinite(full).all()


@pytest.mark.parametrize("case", ["uniform2", "uniform3", "lattice", "pair", "triple", "same"])
def test_median_by_counting_equals_sorted_median(case):
    """The pair-counting median (used where the distances cannot all be listed)
    returns exactly the bandwidth of numpy.median over scipy's pdist, including
    lattice points whose distances tie (even and odd pair counts), two and three
    points, and coincident points (h = 1)."""
    rng = np.random.default_rng(91)
    x = {"uniform2": rng.uniform(size=(57, 2)), "uniform3": rng.uniform(size=(40, 3)),
         "lattice": np.array(list(np.ndindex(5, 4)), dtype=np.float64) * 0.25,
         "pair": rng.uniform(size=(2, 2)), "triple": rng.uniform(size=(3, 3)),
         "same": np.ones((6, 2))}[case]
    n = len(x)
    med = float(np.median(pdist(x)))
    ref = 1.0 if med == 0.0 else med * med / np.log(n)
    got = oracle.median_bandwidth_by_counting(x)
    assert got == oracle.median_bandwidth(x)
    assert abs(got - ref) <= 1e-15 * ref
