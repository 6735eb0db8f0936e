"""GPU parity of ct_svgd_grad against the FP64 oracle (Sec. II-B, eq. 4): the
mixture score, the exact median bandwidth and the Stein flow phi.
Tolerance 1e-5 norm-wise relative error (float32 path vs float64 oracle)."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def _gpu(ct, x, g, h=None):
    dev = torch.device("cuda")
    phi, hu, sc = ct.svgd_grad(torch.as_tensor(x, device=dev), ct.GMM.from_numpy(g, dev), h,
                               return_score=True)
    torch.cuda.synchronize()
    return phi.cpu().numpy(), float(hu.item()), sc.cpu().numpy()


def _oracle(x, g, h=None):
    sc = oracle.gmm_score(x, g.weights, g.means, g.sigmas, g.floor)
    hh = oracle.median_bandwidth(x) if h is None else h
    return oracle.svgd_phi(x, sc, hh), hh, sc


@pytest.mark.parametrize("cfg,T", [("grad_2d", 1000), ("grad_2d", 4096), ("autograd_3d", 777),
                                   ("roofline_2d", 1531)])
def test_parity(ct, cfg, T):
    x, _y, _w, g = W.config_inputs(W.CONFIGS[cfg], T=T, M=16)
    phi, h, sc = _gpu(ct, x, g)
    rphi, rh, rsc = _oracle(x, g)
    e = dict(score=rel(sc, rsc), h=abs(h - rh) / rh, phi=rel(phi, rphi))
    print(cfg, T, " ".join(f"{k}={v:.2e}" for k, v in e.items()))
    assert e["score"] < TOL and e["h"] < 1e-6 and e["phi"] < TOL, e


def test_fixed_bandwidth_and_odd_even_pair_counts(ct):
    x, _y, _w, g = W.config_inputs(W.CONFIGS["grad_2d"], T=301, M=16)
    phi, h, _ = _gpu(ct, x, g, h=0.0123)
    rphi, _, _ = _oracle(x, g, h=0.0123)
    assert h == pytest.approx(0.0123, rel=1e-7)
    assert rel(phi, rphi) < TOL
    for T in (2, 3, 4, 5, 64, 65):        # pair counts 1, 3, 6, 10, 2016, 2080
        xs = x[:T]
        _p, hg, _s = _gpu(ct, xs, g)
        assert abs(hg - oracle.median_bandwidth(xs)) <= 1e-6 * oracle.median_bandwidth(xs)


def test_degenerate_cases(ct):
    g = W.gmm_params(np.random.default_rng(0), 1, 2, 0.05, 0.1)
    x1 = np.array([[0.3, 0.6]], np.float32)
    phi, h, sc = _gpu(ct, x1, g)
    assert h == 1.0
    np.testing.assert_allclose(phi, sc, rtol=1e-6)          # one sample: phi = score
    mu, sg = g.means[0].astype(np.float64), g.sigmas[0].astype(np.float64)
    np.testing.assert_allclose(sc[0], -(x1[0] - mu) / sg ** 2, rtol=1e-6)
    x2 = np.array([[0.3, 0.6], [0.35, 0.58]], np.float32)
    phi, h, sc = _gpu(ct, x2, g)
    rphi, rh, _ = _oracle(x2, g)
    assert abs(h - rh) / rh < 1e-6 and rel(phi, rphi) < TOL
    xc = np.repeat(x1, 7, axis=0)                            # coincident samples: h = 1
    phi, h, sc = _gpu(ct, xc, g)
    assert h == 1.0
    np.testing.assert_allclose(phi, sc, rtol=1e-6)


@pytest.mark.parametrize("cfg,T", [("grad_2d", 20000), ("autograd_3d", 17000), ("grad_2d", 11000),
                                   ("roofline_2d", 92681), ("autograd_3d", 30001),
                                   ("roofline_2d", 24576), ("roofline_2d", 24575)])
def test_bracketed_median_is_exact(ct, cfg, T):
    # large T: the median comes from a sampled bracket and one pass over all pairs (over
    # every pair below T = 24576, over boxes of point groups from there on); the pairs
    # strictly below / at most the returned median must straddle the middle ranks
    x, _y, _w, g = W.config_inputs(W.CONFIGS[cfg], T=T, M=16)
    _phi, h, _sc = _gpu(ct, x, g)
    med2 = h * np.log(T)
    npair = T * (T - 1) // 2
    lt, _ = oracle.pair_count(x, med2 * (1 - 2e-6))
    _, le = oracle.pair_count(x, med2 * (1 + 2e-6))
    assert lt <= npair // 2 and le >= (npair + 1) // 2, (lt, le, npair)


@pytest.mark.parametrize("d,T,spread", [(2, 30011, 0.01), (3, 12289, 0.02), (2, 24577, 0.2)])
def test_box_settled_bracket_is_exact(ct, d, T, spread):
    """Clustered samples (nine tight clusters: after the points are put in cell
    order, the boxes of their groups of 64 settle most pairs of groups without
    evaluating a pair), T not a multiple of 64, coordinates near 100: the pairs
    strictly below / at most the returned median still straddle the middle ranks
    (oracle pair counts).  The wide spread leaves more pairs of groups to the
    pair-by-pair pass."""
    rng = np.random.default_rng(T)
    ctr = rng.uniform(0.0, 1.0, (9, d))
    x = (100.0 + ctr[rng.integers(0, 9, T)] + rng.normal(0.0, spread, (T, d))).astype(np.float32)
    g = W.gmm_params(np.random.default_rng(1), 2, d, 0.05, 0.1)
    g.means[:] += 100.0
    print(f"box-settled bracket d={d} T={T} spread={spread}", flush=True)
    _phi, h, _sc = _gpu(ct, x, g)
    med2 = h * np.log(T)
    npair = T * (T - 1) // 2
    lt, _ = oracle.pair_count(x, med2 * (1 - 2e-6))
    _, le = oracle.pair_count(x, med2 * (1 + 2e-6))
    assert lt <= npair // 2 and le >= (npair + 1) // 2, (lt, le, npair)


def test_bracket_miss_falls_back_to_all_pairs(ct):
    # two coincident clusters of 10000 points: squared distances are 0 (99 990 000
    # pairs) or 0.5 (100 000 000 pairs), so the sampled bracket spans both values,
    # its candidates overflow, and the selection reruns over all pairs.  Both middle
    # ranks fall among the cross pairs: med^2 = 0.5.
    T = 20000
    x = np.full((T, 2), 0.25, np.float32)
    x[T // 2:] = 0.75
    g = W.gmm_params(np.random.default_rng(0), 1, 2, 0.05, 0.1)
    _phi, h, _sc = _gpu(ct, x, g)
    assert h == pytest.approx(0.5 / np.log(T), rel=1e-6)


def test_far_from_coordinate_origin(ct):
    """Samples and mixture shifted far from the coordinate origin: the staging
    subtracts the samples' mean before the bandwidth scale, so phi matches the
    oracle at the same bar as near the origin (the bandwidth is a median of
    differences and does not move)."""
    x, _y, _w, g = W.config_inputs(W.CONFIGS["grad_2d"], T=1500, M=16)
    shift = np.array([250.0, -125.0])
    xs = (x.astype(np.float64) + shift).astype(np.float32)
    gs = W.GMM(g.weights, (g.means.astype(np.float64) + shift).astype(np.float32), g.sigmas,
               g.floor)
    phi, h, sc = _gpu(ct, xs, gs)
    rphi, rh, rsc = _oracle(xs, gs)
    e = dict(score=rel(sc, rsc), h=abs(h - rh) / rh, phi=rel(phi, rphi))
    assert e["score"] < TOL and e["h"] < 1e-6 and e["phi"] < TOL, e
