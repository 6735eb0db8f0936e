"""Pins of the FP64 Sinkhorn oracle against facts fixed by the mathematics
(Sec. II-B, eqs. 5-7): library log-sum-exp, the textbook Sinkhorn-Knopp matrix
scaling, closed forms (translation, identical clouds, single point),
brute-force optimal assignment bounds, invariances, and finite differences."""
import itertools

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment
from scipy.special import logsumexp

import oracle
from oracle.sinkhorn import lse_update



def _cloud(rng, n, d, lo=0.0, hi=1.0):
    return rng.uniform(lo, hi, size=(n, d))


def test_lse_matches_scipy_logsumexp():
    rng = np.random.default_rng(1)
    for d in (2, 3):
        xq, xk = _cloud(rng, 17, d), _cloud(rng, 33, d)
        lw = np.log(rng.uniform(0.1, 1.0, 33))
        pot = rng.normal(size=33) * 0.01
        eps = 0.003
        out, bary = lse_update(xq, xk, lw, pot, eps, want_bary=True)
        C = ((xq[:, None, :] - xk[None, :, :]) ** 2).sum(-1)
        Z = lw[None, :] + (pot[None, :] - C) / eps
        ref = -eps * logsumexp(Z, axis=1)
        np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-15)
        P = np.exp(Z - logsumexp(Z, axis=1, keepdims=True))
        ref_b = np.einsum("ij,ijk->ik", P, xk[None, :, :] - xq[:, None, :])
        np.testing.assert_allclose(bary, ref_b, rtol=1e-11, atol=1e-14)


def _converge(x, y, w=None, eps=0.1, debias=True, tol=1e-12, chunk=200, max_iter=200000):
    """Run the oracle from warm starts until the column residual is below tol."""
    r = oracle.sinkhorn(x, y, w, eps=eps, iters=chunk, debias=debias)
    done = chunk
    while r.resid > tol and done < max_iter:
        init = (r.f, r.g, r.p if r.p is not None else np.zeros(len(x)),
                r.q if r.q is not None else np.zeros(len(y)))
        r = oracle.sinkhorn(x, y, w, eps=eps, iters=chunk, debias=debias, init=init)
        done += chunk
    return r


def test_marginal_residual_below_1e9_and_matches_textbook_scaling():
    """Converged log-domain iterates reproduce Cuturi's dense Sinkhorn-Knopp
    scaling: same plan, potentials f = eps log(u/a), g = eps log(v/b), and the
    dual value equals the primal objective <pi,C> + eps KL(pi | a x b)."""
    rng = np.random.default_rng(2)
    T, M, d, eps = 7, 11, 2, 0.05
    x, y = _cloud(rng, T, d), _cloud(rng, M, d)
    w = rng.uniform(0.5, 2.0, M)
    r = _converge(x, y, w, eps=eps, tol=1e-13)
    assert r.resid < 1e-9
    a = np.full(T, 1.0 / T)
    b = w / w.sum()
    C = ((x[:, None] - y[None]) ** 2).sum(-1)
    K = np.exp(-C / eps)
    u, v = np.ones(T), np.ones(M)
    for _ in range(20000):
        u = a / (K @ v)
        v = b / (K.T @ u)
    P = u[:, None] * K * v[None, :]
    assert np.abs(P.sum(0) - b).sum() < 1e-12
    fk, gk = eps * np.log(u / a), eps * np.log(v / b)
    f1, g1 = oracle.gauge_fix(r.f_plus, r.g, a, b)
    f2, g2 = oracle.gauge_fix(fk, gk, a, b)
    np.testing.assert_allclose(f1, f2, atol=1e-10)
    np.testing.assert_allclose(g1, g2, atol=1e-10)
    primal = (P * C).sum() + eps * (P * np.log(P / (a[:, None] * b[None, :]))).sum()
    assert abs(r.ot_ab - primal) < 1e-10
    # the plan of the oracle's row-exact pair is the textbook plan
    Po = a[:, None] * b[None, :] * np.exp((r.f_plus[:, None] + r.g[None, :] - C) / eps)
    np.testing.assert_allclose(Po, P, atol=1e-11)
    # barycentric offsets: D^y = sum_j P_ij/a_i (y_j - x_i)
    Dy = (P / a[:, None]) @ y - x
    np.testing.assert_allclose(r.bary_y, Dy, atol=1e-10)


@pytest.mark.parametrize("d", [2, 3])
def test_translation_closed_form(d):
    """y_j = x_j + c with equal weights: S = |c|^2, dS/dx_i = -2 a_i c, and the
    weight gradient along any zero-sum direction delta is sum_j delta_j 2c.x_j / sum(w)."""
    rng = np.random.default_rng(3 + d)
    n = 9
    x = _cloud(rng, n, d, 0.2, 0.8)
    c = rng.normal(size=d) * 0.1
    y = x + c
    r = _converge(x, y, eps=0.1, tol=1e-13)
    assert abs(r.value - c @ c) < 1e-10
    np.testing.assert_allclose(r.grad_x, np.tile(-2.0 / n * c, (n, 1)), atol=1e-10)
    delta = rng.normal(size=n)
    delta -= delta.mean()
    expect = np.sum(delta * (2.0 * (x @ c))) / n
    assert abs(delta @ r.grad_w - expect) < 1e-10


def test_identical_clouds_give_zero():
    rng = np.random.default_rng(5)
    x = _cloud(rng, 8, 2)
    r = _converge(x, x.copy(), eps=0.1, tol=1e-13)
    assert abs(r.value) < 1e-11
    assert np.abs(r.grad_x).max() < 1e-11
    assert np.abs(r.grad_w).max() < 1e-11
    # without debiasing the entropic blur leaves a nonzero gradient and value
    r2 = _converge(x, x.copy(), eps=0.1, debias=False, tol=1e-13)
    assert r2.value > 1e-3
    assert np.abs(r2.grad_x).max() > 1e-4


@pytest.mark.parametrize("eps", [1e-3, 0.05, 1.0])
def test_single_point(eps):
    x = np.array([[0.2, 0.7]])
    y = np.array([[0.5, 0.1]])
    r = oracle.sinkhorn(x, y, eps=eps, iters=3)
    diff = x[0] - y[0]
    assert abs(r.value - diff @ diff) < 1e-14
    np.testing.assert_allclose(r.grad_x[0], 2.0 * diff, atol=1e-14)


@pytest.mark.parametrize("n,seed", [(4, 10), (6, 11), (8, 12)])
def test_brute_force_assignment_bounds(n, seed):
    """W = (1/n) min over permutations of sum |x_i - y_s(i)|^2, enumerated, and by
    scipy's assignment solver.  With the relative-entropy regulariser
    W <= OT_eps(a,b) <= W + eps ln n, OT_eps(a,a), OT_eps(b,b) in [0, eps ln n],
    so |S - W| <= eps ln n."""
    rng = np.random.default_rng(seed)
    x, y = _cloud(rng, n, 2), _cloud(rng, n, 2)
    C = ((x[:, None] - y[None]) ** 2).sum(-1)
    best = min(sum(C[i, s[i]] for i in range(n)) for s in itertools.permutations(range(n))) / n
    ri, ci = linear_sum_assignment(C)
    assert abs(best - C[ri, ci].sum() / n) < 1e-14
    for eps in (0.05, 0.01, 0.004):
        r = _converge(x, y, eps=eps, tol=1e-10, chunk=500)
        bound = eps * np.log(n)
        assert best - 1e-12 <= r.ot_ab <= best + bound + 1e-12
        assert -1e-12 <= 0.5 * r.ot_aa <= bound + 1e-12
        assert -1e-12 <= 0.5 * r.ot_bb <= bound + 1e-12
        assert abs(r.value - best) <= bound + 1e-12


def test_small_eps_gradient_tends_to_assignment():
    """As eps -> 0 with a unique optimal assignment s, dS/dx_i -> 2 a_i (x_i - y_s(i))."""
    rng = np.random.default_rng(13)
    n = 4
    x, y = _cloud(rng, n, 2), _cloud(rng, n, 2)
    C = ((x[:, None] - y[None]) ** 2).sum(-1)
    _, sig = linear_sum_assignment(C)
    r = _converge(x, y, eps=5e-4, tol=1e-9, chunk=2000, max_iter=400000)
    expect = 2.0 / n * (x - y[sig])
    np.testing.assert_allclose(r.grad_x, expect, atol=2e-3 * np.abs(expect).max())


def test_invariances():
    rng = np.random.default_rng(14)
    T, M = 6, 9
    x, y = _cloud(rng, T, 2), _cloud(rng, M, 2)
    w = rng.uniform(0.5, 2.0, M)
    eps = 0.05
    r = _converge(x, y, w, eps=eps, tol=1e-13)
    assert r.value >= 0.0
    # weight gradient is centred: sum_j w_j dS/dw_j = 0 (S is 0-homogeneous in w)
    assert abs(w @ r.grad_w) < 1e-14
    # permutation equivariance
    pi, pj = rng.permutation(T), rng.permutation(M)
    rp = _converge(x[pi], y[pj], w[pj], eps=eps, tol=1e-13)
    np.testing.assert_allclose(rp.grad_x, r.grad_x[pi], atol=1e-12)
    np.testing.assert_allclose(rp.grad_w, r.grad_w[pj], atol=1e-12)
    assert abs(rp.value - r.value) < 1e-12
    # scaling: x,y -> lam x, lam y and eps -> lam^2 eps gives S -> lam^2 S, grad -> lam grad
    lam = 1.7
    rs = _converge(lam * x, lam * y, w, eps=lam ** 2 * eps, tol=1e-13)
    assert abs(rs.value - lam ** 2 * r.value) < 1e-12
    np.testing.assert_allclose(rs.grad_x, lam * r.grad_x, atol=1e-12)
    # rescaling all weights changes nothing but the weight gradient's scale
    r3 = _converge(x, y, 3.0 * w, eps=eps, tol=1e-13)
    np.testing.assert_allclose(r3.grad_x, r.grad_x, atol=1e-13)
    np.testing.assert_allclose(r3.grad_w, r.grad_w / 3.0, atol=1e-13)


def _dual(f, g, a, b, C, eps):
    """Entropic dual objective of eq. 5 (relative entropy to a x b) at any pair
    (f, g): <a,f> + <b,g> - eps sum_ij a_i b_j (exp((f_i + g_j - C_ij)/eps) - 1)."""
    E = np.exp((f[:, None] + g[None, :] - C) / eps)
    return a @ f + b @ g - eps * (a @ E @ b - 1.0)


@pytest.mark.parametrize("iters", [1, 3, 8])
def test_value_terms_are_dual_objectives_before_convergence(iters):
    """Away from convergence each OT term of the value is the full dual objective
    at the pair it is read from (the exponential term vanishes because the first
    potential is row-exact for the second), and by weak duality it stays below
    the converged term."""
    rng = np.random.default_rng(16)
    T, M, eps = 7, 10, 0.05
    x, y = _cloud(rng, T, 2), _cloud(rng, M, 2)
    w = rng.uniform(0.5, 2.0, M)
    a, b = np.full(T, 1.0 / T), w / w.sum()
    Cxy = ((x[:, None] - y[None]) ** 2).sum(-1)
    Cxx = ((x[:, None] - x[None]) ** 2).sum(-1)
    Cyy = ((y[:, None] - y[None]) ** 2).sum(-1)
    r = oracle.sinkhorn(x, y, w, eps=eps, iters=iters)
    assert r.resid > 1e-6                      # genuinely not converged
    assert abs(np.max(np.abs(r.p_plus - r.p))) > 1e-6
    assert abs(r.ot_ab - _dual(r.f_plus, r.g, a, b, Cxy, eps)) < 1e-13
    assert abs(r.ot_aa - _dual(r.p_plus, r.p, a, a, Cxx, eps)) < 1e-13
    assert abs(r.ot_bb - _dual(r.q_plus, r.q, b, b, Cyy, eps)) < 1e-13
    c = _converge(x, y, w, eps=eps, tol=1e-13)
    assert r.ot_ab <= c.ot_ab + 1e-13
    assert r.ot_aa <= c.ot_aa + 1e-13
    assert r.ot_bb <= c.ot_bb + 1e-13


def _value_at(x, y, w, eps, init):
    r = oracle.sinkhorn(x, y, w, eps=eps, iters=50, init=init)
    while r.resid > 1e-14:
        r = oracle.sinkhorn(x, y, w, eps=eps, iters=50, init=(r.f, r.g, r.p, r.q))
    return r.value


@pytest.mark.parametrize("debias", [True, False])
def test_gradients_match_central_differences(debias):
    """Envelope-theorem gradients (w.r.t. points and weights) against central
    differences of the converged FP64 objective (eq. 7)."""
    rng = np.random.default_rng(15)
    T, M, eps, h = 6, 9, 0.05, 1e-4
    x, y = _cloud(rng, T, 2), _cloud(rng, M, 2)
    w = rng.uniform(0.5, 2.0, M)
    r = _converge(x, y, w, eps=eps, debias=debias, tol=1e-14)
    init = (r.f, r.g, r.p if r.p is not None else np.zeros(T),
            r.q if r.q is not None else np.zeros(M))

    def val(xx, ww):
        rr = oracle.sinkhorn(xx, y, ww, eps=eps, iters=50, debias=debias, init=init)
        while rr.resid > 1e-14:
            rr = oracle.sinkhorn(xx, y, ww, eps=eps, iters=50, debias=debias,
                                 init=(rr.f, rr.g, rr.p if rr.p is not None else np.zeros(T),
                                       rr.q if rr.q is not None else np.zeros(M)))
        return rr.value

    for (i, k) in [(0, 0), (2, 1), (5, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        fd = (val(xp, w) - val(xm, w)) / (2 * h)
        assert abs(fd - r.grad_x[i, k]) < 1e-8 * max(1.0, abs(fd)), (i, k, fd, r.grad_x[i, k])
    for j in [0, 4, 8]:
        wp, wm = w.copy(), w.copy()
        wp[j] += h
        wm[j] -= h
        fd = (val(x, wp) - val(x, wm)) / (2 * h)
        assert abs(fd - r.grad_w[j]) < 1e-8 * max(1.0, abs(fd)), (j, fd, r.grad_w[j])
