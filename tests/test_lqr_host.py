"""ct_lqr_track (host FP64, Sec. II-C eqs. 9-10) against the oracle's dense
least-squares and Riccati solutions; runs on the CPU (no GPU work involved)."""
import numpy as np
import pytest

import oracle


def _problem(rng, T, n, m):
    A = rng.normal(size=(T, n, n)) * 0.5
    B = rng.normal(size=(T, n, m))
    a = rng.normal(size=(T, n))
    Q = np.diag(rng.uniform(0.5, 2.0, n))
    Q[-1, -1] = 0.0
    R = np.diag(rng.uniform(0.01, 0.1, m))
    return A, B, a, Q, R


@pytest.mark.parametrize("T,n,m", [(1, 1, 1), (9, 3, 2), (60, 4, 2), (41, 6, 3), (33, 8, 8), (17, 5, 1)])
def test_lqr_matches_oracle(ct, T, n, m):
    rng = np.random.default_rng(T * 10 + n)
    A, B, a, Q, R = _problem(rng, T, n, m)
    v, z = ct.lqr_track(A, B, a, Q, R, 0.05)
    vd, zd = oracle.lqr_track_dense(A, B, a, Q, R, 0.05)
    np.testing.assert_allclose(v, vd, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(z, zd, rtol=1e-8, atol=1e-10)


def test_lqr_long_horizon_matches_riccati_oracle(ct):
    rng = np.random.default_rng(5)
    T, n, m = 20000, 3, 2
    s = rng.normal(size=(T, 3))
    u = rng.normal(size=(T, 2))
    A, B = oracle.dynamics_jac("unicycle", s, u)
    a = rng.normal(size=(T, n)) * 0.1
    Q = np.diag([1.0, 1.0, 0.0])
    R = 0.01 * np.eye(2)
    v, z = ct.lqr_track(A, B, a, Q, R, 0.01)
    vr, zr = oracle.lqr_track_riccati(A, B, a, Q, R, 0.01)
    np.testing.assert_allclose(v, vr, rtol=1e-7, atol=1e-9)


def test_lqr_rejects_bad_arguments(ct):
    from paper_2511_11514_amd import CtError
    A = np.zeros((3, 2, 2))
    B = np.zeros((3, 2, 1))
    a = np.zeros((3, 2))
    with pytest.raises(CtError):
        ct.lqr_track(A, B, a, np.eye(2), np.eye(1), -1.0)
    with pytest.raises(CtError):                  # R = 0: dt R + B'SB singular
        ct.lqr_track(A, B, a, np.eye(2), np.zeros((1, 1)), 0.1)
    v, z = ct.lqr_track(A, B, a, np.eye(2), np.eye(1), 0.1)
    assert np.all(v == 0) and np.all(z == 0)
