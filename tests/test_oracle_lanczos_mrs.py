"""Pins for the skew-Lanczos process (Fig. 2) and the mrs solver (App. B)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from oracle.lanczos import skew_tridiagonal, splitmix64_raw
from _golden import GOLDEN, rows


def _skew(n, density, seed):
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=rng, data_rvs=rng.standard_normal)
    U = sp.csr_matrix(sp.triu(M - M.T, 1))
    return U


def test_splitmix64_reference_outputs():
    ref = [int(r[0], 16) for r in rows("splitmix64_seed0.txt")]
    got = [int(v) for v in splitmix64_raw(0, 3)]
    assert got == ref
    u = O.splitmix64_uniform(0, 3)
    assert np.all((u >= -1) & (u < 1))
    assert u[0] == (ref[0] >> 11) * 2.0 ** -52 - 1.0


@pytest.mark.parametrize("k", [2, 5, 8])
def test_lanczos_projection_and_spectrum(k):
    U = _skew(300, 0.03, 1)
    J = lambda v: U @ v - U.T @ v
    Q, a = O.skew_lanczos(J, O.start_vector(7, 300), k)
    assert Q.shape == (300, k) and a.size == k - 1
    Sk = skew_tridiagonal(a)
    Jd = J(np.eye(300))
    np.testing.assert_allclose(Q.T @ Jd @ Q, Sk, atol=1e-13)
    np.testing.assert_allclose(Q.T @ Q, np.eye(k), atol=1e-13)
    ritz = np.linalg.eigvals(Sk)
    assert np.abs(ritz.real).max() <= 1e-14 * max(1.0, np.abs(ritz).max())
    Jbar = Jd - Q @ Sk @ Q.T
    np.testing.assert_allclose(Jbar, -Jbar.T, atol=1e-15)


def test_lanczos_extreme_ritz_values_converge():
    U = _skew(200, 0.05, 2)
    J = lambda v: U @ v - U.T @ v
    Q, a = O.skew_lanczos(J, O.start_vector(1, 200), 30)
    ritz = np.abs(np.linalg.eigvals(skew_tridiagonal(a))).max()
    lam = np.abs(np.linalg.eigvals(J(np.eye(200)))).max()
    assert abs(ritz - lam) <= 1e-6 * lam


def test_lanczos_breakdown_symmetric_input():
    """J = 0 (a symmetric input after scaling): alpha_1 = 0, one vector."""
    Q, a = O.skew_lanczos(lambda v: 0 * v, O.start_vector(0, 10), 8)
    assert Q.shape == (10, 1) and a.size == 0


def test_lanczos_golden_2x2():
    t = 3.0
    J = lambda v: np.array([[0, t], [-t, 0]]) @ v
    Q, a = O.skew_lanczos(J, np.array([1.0, 0.0]), 2)
    np.testing.assert_allclose(a, [3.0])
    np.testing.assert_allclose(Q, [[1, 0], [0, 1]], atol=1e-16)


def test_mrs_golden_2x2():
    for r in rows("mrs_2x2.txt"):
        al, t, b1, b2, x1, x2 = map(float, r)
        K = np.array([[0, t], [-t, 0]])
        x, its, h = O.mrs(al, lambda v: K @ v, np.array([b1, b2]), 10, 1e-15)
        np.testing.assert_allclose(x, [x1, x2], rtol=1e-14)
        assert its <= 2


@pytest.mark.parametrize("alpha", [1.0, 0.3, 2.0])
def test_mrs_residual_estimate_monotone_and_exact(alpha):
    U = _skew(120, 0.05, 3)
    K = lambda v: U @ v - U.T @ v
    rng = np.random.default_rng(4)
    b = rng.standard_normal(120)
    x, its, hist = O.mrs(alpha, K, b, 400, 1e-14)
    h = hist[:, 0]
    assert np.all(np.diff(h) <= 1e-15)
    Kd = K(np.eye(120))
    A = alpha * np.eye(120) + Kd
    xd = np.linalg.solve(A, b)
    np.testing.assert_allclose(x, xd, rtol=1e-12 * np.linalg.cond(A), atol=1e-12)
    # the estimate equals the true residual in early steps
    for stop in (1, 2, 5, 10):
        xs, _, hs = O.mrs(alpha, K, b, stop, 0.0, fixed_steps=stop)
        true = np.linalg.norm(b - A @ xs) / np.linalg.norm(b)
        assert abs(true - hs[-1, 0]) <= 1e-12


@pytest.mark.parametrize("n", [3, 6, 10])
def test_mrs_terminates_within_n_steps(n):
    rng = np.random.default_rng(n)
    Kd = rng.standard_normal((n, n))
    Kd = Kd - Kd.T
    b = rng.standard_normal(n)
    x, its, h = O.mrs(1.0, lambda v: Kd @ v, b, n, 0.0, fixed_steps=n)
    assert np.linalg.norm(b - (np.eye(n) + Kd) @ x) / np.linalg.norm(b) <= 1e-13


def test_mrs_zero_operator_one_step():
    b = np.arange(1.0, 6.0)
    x, its, h = O.mrs(2.0, lambda v: 0 * v, b, 10, 1e-12)
    assert its == 1
    np.testing.assert_allclose(x, b / 2.0, rtol=1e-15)


def test_mrs_simultaneous_equals_separate():
    U = _skew(90, 0.06, 5)
    K = lambda v: U @ v - U.T @ v
    B = np.random.default_rng(6).standard_normal((90, 3))
    B[:, 1] *= 100.0
    X, its, _ = O.mrs(1.0, K, B, 25, 0.0, fixed_steps=25)
    for j in range(3):
        xj, _, _ = O.mrs(1.0, K, B[:, j], 25, 0.0, fixed_steps=25)
        np.testing.assert_array_equal(X[:, j], xj)


def test_mrs_zero_column_and_stop_rule():
    U = _skew(60, 0.1, 8)
    K = lambda v: U @ v - U.T @ v
    B = np.random.default_rng(9).standard_normal((60, 3))
    B[:, 2] = 0
    X, its, hist = O.mrs(1.0, K, B, 500, 1e-10)
    assert np.all(X[:, 2] == 0)
    assert hist[-1].max() < 1e-10 and hist[-2].max() >= 1e-10


def test_mrs_fp32_storage_reading():
    """storage=np.float32 stores every basis vector as an FP32 value: with
    float64 storage it is the plain method bit for bit; with float32 on a
    well-conditioned operator it stays within FP32 rounding of the FP64
    result and keeps the minimal-residual decrease."""
    import oracle as O
    rng = np.random.default_rng(3)
    n = 300
    K = rng.standard_normal((n, n)) * 0.05
    K = K - K.T
    b = rng.standard_normal(n)
    op = lambda v: K @ v
    x64, its, h64 = O.mrs(1.0, op, b, 40, 0.0, fixed_steps=40)
    xs, _, hs = O.mrs(1.0, op, b, 40, 0.0, fixed_steps=40, storage=np.float64)
    assert np.array_equal(x64, xs) and np.array_equal(h64, hs)
    seen = []
    op_rec = lambda v: (seen.append(v.copy()), K @ v)[1]
    x32, _, h32 = O.mrs(1.0, op_rec, b, 40, 0.0, fixed_steps=40, storage=np.float32)
    for v in seen:  # every vector the operator saw is FP32-valued
        assert np.array_equal(v, v.astype(np.float32).astype(np.float64))
    assert np.linalg.norm(x32 - x64) <= 1e-5 * np.linalg.norm(x64)
    assert np.all(np.diff(h32[:, 0]) <= 1e-12)
