"""Pins of the oracle's gradient of a solve (value_gradient, solve_adjoint).

Closed forms and finite differences: the directional derivative of
L(v, b) = ||A(v)^-1 b - x_t||^2 by central differences of dense solves pins
the formula dL/da_ij = -lambda_i x_j and dL/db = lambda; the same check
through the oracle's own two-level solve (tight tolerance) pins the composed
path.  Plausible mistakes (transposed indices, dropped sign) fail it."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W


def _problem(m=12, seed=5):
    w = W.implicit_euler_grid(m=m, h=0.1, cfg=0)
    A = sp.csr_matrix(w.A)
    rng = np.random.default_rng(seed)
    xt = rng.standard_normal(A.shape[0])
    return A, w.b.copy(), xt, rng


def _with_values(A, v):
    return sp.csr_matrix((v, A.indices, A.indptr), shape=A.shape)


def _loss_dense(A, b, xt):
    x = np.linalg.solve(A.toarray(), b)
    return float(np.sum((x - xt) ** 2)), x


def test_value_gradient_matches_dense_finite_differences():
    A, b, xt, rng = _problem()
    L0, x = _loss_dense(A, b, xt)
    lam = np.linalg.solve(A.toarray().T, 2.0 * (x - xt))
    g = O.value_gradient(A, lam, x)
    v = A.data.copy()
    for _ in range(4):
        d = rng.standard_normal(v.size)
        eps = 1e-6 * np.linalg.norm(v) / np.linalg.norm(d)
        Lp, _ = _loss_dense(_with_values(A, v + eps * d), b, xt)
        Lm, _ = _loss_dense(_with_values(A, v - eps * d), b, xt)
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - g @ d) <= 1e-6 * max(1.0, abs(fd)), (fd, g @ d)
    # dL/db = lambda
    d = rng.standard_normal(b.size)
    eps = 1e-6 * np.linalg.norm(b) / np.linalg.norm(d)
    fd = (_loss_dense(A, b + eps * d, xt)[0] - _loss_dense(A, b - eps * d, xt)[0]) / (2 * eps)
    assert abs(fd - lam @ d) <= 1e-6 * max(1.0, abs(fd))


def test_value_gradient_catches_transposed_or_unsigned_formula():
    A, b, xt, rng = _problem()
    _, x = _loss_dense(A, b, xt)
    lam = np.linalg.solve(A.toarray().T, 2.0 * (x - xt))
    g = O.value_gradient(A, lam, x)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    wrong_t = -lam[A.indices] * x[rows]      # indices swapped
    wrong_s = lam[rows] * x[A.indices]       # sign dropped
    d = rng.standard_normal(A.nnz)
    v = A.data
    eps = 1e-6 * np.linalg.norm(v) / np.linalg.norm(d)
    fd = (_loss_dense(_with_values(A, v + eps * d), b, xt)[0]
          - _loss_dense(_with_values(A, v - eps * d), b, xt)[0]) / (2 * eps)
    assert abs(fd - g @ d) <= 1e-6 * max(1.0, abs(fd))
    assert abs(fd - wrong_t @ d) > 1e-3 * abs(fd)
    assert abs(fd - wrong_s @ d) > 1e-3 * abs(fd)


def test_two_level_gradient_matches_finite_differences():
    A, b, xt, rng = _problem(m=10)
    opts = O.SolveOptions(tol=1e-13)
    so = O.SetupOptions(k=6, s_pattern="tridiag")

    def loss(Am, bm):
        x, info = O.solve(O.setup(Am, so), bm, opts)
        assert info["converged"]
        return float(np.sum((x - xt) ** 2)), x

    st = O.setup(A, so)
    x, _ = O.solve(st, b, opts)
    lam, info = O.solve_adjoint(st, 2.0 * (x - xt), opts)
    assert info["converged"]
    lam_dense = np.linalg.solve(A.toarray().T, 2.0 * (x - xt))
    assert np.linalg.norm(lam - lam_dense) <= 1e-10 * np.linalg.norm(lam_dense)
    g = O.value_gradient(A, lam, x)
    v = A.data.copy()
    for _ in range(3):
        d = rng.standard_normal(v.size)
        eps = 1e-5 * np.linalg.norm(v) / np.linalg.norm(d)
        fd = (loss(_with_values(A, v + eps * d), b)[0] - loss(_with_values(A, v - eps * d), b)[0]) / (2 * eps)
        assert abs(fd - g @ d) <= 1e-5 * max(1.0, abs(fd)), (fd, g @ d)
