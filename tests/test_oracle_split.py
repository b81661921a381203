"""Pins for A_hat, D, Omega and J_tilde (paper Sec. 3)."""
import numpy as np
import scipy.sparse as sp

import oracle as O
import workloads as W


def _setup_parts(A, pattern="tridiag", gamma=1.0):
    A = O.validate_csr(A)
    m = O.max_product_matching(A)
    Dr, Dc = O.canonical_scaling(A, m)
    Abar = O.permute_scale(A, m, Dr, Dc)
    S, _, _ = O.skew_symmetrizer(Abar, pattern, gamma)
    return Abar, S, O.split_ahat(Abar, S)


def test_jtilde_skew_and_reconstruction():
    Abar, S, p = _setup_parts(W.paper_like(80, 400, seed=5).A)
    n = Abar.shape[0]
    J = O.split.jtilde_apply(p["Jup"], np.eye(n))
    np.testing.assert_array_equal(J, -J.T)
    Ah = (Abar @ S).toarray()
    Jhat = (Ah - Ah.T) / 2
    Om = np.diag(p["Omega"])
    lhs = Om @ (np.diag(p["D"]) + Jhat) @ Om
    rhs = np.diag(np.sign(p["D"])) + J
    np.testing.assert_allclose(lhs, rhs, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(p["Ahat"].toarray(), Ah, rtol=1e-14, atol=1e-15)
    assert np.array_equal(p["N"], np.flatnonzero(p["D"] < 0))


def test_config0_diagonal_close_to_one():
    Abar, S, p = _setup_parts(W.config(0).A)
    assert 0.85 < p["D"].min() and p["D"].max() < 1.1
    assert p["N"].size == 0
    assert p["Jup"].nnz == 9987 and p["Ahat"].nnz == 21909


def test_paper_like_reaches_negative_diagonal():
    """With a small diagonal weight (the paper tries gamma in {0.1, 1, 10}) the
    stand-in family reaches D_i < 0 and so the rank-r correction path."""
    found = False
    for s in range(6):
        Abar, S, p = _setup_parts(W.paper_like(200, 1200, seed=s).A, gamma=0.01)
        found |= p["N"].size > 0
    assert found


def test_skew_symmetry_ratio_triangular():
    """Table 3's off-diagonal skew-symmetry ratio is exactly 1/sqrt(2) when no
    pair (i,j),(j,i) is present, e.g. for a strictly triangular off-diagonal."""
    rng = np.random.default_rng(0)
    X = np.triu(rng.standard_normal((30, 30)), 1) + np.diag(rng.standard_normal(30))
    assert abs(O.split.skew_symmetry_ratio(X) - 1 / np.sqrt(2)) < 1e-15
    K = rng.standard_normal((30, 30))
    assert abs(O.split.skew_symmetry_ratio(K - K.T) - 1.0) < 1e-15
    assert O.split.skew_symmetry_ratio(K + K.T) < 1e-15
