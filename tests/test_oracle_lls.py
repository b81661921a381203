"""Pins for the least-squares skew-symmetrizer (paper Sec. 2, App. A)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W
from _golden import rows


def _abar(A):
    A = O.validate_csr(A)
    m = O.max_product_matching(A)
    Dr, Dc = O.canonical_scaling(A, m)
    return O.permute_scale(A, m, Dr, Dc)


def test_golden_2x2_diagonal():
    for r in rows("lls_2x2.txt"):
        a, b, g = float(r[0]), float(r[1]), float(r[2])
        s1 = float(r[3]) / float(r[4])
        s2 = float(r[5]) / float(r[6])
        Abar = sp.csr_matrix(np.array([[1.0, a], [b, 1.0]]))
        S, B, v = O.skew_symmetrizer(Abar, "diag", g)
        np.testing.assert_allclose(S.diagonal(), [s1, s2], rtol=1e-14)


def test_identity_plus_skew_gives_identity():
    """Abar = I + K with K skew: S = I solves every equation exactly."""
    rng = np.random.default_rng(3)
    n = 40
    K = sp.random(n, n, density=0.1, random_state=rng).toarray()
    K = 0.4 * (K - K.T) / max(1.0, np.abs(K - K.T).max())
    Abar = sp.csr_matrix(np.eye(n) + K)
    S, B, v = O.skew_symmetrizer(Abar, "diag", 1.0)
    np.testing.assert_allclose(S.diagonal(), 1.0, rtol=0, atol=1e-14)


def test_size_identities_diag_pattern():
    """S_d: nnz(B) = nnz(Abar), unknowns = n; rows = n + (nnz - n)/2 for a
    structurally symmetric Abar (the identities behind Table 2)."""
    for A in (W.config(0).A, W.paper_like(300, 1500, seed=1).A):
        Abar = _abar(A)
        n = Abar.shape[0]
        B, v, _, _ = O.build_lls(Abar, O.s_pattern(Abar, "diag"), 1.0)
        assert B.nnz == Abar.nnz
        assert B.shape[1] == n
        P = sp.csr_matrix((np.ones(Abar.nnz), Abar.indices, Abar.indptr), shape=Abar.shape)
        if (P != P.T).nnz == 0:
            assert B.shape[0] == n + (Abar.nnz - n) // 2


def test_size_identities_tridiag_and_config0():
    w = W.config(0)
    Abar = _abar(w.A)
    n = Abar.shape[0]
    B, v, _, _ = O.build_lls(Abar, O.s_pattern(Abar, "tridiag"), 1.0)
    assert B.shape == (12012, 6073) and B.nnz == 29829
    assert B.shape[1] == 3 * n - 2
    B2, _, _, _ = O.build_lls(Abar, O.s_pattern(Abar, "abar"), 1.0)
    assert B2.shape == (13727, 9945) and B2.nnz == 49013


@pytest.mark.parametrize("pattern", ["diag", "tridiag", "abar"])
def test_B_assembly_matches_closed_form_gradient(pattern):
    """B^T (B s - v) equals the closed-form half-gradient pattern(S) o (Abar^T G)
    for an arbitrary S: pins every entry of the entry-by-entry assembly."""
    rng = np.random.default_rng(7)
    Abar = _abar(W.paper_like(60, 300, seed=2).A)
    Spat = O.s_pattern(Abar, pattern)
    B, v, ur, uc = O.build_lls(Abar, Spat, 2.5)
    s = rng.standard_normal(B.shape[1])
    S = sp.csr_matrix((s, (ur, uc)), shape=Abar.shape)
    lhs = B.T @ (B @ s - v)
    grad = O.lls_gradient(Abar, S, 2.5)
    gd = grad.toarray()[ur, uc]
    np.testing.assert_allclose(lhs, gd, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("pattern", ["diag", "tridiag", "abar"])
def test_lls_kkt_and_dense(pattern):
    """The solution is stationary (KKT) and equals dense min-norm lstsq."""
    Abar = _abar(W.paper_like(120, 500, seed=4).A)
    S, B, v = O.skew_symmetrizer(Abar, pattern, 1.0)
    s = O.solve_lls(B, v, dense_limit=0)          # LSQR path
    sd = O.solve_lls(B, v, dense_limit=10 ** 9)   # dense path
    np.testing.assert_allclose(s, sd, rtol=1e-9, atol=1e-11)
    r = B @ sd - v
    kkt = np.linalg.norm(B.T @ r) / (sp.linalg.norm(B) * max(np.linalg.norm(r), 1e-300))
    assert kkt <= 1e-12
    g = O.lls_gradient(Abar, S, 1.0)
    assert np.abs(g.data).max() <= 1e-12 * max(1.0, sp.linalg.norm(B) ** 2)


def test_config0_lsqr_solution_is_stationary():
    Abar = _abar(W.config(0).A)
    S, B, v = O.skew_symmetrizer(Abar, "tridiag", 1.0)
    g = O.lls_gradient(Abar, S, 1.0)
    assert np.abs(g.data).max() <= 1e-13
