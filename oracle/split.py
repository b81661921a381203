"""Splitting of the preprocessed matrix (paper Sec. 3, eq. modified and the
preconditioner eqs. preconditioner / preconditioner2).

A_hat = Abar S, M_hat = (A_hat + A_hat^T)/2, J_hat = (A_hat - A_hat^T)/2.

Reading (the incomplete LDL^T of M_hat reduced to its diagonal): L_tilde = I,
D_tilde = D = diag(A_hat), so the scaled factor is |D|^(1/2) and, with
Omega = |D|^(-1/2),

    J_tilde = Omega J_hat Omega          (exactly skew-symmetric)
    M_r     = sign(D) - I                (1x1 blocks only, value -2)
    P       = sign(D) + J_tilde = Omega (D + J_hat) Omega.

J_tilde is kept as its strictly upper triangle on the structural pattern of
A_hat + A_hat^T (pattern of |Abar||S| and its transpose); the lower triangle
is implied as the negated transpose.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .preprocess import ZeroDiagonal
from .skewsym import _on_pattern, _spones


def ahat_on_pattern(Abar: sp.csr_matrix, S: sp.csr_matrix):
    """(A_hat, P): A_hat = Abar S stored on its structural pattern P (the
    pattern of |Abar||S|, explicit zeros of the product kept)."""
    P = sp.csr_matrix(_spones(Abar) @ _spones(S))
    P.sort_indices()
    return _on_pattern(sp.csr_matrix(Abar @ S), P), P


def symmetric_skew_parts(Ahat: sp.csr_matrix):
    """M_hat = (A_hat + A_hat^T)/2 and J_hat = (A_hat - A_hat^T)/2 (Sec. 3),
    both on the pattern of A_hat + A_hat^T."""
    At = sp.csr_matrix(Ahat.T)
    Mh = sp.csr_matrix((Ahat + At) / 2.0)
    Jh = sp.csr_matrix((Ahat - At) / 2.0)
    Mh.sort_indices()
    Jh.sort_indices()
    return Mh, Jh


def split_ahat(Abar: sp.csr_matrix, S: sp.csr_matrix):
    """Returns dict with Ahat (on its structural pattern), D, Omega, Jup
    (strict upper CSR of J_tilde), N (indices with D_i < 0, increasing)."""
    n = Abar.shape[0]
    Ahat, P = ahat_on_pattern(Abar, S)
    D = Ahat.diagonal()
    if np.any(D == 0):
        raise ZeroDiagonal("diag(Abar S) has a zero entry")
    Omega = 1.0 / np.sqrt(np.abs(D))
    Up = sp.csr_matrix(sp.triu(P + P.T, 1))
    Up.sort_indices()
    Uc = sp.coo_matrix(Up)
    i, j = Uc.row, Uc.col
    a_ij = _on_pattern(Ahat, Up).data                 # Ahat_ij on the upper pattern
    a_ji = _on_pattern(sp.csr_matrix(Ahat.T), Up).data  # Ahat_ji
    u = Omega[i] * Omega[j] * (a_ij - a_ji) / 2.0
    Jup = sp.csr_matrix((u, Up.indices.copy(), Up.indptr.copy()), shape=(n, n))
    N = np.flatnonzero(D < 0)
    return {"Ahat": Ahat, "D": D, "Omega": Omega, "Jup": Jup, "N": N}


def jtilde_apply(Jup: sp.csr_matrix, v: np.ndarray) -> np.ndarray:
    """J_tilde v = U v - U^T v for the strict upper triangle U."""
    return Jup @ v - Jup.T @ v


def skew_symmetry_ratio(X) -> float:
    """||(X - X^T)/2||_F / ||X - diag(X)||_F (the skew-symmetry measure of the
    paper's Table 3)."""
    X = X.toarray() if sp.issparse(X) else np.asarray(X)
    off = X - np.diag(np.diag(X))
    return float(np.linalg.norm((X - X.T) / 2) / np.linalg.norm(off))


def diagonal_distance(X) -> float:
    """||diag(X) - I||_F (Table 3)."""
    X = X.toarray() if sp.issparse(X) else np.asarray(X)
    return float(np.linalg.norm(np.diag(X) - 1.0))
