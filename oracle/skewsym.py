"""Sparse approximate shifted skew-symmetrizer S (paper Sec. 2, eqs. 1-2,
eq. regularized, App. A).

Find S on a given sparsity pattern such that the off-diagonal part of Abar S
is as skew-symmetric as possible and its diagonal as close to one as possible:
one least-squares equation (Abar S)_ij + (Abar S)_ji = 0 for every pair i < j
in the strictly upper pattern of |Abar||S| + (|Abar||S|)^T, and n weighted
equations sqrt(gamma) ((Abar S)_ii - 1) = 0.

Readings:
* The objective is sum over those pairs of ((AS)_ij + (AS)_ji)^2 plus
  gamma * sum_i ((AS)_ii - 1)^2, as the appendix builds it (the Frobenius form
  printed in eq. regularized double counts pairs and diagonal terms).
* The least-squares solution is the minimum-norm one (the appendix uses a
  sparse backslash, which agrees whenever B has full column rank).
* Equations are numbered pairs first (by (min, max) index), then the n
  diagonal ones; unknowns are the pattern entries of S in CSR order.  Neither
  order changes the solution.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import lsqr


def s_pattern(Abar: sp.csr_matrix, kind) -> sp.csr_matrix:
    """Pattern of S (values 1).  kind: 'diag', 'tridiag', 'abar' or a sparse
    matrix whose structure is taken as given (Sec. 2: diagonal, tridiagonal,
    banded, the sparsity of Abar, or user defined)."""
    n = Abar.shape[0]
    if isinstance(kind, str):
        if kind == "diag":
            P = sp.identity(n, format="csr")
        elif kind == "tridiag":
            P = sp.diags([np.ones(n - 1), np.ones(n), np.ones(n - 1)], [-1, 0, 1], format="csr")
        elif kind == "abar":
            P = Abar.copy()
        else:
            raise ValueError(f"unknown S pattern {kind!r}")
    else:
        P = sp.csr_matrix(kind)
    P = sp.csr_matrix((np.ones(P.nnz), P.indices, P.indptr), shape=(n, n))
    P.sum_duplicates()
    P.data[:] = 1.0
    P.sort_indices()
    return P


def _spones(M) -> sp.csr_matrix:
    M = sp.csr_matrix(M)
    return sp.csr_matrix((np.ones(M.nnz), M.indices, M.indptr), shape=M.shape)


def build_lls(Abar: sp.csr_matrix, Spat: sp.csr_matrix, gamma: float):
    """Least-squares matrix B and right-hand side v of the skew-symmetrizer
    problem (Sec. 2; App. A gives the same equations), from the linear map
    s -> Abar S.

    The unknowns are the pattern entries s_u = S[k_u, j_u] (CSR order of the
    pattern).  Entry (i, j) of Abar S is sum_k abar_ik s_kj, so unknown u
    contributes abar_{i k_u} to every entry (i, j_u) with abar_{i k_u} != 0:
    that is the matrix M of the map, one row per structural entry of Abar S.
    The equations are
      * one per unordered pair {i, j}, i != j, with (i, j) or (j, i) in the
        structural pattern of Abar S: row M_(i,j) + M_(j,i), right-hand side 0;
      * one per i: sqrt(gamma) M_(i,i), right-hand side sqrt(gamma).
    Pairs are numbered by (min, max) in increasing order, then the n diagonal
    equations.  Returns (B, v, unknown_rows, unknown_cols)."""
    n = Abar.shape[0]
    P = sp.csr_matrix(Spat)
    P.sort_indices()
    unk_row = np.repeat(np.arange(n), np.diff(P.indptr))
    unk_col = P.indices.astype(np.int64)
    nu = unk_row.size
    # M as (entry i, entry j, unknown, coefficient): column k_u of Abar, placed in column j_u
    Ac = sp.csc_matrix(Abar)
    Ac.sort_indices()
    cnt = np.diff(Ac.indptr)[unk_row]              # entries of Abar's column k_u
    u_of = np.repeat(np.arange(nu), cnt)
    starts = np.repeat(Ac.indptr[unk_row], cnt)
    offs = np.arange(u_of.size) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    ent_i = Ac.indices[starts + offs].astype(np.int64)
    coef = Ac.data[starts + offs]
    ent_j = unk_col[u_of]
    # equation numbers: pairs by (min, max), then the diagonal ones
    off = ent_i != ent_j
    lo = np.minimum(ent_i, ent_j)[off]
    hi = np.maximum(ent_i, ent_j)[off]
    keys = np.unique(lo * n + hi)
    neq = keys.size
    eq = np.empty(ent_i.size, dtype=np.int64)
    eq[off] = np.searchsorted(keys, lo * n + hi)
    eq[~off] = neq + ent_i[~off]
    sg = np.sqrt(gamma)
    val = np.where(off, coef, sg * coef)
    B = sp.csr_matrix((val, (eq, u_of)), shape=(neq + n, nu))  # duplicates summed
    B.sort_indices()
    v = np.concatenate([np.zeros(neq), np.full(n, sg)])
    return B, v, unk_row, unk_col


def solve_lls(B: sp.csr_matrix, v: np.ndarray, dense_limit: int = 2000,
              tol: float = 1e-15, iter_lim: int | None = None) -> np.ndarray:
    """Minimum-norm least-squares solution of B s = v: dense SVD-based lstsq for
    small problems, otherwise LSQR from s = 0 (which converges to the
    minimum-norm solution)."""
    if B.shape[1] <= dense_limit:
        s, *_ = np.linalg.lstsq(B.toarray(), v, rcond=None)
        return s
    it = iter_lim if iter_lim is not None else 20 * B.shape[1]
    out = lsqr(B, v, atol=tol, btol=tol, conlim=1e16, iter_lim=it)
    return out[0]


def skew_symmetrizer(Abar: sp.csr_matrix, pattern="tridiag", gamma: float = 1.0, **kw):
    """S on the requested pattern (App. A).  Returns (S as CSR, B, v)."""
    n = Abar.shape[0]
    Spat = s_pattern(Abar, pattern)
    B, v, ur, uc = build_lls(Abar, Spat, gamma)
    s = solve_lls(B, v, **kw)
    S = sp.csr_matrix((s, (ur, uc)), shape=(n, n))
    S.sort_indices()
    # keep the full pattern even where a value is exactly zero
    S = _on_pattern(S, Spat)
    return S, B, v


def _on_pattern(M: sp.csr_matrix, P: sp.csr_matrix) -> sp.csr_matrix:
    """Values of M on the structure of P (entries of P missing from M are 0)."""
    P = sp.csr_matrix(P)
    P.sort_indices()
    n = P.shape[1]
    Pc = sp.coo_matrix(P)
    key_p = Pc.row.astype(np.int64) * n + Pc.col
    Mc = sp.coo_matrix(M)
    key_m = Mc.row.astype(np.int64) * n + Mc.col
    order = np.argsort(key_m)
    key_m, val_m = key_m[order], Mc.data[order]
    pos = np.searchsorted(key_m, key_p)
    pos = np.minimum(pos, max(key_m.size - 1, 0))
    hit = (key_m.size > 0) & (key_m[pos] == key_p) if key_m.size else np.zeros(key_p.size, bool)
    vals = np.where(hit, val_m[pos] if key_m.size else 0.0, 0.0)
    return sp.csr_matrix((vals, P.indices.copy(), P.indptr.copy()), shape=P.shape)


def lls_gradient(Abar: sp.csr_matrix, S: sp.csr_matrix, gamma: float) -> sp.csr_matrix:
    """Half the gradient of the least-squares objective with respect to the
    pattern entries of S, in closed form: with Y = Abar S,
    G = offdiag(Y + Y^T) + gamma diag(Y - 1), grad = pattern(S) o (Abar^T G).
    Zero at the least-squares solution; independent of how B is assembled."""
    Y = sp.csr_matrix(Abar @ S)
    n = Y.shape[0]
    d = Y.diagonal()
    G = sp.csr_matrix(Y + Y.T)
    G = G - sp.diags(G.diagonal()) + sp.diags(gamma * (d - 1.0))
    full = sp.csr_matrix(Abar.T @ G)
    return _on_pattern(full, S)
