"""Structural preprocessing: Abar = P Dr A Dc (paper Sec. 2, eq. mc64).

The paper calls HSL MC64 (maximum product transversal with scaling): a row
permutation P and diagonal scalings Dr, Dc such that |abar_ii| = 1 and
|abar_ij| <= 1.  The paper fixes only these properties.  The oracle takes:

* matching: a perfect matching maximising prod_j |a_{m[j], j}|, as a minimum
  cost assignment with c_ij = log(max_k |a_kj|) - log |a_ij|.  No perfect
  matching exists iff A is structurally singular.
* scaling (reading, the MC64 dual is not unique): with At = P A (row j of At is
  row m[j] of A) and w_ij = log|at_ii| - log|at_ij| for every off-diagonal
  nonzero, gamma is the shortest-path distance from a virtual source joined to
  every node by a zero-weight edge over the edges i -> j of weight w_ij, i.e.
  the componentwise largest gamma <= 0 with gamma_j <= gamma_i + w_ij.
  Dc = diag(exp(gamma)), the row scale of At row i is exp(-gamma_i) / |at_ii|.

Explicit zeros of the input are dropped (a stored zero is no nonzero).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import min_weight_full_bipartite_matching


class StructurallySingular(ValueError):
    pass


class ZeroDiagonal(ValueError):
    pass


def validate_csr(A) -> sp.csr_matrix:
    """Checks of the input (paper Sec. 1: A square, sparse, invertible).

    Returns a canonical copy (float64, sorted indices, explicit zeros dropped).
    Raises ValueError on non-square, empty, duplicate/unsorted-free violations
    are repaired only for the copy; non-finite values raise.
    """
    A = sp.csr_matrix(A, dtype=np.float64, copy=True)
    n, n2 = A.shape
    if n != n2 or n < 1:
        raise ValueError("A must be square with n >= 1")
    if not np.all(np.isfinite(A.data)):
        raise ValueError("A has non-finite values")
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    return A


def max_product_matching(A: sp.csr_matrix) -> np.ndarray:
    """m[j] = row matched to column j, maximising prod |a_{m[j],j}| (Sec. 2).

    Solved as min-cost perfect matching with c_ij = log(colmax_j) - log|a_ij| >= 0
    (a per-column constant does not change the optimum).  SciPy's LAPJVsp needs
    nonzero weights, so 1 is added to every cost, which shifts every perfect
    matching by n and keeps the optimum.
    """
    C = sp.csc_matrix(abs(A))
    n = C.shape[0]
    colmax = np.zeros(n)
    for j in range(n):
        seg = C.data[C.indptr[j]:C.indptr[j + 1]]
        colmax[j] = seg.max() if seg.size else 0.0
    cols = np.repeat(np.arange(n), np.diff(C.indptr))
    cost = np.log(colmax[cols]) - np.log(C.data) + 1.0
    W = sp.csc_matrix((cost, C.indices, C.indptr), shape=C.shape)
    try:
        rows, matched_cols = min_weight_full_bipartite_matching(W)
    except ValueError as e:
        raise StructurallySingular(str(e)) from e
    m = np.empty(n, dtype=np.int64)
    m[matched_cols] = rows
    return m


def matching_log_product(A: sp.csr_matrix, m: np.ndarray) -> float:
    """sum_j log|a_{m[j], j}| of a matching (objective used when ties exist)."""
    Ad = A.tocsr()
    return float(sum(np.log(abs(Ad[m[j], j])) for j in range(A.shape[0])))


def canonical_scaling(A: sp.csr_matrix, m: np.ndarray):
    """Row/column scalings Dr, Dc for the matching m (reading described above).

    Bellman-Ford relaxation from gamma = 0 (the virtual source).  A negative
    cycle cannot exist for an optimal matching; if relaxation does not settle
    within n+1 sweeps the matching was not optimal and ValueError is raised.
    """
    n = A.shape[0]
    At = A[m, :].tocoo()
    at_diag = np.abs(A[m, :].diagonal())
    if np.any(at_diag == 0):
        raise StructurallySingular("matched entry is zero")
    off = (At.row != At.col) & (At.data != 0)
    i, j = At.row[off], At.col[off]
    w = np.log(at_diag[i]) - np.log(np.abs(At.data[off]))
    gamma = np.zeros(n)
    for _ in range(n + 1):
        new = gamma.copy()
        np.minimum.at(new, j, gamma[i] + w)
        if np.array_equal(new, gamma):
            break
        gamma = new
    else:
        raise ValueError("scaling relaxation did not settle (matching not optimal)")
    # row scale exp(-gamma_i - log|at_ii|), evaluated as exp(-gamma_i)/|at_ii| so
    # that |abar_ii| = 1 holds to rounding even when gamma_i = 0
    Dc = np.exp(gamma)
    Dr = np.empty(n)
    Dr[m] = np.exp(-gamma) / at_diag
    return Dr, Dc


def permute_scale(A: sp.csr_matrix, m: np.ndarray, Dr: np.ndarray, Dc: np.ndarray) -> sp.csr_matrix:
    """Abar = P Dr A Dc, with (P y)_j = y_{m[j]} (eq. mc64)."""
    Abar = sp.diags(Dr[m]) @ A[m, :] @ sp.diags(Dc)
    Abar = sp.csr_matrix(Abar)
    Abar.sort_indices()
    return Abar
