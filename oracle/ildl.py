"""Incomplete LDL^T of M_hat with Bunch-Kaufman pivoting, the scaled factor
and the low-rank term of the general preconditioner (paper Sec. 3: the
factorization of M_hat, eq. absfac, eq. preconditioner, Fig. 1).

TEST INFRASTRUCTURE ONLY (see the package docstring): dense, slow, for small n.

With M_hat = (A_hat + A_hat^T) / 2 symmetric (indefinite in general), the
factorization is a symmetric permutation and a block LDL^T,

    M_hat[perm][:, perm] = L D L^T + E,

L unit lower triangular, D block diagonal with 1x1 and 2x2 blocks, E = 0 for
the complete factorization and supported on the dropped entries otherwise.

Pivoting (Bunch and Kaufman's partial pivoting, the algorithm of the paper's
reference [BunKP76] as LAPACK's symmetric indefinite factorization runs it,
alpha = (1 + sqrt 17) / 8): at position j of the current Schur complement W,
lam = max_{i > j} |W_ij| at row r (the first such row);
  * 1x1 pivot at j if |W_jj| >= alpha lam (this includes lam = 0);
  * otherwise, with sigma = max_{i >= j, i != r} |W_ir|:
    1x1 at j if |W_jj| >= alpha lam (lam / sigma); else a 1x1 pivot at r
    (positions j and r swapped) if |W_rr| >= alpha sigma; else a 2x2 pivot on
    (j, r) (positions j + 1 and r swapped).
A swap exchanges the two rows and columns of W, the two entries of perm and
the two rows of the columns of L already computed.

Elimination (right-looking): for the pivot block P_b (s x s) and the column
block C = W[j+s:, j:j+s] below it, the columns of L are C P_b^-1; each is
thinned by the dropping rules below; then W[j+s:, j+s:] -= L_b P_b L_b^T with
the thinned columns L_b.  Dropping is therefore applied before a column
updates the rest of the matrix, as in a column-by-column incomplete
factorization.

Readings (the paper names a package and its settings, Sec. 4.1, not rules):
* Threshold: an entry l_ij of a computed column is dropped when
  |l_ij| < droptol * ||l_j||_2 (the norm of the column as computed, over the
  rows below the pivot block).  droptol = 0 drops nothing.
* Fill: a column keeps at most ceil(fill * c_j) entries, the largest in
  magnitude (ties to the smaller position), where c_j counts the structural
  nonzeros of the original M_hat in the pivot's column among the rows still
  to be eliminated.  fill = 1 with droptol = 0 is the "as many nonzeros as
  the original matrix per column" variant; fill = inf keeps all.
* A zero column with a zero diagonal (possible only when M_hat has a zero
  row in the current Schur complement) takes the pivot 1, so that |D| is
  invertible; the preconditioner then acts as the identity on that row.
* pivoting = False takes 1x1 pivots in the natural order (an exact zero pivot
  is an error); with droptol = inf this is the diagonal-only reading
  L = I, D = diag(A_hat).

Scaled factor (eq. absfac): for each block B of D, |B| = V |Lambda| V^T from
its eigendecomposition and C_B the lower Cholesky factor of |B| (a 1x1 block
d gives C = sqrt|d|); C = blockdiag(C_B), Lcal = L C (lower triangular:
L is the identity on each 2x2 pivot block and C_B is lower triangular), and

    M_r = C^-1 D C^-T - I     (block diagonal; eigenvalues 0 or -2),
    J_tilde = Lcal^-1 J_hat[perm][:, perm] Lcal^-T.

Low-rank term (Fig. 1): M_r = U_r Sigma_r U_r^T.  Reading: the walk over the
nonzero rows of M_r is done block by block, using the pivot blocks of D
rather than the test M_r(i, i+1) = 0 (which rounding can fool: a 2x2 block
of -2 I has off-diagonal entries of rounding size), and it covers every
block (the printed loop bound i < r stops early when 2x2 blocks occur): a
1x1 block with D_b < 0 gives the column e_p and Sigma = -2; a 2x2 block gives
one column [e_p, e_p+1] v for every eigenpair (lam, v) of its M_r block with
lam < -1 (the exact eigenvalues are 0 and -2), with Sigma = lam.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .preprocess import ZeroDiagonal

ALPHA = (1.0 + math.sqrt(17.0)) / 8.0


@dataclass
class IldlOptions:
    droptol: float = 0.0
    fill: float = math.inf
    pivoting: bool = True


@dataclass
class IldlFactor:
    perm: np.ndarray        # position p holds original index perm[p]
    L: sp.csr_matrix        # unit lower triangular, in positions
    D: sp.csr_matrix        # block diagonal, in positions
    blocks: np.ndarray      # (nblocks, 2): first position, size (1 or 2)
    dropped: int            # entries of L dropped

    @property
    def n(self):
        return self.perm.size


def bk_pivot(W: np.ndarray, j: int):
    """(size, r) of the Bunch-Kaufman pivot at position j of W."""
    n = W.shape[0]
    akk = abs(W[j, j])
    if j == n - 1:
        return 1, j
    col = np.abs(W[j + 1:, j])
    imax = int(np.argmax(col))
    lam = col[imax]
    r = j + 1 + imax
    if max(akk, lam) == 0.0 or akk >= ALPHA * lam:
        return 1, j
    colr = np.abs(W[j:, r])
    colr[r - j] = 0.0
    sigma = colr.max()
    if akk >= ALPHA * lam * (lam / sigma):
        return 1, j
    if abs(W[r, r]) >= ALPHA * sigma:
        return 1, r
    return 2, r


def _swap(W, L, perm, j, a, b):
    """Exchange positions a and b (a, b >= j) of W, perm and L[:, :j]."""
    if a == b:
        return
    W[[a, b], :] = W[[b, a], :]
    W[:, [a, b]] = W[:, [b, a]]
    perm[[a, b]] = perm[[b, a]]
    L[[a, b], :j] = L[[b, a], :j]


def _thin(l: np.ndarray, cap, droptol: float) -> np.ndarray:
    """The dropping rules on one computed column (entries by position)."""
    keep = l != 0.0
    nrm = np.linalg.norm(l)
    if droptol > 0.0 and nrm > 0.0:
        keep &= ~(np.abs(l) < droptol * nrm)
    if cap is not None and keep.sum() > cap:
        idx = np.flatnonzero(keep)
        order = sorted(idx, key=lambda i: (-abs(l[i]), i))
        keep[:] = False
        keep[order[:cap]] = True
    return np.where(keep, l, 0.0)


def ildl(M, opts: IldlOptions | None = None) -> IldlFactor:
    """Incomplete (or, with the default options, complete) Bunch-Kaufman
    LDL^T of the symmetric matrix M (dense W, right-looking)."""
    opts = opts or IldlOptions()
    M = sp.csr_matrix(M)
    n = M.shape[0]
    W = M.toarray().astype(np.float64)
    if not np.array_equal(W, W.T):
        raise ValueError("M is not symmetric")
    struct = M.toarray() != 0.0
    perm = np.arange(n)
    L = np.zeros((n, n))
    D = np.zeros((n, n))
    blocks = []
    dropped = 0
    j = 0
    while j < n:
        s, r = bk_pivot(W, j) if opts.pivoting else (1, j)
        if s == 1:
            _swap(W, L, perm, j, j, r)
        else:
            _swap(W, L, perm, j, j + 1, r)
        Pb = W[j:j + s, j:j + s].copy()
        if s == 1 and Pb[0, 0] == 0.0:
            if opts.pivoting and not np.any(W[j + 1:, j]):
                Pb[0, 0] = 1.0
            else:
                raise ZeroDiagonal(f"zero pivot at position {j}")
        C = W[j + s:, j:j + s]
        Lb = C / Pb[0, 0] if s == 1 else np.linalg.solve(Pb, C.T).T
        rows = perm[j + s:]
        for q in range(s):
            cap = None
            if math.isfinite(opts.fill):
                cap = int(math.ceil(opts.fill * np.count_nonzero(struct[rows, perm[j + q]])))
            before = np.count_nonzero(Lb[:, q])
            Lb[:, q] = _thin(Lb[:, q], cap, opts.droptol)
            dropped += before - np.count_nonzero(Lb[:, q])
        L[j + s:, j:j + s] = Lb
        L[j:j + s, j:j + s] = np.eye(s)
        D[j:j + s, j:j + s] = Pb
        blocks.append((j, s))
        idx = np.flatnonzero(np.any(Lb != 0.0, axis=1))
        if idx.size:
            Lk = Lb[idx]
            W[np.ix_(j + s + idx, j + s + idx)] -= Lk @ Pb @ Lk.T
        j += s
    return IldlFactor(perm=perm, L=sp.csr_matrix(L), D=sp.csr_matrix(D),
                      blocks=np.asarray(blocks, dtype=np.int64).reshape(-1, 2), dropped=dropped)


def abs_block_cholesky(B: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor of |B| = V |Lambda| V^T (eq. absfac) for a 1x1
    or 2x2 symmetric block B."""
    if B.shape == (1, 1):
        return np.array([[math.sqrt(abs(B[0, 0]))]])
    lam, V = np.linalg.eigh(B)
    absB = (V * np.abs(lam)) @ V.T
    absB = (absB + absB.T) / 2.0
    return np.linalg.cholesky(absB)


def scaled_factor(F: IldlFactor):
    """(Lcal, C, Mr): Lcal = L C lower triangular, C = blockdiag of the
    Cholesky factors of |D|'s blocks, Mr = C^-1 D C^-T - I block diagonal."""
    n = F.n
    Cm = np.zeros((n, n))
    Mr = np.zeros((n, n))
    Dd = F.D.toarray()
    for p, s in F.blocks:
        B = Dd[p:p + s, p:p + s]
        Cb = abs_block_cholesky(B)
        Cm[p:p + s, p:p + s] = Cb
        if s == 1:
            Mr[p, p] = math.copysign(1.0, B[0, 0]) - 1.0
        else:
            T = sla.solve_triangular(Cb, B, lower=True)
            Mb = sla.solve_triangular(Cb, T.T, lower=True).T - np.eye(2)
            Mr[p:p + 2, p:p + 2] = (Mb + Mb.T) / 2.0
    Lcal = sp.csr_matrix(F.L @ sp.csr_matrix(Cm))
    Lcal.eliminate_zeros()
    Lcal.sort_indices()
    return Lcal, sp.csr_matrix(Cm), sp.csr_matrix(Mr)


def low_rank(F: IldlFactor, Mr: sp.csr_matrix):
    """(U_r, sigma_r) with Mr = U_r diag(sigma_r) U_r^T (Fig. 1, with the
    readings of the module docstring).  U_r is dense n x r."""
    n = F.n
    cols, sig = [], []
    Md = Mr.toarray()
    for p, s in F.blocks:
        if s == 1:
            if Md[p, p] != 0.0:
                u = np.zeros(n)
                u[p] = 1.0
                cols.append(u)
                sig.append(Md[p, p])
        else:
            lam, V = np.linalg.eigh(Md[p:p + 2, p:p + 2])
            for t in range(2):
                if lam[t] < -1.0:
                    u = np.zeros(n)
                    u[p:p + 2] = V[:, t]
                    cols.append(u)
                    sig.append(lam[t])
    Ur = np.stack(cols, axis=1) if cols else np.zeros((n, 0))
    return Ur, np.asarray(sig, dtype=np.float64)


def lower_solve(Lcal: sp.csr_matrix, v: np.ndarray) -> np.ndarray:
    """Lcal^-1 v (dense triangular solve; small n)."""
    return sla.solve_triangular(Lcal.toarray(), v, lower=True)


def lower_solve_T(Lcal: sp.csr_matrix, v: np.ndarray) -> np.ndarray:
    """Lcal^-T v."""
    return sla.solve_triangular(Lcal.toarray(), v, lower=True, trans="T")
