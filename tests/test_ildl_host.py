"""The library's host incomplete LDL^T (paper Sec. 3: Bunch-Kaufman pivoting
on M_hat, eq. absfac, the low-rank term of Fig. 1) against the oracle's, on
the CPU through asss_ildl_factor (no device is touched).

The pivot sequence is an integer result decided by floating-point
comparisons; both sides take them in FP64 on the same Schur complements
(formed in a different order: left-looking in the library, right-looking in
the oracle), so the permutation and the block sizes are compared exactly and
L, Lcal, D and U_r Sigma_r U_r^T element by element."""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from oracle.ildl import IldlOptions, ildl, low_rank, scaled_factor
from oracle.split import ahat_on_pattern, symmetric_skew_parts
import workloads as W


def _lib():
    import paper_2009_06954_amd as asss
    if not os.path.exists(asss.LIB_PATH):
        pytest.skip("libasss.so not built")
    asss.load()
    return asss


def _mhat(A, s_pattern="tridiag", gamma=1.0):
    A = O.validate_csr(A)
    m = O.max_product_matching(A)
    Dr, Dc = O.canonical_scaling(A, m)
    Abar = O.permute_scale(A, m, Dr, Dc)
    S, _, _ = O.skew_symmetrizer(Abar, s_pattern, gamma)
    Ahat, _ = ahat_on_pattern(Abar, S)
    return sp.csr_matrix(symmetric_skew_parts(Ahat)[0])


def _random_sym(seed, n, weak_diag):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    M = (A + A.T) / 2
    if weak_diag:
        M[np.diag_indices(n)] *= 0.01
    M[np.abs(M) < 0.3] = 0.0
    return sp.csr_matrix(M)


def _compare(M, opts: IldlOptions, tol=1e-12):
    asss = _lib()
    n = M.shape[0]
    g = asss.ildl_factor(M, droptol=opts.droptol, fill=opts.fill, pivoting=opts.pivoting)
    F = ildl(M, opts)
    assert np.array_equal(g["ildl_perm"], F.perm)
    bs = np.zeros(n, dtype=np.int32)
    bs[F.blocks[:, 0]] = F.blocks[:, 1]
    assert np.array_equal(g["ildl_bsize"], bs)
    scale = max(1.0, abs(M).max())
    Lg = sp.csr_matrix((g["ildl_L_val"], g["ildl_L_colind"], g["ildl_L_rowptr"]), shape=(n, n)).toarray()
    Lo = F.L.toarray() - np.eye(n)
    assert np.abs(Lg - Lo).max() <= tol * max(1.0, np.abs(Lo).max())
    Dg = np.zeros((n, n))
    d3 = g["ildl_D"].reshape(n, 3)
    for p in np.flatnonzero(bs):
        Dg[p, p] = d3[p, 0]
        if bs[p] == 2:
            Dg[p + 1, p] = Dg[p, p + 1] = d3[p, 1]
            Dg[p + 1, p + 1] = d3[p, 2]
    assert np.abs(Dg - F.D.toarray()).max() <= tol * scale
    Lcal, _, Mr = scaled_factor(F)
    Lcg = sp.csr_matrix((g["Lcal_val"], g["Lcal_colind"], g["Lcal_rowptr"]), shape=(n, n)).toarray()
    assert np.abs(Lcg - Lcal.toarray()).max() <= tol * max(1.0, np.abs(Lcal.toarray()).max())
    Ur, sig = low_rank(F, Mr)
    assert g["sigma_r"].size == sig.size
    lo = Ur @ np.diag(sig) @ Ur.T
    lg = g["Ur"] @ np.diag(g["sigma_r"]) @ g["Ur"].T
    assert np.abs(lo - lg).max() <= 1e-12
    return F


@pytest.mark.parametrize("seed", range(12))
def test_random_symmetric_complete_and_incomplete(seed):
    """Dense-ish random symmetric matrices (weak diagonals on even seeds force
    2x2 pivots): complete, threshold-dropped and fill-capped factorizations."""
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(5, 60))
    M = _random_sym(seed, n, weak_diag=seed % 2 == 0)
    F = _compare(M, IldlOptions())
    _compare(M, IldlOptions(droptol=1e-1))
    _compare(M, IldlOptions(droptol=1e-2, fill=1.0))
    if seed % 2 == 0:
        assert (F.blocks[:, 1] == 2).any()


def test_implicit_euler_mhat():
    """M_hat of the 45 x 45 implicit-Euler grid (n = 2025), the settings of
    the paper's experiments ildl(1e-2) and a fill cap of one."""
    M = _mhat(W.implicit_euler_grid(m=45, h=0.1, cfg=0).A)
    F = _compare(M, IldlOptions(droptol=1e-2))
    assert F.dropped > 0
    _compare(M, IldlOptions(fill=1.0))


@pytest.mark.parametrize("seed", [0, 2, 5])
def test_stand_in_mhat_with_2x2_pivots(seed):
    """M_hat of stand-in matrices (random off-diagonals, mixed-sign diagonal):
    indefinite, with 2x2 pivots and a low-rank term."""
    M = _mhat(W.paper_like(300, 1800, seed=seed).A, gamma=0.01)
    for opts in (IldlOptions(), IldlOptions(droptol=1e-2), IldlOptions(droptol=1e-1, fill=2.0)):
        F = _compare(M, opts)
    F = ildl(M, IldlOptions(droptol=1e-2))
    assert (F.blocks[:, 1] == 2).any()


def test_without_pivoting_and_the_diagonal_reading():
    """pivoting off: 1x1 pivots in order; with everything dropped L = I and
    D = diag(M)."""
    M = _mhat(W.implicit_euler_grid(m=12, h=0.2, cfg=0).A)
    _compare(M, IldlOptions(pivoting=False, droptol=1e-2))
    asss = _lib()
    g = asss.ildl_factor(M, droptol=math.inf, pivoting=False)
    n = M.shape[0]
    assert np.array_equal(g["ildl_perm"], np.arange(n))
    assert g["ildl_L_colind"].size == 0
    assert np.allclose(g["ildl_D"].reshape(n, 3)[:, 0], M.diagonal(), rtol=0, atol=0)


def test_zero_pivots():
    """A zero column takes the pivot 1 (as in the oracle); a zero pivot that
    pivoting cannot avoid is ZERO_DIAGONAL; a nonsymmetric M is INVALID_ARG."""
    asss = _lib()
    M = sp.csr_matrix(np.array([[2.0, 0, 1], [0, 0, 0], [1, 0, 3]]))
    g = asss.ildl_factor(M)
    assert g["ildl_D"].reshape(3, 3)[1, 0] == 1.0
    _compare(M, IldlOptions())
    Z = sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 2.0]]))
    with pytest.raises(asss.AsssError) as e:
        asss.ildl_factor(Z, pivoting=False)
    assert e.value.name == "ZERO_DIAGONAL"
    with pytest.raises(asss.AsssError) as e:
        asss.ildl_factor(sp.csr_matrix(np.array([[1.0, 2.0], [0.0, 1.0]])))
    assert e.value.name == "INVALID_ARG"
