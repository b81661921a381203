"""Pins for the oracle's matching and scaling (paper Sec. 2, eq. mc64)."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linear_sum_assignment

import oracle as O
import workloads as W
from _golden import keyed


def _random_sparse(n, density, rng):
    M = sp.random(n, n, density=density, random_state=rng, data_rvs=rng.standard_normal).tocsr()
    M = M + sp.diags(rng.uniform(0.1, 1.0, n) * np.where(rng.uniform(size=n) < 0.5, -1, 1))
    M = M[rng.permutation(n), :]
    return O.validate_csr(M)


def test_golden_matching_4x4():
    g = keyed("matching_4x4.txt")
    A = sp.csr_matrix(np.array([[1, 5, 0, 0], [4, 1, 0, 0], [0, 0, 2, 3], [0, 0, 1, 6]], float))
    m = O.max_product_matching(A)
    assert np.array_equal(m, g["m"].astype(int))
    Dr, Dc = O.canonical_scaling(A, m)
    np.testing.assert_allclose(Dc, g["Dc"], rtol=1e-15)
    np.testing.assert_allclose(Dr, g["Dr"], rtol=1e-15)
    Abar = O.permute_scale(A, m, Dr, Dc).toarray()
    np.testing.assert_allclose(Abar, g["Abar"].reshape(4, 4), rtol=1e-15, atol=1e-16)


@pytest.mark.parametrize("seed", range(12))
def test_matching_brute_force(seed):
    """Max-product matching equals exhaustive search over all n! permutations."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 7))
    A = _random_sparse(n, 0.5, rng)
    Ad = A.toarray()
    best, best_val = None, -np.inf
    for p in itertools.permutations(range(n)):
        vals = np.abs(Ad[list(p), range(n)])
        if np.all(vals > 0):
            v = np.sum(np.log(vals))
            if v > best_val + 1e-12:
                best, best_val = np.array(p), v
    m = O.max_product_matching(A)
    assert np.sum(np.log(np.abs(Ad[m, range(n)]))) == pytest.approx(best_val, abs=1e-12)
    assert np.array_equal(m, best)


@pytest.mark.parametrize("n", [50, 200])
def test_matching_vs_dense_assignment(n):
    rng = np.random.default_rng(n)
    A = _random_sparse(n, 0.05, rng)
    Ad = np.abs(A.toarray())
    cost = np.where(Ad > 0, -np.log(np.where(Ad > 0, Ad, 1.0)), 1e6)
    r, c = linear_sum_assignment(cost)
    ref = np.empty(n, int)
    ref[c] = r
    m = O.max_product_matching(A)
    assert np.array_equal(m, ref)


def test_row_dominant_configs_give_identity():
    """Any non-identity permutation multiplies the diagonal product by ratios
    |a_ij|/|a_ii| < 1 when every row is strictly dominated by its diagonal."""
    for A in (W.config(0).A, W.convdiff3d_matrix(8, 100.0), W.convdiff3d_matrix(8, 1000.0)):
        A = O.validate_csr(A)
        d = np.abs(A.diagonal())
        off = abs(A - sp.diags(A.diagonal())).max(axis=1).toarray().ravel()
        assert np.all(off < d)
        m = O.max_product_matching(A)
        assert np.array_equal(m, np.arange(A.shape[0]))
        Dr, Dc = O.canonical_scaling(A, m)
        np.testing.assert_array_equal(Dc, np.ones(A.shape[0]))
        np.testing.assert_allclose(Dr, 1.0 / d, rtol=1e-15)


def test_structurally_singular():
    A = sp.csr_matrix(np.array([[1.0, 2.0, 0], [3.0, 4.0, 0], [5.0, 6.0, 0]]))
    with pytest.raises(O.StructurallySingular):
        O.max_product_matching(O.validate_csr(A))


@pytest.mark.parametrize("seed", range(6))
def test_scaling_properties_and_maximality(seed):
    """|abar_ii| = 1, |abar_ij| <= 1, and gamma is the largest feasible
    potential: gamma <= 0 and each gamma_j < 0 is attained by a tight edge."""
    w = W.paper_like(150, 700, seed=seed)
    A = O.validate_csr(w.A)
    m = O.max_product_matching(A)
    Dr, Dc = O.canonical_scaling(A, m)
    Abar = O.permute_scale(A, m, Dr, Dc)
    np.testing.assert_allclose(np.abs(Abar.diagonal()), 1.0, rtol=1e-13)
    off = abs(Abar - sp.diags(Abar.diagonal()))
    assert off.max() <= 1.0 + 1e-13
    gamma = np.log(Dc)
    assert np.all(gamma <= 0)
    At = A[m, :].tocoo()
    dt = np.abs(A[m, :].diagonal())
    sel = At.row != At.col
    i, j = At.row[sel], At.col[sel]
    wgt = np.log(dt[i]) - np.log(np.abs(At.data[sel]))
    slack = gamma[i] + wgt - gamma[j]
    assert slack.min() >= -1e-12
    for jj in np.flatnonzero(gamma < -1e-12):
        assert np.min(np.abs(slack[j == jj])) <= 1e-12


def test_validate_rejects_nonfinite():
    A = sp.csr_matrix(np.array([[1.0, np.nan], [0.0, 1.0]]))
    with pytest.raises(ValueError):
        O.validate_csr(A)


def test_grid_line_tiles_is_a_tiling_permutation():
    """The input-side ordering helper: a permutation whose consecutive runs of
    m*ty*tz entries are ty x tz blocks of whole x-lines."""
    m, ty, tz = 8, 2, 4
    p = W.grid_line_tiles(m, ty, tz)
    assert p.dtype == np.int32 and np.array_equal(np.sort(p), np.arange(m ** 3))
    run = m * ty * tz
    for t in range(m ** 3 // run):
        q = p[t * run:(t + 1) * run]
        x, y, z = q % m, (q // m) % m, q // (m * m)
        assert np.array_equal(x, np.tile(np.arange(m), ty * tz))
        assert len(set(y)) == ty and len(set(z)) == tz
        assert y.max() - y.min() == ty - 1 and z.max() - z.min() == tz - 1
