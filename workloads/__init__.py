"""Seeded synthetic inputs for the ASSS two-level solver.

This module builds test matrices and right-hand sides only.  It holds none of
the solver's arithmetic, so both the FP64 oracle (``oracle/``) and the GPU
library's tests and benchmark may draw their inputs from it.

Workload families (all draws from NumPy's PCG64, in the order documented per
function):

* ``implicit_euler_grid`` -- A = E + h(R - J) from the implicit Euler step of a
  dissipative Hamiltonian system (paper Sec. 1, eqs. dissHS and the implicit
  Euler system), on an m x m grid graph with a 5-point pattern.
* ``convdiff3d`` -- 7-point first-order upwind discretisation of
  -eps*Laplace(u) + w.grad(u) on the unit cube (a standard nonsymmetric
  benchmark family standing in for large general sparse systems).
* ``batched_implicit_euler`` -- many uneven-sized implicit Euler systems with
  several right-hand sides each.
* ``paper_like`` -- random general sparse matrices with the sizes and densities
  of the paper's test set (Table 1), with a random row permutation and wildly
  varying row scales, so that the matching step is non-trivial.  The paper's
  actual matrices are not available; these only mimic their dimensions.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

BASE_SEED = 200906954


def rng_for(cfg: int) -> np.random.Generator:
    """Generator for configuration number ``cfg`` (seed BASE_SEED + cfg)."""
    return np.random.Generator(np.random.PCG64(BASE_SEED + int(cfg)))


@dataclass
class Workload:
    name: str
    A: sp.csr_matrix
    b: np.ndarray
    x_star: np.ndarray | None = None
    meta: dict = field(default_factory=dict)


def _canonical_csr(M) -> sp.csr_matrix:
    M = sp.csr_matrix(M, dtype=np.float64)
    M.sum_duplicates()
    M.sort_indices()
    M.indptr = M.indptr.astype(np.int64)
    M.indices = M.indices.astype(np.int32)
    return M


# ---------------------------------------------------------------------------
# 2D grid graph, implicit Euler matrix A = E + h (R - J)
# ---------------------------------------------------------------------------

def grid_edges(m: int) -> tuple[np.ndarray, np.ndarray]:
    """Edges of the m x m grid graph, node i = x + m*y.

    Enumeration order: nodes in increasing i (y-major, then x); for each node
    first the edge to (x+1, y), then the edge to (x, y+1).  Returns (lo, hi)
    with lo < hi.
    """
    i = np.arange(m * m, dtype=np.int64)
    x = i % m
    y = i // m
    lo = np.repeat(i, 2)
    hi = np.empty(2 * m * m, dtype=np.int64)
    hi[0::2] = i + 1
    hi[1::2] = i + m
    valid = np.empty(2 * m * m, dtype=bool)
    valid[0::2] = x < m - 1
    valid[1::2] = y < m - 1
    return lo[valid], hi[valid]


@dataclass
class ImplicitEulerParts:
    m: int
    h: float
    E: np.ndarray          # diagonal of E (n)
    lo: np.ndarray         # edge endpoints, lo < hi
    hi: np.ndarray
    g: np.ndarray          # J[lo, hi] = g, J[hi, lo] = -g
    r_weight: float = 0.1  # R = r_weight * (Deg - Adj)

    @property
    def n(self) -> int:
        return self.m * self.m


def implicit_euler_parts(m: int, h: float, rng: np.random.Generator) -> ImplicitEulerParts:
    """Draw E = diag(U(0.5, 2)) (n draws), then g ~ N(0,1) (one per edge)."""
    n = m * m
    E = rng.uniform(0.5, 2.0, size=n)
    lo, hi = grid_edges(m)
    g = rng.standard_normal(lo.size)
    return ImplicitEulerParts(m=m, h=float(h), E=E, lo=lo, hi=hi, g=g)


def assemble_implicit_euler(p: ImplicitEulerParts) -> sp.csr_matrix:
    """A = E + h (R - J) with R = 0.1 (Deg - Adj) and J skew on the grid edges."""
    n = p.n
    deg = np.bincount(p.lo, minlength=n) + np.bincount(p.hi, minlength=n)
    w = p.r_weight
    diag = p.E + p.h * w * deg
    # A[lo, hi] = h(-w - g),  A[hi, lo] = h(-w + g)
    rows = np.concatenate([np.arange(n), p.lo, p.hi])
    cols = np.concatenate([np.arange(n), p.hi, p.lo])
    vals = np.concatenate([diag, p.h * (-w - p.g), p.h * (-w + p.g)])
    return _canonical_csr(sp.coo_matrix((vals, (rows, cols)), shape=(n, n)))


def implicit_euler_grid(m: int = 45, h: float = 0.1, cfg: int = 0) -> Workload:
    """Small implicit Euler grid system (default: 45 x 45, h = 0.1).

    Draw order from PCG64(BASE_SEED + cfg): E (n), g (edges), x* ~ U(-1, 1) (n).
    b = A x*.
    """
    rng = rng_for(cfg)
    parts = implicit_euler_parts(m, h, rng)
    A = assemble_implicit_euler(parts)
    x_star = rng.uniform(-1.0, 1.0, size=A.shape[0])
    b = A @ x_star
    return Workload(name=f"implicit_euler_{m}x{m}_h{h}", A=A, b=b, x_star=x_star,
                    meta={"m": m, "h": h, "parts": parts, "s_pattern": "tridiag", "k": 8})


# ---------------------------------------------------------------------------
# 3D convection-diffusion, first-order upwind
# ---------------------------------------------------------------------------

def convdiff3d_matrix(m: int, peclet: float, wind=(1.0, 0.5, 0.25)) -> sp.csr_matrix:
    """-eps Lap(u) + w.grad(u) on (0,1)^3, Dirichlet, m interior points per axis.

    h = 1/(m+1), eps = max|w| / Pe, rows scaled by h^2, node i = x + m y + m^2 z.
    a_ii = 6 eps + h sum|w_d|; for w_d > 0: a(i, i - e_d) = -eps - h w_d and
    a(i, i + e_d) = -eps (for w_d < 0 the roles of the two neighbours swap).
    """
    wind = tuple(float(v) for v in wind)
    eps = max(abs(v) for v in wind) / float(peclet)
    hh = 1.0 / (m + 1)
    n = m ** 3
    idx = np.arange(n, dtype=np.int64)
    coord = [idx % m, (idx // m) % m, idx // (m * m)]
    strides = [1, m, m * m]
    rows = [idx]
    cols = [idx]
    vals = [np.full(n, 6.0 * eps + hh * sum(abs(v) for v in wind))]
    for d in range(3):
        wd = wind[d]
        back = -eps - hh * wd if wd > 0 else -eps
        fwd = -eps if wd > 0 else -eps + hh * wd
        has_back = coord[d] > 0
        has_fwd = coord[d] < m - 1
        rows += [idx[has_back], idx[has_fwd]]
        cols += [idx[has_back] - strides[d], idx[has_fwd] + strides[d]]
        vals += [np.full(int(has_back.sum()), back), np.full(int(has_fwd.sum()), fwd)]
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=indptr[1:])
    return sp.csr_matrix((vals, cols.astype(np.int32), indptr), shape=(n, n))


def convdiff3d(m: int = 128, peclet: float = 100.0, cfg: int = 1,
               wind=(1.0, 0.5, 0.25)) -> Workload:
    """3D convection-diffusion system; x* ~ U(-1,1) from PCG64(BASE_SEED+cfg), b = A x*."""
    A = convdiff3d_matrix(m, peclet, wind)
    rng = rng_for(cfg)
    x_star = rng.uniform(-1.0, 1.0, size=A.shape[0])
    b = A @ x_star
    return Workload(name=f"convdiff3d_{m}^3_Pe{peclet:g}", A=A, b=b, x_star=x_star,
                    meta={"m": m, "peclet": peclet, "wind": wind, "s_pattern": "abar", "k": 16})


def grid_line_tiles(m: int, ty: int = 4, tz: int = 4) -> np.ndarray:
    """An order of the m^3 grid (node x + m y + m^2 z) in which each run of
    m*ty*tz consecutive positions is one tile of ty x tz whole x-lines: tiles in
    lexicographic (y, z) order, inside a tile lines y-fastest, points x-fastest.
    Returns perm with perm[new] = old (int32)."""
    if m % ty or m % tz:
        raise ValueError("ty and tz must divide m")
    TZ = np.arange(m // tz)[:, None, None, None, None]
    TY = np.arange(m // ty)[None, :, None, None, None]
    z = np.arange(tz)[None, None, :, None, None]
    y = np.arange(ty)[None, None, None, :, None]
    x = np.arange(m)[None, None, None, None, :]
    perm = x + m * ((TY * ty + y) + m * (TZ * tz + z))
    return np.ascontiguousarray(perm.reshape(-1), dtype=np.int32)


# ---------------------------------------------------------------------------
# Batched uneven implicit Euler systems
# ---------------------------------------------------------------------------

def batched_implicit_euler(nsys: int = 64, n_lo: float = 1e4, n_hi: float = 5e5,
                           nrhs: int = 4, cfg: int = 3, h_lo: float = 0.01,
                           h_hi: float = 0.5) -> list[Workload]:
    """Many uneven systems.  Draw order: sizes n_s = exp(U(ln n_lo, ln n_hi)) (nsys),
    h_s ~ U(h_lo, h_hi) (nsys); then per system: E, g (as implicit_euler_parts),
    then B ~ N(0,1) of shape (n_s, nrhs) in column-major draw order."""
    rng = rng_for(cfg)
    sizes = np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=nsys))
    hs = rng.uniform(h_lo, h_hi, size=nsys)
    out = []
    for s in range(nsys):
        m = max(2, int(round(math.sqrt(sizes[s]))))
        parts = implicit_euler_parts(m, float(hs[s]), rng)
        A = assemble_implicit_euler(parts)
        B = rng.standard_normal((nrhs, A.shape[0])).T.copy()
        out.append(Workload(name=f"batched_{s}_m{m}_h{hs[s]:.3f}", A=A, b=B,
                            meta={"m": m, "h": float(hs[s]), "s_pattern": "tridiag", "k": 8}))
    return out


# ---------------------------------------------------------------------------
# Paper-like random general sparse matrices (stand-in for the paper's test set)
# ---------------------------------------------------------------------------

# (name, n, nnz) as listed in the paper's Table 1; rdb1250l uses nnz = 7,300,
# the value implied by its Table 2 row (Table 1 repeats bp_200's count there).
PAPER_SIZES = [
    ("bp_200", 822, 3802), ("bp_600", 822, 4172), ("west0989", 989, 3518),
    ("rajat19", 1157, 3699), ("rdb1250l", 1250, 7300), ("west1505", 1505, 5414),
    ("chebyshev2", 2053, 18447), ("orani678", 2529, 90158),
    ("rdb3200l", 3200, 18880), ("rdb5000", 5000, 29600),
]


def paper_like(n: int, nnz: int, seed: int = 0, row_scale_decades: float = 4.0) -> Workload:
    """Random nonsymmetric sparse matrix with n rows and about nnz nonzeros.

    Draw order from PCG64(BASE_SEED + 1000 + seed): diagonal magnitudes
    U(0.5, 2) (n), diagonal signs (n), off-diagonal column choices, off-diagonal
    values N(0,1), row scales 10^U(-d, d) (n), row permutation (n).
    The right-hand side is b = A * ones (as in the paper's experiments).
    """
    rng = np.random.Generator(np.random.PCG64(BASE_SEED + 1000 + int(seed)))
    dmag = rng.uniform(0.5, 2.0, size=n)
    dsgn = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    n_off = max(0, nnz - n)
    r = rng.integers(0, n, size=n_off)
    c = rng.integers(0, n, size=n_off)
    keep = r != c
    r, c = r[keep], c[keep]
    v = rng.standard_normal(r.size)
    rows = np.concatenate([np.arange(n), r])
    cols = np.concatenate([np.arange(n), c])
    vals = np.concatenate([dmag * dsgn, v])
    M = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    M.sum_duplicates()
    scale = 10.0 ** rng.uniform(-row_scale_decades, row_scale_decades, size=n)
    perm = rng.permutation(n)
    A = sp.diags(scale) @ M
    A = _canonical_csr(A[perm, :])
    b = A @ np.ones(n)
    return Workload(name=f"paper_like_n{n}_s{seed}", A=A, b=b, x_star=np.ones(n),
                    meta={"seed": seed, "s_pattern": "tridiag", "k": 8})


def paper_like_family(scale: float = 1.0, max_n: int | None = None) -> list[Workload]:
    out = []
    for s, (name, n, nnz) in enumerate(PAPER_SIZES):
        nn = max(8, int(round(n * scale)))
        if max_n is not None and nn > max_n:
            continue
        w = paper_like(nn, int(round(nnz * nn / n)), seed=s)
        w.name = f"like_{name}_n{nn}"
        out.append(w)
    return out


# ---------------------------------------------------------------------------
# Configurations used by the benchmark and the parity tests
# ---------------------------------------------------------------------------

def config(cfg: int, **kw):
    """Workload of configuration ``cfg`` (0..4), at full size unless overridden.

    0: 2D implicit Euler, 45 x 45, h = 0.1, S tridiagonal, k = 8
    1: 3D convection-diffusion 128^3, Pe 100, S on the pattern of Abar, k = 16
    2: 3D convection-diffusion 192^3, Pe 1000, same, FP32 inner vs FP64
    3: 64 uneven implicit Euler systems, n in [1e4, 5e5], 4 RHS each
    4: 2D implicit Euler on a 1000 x 1000 grid (differentiation workload)
    """
    if cfg == 0:
        return implicit_euler_grid(m=kw.get("m", 45), h=kw.get("h", 0.1), cfg=0)
    if cfg == 1:
        return convdiff3d(m=kw.get("m", 128), peclet=kw.get("peclet", 100.0), cfg=1)
    if cfg == 2:
        return convdiff3d(m=kw.get("m", 192), peclet=kw.get("peclet", 1000.0), cfg=2)
    if cfg == 3:
        return batched_implicit_euler(nsys=kw.get("nsys", 64), n_lo=kw.get("n_lo", 1e4),
                                      n_hi=kw.get("n_hi", 5e5), nrhs=kw.get("nrhs", 4), cfg=3)
    if cfg == 4:
        return implicit_euler_grid(m=kw.get("m", 1000), h=kw.get("h", 0.1), cfg=4)
    raise ValueError(f"unknown configuration {cfg}")
