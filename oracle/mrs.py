"""Minimal residual solves of shifted skew-symmetric systems, one or several
right-hand sides at once (paper Sec. 3.1; App. B for several right-hand
sides with one shared stopping rule).

For (alpha I + K) x = b with K skew-symmetric, the iterate after t steps is
the minimal residual one over the Krylov space of K and b:

    x_t = V_t y_t,   y_t = argmin_y || r0 e_1 - H_t y ||,   r0 = ||b||,

where V_t = [v_1 .. v_t] comes from the skew-Lanczos recurrence of K started
at v_1 = b / r0,

    K v_j = beta_j v_{j+1} - beta_{j-1} v_{j-1},

and H_t = alpha [I; 0] + T_t is the (t+1) x t matrix with alpha on the
diagonal, beta_j below it and -beta_{j-1} above it, so that
(alpha I + K) V_t = V_{t+1} H_t and the residual norm of x_t equals the
least-squares residual (orthonormal V_{t+1} in exact arithmetic).

This module computes exactly that, in the plainest form that fits in memory:
a first sweep runs the Lanczos recurrence, appends each new column of H to a
QR factorisation by Givens rotations (every earlier rotation applied to the
new column) and reads the residual norm |g_{t+1}| off the rotated
right-hand side; when the stopping rule holds, y solves the triangular
system R y = g, and a second sweep regenerates the same basis vectors (the
same arithmetic on the same inputs) and accumulates x = sum_j y_j v_j.  It
shares no structure with the short recurrences of the paper's listing (no
search directions, no update of x during the iteration); both give the same
iterate up to rounding.

Stopping rule (App. B): all columns step together and stop once the largest
relative residual norm max_j |g_{t+1,j}| / r0_j is below tol, or after maxit
steps; ``fixed_steps > 0`` runs exactly that many steps (trajectory checks).

Readings:
* A zero right-hand-side column keeps x_j = 0 and a residual ratio of 0 (the
  listing would divide by r0_j = 0).
* A breakdown beta_j = 0 means the Krylov space is invariant: the next basis
  vector is 0, the least-squares residual is 0 from then on, and later steps
  add nothing to x.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular


def _colnorms(M: np.ndarray) -> np.ndarray:
    """2-norm of every column, one column at a time (so a column's norm does
    not depend on how many columns run together)."""
    return np.array([np.linalg.norm(np.ascontiguousarray(M[:, j])) for j in range(M.shape[1])])


def _lanczos_sweep(K_apply, V1: np.ndarray, steps: int, visit, store=None):
    """Skew-Lanczos recurrence from the orthonormal start columns V1 (n, nrhs):
    calls visit(j, v_j, beta_j) for j = 1..steps with v_j the j-th basis
    vectors and beta_j = ||K v_j + beta_{j-1} v_{j-1}|| (the subdiagonal entry
    of column j); the next vector is v_{j+1} = (K v_j + beta_{j-1} v_{j-1}) / beta_j
    (zero where beta_j = 0), rounded by `store` when given."""
    v_prev = np.zeros_like(V1)
    v = V1
    beta_prev = np.zeros(V1.shape[1])
    for j in range(1, steps + 1):
        w = K_apply(v) + v_prev * beta_prev
        beta = _colnorms(w)
        if not visit(j, v, beta):
            return
        nz = beta > 0
        v_next = np.where(nz, w / np.where(nz, beta, 1.0), 0.0)
        if store is not None:
            v_next = store(v_next)
        v_prev, v, beta_prev = v, v_next, beta


class _GivensQR:
    """QR factorisation of the growing (t+1) x t matrix H of one column, by
    Givens rotations, with the rotated right-hand side g (g = r0 e_1 at the
    start).  After appending column t, |g[t]| is the least-squares residual.
    The columns of R are kept as a list (column l has l + 2 rows)."""

    def __init__(self, r0: float):
        self.cols = []
        self.g = [r0]
        self.cs, self.sn = [], []

    def append(self, col: np.ndarray) -> float:
        """col: the new column of H, length t + 2 (rows 0..t+1 of column t)."""
        t = len(self.cols)
        h = np.array(col, dtype=np.float64)
        for i, (c, s) in enumerate(zip(self.cs, self.sn)):  # earlier rotations, in order
            a, b = h[i], h[i + 1]
            h[i], h[i + 1] = c * a + s * b, -s * a + c * b
        rr = np.hypot(h[t], h[t + 1])
        c, s = (1.0, 0.0) if rr == 0.0 else (h[t] / rr, h[t + 1] / rr)
        h[t], h[t + 1] = rr, 0.0
        self.cs.append(c)
        self.sn.append(s)
        a = self.g[t]
        self.g[t] = c * a
        self.g.append(-s * a)
        self.cols.append(h)
        return abs(self.g[t + 1])

    def solve(self) -> np.ndarray:
        """y with R[:t, :t] y = g[:t] (back substitution)."""
        t = len(self.cols)
        R = np.zeros((t, t))
        for l, h in enumerate(self.cols):
            R[: l + 1, l] = h[: l + 1]
        return solve_triangular(R, np.asarray(self.g[:t]), lower=False)


def mrs(alpha: float, K_apply, b: np.ndarray, maxit: int, tol: float, fixed_steps: int = 0,
        storage=None):
    """Returns (x, its, relres_hist) with x of b's shape, its the number of
    steps taken and relres_hist of shape (its+1, nrhs) (row 0 is 1 for a
    nonzero column, 0 for a zero one).

    storage: None (FP64 throughout) or a NumPy dtype such as np.float32 in
    which the basis vectors are stored: every v_j is rounded to it (the
    arithmetic stays FP64).  This is the reading taken for an inner solve
    that keeps its vectors in FP32; the reference for such a solve is then
    its residual, not its iterates."""
    single = b.ndim == 1
    B = b.reshape(b.shape[0], -1).astype(np.float64, copy=False)
    n, nrhs = B.shape
    r0 = _colnorms(B)
    live = r0 > 0
    store = None if storage is None else (lambda a: a.astype(storage).astype(np.float64))
    V1 = np.where(live, B / np.where(live, r0, 1.0), 0.0)
    if store is not None:
        V1 = store(V1)
    limit = fixed_steps if fixed_steps > 0 else maxit
    qrs = [_GivensQR(r0[c]) for c in range(nrhs)]
    hist = [np.where(live, 1.0, 0.0)]
    beta_prev = np.zeros(nrhs)
    state = {"its": 0}

    # first sweep: columns of H, their QR, residual norms, the stopping step
    def first(j, v, beta):
        rel = np.zeros(nrhs)
        for c in range(nrhs):
            if not live[c]:
                continue
            col = np.zeros(j + 1)
            if j >= 2:
                col[j - 2] = -beta_prev[c]
            col[j - 1] = alpha
            col[j] = beta[c]
            rel[c] = qrs[c].append(col) / r0[c]
        hist.append(rel)
        beta_prev[:] = beta
        state["its"] = j
        return fixed_steps > 0 or rel.max() >= tol

    _lanczos_sweep(K_apply, V1, limit, first, store)
    its = state["its"]
    Y = np.zeros((its, nrhs))
    for c in range(nrhs):
        if live[c]:
            Y[:, c] = qrs[c].solve()

    # second sweep: the same basis again, x = V_its y
    x = np.zeros((n, nrhs))

    def second(j, v, beta):
        x[:] += v * Y[j - 1]
        return j < its

    if its > 0:
        _lanczos_sweep(K_apply, V1, its, second, store)
    x = x[:, 0] if single else x
    return x, its, np.asarray(hist)
