"""Minimal residual method for shifted skew-symmetric systems, with
simultaneous iterations for several right-hand sides (paper Sec. 3.1 and
App. B).

Solves (alpha I + K) X = B for skew-symmetric K given as an operator on
(n, nrhs) arrays.  Each column runs its own short recurrence (a skew Lanczos
recurrence q_new = K q + beta q_old followed by a Givens QR update of the
shifted tridiagonal matrix), all columns share one operator application per
iteration, and the loop stops when the largest residual estimate
|s_j| / r0_j falls below tol.

Readings:
* A zero right-hand-side column keeps x_j = 0 and a residual ratio of 0 (the
  appendix would divide by r0_j = 0).
* ``fixed_steps > 0`` runs exactly that many iterations and ignores tol
  (used to compare trajectories).
"""
from __future__ import annotations

import numpy as np


def _colnorms(M: np.ndarray) -> np.ndarray:
    """2-norm of every column, one column at a time (so a column's norm does
    not depend on how many columns run together)."""
    return np.array([np.linalg.norm(np.ascontiguousarray(M[:, j])) for j in range(M.shape[1])])


def mrs(alpha: float, K_apply, b: np.ndarray, maxit: int, tol: float, fixed_steps: int = 0):
    """Returns (x, its, relres_hist) with x of b's shape, its the number of
    iterations run and relres_hist of shape (its+1, nrhs)."""
    single = b.ndim == 1
    B = b.reshape(b.shape[0], -1).astype(np.float64, copy=False)
    n, nrhs = B.shape
    x = np.zeros((n, nrhs))
    r0 = _colnorms(B)
    live = r0 > 0
    safe_r0 = np.where(live, r0, 1.0)
    s = r0.copy()
    q = np.where(live, B / safe_r0, 0.0)
    beta = np.zeros(nrhs)
    theta1 = np.full(nrhs, float(alpha))
    c_old = np.ones(nrhs)
    s_old = np.zeros(nrhs)
    delta_old = np.zeros(nrhs)
    q_old = np.zeros((n, nrhs))
    p_old = np.zeros((n, nrhs))
    p_old2 = np.zeros((n, nrhs))
    hist = [np.where(live, 1.0, 0.0)]
    limit = fixed_steps if fixed_steps > 0 else maxit
    its = 0
    for i in range(1, limit + 1):
        q_new = K_apply(q) + q_old * beta
        q_old = q
        beta = _colnorms(q_new)
        nz = beta != 0
        q = np.where(nz, q_new / np.where(nz, beta, 1.0), q_new)
        theta = np.sqrt(theta1 * theta1 + beta * beta)
        c_k = theta1 / theta
        s_k = beta / theta
        delta = -s_old * beta
        theta1 = c_old * theta
        p = (q_old - p_old2 * delta_old) / theta
        x = x + p * (s * c_k)
        s = -s * s_k
        relres = np.abs(s) / safe_r0
        hist.append(relres)
        its = i
        if fixed_steps <= 0 and relres.max() < tol:
            break
        p_old2 = p_old
        p_old = p
        s_old = s_k
        c_old = c_k
        delta_old = delta
    x = x[:, 0] if single else x
    return x, its, np.asarray(hist)
