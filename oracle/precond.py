"""Deflated shifted skew-symmetric preconditioner (paper Sec. 3.2, eqs.
preconditioner and smw; the one-time data of Sec. 4.1).

With Q_k, S_k from the skew-Lanczos process:

    J_bar  = J_tilde - Q_k S_k Q_k^T          (still skew-symmetric)
    S_bar  = I + J_bar
    U_bar  = [Q_k, U_r],  Sigma_bar = blkdiag(S_k, Sigma_r),  Sigma_r = -2 I_r
    P      = U_bar Sigma_bar U_bar^T + S_bar

where U_r = [e_i : D_i < 0] (the 1x1 blocks of the low-rank decomposition of
Fig. 1 -- with a diagonal D_tilde no 2x2 blocks arise).  For the general
incomplete LDL^T (oracle.ildl) J_tilde is an operator (two triangular solves
around J_hat) and U_r, Sigma_r come from Fig. 1 with 2x2 blocks; the
formulas below are the same.

Reading of eq. smw (the printed inner matrix (Sigma + U^T S^-1 U)^-1 needs
Sigma^-1, and S_k is singular for odd k): the inverse-free form

    X = S_bar^-1 U_bar,  G = U_bar^T X,  C = I + Sigma_bar G,
    P^-1 v = y - X C^-1 Sigma_bar U_bar^T y,   y = S_bar^-1 v,

and for the transpose (adjoint solves)

    P^-T v = S_bar^-T (v - U_bar Sigma_bar^T C^-T X^T v),  S_bar^T = I - J_bar.

X is computed once with the simultaneous mrs of App. B; every application of
P^-1 runs mrs on S_bar with a single right-hand side.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .lanczos import skew_tridiagonal
from .mrs import mrs
from .split import jtilde_apply


class Preconditioner:
    """Jup, N: the diagonal reading (J_tilde from its strict upper triangle,
    U_r = unit vectors at N, Sigma_r = -2 I).  jtilde, Ur, sigma_r: the
    general one (J_tilde as an operator on vectors or column blocks, U_r and
    the diagonal of Sigma_r given)."""

    def __init__(self, Jup, N, Q, alpha, x_tol=1e-10, x_maxit=2000, jtilde=None, Ur=None,
                 sigma_r=None):
        self.Jup = Jup
        self._jt = jtilde
        self.n = Q.shape[0]
        self.Q = Q
        self.k = Q.shape[1]
        self.Sk = skew_tridiagonal(alpha) if self.k > 0 else np.zeros((0, 0))
        if Ur is None:
            self.N = np.asarray(N, dtype=np.int64)
            r = self.N.size
            Ur = np.zeros((self.n, r))
            Ur[self.N, np.arange(r)] = 1.0
            sigma_r = -2.0 * np.ones(r)
        else:
            r = Ur.shape[1]
            self.N = np.zeros(0, dtype=np.int64)
        self.r = r
        self.U = np.concatenate([Q, Ur], axis=1)
        m = self.k + r
        self.Sigma = np.zeros((m, m))
        self.Sigma[:self.k, :self.k] = self.Sk
        self.Sigma[self.k:, self.k:] = np.diag(np.asarray(sigma_r, dtype=np.float64))
        self.x_its = 0
        if m > 0:
            self.X, self.x_its, _ = mrs(1.0, self.jbar, self.U, x_maxit, x_tol)
            self.G = self.U.T @ self.X
            self.C = np.eye(m) + self.Sigma @ self.G
            self.lu = sla.lu_factor(self.C)
        else:
            self.X = np.zeros((self.n, 0))
            self.G = self.C = np.zeros((0, 0))
            self.lu = None

    def jtilde(self, v):
        if self._jt is not None:
            return self._jt(v)
        return jtilde_apply(self.Jup, v)

    def jbar(self, v):
        """J_bar v = J_tilde v - Q_k (S_k (Q_k^T v)) (Sec. 3.2)."""
        out = self.jtilde(v)
        if self.k > 0:
            out = out - self.Q @ (self.Sk @ (self.Q.T @ v))
        return out

    def jbar_neg(self, v):
        return -self.jbar(v)

    def apply(self, v, tol, maxit, fixed_steps=0):
        """P^-1 v; returns (z, inner iterations)."""
        y, its, _ = mrs(1.0, self.jbar, v, maxit, tol, fixed_steps)
        if self.lu is not None:
            t = self.Sigma @ (self.U.T @ y)
            y = y - self.X @ sla.lu_solve(self.lu, t)
        return y, its

    def apply_T(self, v, tol, maxit, fixed_steps=0):
        """P^-T v; returns (z, inner iterations)."""
        w = v
        if self.lu is not None:
            t = sla.lu_solve(self.lu, self.X.T @ v, trans=1)
            w = v - self.U @ (self.Sigma.T @ t)
        y, its, _ = mrs(1.0, self.jbar_neg, w, maxit, tol, fixed_steps)
        return y, its

    def dense_P(self):
        """P as a dense matrix (tests only, small n)."""
        n = self.n
        Jt = self.jtilde(np.eye(n))
        Jb = Jt - self.Q @ self.Sk @ self.Q.T if self.k > 0 else Jt
        return np.eye(n) + Jb + self.U @ self.Sigma @ self.U.T
