"""Differentiable solve x = A^-1 b on top of libasss.

For a scalar loss L(x): dL/db = lambda with A^T lambda = dL/dx, solved by
asss_solve_adjoint (the transposed two-level scheme), and dL/da_ij =
-lambda_i x_j on the stored entries of A, formed by asss_value_gradient.

    op = LinearSolve(A_csr, k=8, s_pattern="tridiag", tol=1e-12)
    x = op(values, b)          # values: A's nonzeros in its CSR order
    L = ((x - xt) ** 2).sum(); L.backward()

The preconditioner is built once from the matrix given to LinearSolve.  A
call with other values moves them into the handle (asss_update_values): the
solve is then exact for the new A to its tolerance, with the old
preconditioner.  Both the forward and the backward solve run on the GPU.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import torch

from . import setup as _setup


class LinearSolve:
    """x = A(values)^-1 b for a fixed sparsity pattern, differentiable in the
    values and in b."""

    def __init__(self, A, device="cuda", tol=1e-10, solve_opts=None, **setup_opts):
        A = sp.csr_matrix(A, copy=True)
        if not A.has_canonical_format:
            A.sum_duplicates()
            A.sort_indices()
        if np.any(A.data == 0.0):
            # the library drops stored zeros at setup (a stored zero is no
            # nonzero of A), so such an entry could never take another value
            # in a later call: refuse it here rather than after a step
            raise ValueError("A has stored zeros: remove them (A.eliminate_zeros()) or give them nonzero values")
        self.n = A.shape[0]
        self.indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
        self.indices = np.ascontiguousarray(A.indices, dtype=np.int32)
        self.values0 = np.ascontiguousarray(A.data, dtype=np.float64)
        self.handle = _setup(A, **setup_opts)
        self.rowptr_dev = torch.from_numpy(self.indptr).to(device)
        self.colind_dev = torch.from_numpy(self.indices).to(device)
        self.solve_opts = dict(tol=tol)
        if solve_opts:
            self.solve_opts.update(solve_opts)
        self._current = self.values0.copy()  # values the handle holds now
        self.last_info = None

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def matrix(self, values) -> sp.csr_matrix:
        v = values.detach().cpu().numpy() if isinstance(values, torch.Tensor) else np.asarray(values)
        return sp.csr_matrix((v.astype(np.float64), self.indices, self.indptr), shape=(self.n, self.n))

    def _use(self, values):
        v = values.detach().to("cpu", torch.float64).numpy()
        if v.shape != (self.nnz,):
            raise ValueError(f"expected {self.nnz} values")
        if not np.array_equal(v, self._current):
            self.handle.update_values(self.matrix(v))
            self._current = v.copy()

    def __call__(self, values, b):
        return _Solve.apply(values, b, self)

    def close(self):
        self.handle.close()


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, b, op: LinearSolve):
        op._use(values)
        x, info = op.handle.solve(b.detach().contiguous(), **op.solve_opts)
        op.last_info = info
        if info["status"] != "OK":
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.op = op
        ctx.save_for_backward(values, x)
        return x

    @staticmethod
    def backward(ctx, gx):
        values, x = ctx.saved_tensors
        op = ctx.op
        op._use(values)  # the handle may have moved on to other values since
        lam, info = op.handle.solve_adjoint(gx.detach().contiguous(), **op.solve_opts)
        if info["status"] != "OK":
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        gvals = None
        if ctx.needs_input_grad[0]:
            gvals = op.handle.value_gradient(op.rowptr_dev, op.colind_dev, lam, x)
            gvals = gvals.to(values.device)
        gb = lam if ctx.needs_input_grad[1] else None
        return gvals, gb, None
