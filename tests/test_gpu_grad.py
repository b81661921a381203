"""Differentiation of the solve on the GPU (through the C ABI): the autograd
function against the oracle's adjoint gradient, value updates under a frozen
preconditioner, finite-difference checks through a torch assembly of A, and
the error paths of the two entries."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_06954_amd as asss
    asss.load()
    return asss


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


class EulerAssembly:
    """A = E + h (R - J) on an m x m grid as a differentiable torch function of
    (E, r, g): E diagonal, r per-edge diffusion weights (R = Deg_r - Adj_r),
    g per-edge skew values (J_lo,hi = g, J_hi,lo = -g).  Values come out in
    the canonical CSR order of the pattern."""

    def __init__(self, m, h=0.1, cfg=4):
        p = W.implicit_euler_parts(m, h, W.rng_for(cfg))
        n = m * m
        self.n, self.h = n, h
        self.lo, self.hi = p.lo.astype(np.int64), p.hi.astype(np.int64)
        rows = np.concatenate([np.arange(n), self.lo, self.hi])
        cols = np.concatenate([np.arange(n), self.hi, self.lo])
        order = np.lexsort((cols, rows))
        self.order = torch.from_numpy(order)
        rs, cs = rows[order], cols[order]
        self.indptr = np.concatenate([[0], np.cumsum(np.bincount(rs, minlength=n))]).astype(np.int64)
        self.indices = cs.astype(np.int32)
        self.E0 = torch.from_numpy(p.E.copy())
        self.r0 = torch.full((self.lo.size,), p.r_weight, dtype=torch.float64)
        self.g0 = torch.from_numpy(p.g.copy())

    def values(self, E, r, g):
        lo, hi = torch.from_numpy(self.lo), torch.from_numpy(self.hi)
        deg = torch.zeros(self.n, dtype=torch.float64).index_add(0, lo, r).index_add(0, hi, r)
        v = torch.cat([E + self.h * deg, self.h * (-r - g), self.h * (-r + g)])
        return v[self.order]

    def matrix(self, v):
        return sp.csr_matrix((v.detach().numpy(), self.indices, self.indptr), shape=(self.n, self.n))


def test_autograd_matches_oracle_adjoint_gradient():
    asss = _lib()
    from paper_2009_06954_amd.autograd import LinearSolve
    w = W.config(0)
    A = sp.csr_matrix(w.A)
    rng = np.random.default_rng(11)
    xt = rng.standard_normal(A.shape[0])
    print(f"[grad] cfg0 n={A.shape[0]}", flush=True)
    op = LinearSolve(A, k=8, s_pattern="tridiag", tol=1e-12)
    vals = torch.tensor(op.values0, requires_grad=True)
    b = torch.tensor(w.b, device="cuda", requires_grad=True)
    x = op(vals, b)
    L = ((x - torch.from_numpy(xt).cuda()) ** 2).sum()
    L.backward()
    st = O.setup(A, O.SetupOptions(k=8, s_pattern="tridiag"))
    xo, io = O.solve(st, w.b, O.SolveOptions(tol=1e-12))
    lo, il = O.solve_adjoint(st, 2.0 * (xo - xt), O.SolveOptions(tol=1e-12))
    go = O.value_gradient(A, lo, xo)
    assert _rel(_np(x), xo) <= 1e-10
    assert _rel(vals.grad.numpy(), go) <= 1e-9
    assert _rel(_np(b.grad), lo) <= 1e-9
    op.close()


def test_update_values_solves_the_new_matrix():
    asss = _lib()
    from paper_2009_06954_amd.autograd import LinearSolve
    w = W.config(0)
    A = sp.csr_matrix(w.A)
    op = LinearSolve(A, k=8, s_pattern="tridiag", tol=1e-12)
    b = torch.tensor(w.b, device="cuda")
    x0 = _np(op(torch.tensor(op.values0), b))
    rng = np.random.default_rng(3)
    v2 = op.values0 * (1.0 + 0.05 * rng.standard_normal(op.nnz))
    x2 = _np(op(torch.tensor(v2), b))
    assert op.last_info["relres_true"] <= 1e-12
    ref2 = spla.spsolve(sp.csc_matrix(op.matrix(v2)), w.b)
    assert _rel(x2, ref2) <= 1e-10
    x0b = _np(op(torch.tensor(op.values0), b))  # back to the setup values
    assert _rel(x0b, x0) <= 1e-10
    op.close()


def test_update_values_and_gradient_reject_bad_input():
    asss = _lib()
    w = W.config(0)
    A = sp.csr_matrix(w.A)
    n = A.shape[0]
    h = asss.setup(A, k=4, s_pattern="tridiag")
    extra = A.tolil()
    extra[0, n - 1] = 1.0  # outside the pattern
    with pytest.raises(asss.AsssError, match="INVALID_ARG"):
        h.update_values(extra.tocsr())
    Z = A.copy()
    Z.data[:] = 0.0
    Z.data[A.indptr[:-1]] = 1.0  # zeros inside the pattern are allowed
    h.update_values(Z)
    with pytest.raises(ValueError):
        h.update_values(sp.identity(n + 1, format="csr"))
    lam = torch.ones(n, dtype=torch.float64, device="cuda")
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    rp = torch.from_numpy(A.indptr.astype(np.int64)).cuda()
    ci = torch.from_numpy(A.indices.astype(np.int32)).cuda()
    g = h.value_gradient(rp, ci, lam, x)
    assert np.allclose(_np(g), -1.0)
    bad = ci.clone()
    bad[5] = n  # column out of range: skipped and reported
    with pytest.raises(asss.AsssError, match="INVALID_CSR"):
        h.value_gradient(rp, bad, lam, x)
    badp = rp.clone()
    badp[3] = badp[4] + 1  # decreasing row pointer
    with pytest.raises(asss.AsssError, match="INVALID_CSR"):
        h.value_gradient(badp, ci, lam, x)
    h.close()


def _fd_check(m, ndir, seed=7):
    asss = _lib()
    from paper_2009_06954_amd.autograd import LinearSolve
    asm = EulerAssembly(m)
    theta0 = [asm.E0, asm.r0, asm.g0]
    rng = np.random.default_rng(seed)
    b0 = torch.from_numpy(rng.standard_normal(asm.n))
    xt = torch.from_numpy(rng.standard_normal(asm.n)).cuda()
    v0 = asm.values(*theta0)
    op = LinearSolve(asm.matrix(v0), k=8, s_pattern="tridiag", tol=1e-12,
                     solve_opts=dict(restart_m=64))
    assert np.array_equal(op.indices, asm.indices) and np.array_equal(op.indptr, asm.indptr)

    def loss(params, b):
        x = op(asm.values(*params), b.cuda())
        return ((x - xt) ** 2).sum()

    params = [t.clone().requires_grad_(True) for t in theta0]
    bb = b0.clone().requires_grad_(True)
    L = loss(params, bb)
    L.backward()
    grads = [p.grad.numpy() for p in params] + [bb.grad.numpy()]
    flat0 = np.concatenate([t.numpy() for t in theta0] + [b0.numpy()])
    sizes = [t.numel() for t in theta0] + [asm.n]
    worst = 0.0
    for j in range(ndir):
        d = rng.standard_normal(flat0.size)
        eps = 1e-5 * np.linalg.norm(flat0) / np.linalg.norm(d)

        def at(s):
            parts = np.split(flat0 + s * eps * d, np.cumsum(sizes)[:-1])
            with torch.no_grad():
                return float(loss([torch.from_numpy(q) for q in parts[:3]], torch.from_numpy(parts[3])))

        fd = (at(1.0) - at(-1.0)) / (2 * eps)
        an = float(np.concatenate(grads) @ d)
        err = abs(fd - an) / max(abs(fd), 1e-300)
        worst = max(worst, err)
        print(f"[fd] m={m} dir {j}: fd={fd:.10e} adjoint={an:.10e} rel={err:.2e}", flush=True)
    op.close()
    assert worst <= 1e-5, worst


def test_finite_differences_through_assembly():
    _fd_check(m=200, ndir=8)


def test_finite_differences_million_unknowns():
    """The differentiation workload: 1000 x 1000 grid (n = 1e6), 32 random
    directions over (E, R weights, J values, b), solves at tol 1e-12."""
    _fd_check(m=1000, ndir=32)
