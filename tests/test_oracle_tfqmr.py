"""Pins of the oracle's TFQMR outer iteration (the outer method of the paper's
experiments, Sec. 4.1).

* exact preconditioner (Abar = I + K): the preconditioned operator is the
  identity and TFQMR stops after one half step;
* the w vectors of TFQMR after every second half step are the residuals of
  CGS (Sonneveld) on the same preconditioned operator with the same shadow
  vector; an independent textbook CGS on the dense preconditioned operator
  pins the alpha / beta / u / v / w recurrences;
* the quasi-minimal residual bound ||r_m|| <= tau_m sqrt(m + 1) holds for the
  recorded iterates (pins theta, c, tau, eta and the update of x);
* solutions and adjoints against dense solves, and finite termination on a
  tiny system."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W

EXACT_INNER = dict(inner_tol=1e-15, inner_maxit=5000)


@pytest.fixture(scope="module")
def cfg0_setup():
    return O.setup(W.config(0).A, O.SetupOptions(k=8, s_pattern="tridiag"))


def _small(n=40, seed=6):
    w = W.implicit_euler_grid(m=int(np.sqrt(n)), h=0.2, cfg=0)
    st = O.setup(w.A, O.SetupOptions(k=4, s_pattern="tridiag", x_tol=1e-15, x_maxit=5000))
    return st, w


def test_identity_plus_skew_one_half_step():
    rng = np.random.default_rng(2)
    n = 50
    K = sp.random(n, n, density=0.1, random_state=rng).toarray()
    K = 0.5 * (K - K.T)
    A = sp.csr_matrix(np.eye(n) + K)
    st = O.setup(A, O.SetupOptions(k=3, s_pattern="diag", x_tol=1e-15, x_maxit=5000))
    b = rng.standard_normal(n)
    x, info = O.solve(st, b, O.SolveOptions(tol=1e-12, outer="tfqmr", **EXACT_INNER))
    assert info["converged"] and info["outer_its"] == 1
    np.testing.assert_allclose(x, np.linalg.solve(A.toarray(), b), rtol=1e-11)


def _cgs_residual_norms(B, b, steps):
    """Textbook conjugate gradient squared (Sonneveld 1989), x0 = 0, r* = r0."""
    r = b.copy()
    rs = r.copy()
    u = r.copy()
    p = r.copy()
    out = []
    rho = rs @ r
    for _ in range(steps):
        Ap = B @ p
        alpha = rho / (Ap @ rs)
        q = u - alpha * Ap
        r = r - alpha * (B @ (u + q))
        out.append(np.linalg.norm(r))
        rho_new = rs @ r
        beta = rho_new / rho
        rho = rho_new
        u = r + beta * q
        p = u + beta * (q + beta * p)
    return np.array(out)


def test_w_vectors_are_cgs_residuals():
    st, w = _small(n=64)
    n = st.n
    o = O.SolveOptions(tol=1e-14, outer="tfqmr", record=True, max_outer=12, **EXACT_INNER)
    prec = lambda v: st.prec.apply(v, o.inner_tol, o.inner_maxit, 0)[0]
    Pinv = np.column_stack([prec(e) for e in np.eye(n)])
    B = np.column_stack([st.op(Pinv[:, j]) for j in range(n)])
    rhs = st.rhs(w.b)
    x, info = O.solve(st, w.b, o)
    wn = np.array(info["w_norms"])
    steps = 5
    cgs = _cgs_residual_norms(B, rhs, steps)
    # w after half steps 1, 3, 5, ... (0-based) is w_2, w_4, ...: the CGS residuals
    np.testing.assert_allclose(wn[1:2 * steps:2], cgs, rtol=1e-8)


def test_quasi_residual_bound_holds():
    st, w = _small(n=64)
    o = O.SolveOptions(tol=1e-13, outer="tfqmr", record=True, **EXACT_INNER)
    x, info = O.solve(st, w.b, o)
    assert info["converged"]
    rhs = st.rhs(w.b)
    bn = np.linalg.norm(rhs)
    for m, (xm, hb) in enumerate(zip(info["x_hist"], info["hist"])):
        r = np.linalg.norm(rhs - st.op(xm))
        assert r <= hb * bn * (1 + 1e-8) + 1e-14 * bn, (m, r, hb * bn)


def test_config0_solution_and_adjoint_vs_dense(cfg0_setup):
    w = W.config(0)
    x, info = O.solve(cfg0_setup, w.b, O.SolveOptions(tol=1e-12, outer="tfqmr"))
    assert info["converged"] and info["relres_true"] <= 1e-12
    xd = np.linalg.solve(w.A.toarray(), w.b)
    assert np.linalg.norm(x - xd) <= 4 * 1e-12 * 4 * np.linalg.norm(xd)
    g = np.random.default_rng(3).standard_normal(w.A.shape[0])
    lam, info = O.solve_adjoint(cfg0_setup, g, O.SolveOptions(tol=1e-12, outer="tfqmr"))
    ld = np.linalg.solve(w.A.toarray().T, g)
    assert info["converged"]
    assert np.linalg.norm(lam - ld) <= 1e-9 * np.linalg.norm(ld)


def test_tiny_terminates():
    rng = np.random.default_rng(4)
    n = 8
    A = sp.csr_matrix(np.eye(n) * 3 + rng.standard_normal((n, n)))
    st = O.setup(A, O.SetupOptions(k=2, x_tol=1e-15, x_maxit=1000))
    b = rng.standard_normal(n)
    x, info = O.solve(st, b, O.SolveOptions(tol=1e-12, outer="tfqmr", **EXACT_INNER))
    assert info["converged"] and info["outer_its"] <= 2 * n + 2
    np.testing.assert_allclose(x, np.linalg.solve(A.toarray(), b), rtol=1e-9)


def test_unknown_outer_method_rejected(cfg0_setup):
    with pytest.raises(ValueError):
        O.solve(cfg0_setup, W.config(0).b, O.SolveOptions(outer="bicgstab"))
