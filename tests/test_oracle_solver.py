"""Pins for the preconditioner (Sec. 3.2, eq. smw) and the whole two-level
solve (Sec. 3, Sec. 4.1)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W

EXACT = dict(tol=1e-15, maxit=5000)


def _neg_case():
    """A stand-in matrix whose preprocessed diagonal has negative entries."""
    for s in range(10):
        A = W.paper_like(200, 1200, seed=s).A
        st = O.setup(A, O.SetupOptions(k=5, gamma=0.01, s_pattern="tridiag"))
        if st.N.size > 0:
            return st
    raise AssertionError("no case with negative diagonal found")


@pytest.fixture(scope="module")
def neg_setup():
    return _neg_case()


@pytest.fixture(scope="module")
def cfg0_setup():
    return O.setup(W.config(0).A, O.SetupOptions(k=8, s_pattern="tridiag"))


def _dense_P(st):
    n = st.n
    Jt = O.split.jtilde_apply(st.Jup, np.eye(n))
    return np.diag(np.sign(st.D)) + Jt


@pytest.mark.parametrize("k", [0, 1, 4, 5])
def test_combined_lowrank_form_equals_sign_plus_skew(k):
    """U_bar Sigma_bar U_bar^T + S_bar = sign(D) + J_tilde (eq. preconditioner)."""
    st = O.setup(W.paper_like(120, 700, seed=1).A, O.SetupOptions(k=k, gamma=0.01))
    np.testing.assert_allclose(st.prec.dense_P(), _dense_P(st), atol=1e-13)


@pytest.mark.parametrize("k", [4, 5, 8])
def test_smw_apply_equals_dense_solve(k):
    st = O.setup(W.config(0, m=20).A, O.SetupOptions(k=k, x_tol=1e-15, x_maxit=5000))
    P = _dense_P(st)
    v = np.random.default_rng(k).standard_normal(st.n)
    z, _ = st.prec.apply(v, **EXACT)
    np.testing.assert_allclose(z, np.linalg.solve(P, v), rtol=1e-12, atol=1e-12)
    zt, _ = st.prec.apply_T(v, **EXACT)
    np.testing.assert_allclose(zt, np.linalg.solve(P.T, v), rtol=1e-12, atol=1e-12)


def test_smw_apply_with_negative_diagonal(neg_setup):
    st = neg_setup
    st2 = O.setup(st.A, O.SetupOptions(k=5, gamma=0.01, x_tol=1e-15, x_maxit=20000))
    assert st2.N.size > 0
    P = _dense_P(st2)
    v = np.random.default_rng(0).standard_normal(st2.n)
    z, _ = st2.prec.apply(v, tol=1e-15, maxit=20000)
    ref = np.linalg.solve(P, v)
    assert np.linalg.norm(z - ref) <= 1e-9 * np.linalg.norm(ref)


def test_printed_smw_inner_matrix_is_not_the_inverse():
    """The inner matrix printed in eq. smw, (Sigma + U^T S^-1 U)^-1, does not
    give P^-1 (SMW needs Sigma^-1 there): documents the reading taken."""
    st = O.setup(W.config(0, m=20).A, O.SetupOptions(k=4, x_tol=1e-15, x_maxit=5000))
    pr = st.prec
    v = np.random.default_rng(1).standard_normal(st.n)
    y, _, _ = O.mrs(1.0, pr.jbar, v, 5000, 1e-15)
    printed = y - pr.X @ np.linalg.solve(pr.Sigma + pr.G, pr.U.T @ y)
    ref = np.linalg.solve(_dense_P(st), v)
    assert np.linalg.norm(printed - ref) > 1e-3 * np.linalg.norm(ref)


def test_identity_plus_skew_one_outer_iteration():
    """Abar = I + K: S = I (diagonal pattern), P equals the scaled operator,
    so an exact inner solve makes FGMRES converge in one step."""
    rng = np.random.default_rng(2)
    n = 50
    K = sp.random(n, n, density=0.1, random_state=rng).toarray()
    K = 0.5 * (K - K.T)
    A = sp.csr_matrix(np.eye(n) + K)
    st = O.setup(A, O.SetupOptions(k=3, s_pattern="diag", x_tol=1e-15, x_maxit=5000))
    b = rng.standard_normal(n)
    x, info = O.solve(st, b, O.SolveOptions(tol=1e-12, inner_tol=1e-15, inner_maxit=5000))
    assert info["converged"] and info["outer_its"] == 1
    np.testing.assert_allclose(x, np.linalg.solve(A.toarray(), b), rtol=1e-11)


def test_config0_solution_vs_dense(cfg0_setup):
    w = W.config(0)
    x, info = O.solve(cfg0_setup, w.b, O.SolveOptions(tol=1e-12))
    assert info["converged"] and info["relres_true"] <= 1e-12
    xd = np.linalg.solve(w.A.toarray(), w.b)
    assert np.linalg.norm(x - xd) <= 4 * 1e-12 * 4 * np.linalg.norm(xd)
    h = np.asarray(info["hist"])
    assert np.all(np.diff(h) <= 1e-15)
    assert info["k_eff"] == 8 and info["rank_r"] == 0


def test_config0_adjoint_vs_dense(cfg0_setup):
    w = W.config(0)
    g = np.random.default_rng(3).standard_normal(w.A.shape[0])
    lam, info = O.solve_adjoint(cfg0_setup, g, O.SolveOptions(tol=1e-12))
    ld = np.linalg.solve(w.A.toarray().T, g)
    assert info["converged"]
    assert np.linalg.norm(lam - ld) <= 1e-9 * np.linalg.norm(ld)


def test_negative_diagonal_solve_and_adjoint(neg_setup):
    st = neg_setup
    b = st.A @ np.ones(st.n)
    x, info = O.solve(st, b, O.SolveOptions(tol=1e-10))
    assert info["converged"] and info["rank_r"] > 0
    xd = np.linalg.solve(st.A.toarray(), b)
    kappa = np.linalg.cond(st.A.toarray())
    assert np.linalg.norm(x - xd) <= 10 * kappa * 1e-10 * np.linalg.norm(xd)
    g = np.random.default_rng(5).standard_normal(st.n)
    lam, info = O.solve_adjoint(st, g, O.SolveOptions(tol=1e-10))
    assert info["converged"]


def test_tiny_terminates_within_n_outer_steps():
    rng = np.random.default_rng(4)
    n = 8
    A = sp.csr_matrix(np.eye(n) * 3 + rng.standard_normal((n, n)))
    st = O.setup(A, O.SetupOptions(k=2, x_tol=1e-15, x_maxit=1000))
    b = rng.standard_normal(n)
    x, info = O.solve(st, b, O.SolveOptions(tol=1e-13, restart_m=n, inner_tol=1e-15, inner_maxit=1000))
    assert info["converged"] and info["outer_its"] <= n


def test_restarts_and_limits(cfg0_setup):
    w = W.config(0)
    x, info = O.solve(cfg0_setup, w.b, O.SolveOptions(tol=1e-10, restart_m=2))
    assert info["converged"] and info["cycles"] > 1
    x, info = O.solve(cfg0_setup, w.b, O.SolveOptions(tol=1e-10, max_outer=1))
    assert not info["converged"] and info["outer_its"] == 1
    x, info = O.solve(cfg0_setup, np.zeros(w.A.shape[0]))
    assert info["converged"] and np.all(x == 0)
    b = w.b.copy()
    b[3] = np.nan
    with pytest.raises(ValueError):
        O.solve(cfg0_setup, b)


def test_fixed_inner_steps(cfg0_setup):
    w = W.config(0)
    x, info = O.solve(cfg0_setup, w.b, O.SolveOptions(tol=1e-8, fixed_inner_steps=30))
    assert info["converged"]
    assert info["inner_its_total"] == 30 * info["outer_its"]


def test_initial_guess(cfg0_setup):
    """Starting from x0: the exact solution returns at once, unchanged; a
    random or a nearby x0 reaches the dense solution with the true residual
    below tol * ||b|| (not ||b - A x0||); the nearby start takes fewer outer
    steps; the adjoint likewise; a non-finite x0 is refused."""
    st = cfg0_setup
    w = W.config(0)
    A, b = w.A, w.b
    Ad = A.toarray()
    xd = np.linalg.solve(Ad, b)
    kappa = np.linalg.cond(Ad)
    o = O.SolveOptions(tol=1e-10)
    x, info = O.solve(st, b, o, x0=xd)
    assert info["converged"] and info["outer_its"] == 0 and np.array_equal(x, xd)
    _, info_zero = O.solve(st, b, o)
    rng = np.random.default_rng(3)
    for x0 in (rng.standard_normal(st.n), xd + 1e-4 * rng.standard_normal(st.n)):
        x, info = O.solve(st, b, o, x0=x0)
        assert info["converged"]
        assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
        assert np.linalg.norm(x - xd) <= 2 * kappa * 1e-10 * np.linalg.norm(xd)
    assert info["outer_its"] < info_zero["outer_its"]
    lamd = np.linalg.solve(Ad.T, b)
    lam, info = O.solve_adjoint(st, b, o, x0=lamd + 1e-4 * rng.standard_normal(st.n))
    assert info["converged"] and np.linalg.norm(lam - lamd) <= 2 * kappa * 1e-10 * np.linalg.norm(lamd)
    with pytest.raises(ValueError):
        O.solve(st, b, o, x0=np.full(st.n, np.nan))


@pytest.mark.parametrize("case", ["cfg0", "neg"])
def test_smw_preconditioner_does_not_depend_on_the_deflation_basis(case, cfg0_setup, neg_setup):
    """Eq. smw adds back, through the low-rank term, exactly what the deflation
    of J_tilde takes out, so P^-1 applied as mrs on I + J_tilde - Q S_k Q^T plus
    the SMW correction is the inverse of the same P for any basis Q used
    consistently (Sec. 3.2).  Checked on the Lanczos basis rounded to FP32
    values and on a basis perturbed by 1e-3 (no longer a Lanczos basis), with
    and without negative diagonal entries (r = 0 and r > 0): P^-1 v agrees with
    a dense solve with the unperturbed P.  This is what lets the library store
    its deflation basis as FP32 values in the FP64 path."""
    from oracle.precond import Preconditioner
    st = cfg0_setup if case == "cfg0" else neg_setup
    assert (st.N.size > 0) == (case == "neg")
    P = st.prec.dense_P()
    v = np.random.default_rng(41).standard_normal(P.shape[0])
    zd = np.linalg.solve(P, v)
    rng = np.random.default_rng(42)
    for Q in (st.Q.astype(np.float32).astype(np.float64),
              st.Q + 1e-3 * rng.standard_normal(st.Q.shape)):
        pr = Preconditioner(st.prec.Jup, st.N, Q, st.alpha)
        z, its = pr.apply(v, 1e-14, 5000)
        assert its > 0
        assert np.linalg.norm(z - zd) <= 1e-9 * np.linalg.norm(zd)
