"""The two-level scheme end to end (paper Sec. 3, eq. modified, eqs.
preconditioner / smw, Sec. 4.1).

Setup (independent of b, done once):
    m, Dr, Dc          max-product matching and scaling          (Sec. 2)
    S                  least-squares skew-symmetrizer            (Sec. 2, App. A)
    A_hat = Abar S,  D, Omega, J_tilde, N                        (Sec. 3)
    Q_k, S_k           skew-Lanczos                              (Fig. 2)
    X, G, C            one-time SMW data                          (Sec. 4.1)

Solve: the outer Krylov method runs on the scaled system
    A_chk x_chk = b_chk,   A_chk = Omega Abar S Omega,   b_chk = Omega P Dr b,
    x = Dc S Omega x_chk,
right-preconditioned with P (eq. preconditioner).

Readings:
* Outer method: flexible GMRES(m) (the paper says "a Krylov subspace method";
  the inner solve is inexact, so the preconditioner changes from step to step
  and the flexible variant stores the preconditioned vectors z_j).  Arnoldi
  with classical Gram-Schmidt and one reorthogonalisation pass whenever the
  norm drops below 1/sqrt(10) of its value (Daniel-Gragg-Kaufman-Stewart
  criterion with eta = 1/sqrt(10): the orthogonality lost in one pass is then
  a small multiple of the rounding unit; with eta = 1/sqrt(2) the second pass
  ran in every step on the convection-diffusion family without changing a
  single iterate count); Givens rotations on the Hessenberg matrix.
* Stopping: the implicit residual |g_{j+1}| <= thr only triggers a check; the
  solve is converged when the true residual ||b - A x|| <= tol ||b|| on the
  original system.  The true residual is also checked at every restart.  If
  the implicit test passed but the true one failed, thr is multiplied by
  0.5 * tol / relres_true and the method restarts.  thr starts at
  tol * ||b_chk||.  max_outer counts Arnoldi steps over all cycles.
* Inner solves: mrs on S_bar with tolerance inner_tol and at most inner_maxit
  iterations (the paper uses the outer criterion for both levels).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .lanczos import DEFAULT_SEED, skew_lanczos, start_vector
from .precond import Preconditioner
from .preprocess import canonical_scaling, max_product_matching, permute_scale, validate_csr
from .skewsym import skew_symmetrizer
from .split import jtilde_apply, split_ahat


@dataclass
class SetupOptions:
    gamma: float = 1.0
    s_pattern: object = "tridiag"
    k: int = 20
    lanczos_seed: int = DEFAULT_SEED
    x_tol: float = 1e-10
    x_maxit: int = 2000
    lls_dense_limit: int = 2000


@dataclass
class SolveOptions:
    tol: float = 1e-8
    restart_m: int = 64
    max_outer: int = 2000
    inner_tol: float = 1e-5
    inner_maxit: int = 1000
    fixed_inner_steps: int = 0
    outer: str = "fgmres"  # or "tfqmr"
    record: bool = False   # tfqmr: keep x_chk and ||w|| after every half step
                           # (info["x_hist"], info["w_norms"])


@dataclass
class OracleSetup:
    A: sp.csr_matrix
    m: np.ndarray
    Dr: np.ndarray
    Dc: np.ndarray
    Abar: sp.csr_matrix
    S: sp.csr_matrix
    Ahat: sp.csr_matrix
    D: np.ndarray
    Omega: np.ndarray
    Jup: sp.csr_matrix
    N: np.ndarray
    Q: np.ndarray
    alpha: np.ndarray
    prec: Preconditioner
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.A.shape[0]

    @property
    def rank_r(self):
        return self.N.size

    # outer operator and its transpose (Sec. 3, eq. modified with the scaling)
    def op(self, z):
        return self.Omega * (self.Abar @ (self.S @ (self.Omega * z)))

    def op_T(self, z):
        return self.Omega * (self.S.T @ (self.Abar.T @ (self.Omega * z)))

    def rhs(self, b):
        """b_chk = Omega P Dr b."""
        return self.Omega * (self.Dr[self.m] * b[self.m])

    def back(self, x_chk):
        """x = Dc S Omega x_chk."""
        return self.Dc * (self.S @ (self.Omega * x_chk))

    def rhs_T(self, g):
        """g_chk = Omega S^T Dc g (adjoint)."""
        return self.Omega * (self.S.T @ (self.Dc * g))

    def back_T(self, l_chk):
        """lambda = Dr P^T Omega l_chk (adjoint)."""
        lam = np.empty(self.n)
        lam[self.m] = self.Dr[self.m] * (self.Omega * l_chk)
        return lam


def setup(A, opts: SetupOptions | None = None) -> OracleSetup:
    opts = opts or SetupOptions()
    A = validate_csr(A)
    m = max_product_matching(A)
    Dr, Dc = canonical_scaling(A, m)
    Abar = permute_scale(A, m, Dr, Dc)
    S, B, v = skew_symmetrizer(Abar, opts.s_pattern, opts.gamma, dense_limit=opts.lls_dense_limit)
    parts = split_ahat(Abar, S)
    Jup = parts["Jup"]
    n = A.shape[0]
    q1 = start_vector(opts.lanczos_seed, n)
    Q, alpha = skew_lanczos(lambda v_: jtilde_apply(Jup, v_), q1, opts.k)
    prec = Preconditioner(Jup, parts["N"], Q, alpha, opts.x_tol, opts.x_maxit)
    return OracleSetup(A=A, m=m, Dr=Dr, Dc=Dc, Abar=Abar, S=S, Ahat=parts["Ahat"],
                       D=parts["D"], Omega=parts["Omega"], Jup=Jup, N=parts["N"],
                       Q=Q, alpha=alpha, prec=prec, extra={"B_shape": B.shape, "B_nnz": B.nnz})


@dataclass
class IldlOracleSetup:
    """The two-level scheme with the general incomplete LDL^T of M_hat
    (Sec. 3, eqs. absfac and preconditioner; oracle.ildl).  The outer method
    runs in the positions of the factorization:

        A_chk = Lcal^-1 A_hat[perm][:, perm] Lcal^-T,
        b_chk = Lcal^-1 (P Dr b)[perm],
        x_hat[perm] = Lcal^-T x_chk,  x = Dc S x_hat,

    right-preconditioned with P = M_r + I + J_tilde (deflated, in the SMW form
    of oracle.precond).  The Lanczos start vector is indexed by positions."""
    A: sp.csr_matrix
    m: np.ndarray
    Dr: np.ndarray
    Dc: np.ndarray
    Abar: sp.csr_matrix
    S: sp.csr_matrix
    Ahat: sp.csr_matrix
    factor: object          # oracle.ildl.IldlFactor
    Lcal: sp.csr_matrix
    Mr: sp.csr_matrix
    Ur: np.ndarray
    sigma_r: np.ndarray
    Ap: sp.csr_matrix       # A_hat[perm][:, perm]
    Jp: sp.csr_matrix       # J_hat[perm][:, perm]
    Q: np.ndarray
    alpha: np.ndarray
    prec: Preconditioner
    Ld: np.ndarray = None   # Lcal as a dense array (triangular solves)

    @property
    def n(self):
        return self.A.shape[0]

    @property
    def rank_r(self):
        return self.Ur.shape[1]

    @property
    def perm(self):
        return self.factor.perm

    def lsolve(self, v):
        return sla.solve_triangular(self.Ld, v, lower=True)

    def lsolve_T(self, v):
        return sla.solve_triangular(self.Ld, v, lower=True, trans="T")

    def jtilde(self, v):
        """J_tilde v = Lcal^-1 J_hat_p Lcal^-T v."""
        return self.lsolve(self.Jp @ self.lsolve_T(v))

    def op(self, z):
        return self.lsolve(self.Ap @ self.lsolve_T(z))

    def op_T(self, z):
        return self.lsolve(self.Ap.T @ self.lsolve_T(z))

    def rhs(self, b):
        bh = self.Dr[self.m] * b[self.m]
        return self.lsolve(bh[self.perm])

    def back(self, x_chk):
        xh = np.empty(self.n)
        xh[self.perm] = self.lsolve_T(x_chk)
        return self.Dc * (self.S @ xh)

    def rhs_T(self, g):
        gh = self.S.T @ (self.Dc * g)
        return self.lsolve(gh[self.perm])

    def back_T(self, l_chk):
        y = np.empty(self.n)
        y[self.perm] = self.lsolve_T(l_chk)
        lam = np.empty(self.n)
        lam[self.m] = self.Dr[self.m] * y
        return lam


def setup_ildl(A, opts: SetupOptions | None = None, iopts=None) -> IldlOracleSetup:
    """Setup with the incomplete LDL^T of M_hat (Sec. 3): matching, scaling
    and S as in setup(); then M_hat, J_hat, the factorization, the scaled
    factor, the low-rank term (Fig. 1), the skew-Lanczos basis of J_tilde
    (Fig. 2) and the SMW data."""
    from .ildl import IldlOptions, ildl, low_rank, scaled_factor
    from .split import ahat_on_pattern, symmetric_skew_parts
    opts = opts or SetupOptions()
    iopts = iopts or IldlOptions()
    A = validate_csr(A)
    m = max_product_matching(A)
    Dr, Dc = canonical_scaling(A, m)
    Abar = permute_scale(A, m, Dr, Dc)
    S, _, _ = skew_symmetrizer(Abar, opts.s_pattern, opts.gamma, dense_limit=opts.lls_dense_limit)
    Ahat, _ = ahat_on_pattern(Abar, S)
    Mh, Jh = symmetric_skew_parts(Ahat)
    F = ildl(Mh, iopts)
    Lcal, _, Mr = scaled_factor(F)
    Ur, sig = low_rank(F, Mr)
    p = F.perm
    Ap = sp.csr_matrix(Ahat[p][:, p])
    Jp = sp.csr_matrix(Jh[p][:, p])
    st = IldlOracleSetup(A=A, m=m, Dr=Dr, Dc=Dc, Abar=Abar, S=S, Ahat=Ahat, factor=F, Lcal=Lcal,
                         Mr=Mr, Ur=Ur, sigma_r=sig, Ap=Ap, Jp=Jp, Q=None, alpha=None, prec=None,
                         Ld=Lcal.toarray())
    n = A.shape[0]
    Q, alpha = skew_lanczos(st.jtilde, start_vector(opts.lanczos_seed, n), opts.k)
    st.Q, st.alpha = Q, alpha
    st.prec = Preconditioner(None, None, Q, alpha, opts.x_tol, opts.x_maxit, jtilde=st.jtilde,
                             Ur=Ur, sigma_r=sig)
    return st


def _fgmres(op, prec_apply, rhs, back, true_relres, o: SolveOptions):
    """Flexible GMRES(m) with the stopping rule described in the module doc."""
    n = rhs.size
    info = dict(converged=False, outer_its=0, inner_its_total=0, inner_its_max=0,
                relres_true=np.nan, relres_implicit=np.nan, cycles=0, hist=[], reorth=0)
    bn = np.linalg.norm(rhs)
    x_chk = np.zeros(n)
    if bn == 0.0:
        info.update(converged=True, relres_true=0.0, relres_implicit=0.0)
        return x_chk, info
    thr = o.tol * bn
    m = max(1, o.restart_m)
    first = True
    while True:
        r = rhs.copy() if first else rhs - op(x_chk)
        first = False
        beta = np.linalg.norm(r)
        info["cycles"] += 1
        V = np.zeros((n, m + 1))
        Z = np.zeros((n, m))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        j_used = 0
        implicit_ok = beta <= thr
        if beta > 0:
            V[:, 0] = r / beta
            for j in range(m):
                z, its = prec_apply(V[:, j])
                info["inner_its_total"] += its
                info["inner_its_max"] = max(info["inner_its_max"], its)
                Z[:, j] = z
                w = op(z)
                wn = np.linalg.norm(w)
                h = V[:, :j + 1].T @ w
                w = w - V[:, :j + 1] @ h
                hn = np.linalg.norm(w)
                if hn * hn < 0.1 * wn * wn:          # DGKS: one reorthogonalisation pass
                    h2 = V[:, :j + 1].T @ w
                    w = w - V[:, :j + 1] @ h2
                    h = h + h2
                    hn = np.linalg.norm(w)
                    info["reorth"] += 1
                H[:j + 1, j] = h
                H[j + 1, j] = hn
                if hn != 0.0:
                    V[:, j + 1] = w / hn
                for i in range(j):
                    a, b_ = H[i, j], H[i + 1, j]
                    H[i, j] = cs[i] * a + sn[i] * b_
                    H[i + 1, j] = -sn[i] * a + cs[i] * b_
                rr = np.hypot(H[j, j], H[j + 1, j])
                if rr == 0.0:
                    cs[j], sn[j] = 1.0, 0.0
                else:
                    cs[j], sn[j] = H[j, j] / rr, H[j + 1, j] / rr
                H[j, j] = rr
                H[j + 1, j] = 0.0
                g[j + 1] = -sn[j] * g[j]
                g[j] = cs[j] * g[j]
                info["outer_its"] += 1
                j_used = j + 1
                implicit_ok = abs(g[j + 1]) <= thr
                info["hist"].append(abs(g[j + 1]) / bn)
                if implicit_ok or hn == 0.0 or info["outer_its"] >= o.max_outer:
                    break
            y = np.zeros(j_used)
            for i in range(j_used - 1, -1, -1):          # back substitution
                y[i] = (g[i] - H[i, i + 1:j_used] @ y[i + 1:j_used]) / H[i, i]
            x_chk = x_chk + Z[:, :j_used] @ y
        info["relres_implicit"] = abs(g[j_used]) / bn
        relres = true_relres(back(x_chk))
        info["relres_true"] = relres
        if relres <= o.tol:
            info["converged"] = True
            break
        if info["outer_its"] >= o.max_outer or j_used == 0:
            break          # j_used == 0: zero scaled residual, a restart cannot move
        if implicit_ok:
            thr = thr * 0.5 * o.tol / relres
    return x_chk, info


def _tfqmr(op, prec_apply, rhs, back, true_relres, o: SolveOptions):
    """Transpose-free QMR (Freund 1993) on A_chk P^-1 y = rhs, x_chk = P^-1 y:
    the outer method of the paper's experiments (Sec. 4.1).

    Right preconditioning with the iterate kept in x_chk coordinates: every
    vector u that enters a product gets z = P^-1 u once, the product is
    A_chk z, and the direction d (a combination of the u's) is carried as
    P^-1 d, built from the same z's.  With an exact preconditioner this is
    the textbook method; with the inexact inner solve the update of x_chk
    stays consistent with the products actually formed.  Two half steps per
    iteration (m even: new alpha, u_{m+1} = u_m - alpha v_m; m odd: new rho,
    beta, u_{m+1} = w_{m+1} + beta u_m, v_{m+1}); quasi-minimal residual
    bound ||r_{m+1}|| <= tau_{m+1} sqrt(m + 2).  Stopping as for FGMRES: the
    bound only triggers the true-residual check; a failed check restarts the
    method from x_chk with the threshold tightened; a breakdown ((v, r*) = 0
    or rho = 0) also restarts.  outer_its counts half steps."""
    n = rhs.size
    info = dict(converged=False, outer_its=0, inner_its_total=0, inner_its_max=0,
                relres_true=np.nan, relres_implicit=np.nan, cycles=0, hist=[], reorth=0)
    bn = np.linalg.norm(rhs)
    x_chk = np.zeros(n)
    if bn == 0.0:
        info.update(converged=True, relres_true=0.0, relres_implicit=0.0)
        return x_chk, info
    thr = o.tol * bn

    def pre(u):
        z, its = prec_apply(u)
        info["inner_its_total"] += its
        info["inner_its_max"] = max(info["inner_its_max"], its)
        return z

    first = True
    while True:
        r = rhs.copy() if first else rhs - op(x_chk)
        first = False
        info["cycles"] += 1
        tau = np.linalg.norm(r)
        tau0 = tau
        implicit_ok = tau <= thr
        bound = tau
        if not implicit_ok:
            rstar = r.copy()
            rho = rstar @ r
            w = r.copy()
            u = r.copy()
            z = pre(u)          # P^-1 u_0
            Au = op(z)          # A_chk P^-1 u_0
            v = Au.copy()
            dz = np.zeros(n)
            theta = eta = 0.0
            alpha = 0.0
            m = 0
            while True:
                if m % 2 == 0:
                    sigma = v @ rstar
                    if sigma == 0.0 or rho == 0.0:
                        break                       # breakdown: restart
                    alpha = rho / sigma
                    u_next = u - alpha * v
                    zm, Aum = z, Au                 # u_m = u (product known)
                else:
                    zm = pre(u)                     # u_m = u_next of the even step
                    Aum = op(zm)
                w = w - alpha * Aum
                dz = zm + (theta * theta / alpha) * eta * dz
                theta = np.linalg.norm(w) / tau
                if o.record:
                    info.setdefault("w_norms", []).append(np.linalg.norm(w))
                c = 1.0 / np.sqrt(1.0 + theta * theta)
                tau = tau * theta * c
                eta = c * c * alpha
                x_chk = x_chk + eta * dz
                info["outer_its"] += 1
                bound = tau * np.sqrt(m + 2.0)
                info["hist"].append(bound / bn)
                if o.record:
                    info.setdefault("x_hist", []).append(x_chk.copy())
                implicit_ok = bound <= thr
                if implicit_ok or info["outer_its"] >= o.max_outer:
                    break
                if m % 2 == 1:
                    rho_new = w @ rstar
                    if rho_new == 0.0:
                        break                       # breakdown: restart
                    beta = rho_new / rho
                    rho = rho_new
                    u_new = w + beta * u
                    z = pre(u_new)
                    Au_new = op(z)
                    v = Au_new + beta * (Aum + beta * v)
                    u, Au = u_new, Au_new
                else:
                    u = u_next
                m += 1
        info["relres_implicit"] = bound / bn
        relres = true_relres(back(x_chk))
        info["relres_true"] = relres
        if relres <= o.tol:
            info["converged"] = True
            break
        if info["outer_its"] >= o.max_outer or tau0 == 0.0:
            break          # zero scaled residual: a restart cannot move
        if implicit_ok:
            thr = thr * 0.5 * o.tol / relres
    return x_chk, info


def _outer(o: SolveOptions):
    if o.outer == "fgmres":
        return _fgmres
    if o.outer == "tfqmr":
        return _tfqmr
    raise ValueError(f"unknown outer method {o.outer!r}")


def _from_x0(solve_fn, M, st, b, o, x0):
    """Start from an initial guess x0 (not in the paper; the solver's option).
    The outer method corrects r0 = b - M x0 to the relative tolerance
    tol ||b|| / ||r0||, and x = x0 + d: the right-preconditioned residual of
    the transformed x0 is the transformed r0, so this is the iteration started
    at x0 without applying S^-1.  The true residual reported is that of x
    against b."""
    x0 = np.asarray(x0, dtype=np.float64)
    if not np.all(np.isfinite(x0)):
        raise ValueError("x0 has non-finite entries")
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return solve_fn(st, b, o)
    r0 = b - M @ x0
    rn = np.linalg.norm(r0)
    if rn <= o.tol * bn:
        return x0.copy(), dict(converged=True, outer_its=0, inner_its_total=0, inner_its_max=0,
                               relres_true=rn / bn, relres_implicit=0.0, cycles=0,
                               k_eff=st.Q.shape[1], rank_r=st.rank_r)
    d, info = solve_fn(st, r0, dataclasses.replace(o, tol=o.tol * bn / rn))
    x = x0 + d
    rel = np.linalg.norm(b - M @ x) / bn
    info.update(relres_true=rel, converged=bool(rel <= o.tol))
    return x, info


def solve(st: OracleSetup, b: np.ndarray, o: SolveOptions | None = None, x0=None):
    """x with A x = b (Sec. 3), from x0 if given.  Returns (x, info)."""
    o = o or SolveOptions()
    b = np.asarray(b, dtype=np.float64)
    if not np.all(np.isfinite(b)):
        raise ValueError("b has non-finite entries")
    if x0 is not None:
        return _from_x0(solve, st.A, st, b, o, x0)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros(st.n), dict(converged=True, outer_its=0, inner_its_total=0,
                                    inner_its_max=0, relres_true=0.0, relres_implicit=0.0,
                                    cycles=0, k_eff=st.Q.shape[1], rank_r=st.rank_r)

    def true_relres(x):
        return np.linalg.norm(b - st.A @ x) / bn

    prec = lambda v: st.prec.apply(v, o.inner_tol, o.inner_maxit, o.fixed_inner_steps)
    x_chk, info = _outer(o)(st.op, prec, st.rhs(b), st.back, true_relres, o)
    info.update(k_eff=st.Q.shape[1], rank_r=st.rank_r)
    return st.back(x_chk), info


def solve_adjoint(st: OracleSetup, g: np.ndarray, o: SolveOptions | None = None, x0=None):
    """lambda with A^T lambda = g: FGMRES on A_chk^T right-preconditioned with P^T,
    from x0 if given.  Returns (lambda, info)."""
    o = o or SolveOptions()
    g = np.asarray(g, dtype=np.float64)
    if not np.all(np.isfinite(g)):
        raise ValueError("g has non-finite entries")
    if x0 is not None:
        return _from_x0(solve_adjoint, st.A.T.tocsr(), st, g, o, x0)
    gn = np.linalg.norm(g)
    if gn == 0.0:
        return np.zeros(st.n), dict(converged=True, outer_its=0, inner_its_total=0,
                                    inner_its_max=0, relres_true=0.0, relres_implicit=0.0,
                                    cycles=0, k_eff=st.Q.shape[1], rank_r=st.rank_r)

    def true_relres(lam):
        return np.linalg.norm(g - st.A.T @ lam) / gn

    prec = lambda v: st.prec.apply_T(v, o.inner_tol, o.inner_maxit, o.fixed_inner_steps)
    l_chk, info = _outer(o)(st.op_T, prec, st.rhs_T(g), st.back_T, true_relres, o)
    info.update(k_eff=st.Q.shape[1], rank_r=st.rank_r)
    return st.back_T(l_chk), info


def value_gradient(A, lam: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Derivative of a loss L(x) with respect to the stored values of A, for
    x = A^-1 b and lam = A^-T dL/dx.

    Differentiating A x = b gives A dx = -dA x, so dL = lam^T dx =
    -sum_ij lam_i dA_ij x_j: the entry (i, j) gets -lam_i x_j.  Returned in
    the order of A's CSR storage (the adjoint is the transposed two-level
    scheme, Sec. 3 eqs. modified and smw taken by transposition)."""
    import scipy.sparse as sp
    A = sp.csr_matrix(A)
    out = np.empty(A.nnz)
    for i in range(A.shape[0]):
        for e in range(A.indptr[i], A.indptr[i + 1]):
            out[e] = -lam[i] * x[A.indices[e]]
    return out
