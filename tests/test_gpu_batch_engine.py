"""The lockstep batch engine of asss_solve_batched: all systems' rows
concatenated, one persistent work-queue launch per inner step for every
system (replayed from HIP graph chunks), segmented outer kernels, one host
round trip per outer step.  Checked against the oracle's per-system solves on
a subset of the 64-system draw of the batched workload, against the
per-system worker path, and on restarts, uneven column counts, zero columns,
r > 0 and repeated solves."""
import numpy as np
import pytest
import scipy.sparse as sp

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


def _colmajor(B):
    return torch.from_numpy(np.ascontiguousarray(B.T)).cuda().t()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def draw():
    """The 64 systems of the batched workload (n log-uniform in [1e4, 5e5],
    h ~ U(0.01, 0.5), 4 right-hand sides each), set up once."""
    asss = _lib()
    ws = W.batched_implicit_euler(nsys=64, nrhs=4, cfg=3)
    print(f"[engine] 64 systems, n {min(w.A.shape[0] for w in ws)}..{max(w.A.shape[0] for w in ws)}", flush=True)
    hs = [asss.setup(w.A, k=8, s_pattern="tridiag") for w in ws]
    Bs = [_colmajor(w.b) for w in ws]
    yield asss, ws, hs, Bs
    for h in hs:
        h.close()


def _subset(ws, count=4, nmax=40000):
    """The smallest systems of the draw (the oracle solves them in seconds)."""
    order = sorted(range(len(ws)), key=lambda s: ws[s].A.shape[0])
    return [s for s in order if ws[s].A.shape[0] <= nmax][:count]


def test_engine_mixed_precision_on_the_draw(draw):
    """The workload's options (FP32 inner, FGMRES(64), inner tolerance 1e-2,
    tol 1e-8): every column converges with its true residual (recomputed on
    the host) below 1e-8, and on the smallest systems x lies within 1e-7 of
    the FP64 oracle's x (kappa of these systems is a few units)."""
    asss, ws, hs, Bs = draw
    Xs, infos = asss.solve_batched(hs, Bs, tol=1e-8, inner_fp32=True, restart_m=64, inner_tol=1e-2,
                                   batch_engine="lockstep")
    for s, w in enumerate(ws):
        X = Xs[s].detach().cpu().numpy()
        for j in range(4):
            inf = infos[s][j]
            assert inf["converged"] == 1, (s, j, inf)
            r = np.linalg.norm(w.b[:, j] - w.A @ X[:, j]) / np.linalg.norm(w.b[:, j])
            assert r <= 1e-8 * 1.01, (s, j, r)
    for s in _subset(ws):
        w = ws[s]
        st = O.setup(w.A, O.SetupOptions(k=8, s_pattern="tridiag"))
        X = Xs[s].detach().cpu().numpy()
        for j in range(4):
            xo, _ = O.solve(st, w.b[:, j], O.SolveOptions(tol=1e-13))
            err = _rel(X[:, j], xo)
            print(f"[engine] system {s} n={w.A.shape[0]} col {j}: mixed vs oracle {err:.2e}", flush=True)
            assert err <= 1e-7


def test_engine_fp64_parity_on_the_draw(draw):
    """P1 on the subset: FP64 inner, both solved to 1e-12 / 1e-13, x within
    1e-10 of the oracle's."""
    asss, ws, hs, Bs = draw
    sub = _subset(ws)
    Xs, infos = asss.solve_batched([hs[s] for s in sub], [Bs[s] for s in sub], tol=1e-12, inner_fp32=False,
                                   restart_m=64, inner_tol=1e-5, batch_engine="lockstep")
    for q, s in enumerate(sub):
        w = ws[s]
        st = O.setup(w.A, O.SetupOptions(k=8, s_pattern="tridiag"))
        X = Xs[q].detach().cpu().numpy()
        for j in range(4):
            assert infos[q][j]["converged"] == 1
            xo, _ = O.solve(st, w.b[:, j], O.SolveOptions(tol=1e-13))
            assert _rel(X[:, j], xo) <= 1e-10, (s, j)


def test_engine_matches_workers(draw):
    """The engine and the per-system workers solve the same columns to the
    same x (FP64 inner, tol 1e-12) on eight systems of the draw."""
    asss, ws, hs, Bs = draw
    sub = list(range(0, 64, 8))
    kw = dict(tol=1e-12, inner_fp32=False, restart_m=64, inner_tol=1e-5)
    Xe, ie = asss.solve_batched([hs[s] for s in sub], [Bs[s] for s in sub], batch_engine="lockstep", **kw)
    Xw, iw = asss.solve_batched([hs[s] for s in sub], [Bs[s] for s in sub], batch_engine="workers", **kw)
    for q in range(len(sub)):
        a, b = Xe[q].detach().cpu().numpy(), Xw[q].detach().cpu().numpy()
        for j in range(4):
            assert ie[q][j]["converged"] == 1 and iw[q][j]["converged"] == 1
            assert _rel(a[:, j], b[:, j]) <= 1e-9, (q, j)


def test_engine_repeated_solves(draw):
    """Three solves in a row (graph replays with eager work and
    synchronisations between them) give the same solutions to rounding."""
    asss, ws, hs, Bs = draw
    sub = list(range(3, 64, 16))
    kw = dict(tol=1e-8, inner_fp32=True, restart_m=64, inner_tol=1e-2, batch_engine="lockstep")
    ref = None
    for rep in range(3):
        Xs, infos = asss.solve_batched([hs[s] for s in sub], [Bs[s] for s in sub], **kw)
        torch.cuda.synchronize()
        cur = [X.detach().cpu().numpy() for X in Xs]
        if ref is None:
            ref = cur
        else:
            for a, b in zip(cur, ref):
                assert _rel(a, b) <= 1e-12


def _stand_in_with_r():
    for seed in range(10):
        A = W.paper_like(200, 1200, seed=seed).A
        st = O.setup(A, O.SetupOptions(k=5, gamma=0.01))
        if st.N.size > 0:
            return A, st
    pytest.skip("no negative-diagonal case")


def test_engine_restarts_and_uneven_columns():
    """Short restarts (m = 3), so that columns end and restart cycles at
    different steps; systems with 4, 1 and 3 right-hand sides, one of them
    zero; against the oracle (same restart length) and dense solves."""
    asss = _lib()
    ws = W.batched_implicit_euler(nsys=3, n_lo=400, n_hi=2500, nrhs=4, cfg=3)
    hs = [asss.setup(w.A, k=8, s_pattern="tridiag") for w in ws]
    sts = [O.setup(w.A, O.SetupOptions(k=8, s_pattern="tridiag")) for w in ws]
    rng = np.random.default_rng(4)
    nr = [4, 1, 3]
    Bn = [rng.standard_normal((w.A.shape[0], r)) for w, r in zip(ws, nr)]
    Bn[2][:, 1] = 0.0  # a zero right-hand side
    try:
        Xs, infos = asss.solve_batched(hs, [_colmajor(B) for B in Bn], tol=1e-10, inner_fp32=False, restart_m=3,
                                       inner_tol=1e-6, batch_engine="lockstep")
        for s, (w, B, st) in enumerate(zip(ws, Bn, sts)):
            X = Xs[s].detach().cpu().numpy()
            Ad = w.A.toarray()
            bound = max(1e-9, 10 * np.linalg.cond(Ad) * 1e-10)
            for j in range(B.shape[1]):
                inf = infos[s][j]
                assert inf["converged"] == 1, (s, j, inf)
                if not B[:, j].any():
                    assert not X[:, j].any() and inf["outer_its"] == 0
                    continue
                assert inf["cycles"] >= 2
                xo, _ = O.solve(st, B[:, j], O.SolveOptions(tol=1e-12, restart_m=3, inner_tol=1e-6))
                assert _rel(X[:, j], np.linalg.solve(Ad, B[:, j])) <= bound, (s, j)
                assert _rel(X[:, j], xo) <= bound, (s, j)
    finally:
        for h in hs:
            h.close()


def test_engine_low_rank_term():
    """A stand-in matrix with negative diagonal entries after the
    skew-symmetrizer (r > 0: the low-rank term of Fig. 1 in the SMW form),
    batched with two implicit-Euler systems, b = A 1 for the stand-in (as in
    its one-system test; kappa ~ 1e10): every column reaches tol on its true
    residual (recomputed on the host), the stand-in's x agrees with the
    one-system solve and the oracle's within 10 kappa tol, and the other
    systems match the oracle."""
    asss = _lib()
    A, st_neg = _stand_in_with_r()
    ws = W.batched_implicit_euler(nsys=2, n_lo=400, n_hi=1500, nrhs=4, cfg=3)
    mats = [A] + [w.A for w in ws]
    hs = [asss.setup(A, k=5, gamma=0.01)] + [asss.setup(w.A, k=8, s_pattern="tridiag") for w in ws]
    rng = np.random.default_rng(5)
    Bn = [np.stack([A @ np.ones(A.shape[0]), A @ np.ones(A.shape[0])], axis=1)]
    Bn += [rng.standard_normal((M.shape[0], 2)) for M in mats[1:]]
    try:
        assert hs[0].info()["rank_r"] == st_neg.N.size > 0
        Xs, infos = asss.solve_batched(hs, [_colmajor(B) for B in Bn], tol=1e-10, inner_fp32=False, restart_m=64,
                                       batch_engine="lockstep")
        kappa = np.linalg.cond(A.toarray())
        x1, i1 = hs[0].solve(torch.from_numpy(Bn[0][:, 0].copy()).cuda(), tol=1e-10)
        xo, _ = O.solve(st_neg, Bn[0][:, 0], O.SolveOptions(tol=1e-10))
        for s, (M, B) in enumerate(zip(mats, Bn)):
            X = Xs[s].detach().cpu().numpy()
            for j in range(2):
                print(f"[engine] low-rank batch: system {s} col {j}: {infos[s][j]['outer_its']} outer, "
                      f"relres {infos[s][j]['relres_true']:.2e}", flush=True)
                assert infos[s][j]["converged"] == 1, (s, j, infos[s][j])
                r = np.linalg.norm(B[:, j] - M @ X[:, j]) / np.linalg.norm(B[:, j])
                assert r <= 1.01e-10, (s, j, r)
                if s == 0:
                    bound = max(1e-9, 10 * kappa * 1e-10)
                    assert _rel(X[:, j], x1.cpu().numpy()) <= bound and _rel(X[:, j], xo) <= bound
                else:
                    st = O.setup(M, O.SetupOptions(k=8, s_pattern="tridiag"))
                    xr, _ = O.solve(st, B[:, j], O.SolveOptions(tol=1e-12))
                    assert _rel(X[:, j], xr) <= 1e-9
        assert i1["status"] == "OK"
    finally:
        for h in hs:
            h.close()
