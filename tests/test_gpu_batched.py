"""Batched solves (several uneven systems, several right-hand sides each)
through asss_solve_batched: FGMRES columns of a system advance in lockstep
with one simultaneous inner mrs (App. B) per step.  Checked against the oracle
(per-system solves) and dense solves, against column-by-column solves, and on
the error path."""
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
    """(n, nrhs) float64 CUDA tensor with column-major storage."""
    return torch.from_numpy(np.ascontiguousarray(B.T)).cuda().t()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def batch():
    asss = _lib()
    ws = W.batched_implicit_euler(nsys=4, n_lo=400, n_hi=3000, nrhs=4, cfg=3)
    nr = [4, 3, 1, 2]
    hs = [asss.setup(w.A, k=8, s_pattern="tridiag") for w in ws]
    print("[batch] sizes", [w.A.shape[0] for w in ws], "h", [round(w.meta["h"], 3) for w in ws], flush=True)
    yield asss, ws, nr, hs
    for h in hs:
        h.close()


def test_batched_against_oracle_and_dense(batch):
    asss, ws, nr, hs = batch
    Bs = [_colmajor(w.b[:, :r]) for w, r in zip(ws, nr)]
    Xs, infos = asss.solve_batched(hs, Bs, tol=1e-10)
    for s, (w, r) in enumerate(zip(ws, nr)):
        X = Xs[s].detach().cpu().numpy()
        st = O.setup(w.A, O.SetupOptions(k=8, s_pattern="tridiag"))
        Ad = w.A.toarray()
        kappa = np.linalg.cond(Ad)
        for j in range(r):
            inf = infos[s][j]
            assert inf["converged"] == 1 and inf["relres_true"] <= 1e-10, inf
            xo, io = O.solve(st, w.b[:, j], O.SolveOptions(tol=1e-12))
            xd = np.linalg.solve(Ad, w.b[:, j])
            bound = max(1e-9, 10 * kappa * 1e-10)
            assert _rel(X[:, j], xd) <= bound and _rel(X[:, j], xo) <= bound, (s, j, kappa)


def test_batched_block_matches_single_columns(batch):
    asss, ws, nr, hs = batch
    w, h = ws[0], hs[0]
    B = w.b[:, :4]
    Xs, infos = asss.solve_batched([h], [_colmajor(B)], tol=1e-12)
    X = Xs[0].detach().cpu().numpy()
    for j in range(4):
        x, info = h.solve(torch.from_numpy(B[:, j].copy()).cuda(), tol=1e-12)
        assert info["status"] == "OK"
        assert _rel(X[:, j], x.cpu().numpy()) <= 1e-9
    # the block shares one inner solve per outer step: its inner count is the
    # same for every column of the block
    assert len({i["inner_its_total"] for i in infos[0]}) <= 4


def test_batched_mixed_precision_and_tfqmr(batch):
    asss, ws, nr, hs = batch
    Bs = [_colmajor(w.b[:, :r]) for w, r in zip(ws, nr)]
    for kw in (dict(inner_fp32=True), dict(outer="tfqmr")):
        Xs, infos = asss.solve_batched(hs, Bs, tol=1e-8, **kw)
        for s, (w, r) in enumerate(zip(ws, nr)):
            X = Xs[s].detach().cpu().numpy()
            Ad = w.A.toarray()
            kappa = np.linalg.cond(Ad)
            for j in range(r):
                assert infos[s][j]["relres_true"] <= 1e-8, (kw, s, j)
                xd = np.linalg.solve(Ad, w.b[:, j])
                assert _rel(X[:, j], xd) <= max(1e-7, 10 * kappa * 1e-8), (kw, s, j)


def test_batched_rejects_nonfinite(batch):
    asss, ws, nr, hs = batch
    B = ws[1].b[:, :3].copy()
    B[7, 2] = np.nan
    with pytest.raises(asss.AsssError, match="NONFINITE"):
        asss.solve_batched([hs[0], hs[1]], [_colmajor(ws[0].b[:, :2]), _colmajor(B)], tol=1e-8)


def test_batched_many_deflation_vectors():
    """k = 20 exceeds the 4-column kernels: the batched solve falls back to
    one column at a time and still matches dense solves."""
    asss = _lib()
    w = W.batched_implicit_euler(nsys=1, n_lo=900, n_hi=1200, nrhs=3, cfg=3)[0]
    h = asss.setup(w.A, k=20, s_pattern="tridiag")
    Xs, infos = asss.solve_batched([h], [_colmajor(w.b)], tol=1e-10)
    X = Xs[0].detach().cpu().numpy()
    Ad = w.A.toarray()
    for j in range(3):
        assert infos[0][j]["converged"] == 1
        assert _rel(X[:, j], np.linalg.solve(Ad, w.b[:, j])) <= max(1e-8, 10 * np.linalg.cond(Ad) * 1e-10)
    h.close()


def test_batched_same_handle_twice_and_many_systems(batch):
    """Systems run concurrently on worker streams; a handle listed twice stays
    on one worker.  Every column matches its own single solve."""
    asss, ws, nr, hs = batch
    order = [0, 1, 0, 2, 3, 1]
    Bs = [_colmajor(ws[i].b[:, :2]) for i in order]
    Xs, infos = asss.solve_batched([hs[i] for i in order], Bs, tol=1e-11)
    for t, i in enumerate(order):
        X = Xs[t].detach().cpu().numpy()
        for j in range(2):
            assert infos[t][j]["converged"] == 1
            x, _ = hs[i].solve(torch.from_numpy(ws[i].b[:, j].copy()).cuda(), tol=1e-11)
            assert _rel(X[:, j], x.cpu().numpy()) <= 1e-8


def test_batched_with_torch_allocator_and_autotune():
    """Handles whose memory comes from torch's caching allocator grow their
    lockstep workspace from the worker threads of the batched solve; row
    blocks chosen by the autotuner.  Every column matches a dense solve and
    all memory goes back to torch at destroy."""
    asss = _lib()
    ws = W.batched_implicit_euler(nsys=3, n_lo=1500, n_hi=6000, nrhs=4, cfg=3)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    hs = [asss.setup(w.A, k=8, s_pattern="tridiag", allocator="torch", autotune=True) for w in ws]
    for h in hs:
        i = h.info()
        assert i["tune_n"] >= 2 and i["row_block"] in i["tune_rows"]
    Bs = [_colmajor(w.b) for w in ws] + [_colmajor(ws[0].b[:, :2])]
    Xs, infos = asss.solve_batched(hs + hs[:1], Bs, tol=1e-10)
    for s, w in enumerate(ws + ws[:1]):
        X = Xs[s].detach().cpu().numpy()
        Ad = w.A.toarray()
        tol_x = max(1e-8, 10 * np.linalg.cond(Ad) * 1e-10)
        for j in range(X.shape[1]):
            assert infos[s][j]["converged"] == 1
            assert _rel(X[:, j], np.linalg.solve(Ad, w.b[:, j])) <= tol_x
    del Xs, Bs
    for h in hs:
        h.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


def test_batch_streams_option(batch):
    """The per-system workers: any number of worker streams gives the same columns up to the solve's
    tolerance (the in-block LDS scatter adds in a run-dependent order);
    values outside [0, 16] are refused."""
    asss, ws, nr, hs = batch
    Bs = [_colmajor(w.b[:, :r]) for w, r in zip(ws, nr)]
    ref, _ = asss.solve_batched(hs, Bs, tol=1e-11, batch_streams=1, batch_engine="workers")
    for ns in (2, 3, 16):
        Xs, infos = asss.solve_batched(hs, Bs, tol=1e-11, batch_streams=ns, batch_engine="workers")
        for s in range(len(ws)):
            assert all(i["converged"] == 1 for i in infos[s])
            assert _rel(Xs[s].cpu().numpy(), ref[s].cpu().numpy()) <= 1e-8
    for bad in (-1, 17):
        with pytest.raises(asss.AsssError) as e:
            asss.solve_batched(hs, Bs, tol=1e-8, batch_streams=bad)
        assert e.value.name == "INVALID_ARG"


def test_batched_initial_guesses(batch):
    """X0s: every column starts from its own guess (one at a time) and reaches
    the dense solution; exact guesses come back after no outer step."""
    asss, ws, nr, hs = batch
    Bs = [_colmajor(w.b[:, :r]) for w, r in zip(ws, nr)]
    Xd = [np.linalg.solve(w.A.toarray(), w.b[:, :r]) for w, r in zip(ws, nr)]
    rng = np.random.default_rng(11)
    X0 = [_colmajor(x + 1e-3 * rng.standard_normal(x.shape)) for x in Xd]
    Xs, infos = asss.solve_batched(hs, Bs, X0s=X0, tol=1e-11)
    for s, w in enumerate(ws):
        X = Xs[s].detach().cpu().numpy()
        kappa = np.linalg.cond(w.A.toarray())
        for j in range(nr[s]):
            assert infos[s][j]["converged"] == 1
            assert _rel(X[:, j], Xd[s][:, j]) <= max(1e-8, 10 * kappa * 1e-11)
    Xs, infos = asss.solve_batched(hs, Bs, X0s=[_colmajor(x) for x in Xd], tol=1e-8)
    assert all(i["outer_its"] == 0 for row in infos for i in row)
