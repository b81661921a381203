"""The caller's order of the inner system (setup option reorder = 3,
inner_perm): a symmetric permutation of J_tilde that must be invisible in
every result (exported Q_k, the skew operator, the inner mrs, full solves) up
to rounding, checked against the FP64 oracle; bad permutations are rejected;
on a 3D grid, tiles of whole x-lines keep more pairs inside a row block than
the natural order."""
import numpy as np
import pytest

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


def _cuda(v):
    return torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda()


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def test_random_caller_order_matches_the_oracle():
    asss = _lib()
    w = W.config(0, m=40)
    n = w.A.shape[0]
    st = O.setup(w.A, O.SetupOptions(k=6))
    perm = np.random.default_rng(5).permutation(n)
    print(f"[order] random permutation, n={n}", flush=True)
    hp = asss.setup(w.A, k=6, reorder=perm, row_block=64)
    hn = asss.setup(w.A, k=6, reorder="none", row_block=64)
    ip = hp.info()
    assert ip["reordered"] == 1 and hn.info()["reordered"] == 0
    assert ip["cross_pairs_natural"] == hn.info()["cross_pairs_used"]
    assert _rel(hp.array("Q").reshape(6, -1).T, st.Q) <= 1e-10
    v = np.random.default_rng(31).standard_normal(n)
    for op, ref in (("skew", st.prec.jtilde(v)), ("mrs", O.mrs(1.0, st.prec.jbar, v, 20, 0.0, 20)[0])):
        kw = {"fixed_inner_steps": 20} if op == "mrs" else {}
        op_p, _ = hp.apply(op, _cuda(v), **kw)
        op_n, _ = hn.apply(op, _cuda(v), **kw)
        assert _rel(_np(op_p), _np(op_n)) <= 1e-12, op
        assert _rel(_np(op_p), ref) <= 1e-10, op
    xo, _ = O.solve(st, w.b, O.SolveOptions(tol=1e-12))
    for mixed in (False, True):
        x, info = hp.solve(_cuda(w.b), tol=1e-12 if not mixed else 1e-8, inner_fp32=mixed)
        assert info["status"] == "OK"
        assert _rel(_np(x), xo) <= (1e-10 if not mixed else 1e-7)
    lam_p, _ = hp.solve_adjoint(_cuda(w.b), tol=1e-12)
    lam_n, _ = hn.solve_adjoint(_cuda(w.b), tol=1e-12)
    assert _rel(_np(lam_p), _np(lam_n)) <= 1e-10
    hp.close()
    hn.close()


def test_bad_caller_order_is_rejected():
    asss = _lib()
    w = W.config(0, m=12)
    n = w.A.shape[0]
    for bad in (np.zeros(n, np.int32), np.arange(1, n + 1), np.r_[np.arange(n - 1), -1]):
        with pytest.raises(asss.AsssError) as e:
            asss.setup(w.A, k=4, reorder=bad)
        assert e.value.name == "INVALID_ARG"
    with pytest.raises(ValueError):
        asss.setup(w.A, k=4, reorder=np.arange(n - 1))


def test_line_tiles_on_a_3d_grid():
    """48^3 convection-diffusion, blocks of 768 rows: one 48 x 4 x 4 tile of
    x-lines per block against 16 consecutive x-lines of one plane."""
    asss = _lib()
    m = 48
    w = W.convdiff3d(m=m, peclet=100.0, cfg=1)
    perm = W.grid_line_tiles(m, 4, 4)
    print(f"[order] {m}^3 line tiles 4x4, row_block 768", flush=True)
    ht = asss.setup(w.A, k=8, s_pattern="tridiag", reorder=perm, row_block=768)
    hn = asss.setup(w.A, k=8, s_pattern="tridiag", row_block=768)
    it, i_n = ht.info(), hn.info()
    print(f"[order] stored entries a {i_n['sell_entries_a']} -> {it['sell_entries_a']}, "
          f"b {i_n['sell_entries_b']} -> {it['sell_entries_b']}", flush=True)
    assert it["cross_pairs_used"] < 0.7 * i_n["cross_pairs_used"]
    assert it["sell_entries_a"] + it["sell_entries_b"] < i_n["sell_entries_a"] + i_n["sell_entries_b"]
    assert it["skew_form"] == 3  # offset slots
    v = np.random.default_rng(3).uniform(-1, 1, m ** 3)
    yt, _ = ht.apply("skew", _cuda(v))
    yn, _ = hn.apply("skew", _cuda(v))
    assert _rel(_np(yt), _np(yn)) <= 1e-13
    b = _cuda(w.b)
    for mixed in (False, True):
        xt, infot = ht.solve(b, tol=1e-10, restart_m=100, inner_tol=0.2, inner_fp32=mixed)
        xn, infon = hn.solve(b, tol=1e-10, restart_m=100, inner_tol=0.2, inner_fp32=mixed)
        assert infot["status"] == "OK" and infon["status"] == "OK"
        a = _np(xt)
        assert np.linalg.norm(w.b - w.A @ a) <= 1.01e-10 * np.linalg.norm(w.b)
        assert _rel(a, _np(xn)) <= 1e-6
    # the caller's order with the row-block autotuner: candidates packed in that order
    ha = asss.setup(w.A, k=8, s_pattern="tridiag", reorder=perm, autotune=True)
    ia = ha.info()
    assert ia["reordered"] == 1 and ia["tune_n"] >= 2 and ia["row_block"] in ia["tune_rows"]
    xa, infoa = ha.solve(b, tol=1e-10, restart_m=100, inner_tol=0.2)
    assert infoa["status"] == "OK"
    assert np.linalg.norm(w.b - w.A @ _np(xa)) <= 1.01e-10 * np.linalg.norm(w.b)
    ha.close()
    ht.close()
    hn.close()


def test_library_grid_order():
    """reorder="grid": the library finds the lexicographic 3D grid in the
    pattern of Abar and lays the inner system out in tiles of whole x-lines;
    on 64^3 (automatic row block 256) that is the 2 x 2 line tiling the
    caller could pass, and the solution does not change.  A 2D grid and a
    random pattern keep the natural order."""
    asss = _lib()
    m = 64
    w = W.convdiff3d(m=m, peclet=100.0, cfg=1)
    hg = asss.setup(w.A, k=8, s_pattern="tridiag", reorder="grid")
    hc = asss.setup(w.A, k=8, s_pattern="tridiag", reorder=W.grid_line_tiles(m, 2, 2), row_block=256)
    ig, ic = hg.info(), hc.info()
    assert ig["reordered"] == 1 and ig["row_block"] == 256
    for key in ("cross_pairs_used", "sell_entries_a", "sell_entries_b", "skew_form"):
        assert ig[key] == ic[key], key
    b = _cuda(w.b)
    xg, info = hg.solve(b, tol=1e-10, restart_m=100, inner_tol=0.2)
    assert info["status"] == "OK"
    assert np.linalg.norm(w.b - w.A @ _np(xg)) <= 1.01e-10 * np.linalg.norm(w.b)
    hg.close()
    hc.close()
    for A in (W.config(0).A, W.paper_like(2000, 12000, seed=1).A):
        h = asss.setup(A, k=4, reorder="grid")
        assert h.info()["reordered"] == 0
        h.close()
