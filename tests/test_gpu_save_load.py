"""Saved setups (asss_save / asss_load): a loaded handle has the saved
matching, scalings and S bit for bit, rebuilds A_hat, D and J_tilde from them
exactly, the skew-Lanczos vectors to rounding, and solves like the saved
handle and the oracle; the layout (caller's order, autotuned row block,
column form) and values set by asss_update_values survive the round trip."""
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


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_round_trip_matches_saved_handle_and_oracle(tmp_path):
    asss = _lib()
    w = W.config(0)
    h = asss.setup(w.A, k=8, s_pattern="tridiag")
    path = tmp_path / "cfg0.asss"
    h.save(path)
    g = asss.load_handle(path)
    ih, ig = h.info(), g.info()
    for key in ("n", "nnz_a", "nnz_s", "nnz_ahat", "nh", "k_eff", "rank_r", "row_block", "nblocks",
                "sell_entries_a", "sell_entries_b", "skew_form", "reordered"):
        assert ih[key] == ig[key], key
    assert ig["lls_its"] == 0  # no least-squares solve on load
    for name in ("match", "Dr", "Dc", "S_rowptr", "S_colind", "S_val", "D", "J_rowptr", "J_colind", "J_val"):
        assert np.array_equal(h.array(name), g.array(name)), name
    n = w.A.shape[0]
    assert _rel(g.array("Q").reshape(8, n).T, h.array("Q").reshape(8, n).T) <= 1e-10
    b = torch.from_numpy(w.b).cuda()
    x1, i1 = h.solve(b, tol=1e-12)
    x2, i2 = g.solve(b, tol=1e-12)
    assert i1["status"] == "OK" and i2["status"] == "OK"
    st = O.setup(w.A, O.SetupOptions(k=8, s_pattern="tridiag"))
    xo, _ = O.solve(st, w.b, O.SolveOptions(tol=1e-12))
    assert _rel(_np(x2), _np(x1)) <= 1e-11 and _rel(_np(x2), xo) <= 1e-10
    h.close()
    g.close()


def test_round_trip_keeps_layout_and_updated_values(tmp_path):
    asss = _lib()
    m = 24
    w = W.convdiff3d(m=m, peclet=100.0, cfg=1)
    h = asss.setup(w.A, k=8, s_pattern="abar", reorder=W.grid_line_tiles(m, 4, 2), autotune=True)
    A2 = w.A.copy()
    A2.data = A2.data * (1.0 + 0.01 * np.random.default_rng(4).standard_normal(A2.nnz))
    h.update_values(A2)
    path = tmp_path / "cd.asss"
    h.save(path)
    g = asss.load_handle(path, allocator="torch")
    ih, ig = h.info(), g.info()
    for key in ("row_block", "skew_form", "reordered", "nh", "k_eff"):
        assert ih[key] == ig[key], key
    assert ig["reordered"] == 1 and ig["tune_n"] == 0
    b = torch.from_numpy(w.b).cuda()
    x, info = g.solve(b, tol=1e-10, restart_m=100, inner_tol=0.2)
    assert info["status"] == "OK"
    assert np.linalg.norm(w.b - A2 @ _np(x)) <= 1.01e-10 * np.linalg.norm(w.b)  # the updated matrix
    h.close()
    g.close()
