"""Row-block autotuner (setup option autotune): the layout it keeps is the
fastest of the candidates it timed, it is the layout an explicit row_block of
that size gives, and it holds the same operator as the automatic size (the
skew operator J_tilde, the FP64 inner mrs solve of App. B and the outer
solve agree to rounding).  Sizes: a 64^3 convection-diffusion grid
(n = 262,144, automatic row block 256, candidates 64 ... 1024)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def handles():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_06954_amd as asss
    asss.load()
    w = W.convdiff3d(m=64, peclet=100.0, cfg=1)
    print("[autotune] setup with autotune, n =", w.A.shape[0], flush=True)
    ht = asss.setup(w.A, k=8, s_pattern="tridiag", autotune=True)
    print("[autotune]", {k: v for k, v in ht.info().items() if k.startswith("tune") or k == "row_block"},
          flush=True)
    h0 = asss.setup(w.A, k=8, s_pattern="tridiag")
    hr = asss.setup(w.A, k=8, s_pattern="tridiag", row_block=ht.info()["row_block"])
    yield dict(w=w, ht=ht, h0=h0, hr=hr)
    for h in (ht, h0, hr):
        h.close()


def test_autotune_keeps_the_fastest_candidate(handles):
    it, i0 = handles["ht"].info(), handles["h0"].info()
    n = i0["n"]
    assert i0["tune_n"] == 0 and i0["row_block"] == 256
    assert it["tune_rows"] == [64, 128, 256, 512, 1024]
    assert all(t > 0 for t in it["tune_us"]) and it["tune_s"] > 0
    best = it["tune_rows"][int(np.argmin(it["tune_us"]))]
    assert it["row_block"] == best and it["nblocks"] == -(-n // best)


def test_autotuned_layout_equals_explicit_row_block(handles):
    it, ir = handles["ht"].info(), handles["hr"].info()
    for key in ("row_block", "nblocks", "sell_entries_a", "sell_entries_b", "narrow_b_columns", "skew_form",
                "cross_pairs_natural", "k_eff"):
        assert it[key] == ir[key], key


def test_autotuned_handle_applies_the_same_operators(handles):
    ht, h0 = handles["ht"], handles["h0"]
    n = handles["w"].A.shape[0]
    v = torch.from_numpy(np.random.default_rng(7).uniform(-1, 1, n)).cuda()
    # skew: rounding of a different summation order; mrs at inner tolerance
    # 1e-12: both residuals <= 1e-12 |v| and |(I + J)^-1| <= 1 for skew J
    for op, rel in (("skew", 1e-13), ("mrs", 1e-9)):
        yt, _ = ht.apply(op, v, inner_tol=1e-12, inner_maxit=3000)
        y0, _ = h0.apply(op, v, inner_tol=1e-12, inner_maxit=3000)
        a, b = _np(yt), _np(y0)
        assert np.linalg.norm(a - b) <= rel * np.linalg.norm(b), op


def test_autotuned_handle_solves_to_the_same_solution(handles):
    w, ht, h0 = handles["w"], handles["ht"], handles["h0"]
    b = torch.from_numpy(w.b).cuda()
    xt, it = ht.solve(b, tol=1e-11, restart_m=100, inner_tol=0.2)
    x0, i0 = h0.solve(b, tol=1e-11, restart_m=100, inner_tol=0.2)
    assert it["converged"] and i0["converged"]
    a, c = _np(xt), _np(x0)
    for x in (a, c):
        assert np.linalg.norm(w.b - w.A @ x) <= 1.01e-11 * np.linalg.norm(w.b)
    # two solutions with relative residuals <= 1e-11 on a matrix with
    # condition number well below 1e4
    assert np.linalg.norm(a - c) <= 1e-7 * np.linalg.norm(c)
