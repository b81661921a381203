"""asss_solve_noalloc (the allocation-free solve) against asss_solve through
the C ABI: equal results on two calls in a row, the second on a smaller
system, so that the shared fixed workspace is reused with leftover contents;
a problem beyond the fixed workspace is refused."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_06954_amd as asss
    asss.load()
    return asss


def _pair(asss, m, k):
    w = W.implicit_euler_grid(m=m, h=0.1, cfg=0)
    h = asss.setup(w.A, k=k, s_pattern="tridiag")
    return w, h


@pytest.mark.parametrize("outer", ["fgmres", "tfqmr"])
def test_noalloc_matches_solve_on_two_calls(outer):
    asss = _lib()
    w1, h1 = _pair(asss, 45, 8)   # n = 2025
    w2, h2 = _pair(asss, 30, 6)   # n = 900: the second call is smaller
    try:
        for w, h, m in ((w1, h1, 64), (w2, h2, 30)):
            n = w.A.shape[0]
            print(f"[noalloc] outer={outer} n={n} restart={m}", flush=True)
            b = torch.from_numpy(w.b).cuda()
            kw = dict(tol=1e-10, restart_m=m, outer=outer)
            x_ref, i_ref = h.solve(b, **kw)
            out = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
            x_na, i_na = h.solve_noalloc(b, out, **kw)
            torch.cuda.synchronize()
            assert x_na.data_ptr() == out.data_ptr()
            assert i_na["status"] == "OK" and i_na["relres_true"] <= 1e-10
            assert i_na["outer_its"] == i_ref["outer_its"]
            assert i_na["inner_its_total"] == i_ref["inner_its_total"]
            xr, xn = x_ref.cpu().numpy(), x_na.cpu().numpy()
            assert np.linalg.norm(xn - xr) <= 1e-15 * np.linalg.norm(xr), np.linalg.norm(xn - xr)
            # a solve from an initial guess uses the two extra workspace vectors
            x0 = x_ref * (1 + 1e-3)
            x_ref0, _ = h.solve(b, x0=x0, **kw)
            x_na0, i_na0 = h.solve_noalloc(b, torch.empty_like(b), x0=x0, **kw)
            torch.cuda.synchronize()
            assert i_na0["status"] == "OK"
            assert torch.equal(x_ref0, x_na0)
    finally:
        h1.close()
        h2.close()


def test_noalloc_refuses_beyond_its_workspace():
    """n (2 m + 3) 8 bytes above the fixed 128 MiB: INVALID_ARG, x untouched;
    the same handle then solves normally through both entry points."""
    asss = _lib()
    w, h = _pair(asss, 200, 4)    # n = 40,000: 256 MB of workspace at m = 250
    try:
        b = torch.from_numpy(w.b).cuda()
        out = torch.zeros_like(b)
        with pytest.raises(asss.AsssError) as e:
            h.solve_noalloc(b, out, restart_m=250, tol=1e-8)
        assert e.value.name == "INVALID_ARG" and "workspace" in str(e.value)
        assert float(out.abs().max()) == 0.0
        x, info = h.solve_noalloc(b, out, restart_m=64, tol=1e-8)
        assert info["status"] == "OK"
        xr, _ = h.solve(b, restart_m=64, tol=1e-8)
        assert torch.equal(x, xr)
    finally:
        h.close()
