"""Host setup stages (no GPU) against the oracle: the C++ matching, canonical
scaling, Abar, the pattern of S and the least-squares system of App. A are
run through a small harness on the CPU (the device LSQR is not involved), and,
fed the oracle's S values, the C++ A_hat, D, Omega and J_tilde.  Matching
indices bit-exact (random real entries make a tie in the optimum a
probability-zero event; the stand-ins and the large-h implicit-Euler systems
match 299 / 300 / 299, 20 and 8 columns off the diagonal); scalings, Abar, D,
Omega, J_tilde to 1e-13; the
least-squares system through its normal equations B^T B and B^T v (which do
not depend on the order of equations and unknowns) to 1e-13."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2009_06954_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("hs")
    exe = str(d / "check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-pthread", f"-I{CSRC}",
                    os.path.join(ROOT, "tests", "host_setup_check.cpp"),
                    os.path.join(CSRC, "host_setup.cpp"), "-o", exe], check=True)
    return exe, d


def _run(harness, A, kind, svals):
    exe, d = harness
    A = sp.csr_matrix(A)
    A.sort_indices()
    fin, fout = str(d / "in.bin"), str(d / "out.bin")
    with open(fin, "wb") as f:
        np.array([A.shape[0], A.nnz], np.int64).tofile(f)
        np.array([kind], np.int32).tofile(f)
        A.indptr.astype(np.int64).tofile(f)
        A.indices.astype(np.int32).tofile(f)
        A.data.astype(np.float64).tofile(f)
        np.array([len(svals)], np.int64).tofile(f)
        np.asarray(svals, np.float64).tofile(f)
    r = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    raw = open(fout, "rb").read()
    pos = 0
    out = []

    def take(dt):
        nonlocal pos
        cnt = int(np.frombuffer(raw, np.int64, 1, pos)[0])
        pos += 8
        a = np.frombuffer(raw, dt, cnt, pos).copy()
        pos += cnt * np.dtype(dt).itemsize
        return a

    names = [("m", np.int32), ("Dr", np.float64), ("Dc", np.float64), ("Abar_ptr", np.int64),
             ("Abar_col", np.int32), ("Abar_val", np.float64), ("S_ptr", np.int64), ("S_col", np.int32),
             ("B_shape", np.int64), ("B_ptr", np.int64), ("B_col", np.int32), ("B_val", np.float64),
             ("rhs", np.float64)]
    if len(svals):
        names += [("D", np.float64), ("Omega", np.float64), ("J_ptr", np.int64), ("J_col", np.int32),
                  ("J_val", np.float64)]
    res = {}
    for name, dt in names:
        res[name] = take(dt)
    return res


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _cases():
    cases = [("cfg0 45x45", W.config(0).A, "tridiag", 1), ("cfg0 abar pattern", W.config(0, m=20).A, "abar", 2)]
    for s in range(3):  # random row permutations and row scales: non-identity matchings
        w = W.paper_like(300, 1800, seed=s)
        cases.append((f"paper-like seed {s}", w.A, "tridiag", 1))
    ws = W.batched_implicit_euler(nsys=2, n_lo=400, n_hi=900, nrhs=1, cfg=3, h_lo=0.3, h_hi=0.5)
    cases += [(f"implicit Euler h={w.meta['h']:.2f}", w.A, "tridiag", 1) for w in ws]
    return cases


@pytest.mark.parametrize("name,A,pattern,kind", _cases(), ids=[c[0] for c in _cases()])
def test_host_setup_matches_oracle(harness, name, A, pattern, kind):
    st = O.setup(A, O.SetupOptions(k=0, s_pattern=pattern))
    S = st.S.tocsr()
    S.sort_indices()
    r = _run(harness, A, kind, S.data)
    n = A.shape[0]
    # matching: the optimum is unique here, so the indices must agree exactly
    assert np.array_equal(r["m"], st.m.astype(np.int32)), name
    assert _rel(r["Dr"], st.Dr) <= 1e-13 and _rel(r["Dc"], st.Dc) <= 1e-13
    Ab = sp.csr_matrix((r["Abar_val"], r["Abar_col"], r["Abar_ptr"]), shape=(n, n))
    assert abs(Ab - st.Abar).max() <= 1e-13 * abs(st.Abar).max()
    assert np.array_equal(r["S_ptr"], S.indptr) and np.array_equal(r["S_col"], S.indices)
    # least-squares system: same size, same normal equations (unknowns mapped
    # from the harness's row-major order to the oracle's column-major order)
    Bo, vo, urow, ucol = O.skewsym.build_lls(st.Abar, S, 1.0)
    nrows, ncols, nnzB = (int(t) for t in r["B_shape"])
    assert (nrows, ncols) == Bo.shape and nnzB == Bo.nnz
    Bc = sp.csr_matrix((r["B_val"], r["B_col"], r["B_ptr"]), shape=(nrows, ncols))
    rowmajor = {(int(i), int(j)): t for t, (i, j) in
                enumerate(zip(np.repeat(np.arange(n), np.diff(S.indptr)), S.indices))}
    perm = np.array([rowmajor[(int(i), int(j))] for i, j in zip(urow, ucol)])
    Bc = Bc[:, perm]
    G, Go = (Bc.T @ Bc).toarray(), (Bo.T @ Bo).toarray()
    assert np.abs(G - Go).max() <= 1e-13 * np.abs(Go).max()
    assert _rel(Bc.T @ r["rhs"], Bo.T @ vo) <= 1e-13
    # A_hat = Abar S, D, Omega and J_tilde from the same S values
    assert _rel(r["D"], st.D) <= 1e-13 and _rel(r["Omega"], st.Omega) <= 1e-13
    Ju = st.Jup.tocsr()
    Ju.sort_indices()
    assert np.array_equal(r["J_ptr"], Ju.indptr) and np.array_equal(r["J_col"], Ju.indices)
    assert _rel(r["J_val"], Ju.data) <= 1e-13


def test_host_setup_under_sanitizers(tmp_path):
    """The setup stages built with AddressSanitizer and UndefinedBehaviorSanitizer
    (g++, host code only) run clean on a stand-in with a non-identity
    matching and still agree with the oracle."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "check_san")
    r = subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-pthread", "-fsanitize=address,undefined",
                        "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", f"-I{CSRC}",
                        os.path.join(ROOT, "tests", "host_setup_check.cpp"),
                        os.path.join(CSRC, "host_setup.cpp"), "-o", exe], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    os.environ.setdefault("ASAN_OPTIONS", "detect_leaks=1:abort_on_error=1")
    A = W.paper_like(300, 1800, seed=1).A
    st = O.setup(A, O.SetupOptions(k=0, s_pattern="tridiag"))
    S = st.S.tocsr()
    S.sort_indices()
    res = _run((exe, tmp_path), A, 1, S.data)
    assert np.array_equal(res["m"], st.m.astype(np.int32))
    assert _rel(res["J_val"], st.Jup.tocsr().sorted_indices().data) <= 1e-13
