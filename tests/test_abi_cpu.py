"""CPU checks of the boundary: the library loads without a GPU and exports
every entry point that include/asss.h declares; the Python structs match the
header's field lists; option defaults follow the documented values."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "asss.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(asss_[a-z_]+)\s*\(", text)))


def _lib():
    import paper_2009_06954_amd as asss
    if not os.path.exists(asss.LIB_PATH):
        pytest.skip("libasss.so not built")
    return asss, asss.load()


def test_header_functions_are_exported():
    asss, lib = _lib()
    declared = _declared_functions()
    assert len(declared) >= 11
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(asss.EXPORTED) == declared


def _header_struct_fields(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", text)
    body = m.group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        parts = decl.replace("*", " ").split()
        names = " ".join(parts[1:]).replace(",", " ").split()
        if parts[0] == "const":
            names = " ".join(parts[2:]).replace(",", " ").split()
        fields += [re.sub(r"\[\d+\]$", "", f) for f in names]
    return fields


@pytest.mark.parametrize("cname,pyname", [("asss_csr_t", "CsrT"), ("asss_setup_opts_t", "SetupOpts"),
                                          ("asss_solve_opts_t", "SolveOpts"), ("asss_info_t", "Info"),
                                          ("asss_handle_info_t", "HandleInfo")])
def test_struct_layouts_match_header(cname, pyname):
    import paper_2009_06954_amd as asss
    py = [f for f, _ in getattr(asss, pyname)._fields_]
    assert py == _header_struct_fields(cname)


def test_defaults():
    asss, lib = _lib()
    o = asss.SetupOpts()
    lib.asss_default_setup_opts(ctypes.byref(o))
    assert o.gamma == 1.0 and o.s_pattern == 1 and o.k == 20 and o.lanczos_seed == 0x2009069540
    assert o.x_tol == 1e-10 and o.inner_fp32 == 0 and o.row_block == 0 and o.autotune == 0
    s = asss.SolveOpts()
    lib.asss_default_solve_opts(ctypes.byref(s))
    assert s.tol == 1e-8 and s.restart_m == 64 and s.inner_fp32 == -1


def test_null_arguments_are_rejected_without_gpu():
    asss, lib = _lib()
    st = lib.asss_setup(None, None, None, None)
    assert st == -1
    assert b"null" in lib.asss_last_error()
    assert lib.asss_destroy(None) == 0
    assert lib.asss_solve(None, None, None, None, None, None) == -1


def test_missing_library_fails_loudly(tmp_path):
    import paper_2009_06954_amd as asss
    with pytest.raises(ImportError):
        asss._lib_saved = asss._lib
        try:
            asss._lib = None
            asss.load(str(tmp_path / "nope.so"))
        finally:
            asss._lib = asss._lib_saved


def test_load_rejects_bad_files_without_gpu(tmp_path):
    """asss_load checks the file before any device call: a missing file, a
    foreign file and a truncated saved setup are INVALID_ARG."""
    asss, lib = _lib()
    out = ctypes.c_void_p()
    assert lib.asss_load(str(tmp_path / "missing.bin").encode(), None, None, ctypes.byref(out)) == -1
    assert b"cannot open" in lib.asss_last_error()
    bad = tmp_path / "foreign.bin"
    bad.write_bytes(b"not a saved setup at all")
    assert lib.asss_load(str(bad).encode(), None, None, ctypes.byref(out)) == -1
    trunc = tmp_path / "trunc.bin"
    trunc.write_bytes(b"ASSSSAV1" + (5).to_bytes(8, "little") + b"\x00" * 12)
    assert lib.asss_load(str(trunc).encode(), None, None, ctypes.byref(out)) == -1
    assert b"truncated" in lib.asss_last_error() and not out.value


@pytest.mark.parametrize("field,value,word", [("deflation", 2, b"deflation"), ("reorder", 2, b"reorder"),
                                              ("deflation", 4, b"deflation"), ("k", 33, b"k must")])
def test_unprovided_modes_are_refused_without_gpu(field, value, word):
    """Options are checked before any device call: the recurrence form of the
    deflation (deflation = 2, unstable) and the BFS block order (reorder = 2)
    are not provided and, like out-of-range values, give INVALID_ARG."""
    import numpy as np
    asss, lib = _lib()
    rp = np.array([0, 1, 2], dtype=np.int64)
    ci = np.array([0, 1], dtype=np.int32)
    va = np.array([1.0, 2.0])
    csr = asss.CsrT(2, 2, rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
    o = asss.SetupOpts()
    lib.asss_default_setup_opts(ctypes.byref(o))
    setattr(o, field, value)
    out = ctypes.c_void_p()
    assert lib.asss_setup(ctypes.byref(csr), ctypes.byref(o), None, ctypes.byref(out)) == -1
    assert word in lib.asss_last_error() and not out.value
