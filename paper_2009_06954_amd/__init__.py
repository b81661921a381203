"""Python binding of libasss (include/asss.h): the solve phase of the two-level
ASSS + mrs scheme of Manguoglu & Mehrmann on MI355X (gfx950).

Argument marshalling only: every step of the method runs in libasss.  The
library must have been built (``python -m paper_2009_06954_amd.build``);
there is no fallback.

    import paper_2009_06954_amd as asss
    h = asss.setup(A_scipy_csr, k=16, s_pattern="abar")
    x, info = h.solve(b_cuda_float64)

PyTorch provides device memory and the current HIP stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libasss.so")

OK, NOT_CONVERGED = 0, 1
_STATUS_NAMES = {
    0: "OK", 1: "NOT_CONVERGED", -1: "INVALID_ARG", -2: "INVALID_CSR",
    -3: "STRUCTURALLY_SINGULAR", -4: "ZERO_DIAGONAL", -5: "LLS", -6: "NONFINITE",
    -7: "HIP", -8: "OOM", -9: "INTERNAL",
}
S_PATTERNS = {"diag": 0, "tridiag": 1, "abar": 2, "user": 3}
OPS = {"skew": 0, "deflated": 1, "outer": 2, "outer_t": 3, "mrs": 4, "prec": 5, "prec_t": 6,
       "A": 7, "AT": 8}
ARRAYS = {"match": (0, np.int32), "Dr": (1, np.float64), "Dc": (2, np.float64),
          "S_rowptr": (3, np.int64), "S_colind": (4, np.int32), "S_val": (5, np.float64),
          "D": (6, np.float64), "J_rowptr": (7, np.int64), "J_colind": (8, np.int32),
          "J_val": (9, np.float64), "Q": (10, np.float64), "alpha": (11, np.float64),
          "X": (12, np.float64), "neg": (13, np.int32),
          # the incomplete LDL^T (precond="ildl"), in the factorization's positions
          "ildl_perm": (14, np.int32), "ildl_L_rowptr": (15, np.int64), "ildl_L_colind": (16, np.int32),
          "ildl_L_val": (17, np.float64), "ildl_bsize": (18, np.int32), "ildl_D": (19, np.float64),
          "Lcal_rowptr": (20, np.int64), "Lcal_colind": (21, np.int32), "Lcal_val": (22, np.float64),
          "Ur": (23, np.float64), "sigma_r": (24, np.float64)}
PRECONDS = {"diag": 0, "ildl": 1}

EXPORTED = ["asss_default_setup_opts", "asss_default_solve_opts", "asss_setup", "asss_solve",
            "asss_solve_noalloc", "asss_solve_adjoint", "asss_solve_batched", "asss_destroy", "asss_last_error",
            "asss_get_handle_info", "asss_get_array", "asss_apply", "asss_update_values",
            "asss_value_gradient", "asss_save", "asss_load", "asss_ildl_factor", "asss_ildl_get",
            "asss_ildl_destroy"]


class CsrT(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("colind", C.c_void_p), ("val", C.c_void_p)]


class SetupOpts(C.Structure):
    _fields_ = [("gamma", C.c_double), ("s_pattern", C.c_int32), ("s_rowptr", C.c_void_p),
                ("s_colind", C.c_void_p), ("k", C.c_int32), ("lanczos_seed", C.c_uint64),
                ("inner_fp32", C.c_int32), ("x_tol", C.c_double), ("x_maxit", C.c_int32),
                ("lls_tol", C.c_double), ("lls_maxit", C.c_int32), ("row_block", C.c_int32),
                ("verbose", C.c_int32), ("deflation", C.c_int32), ("reorder", C.c_int32),
                ("allocator", C.c_void_p), ("autotune", C.c_int32), ("inner_perm", C.c_void_p),
                ("skew_form", C.c_int32), ("s_val", C.c_void_p), ("q_basis", C.c_void_p),
                ("q_alpha", C.c_void_p), ("precond", C.c_int32), ("ildl_droptol", C.c_double),
                ("ildl_fill", C.c_double), ("ildl_pivoting", C.c_int32), ("ildl_explicit", C.c_int32),
                ("step_threads", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class AllocatorT(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


def torch_allocator():
    """asss_allocator_t backed by torch's caching allocator on the current
    device (the returned object must outlive the handle; Handle keeps it)."""
    import torch
    dev = torch.cuda.current_device()

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev)
        except RuntimeError:  # out of memory: the library reports ASSS_ERR_OOM
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    a = AllocatorT(ALLOC_FN(_alloc), FREE_FN(_free), None)
    a._keep = (_alloc, _free)
    return a


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart_m", C.c_int32), ("max_outer", C.c_int32),
                ("inner_tol", C.c_double), ("inner_maxit", C.c_int32),
                ("fixed_inner_steps", C.c_int32), ("inner_fp32", C.c_int32), ("outer", C.c_int32),
                ("batch_streams", C.c_int32), ("use_x0", C.c_int32), ("batch_engine", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("converged", C.c_int32), ("outer_its", C.c_int32), ("inner_its_total", C.c_int32),
                ("inner_its_max", C.c_int32), ("k_eff", C.c_int32), ("rank_r", C.c_int32),
                ("cycles", C.c_int32), ("inner_launches", C.c_int32), ("relres_true", C.c_double),
                ("relres_implicit", C.c_double), ("setup_host_s", C.c_double),
                ("setup_device_s", C.c_double), ("solve_s", C.c_double),
                ("inner_kernel_s", C.c_double), ("reorth", C.c_int32), ("reserved", C.c_int32)]

    def to_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class HandleInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz_a", C.c_int64), ("nnz_s", C.c_int64),
                ("nnz_ahat", C.c_int64), ("nh", C.c_int64), ("lls_rows", C.c_int64),
                ("lls_nnz", C.c_int64), ("k_eff", C.c_int32), ("rank_r", C.c_int32),
                ("lls_its", C.c_int32), ("x_its", C.c_int32), ("row_block", C.c_int32),
                ("nblocks", C.c_int32), ("sell_entries_a", C.c_int64),
                ("sell_entries_b", C.c_int64), ("lls_relres", C.c_double), ("lls_kkt", C.c_double),
                ("lanczos_orth_err", C.c_double), ("deflation_mode", C.c_int32), ("reordered", C.c_int32),
                ("cross_pairs_natural", C.c_int64), ("cross_pairs_used", C.c_int64),
                ("narrow_b_columns", C.c_int32), ("skew_form", C.c_int32), ("tune_n", C.c_int32),
                ("tune_rows", C.c_int32 * 8), ("tune_us", C.c_double * 8), ("tune_s", C.c_double),
                ("precond", C.c_int32), ("ildl_n2x2", C.c_int32), ("ildl_levels_lower", C.c_int32),
                ("ildl_levels_upper", C.c_int32), ("ildl_nnz_l", C.c_int64), ("ildl_dropped", C.c_int64),
                ("step_threads", C.c_int32), ("step_threads_fp64", C.c_int32), ("ildl_explicit", C.c_int32),
                ("outer_ell", C.c_int32)]

    def to_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        nt = self.tune_n
        d["tune_rows"] = list(self.tune_rows)[:nt]
        d["tune_us"] = list(self.tune_us)[:nt]
        return d


class AsssError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS_NAMES.get(status, status)} ({status}): {msg}")
        self.status = status
        self.name = _STATUS_NAMES.get(status, str(status))


_lib = None


def load(path: str = LIB_PATH):
    """Load libasss.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2009_06954_amd.build`")
    lib = C.CDLL(path)
    lib.asss_last_error.restype = C.c_char_p
    lib.asss_default_setup_opts.argtypes = [C.POINTER(SetupOpts)]
    lib.asss_default_solve_opts.argtypes = [C.POINTER(SolveOpts)]
    lib.asss_setup.argtypes = [C.POINTER(CsrT), C.POINTER(SetupOpts), C.c_void_p, C.POINTER(C.c_void_p)]
    lib.asss_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(SolveOpts),
                               C.POINTER(Info), C.c_void_p]
    lib.asss_solve_adjoint.argtypes = lib.asss_solve.argtypes
    lib.asss_solve_noalloc.argtypes = lib.asss_solve.argtypes
    lib.asss_solve_batched.argtypes = [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                       C.POINTER(SolveOpts), C.POINTER(Info), C.c_void_p]
    lib.asss_update_values.argtypes = [C.c_void_p, C.POINTER(CsrT), C.c_void_p]
    lib.asss_value_gradient.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p]
    lib.asss_destroy.argtypes = [C.c_void_p]
    lib.asss_get_handle_info.argtypes = [C.c_void_p, C.POINTER(HandleInfo)]
    lib.asss_get_array.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_int64)]
    lib.asss_apply.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(SolveOpts),
                               C.POINTER(C.c_int32), C.c_void_p]
    lib.asss_save.argtypes = [C.c_void_p, C.c_char_p]
    lib.asss_load.argtypes = [C.c_char_p, C.POINTER(SetupOpts), C.c_void_p, C.POINTER(C.c_void_p)]
    lib.asss_ildl_factor.argtypes = [C.POINTER(CsrT), C.c_double, C.c_double, C.c_int32, C.POINTER(C.c_void_p)]
    lib.asss_ildl_get.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_int64)]
    lib.asss_ildl_destroy.argtypes = [C.c_void_p]
    for f in EXPORTED:
        if f != "asss_last_error":
            getattr(lib, f).restype = None if f.startswith("asss_default") else C.c_int32
    _lib = lib
    return lib


def _check(status, allow_soft=True):
    if status < 0 or (status > 0 and not allow_soft):
        raise AsssError(status, _lib.asss_last_error().decode())
    return status


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _csr_arrays(A, canonicalize=True):
    import scipy.sparse as sp
    if hasattr(A, "crow_indices"):  # torch sparse CSR (CPU)
        rp = A.crow_indices().numpy().astype(np.int64)
        ci = A.col_indices().numpy().astype(np.int32)
        va = A.values().numpy().astype(np.float64)
        n = A.shape[0]
    else:
        A = sp.csr_matrix(A, copy=True)
        if canonicalize:
            A.sum_duplicates()
            A.sort_indices()
        rp = np.ascontiguousarray(A.indptr, dtype=np.int64)
        ci = np.ascontiguousarray(A.indices, dtype=np.int32)
        va = np.ascontiguousarray(A.data, dtype=np.float64)
        n = A.shape[0]
    return n, rp, ci, va


OUTER = {"fgmres": 0, "tfqmr": 1}


def solve_options(tol=1e-8, restart_m=64, max_outer=2000, inner_tol=1e-5, inner_maxit=1000,
                  fixed_inner_steps=0, inner_fp32=None, outer="fgmres", batch_streams=0,
                  use_x0=False, batch_engine="auto") -> SolveOpts:
    o = SolveOpts()
    load().asss_default_solve_opts(C.byref(o))
    o.tol, o.restart_m, o.max_outer = tol, restart_m, max_outer
    o.inner_tol, o.inner_maxit, o.fixed_inner_steps = inner_tol, inner_maxit, fixed_inner_steps
    o.inner_fp32 = -1 if inner_fp32 is None else int(bool(inner_fp32))
    o.outer = OUTER[outer]
    o.batch_streams = batch_streams
    o.use_x0 = int(bool(use_x0))
    o.batch_engine = {"auto": 0, "lockstep": 1, "workers": 2}[batch_engine]
    return o


class Handle:
    """A preprocessed matrix on the GPU (owns all its device memory)."""

    def __init__(self, ptr, n, keep=None):
        self._h = C.c_void_p(ptr)
        self.n = n
        self._keep = keep  # the allocator callbacks must outlive the handle

    def close(self):
        if self._h and self._h.value:
            _check(load().asss_destroy(self._h))
            self._h = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, v):
        import torch
        if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.float64
                and v.is_contiguous() and v.numel() == self.n):
            raise ValueError(f"expected a contiguous CUDA float64 tensor of length {self.n}")
        return v

    def _start(self, out, like, x0):
        import torch
        x = self._vec(out) if out is not None else torch.empty_like(like)
        if x0 is not None:
            x.copy_(self._vec(x0))
        return x

    def solve(self, b, out=None, stream=None, x0=None, **opts):
        """x = A^-1 b, from x0 if given (else from 0).  Returns (x, info dict);
        info['status'] is OK or NOT_CONVERGED."""
        b = self._vec(b)
        x = self._start(out, b, x0)
        opts["use_x0"] = x0 is not None
        info = Info()
        st = _check(load().asss_solve(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                      C.byref(solve_options(**opts)), C.byref(info), _stream(stream)))
        d = info.to_dict()
        d["status"] = _STATUS_NAMES[st]
        return x, d

    def solve_noalloc(self, b, out, stream=None, x0=None, **opts):
        """x = A^-1 b through asss_solve_noalloc (no device allocation inside
        the call; the workspace is the library's fixed array).  `out` is the
        caller's x (contiguous CUDA float64, length n).  Returns (out, info)."""
        b = self._vec(b)
        x = self._vec(out)
        if x0 is not None:
            x.copy_(self._vec(x0))
        opts["use_x0"] = x0 is not None
        info = Info()
        st = _check(load().asss_solve_noalloc(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                              C.byref(solve_options(**opts)), C.byref(info), _stream(stream)))
        d = info.to_dict()
        d["status"] = _STATUS_NAMES[st]
        return x, d

    def solve_adjoint(self, g, out=None, stream=None, x0=None, **opts):
        """lambda = A^-T g, from x0 if given.  Returns (lambda, info dict)."""
        g = self._vec(g)
        lam = self._start(out, g, x0)
        opts["use_x0"] = x0 is not None
        info = Info()
        st = _check(load().asss_solve_adjoint(self._h, C.c_void_p(g.data_ptr()), C.c_void_p(lam.data_ptr()),
                                              C.byref(solve_options(**opts)), C.byref(info), _stream(stream)))
        d = info.to_dict()
        d["status"] = _STATUS_NAMES[st]
        return lam, d

    def apply(self, op, v, out=None, stream=None, **opts):
        """One operator of the method (see asss_apply).  Returns (out, inner_its)."""
        import torch
        v = self._vec(v)
        o = self._vec(out) if out is not None else torch.empty_like(v)
        its = C.c_int32(0)
        _check(load().asss_apply(self._h, OPS[op], C.c_void_p(v.data_ptr()), C.c_void_p(o.data_ptr()),
                                 C.byref(solve_options(**opts)), C.byref(its), _stream(stream)))
        return o, its.value

    def update_values(self, A, stream=None):
        """Give A new values on the pattern used at setup; the preconditioner
        stays as built (see asss_update_values)."""
        n, rp, ci, va = _csr_arrays(A)
        if n != self.n:
            raise ValueError(f"expected an n = {self.n} matrix")
        csr = CsrT(n, int(rp[-1]), rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
        _check(load().asss_update_values(self._h, C.byref(csr), _stream(stream)))

    def value_gradient(self, rowptr, colind, lam, x, out=None, stream=None):
        """grad[e] = -lam[i] x[colind[e]] over the CSR pattern (rowptr int64 and
        colind int32 CUDA tensors), i.e. dL/dA for x = A^-1 b, A^T lam = dL/dx."""
        import torch
        lam, x = self._vec(lam), self._vec(x)
        if not (rowptr.is_cuda and rowptr.dtype == torch.int64 and rowptr.is_contiguous()
                and rowptr.numel() == self.n + 1 and colind.is_cuda and colind.dtype == torch.int32
                and colind.is_contiguous()):
            raise ValueError("rowptr must be CUDA int64 (n + 1), colind CUDA int32")
        nnz = colind.numel()
        if out is not None and not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64
                                    and out.is_contiguous() and out.numel() == nnz):
            raise ValueError(f"out must be a contiguous CUDA float64 tensor of length {nnz}")
        g = out if out is not None else torch.empty(nnz, dtype=torch.float64, device=x.device)
        _check(load().asss_value_gradient(self._h, nnz, C.c_void_p(rowptr.data_ptr()),
                                          C.c_void_p(colind.data_ptr()), C.c_void_p(lam.data_ptr()),
                                          C.c_void_p(x.data_ptr()), C.c_void_p(g.data_ptr()),
                                          _stream(stream)))
        return g

    def save(self, path):
        """Write the setup to `path` (asss_save); `load_handle` reads it back."""
        _check(load().asss_save(self._h, os.fsencode(path)))

    def info(self) -> dict:
        hi = HandleInfo()
        _check(load().asss_get_handle_info(self._h, C.byref(hi)))
        return hi.to_dict()

    def array(self, name) -> np.ndarray:
        which, dt = ARRAYS[name]
        cnt = C.c_int64(0)
        _check(load().asss_get_array(self._h, which, None, C.byref(cnt)))
        out = np.empty(cnt.value, dtype=dt)
        if cnt.value:
            _check(load().asss_get_array(self._h, which, C.c_void_p(out.ctypes.data), C.byref(cnt)))
        return out


SKEW_FORMS = {"auto": 0, "wide": 1, "narrow": 2, "slots": 3}


def setup(A, gamma=1.0, s_pattern="tridiag", k=20, lanczos_seed=0x2009069540, inner_fp32=False,
          x_tol=1e-10, x_maxit=2000, lls_tol=1e-15, lls_maxit=20000, row_block=0, verbose=False,
          stream=None, canonicalize=True, deflation="auto", reorder="auto", allocator=None,
          autotune=False, skew_form="auto", s_values=None, q_basis=None, q_alpha=None, precond="diag",
          ildl_droptol=0.0, ildl_fill=float("inf"), ildl_pivoting=True, ildl_explicit="auto",
          step_threads=0) -> Handle:
    """Preprocess A (scipy CSR or torch sparse CSR on the CPU, float64) on the GPU.
    canonicalize: sum duplicates and sort column indices of a SciPy input first
    (otherwise the library rejects such input with INVALID_CSR).
    allocator: None (the library's hipMalloc) or "torch" (torch's caching
    allocator holds all device memory of the handle).
    autotune: time the inner step for several row-block sizes at setup and keep
    the fastest (row_block must be 0; see info()["tune_rows"], ["tune_us"]).
    reorder: "auto"/"none" (natural order of the inner system), "grid" (tiles
    of whole lines when A's pattern is a lexicographic 3D grid, else natural)
    or an integer array perm of length n (inner row i is row perm[i]).
    s_values: None (S from the least-squares problem of App. A) or the values
    of S on its pattern in CSR order (float64, length nnz of the pattern): the
    least-squares solve is skipped.
    q_basis, q_alpha: None (deflation basis from skew-Lanczos) or Q_k (n x k,
    A's row order) and the k - 1 coefficients of S_k: the Lanczos run is
    skipped and this basis is used (the preconditioner P does not depend on it).
    skew_form: storage of J_tilde's columns: "auto", "wide" (32-bit), "narrow"
    (16-bit deltas) or "slots" (one offset per slot, no per-entry columns).
    deflation: "auto"/"explicit" or "explicit_fp32_basis" (the
    Lanczos vectors rounded to FP32 values and used so everywhere: same
    preconditioner P, FP64 arithmetic, half the basis bytes in the FP64 inner
    step; see asss_setup_opts_t.deflation).
    precond: "diag" (L = I, D = diag(A_hat)) or "ildl" (incomplete LDL^T of
    M_hat with Bunch-Kaufman pivoting; ildl_droptol, ildl_fill and
    ildl_pivoting as in asss_setup_opts_t; reorder must stay "auto";
    ildl_explicit: "auto", True (J_tilde formed at setup, inner steps on the
    sliced kernels) or False (two triangular solves per inner step)).
    step_threads: workgroup size of the one-column inner step (0 = chosen
    per precision, 256 or 512 in both; asss_setup_opts_t)."""
    lib = load()
    n, rp, ci, va = _csr_arrays(A, canonicalize)
    csr = CsrT(n, int(rp[-1]), rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
    o = SetupOpts()
    lib.asss_default_setup_opts(C.byref(o))
    keep = []
    if isinstance(s_pattern, str):
        o.s_pattern = S_PATTERNS[s_pattern]
    else:
        _, srp, sci, _ = _csr_arrays(s_pattern)
        keep += [srp, sci]
        o.s_pattern = S_PATTERNS["user"]
        o.s_rowptr, o.s_colind = srp.ctypes.data, sci.ctypes.data
    o.gamma, o.k, o.lanczos_seed, o.inner_fp32 = gamma, k, lanczos_seed, int(bool(inner_fp32))
    o.x_tol, o.x_maxit, o.lls_tol, o.lls_maxit = x_tol, x_maxit, lls_tol, lls_maxit
    o.row_block, o.verbose = row_block, int(bool(verbose))
    o.autotune = int(bool(autotune))
    o.skew_form = SKEW_FORMS[skew_form]
    o.precond = PRECONDS[precond]
    o.ildl_droptol, o.ildl_fill, o.ildl_pivoting = ildl_droptol, ildl_fill, int(bool(ildl_pivoting))
    o.ildl_explicit = -1 if ildl_explicit == "auto" else int(bool(ildl_explicit))
    o.step_threads = int(step_threads)
    if s_values is not None:
        sv = np.ascontiguousarray(s_values, dtype=np.float64)
        keep.append(sv)
        o.s_val = sv.ctypes.data
    if q_basis is not None:
        qb = np.asfortranarray(q_basis, dtype=np.float64)
        if qb.shape != (n, k):
            raise ValueError(f"q_basis must be n x k = {n} x {k}")
        qa = np.ascontiguousarray(q_alpha if q_alpha is not None else np.zeros(0), dtype=np.float64)
        if qa.shape != (max(k - 1, 0),):
            raise ValueError("q_alpha must hold k - 1 values")
        keep += [qb, qa]
        o.q_basis, o.q_alpha = qb.ctypes.data, qa.ctypes.data
    o.deflation = {"auto": 0, "explicit": 1, "explicit_fp32_basis": 3}[deflation]
    if isinstance(reorder, str):
        o.reorder = {"auto": 0, "none": 1, "grid": 4}[reorder]
    else:  # the caller's order of the inner system: inner row i is row reorder[i]
        perm = np.ascontiguousarray(reorder, dtype=np.int32)
        if perm.shape != (n,):
            raise ValueError("reorder must be 'auto', 'none', 'grid' or a permutation of length n")
        keep.append(perm)
        o.reorder, o.inner_perm = 3, perm.ctypes.data
    alloc = None
    if allocator == "torch":
        alloc = torch_allocator()
        o.allocator = C.cast(C.pointer(alloc), C.c_void_p)
    elif allocator is not None:
        raise ValueError("allocator must be None or 'torch'")
    out = C.c_void_p()
    _check(lib.asss_setup(C.byref(csr), C.byref(o), _stream(stream), C.byref(out)))
    return Handle(out.value, n, keep=alloc)


def load_handle(path, stream=None, allocator=None, verbose=False) -> Handle:
    """A handle from a file written by Handle.save (asss_load): the matching,
    scalings and S are read, the rest of the setup is rebuilt."""
    lib = load()
    o = SetupOpts()
    lib.asss_default_setup_opts(C.byref(o))
    o.verbose = int(bool(verbose))
    alloc = None
    if allocator == "torch":
        alloc = torch_allocator()
        o.allocator = C.cast(C.pointer(alloc), C.c_void_p)
    elif allocator is not None:
        raise ValueError("allocator must be None or 'torch'")
    out = C.c_void_p()
    _check(lib.asss_load(os.fsencode(path), C.byref(o), _stream(stream), C.byref(out)))
    hi = HandleInfo()
    _check(lib.asss_get_handle_info(out, C.byref(hi)))
    return Handle(out.value, int(hi.n), keep=alloc)


def solve_batched(handles, Bs, stream=None, X0s=None, **opts):
    """Solve several systems, each with several right-hand sides (B: n_s x nrhs_s
    CUDA float64, column-major i.e. the transpose of a contiguous (nrhs, n)
    tensor is expected as B.T), from the initial guesses X0s (same shapes) if
    given.  Returns (list of X, list of info lists)."""
    import torch
    lib = load()
    ns = len(handles)
    Xs, nr = [], []
    for h, B in zip(handles, Bs):
        if B.dim() == 1:
            B = B[:, None]
        if not (B.is_cuda and B.dtype == torch.float64 and B.shape[0] == h.n and B.t().is_contiguous()):
            raise ValueError("each B must be a column-major (n, nrhs) CUDA float64 tensor")
        Xs.append(torch.empty_like(B))
        nr.append(B.shape[1])
    if X0s is not None:
        for X, X0 in zip(Xs, X0s):
            X.copy_(X0.reshape(X.shape))
        opts["use_x0"] = True
    maxr = max(nr) if nr else 0
    hs = (C.c_void_p * ns)(*[h._h.value for h in handles])
    nra = (C.c_int32 * ns)(*nr)
    bp = (C.c_void_p * ns)(*[B.data_ptr() for B in Bs])
    xp = (C.c_void_p * ns)(*[X.data_ptr() for X in Xs])
    infos = (Info * max(1, ns * maxr))()
    _check(lib.asss_solve_batched(ns, hs, nra, bp, xp, C.byref(solve_options(**opts)), infos, _stream(stream)))
    out_infos = [[infos[s * maxr + j].to_dict() for j in range(nr[s])] for s in range(ns)]
    return Xs, out_infos


ILDL_ARRAYS = ("ildl_perm", "ildl_L_rowptr", "ildl_L_colind", "ildl_L_val", "ildl_bsize", "ildl_D",
               "Lcal_rowptr", "Lcal_colind", "Lcal_val", "Ur", "sigma_r")


def ildl_factor(M, droptol=0.0, fill=float("inf"), pivoting=True) -> dict:
    """The library's incomplete LDL^T of a symmetric matrix M (host only, no
    GPU): asss_ildl_factor, then every ASSS_ARR_ILDL_* / LCAL / UR / SIGMA_R
    array.  Ur is returned as an n x r array."""
    lib = load()
    n, rp, ci, va = _csr_arrays(M)
    csr = CsrT(n, int(rp[-1]), rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
    f = C.c_void_p()
    _check(lib.asss_ildl_factor(C.byref(csr), droptol, fill, int(bool(pivoting)), C.byref(f)))
    try:
        out = {}
        for name in ILDL_ARRAYS:
            which, dt = ARRAYS[name]
            cnt = C.c_int64(0)
            _check(lib.asss_ildl_get(f, which, None, C.byref(cnt)))
            a = np.empty(cnt.value, dtype=dt)
            if cnt.value:
                _check(lib.asss_ildl_get(f, which, C.c_void_p(a.ctypes.data), C.byref(cnt)))
            out[name] = a
        r = out["sigma_r"].size
        out["Ur"] = out["Ur"].reshape(r, n).T if r else np.zeros((n, 0))
        return out
    finally:
        lib.asss_ildl_destroy(f)
