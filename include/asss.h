/*
 * asss.h -- C ABI of libasss, a gfx950 (MI355X) implementation of the solve
 * phase of the two-level iterative scheme of Manguoglu & Mehrmann, "A
 * two-level iterative scheme for general sparse linear systems based on
 * approximate skew-symmetrizers".
 *
 * A general sparse invertible A x = b (paper Sec. 1 eq. 1, Sec. 3 eq. sys) is
 * preprocessed once (asss_setup):
 *   - row permutation and scalings, Abar = P Dr A Dc with |abar_ii| = 1 and
 *     |abar_ij| <= 1 (Sec. 2, eq. mc64);
 *   - a sparse skew-symmetrizer S on a user-chosen pattern from a weighted
 *     least-squares problem (Sec. 2, eqs. 1-2 and regularized; App. A);
 *   - A_hat = Abar S split into D = diag(A_hat) and the skew part J_hat
 *     (Sec. 3, eq. modified); Omega = |D|^(-1/2), J_tilde = Omega J_hat Omega;
 *   - k skew-Lanczos vectors Q_k, S_k (Fig. 2), the deflated J_bar =
 *     J_tilde - Q_k S_k Q_k^T, and the one-time Sherman-Morrison-Woodbury data
 *     for the rank-(k+r) term (Sec. 3.2, eqs. preconditioner and smw; Sec. 4.1).
 * Each solve (asss_solve) runs flexible GMRES (or TFQMR, Sec. 4.1) on the
 * scaled system Omega Abar S Omega, right-preconditioned with
 * P = sign(D) + J_tilde, where P^-1 is applied through the SMW form around an
 * inner minimal residual solve (mrs, Sec. 3.1 and App. B) on I + J_bar.
 * With the setup option precond = ASSS_PRECOND_ILDL the symmetric part
 * M_hat = (A_hat + A_hat^T) / 2 is instead factorized incompletely, M_hat ~
 * L D L^T with Bunch-Kaufman pivoting (Sec. 3), Lcal = L |D|^(1/2) as in eq.
 * absfac, J_tilde = Lcal^-1 J_hat Lcal^-T, and the low-rank term of Fig. 1
 * carries the negative eigenvalues of D (1x1 and 2x2 blocks).  The
 * adjoint solve (A^T lambda = g), batched solves of several systems with
 * several right-hand sides, value gradients of a solve, and saved setups use
 * the same preconditioner.
 *
 * Conventions
 *   - Every function returns asss_status_t: 0 = ASSS_OK, > 0 = soft status
 *     (outputs written), < 0 = error (outputs untouched, asss_last_error()
 *     describes it).
 *   - Host pointers are read during the call only and stay owned by the
 *     caller.  Device pointers (b, x, g, lambda, in/out vectors) are owned by
 *     the caller, must hold FP64 data of the stated length, and are used only
 *     on the given HIP stream; they must stay valid until that stream has
 *     finished the call's work (the call itself synchronises the stream
 *     before it returns).
 *   - A handle owns all its device memory (allocated with hipMalloc, or the
 *     caller's allocator, on the device current at asss_setup) and is not
 *     thread-safe: one call at a time per handle.  An output vector must not
 *     overlap its right-hand side (INVALID_ARG).
 *   - hip_stream is a hipStream_t (NULL = the default stream).
 */
#ifndef ASSS_H
#define ASSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t asss_status_t;
enum {
  ASSS_OK = 0,
  ASSS_NOT_CONVERGED = 1,            /* best iterate written, info filled */
  ASSS_ERR_INVALID_ARG = -1,
  ASSS_ERR_INVALID_CSR = -2,         /* unsorted / duplicate / out-of-range columns */
  ASSS_ERR_STRUCTURALLY_SINGULAR = -3, /* no perfect matching exists (Sec. 2) */
  ASSS_ERR_ZERO_DIAGONAL = -4,       /* diag(Abar S) has a zero: Omega undefined */
  ASSS_ERR_LLS = -5,                 /* least-squares solve for S failed */
  ASSS_ERR_NONFINITE = -6,           /* NaN/Inf in an input */
  ASSS_ERR_HIP = -7,                 /* a HIP runtime call failed */
  ASSS_ERR_OOM = -8,
  ASSS_ERR_INTERNAL = -9
};

typedef struct asss_handle_s* asss_handle_t;

/* Sparse matrix in CSR form, HOST memory: rowptr[n+1] (rowptr[0] = 0,
 * non-decreasing, rowptr[n] = nnz), colind[nnz] strictly increasing within a
 * row and in [0, n), val[nnz] finite.  Stored zeros are ignored (a zero value
 * is not a nonzero of A). */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t* rowptr;
  const int32_t* colind;
  const double* val;
} asss_csr_t;

/* Sparsity pattern of S (Sec. 2: diagonal, tridiagonal, the sparsity of
 * Abar, or user defined; the experiments of Sec. 4 use the tridiagonal one). */
enum {
  ASSS_S_DIAG = 0,
  ASSS_S_TRIDIAG = 1,
  ASSS_S_PATTERN_OF_ABAR = 2,
  ASSS_S_USER = 3          /* s_rowptr / s_colind, a CSR pattern in Abar's index space */
};

/* Preconditioner of the inner level (Sec. 3, eqs. preconditioner and absfac). */
enum {
  ASSS_PRECOND_DIAG = 0,   /* L = I, D = diag(A_hat): P = sign(D) + Omega J_hat Omega */
  ASSS_PRECOND_ILDL = 1    /* incomplete LDL^T of M_hat with Bunch-Kaufman pivoting */
};

/* Device memory provider for a handle, e.g. a framework's caching allocator.
 * alloc returns at least `bytes` bytes of device memory (256-byte aligned)
 * usable on the handle's device, or NULL (the entry point then fails with
 * ASSS_ERR_OOM); free gives it back.  Both are called from the calling thread
 * of asss_setup, of the solve entry points (workspaces are grown on first use)
 * and of asss_destroy, with ctx passed through, and from the worker threads of
 * asss_solve_batched, several at once for different handles: they must be
 * thread-safe.  The functions and ctx must stay valid until the handle is
 * destroyed (the structure itself is copied).
 * The callbacks take no stream (a stream-ordered allocator would get one):
 * a handle's buffers serve every stream its calls are given, they are taken
 * at setup or on first use, and given back by asss_destroy (after a device
 * synchronisation) or when a workspace grows (every entry point synchronises
 * its stream before it returns), so no kernel can still be reading memory
 * that is given back. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} asss_allocator_t;

typedef struct {
  double gamma;            /* weight of the diagonal equations (eq. regularized), default 1 */
  int32_t s_pattern;       /* ASSS_S_*, default ASSS_S_TRIDIAG */
  const int64_t* s_rowptr; /* USER pattern (host, n+1), else NULL */
  const int32_t* s_colind; /* USER pattern (host), else NULL */
  int32_t k;               /* skew-Lanczos vectors (Fig. 2), default 20; 0 = no deflation */
  uint64_t lanczos_seed;   /* start vector: SplitMix64 stream of this seed, default 0x2009069540 */
  int32_t inner_fp32;      /* default precision of the inner mrs: 0 = FP64, 1 = FP32 */
  double x_tol;            /* tolerance of the one-time multi-RHS mrs for X, default 1e-10 */
  int32_t x_maxit;         /* default 2000 */
  double lls_tol;          /* LSQR atol = btol for S, default 1e-15 */
  int32_t lls_maxit;       /* default 20000 */
  int32_t row_block;       /* rows per LDS block of the skew operator, 0 = automatic */
  int32_t verbose;         /* 0 = silent, 1 = timing lines on stderr */
  int32_t deflation;       /* how the inner step applies Q_k S_k Q_k^T (Sec. 3.2):
                              0 or 1 = explicitly: Q_k^T q recomputed from the k Lanczos
                                  vectors every step (default);
                              2 = not provided (INVALID_ARG): a form that keeps Q_k^T q_t
                                  through the Lanczos relation instead of the k vectors
                                  loses orthogonality within a few dozen steps;
                              3 = explicitly, with the Lanczos vectors rounded to FP32
                                  values at setup and that basis used everywhere (the
                                  deflated inner operator, U_bar, X, G): the SMW form of
                                  eq. smw then gives back the same P = sign(D) + J_tilde
                                  (the low-rank term adds back what the deflation takes
                                  out, for any basis), arithmetic stays FP64, and the
                                  FP64 inner step reads the basis as 4-byte values.  The
                                  deflated operator and single mrs solves then differ
                                  from those of the unrounded basis by its rounding */
  int32_t reorder;         /* order of the inner system (a symmetric permutation of
                              J_tilde, invisible to the caller):
                              0 or 1 = natural order (default);
                              2 = not provided (INVALID_ARG);
                              3 = the caller's order in inner_perm.  For a grid, an
                                  order in which each block of row_block rows is a
                                  compact tile of whole grid lines keeps more pairs
                                  inside a block than the natural order and keeps
                                  the neighbours of a wavefront at common offsets;
                              4 = that order found by the library: when the pattern
                                  of Abar is a lexicographic 3D grid (positive column
                                  offsets exactly 1, m1 and m1 m2, with m1 m2 | n),
                                  tiles of ty x tz whole x-lines, ty tz the largest
                                  power of two with m1 ty tz <= 1.5 times the
                                  automatic row block (or row_block if given) and a
                                  multiple of 64 within 4096, ty | m2, tz | m3, as
                                  square as possible, one tile per row block (4 x 4
                                  lines at 128^3 and 192^3); otherwise the natural
                                  order */
  const asss_allocator_t* allocator; /* device memory of the handle; NULL = hipMalloc / hipFree */
  int32_t autotune;        /* row-block autotuner (only with row_block = 0):
                              0 = the automatic size (default);
                              1 = at the end of setup, pack J_tilde for the automatic size
                                  and up to two halvings and doublings of it within
                                  [64, 4096], time the fused inner step on each (HIP events,
                                  the handle's deflation and default inner precision, one
                                  right-hand side) and keep the fastest layout.  Costs one
                                  host packing and a few ms of GPU time per candidate;
                                  the result is in asss_handle_info_t.tune_* */
  const int32_t* inner_perm; /* reorder = 3: host array of n entries, inner row i is row
                              inner_perm[i] of J_tilde (new -> old); read during setup
                              only; must be a permutation of 0..n-1 (INVALID_ARG else).
                              Solutions do not depend on it beyond rounding */
  int32_t skew_form;       /* column form of the sliced J_tilde storage:
                              0 = automatic (default): offset slots when they store at
                                  most 1.2x the entries of the per-entry forms (grid
                                  patterns), else 16-bit off-block deltas when they fit,
                                  else 32-bit columns;
                              1 = 32-bit off-block columns;
                              2 = 16-bit off-block column deltas (INVALID_ARG if a slot
                                  spans 2^16 columns or more);
                              3 = offset slots: every slot of a 64-row slice is one offset
                                  d (column = row + d), no per-entry columns; INVALID_ARG
                                  if that stores more than 16x the entries */
  const double* s_val;     /* NULL (default): S solves the least-squares problem of App. A.
                              Else host array of the values of S on its pattern (CSR order
                              of the pattern that s_pattern selects, columns increasing),
                              read during setup only; the least-squares solve is skipped
                              and S is taken as given (e.g. an S computed earlier for the
                              same pattern).  NONFINITE if a value is NaN/Inf */
  const double* q_basis;   /* NULL (default): the deflation basis Q_k comes from k - 1 steps
                              of skew-Lanczos (Fig. 2) from the SplitMix64 start vector.
                              Else host array, n x k column-major in A's row order, with
                              q_alpha (k - 1 values): Q_k and the coefficients of S_k are
                              taken as given and the Lanczos run is skipped (k_eff = k).
                              Any basis gives the same preconditioner P through eq. smw;
                              the basis only changes how fast the inner solve converges.
                              Read during setup only; NONFINITE on NaN/Inf */
  const double* q_alpha;   /* with q_basis: super-diagonal of S_k (k - 1 values) */
  int32_t precond;         /* ASSS_PRECOND_DIAG (default) or ASSS_PRECOND_ILDL: the incomplete
                              factorization M_hat[p][:, p] = L D L^T + E, D with 1x1 and 2x2
                              blocks (Sec. 3).  The scaled system then runs in the
                              factorization's positions p: A_chk = Lcal^-1 A_hat_p Lcal^-T,
                              Lcal = L C with C the block Cholesky factor of |D| (eq. absfac),
                              P = C^-1 D C^-T + J_tilde with J_tilde = Lcal^-1 J_hat_p Lcal^-T,
                              deflated and corrected in the SMW form as above; every product
                              with J_tilde is two sparse triangular solves around J_hat_p,
                              run level by level in one workgroup (sizes of the paper's
                              problems: n up to some 10^4).  Needs reorder = 0, deflation 0/1,
                              autotune = 0 (INVALID_ARG else); ZERO_DIAGONAL if a zero pivot
                              cannot be avoided (pivoting off, or a zero pivot with a nonzero
                              column).  Q and X of asss_get_array are then in positions */
  double ildl_droptol;     /* drop l_ij when |l_ij| < ildl_droptol ||l_j||_2, the norm of column j
                              of L as computed (entries below its pivot block), default 0 */
  double ildl_fill;        /* keep at most ceil(ildl_fill c_j) entries of column j of L, the
                              largest in magnitude, c_j = nonzeros of M_hat's column j among the
                              rows still to be eliminated; default +inf (no cap).  Dropping is
                              applied to each column before it updates the rest of the matrix */
  int32_t ildl_pivoting;   /* 1 (default): Bunch-Kaufman partial pivoting, alpha = (1 + sqrt 17)/8;
                              0: 1x1 pivots in the natural order */
  int32_t ildl_explicit;   /* with precond = ASSS_PRECOND_ILDL: 1 forms J_tilde = Lcal^-1 J_hat_p
                              Lcal^-T and the outer operator Lcal^-1 A_hat_p Lcal^-T explicitly at
                              setup (n columns each of the two triangular solves around J_hat_p,
                              A_hat_p; dense in general: 3.5 n^2 doubles of device memory), runs
                              the inner solve with the fused kernel of the diagonal reading on the
                              dense J_tilde and the outer products as dense row products; 0
                              applies both as two level-scheduled triangular solves per product;
                              -1 (default): 1 when n <= 12288 and the device memory holds them
                              (else 0).  The same operators up to rounding; other values:
                              INVALID_ARG */
  int32_t step_threads;    /* workgroup size of the one-column inner step: 0 (default) chooses
                              512 in FP64, and in FP32 512 when its row blocks fill whole rounds
                              of 512 resident workgroups clearly better than of 1,024 (2 and 4
                              per compute unit), else 256; 256 or 512 force it in both.  Results
                              are the same up to rounding order; other values: INVALID_ARG */
} asss_setup_opts_t;

typedef struct {
  double tol;              /* true relative residual ||b - A x|| / ||b||, default 1e-8 */
  int32_t restart_m;       /* FGMRES restart length, default 64 (TFQMR: unused) */
  int32_t max_outer;       /* total Arnoldi steps (TFQMR: half steps), default 2000 */
  double inner_tol;        /* mrs relative tolerance, default 1e-5 */
  int32_t inner_maxit;     /* default 1000 */
  int32_t fixed_inner_steps; /* > 0: every mrs runs exactly this many steps */
  int32_t inner_fp32;      /* -1 = handle default, 0 = FP64, 1 = FP32 inner */
  int32_t outer;           /* ASSS_OUTER_FGMRES (default) or ASSS_OUTER_TFQMR, the
                              transpose-free QMR of the paper's experiments (Sec. 4.1) */
  int32_t batch_streams;   /* asss_solve_batched only: concurrent worker streams (one host
                              thread each), 1..16; 0 = 16 (default) */
  int32_t use_x0;          /* 0 (default): start from x = 0.  1: the output vector holds
                              the initial guess x0 on entry (NONFINITE if it has NaN/Inf);
                              the outer method corrects r0 = b - A x0 to tol ||b|| and
                              returns x0 + d.  Batched solves then run column by column */
  int32_t batch_engine;    /* asss_solve_batched only: 0 (default) = all systems in one lockstep
                              (rows of all systems concatenated; one persistent work-queue
                              launch per inner step for every system, captured in HIP graph
                              chunks; segmented outer kernels; the Hessenberg updates of all
                              columns on the device; one host round trip per outer step for
                              all columns) when every system qualifies (FGMRES from
                              zero, no fixed inner steps, <= 4 right-hand sides, k <= 16,
                              k + r <= 256, natural inner order, one device, one inner
                              precision), else per-system workers; 1 = the lockstep engine or
                              INVALID_ARG; 2 = per-system workers */
} asss_solve_opts_t;

enum { ASSS_OUTER_FGMRES = 0, ASSS_OUTER_TFQMR = 1 };

typedef struct {
  int32_t converged;
  int32_t outer_its;
  int32_t inner_its_total;
  int32_t inner_its_max;
  int32_t k_eff;           /* Lanczos vectors actually produced */
  int32_t rank_r;          /* number of negative entries of D */
  int32_t cycles;          /* FGMRES cycles (restarts + 1) */
  int32_t inner_launches;  /* launches of the fused mrs iteration kernel */
  double relres_true;      /* ||b - A x|| / ||b|| in FP64 on the original A */
  double relres_implicit;  /* FGMRES estimate on the scaled system */
  double setup_host_s;
  double setup_device_s;
  double solve_s;
  double inner_kernel_s;   /* HIP-event time of those launches (back to back on the stream) */
  int32_t reorth;          /* Arnoldi steps that needed the second Gram-Schmidt pass */
  int32_t reserved;
} asss_info_t;

/* Defaults of the option structs. */
void asss_default_setup_opts(asss_setup_opts_t* o);
void asss_default_solve_opts(asss_solve_opts_t* o);

/* Preprocess A (copied) and build the device data of the preconditioner.
 * Errors: INVALID_ARG, INVALID_CSR, NONFINITE, STRUCTURALLY_SINGULAR,
 * ZERO_DIAGONAL, LLS, HIP, OOM.  On success *out receives a new handle. */
asss_status_t asss_setup(const asss_csr_t* A, const asss_setup_opts_t* opts,
                         void* hip_stream, asss_handle_t* out);

/* x = A^-1 b (device FP64 vectors of length n).  ASSS_NOT_CONVERGED when
 * max_outer was reached (x holds the last iterate).  NONFINITE if b has a
 * NaN/Inf (x untouched).  info may be NULL. */
asss_status_t asss_solve(asss_handle_t h, const double* b_dev, double* x_dev,
                         const asss_solve_opts_t* o, asss_info_t* info, void* hip_stream);

/* For callers that cannot allocate device memory during a solve (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * asss_solve with the Krylov workspace (FGMRES: 2 restart_m + 1 vectors;
 * TFQMR: 13) and the two vectors of a solve from x0 placed in a fixed device
 * array of 128 MiB that the library holds per GPU until the process ends,
 * instead of memory the handle allocates (asss_solve grows the handle's
 * workspace on first use).  It calls no hipMalloc, hipFree or allocating
 * routine; the handle itself comes from asss_setup as usual, and b, x are the
 * caller's.  Limit: n (2 m + 3) 8 bytes <= 128 MiB with m = restart_m (FGMRES)
 * or 6 (TFQMR), e.g. n <= 127,000 at m = 64; larger problems are refused with
 * ASSS_ERR_INVALID_ARG and a message giving both sizes.  Results equal those of
 * asss_solve with the same options.  Every call on a GPU shares that GPU's
 * array and leaves its contents behind (nothing in it must start at zero):
 * calls that overlap in time on one GPU, from any thread or stream, race and
 * must not be made. */
asss_status_t asss_solve_noalloc(asss_handle_t h, const double* b_dev, double* x_dev,
                                 const asss_solve_opts_t* o, asss_info_t* info, void* hip_stream);

/* lambda = A^-T g: the same scheme on the transposed system, with P^-T
 * applied as S_bar^-T (v - U_bar Sigma_bar^T C^-T X^T v) (derived from eq.
 * smw by transposition). */
asss_status_t asss_solve_adjoint(asss_handle_t h, const double* g_dev, double* lambda_dev,
                                 const asss_solve_opts_t* o, asss_info_t* info,
                                 void* hip_stream);

/* ---- Differentiation ----------------------------------------------------
 * For x = A^-1 b and a scalar loss L(x): dL/db = lambda with A^T lambda =
 * dL/dx (asss_solve_adjoint), and dL/da_ij = -lambda_i x_j on the stored
 * entries of A (differentiating A x = b; the transposed solve is the adjoint
 * of the scheme, Sec. 3 eqs. modified and smw taken by transposition). */

/* Replace the values of A (host CSR, n as at setup) while keeping everything
 * built from the old values: matching, scaling, S, Omega, J_tilde, Q_k, X, C,
 * i.e. the preconditioner is frozen and only the outer operator, the true
 * residual and the adjoint use the new values.  Solves then return
 * A_new^-1 b to their tolerance (convergence may degrade as A_new drifts from
 * the matrix the preconditioner was built for).  The caller's entries must
 * lie in the pattern given at setup (explicit zeros there were dropped; a
 * zero outside the pattern is ignored, a nonzero outside it is INVALID_ARG;
 * stored entries the caller omits become zero).  INVALID_CSR / NONFINITE as
 * for asss_setup.  Synchronizes hip_stream. */
asss_status_t asss_update_values(asss_handle_t h, const asss_csr_t* A, void* hip_stream);

/* grad_dev[e] = -lambda_dev[i] * x_dev[colind_dev[e]] for every entry e of
 * row i of the caller's CSR pattern (device arrays: rowptr n+1 int64, colind
 * nnz int32, lambda, x length n FP64, grad nnz FP64, all owned by the caller).
 * Row pointers outside [0, nnz] or decreasing, and columns outside [0, n),
 * are skipped and reported as INVALID_CSR after the kernel (other entries are
 * written).  Synchronizes hip_stream. */
asss_status_t asss_value_gradient(asss_handle_t h, int64_t nnz, const int64_t* rowptr_dev,
                                  const int32_t* colind_dev, const double* lambda_dev,
                                  const double* x_dev, double* grad_dev, void* hip_stream);

/* Several systems, each with several right-hand sides: system s has
 * nrhs[s] columns in B_dev[s] / X_dev[s] (device, n_s x nrhs[s], column-major).
 * With FGMRES the columns of a system advance in lockstep in groups of up to
 * 4: one simultaneous mrs solve (App. B) per outer step serves the group, so
 * each inner step reads J_tilde and Q_k once for all its columns; the inner
 * stop rule is the maximum over the group.  Each column restarts and stops on
 * its own true residual.  With TFQMR, or with more than 16 deflation vectors,
 * the columns are solved one at a time.  Systems run concurrently on up to
 * batch_streams (default 16) internal streams (one host thread each; all work on
 * one handle stays on one of them), ordered after hip_stream; the call returns
 * when all are done.
 * All right-hand sides are checked for NaN/Inf first (NONFINITE, nothing
 * solved).  infos: nsys * max(nrhs) entries, row s * max(nrhs) + j (may be
 * NULL); inner_kernel_s / inner_launches are those of the column's group.
 * Returns the worst status over all columns. */
asss_status_t asss_solve_batched(int32_t nsys, const asss_handle_t* hs, const int32_t* nrhs,
                                 const double* const* B_dev, double* const* X_dev,
                                 const asss_solve_opts_t* o, asss_info_t* infos,
                                 void* hip_stream);

asss_status_t asss_destroy(asss_handle_t h);

/* Saved setups: the expensive results of asss_setup written to a file and read
 * back without recomputing them (the setup handle is the checkpoint; the paper
 * reuses one preprocessing for many right-hand sides, Sec. 4.1).
 *
 * asss_save writes A (its current values), the matching and scalings (Sec. 2),
 * S (pattern and values, Sec. 2 / App. A), the inner order and the setup
 * options (with the row-block size and column form in use) to `path`.
 *
 * asss_load reads such a file and builds a handle from it: the matching,
 * scaling and least-squares solve for S are skipped; A_hat, D, J_tilde, its
 * sliced storage, the skew-Lanczos vectors and the SMW data are rebuilt (so
 * the handle equals the saved one up to rounding).  From `opts` (may be NULL)
 * only `allocator` and `verbose` are used.  A missing, truncated or
 * inconsistent file is INVALID_ARG, detected before any device call. */
asss_status_t asss_save(asss_handle_t h, const char* path);
asss_status_t asss_load(const char* path, const asss_setup_opts_t* opts, void* hip_stream,
                        asss_handle_t* out);

/* Thread-local description of the last error (never NULL). */
const char* asss_last_error(void);

/* ---- Inspection (used by parity tests and diagnostics) ------------------ */

typedef struct {
  int64_t n, nnz_a, nnz_s, nnz_ahat, nh, lls_rows, lls_nnz;
  int32_t k_eff, rank_r, lls_its, x_its;
  int32_t row_block, nblocks;
  int64_t sell_entries_a, sell_entries_b; /* stored skew entries: in-block upper, off-block both */
  double lls_relres, lls_kkt;             /* LSQR stopping quantities */
  double lanczos_orth_err;                /* max |Q_k^T Q_k - I| */
  int32_t deflation_mode;                 /* 0 none, 1 explicit, 3 explicit with the FP32-valued basis */
  int32_t reordered;                      /* 1 if the inner system uses block order */
  int64_t cross_pairs_natural;            /* strictly upper pairs straddling two row blocks */
  int64_t cross_pairs_used;               /* the same in the order used */
  int32_t narrow_b_columns;               /* 1: off-block columns stored as 16-bit deltas
                                             from per-slot bases (grid-like patterns) */
  int32_t skew_form;                      /* column form used: 1 32-bit, 2 16-bit deltas,
                                             3 offset slots (see asss_setup_opts_t) */
  int32_t tune_n;                         /* row-block candidates timed (0: no autotune) */
  int32_t tune_rows[8];                   /* their row_block values, ascending */
  double tune_us[8];                      /* their inner-step times (microseconds) */
  double tune_s;                          /* wall time of the autotuner */
  int32_t precond;                        /* ASSS_PRECOND_* of the handle */
  int32_t ildl_n2x2;                      /* 2x2 pivot blocks of the incomplete LDL^T */
  int32_t ildl_levels_lower;              /* levels of the forward solve with Lcal */
  int32_t ildl_levels_upper;              /* levels of the backward solve with Lcal^T */
  int64_t ildl_nnz_l;                     /* strictly lower entries of L */
  int64_t ildl_dropped;                   /* entries of L dropped by droptol and fill */
  int32_t step_threads;                   /* workgroup size of the one-column FP32 inner step */
  int32_t step_threads_fp64;              /* the same for the FP64 inner step */
  int32_t ildl_explicit;                  /* 1: J_tilde of the incomplete LDL^T formed at setup */
  int32_t outer_ell;                      /* 1: the outer operator's products Abar, S (and their
                                             transposes) read sliced ELL copies, 64-row slices with
                                             at most 16 slots (rows that short) */
} asss_handle_info_t;

asss_status_t asss_get_handle_info(asss_handle_t h, asss_handle_info_t* out);

/* Copy an internal array to host memory.  *count receives the number of
 * elements; if dst is NULL only the count is returned.  Element types:
 * MATCH, NEG, S_COLIND, J_COLIND int32; S_ROWPTR, J_ROWPTR int64; others FP64.
 * Q and X are column-major n x k_eff and n x (k_eff + r). */
enum {
  ASSS_ARR_MATCH = 0,   /* m[j]: row of A matched to column j */
  ASSS_ARR_DR = 1, ASSS_ARR_DC = 2,
  ASSS_ARR_S_ROWPTR = 3, ASSS_ARR_S_COLIND = 4, ASSS_ARR_S_VAL = 5,
  ASSS_ARR_D = 6,       /* diag(A_hat) */
  ASSS_ARR_J_ROWPTR = 7, ASSS_ARR_J_COLIND = 8, ASSS_ARR_J_VAL = 9, /* strict upper J_tilde */
  ASSS_ARR_Q = 10, ASSS_ARR_ALPHA = 11, ASSS_ARR_X = 12, ASSS_ARR_NEG = 13,
  /* the incomplete LDL^T of a handle with precond = ASSS_PRECOND_ILDL (count 0 otherwise),
     and of an asss_ildl_t: */
  ASSS_ARR_ILDL_PERM = 14,     /* int32 n: position p holds index perm[p] of Abar */
  ASSS_ARR_ILDL_L_ROWPTR = 15, /* int64 n+1: strictly lower part of the unit factor L, positions */
  ASSS_ARR_ILDL_L_COLIND = 16, /* int32 */
  ASSS_ARR_ILDL_L_VAL = 17,    /* FP64 */
  ASSS_ARR_ILDL_BSIZE = 18,    /* int32 per position: 1, or 2 at the first position of a 2x2 block and
                                  0 at its second */
  ASSS_ARR_ILDL_D = 19,        /* FP64 3 per position p: (d_pp, d_{p+1,p}, d_{p+1,p+1}) at the first
                                  position of a block (zeros at the others; d of a 1x1 block in the first) */
  ASSS_ARR_LCAL_ROWPTR = 20,   /* int64 n+1: Lcal = L C, lower triangular with its diagonal, positions */
  ASSS_ARR_LCAL_COLIND = 21,   /* int32 */
  ASSS_ARR_LCAL_VAL = 22,      /* FP64 */
  ASSS_ARR_UR = 23,            /* FP64 n x r column-major: U_r of the low-rank term, positions */
  ASSS_ARR_SIGMA_R = 24        /* FP64 r: the diagonal of Sigma_r */
};
asss_status_t asss_get_array(asss_handle_t h, int32_t which, void* dst, int64_t* count);

/* Apply one operator of the method to a device FP64 vector (length n):
 *   OP_SKEW       out = J_tilde in                    (FP64, or FP32 if o->inner_fp32 == 1)
 *   OP_DEFLATED   out = J_bar in
 *   OP_OUTER      out = Omega Abar S Omega in
 *   OP_OUTER_T    out = (Omega Abar S Omega)^T in
 *   OP_MRS        out = mrs solution of (I + J_bar) out = in   (o: inner_tol/maxit/fixed)
 *   OP_PREC       out = P^-1 in   (eq. smw around mrs)
 *   OP_PREC_T     out = P^-T in
 *   OP_A, OP_AT   out = A in, A^T in
 * *inner_its (may be NULL) receives the mrs iteration count. */
enum {
  ASSS_OP_SKEW = 0, ASSS_OP_DEFLATED = 1, ASSS_OP_OUTER = 2, ASSS_OP_OUTER_T = 3,
  ASSS_OP_MRS = 4, ASSS_OP_PREC = 5, ASSS_OP_PREC_T = 6, ASSS_OP_A = 7, ASSS_OP_AT = 8
};
asss_status_t asss_apply(asss_handle_t h, int32_t op, const double* in_dev, double* out_dev,
                         const asss_solve_opts_t* o, int32_t* inner_its, void* hip_stream);

/* ---- The incomplete LDL^T alone, on the host (no device is used) --------
 * For inspection and tests: the Bunch-Kaufman incomplete factorization of a
 * symmetric matrix M (host CSR, exactly symmetric in pattern and values, else
 * INVALID_ARG) with the options of asss_setup_opts_t, its scaled factor and
 * low-rank term, exactly as a handle with precond = ASSS_PRECOND_ILDL builds
 * them from M_hat.  asss_ildl_get reads the ASSS_ARR_ILDL_* / LCAL / UR /
 * SIGMA_R arrays as asss_get_array does.  ZERO_DIAGONAL as for asss_setup. */
typedef struct asss_ildl_s* asss_ildl_t;
asss_status_t asss_ildl_factor(const asss_csr_t* M, double droptol, double fill, int32_t pivoting,
                               asss_ildl_t* out);
asss_status_t asss_ildl_get(asss_ildl_t f, int32_t which, void* dst, int64_t* count);
asss_status_t asss_ildl_destroy(asss_ildl_t f);

#ifdef __cplusplus
}
#endif
#endif /* ASSS_H */
