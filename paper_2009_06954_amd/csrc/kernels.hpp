// Device data structures and kernel launchers of libasss (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace asss {

constexpr int WG = 256;        // threads per workgroup of the streaming kernels
constexpr int KMAX = 32;       // largest k the fused mrs kernels accept
constexpr int NRMAX = 4;       // columns of the multi-column mrs kernels
constexpr int RED_SLOTS = 136; // values per workgroup partial (>= (16+1)*4, >= restart + 1)

// CSR on the device, FP64 values.
struct DCsr {
  int64_t nrows = 0, ncols = 0, nnz = 0;
  int64_t* ptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
  int lanes = 1;  // lanes per row of the vector SpMV kernel; 0: one row per thread
};

// Sliced skew operator (see host_setup.hpp: SkewSell).
template <typename T>
struct DSkew {
  int32_t n = 0, R = 0, nblocks = 0, nslices = 0;
  const int32_t* a_width = nullptr;
  const int32_t* b_width = nullptr;
  const int64_t* a_off = nullptr;
  const int64_t* b_off = nullptr;
  const uint16_t* a_col = nullptr;
  const int32_t* b_col = nullptr;   // wide part-b columns (b_narrow == 0)
  const uint16_t* b_cd = nullptr;   // narrow: column = b_base[b_off / 64 + slot] + b_cd
  const int32_t* b_base = nullptr;  // slots: column of lane 0 = first row of the slice + d
  const int32_t* a_doff = nullptr;  // slots: part-a offset d > 0 per slot (a_off / 64 + slot)
  int32_t b_narrow = 0;
  int32_t form = 1;                 // 1: 32-bit part-b columns, 2: 16-bit deltas, 3: offset slots
  int32_t threads = 0;              // workgroup size of the one-column FP32 inner step (0: 256)
  // explicit form (dense != nullptr): J_tilde row-major, n x n, leading
  // dimension dense_ld, exactly skew; the block pass is a dense row product
  const T* dense = nullptr;
  int64_t dense_ld = 0;
  const T* a_val = nullptr;
  const T* b_val = nullptr;
};

// Scalar state of one mrs column (App. B): the Givens recurrence plus the
// bookkeeping of the deferred normalisation and of the p/x update that is
// applied one iteration late (fused into the next operator pass).
struct MrsCol {
  double nu;          // q_t = w_t / nu
  double nu_old;      // q_{t-1} = w_{t-1} / nu_old
  double beta_prev;   // beta_{t-1}
  double theta1, c_old, s_old, delta_old, g, r0;
  double pend_theta, pend_delta, pend_coef;
  int32_t has_pending, live;
};

static_assert(sizeof(MrsCol) % 8 == 0, "MrsCol is copied as doubles");

enum { MRS_RUNNING = 0, MRS_CONVERGED = 1, MRS_DONE = 2 };

struct MrsState {
  int32_t its, status, nr, k;
  int32_t maxit, fixed, sign, pad;
  double tol, alpha, relres_max;
  double cvec[KMAX * NRMAX];   // S_k (Q_k^T q_t) per column, column c at [c * KMAX]
  MrsCol col[NRMAX];
};

// Per-solve device buffers of the inner mrs (inner precision T, n x NR row-major).
template <typename T>
struct MrsBufs {
  T* w[3];
  T* p[2];
  T* x;
};

struct Reducer {
  double* partials = nullptr;   // [max_groups * RED_SLOTS]
  unsigned* tickets = nullptr;  // one per reduction site
  int max_groups = 0;
};

// ---- launchers (all asynchronous on `s`) ----------------------------------

// y = rs o (M (cs o x))   [mode 0],  y = b - rs o (M (cs o x))   [mode 1]
void spmv(const DCsr& M, const double* x, double* y, const double* rs, const double* cs,
          int mode, const double* b, hipStream_t s);

// y = J_tilde x on the sliced layout (T precision in and out).
template <typename T>
void skew_spmv(const DSkew<T>& J, const T* x, T* y, hipStream_t s);

// out[l * nr + c] = sum_i A[l * lda + i] * B[i * nr + c] for l < ka, c < nr
// (FP64 accumulation, deterministic order), reduced into `out` on the device.
// If M != nullptr (nr == 1), out = M (ka x ka, row-major) applied to that product.
template <typename TA, typename TB>
void gemm_tn(int64_t n, int ka, const TA* A, int64_t lda, const TB* B, int nr, double* out,
             const double* M, Reducer& red, int site, hipStream_t s);

// y[i] += sign * sum_l A[l * lda + i] * t[l]   (y, A FP64; t device FP64)
void gemv_acc(int64_t n, int kt, const double* A, int64_t lda, const double* t, double sign,
              double* y, hipStream_t s);

// y += sign * A t and *nrm2 = ||y||^2 (deterministic reduction)
void gemv_acc_norm(int64_t n, int kt, const double* A, int64_t lda, const double* t, double sign,
                   double* y, double* nrm2, Reducer& red, int site, hipStream_t s);

// y = a * x (FP64)   and   y = x / sqrt(*nrm2) (device scalar)
void scale(int64_t n, double a, const double* x, double* y, hipStream_t s);
void normalize(int64_t n, const double* x, const double* nrm2, double* y, hipStream_t s);
void axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);  // y = a x + b y
// y[j] = omega[j] * (dr[j] * x[m[j]])
void gather_scale(int64_t n, const int32_t* m, const double* dr, const double* omega, const double* x,
                  double* y, hipStream_t s);
// y[m[j]] = dr[j] * (omega[j] * x[j])
void scatter_scale(int64_t n, const int32_t* m, const double* dr, const double* omega, const double* x,
                   double* y, hipStream_t s);
void cast_d2f(int64_t n, const double* x, float* y, hipStream_t s);
void cast_f2d(int64_t n, const float* x, double* y, hipStream_t s);
void splitmix_vector(int64_t n, uint64_t seed, double* y, hipStream_t s);
// non-finite check: *flag = 1 if any entry of x is NaN/Inf
void check_finite(int64_t n, const double* x, int* flag, hipStream_t s);
// Qs (sliced, nslices * 64 * k, zero padded) from column-major Q (n x k)
template <typename T>
void slice_columns(int64_t n, int k, const T* Q, T* Qs, hipStream_t s);

// ---- inner mrs --------------------------------------------------------------

struct MrsLaunch {
  int64_t n;
  int nr;           // active columns (<= NR of the kernel)
  int k;            // deflation vectors (0 = none)
  const double* alpha_dev;  // k-1 skew-Lanczos coefficients
  int sign;         // +1: K = J_bar,  -1: K = -J_bar
  // Q_k in sliced layout for the iteration kernel: row i, column l at
  // (i / 64) * (kq * 64) + l * 64 + i % 64 (each 64-row slice contiguous;
  // kq = k for one system, the batch's largest k in a batched launch)
  const void* Qs;
  int kq;
  // G = Q_k^T Q_k (k x k, FP64) of Q_k as stored in the inner precision: the
  // iteration kernel forms Q_k^T q_new as Q_k^T a - sign G c (see k_mrs_iter)
  const double* gram;
  // 1: Qs holds FP32 values for an FP64 kernel (a deflation basis rounded to
  // FP32 values at setup, so that the FP32 copy is exact)
  int q32;
};

// A batch of systems for the batched inner kernels: rows of all systems
// concatenated, each system padded to whole blocks of the common row block;
// per system its state, partial sums, ticket, Lanczos coefficients, Gram
// matrix (FP64 kernels) and number of deflation vectors.
struct MrsBatchSys {
  MrsState* st;
  double* partials;      // nblocks * RED_SLOTS values
  unsigned* ticket;
  const double* alpha;   // k - 1 skew-Lanczos coefficients
  const double* gram;    // k x k, Q_k^T Q_k of the stored inner-precision basis
  int k;                 // deflation vectors of this system (<= kq)
  int nblocks;           // row blocks of this system
  int first_block;       // its first block in the batch
  int pad;
};

struct MrsBatch {
  int64_t n;             // rows of the batch (padded)
  int nblocks;           // row blocks of the batch
  int kq;                // stride of the sliced basis (largest k)
  int sign;              // +1: K = J_bar
  const MrsBatchSys* sys;
  const int32_t* block_sys;  // system of every block
  unsigned* queue;           // work-queue counter (0 between launches)
  const void* Qs;            // sliced basis of the batch (inner precision)
};

// Batched start and step (all systems of B; rhs column c of the batch at
// rhs + c * ldr, no inner permutation).  `groups` workgroups take the row
// blocks from B.queue.
template <typename T, int NR>
void mrs_init_batched(const MrsBatch& B, const DSkew<T>& J, const double* rhs, int64_t ldr, MrsBufs<T>& buf,
                      double tol, int maxit, int fixed, int kf, int groups, hipStream_t s);
template <typename T, int NR>
void mrs_iter_batched(const MrsBatch& B, const DSkew<T>& J, MrsBufs<T>& buf, int kf, int groups, hipStream_t s);

// Initialise: w1 = rhs (col c at rhs + c * ldr), zero the other buffers,
// r0 = ||rhs_c||, d = Q^T q_1, c = S_k d.
// perm (new -> old, may be null): row i of the inner system is row perm[i] of rhs.
template <typename T, int NR>
void mrs_init(const MrsLaunch& L, const double* rhs, int64_t ldr, const int32_t* perm, const T* Q,
              MrsBufs<T>& buf, MrsState* st, double tol, int maxit, int fixed, Reducer& red,
              hipStream_t s);

// One iteration of App. B (or the final deferred update once converged, or
// nothing once done), fused with the skew operator and the deflation.
template <typename T, int NR>
void mrs_iter(const MrsLaunch& L, const DSkew<T>& J, const T* Q, MrsBufs<T>& buf, MrsState* st,
              Reducer& red, hipStream_t s);

// Copy the inner solution out: out (FP64, column c at out + c * ldo) = x.
template <typename T, int NR>
void mrs_output(int64_t n, int nr, const MrsBufs<T>& buf, const int32_t* perm, double* out, int64_t ldo,
                hipStream_t s);

// g[e] = -lam[i] x[col[e]] over the entries e of every row i of a CSR pattern
// (device arrays, checked while read: *bad = 1 on an invalid entry range or column)
void csr_value_grad(int64_t n, int64_t nnz, const int64_t* ptr, const int32_t* col, const double* lam,
                    const double* x, double* g, int* bad, hipStream_t s);

// y[i] = x[perm[i]] (gather) and y[perm[i]] = x[i] (scatter), FP64
void permute_gather(int64_t n, const int32_t* perm, const double* x, double* y, hipStream_t s);
void permute_scatter(int64_t n, const int32_t* perm, const double* x, double* y, hipStream_t s);

}  // namespace asss
