// Device side of the Hessenberg least-squares problem of flexible GMRES
// (definitions in outer.hip).  Each outer column owns a workspace of
// hess_slot(cap) doubles in device memory for restart lengths m <= cap:
// H ((m+1) x m, leading dimension m), the rotations cs and sn, the rotated
// right-hand side g, its entries before rotation gp, the cycle's solution y
// and HESS_OUT values read back by the host.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace asss {

constexpr int HESS_MMAX = 250;
constexpr int HESS_OUT = 8;
constexpr int64_t hess_slot(int cap) { return (int64_t)(cap + 1) * cap + 5 * (int64_t)cap + 1 + HESS_OUT; }
constexpr int64_t HESS_SLOT = hess_slot(HESS_MMAX);

// out[0] = |g_{j+1}| after step j (the residual estimate of the scaled
// system), out[1] = h_{j+1,j}, out[2] = 1 when step j needs a second
// Gram-Schmidt pass (nothing else was done), out[3] = 1 when out[0] <= thr.
// Single column (cap = HESS_MMAX): out lies in the workspace.
double* hess_out(double* W);
// the combination y of the preconditioned vectors, written by hess_solve
double* hess_y(double* W);

// Start of a cycle: g = beta e_1.
void hess_reset(double* W, double beta, hipStream_t s);
// Step j: the Hessenberg column from the Gram-Schmidt coefficients h1 (j + 1
// values, then ||w||^2 and the squared norm after the pass) and, in mode 1,
// h2 (j + 1 values of the second pass, then the squared norm after it);
// earlier rotations, the new rotation, the residual estimate and the test
// against thr.  Repeating a step with the same inputs gives the same result.
void hess_step(double* W, const double* h1, const double* h2, int j, int m, int mode, double thr, hipStream_t s);
// End of a cycle: y = R^-1 g over the first jused columns.
void hess_solve(double* W, int jused, int m, hipStream_t s);

// The same for ncol columns at once (workspace of column q at W + q
// hess_slot(cap), one wavefront per column).  reset: columns with beta[q] >= 0.
// step: columns with jv[q] >= 0 (and sel[q] != 0 in mode 1); coefficients
// of column q at h1 + q ldh (h2 + q ldh), ||w||^2 in wn2[q], the squared
// norm after the pass in hn2[q], threshold thr[q]; out + q HESS_OUT as above.
// solve: columns with jused[q] > 0, y of column q at y + q m.
void hess_reset_batched(double* W, int cap, int ncol, const double* beta, hipStream_t s);
void hess_step_batched(double* W, int cap, int m, int ncol, const int32_t* jv, const int32_t* sel, int mode,
                       const double* h1, const double* h2, int ldh, const double* wn2, const double* hn2,
                       const double* thr, double* out, hipStream_t s);
void hess_solve_batched(double* W, int cap, int m, int ncol, const int32_t* jused, double* y, hipStream_t s);

// y = M x for a dense row-major n x n matrix M (leading dimension n): one
// wave per row, coalesced row loads, a fixed summation order.
void dense_rows(int64_t n, const double* M, const double* x, double* y, hipStream_t s);

// Sliced ELL copy of a CSR matrix whose rows have at most SELL_MAXW entries:
// slices of 64 rows (the last one filled up with empty rows), slice s holds
// width[s] slots (its longest row) at off[s], slot u of row 64 s + l at
// off[s] + 64 u + l; a row's entries in its CSR order, then padding with value
// 0 and the column of the row's first entry (column 0 for an empty row).
constexpr int SELL_MAXW = 16;
struct DSell {
  int64_t nrows = 0;  // 0: no copy
  int64_t entries = 0;  // stored slots, padding included
  const int32_t* width = nullptr;
  const int64_t* off = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
};
// y = rs o (M (cs o x)) (rs, cs may be null), one row per thread; the same
// products and summation order as the one-row-per-thread CSR kernel.
void spmv_sell(const DSell& M, const double* x, double* y, const double* rs, const double* cs, hipStream_t s);
// y = sa (M x) + sb y (y is not read when sb == 0; x and y must not overlap),
// the same row sums.  With part (ceil(nrows / 256) values), part[b] = the sum
// of the new y_i^2 over rows 256 b .. 256 b + 255; sum_parts then adds the
// np values of part in a fixed order into out[0] (part must hold np + 256
// values: the 256 after the np take partial sums).
void spmv_sell_acc(const DSell& M, const double* x, double* y, double sa, double sb, double* part,
                   hipStream_t s);
void sum_parts(int64_t np, double* part, double* out, hipStream_t s);

// The copy is built on the device from CSR arrays of n rows (ptr n + 1 int64,
// col int32, val FP64, sorted rows): ell_widths writes the ceil(n / 64) slice
// widths (each slice's longest row, clamped to INT32_MAX); with width and off
// in place (off[s] = 64 x the widths before s), ell_fill writes every slot,
// padding included.  Running ell_fill again after new values of the same
// pattern refreshes the copy.
void ell_widths(int64_t n, const int64_t* ptr, int32_t* width, hipStream_t s);
void ell_fill(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, const int32_t* width,
              const int64_t* off, int32_t* ecol, double* eval, hipStream_t s);

}  // namespace asss
