// Device side of the Hessenberg least-squares problem of flexible GMRES
// (definitions in outer.hip).  Each outer column owns a workspace of
// HESS_SLOT doubles in device memory; restart lengths up to HESS_MMAX.
#pragma once

#include <hip/hip_runtime.h>

namespace asss {

constexpr int HESS_MMAX = 250;
// H ((m+1) x m), cs, sn, g (rotated), gp (before rotation), y, out
constexpr int HESS_SLOT = (HESS_MMAX + 1) * HESS_MMAX + 5 * HESS_MMAX + 16;

// out[0] = |g_{j+1}| after step j (the residual estimate of the scaled
// system), out[1] = h_{j+1,j}, out[2] = 1 when step j needs a second
// Gram-Schmidt pass (nothing else was done), out[3] = 1 when out[0] <= thr,
// out[4] = |g_jused| after hess_solve.
constexpr int HESS_OUT = 8;
double* hess_out(double* W);
// the combination y of the preconditioned vectors, written by hess_solve
double* hess_y(double* W);

// Start of a cycle: g = beta e_1.
void hess_reset(double* W, double beta, hipStream_t s);
// Step j: the Hessenberg column from the Gram-Schmidt coefficients h1 (j + 1
// values, then ||w||^2 and the norm after the pass) and, in mode 1, h2 (j + 1
// values of the second pass, then the norm after it); earlier rotations, the
// new rotation and the residual estimate; thr: the stopping threshold of the
// estimate.  Repeating a step with the same inputs gives the same result.
void hess_step(double* W, const double* h1, const double* h2, int j, int m, int mode, double thr, hipStream_t s);
// End of a cycle: y = R^-1 g over the first jused columns.
void hess_solve(double* W, int jused, int m, hipStream_t s);

}  // namespace asss
