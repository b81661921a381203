// The Hessenberg part of flexible GMRES on the device, in FP64: the column of
// an Arnoldi step from its Gram-Schmidt coefficients, the Givens rotations of
// its QR factorization, the rotated right-hand side whose last entry is the
// residual estimate, the stopping test on it, and at the end of a cycle the
// small triangular solve for the combination of the preconditioned vectors.
// The work is O(j) per step (j <= 250) and sequential: one thread does it, so
// the result does not depend on timing.
#include <hip/hip_runtime.h>

#include "outer_kernels.hpp"

namespace asss {

namespace {

// Workspace of one column (doubles): H row-major (m+1) x m at 0 (leading
// dimension m), then cs, sn, g, gp (MMAX + 1), y, out.
constexpr int OFF_CS = (HESS_MMAX + 1) * HESS_MMAX;
constexpr int OFF_SN = OFF_CS + HESS_MMAX;
constexpr int OFF_G = OFF_SN + HESS_MMAX;
constexpr int OFF_GP = OFF_G + HESS_MMAX;
constexpr int OFF_Y = OFF_GP + HESS_MMAX + 1;
constexpr int OFF_OUT = OFF_Y + HESS_MMAX;
static_assert(OFF_OUT + HESS_OUT <= HESS_SLOT, "Hessenberg workspace");

__global__ void k_hess_reset(double* W, double beta) {
  const int t = threadIdx.x;
  if (t == 0) W[OFF_GP] = beta;
  if (t < HESS_OUT) W[OFF_OUT + t] = 0.0;
}

// gp[j] is the entry j of the right-hand side before step j's rotation, so
// the step reads only values no later step of the cycle writes and can be
// repeated.  Mode 0 with ||w'||^2 < 0.1 ||w||^2 (the vector kept less than
// 1/sqrt(10) of its norm in the first pass) only flags the second pass.
// One wavefront: the lanes stage the column and the earlier rotations in
// LDS, lane 0 applies the rotations (a chain of dependent FMAs whose LDS
// loads do not depend on it), the lanes write the column back.
__global__ void __launch_bounds__(64) k_hess_step(double* W, const double* h1, const double* h2, int j, int m,
                                                   int mode, double thr) {
  __shared__ double col[HESS_MMAX + 1], c_s[HESS_MMAX], s_s[HESS_MMAX];
  const int t = threadIdx.x;
  double* out = W + OFF_OUT;
  double hn2;
  if (mode == 0) {
    hn2 = h1[j + 2];
    if (hn2 < 0.1 * h1[j + 1]) {
      if (t == 0) out[2] = 1.0;
      return;
    }
    for (int i = t; i <= j; i += 64) col[i] = h1[i];
  } else {
    for (int i = t; i <= j; i += 64) col[i] = h1[i] + h2[i];
    hn2 = h2[j + 1];
  }
  for (int i = t; i < j; i += 64) {
    c_s[i] = W[OFF_CS + i];
    s_s[i] = W[OFF_SN + i];
  }
  __syncthreads();
  if (t == 0) {
    const double hn = sqrt(hn2);
    double a = col[0];
    for (int i = 0; i < j; ++i) {  // the rotations of the earlier columns
      const double b = col[i + 1];
      col[i] = c_s[i] * a + s_s[i] * b;
      a = -s_s[i] * a + c_s[i] * b;
    }
    const double rr = hypot(a, hn);
    double c = 1.0, sv = 0.0;
    if (rr != 0.0) {
      c = a / rr;
      sv = hn / rr;
    }
    W[OFF_CS + j] = c;
    W[OFF_SN + j] = sv;
    col[j] = rr;
    const double gj = W[OFF_GP + j];
    W[OFF_G + j] = c * gj;
    const double gn = -sv * gj;
    W[OFF_GP + j + 1] = gn;
    out[0] = fabs(gn);
    out[1] = hn;
    out[2] = 0.0;
    out[3] = fabs(gn) <= thr ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int i = t; i <= j; i += 64) W[i * m + j] = col[i];
  if (t == 0) W[(j + 1) * m + j] = 0.0;
}

// Back substitution by columns in one wavefront: lane l keeps the entries
// g_i with i = l (mod 64) in registers; for i = jused-1 down to 0 the owner
// forms y_i, broadcasts it, and every lane removes R_{:,i} y_i from its
// entries above i.
__global__ void __launch_bounds__(64) k_hess_solve(double* W, int jused, int m) {
  constexpr int PER = (HESS_MMAX + 63) / 64;
  const int t = threadIdx.x;
  const double* H = W;
  double r[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = t + 64 * q;
    r[q] = i < jused ? W[OFF_G + i] : 0.0;
  }
  for (int i = jused - 1; i >= 0; --i) {
    const int owner = i & 63, q_i = i >> 6;
    double mine = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q)
      if (q == q_i) mine = r[q];
    double yi = mine / H[i * m + i];
    yi = __shfl(yi, owner, 64);
    if (t == owner) W[OFF_Y + i] = yi;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int l = t + 64 * q;
      if (l < i) r[q] -= H[l * m + i] * yi;
    }
  }
  if (t == 0) W[OFF_OUT + 4] = fabs(W[OFF_GP + jused]);
}

}  // namespace

double* hess_out(double* W) { return W + OFF_OUT; }
double* hess_y(double* W) { return W + OFF_Y; }

void hess_reset(double* W, double beta, hipStream_t s) {
  hipLaunchKernelGGL(k_hess_reset, dim3(1), dim3(64), 0, s, W, beta);
}

void hess_step(double* W, const double* h1, const double* h2, int j, int m, int mode, double thr, hipStream_t s) {
  hipLaunchKernelGGL(k_hess_step, dim3(1), dim3(64), 0, s, W, h1, h2, j, m, mode, thr);
}

void hess_solve(double* W, int jused, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_hess_solve, dim3(1), dim3(64), 0, s, W, jused, m);
}

}  // namespace asss
