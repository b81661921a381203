// The Hessenberg part of flexible GMRES on the device, in FP64: the column of
// an Arnoldi step from its Gram-Schmidt coefficients, the Givens rotations of
// its QR factorization, the rotated right-hand side whose last entry is the
// residual estimate, the stopping test on it, and at the end of a cycle the
// small triangular solve for the combination of the preconditioned vectors.
// The work is O(j) per step (j <= 250) and sequential: one wavefront per
// column, and the rotation chain in one lane, so the result does not depend
// on timing.  Also the dense outer operator of the incomplete LDL^T formed
// at setup (dense_rows).
#include <hip/hip_runtime.h>

#include "outer_kernels.hpp"

namespace asss {

namespace {

// Offsets (doubles) in a column's workspace for restart lengths up to cap.
struct Lay {
  int cap;
  __host__ __device__ int64_t cs() const { return (int64_t)(cap + 1) * cap; }
  __host__ __device__ int64_t sn() const { return cs() + cap; }
  __host__ __device__ int64_t g() const { return sn() + cap; }
  __host__ __device__ int64_t gp() const { return g() + cap; }
  __host__ __device__ int64_t y() const { return gp() + cap + 1; }
  __host__ __device__ int64_t out() const { return y() + cap; }
};
static_assert(hess_slot(HESS_MMAX) == (int64_t)(HESS_MMAX + 1) * HESS_MMAX + 5 * HESS_MMAX + 1 + HESS_OUT,
              "workspace size");

__device__ void reset_column(double* W, const Lay& L, double beta, double* out) {
  const int t = threadIdx.x;
  if (t == 0) W[L.gp()] = beta;
  if (t < HESS_OUT) out[t] = 0.0;
}

// gp[j] is the entry j of the right-hand side before step j's rotation, so
// the step reads only values no later step of the cycle writes and can be
// repeated.  The caller's lanes have put the new column (j + 1 values) in
// col; the lanes stage the earlier rotations in LDS, lane 0 applies them (a
// chain of dependent FMAs whose LDS loads do not depend on it) and the new
// one, and the lanes write the column back.  One wavefront per column.
__device__ void rotate_column(double* W, const Lay& L, int j, int m, double hn2, double thr, double* col,
                              double* c_s, double* s_s, double* out) {
  const int t = threadIdx.x;
  for (int i = t; i < j; i += 64) {
    c_s[i] = W[L.cs() + i];
    s_s[i] = W[L.sn() + i];
  }
  __syncthreads();
  if (t == 0) {
    const double hn = sqrt(fmax(hn2, 0.0));
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
    W[L.cs() + j] = c;
    W[L.sn() + j] = sv;
    col[j] = rr;
    const double gj = W[L.gp() + j];
    W[L.g() + j] = c * gj;
    const double gn = -sv * gj;
    W[L.gp() + j + 1] = gn;
    out[0] = fabs(gn);
    out[1] = hn;
    out[2] = 0.0;
    out[3] = fabs(gn) <= thr ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int i = t; i <= j; i += 64) W[(int64_t)i * m + j] = col[i];
  if (t == 0) W[(int64_t)(j + 1) * m + j] = 0.0;
}

// Mode 0 with ||w'||^2 < 0.1 ||w||^2 (the vector kept less than 1/sqrt(10)
// of its norm in the first pass) only flags the second pass.
__device__ void step_column(double* W, const Lay& L, int j, int m, int mode, const double* h1, const double* h2,
                            double wn2, double hn2, double thr, double* out) {
  __shared__ double col[HESS_MMAX + 1], c_s[HESS_MMAX], s_s[HESS_MMAX];
  const int t = threadIdx.x;
  if (mode == 0) {
    if (hn2 < 0.1 * wn2) {
      if (t == 0) out[2] = 1.0;
      return;
    }
    for (int i = t; i <= j; i += 64) col[i] = h1[i];
  } else {
    for (int i = t; i <= j; i += 64) col[i] = h1[i] + h2[i];
  }
  rotate_column(W, L, j, m, hn2, thr, col, c_s, s_s, out);
}

// Back substitution by columns in one wavefront: lane l keeps the entries
// g_i with i = l (mod 64) in registers; for i = jused-1 down to 0 the owner
// forms y_i, broadcasts it, and every lane removes R_{:,i} y_i from its
// entries above i.
__device__ void solve_column(const double* W, const Lay& L, int jused, int m, double* y) {
  constexpr int PER = (HESS_MMAX + 63) / 64;
  const int t = threadIdx.x;
  double r[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = t + 64 * q;
    r[q] = i < jused ? W[L.g() + i] : 0.0;
  }
  for (int i = jused - 1; i >= 0; --i) {
    const int owner = i & 63, q_i = i >> 6;
    double mine = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q)
      if (q == q_i) mine = r[q];
    double yi = mine / W[(int64_t)i * m + i];
    yi = __shfl(yi, owner, 64);
    if (t == owner) y[i] = yi;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int l = t + 64 * q;
      if (l < i) r[q] -= W[(int64_t)l * m + i] * yi;
    }
  }
}

__global__ void __launch_bounds__(64) k_hess_reset(double* W, double beta) {
  const Lay L{HESS_MMAX};
  reset_column(W, L, beta, W + L.out());
}

// h1: j + 1 coefficients, ||w||^2 at h1[j + 1], the squared norm after the
// pass at h1[j + 2]; h2 (mode 1): j + 1 coefficients, the squared norm after
// the second pass at h2[j + 1].
__global__ void __launch_bounds__(64) k_hess_step(double* W, const double* h1, const double* h2, int j, int m,
                                                   int mode, double thr) {
  const Lay L{HESS_MMAX};
  const double wn2 = h1[j + 1];
  const double hn2 = mode == 0 ? h1[j + 2] : h2[j + 1];
  step_column(W, L, j, m, mode, h1, h2, wn2, hn2, thr, W + L.out());
}

__global__ void __launch_bounds__(64) k_hess_solve(double* W, int jused, int m) {
  const Lay L{HESS_MMAX};
  solve_column(W, L, jused, m, W + L.y());
}

__global__ void __launch_bounds__(64) k_hess_reset_batched(double* W, int cap, const double* beta) {
  const int q = blockIdx.x;
  const double b = beta[q];
  if (b < 0.0) return;
  const Lay L{cap};
  double* Wq = W + (int64_t)q * hess_slot(cap);
  reset_column(Wq, L, b, Wq + L.out());
}

__global__ void __launch_bounds__(64) k_hess_step_batched(double* W, int cap, int m, const int32_t* jv,
                                                           const int32_t* sel, int mode, const double* h1,
                                                           const double* h2, int ldh, const double* wn2,
                                                           const double* hn2, const double* thr, double* out) {
  const int q = blockIdx.x;
  const int j = jv[q];
  if (j < 0 || (mode == 1 && sel[q] == 0)) return;
  const Lay L{cap};
  step_column(W + (int64_t)q * hess_slot(cap), L, j, m, mode, h1 + (int64_t)q * ldh,
              mode == 1 ? h2 + (int64_t)q * ldh : nullptr, wn2[q], hn2[q], thr[q], out + (int64_t)q * HESS_OUT);
}

__global__ void __launch_bounds__(64) k_hess_solve_batched(double* W, int cap, int m, const int32_t* jused,
                                                            double* y) {
  const int q = blockIdx.x;
  const int ju = jused[q];
  if (ju <= 0) return;
  const Lay L{cap};
  solve_column(W + (int64_t)q * hess_slot(cap), L, ju, m, y + (int64_t)q * m);
}

__global__ void __launch_bounds__(256) k_dense_rows(int64_t n, const double* __restrict__ M,
                                                    const double* __restrict__ x, double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  const double* __restrict__ row = M + r * n;
  double acc = 0.0;
  int64_t j = lane;
  for (; j + 7 * 64 < n; j += 8 * 64) {
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = __builtin_nontemporal_load(&row[j + u * 64]);
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += a[u] * x[j + u * 64];
  }
  for (; j < n; j += 64) acc += row[j] * x[j];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) y[r] = acc;
}

// One row per thread, a slice per wave: the slot loads of a wave are 64
// consecutive values (coalesced), all of a row's loads are issued before its
// gathers, and the row is summed in its CSR order.  ACC: y = sa sum + sb y.
__device__ __forceinline__ double sell_row(int64_t sl, int lane, const int32_t* __restrict__ width,
                                           const int64_t* __restrict__ off, const int32_t* __restrict__ col,
                                           const double* __restrict__ val, const double* __restrict__ x,
                                           const double* __restrict__ cs) {
  const int w = __builtin_amdgcn_readfirstlane(width[sl]);
  const int64_t base = off[sl] + lane;
  int32_t c[SELL_MAXW];
  double v[SELL_MAXW];
#pragma unroll
  for (int u = 0; u < SELL_MAXW; ++u)
    if (u < w) {
      c[u] = __builtin_nontemporal_load(&col[base + (int64_t)u * 64]);
      v[u] = __builtin_nontemporal_load(&val[base + (int64_t)u * 64]);
    }
  double sum = 0.0;
#pragma unroll
  for (int u = 0; u < SELL_MAXW; ++u)
    if (u < w) sum += v[u] * (cs ? cs[c[u]] * x[c[u]] : x[c[u]]);
  return sum;
}

// ACC: y = sa sum + sb y, and with part, the block's sum of the new y_i^2 in
// part[blockIdx.x] (wave sums, then the four waves in a fixed order).
template <bool ACC>
__global__ void __launch_bounds__(256) k_spmv_sell(int64_t n, const int32_t* __restrict__ width,
                                                   const int64_t* __restrict__ off, const int32_t* __restrict__ col,
                                                   const double* __restrict__ val, const double* __restrict__ x,
                                                   double* __restrict__ y, const double* __restrict__ rs,
                                                   const double* __restrict__ cs, double sa, double sb,
                                                   double* __restrict__ part) {
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t sl = row >> 6;
  const int lane = threadIdx.x & 63;
  if (!ACC) {
    if (sl * 64 >= n) return;  // the whole wave is past the last slice
    const double sum = sell_row(sl, lane, width, off, col, val, x, cs);
    if (row < n) y[row] = rs ? rs[row] * sum : sum;
    return;
  }
  double yv = 0.0;
  if (sl * 64 < n) {
    const double sum = sell_row(sl, lane, width, off, col, val, x, cs);
    if (row < n) {
      yv = sb == 0.0 ? sa * sum : sa * sum + sb * y[row];
      y[row] = yv;
    }
  }
  if (part) {  // the same for the whole grid: every thread reaches the barrier
    __shared__ double wsum[4];
    double q = yv * yv;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) q += __shfl_xor(q, o, 64);
    if (lane == 0) wsum[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
  }
}

// out[b] = the sum of workgroup b's contiguous share of part[0 .. np): thread
// t adds its values t, t + 1024, ... of the share in turn, then a fixed tree
// over the threads.
__global__ void __launch_bounds__(1024) k_sum_parts(int64_t np, const double* __restrict__ part,
                                                    double* __restrict__ out) {
  __shared__ double red[1024];
  const int64_t chunk = (np + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < np ? lo + chunk : np;
  double a = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 1024) a += part[i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int h = 512; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// One wave per slice, one lane per row: the row lengths' maximum over the wave.
__global__ void __launch_bounds__(256) k_ell_widths(int64_t n, const int64_t* __restrict__ ptr,
                                                    int32_t* __restrict__ width) {
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t sl = row >> 6;
  if (sl * 64 >= n) return;  // the whole wave is past the last slice
  int len = 0;
  if (row < n) {
    const int64_t l = ptr[row + 1] - ptr[row];
    len = l < (int64_t)INT32_MAX ? (int)l : INT32_MAX;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) len = max(len, __shfl_xor(len, o, 64));
  if ((threadIdx.x & 63) == 0) width[sl] = len;
}

// One thread per row of the padded slices: its entries in CSR order, then the
// padding (value 0, the column of its first entry, column 0 if it has none).
__global__ void __launch_bounds__(256) k_ell_fill(int64_t n, const int64_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ col, const double* __restrict__ val,
                                                  const int32_t* __restrict__ width,
                                                  const int64_t* __restrict__ off, int32_t* __restrict__ ecol,
                                                  double* __restrict__ eval) {
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t sl = row >> 6;
  if (sl * 64 >= n) return;
  const int lane = threadIdx.x & 63;
  const int w = width[sl];
  const int64_t b = row < n ? ptr[row] : 0, e = row < n ? ptr[row + 1] : 0;
  const int32_t pad = e > b ? col[b] : 0;
  const int64_t base = off[sl] + lane;
  for (int u = 0; u < w; ++u) {
    const bool real = b + u < e;
    ecol[base + (int64_t)u * 64] = real ? col[b + u] : pad;
    eval[base + (int64_t)u * 64] = real ? val[b + u] : 0.0;
  }
}

}  // namespace

void ell_widths(int64_t n, const int64_t* ptr, int32_t* width, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_ell_widths, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, ptr, width);
}

void ell_fill(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, const int32_t* width,
              const int64_t* off, int32_t* ecol, double* eval, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_ell_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, ptr, col, val, width, off,
                       ecol, eval);
}

void spmv_sell(const DSell& M, const double* x, double* y, const double* rs, const double* cs, hipStream_t s) {
  if (M.nrows > 0)
    hipLaunchKernelGGL(k_spmv_sell<false>, dim3((unsigned)((M.nrows + 255) / 256)), dim3(256), 0, s, M.nrows,
                       M.width, M.off, M.col, M.val, x, y, rs, cs, 1.0, 0.0, nullptr);
}

void spmv_sell_acc(const DSell& M, const double* x, double* y, double sa, double sb, double* part, hipStream_t s) {
  if (M.nrows > 0)
    hipLaunchKernelGGL(k_spmv_sell<true>, dim3((unsigned)((M.nrows + 255) / 256)), dim3(256), 0, s, M.nrows,
                       M.width, M.off, M.col, M.val, x, y, nullptr, nullptr, sa, sb, part);
}

void sum_parts(int64_t np, double* part, double* out, hipStream_t s) {
  constexpr int G = 256;
  if (np > 4 * 1024) {  // one workgroup alone reads a long part array slowly
    hipLaunchKernelGGL(k_sum_parts, dim3(G), dim3(1024), 0, s, np, part, part + np);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(1024), 0, s, (int64_t)G, part + np, out);
  } else {
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(1024), 0, s, np, part, out);
  }
}

void dense_rows(int64_t n, const double* M, const double* x, double* y, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_dense_rows, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, M, x, y);
}

double* hess_out(double* W) { return W + Lay{HESS_MMAX}.out(); }
double* hess_y(double* W) { return W + Lay{HESS_MMAX}.y(); }

void hess_reset(double* W, double beta, hipStream_t s) {
  hipLaunchKernelGGL(k_hess_reset, dim3(1), dim3(64), 0, s, W, beta);
}

void hess_step(double* W, const double* h1, const double* h2, int j, int m, int mode, double thr, hipStream_t s) {
  hipLaunchKernelGGL(k_hess_step, dim3(1), dim3(64), 0, s, W, h1, h2, j, m, mode, thr);
}

void hess_solve(double* W, int jused, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_hess_solve, dim3(1), dim3(64), 0, s, W, jused, m);
}

void hess_reset_batched(double* W, int cap, int ncol, const double* beta, hipStream_t s) {
  if (ncol > 0) hipLaunchKernelGGL(k_hess_reset_batched, dim3(ncol), dim3(64), 0, s, W, cap, beta);
}

void hess_step_batched(double* W, int cap, int m, int ncol, const int32_t* jv, const int32_t* sel, int mode,
                       const double* h1, const double* h2, int ldh, const double* wn2, const double* hn2,
                       const double* thr, double* out, hipStream_t s) {
  if (ncol > 0)
    hipLaunchKernelGGL(k_hess_step_batched, dim3(ncol), dim3(64), 0, s, W, cap, m, jv, sel, mode, h1, h2, ldh, wn2,
                       hn2, thr, out);
}

void hess_solve_batched(double* W, int cap, int m, int ncol, const int32_t* jused, double* y, hipStream_t s) {
  if (ncol > 0) hipLaunchKernelGGL(k_hess_solve_batched, dim3(ncol), dim3(64), 0, s, W, cap, m, jused, y);
}

}  // namespace asss
