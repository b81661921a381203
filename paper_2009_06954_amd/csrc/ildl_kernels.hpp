// Device side of the general incomplete LDL^T preconditioner (paper Sec. 3):
// level-scheduled triangular solves with the scaled factor Lcal, the
// "sandwich" products Lcal^-1 M Lcal^-T, and the whole inner mrs solve on
// I + J_bar with J_tilde = Lcal^-1 J_hat Lcal^-T in one persistent workgroup.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace asss {

// Threads of the one workgroup that runs a triangular solve: the solve is a
// chain of levels, each level a __syncthreads() apart, so it runs on one CU
// where a barrier costs a fraction of a microsecond instead of a grid-wide
// synchronisation.
constexpr int TRI_WG = 1024;

// A triangular factor for a level-scheduled solve T y = b, stored level by
// level.  The e-th row of the schedule is row[e], with inverse diagonal
// dinv[e]; level l holds schedule rows lev_ptr[l] .. lev_ptr[l+1] - 1 and is
// solved with lev_lpr[l] lanes per row (a power of two up to 64: long rows
// spread their entries over a group of lanes that sums with shuffles).  The
// off-diagonal entries of a level form one padded block (ELL) at
// lev_base[l]: with N = rows * lpr slots (slot = local row * lpr + lane in
// the group), the t-th entry of a slot (the row's entry lane + t * lpr) is at
// lev_base[l] + t * N + slot, t < lev_w[l]; padding holds value 0 and the
// column of a row of level 0 (solved before any level that reads it).  Every
// address of a level's block is so known from per-level scalars: its loads
// are issued ahead without waiting for anything.  The entry arrays carry a
// tail of TRI_WG padding entries.
template <typename T>
struct DTri {
  int32_t n = 0, nlev = 0;
  int32_t wave = 0;                  // 1: every level fits one wave in one pass, <= 4 entries per lane
  const int32_t* lev_ptr = nullptr;  // nlev + 1
  const int32_t* lev_lpr = nullptr;  // nlev
  const int32_t* lev_w = nullptr;    // nlev: entries per slot
  const int32_t* lev_base = nullptr; // nlev: offset of the level's block
  const int32_t* row = nullptr;      // n
  const int32_t* ecol = nullptr;
  const T* eval = nullptr;
  const T* dinv = nullptr;           // n: 1 / diagonal, in schedule order
};

// Square CSR with 32-bit offsets (the operators between the two solves),
// read with lpr lanes per row.
template <typename T>
struct DCsr32 {
  int32_t n = 0, lpr = 1;
  const int32_t* ptr = nullptr;
  const int32_t* col = nullptr;
  const T* val = nullptr;
};

// Largest n whose solution vector the triangular solves keep in LDS (40 KiB,
// so that a workgroup with the kernels' other shared arrays stays within
// 64 KiB); beyond it the vector stays in global memory.
template <typename T>
constexpr int tri_lds_rows() { return (40 * 1024) / (int)sizeof(T); }

// out = Lf^-1 (M (Lb^-1 in)): Lb the upper factor Lcal^T, Lf the lower Lcal.
// Arithmetic in T; in and out FP64.  t0 .. t3: n values of scratch each.
template <typename T>
void ildl_sandwich(const DTri<T>& Lb, const DCsr32<T>& M, const DTri<T>& Lf, const double* in, double* out,
                   T* t0, T* t1, T* t2, T* t3, hipStream_t s);

// Columns j0 .. j0 + nc - 1 of Lcal^-1 M Lcal^-T in FP64, column j at
// out + j n, nc workgroups at once; scratch: 4 n nc values.
void ildl_columns(const DTri<double>& Lb, const DCsr32<double>& M, const DTri<double>& Lf, int64_t j0, int nc,
                  double* out, double* scratch, hipStream_t s);

// out = F^-1 in (FP64); in and out may not alias; bs: n values of scratch.
void ildl_trsv(const DTri<double>& F, const double* in, double* out, double* bs, hipStream_t s);

// The arguments of one inner solve on I + J_bar (sign = -1: its transpose).
template <typename T>
struct IldlMrsArgs {
  int32_t n = 0, k = 0, sign = 1;
  const double* alpha = nullptr;  // k - 1 skew-Lanczos coefficients
  const T* Q = nullptr;           // n x k column-major, in positions
  const double* gram = nullptr;   // Q^T Q of the stored basis (k x k)
  DTri<T> Lb, Lf;
  DCsr32<T> J;                    // J_hat in positions, both triangles
  const double* rhs = nullptr;    // n (FP64)
  double* out = nullptr;          // n (FP64)
  MrsBufs<T> buf;                 // three w, two p, x: n each
  T* y = nullptr;                 // n: Lcal^-T q
  T* z = nullptr;                 // n: J_hat Lcal^-T q
  T* u = nullptr;                 // n: J_tilde q
  T* bs = nullptr;                // n: a triangular solve's right-hand side in schedule order
  MrsState* st = nullptr;
  double tol = 0.0;
  int32_t maxit = 0, fixed = 0;
};

// The whole inner solve (start, steps, final deferred update, output) in one
// launch of one workgroup; st holds the iteration count and residual after.
template <typename T>
void ildl_mrs(const IldlMrsArgs<T>& a, hipStream_t s);

}  // namespace asss
