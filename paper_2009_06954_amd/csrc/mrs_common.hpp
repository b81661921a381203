// Device code shared by the inner mrs kernels (kernels.hip, ildl.hip): wave
// sums, the scalar part of one App. B step and of its start.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace asss {

// v moved across lanes by one DPP pattern (the two 32-bit halves separately);
// lanes outside ROW_MASK get 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave in a fixed order, with DPP lane moves (VALU)
// instead of LDS permutes: pairs and quads (quad_perm), rows of 16 (row_ror 4
// and 8: every lane then holds its row's sum), then row 1 += row 0 and row 3
// += row 2 (row_bcast:15), rows 2-3 += rows 0-1 (row_bcast:31); lane 63 holds
// the total, which is returned to every lane.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x124, 0xf>(v);  // row_ror:4
  v += dpp_move<0x128, 0xf>(v);  // row_ror:8
  v += dpp_move<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}


// S_k d for the skew tridiagonal S_k (superdiagonal +alpha, subdiagonal -alpha).
__device__ __forceinline__ double sk_times(const double* alpha, const double* d, int k, int l) {
  double r = 0.0;
  if (l + 1 < k) r += alpha[l] * d[l + 1];
  if (l >= 1) r -= alpha[l - 1] * d[l - 1];
  return r;
}

// How the iteration kernel forms Q_k^T q_new for the next deflation
// coefficients.  FP64 kernels stream each Q_k row once and take
// Q_k^T q_new = Q_k^T a - sign G c (G = Q_k^T Q_k), which needs no register
// copy of the row.  FP32 kernels project the stored (rounded) q_new itself:
// the rounding of the deflation term Q_k c, about 2^-24 |Q_k| |c| per entry, is
// then part of q_new and never drifts; with coefficients |c| ~ alpha ~ 1e4
// (Peclet 1000) the G form let the deflation lose ~1e-3 per step in FP32
// (30 steps at 24^3: true residual 0.67 against 0.07 with the direct form).
template <typename T>
__device__ constexpr bool direct_projection() { return sizeof(T) == 4; }

// What the last workgroup of an iteration needs besides the reduced values,
// copied to LDS by every workgroup at the start of the launch (the copies'
// latency hides behind the launch's main work instead of adding to the serial
// tail of the last workgroup).
template <int NR, int KF>
struct MrsTail {
  static constexpr int KF1 = KF > 0 ? KF : 1;
  MrsCol col[NR];
  double cvt[NR][KF1];   // deflation coefficients c as applied (rounded to T)
  double alpha[KF1];     // skew-Lanczos coefficients
  double gram[KF1 * KF1];
};

// The tail's values in registers: every thread of the NT-thread workgroup
// loads at most one column-state word, one c, one alpha and NG Gram entries.
// Loaded at the start of a launch and written to LDS after the block's w is
// staged, so that these loads overlap the staging loads instead of adding
// round trips of their own.
template <int NR, int KF, int NT = WG>
struct MrsTailRegs {
  static constexpr int NC = NR * (int)sizeof(MrsCol) / 8;
  static constexpr int KF1 = KF > 0 ? KF : 1;
  static constexpr int NG = (KF1 * KF1 + NT - 1) / NT;
  static_assert(NC <= NT && NR * KF1 <= NT && KF1 <= NT, "one tail word per thread");
  double col, cvt, alpha, gram[NG];
};

template <typename T, int NR, int KF, int NT = WG>
__device__ __forceinline__ void mrs_tail_load(MrsTailRegs<NR, KF, NT>& r, const MrsState* st, const MrsLaunch& L) {
  using R = MrsTailRegs<NR, KF, NT>;
  const int e = threadIdx.x, k = L.k;
  r.col = e < R::NC ? reinterpret_cast<const double*>(st->col)[e] : 0.0;
  r.cvt = r.alpha = 0.0;
#pragma unroll
  for (int u = 0; u < R::NG; ++u) r.gram[u] = 0.0;
  if (KF > 0 && k > 0) {
    if (e < k - 1) r.alpha = L.alpha_dev[e];
    if (!direct_projection<T>()) {
      if (e < NR * k) r.cvt = st->cvec[(e / k) * KMAX + e % k];  // rounded to T at the store
#pragma unroll
      for (int u = 0; u < R::NG; ++u)
        if (e + u * NT < k * k) r.gram[u] = L.gram[e + u * NT];
    }
  }
}

template <typename T, int NR, int KF, int NT = WG>
__device__ __forceinline__ void mrs_tail_store(MrsTail<NR, KF>& tl, const MrsTailRegs<NR, KF, NT>& r, int k) {
  using R = MrsTailRegs<NR, KF, NT>;
  const int e = threadIdx.x;
  if (e < R::NC) reinterpret_cast<double*>(tl.col)[e] = r.col;
  if (KF > 0 && k > 0) {
    if (e < k - 1) tl.alpha[e] = r.alpha;
    if (!direct_projection<T>()) {
      if (e < NR * k) tl.cvt[e / k][e % k] = (double)(T)r.cvt;
#pragma unroll
      for (int u = 0; u < R::NG; ++u)
        if (e + u * NT < k * k) tl.gram[e + u * NT] = r.gram[u];
    }
  }
}

template <typename T, int NR, int KF>
__device__ void mrs_scalar_update(MrsState* st, const double* res, int k, const MrsTail<NR, KF>& tl,
                                  int fixed, int maxit, double tol, int t, int sign) {
  // res: [KF+1][NR] with row 0 = ||w_new||^2 and rows 1..k either Q^T w_new
  // itself (direct projection, FP32 kernels) or Q^T a, where a = sign u +
  // beta q_old is w_new before the deflation term: w_new = a - sign Q c with c
  // the deflation coefficients as applied (rounded to T), so
  // Q^T w_new = Q^T a - sign G c, G = Q^T Q (FP64 kernels).
  __shared__ double dsh[NRMAX][KMAX];
  __shared__ double s_relmax[NRMAX], s_nu[NRMAX];
  __shared__ int s_live[NRMAX];
  const int c = threadIdx.x;
  if (c < NR) {
    MrsCol col = tl.col[c];
    double rel = 0.0;
    if (col.live) {
      const double beta = sqrt(res[c]);
      const double theta = sqrt(col.theta1 * col.theta1 + beta * beta);
      const double ck = col.theta1 / theta;
      const double sk = beta / theta;
      const double delta_new = -col.s_old * beta;
      const double theta1_new = col.c_old * theta;
      col.pend_theta = theta;
      col.pend_delta = col.delta_old;
      col.pend_coef = col.g * ck;
      col.has_pending = 1;
      col.g = -col.g * sk;
      col.delta_old = delta_new;
      col.s_old = sk;
      col.c_old = ck;
      col.theta1 = theta1_new;
      col.nu_old = col.nu;
      col.nu = (beta != 0.0) ? beta : 1.0;
      col.beta_prev = beta;
      rel = fabs(col.g) / col.r0;
    } else {
      col.pend_theta = 1.0;
      col.pend_delta = 0.0;
      col.pend_coef = 0.0;
      col.has_pending = 1;
    }
    s_relmax[c] = rel;
    s_nu[c] = col.nu;
    s_live[c] = col.live;
    st->col[c] = col;
  }
  __syncthreads();
  // d = Q^T q_new = Q^T w_new / nu_new
  for (int e = threadIdx.x; e < NR * k; e += WG) {
    const int cc = e / k, l = e % k;
    double gc = 0.0;
    if (!direct_projection<T>())
      for (int m = 0; m < k; ++m) gc += tl.gram[l * k + m] * tl.cvt[cc][m];
    dsh[cc][l] = s_live[cc] ? (res[(1 + l) * NR + cc] - (double)sign * gc) / s_nu[cc] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NR * k; e += WG) {
    int cc = e / k, l = e % k;
    st->cvec[cc * KMAX + l] = sk_times(tl.alpha, dsh[cc], k, l);
  }
  if (threadIdx.x == 0) {
    double rmax = 0.0;
    for (int cc = 0; cc < NR; ++cc) rmax = fmax(rmax, s_relmax[cc]);
    st->relres_max = rmax;
    st->its = t;
    int status = MRS_RUNNING;
    if (fixed > 0) {
      if (t >= fixed) status = MRS_CONVERGED;
    } else if (rmax < tol || t >= maxit) {
      status = MRS_CONVERGED;
    }
    st->status = status;
  }
}

// The last block of a start: the column states (r0 = ||b||, App. B's
// initial Givens values), d = Q_k^T q_1 and c = S_k d, and the solve state.
template <int NR>
__device__ void mrs_init_finish(const MrsLaunch& L, MrsState* st, const double* res, double tol, int maxit,
                                int fixed) {
  const int k = L.k;
  __shared__ double dsh[NRMAX][KMAX];
  __shared__ int s_any;
  if (threadIdx.x == 0) s_any = 0;
  __syncthreads();
  const int c = threadIdx.x;
  if (c < NR) {
    MrsCol col;
    const double r0 = sqrt(res[c]);
    col.live = (c < L.nr && r0 > 0.0) ? 1 : 0;
    col.r0 = col.live ? r0 : 1.0;
    col.nu = col.r0;
    col.nu_old = 1.0;
    col.beta_prev = 0.0;
    col.theta1 = 1.0;  // alpha = 1 (S_bar = I + J_bar)
    col.c_old = 1.0;
    col.s_old = 0.0;
    col.delta_old = 0.0;
    col.g = col.live ? r0 : 0.0;
    col.pend_theta = 1.0;
    col.pend_delta = 0.0;
    col.pend_coef = 0.0;
    col.has_pending = 0;
    for (int l = 0; l < k; ++l) dsh[c][l] = col.live ? res[(1 + l) * NR + c] / col.nu : 0.0;
    st->col[c] = col;
    if (col.live) atomicOr(&s_any, 1);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NR * k; e += WG) {
    int cc = e / k, l = e % k;
    st->cvec[cc * KMAX + l] = sk_times(L.alpha_dev, dsh[cc], k, l);
  }
  if (threadIdx.x == 0) {
    st->its = 0;
    st->status = s_any ? MRS_RUNNING : MRS_DONE;
    st->nr = L.nr;
    st->k = k;
    st->maxit = maxit;
    st->fixed = fixed;
    st->sign = L.sign;
    st->tol = tol;
    st->alpha = 1.0;
    st->relres_max = s_any ? 1.0 : 0.0;
  }
}

}  // namespace asss
