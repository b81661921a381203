// gfx950 kernels of the general incomplete LDL^T preconditioner (paper Sec. 3,
// eqs. absfac and preconditioner): every product with J_tilde = Lcal^-1 J_hat
// Lcal^-T, with the outer operator Lcal^-1 A_hat Lcal^-T and the transforms
// of the right-hand side and the solution needs sparse triangular solves.
//
// A triangular solve is a chain of dependent levels (rows whose earlier rows
// are all known); across levels nothing can overlap, within a level every row
// is independent.  The solves here run in one workgroup of 1024 threads: the
// rows of a level are spread over the threads and consecutive levels are one
// __syncthreads() apart, a fraction of a microsecond on one CU, where a
// grid-wide synchronisation between levels would cost microseconds.  The
// factors of the paper's problems (a few thousand rows) stay in the CU's
// caches and the L2 from one step to the next.
//
// The inner mrs solve (App. B) then runs entirely in one launch of that
// workgroup: start, every step (the two triangular solves and J_hat between
// them, the deflation, the norms and projections, the scalar recurrence) and
// the final deferred update, with no host round trip and no grid reduction.
// Its scalar recurrence and its state are those of the sliced kernels
// (mrs_common.hpp), so the iterates are the same function of J_tilde.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ildl_kernels.hpp"
#include "mrs_common.hpp"

namespace asss {

namespace {

// Sum over the lpr lanes of an aligned group (lpr a power of two <= 64).
template <typename T>
__device__ __forceinline__ T group_sum(T v, int lpr) {
  for (int o = lpr >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// What a lane needs of its slot in one level, loaded ahead: the first PF
// entries of the slot, the row, its right-hand side (schedule order) and
// inverse diagonal.  None of it depends on the solution and every address
// comes from per-level scalars, so the loads of a level are issued two levels
// before it is solved, with no branch and no wait between them, and stay in
// flight across the separations of the levels (which wait for LDS only).
template <typename T, int PF>
struct LevelRow {
  int e0, sc, row, lpr, w, base, nslots;
  bool active;  // the thread's wave has a slot in this level (wave-uniform)
  bool valid;   // the thread's slot exists in this level
  int col[PF];
  T val[PF];
  T b, d;
};

template <typename T, int PF, int NT>
__device__ __forceinline__ void load_level(const DTri<T>& F, const T* __restrict__ bs, int l, LevelRow<T, PF>& r) {
  const int slot = threadIdx.x;  // < NT
  r.lpr = F.lev_lpr[l];
  r.e0 = F.lev_ptr[l];
  r.nslots = (F.lev_ptr[l + 1] - r.e0) * r.lpr;
  r.w = F.lev_w[l];
  r.base = F.lev_base[l];
  // a wave with no slot in this level loads nothing (in the workgroup form
  // most waves of a narrow level are idle: their loads would only queue in
  // the CU's memory pipeline ahead of the busy wave's)
  r.active = (int)(threadIdx.x & ~63u) < r.nslots;
  if (!r.active) return;
  r.valid = slot < r.nslots;
  r.sc = min(slot, r.nslots - 1);  // a slot that exists: its loads stay in bounds
  const int e = r.e0 + r.sc / r.lpr;
  r.row = F.row[e];
  r.d = F.dinv[e];
  r.b = bs[e];
  const int wl = max(r.w - 1, 0);
#pragma unroll
  for (int t = 0; t < PF; ++t) {
    const int idx = r.base + min(t, wl) * r.nslots + r.sc;  // within the level's block or the tail
    r.col[t] = F.ecol[idx];
    r.val[t] = F.eval[idx];
  }
}

// Level l from the thread's loaded slot r (every thread calls it; groups of
// lpr lanes share a row): the group's gathered products, summed with
// shuffles, and y[row] = (b - sum) times the inverse diagonal by lane 0; the
// slots of a level wider than NT threads in further passes with plain loads.
template <typename T, int PF, int NT>
__device__ __forceinline__ void solve_level(const DTri<T>& F, const T* __restrict__ bs, T* __restrict__ y,
                                            const LevelRow<T, PF>& r) {
  if (!r.active) return;
  const int lpr = r.lpr;
  const int j = threadIdx.x & (lpr - 1);
  T acc = T(0);
#pragma unroll
  for (int t = 0; t < PF; ++t) {
    // a loaded entry past the slot's count is not used: the product is
    // discarded, never multiplied by 0 (its y may not be solved yet)
    const T p = r.val[t] * y[r.col[t]];
    acc += (t < r.w) ? p : T(0);
  }
  for (int t = PF; t < r.w; ++t) {
    const int idx = r.base + t * r.nslots + r.sc;
    acc += F.eval[idx] * y[F.ecol[idx]];
  }
  acc = group_sum(acc, lpr);
  if (r.valid && j == 0) y[r.row] = (r.b - acc) * r.d;
  for (int s2 = (int)threadIdx.x + NT; s2 < r.nslots; s2 += NT) {
    T a2 = T(0);
    for (int t = 0; t < r.w; ++t) {
      const int idx = r.base + t * r.nslots + s2;
      a2 += F.eval[idx] * y[F.ecol[idx]];
    }
    a2 = group_sum(a2, lpr);
    if (j == 0) {
      const int e = r.e0 + s2 / lpr;
      y[F.row[e]] = (bs[e] - a2) * F.dinv[e];
    }
  }
}

// The levels of a solve taken by NT threads (the whole workgroup, or one
// wave), the row data of level l + 2 loaded while level l is solved, into
// one of three register sets (the loop is unrolled by three, so no copy
// forces a wait); sync() separates the levels.
template <typename T, int NT, class Sync>
__device__ __forceinline__ void trsv_levels(const DTri<T>& F, const T* __restrict__ b, T* __restrict__ y,
                                            const T* __restrict__ bs, Sync sync) {
  constexpr int PF = 4;
  LevelRow<T, PF> ra, rb, rc;
  const int nl = F.nlev;
  if (nl > 0) load_level<T, PF, NT>(F, bs, 0, ra);
  if (nl > 1) load_level<T, PF, NT>(F, bs, 1, rb);
  for (int l = 0; l < nl; l += 3) {
    if (l + 2 < nl) load_level<T, PF, NT>(F, bs, l + 2, rc);
    solve_level<T, PF, NT>(F, bs, y, ra);
    sync();
    if (l + 1 >= nl) break;
    if (l + 3 < nl) load_level<T, PF, NT>(F, bs, l + 3, ra);
    solve_level<T, PF, NT>(F, bs, y, rb);
    sync();
    if (l + 2 >= nl) break;
    if (l + 4 < nl) load_level<T, PF, NT>(F, bs, l + 4, rb);
    solve_level<T, PF, NT>(F, bs, y, rc);
    sync();
  }
}

// y = T^-1 b by levels (every thread of the workgroup calls it).  A group of
// lpr lanes takes one row of the level: its lanes gather entries
// j, j + lpr, ... of the row, the group sums them with shuffles, and lane 0
// scales by the inverse diagonal.  The right-hand side is first copied into
// schedule order (bs, n values of scratch), so that all row data of a level
// is at addresses known without a dependent load, and that data is loaded two
// levels ahead; it stays in flight across the separations of the levels,
// which wait for LDS operations only.
// Narrow factors (F.wave: every level fits one wave in one pass)
// with y in LDS are solved by wave 0 alone: consecutive levels of one wave
// need no workgroup barrier (its LDS operations complete in program order;
// a wavefront-scope fence keeps the compiler from reordering them), and the
// other 15 waves do not spend issue slots on levels they have no rows in.
// Wider factors, or y in global memory, use the whole workgroup with one
// barrier per level.
template <typename T, bool YLDS>
__device__ __forceinline__ void trsv_block(const DTri<T>& F, const T* __restrict__ b, T* __restrict__ y,
                                           T* __restrict__ bs) {
  for (int e = threadIdx.x; e < F.n; e += TRI_WG) bs[e] = b[F.row[e]];
  __syncthreads();
  if (YLDS && F.wave) {
    if (threadIdx.x < 64)
      trsv_levels<T, 64>(F, b, y, bs, [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      });
    __syncthreads();
  } else {
    trsv_levels<T, TRI_WG>(F, b, y, bs, [] { __syncthreads(); });
  }
}

// z = M y with M.lpr lanes per row (entries of a lane summed in stored order).
template <typename T>
__device__ __forceinline__ void spmv_block(const DCsr32<T>& M, const T* __restrict__ y, T* __restrict__ z) {
  const int lpr = M.lpr;
  const int j = threadIdx.x & (lpr - 1);
  for (int i = threadIdx.x / lpr; i < M.n; i += TRI_WG / lpr) {
    T acc = T(0);
    const int q1 = M.ptr[i + 1];
    for (int q = M.ptr[i] + j; q < q1; q += lpr) acc += M.val[q] * y[M.col[q]];
    acc = group_sum(acc, lpr);
    if (j == 0) z[i] = acc;
  }
  __syncthreads();
}

// Sum NV values over the 16 waves of the workgroup in a fixed order.
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], double* lds /* [16 NV] */, double* res) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const double s = wave_sum(v[j]);
    if (lane == 0) lds[wave * NV + j] = s;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < NV; j += TRI_WG) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < TRI_WG / 64; ++w) s += lds[w * NV + j];
    res[j] = s;
  }
  __syncthreads();
}

}  // namespace

// Dynamic LDS of the one-workgroup kernels (the solution vector of the
// triangular solves when it fits).
template <typename T>
__device__ __forceinline__ T* tri_lds() {
  extern __shared__ __align__(16) unsigned char tri_smem[];
  return reinterpret_cast<T*>(tri_smem);
}

template <typename T, bool YLDS>
__global__ __launch_bounds__(TRI_WG) void k_ildl_sandwich(DTri<T> Lb, DCsr32<T> M, DTri<T> Lf,
                                                          const double* __restrict__ in, double* __restrict__ out,
                                                          T* t0, T* t1, T* t2, T* t3) {
  const int n = Lb.n;
  T* y = YLDS ? tri_lds<T>() : t1;
  for (int i = threadIdx.x; i < n; i += TRI_WG) t0[i] = (T)in[i];
  __syncthreads();
  trsv_block<T, YLDS>(Lb, t0, y, t3);
  spmv_block<T>(M, y, t2);
  trsv_block<T, YLDS>(Lf, t2, y, t3);
  for (int i = threadIdx.x; i < n; i += TRI_WG) out[i] = (double)y[i];
}

// Columns j0, j0 + 1, ... of Lcal^-1 M Lcal^-T (M applied to the unit
// vectors), one workgroup per column, each with four n-vectors of scratch of
// its own (t0..t3 at scratch + 4 n b): many columns in flight at once.
template <bool YLDS>
__global__ __launch_bounds__(TRI_WG) void k_ildl_columns(DTri<double> Lb, DCsr32<double> M, DTri<double> Lf,
                                                         int64_t j0, double* __restrict__ out, double* scratch) {
  const int n = Lb.n;
  const int64_t j = j0 + blockIdx.x;
  double* t0 = scratch + (int64_t)blockIdx.x * 4 * n;
  double* t1 = t0 + n;
  double* t2 = t1 + n;
  double* t3 = t2 + n;
  double* y = YLDS ? tri_lds<double>() : t1;
  for (int i = threadIdx.x; i < n; i += TRI_WG) t0[i] = (i == j) ? 1.0 : 0.0;
  __syncthreads();
  trsv_block<double, YLDS>(Lb, t0, y, t3);
  spmv_block<double>(M, y, t2);
  trsv_block<double, YLDS>(Lf, t2, y, t3);
  for (int i = threadIdx.x; i < n; i += TRI_WG) out[j * n + i] = y[i];
}

template <bool YLDS>
__global__ __launch_bounds__(TRI_WG) void k_ildl_trsv(DTri<double> F, const double* __restrict__ in,
                                                      double* __restrict__ out, double* __restrict__ bs) {
  double* y = YLDS ? tri_lds<double>() : out;
  trsv_block<double, YLDS>(F, in, y, bs);
  if (YLDS)
    for (int i = threadIdx.x; i < F.n; i += TRI_WG) out[i] = y[i];
}

template <typename T>
void ildl_sandwich(const DTri<T>& Lb, const DCsr32<T>& M, const DTri<T>& Lf, const double* in, double* out,
                   T* t0, T* t1, T* t2, T* t3, hipStream_t s) {
  if (Lb.n <= tri_lds_rows<T>())
    hipLaunchKernelGGL((k_ildl_sandwich<T, true>), dim3(1), dim3(TRI_WG), (size_t)Lb.n * sizeof(T), s, Lb, M, Lf,
                       in, out, t0, t1, t2, t3);
  else
    hipLaunchKernelGGL((k_ildl_sandwich<T, false>), dim3(1), dim3(TRI_WG), 0, s, Lb, M, Lf, in, out, t0, t1, t2,
                       t3);
}
template void ildl_sandwich<double>(const DTri<double>&, const DCsr32<double>&, const DTri<double>&,
                                    const double*, double*, double*, double*, double*, double*, hipStream_t);
template void ildl_sandwich<float>(const DTri<float>&, const DCsr32<float>&, const DTri<float>&,
                                   const double*, double*, float*, float*, float*, float*, hipStream_t);

void ildl_columns(const DTri<double>& Lb, const DCsr32<double>& M, const DTri<double>& Lf, int64_t j0, int nc,
                  double* out, double* scratch, hipStream_t s) {
  if (nc <= 0) return;
  if (Lb.n <= tri_lds_rows<double>())
    hipLaunchKernelGGL((k_ildl_columns<true>), dim3(nc), dim3(TRI_WG), (size_t)Lb.n * sizeof(double), s, Lb, M, Lf,
                       j0, out, scratch);
  else
    hipLaunchKernelGGL((k_ildl_columns<false>), dim3(nc), dim3(TRI_WG), 0, s, Lb, M, Lf, j0, out, scratch);
}

void ildl_trsv(const DTri<double>& F, const double* in, double* out, double* bs, hipStream_t s) {
  if (F.n <= tri_lds_rows<double>())
    hipLaunchKernelGGL((k_ildl_trsv<true>), dim3(1), dim3(TRI_WG), (size_t)F.n * sizeof(double), s, F, in, out,
                       bs);
  else
    hipLaunchKernelGGL((k_ildl_trsv<false>), dim3(1), dim3(TRI_WG), 0, s, F, in, out, bs);
}

// The inner solve.  Each step is the step of the sliced kernel (k_mrs_iter)
// with u = J_tilde q computed by the two triangular solves around J_hat
// instead of the sliced skew product: the normalisation by 1/nu and the p, x
// update of the previous step are deferred into the pass over the rows in the
// same way, the reduced values (||w_new||^2 and Q_k^T a, or Q_k^T w_new in
// FP32) have the same layout, and mrs_scalar_update advances the same state.
template <typename T, int KF, bool YLDS>
__global__ __launch_bounds__(TRI_WG) void k_ildl_mrs(IldlMrsArgs<T> A) {
  constexpr int NV = KF + 1;
  constexpr int KF1 = KF > 0 ? KF : 1;
  __shared__ double red_lds[(TRI_WG / 64) * NV];
  __shared__ double res[NV];
  __shared__ MrsTail<1, KF> tail;
  __shared__ double sst_raw[sizeof(MrsState) / 8];
  const MrsState& sst = *reinterpret_cast<const MrsState*>(sst_raw);
  const int n = A.n, k = A.k;
  const int tid = threadIdx.x;

  // ---- start: w_1 = rhs, the other vectors 0, r0 = ||rhs||, Q_k^T rhs
  {
    double acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    for (int i = tid; i < n; i += TRI_WG) {
      const double b = A.rhs[i];
      A.buf.w[1][i] = (T)b;
      A.buf.w[0][i] = T(0);
      A.buf.w[2][i] = T(0);
      A.buf.p[0][i] = T(0);
      A.buf.p[1][i] = T(0);
      A.buf.x[i] = T(0);
      acc[0] += b * b;
#pragma unroll
      for (int l = 0; l < KF; ++l)
        if (l < k) acc[1 + l] += (double)A.Q[(int64_t)l * n + i] * (double)(T)b;
    }
    block_reduce<NV>(acc, red_lds, res);
    MrsLaunch L{};
    L.n = n;
    L.nr = 1;
    L.k = k;
    L.alpha_dev = A.alpha;
    L.sign = A.sign;
    mrs_init_finish<1>(L, A.st, res, A.tol, A.maxit, A.fixed);
    __syncthreads();
  }

  const T sgn = (T)A.sign;
  // every step either advances the count (stopping at maxit, or at the fixed
  // count) or finishes: the loop ends within that many passes plus two
  const int passes = (A.fixed > 0 ? A.fixed : A.maxit) + 2;
  for (int guard = 0; guard < passes; ++guard) {
    // the state as the previous step left it (written by this workgroup;
    // atomic loads so that no copy of it is served from the scalar cache)
    for (int e = tid; e < (int)(sizeof(MrsState) / 8); e += TRI_WG)
      sst_raw[e] = __hip_atomic_load(reinterpret_cast<double*>(A.st) + e, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
    const int status = sst.status;
    if (status == MRS_DONE) break;
    const int t = sst.its + 1;
    const T* __restrict__ wcur = A.buf.w[t % 3];
    const T* __restrict__ wold = A.buf.w[(t + 2) % 3];
    T* __restrict__ wnew = A.buf.w[(t + 1) % 3];
    T* __restrict__ pb = A.buf.p[(t + 1) % 2];
    T* __restrict__ x = A.buf.x;
    // the column's coefficients are read from the LDS copy of the state where
    // they are used (after the operator), not held in registers across it
    auto coefs = [&](T& inv_nu, T& inv_nu_old, T& beta_prev, T& pend_delta, T& inv_pend_theta, T& pend_coef,
                     bool& pend) {
      const MrsCol& col = sst.col[0];
      pend = col.has_pending != 0;
      inv_nu = (T)(1.0 / col.nu);
      inv_nu_old = (T)(1.0 / col.nu_old);
      beta_prev = (T)col.beta_prev;
      pend_delta = (T)col.pend_delta;
      inv_pend_theta = (T)(1.0 / col.pend_theta);
      pend_coef = (T)col.pend_coef;
    };
    T inv_nu, inv_nu_old, beta_prev, pend_delta, inv_pend_theta, pend_coef;
    bool pend;

    if (status == MRS_CONVERGED) {  // last deferred update, then done
      coefs(inv_nu, inv_nu_old, beta_prev, pend_delta, inv_pend_theta, pend_coef, pend);
      if (pend)
        for (int i = tid; i < n; i += TRI_WG) {
          const T qold = wold[i] * inv_nu_old;
          const T p = (qold - pend_delta * pb[i]) * inv_pend_theta;
          x[i] += pend_coef * p;
        }
      __syncthreads();
      if (tid == 0) A.st->status = MRS_DONE;
      break;
    }
    // what mrs_scalar_update needs besides the reduced values
    if (tid < (int)(sizeof(MrsCol) / 8))
      reinterpret_cast<double*>(tail.col)[tid] = reinterpret_cast<const double*>(&sst.col[0])[tid];
    if (KF > 0 && tid < k) {
      if (tid < k - 1) tail.alpha[tid] = A.alpha[tid];
      if (!direct_projection<T>()) tail.cvt[0][tid] = (double)(T)sst.cvec[tid];
    }
    if (KF > 0 && !direct_projection<T>())
      for (int e = tid; e < k * k; e += TRI_WG) tail.gram[e] = A.gram[e];

    // u = J_tilde w_t = Lcal^-1 J_hat Lcal^-T w_t (both solves into LDS when
    // the vector fits)
    T* const yv = YLDS ? tri_lds<T>() : A.y;
    T* const uv = YLDS ? tri_lds<T>() : A.u;
    trsv_block<T, YLDS>(A.Lb, wcur, yv, A.bs);
    spmv_block<T>(A.J, yv, A.z);
    trsv_block<T, YLDS>(A.Lf, A.z, uv, A.bs);
    coefs(inv_nu, inv_nu_old, beta_prev, pend_delta, inv_pend_theta, pend_coef, pend);
    T cv[KF1];
#pragma unroll
    for (int l = 0; l < KF1; ++l) cv[l] = (KF > 0 && l < k) ? (T)sst.cvec[l] : T(0);

    double acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    for (int i = tid; i < n; i += TRI_WG) {
      const T u = uv[i] * inv_nu;
      const T qold = wold[i] * inv_nu_old;
      const T a = sgn * u + beta_prev * qold;
      T defl = T(0);
      T qrow[KF1];
#pragma unroll
      for (int l = 0; l < KF; ++l) {
        T q = T(0);
        if (l < k) q = A.Q[(int64_t)l * n + i];
        qrow[l] = q;
        defl += q * cv[l];
        if constexpr (!direct_projection<T>()) acc[1 + l] += (double)q * (double)a;
      }
      const T qn = sgn * (u - defl) + beta_prev * qold;
      wnew[i] = qn;
      acc[0] += (double)qn * (double)qn;
      if constexpr (direct_projection<T>()) {
#pragma unroll
        for (int l = 0; l < KF; ++l) acc[1 + l] += (double)qrow[l] * (double)qn;
      }
      if (pend) {
        const T p = (qold - pend_delta * pb[i]) * inv_pend_theta;
        pb[i] = p;
        x[i] += pend_coef * p;
      }
    }
    block_reduce<NV>(acc, red_lds, res);
    mrs_scalar_update<T, 1, KF>(A.st, res, k, tail, sst.fixed, sst.maxit, sst.tol, t, A.sign);
    __syncthreads();
  }
  __syncthreads();
  for (int i = tid; i < n; i += TRI_WG) A.out[i] = (double)A.buf.x[i];
}

template <typename T, bool YLDS>
void launch_ildl_mrs(const IldlMrsArgs<T>& a, hipStream_t s) {
  const size_t lds = YLDS ? (size_t)a.n * sizeof(T) : 0;
  const int k = a.k;
  if (k <= 0)
    hipLaunchKernelGGL((k_ildl_mrs<T, 0, YLDS>), dim3(1), dim3(TRI_WG), lds, s, a);
  else if (k <= 8)
    hipLaunchKernelGGL((k_ildl_mrs<T, 8, YLDS>), dim3(1), dim3(TRI_WG), lds, s, a);
  else if (k <= 16)
    hipLaunchKernelGGL((k_ildl_mrs<T, 16, YLDS>), dim3(1), dim3(TRI_WG), lds, s, a);
  else
    hipLaunchKernelGGL((k_ildl_mrs<T, 32, YLDS>), dim3(1), dim3(TRI_WG), lds, s, a);
}

template <typename T>
void ildl_mrs(const IldlMrsArgs<T>& a, hipStream_t s) {
  if (a.n <= tri_lds_rows<T>()) launch_ildl_mrs<T, true>(a, s);
  else launch_ildl_mrs<T, false>(a, s);
}
template void ildl_mrs<double>(const IldlMrsArgs<double>&, hipStream_t);
template void ildl_mrs<float>(const IldlMrsArgs<float>&, hipStream_t);

}  // namespace asss
