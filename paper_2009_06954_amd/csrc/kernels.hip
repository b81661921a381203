// gfx950 kernels of libasss: CSR SpMV, the sliced skew-symmetric SpMV with an
// LDS scatter, the fused inner mrs iteration (paper App. B) with the deflation
// projector (Sec. 3.2) and one deterministic grid reduction per iteration,
// tall-skinny products for the outer orthogonalisation and the SMW term, and
// small vector kernels.  All of it is bandwidth bound: no matrix cores.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "mrs_common.hpp"

namespace asss {

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------

// Reduce NV per-thread values over the workgroup of NT threads; results in
// res[0..NV).  Fixed order (wave butterflies, then waves in order), so the
// result does not depend on timing.
template <int NV, int NT = WG>
__device__ __forceinline__ void wg_reduce(double (&v)[NV], double* lds /* [NT/64 * NV] */,
                                          double* res /* [NV] */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    double s = wave_sum(v[j]);
    if (lane == 0) lds[wave * NV + j] = s;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < NV; j += NT) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += lds[w * NV + j];
    res[j] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ void store_partial(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_partial(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last-arriving workgroup detection.  Every workgroup publishes its partials
// with agent-scope atomic stores (write-through to the device coherence point)
// and waits for them to complete before taking a ticket; exactly one workgroup
// (the last) gets true and then reads all partials with agent-scope atomic
// loads.  Only the partials cross workgroups inside a kernel, so no
// release/acquire fence (which would write back or invalidate the whole L2 of
// the XCD) is needed; everything else reaches the next kernel at the launch
// boundary.
__device__ __forceinline__ bool arrive_last(unsigned* ticket, unsigned total) {
  __shared__ unsigned s_last;
  __builtin_amdgcn_s_waitcnt(0);  // this thread's partial stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (t == total - 1) ? 1u : 0u;
  }
  __syncthreads();
  return s_last != 0;
}

__device__ __forceinline__ void reset_ticket(unsigned* ticket) {
  if (threadIdx.x == 0) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Partials in column layout: value j of workgroup g at partials[j * ngroups + g],
// so that the last workgroup reads each value's partials with coalesced loads.
template <int NV>
__device__ __forceinline__ void publish_partials(double* partials, const double* res) {
  for (int j = threadIdx.x; j < NV; j += WG)
    store_partial(partials + (int64_t)j * gridDim.x + blockIdx.x, res[j]);
}

// The same for block g of ng blocks (a system's blocks in a batched launch).
template <int NV, int NT = WG>
__device__ __forceinline__ void publish_partials_at(double* partials, const double* res, int g, int ng) {
  for (int j = threadIdx.x; j < NV; j += NT) store_partial(partials + (int64_t)j * ng + g, res[j]);
}

// In the last workgroup: res[j] = sum over groups g of partials[j * ngroups + g].
// Thread t adds groups t, t + WG, t + 2 WG, ... in that order, then the
// workgroup reduction runs in its fixed order, so the result does not depend
// on timing.  The atomic loads stay in program order, so all loads of a batch
// of B groups are written before any of their sums: one memory round trip per
// batch instead of one per value.
template <int NV, int NT = WG>
__device__ __forceinline__ void final_reduce(const double* partials, int ngroups, double* lds,
                                             double* res) {
  constexpr int B = NV <= 20 ? 2 : 1;
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  int g = threadIdx.x;
  for (; g + (B - 1) * NT < ngroups; g += B * NT) {
    double v[B][NV];
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int j = 0; j < NV; ++j) v[b][j] = load_partial(partials + (int64_t)j * ngroups + g + b * NT);
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int j = 0; j < NV; ++j) acc[j] += v[b][j];
  }
  for (; g < ngroups; g += NT) {
    double v[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = load_partial(partials + (int64_t)j * ngroups + g);
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] += v[j];
  }
  wg_reduce<NV, NT>(acc, lds, res);
}

// sum over g = g0, g0 + step, ... < ng of P[g * stride + o], eight independent
// chains (fixed order for given arguments).
__device__ __forceinline__ double strided_sum(const double* P, int g0, int ng, int step,
                                              int64_t stride, int o) {
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int g = g0;
  for (; g + 7 * step < ng; g += 8 * step) {
    double v[8];  // all eight loads in flight before the sums (see final_reduce)
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = load_partial(P + (int64_t)(g + u * step) * stride + o);
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += v[u];
  }
  for (; g < ng; g += step) a[0] += load_partial(P + (int64_t)g * stride + o);
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// ---------------------------------------------------------------------------
// CSR SpMV (outer operator, true residual, least-squares matrices)
// ---------------------------------------------------------------------------

template <int LANES>
__global__ __launch_bounds__(WG) void k_spmv(int64_t nrows, const int64_t* __restrict__ ptr,
                                             const int32_t* __restrict__ col,
                                             const double* __restrict__ val,
                                             const double* __restrict__ x, double* __restrict__ y,
                                             const double* __restrict__ rs,
                                             const double* __restrict__ cs, int mode,
                                             const double* __restrict__ b) {
  const int64_t gid = (int64_t)blockIdx.x * WG + threadIdx.x;
  const int64_t row = gid / LANES;
  const int sub = (int)(gid % LANES);
  double sum = 0.0;
  if (row < nrows) {
    const int64_t e = ptr[row + 1];
    // the matrix is streamed once: non-temporal loads keep it from pushing
    // the gathered vector out of L2
    if (cs) {
      for (int64_t p = ptr[row] + sub; p < e; p += LANES) {
        const int32_t c = __builtin_nontemporal_load(&col[p]);
        sum += __builtin_nontemporal_load(&val[p]) * (cs[c] * x[c]);
      }
    } else {
      for (int64_t p = ptr[row] + sub; p < e; p += LANES)
        sum += __builtin_nontemporal_load(&val[p]) * x[__builtin_nontemporal_load(&col[p])];
    }
  }
#pragma unroll
  for (int off = LANES / 2; off >= 1; off >>= 1) sum += __shfl_xor(sum, off, LANES);
  if (row < nrows && sub == 0) {
    double r = rs ? rs[row] * sum : sum;
    y[row] = (mode == 1) ? b[row] - r : r;
  }
}

// One row per thread, for matrices whose rows are all short (lanes == 0): the
// column indices and values of up to 8 entries are loaded before any of their
// gathers, so a thread has a whole grid-stencil row in flight at once instead
// of one entry per lane and a cross-lane sum (7-point rows at 128^3: 75 -> 40 us).
// Entries are summed in row order.
__global__ __launch_bounds__(WG) void k_spmv_rows(int64_t nrows, const int64_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ col,
                                                  const double* __restrict__ val,
                                                  const double* __restrict__ x, double* __restrict__ y,
                                                  const double* __restrict__ rs,
                                                  const double* __restrict__ cs, int mode,
                                                  const double* __restrict__ b) {
  const int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (row >= nrows) return;
  const int64_t e = ptr[row + 1];
  double sum = 0.0;
  for (int64_t p0 = ptr[row]; p0 < e; p0 += 8) {
    int32_t c[8];
    double v[8];
    // plain loads: the lanes of a wave read interleaved parts of the same cache
    // lines in successive u, which non-temporal loads would fetch again (100 us)
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (p0 + u < e) {
        c[u] = col[p0 + u];
        v[u] = val[p0 + u];
      }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (p0 + u < e) sum += v[u] * (cs ? cs[c[u]] * x[c[u]] : x[c[u]]);
  }
  const double r = rs ? rs[row] * sum : sum;
  y[row] = (mode == 1) ? b[row] - r : r;
}

void spmv(const DCsr& M, const double* x, double* y, const double* rs, const double* cs, int mode,
          const double* b, hipStream_t s) {
  if (M.nrows == 0) return;
  if (M.lanes == 0) {
    hipLaunchKernelGGL(k_spmv_rows, dim3((unsigned)((M.nrows + WG - 1) / WG)), dim3(WG), 0, s, M.nrows, M.ptr,
                       M.col, M.val, x, y, rs, cs, mode, b);
    return;
  }
  int64_t threads = M.nrows * M.lanes;
  dim3 grid((unsigned)((threads + WG - 1) / WG));
#define ASSS_SPMV(L)                                                                              \
  case L:                                                                                         \
    hipLaunchKernelGGL(k_spmv<L>, grid, dim3(WG), 0, s, M.nrows, M.ptr, M.col, M.val, x, y, rs, \
                       cs, mode, b);                                                              \
    break;
  switch (M.lanes) {
    ASSS_SPMV(1)
    ASSS_SPMV(2)
    ASSS_SPMV(4)
    ASSS_SPMV(8)
    ASSS_SPMV(16)
    ASSS_SPMV(32)
    default:
      ASSS_SPMV(64)
  }
#undef ASSS_SPMV
}

// Row block of this workgroup.  Workgroups are dispatched to the 8 XCDs round
// robin (workgroup b on XCD b mod 8), and each XCD has its own L2.  In FP32 XCD
// x gets one contiguous eighth of the row blocks, so blocks that are
// neighbours in index space -- whose w entries the part-b gathers read --
// share an L2 at any grid size (in natural order a block's z neighbours are a
// plane of rows away: 8 blocks at 128^3, 18 at 192^3).  The FP32 step is
// latency bound and gains (128^3: 87.6 -> 83.7 us, 192^3: 358.7 -> 350.7 us);
// the bandwidth-bound FP64 step loses (142.9 -> 149.7 us, 523.5 -> 533.9 us)
// and keeps the natural order, where all XCDs stream neighbouring blocks.
template <typename T>
__device__ __forceinline__ int xcd_block() {
  constexpr int NXCD = 8;
  const int nb = gridDim.x, b = blockIdx.x;
  if (sizeof(T) != 4) return b;
  const int q = nb / NXCD, r = nb % NXCD;
  const int x = b % NXCD, k = b / NXCD;
  return x * q + min(x, r) + k;
}

// ---------------------------------------------------------------------------
// Sliced skew SpMV: the part shared by the standalone operator and the mrs step.
// One workgroup per block of R rows; wave w handles slices w, w + 4, ... of it,
// P slices at a time (P = 2 for one column: twice the loads in flight per wave).
// w_src(jl) reads the gathered vector at local row jl (LDS or global).
// Accumulates the block's results into acc_lds[il * NR + c], which is FP64 in
// both precisions: LDS float atomics (ds_add_f32) are slow on this chip (the
// FP32 step spent about 24 of its 120 us in them), ds_add_f64 is not, and the
// FP64 sums round to T once when read.
// ---------------------------------------------------------------------------

// FORM: 1 = 32-bit part-b columns, 2 = 16-bit part-b deltas from a per-slot
// base, 3 = offset slots (no per-entry columns: every lane of a slot reads
// column row + d; padding lanes, whose value is 0, are clamped into the block
// for part a and into [0, n) for part b).
template <typename T, int NR, bool STAGE, int FORM, int NT = WG>
__device__ __forceinline__ void skew_block_pass_form(const DSkew<T>& J, int64_t row0, int nrow,
                                                     const T* __restrict__ wg, const T* w_lds,
                                                     double* acc_lds) {
  // Each round handles up to U in-block entries and U off-block entries of
  // every row of the P slices; all of a round's loads are issued before any of
  // its arithmetic (the widths are wave-uniform, so the guards do not diverge).
  // The entries are streamed once per launch: non-temporal loads keep them
  // from evicting the w vector from L2, which the part-b gathers of the
  // neighbouring blocks re-read (measured: FP64 step 185 -> 150 us, FP32
  // 138 -> 124 us on the 128^3 workload).
  constexpr int P = (NR == 1) ? 2 : 1;
  constexpr int U = (NR == 1) ? 4 : 8;
  constexpr int NW = NT / 64;
  constexpr bool NARROW = FORM == 2, SLOTS = FORM == 3;
  // the wave index is uniform: said so, the slice metadata below comes in
  // through scalar loads instead of a vector round trip per slice
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nsl = (nrow + 63) >> 6;
  const int64_t s0 = row0 >> 6;
  for (int sl0 = wave; sl0 < nsl; sl0 += P * NW) {
    int wa[P], wb[P], il[P];
    bool valid[P];
    const uint16_t* __restrict__ acol[P];
    const T* __restrict__ aval[P];
    const int32_t* __restrict__ bcol[P];
    const uint16_t* __restrict__ bcd[P];
    const int32_t* __restrict__ bbase[P];
    const int32_t* __restrict__ adoff[P];
    const T* __restrict__ bval[P];
    T acc[P][NR], wi[P][NR];
    int wmax = 0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int sl = sl0 + p * NW;
      const bool has = sl < nsl;  // wave-uniform
      const int64_t s = s0 + (has ? sl : 0);
      wa[p] = has ? __builtin_amdgcn_readfirstlane(J.a_width[s]) : 0;
      wb[p] = has ? __builtin_amdgcn_readfirstlane(J.b_width[s]) : 0;
      wmax = max(wmax, max(wa[p], wb[p]));
      il[p] = sl * 64 + lane;
      valid[p] = has && il[p] < nrow;
      acol[p] = J.a_col + J.a_off[s] + lane;
      aval[p] = J.a_val + J.a_off[s] + lane;
      bcol[p] = J.b_col + J.b_off[s] + lane;
      bcd[p] = J.b_cd + J.b_off[s] + lane;
      bbase[p] = J.b_base + (J.b_off[s] >> 6);
      adoff[p] = J.a_doff + (J.a_off[s] >> 6);
      bval[p] = J.b_val + J.b_off[s] + lane;
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        acc[p][c] = T(0);
        wi[p][c] = valid[p] ? (STAGE ? w_lds[il[p] * NR + c] : wg[(row0 + il[p]) * NR + c]) : T(0);
      }
    }
    const int rounds = (wmax + U - 1) / U;
    for (int r = 0; r < rounds; ++r) {
      const int l0 = r * U;
      int jl[P][U];
      T va[P][U];
      int32_t jb[P][U];
      T vb[P][U];
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (l0 + u < wa[p]) {
            if (SLOTS)  // d > 0 (uniform); padding lanes past the block end clamp to its last row
              jl[p][u] = min(il[p] + adoff[p][l0 + u], nrow - 1);
            else
              jl[p][u] = __builtin_nontemporal_load(&acol[p][(l0 + u) * 64]);
            va[p][u] = __builtin_nontemporal_load(&aval[p][(l0 + u) * 64]);
          }
          if (l0 + u < wb[p]) {
            // narrow: the 16-bit delta now, its slot base (uniform) at the gather;
            // slots: no column load at all
            if (NARROW)
              jb[p][u] = (int32_t)__builtin_nontemporal_load(&bcd[p][(l0 + u) * 64]);
            else if (!SLOTS)
              jb[p][u] = __builtin_nontemporal_load(&bcol[p][(l0 + u) * 64]);
            vb[p][u] = __builtin_nontemporal_load(&bval[p][(l0 + u) * 64]);
          }
        }
      T wj[P][U][NR];
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (l0 + u < wb[p]) {
            const int32_t col = SLOTS    ? min(max(bbase[p][l0 + u] + lane, 0), J.n - 1)
                                : NARROW ? bbase[p][l0 + u] + jb[p][u]
                                         : jb[p][u];
#pragma unroll
            for (int c = 0; c < NR; ++c) wj[p][u][c] = wg[(int64_t)col * NR + c];
          }
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (l0 + u < wa[p]) {
#pragma unroll
            for (int c = 0; c < NR; ++c) {
              const T w = STAGE ? w_lds[jl[p][u] * NR + c] : wg[(row0 + jl[p][u]) * NR + c];
              acc[p][c] += va[p][u] * w;
              if (valid[p]) atomicAdd(&acc_lds[jl[p][u] * NR + c], (double)(-va[p][u] * wi[p][c]));
            }
          }
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (l0 + u < wb[p]) {
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[p][c] += vb[p][u] * wj[p][u][c];
          }
    }
#pragma unroll
    for (int p = 0; p < P; ++p)
      if (valid[p]) {
#pragma unroll
        for (int c = 0; c < NR; ++c) atomicAdd(&acc_lds[il[p] * NR + c], (double)acc[p][c]);
      }
  }
}

// The explicit (dense) operator: acc_lds[il] = sum_j J[row0 + il][j] w_j for
// the block's rows, one wave per row (rows round-robin over the waves), the
// lanes over the columns with coalesced loads of the row, eight loads in
// flight per lane, a wave sum in a fixed order.
template <typename T, int NR, int NT>
__device__ __forceinline__ void dense_block_pass(const DSkew<T>& J, int64_t row0, int nrow,
                                                 const T* __restrict__ wg, double* acc_lds) {
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t n = J.n;
  for (int r = wave; r < nrow; r += NT / 64) {
    const T* __restrict__ row = J.dense + (row0 + r) * J.dense_ld;
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0.0;
    int64_t j = lane;
    for (; j + 7 * 64 < n; j += 8 * 64) {
      T a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = __builtin_nontemporal_load(&row[j + u * 64]);
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] += (double)a[u] * (double)wg[(j + u * 64) * NR + c];
    }
    for (; j < n; j += 64)
#pragma unroll
      for (int c = 0; c < NR; ++c) acc[c] += (double)row[j] * (double)wg[j * NR + c];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      const double sum = wave_sum(acc[c]);
      if (lane == 0) acc_lds[r * NR + c] = sum;
    }
  }
}

// The column form is fixed per matrix: one uniform branch per launch.
template <typename T, int NR, bool STAGE, int NT = WG>
__device__ __forceinline__ void skew_block_pass(const DSkew<T>& J, int64_t row0, int nrow,
                                                const T* __restrict__ wg, const T* w_lds,
                                                double* acc_lds) {
  if (J.form == 3)
    skew_block_pass_form<T, NR, STAGE, 3, NT>(J, row0, nrow, wg, w_lds, acc_lds);
  else if (J.form == 2)
    skew_block_pass_form<T, NR, STAGE, 2, NT>(J, row0, nrow, wg, w_lds, acc_lds);
  else
    skew_block_pass_form<T, NR, STAGE, 1, NT>(J, row0, nrow, wg, w_lds, acc_lds);
}

template <typename T>
__global__ __launch_bounds__(WG) void k_skew_spmv(DSkew<T> J, const T* __restrict__ x,
                                                  T* __restrict__ y) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* acc_lds = reinterpret_cast<double*>(smem_raw);
  T* w_lds = reinterpret_cast<T*>(acc_lds + J.R);
  const int64_t row0 = (int64_t)xcd_block<T>() * J.R;
  const int nrow = (int)min((int64_t)J.R, (int64_t)J.n - row0);
  for (int r = threadIdx.x; r < nrow; r += WG) {
    w_lds[r] = x[row0 + r];
    acc_lds[r] = 0.0;
  }
  __syncthreads();
  skew_block_pass<T, 1, true>(J, row0, nrow, x, w_lds, acc_lds);
  __syncthreads();
  for (int r = threadIdx.x; r < nrow; r += WG) y[row0 + r] = (T)acc_lds[r];
}

template <typename T>
void skew_spmv(const DSkew<T>& J, const T* x, T* y, hipStream_t s) {
  size_t lds = (size_t)J.R * (sizeof(double) + sizeof(T));
  hipLaunchKernelGGL(k_skew_spmv<T>, dim3(J.nblocks), dim3(WG), lds, s, J, x, y);
}
template void skew_spmv<double>(const DSkew<double>&, const double*, double*, hipStream_t);
template void skew_spmv<float>(const DSkew<float>&, const float*, float*, hipStream_t);

// ---------------------------------------------------------------------------
// Tall-skinny products: out = A^T B (A: n x ka column-major, B: n x nr row-major)
// ---------------------------------------------------------------------------

constexpr int GT_COLS = 8;      // output columns of A per workgroup (blockIdx.y)
constexpr int GT_MAXOUT = 512;  // ka * nr limit

// Each thread streams rows (coalesced over i) and keeps GT_COLS x NR running
// sums; workgroups write partials, the last one sums them in a fixed order.
template <typename TA, typename TB, int NR>
__global__ __launch_bounds__(WG) void k_gemm_tn(int64_t n, int ka, const TA* __restrict__ A,
                                                int64_t lda, const TB* __restrict__ B,
                                                double* __restrict__ out,
                                                const double* __restrict__ M, double* partials,
                                                unsigned* ticket) {
  constexpr int NV = GT_COLS * NR;
  __shared__ double lds[(WG / 64) * NV];
  __shared__ double res[NV];
  const int l0 = blockIdx.y * GT_COLS;
  const int nl = min(GT_COLS, ka - l0);
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  // two rows per thread and round (i and i + stride), all their loads issued
  // before the products: twice the loads in flight of one row per round
  // (190 basis vectors of 2M rows: 728 -> 538 us with 512 x-groups)
  const int64_t stride = (int64_t)gridDim.x * WG;
  int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  for (; i + stride < n; i += 2 * stride) {
    double b0[NR], b1[NR], a0[GT_COLS], a1[GT_COLS];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      b0[c] = (double)B[i * NR + c];
      b1[c] = (double)B[(i + stride) * NR + c];
    }
#pragma unroll
    for (int q = 0; q < GT_COLS; ++q)
      if (q < nl) {
        a0[q] = (double)__builtin_nontemporal_load(&A[(int64_t)(l0 + q) * lda + i]);
        a1[q] = (double)__builtin_nontemporal_load(&A[(int64_t)(l0 + q) * lda + i + stride]);
      }
#pragma unroll
    for (int q = 0; q < GT_COLS; ++q)
      if (q < nl) {
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[q * NR + c] += a0[q] * b0[c] + a1[q] * b1[c];
      }
  }
  for (; i < n; i += stride) {
    double b[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) b[c] = (double)B[i * NR + c];
#pragma unroll
    for (int q = 0; q < GT_COLS; ++q) {
      if (q < nl) {
        const double a = (double)__builtin_nontemporal_load(&A[(int64_t)(l0 + q) * lda + i]);
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[q * NR + c] += a * b[c];
      }
    }
  }
  wg_reduce<NV>(acc, lds, res);
  const int nout = ka * NR;
  const int gx = gridDim.x;
  // partial layout: [bx][o], o = l * NR + c over all ka columns
  for (int j = threadIdx.x; j < nl * NR; j += WG)
    store_partial(partials + (int64_t)blockIdx.x * nout + l0 * NR + j, res[j]);
  if (!arrive_last(ticket, gridDim.x * gridDim.y)) return;
  __shared__ double red[GT_MAXOUT];
  __shared__ double tmp[WG];
  for (int o0 = 0; o0 < nout; o0 += WG) {
    const int cnt = min(WG, nout - o0);
    const int per = max(1, WG / cnt);
    const int o = o0 + threadIdx.x / per, gs = threadIdx.x % per;
    if (threadIdx.x / per < cnt) tmp[threadIdx.x] = strided_sum(partials, gs, gx, per, nout, o);
    __syncthreads();
    if (threadIdx.x < cnt) {
      double sacc = 0.0;
      for (int q = 0; q < per; ++q) sacc += tmp[threadIdx.x * per + q];
      red[o0 + threadIdx.x] = sacc;
    }
    __syncthreads();
  }
  if (M) {  // out = M * red (NR == 1)
    for (int i = threadIdx.x; i < ka; i += WG) {
      double sacc = 0.0;
      for (int j = 0; j < ka; ++j) sacc += M[i * ka + j] * red[j];
      out[i] = sacc;
    }
  } else {
    for (int o = threadIdx.x; o < nout; o += WG) out[o] = red[o];
  }
  reset_ticket(ticket);
}

template <typename TA, typename TB>
void gemm_tn(int64_t n, int ka, const TA* A, int64_t lda, const TB* B, int nr, double* out,
             const double* M, Reducer& red, int site, hipStream_t s) {
  const int nout = ka * nr;
  if (nout > GT_MAXOUT || nout < 1 || (nr != 1 && nr != NRMAX)) return;  // callers respect these
  const int gy = (ka + GT_COLS - 1) / GT_COLS;
  int gx = (int)std::min<int64_t>((n + WG - 1) / WG, 512);
  gx = std::max(1, std::min<int>(gx, (int)((int64_t)red.max_groups * RED_SLOTS / nout)));
  if (nr == 1)
    hipLaunchKernelGGL((k_gemm_tn<TA, TB, 1>), dim3(gx, gy), dim3(WG), 0, s, n, ka, A, lda, B, out, M,
                       red.partials, red.tickets + site);
  else
    hipLaunchKernelGGL((k_gemm_tn<TA, TB, NRMAX>), dim3(gx, gy), dim3(WG), 0, s, n, ka, A, lda, B, out,
                       M, red.partials, red.tickets + site);
}
template void gemm_tn<double, double>(int64_t, int, const double*, int64_t, const double*, int,
                                      double*, const double*, Reducer&, int, hipStream_t);
template void gemm_tn<double, float>(int64_t, int, const double*, int64_t, const float*, int,
                                     double*, const double*, Reducer&, int, hipStream_t);
template void gemm_tn<float, float>(int64_t, int, const float*, int64_t, const float*, int,
                                    double*, const double*, Reducer&, int, hipStream_t);

// ---------------------------------------------------------------------------
// Small vector kernels
// ---------------------------------------------------------------------------

static inline dim3 grid_for(int64_t n) { return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + WG - 1) / WG, 65535 * 4))); }

__global__ __launch_bounds__(WG) void k_gemv_acc(int64_t n, int kt, const double* __restrict__ A,
                                                 int64_t lda, const double* __restrict__ t,
                                                 double sign, double* __restrict__ y) {
  __shared__ double ts[1024];
  for (int l = threadIdx.x; l < kt && l < 1024; l += WG) ts[l] = t[l];
  __syncthreads();
  // two rows per thread and round (i and i + stride), as in k_gemm_tn
  const int64_t stride = (int64_t)gridDim.x * WG;
  int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  for (; i + stride < n; i += 2 * stride) {
    double s0 = 0.0, s1 = 0.0;
    for (int l = 0; l < kt; ++l) {
      const double a0 = __builtin_nontemporal_load(&A[(int64_t)l * lda + i]);
      const double a1 = __builtin_nontemporal_load(&A[(int64_t)l * lda + i + stride]);
      s0 += a0 * ts[l];
      s1 += a1 * ts[l];
    }
    y[i] += sign * s0;
    y[i + stride] += sign * s1;
  }
  for (; i < n; i += stride) {
    double sacc = 0.0;
    for (int l = 0; l < kt; ++l) sacc += __builtin_nontemporal_load(&A[(int64_t)l * lda + i]) * ts[l];
    y[i] += sign * sacc;
  }
}
void gemv_acc(int64_t n, int kt, const double* A, int64_t lda, const double* t, double sign,
              double* y, hipStream_t s) {
  if (kt <= 0 || n <= 0) return;
  if (kt > 1024) kt = 1024;  // callers pass at most 512 (k + r and restart bounds)
  // at most 1024 workgroups, so that every thread has two rows in flight
  const dim3 grid((unsigned)std::min<int64_t>((n + WG - 1) / WG, 1024));
  hipLaunchKernelGGL(k_gemv_acc, grid, dim3(WG), 0, s, n, kt, A, lda, t, sign, y);
}

// y += sign * A t, then ||y||^2 reduced into *nrm2 (last workgroup, fixed order).
__global__ __launch_bounds__(WG) void k_gemv_acc_norm(int64_t n, int kt, const double* __restrict__ A,
                                                      int64_t lda, const double* __restrict__ t,
                                                      double sign, double* __restrict__ y,
                                                      double* nrm2, double* partials, unsigned* ticket) {
  __shared__ double ts[1024];
  __shared__ double lds[WG / 64];
  __shared__ double res[1];
  for (int l = threadIdx.x; l < kt && l < 1024; l += WG) ts[l] = t[l];
  __syncthreads();
  double acc[1] = {0.0};
  const int64_t stride = (int64_t)gridDim.x * WG;
  int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  for (; i + stride < n; i += 2 * stride) {
    double s0 = 0.0, s1 = 0.0;
    for (int l = 0; l < kt; ++l) {
      const double a0 = __builtin_nontemporal_load(&A[(int64_t)l * lda + i]);
      const double a1 = __builtin_nontemporal_load(&A[(int64_t)l * lda + i + stride]);
      s0 += a0 * ts[l];
      s1 += a1 * ts[l];
    }
    const double v0 = y[i] + sign * s0, v1 = y[i + stride] + sign * s1;
    y[i] = v0;
    y[i + stride] = v1;
    acc[0] += v0 * v0 + v1 * v1;
  }
  for (; i < n; i += stride) {
    double sacc = 0.0;
    for (int l = 0; l < kt; ++l) sacc += __builtin_nontemporal_load(&A[(int64_t)l * lda + i]) * ts[l];
    const double v = y[i] + sign * sacc;
    y[i] = v;
    acc[0] += v * v;
  }
  wg_reduce<1>(acc, lds, res);
  publish_partials<1>(partials, res);
  if (!arrive_last(ticket, gridDim.x)) return;
  final_reduce<1>(partials, gridDim.x, lds, res);
  if (threadIdx.x == 0) *nrm2 = res[0];
  reset_ticket(ticket);
}
void gemv_acc_norm(int64_t n, int kt, const double* A, int64_t lda, const double* t, double sign,
                   double* y, double* nrm2, Reducer& red, int site, hipStream_t s) {
  if (n <= 0) return;
  if (kt > 1024) kt = 1024;
  int groups = (int)std::min<int64_t>((n + WG - 1) / WG, 1024);
  hipLaunchKernelGGL(k_gemv_acc_norm, dim3(groups), dim3(WG), 0, s, n, kt, A, lda, t, sign, y, nrm2,
                     red.partials, red.tickets + site);
}

__global__ void k_scale(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) y[i] = a * x[i];
}
void scale(int64_t n, double a, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, grid_for(n), dim3(WG), 0, s, n, a, x, y);
}

__global__ void k_normalize(int64_t n, const double* __restrict__ x, const double* nrm2,
                            double* __restrict__ y) {
  const double inv = 1.0 / sqrt(*nrm2);
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) y[i] = x[i] * inv;
}
void normalize(int64_t n, const double* x, const double* nrm2, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize, grid_for(n), dim3(WG), 0, s, n, x, nrm2, y);
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG)
    y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];
}
void axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, grid_for(n), dim3(WG), 0, s, n, a, x, b, y);
}

__global__ void k_gather_scale(int64_t n, const int32_t* __restrict__ m, const double* __restrict__ dr,
                               const double* __restrict__ om, const double* __restrict__ x,
                               double* __restrict__ y) {
  for (int64_t j = (int64_t)blockIdx.x * WG + threadIdx.x; j < n; j += (int64_t)gridDim.x * WG)
    y[j] = om[j] * (dr[j] * x[m[j]]);
}
void gather_scale(int64_t n, const int32_t* m, const double* dr, const double* omega, const double* x,
                  double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_scale, grid_for(n), dim3(WG), 0, s, n, m, dr, omega, x, y);
}

__global__ void k_scatter_scale(int64_t n, const int32_t* __restrict__ m, const double* __restrict__ dr,
                                const double* __restrict__ om, const double* __restrict__ x,
                                double* __restrict__ y) {
  for (int64_t j = (int64_t)blockIdx.x * WG + threadIdx.x; j < n; j += (int64_t)gridDim.x * WG)
    y[m[j]] = dr[j] * (om[j] * x[j]);
}
void scatter_scale(int64_t n, const int32_t* m, const double* dr, const double* omega, const double* x,
                   double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_scale, grid_for(n), dim3(WG), 0, s, n, m, dr, omega, x, y);
}

__global__ void k_cast_d2f(int64_t n, const double* __restrict__ x, float* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) y[i] = (float)x[i];
}
__global__ void k_cast_f2d(int64_t n, const float* __restrict__ x, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) y[i] = (double)x[i];
}
void cast_d2f(int64_t n, const double* x, float* y, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_d2f, grid_for(n), dim3(WG), 0, s, n, x, y);
}
void cast_f2d(int64_t n, const float* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_f2d, grid_for(n), dim3(WG), 0, s, n, x, y);
}

// SplitMix64 (Steele, Lea, Flood 2014): output i of the stream started at
// state `seed` is mix(seed + (i+1) * 0x9E3779B97F4A7C15); the top 53 bits
// give u in [0,1) and the value is 2u - 1.
__global__ void k_splitmix(int64_t n, uint64_t seed, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    y[i] = (double)(z >> 11) * 0x1p-52 - 1.0;
  }
}
void splitmix_vector(int64_t n, uint64_t seed, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_splitmix, grid_for(n), dim3(WG), 0, s, n, seed, y);
}

template <typename T>
__global__ void k_slice_columns(int64_t n, int k, const T* __restrict__ Q, T* __restrict__ Qs) {
  const int64_t total = ((n + 63) / 64) * 64;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < total; i += (int64_t)gridDim.x * WG)
    for (int l = 0; l < k; ++l)
      Qs[(i >> 6) * (int64_t)(k * 64) + l * 64 + (i & 63)] = i < n ? Q[(int64_t)l * n + i] : T(0);
}
template <typename T>
void slice_columns(int64_t n, int k, const T* Q, T* Qs, hipStream_t s) {
  hipLaunchKernelGGL(k_slice_columns<T>, grid_for(n + 64), dim3(WG), 0, s, n, k, Q, Qs);
}
template void slice_columns<double>(int64_t, int, const double*, double*, hipStream_t);
template void slice_columns<float>(int64_t, int, const float*, float*, hipStream_t);

__global__ void k_check_finite(int64_t n, const double* __restrict__ x, int* flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG)
    bad |= !isfinite(x[i]);
  if (bad) *flag = 1;
}
void check_finite(int64_t n, const double* x, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_finite, grid_for(n), dim3(WG), 0, s, n, x, flag);
}

// ---------------------------------------------------------------------------
// Inner mrs (App. B) on S_bar = I + J_bar, J_bar = J_tilde - Q_k S_k Q_k^T
// ---------------------------------------------------------------------------

template <typename T, int NR, int KF>
__global__ __launch_bounds__(WG) void k_mrs_init(MrsLaunch L, const double* __restrict__ rhs,
                                                 int64_t ldr, const int32_t* __restrict__ perm,
                                                 const T* __restrict__ Q,
                                                 MrsBufs<T> buf, MrsState* st, double tol,
                                                 int maxit, int fixed, double* partials,
                                                 unsigned* ticket) {
  constexpr int NV = (KF + 1) * NR;
  __shared__ double lds[(WG / 64) * NV];
  __shared__ double res[NV];
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  const int64_t n = L.n;
  const int k = L.k;
  const int64_t stride = (int64_t)gridDim.x * WG;
  int64_t i0 = (int64_t)blockIdx.x * WG + threadIdx.x;
  if constexpr (NR == 1 && sizeof(T) == 8) {
    // one FP64 column: two rows per thread and round (i and i + stride), their
    // loads issued before the sums (128^3, k = 16: 115 -> 86 us; the FP32 start
    // does not gain, 62 -> 67 us, and keeps one row per round)
    for (; i0 + stride < n; i0 += 2 * stride) {
      const int64_t i1 = i0 + stride;
      const int64_t src0 = perm ? (int64_t)perm[i0] : i0, src1 = perm ? (int64_t)perm[i1] : i1;
      const double b0 = L.nr > 0 ? rhs[src0] : 0.0, b1 = L.nr > 0 ? rhs[src1] : 0.0;
      double q0[KF > 0 ? KF : 1], q1[KF > 0 ? KF : 1];
#pragma unroll
      for (int l = 0; l < KF; ++l)
        if (l < k) {
          q0[l] = (double)Q[(int64_t)l * n + i0];
          q1[l] = (double)Q[(int64_t)l * n + i1];
        }
      buf.w[1][i0] = (T)b0;
      buf.w[1][i1] = (T)b1;
      buf.w[0][i0] = T(0); buf.w[0][i1] = T(0);
      buf.w[2][i0] = T(0); buf.w[2][i1] = T(0);
      buf.p[0][i0] = T(0); buf.p[0][i1] = T(0);
      buf.p[1][i0] = T(0); buf.p[1][i1] = T(0);
      buf.x[i0] = T(0); buf.x[i1] = T(0);
      acc[0] += b0 * b0 + b1 * b1;
#pragma unroll
      for (int l = 0; l < KF; ++l)
        if (l < k) acc[1 + l] += q0[l] * (double)(T)b0 + q1[l] * (double)(T)b1;
    }
  }
  if constexpr (NR == 1 && sizeof(T) == 4 && KF > 0) {
    // one FP32 column: a pair of adjacent rows per thread and round, with
    // 8-byte loads and stores (the basis from its sliced copy, where rows 2t
    // and 2t + 1 of a slot are adjacent and slices are padded with zeros);
    // the start is bound by the number of memory instructions per row, which
    // this halves.  Needs 8-byte aligned buffers and permutation (checked
    // here, else the row loop below runs).
    const uintptr_t mis = ((uintptr_t)buf.w[0] | (uintptr_t)buf.w[1] | (uintptr_t)buf.w[2] |
                           (uintptr_t)buf.p[0] | (uintptr_t)buf.p[1] | (uintptr_t)buf.x | (uintptr_t)perm |
                           (uintptr_t)L.Qs) & 7u;
    if (mis == 0 && L.Qs != nullptr && L.kq == k) {
      const float* __restrict__ Qs = (const float*)L.Qs;
      const int64_t np = (n + 1) >> 1;
      for (int64_t pi = i0; pi < np; pi += stride) {
        const int64_t i = 2 * pi;
        const bool two = i + 1 < n;
        int64_t s0 = i, s1 = i + 1;
        if (perm) {
          if (two) {
            const int2 pp = *reinterpret_cast<const int2*>(perm + i);
            s0 = pp.x;
            s1 = pp.y;
          } else {
            s0 = perm[i];
          }
        }
        float2 q[KF];
        const int64_t qb = (i >> 6) * (int64_t)(k * 64) + (i & 63);
#pragma unroll
        for (int l = 0; l < KF; ++l)
          if (l < k) q[l] = *reinterpret_cast<const float2*>(Qs + qb + l * 64);
        const double b0 = L.nr > 0 ? rhs[s0] : 0.0;
        const double b1 = (L.nr > 0 && two) ? rhs[s1] : 0.0;
        const float f0 = (float)b0, f1 = (float)b1;
        if (two) {
          const float2 z = make_float2(0.f, 0.f);
          *reinterpret_cast<float2*>(buf.w[1] + i) = make_float2(f0, f1);
          *reinterpret_cast<float2*>(buf.w[0] + i) = z;
          *reinterpret_cast<float2*>(buf.w[2] + i) = z;
          *reinterpret_cast<float2*>(buf.p[0] + i) = z;
          *reinterpret_cast<float2*>(buf.p[1] + i) = z;
          *reinterpret_cast<float2*>(buf.x + i) = z;
        } else {
          buf.w[1][i] = f0;
          buf.w[0][i] = 0.f;
          buf.w[2][i] = 0.f;
          buf.p[0][i] = 0.f;
          buf.p[1][i] = 0.f;
          buf.x[i] = 0.f;
        }
        acc[0] += b0 * b0 + b1 * b1;
#pragma unroll
        for (int l = 0; l < KF; ++l)
          if (l < k) acc[1 + l] += (double)q[l].x * (double)f0 + (double)q[l].y * (double)f1;
      }
      i0 = n;
    }
  }
  for (int64_t i = i0; i < n; i += stride) {
    double b[NR];
    const int64_t src = perm ? (int64_t)perm[i] : i;
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      b[c] = c < L.nr ? rhs[(int64_t)c * ldr + src] : 0.0;
      buf.w[1][i * NR + c] = (T)b[c];
      buf.w[0][i * NR + c] = T(0);
      buf.w[2][i * NR + c] = T(0);
      buf.p[0][i * NR + c] = T(0);
      buf.p[1][i * NR + c] = T(0);
      buf.x[i * NR + c] = T(0);
      acc[c] += b[c] * b[c];
    }
#pragma unroll
    for (int l = 0; l < KF; ++l) {
      if (l < k) {
        const double q = (double)Q[(int64_t)l * n + i];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[(1 + l) * NR + c] += q * (double)(T)b[c];
      }
    }
  }
  wg_reduce<NV>(acc, lds, res);
  publish_partials<NV>(partials, res);
  if (!arrive_last(ticket, gridDim.x)) return;
  final_reduce<NV>(partials, gridDim.x, lds, res);
  mrs_init_finish<NR>(L, st, res, tol, maxit, fixed);
  reset_ticket(ticket);
}

// Batched start: every block of the batch (taken from the work queue) loads
// its rows' right-hand sides, zeroes the other buffers and sums ||b||^2 and
// Q_k^T b for its system; the last block of a system runs mrs_init_finish.
template <typename T, int NR, int KF>
__global__ __launch_bounds__(WG) void k_mrs_init_batched(MrsBatch B, int R, const double* __restrict__ rhs,
                                                         int64_t ldr, MrsBufs<T> buf, double tol, int maxit,
                                                         int fixed) {
  constexpr int NV = (KF + 1) * NR;
  __shared__ double lds[(WG / 64) * NV];
  __shared__ double res[NV];
  __shared__ int s_item;
  const T* __restrict__ Qs = reinterpret_cast<const T*>(B.Qs);
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)__hip_atomic_fetch_add(B.queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int b = s_item;
    __syncthreads();
    if (b >= B.nblocks) {
      if (threadIdx.x == 0 && b == B.nblocks + (int)gridDim.x - 1)
        __hip_atomic_store(B.queue, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    const MrsBatchSys& sys = B.sys[B.block_sys[b]];
    const int k = sys.k;
    double acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    const int64_t row0 = (int64_t)b * R;
    const int64_t row1 = min(row0 + R, B.n);
    for (int64_t i = row0 + threadIdx.x; i < row1; i += WG) {
      double bv[NR];
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        bv[c] = rhs[(int64_t)c * ldr + i];
        buf.w[1][i * NR + c] = (T)bv[c];
        buf.w[0][i * NR + c] = T(0);
        buf.w[2][i * NR + c] = T(0);
        buf.p[0][i * NR + c] = T(0);
        buf.p[1][i * NR + c] = T(0);
        buf.x[i * NR + c] = T(0);
        acc[c] += bv[c] * bv[c];
      }
      const T* qs = Qs + (i >> 6) * (int64_t)(B.kq * 64) + (i & 63);
#pragma unroll
      for (int l = 0; l < KF; ++l)
        if (l < k) {
          const double q = (double)qs[l * 64];
#pragma unroll
          for (int c = 0; c < NR; ++c) acc[(1 + l) * NR + c] += q * (double)(T)bv[c];
        }
    }
    wg_reduce<NV>(acc, lds, res);
    const int g = b - sys.first_block;
    publish_partials_at<NV>(sys.partials, res, g, sys.nblocks);
    if (arrive_last(sys.ticket, sys.nblocks)) {
      final_reduce<NV>(sys.partials, sys.nblocks, lds, res);
      MrsLaunch L{};
      L.nr = NR;
      L.k = k;
      L.alpha_dev = sys.alpha;
      L.sign = B.sign;
      mrs_init_finish<NR>(L, sys.st, res, tol, maxit, fixed);
      reset_ticket(sys.ticket);
    }
    __syncthreads();
  }
}

// One inner step (App. B), or the final deferred update once converged, or
// nothing once done, on rows [row0, row0 + nrow) of one system: block g of
// that system's ng blocks, whose partial sums go to `partials` (value j of
// block g at j * ng + g) and whose last block, found with `ticket`, runs the
// scalar recurrence.  Shared by the one-system kernel (one block per
// workgroup) and the batched work-queue kernel (blocks of many systems).
template <typename T, int NR, int KF, bool STAGE, typename TQ, int NT = WG, bool DENSE = false>
__device__ __forceinline__ void mrs_iter_block(const MrsLaunch& L, const DSkew<T>& J, const MrsBufs<T>& buf,
                                               MrsState* st, double* partials, unsigned* ticket,
                                               int64_t row0, int nrow, int g, int ng, double* acc_lds,
                                               T* w_lds, bool pairs = false) {
  constexpr int NV = (KF + 1) * NR;
  __shared__ double lds[(NT / 64) * NV];
  __shared__ double res[NV];
  // The state was written by the previous launch and is not written before
  // the end of this one: every thread reads it with uniform (scalar) loads, so
  // the per-column coefficients and the deflation coefficients c live in
  // scalar registers rather than in LDS or vector registers.
  // Everything below is loaded before the status test, so that the loads go
  // out together instead of after a round trip for the status (the values
  // are in bounds and unused when the solve is done).
  const int k = L.k;
  const int status = st->status;
  const int t = st->its + 1;
  const bool pend = st->col[0].has_pending != 0;
  constexpr int KF1 = KF > 0 ? KF : 1;
  T inv_nu[NR], inv_nu_old[NR], beta_prev[NR], pend_delta[NR], inv_pend_theta[NR], pend_coef[NR];
  T cv[NR][KF1];
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    const MrsCol& col = st->col[c];
    inv_nu[c] = (T)(1.0 / col.nu);
    inv_nu_old[c] = (T)(1.0 / col.nu_old);
    beta_prev[c] = (T)col.beta_prev;
    pend_delta[c] = (T)col.pend_delta;
    inv_pend_theta[c] = (T)(1.0 / col.pend_theta);
    pend_coef[c] = (T)col.pend_coef;
#pragma unroll
    for (int l = 0; l < KF1; ++l) {
      // loaded for every l < KF1 <= KMAX (in bounds) and selected after: a load
      // under the condition l < k became one scalar load and wait per l, a
      // chain of 16 round trips at the start of every launch
      const T v = (T)st->cvec[c * KMAX + l];
      cv[c][l] = (KF > 0 && l < k) ? v : T(0);
    }
  }
  const int st_fixed = st->fixed, st_maxit = st->maxit;
  const double st_tol = st->tol;
  if (status == MRS_DONE) return;
  __shared__ MrsTail<NR, KF> tail;
  MrsTailRegs<NR, KF, NT> tail_r;
  if (status == MRS_RUNNING) mrs_tail_load<T, NR, KF, NT>(tail_r, st, L);
  const T* __restrict__ wcur = buf.w[t % 3];
  const T* __restrict__ wold = buf.w[(t + 2) % 3];
  T* __restrict__ wnew = buf.w[(t + 1) % 3];
  T* __restrict__ pb = buf.p[(t + 1) % 2];
  T* __restrict__ x = buf.x;

  if (status == MRS_CONVERGED) {
    // last deferred update: p_T and x += g_T c_T p_T
    if (pend) {
      for (int il = threadIdx.x; il < nrow; il += NT) {
        const int64_t i = row0 + il;
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          const T qold = wold[i * NR + c] * inv_nu_old[c];
          const T p = (qold - pend_delta[c] * pb[i * NR + c]) * inv_pend_theta[c];
          x[i * NR + c] += pend_coef[c] * p;
        }
      }
    }
    if (!arrive_last(ticket, ng)) return;
    if (threadIdx.x == 0) st->status = MRS_DONE;
    reset_ticket(ticket);
    return;
  }

  // operator pass: acc_lds = J_tilde w_t on this block
  for (int r = threadIdx.x; r < nrow * NR; r += NT) {
    acc_lds[r] = 0.0;
    if (STAGE) w_lds[r] = wcur[row0 * NR + r];
  }
  mrs_tail_store<T, NR, KF, NT>(tail, tail_r, k);  // status is MRS_RUNNING here
  __syncthreads();
  if constexpr (DENSE) dense_block_pass<T, NR, NT>(J, row0, nrow, wcur, acc_lds);
  else skew_block_pass<T, NR, STAGE, NT>(J, row0, nrow, wcur, w_lds, acc_lds);
  __syncthreads();

  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  const T sgn = (T)L.sign;
  int il_start = threadIdx.x;
  if constexpr (NR == 1 && sizeof(T) == 4 && sizeof(TQ) == 4 && KF > 0) {
    // one FP32 column: a pair of adjacent rows per thread, 8-byte loads and
    // stores of the vectors and of the basis (rows 2t, 2t + 1 of a slot are
    // adjacent in the sliced copy, whose slices are padded with zeros), the
    // same arithmetic per row; the update is bound by memory instructions
    // per row, which this halves.  Needs 8-byte aligned vectors and an even
    // first row (checked; else the row loop below runs).
    const uintptr_t mis = ((uintptr_t)wold | (uintptr_t)wnew | (uintptr_t)pb | (uintptr_t)x |
                           (uintptr_t)L.Qs | (uintptr_t)(row0 & 1)) & 7u;
    if (pairs && mis == 0) {
      for (int il = 2 * (int)threadIdx.x; il < nrow; il += 2 * NT) {
        const int64_t i = row0 + il;
        const bool two = il + 1 < nrow;
        const float2 wo = two ? *reinterpret_cast<const float2*>(wold + i) : make_float2(wold[i], 0.f);
        const float u0 = (T)acc_lds[il] * inv_nu[0];
        const float u1 = two ? (T)acc_lds[il + 1] * inv_nu[0] : 0.f;
        const float qo0 = wo.x * inv_nu_old[0], qo1 = wo.y * inv_nu_old[0];
        const TQ* __restrict__ qs = reinterpret_cast<const TQ*>(L.Qs) + (i >> 6) * (int64_t)(L.kq * 64) + (i & 63);
        float2 qrow[KF];
        float d0 = 0.f, d1 = 0.f;
#pragma unroll
        for (int l = 0; l < KF; ++l) {
          float2 q = make_float2(0.f, 0.f);
          if (l < k) q = two ? *reinterpret_cast<const float2*>(qs + l * 64) : make_float2(qs[l * 64], 0.f);
          qrow[l] = q;
          d0 += q.x * cv[0][l];
          d1 += q.y * cv[0][l];
        }
        const float qn0 = sgn * (u0 - d0) + beta_prev[0] * qo0;
        const float qn1 = sgn * (u1 - d1) + beta_prev[0] * qo1;
        if (two) *reinterpret_cast<float2*>(wnew + i) = make_float2(qn0, qn1);
        else wnew[i] = qn0;
        acc[0] += (double)qn0 * (double)qn0 + (double)qn1 * (double)qn1;
#pragma unroll
        for (int l = 0; l < KF; ++l)
          acc[1 + l] += (double)qrow[l].x * (double)qn0 + (double)qrow[l].y * (double)qn1;
        if (pend) {
          const float2 pv = two ? *reinterpret_cast<const float2*>(pb + i) : make_float2(pb[i], 0.f);
          const float2 xv = two ? *reinterpret_cast<const float2*>(x + i) : make_float2(x[i], 0.f);
          const float p0 = (qo0 - pend_delta[0] * pv.x) * inv_pend_theta[0];
          const float p1 = (qo1 - pend_delta[0] * pv.y) * inv_pend_theta[0];
          const float x0 = xv.x + pend_coef[0] * p0, x1 = xv.y + pend_coef[0] * p1;
          if (two) {
            *reinterpret_cast<float2*>(pb + i) = make_float2(p0, p1);
            *reinterpret_cast<float2*>(x + i) = make_float2(x0, x1);
          } else {
            pb[i] = p0;
            x[i] = x0;
          }
        }
      }
      il_start = nrow;
    }
  }
  for (int il = il_start; il < nrow; il += NT) {
    const int64_t i = row0 + il;
    T defl[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) defl[c] = T(0);
    T u[NR], qold[NR], a[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      u[c] = (T)acc_lds[il * NR + c] * inv_nu[c];
      qold[c] = wold[i * NR + c] * inv_nu_old[c];
      a[c] = sgn * u[c] + beta_prev[c] * qold[c];
    }
    // Q row i streams once (non-temporal for an FP64 basis, where it helps:
    // 161 -> 150 us; for an FP32 basis it costs 124 -> 132 us).  TQ = float in
    // an FP64 kernel: the basis is stored as FP32 values.
    const TQ* __restrict__ qs = reinterpret_cast<const TQ*>(L.Qs) + (i >> 6) * (int64_t)(L.kq * 64) + (i & 63);
    constexpr bool DIRECT = direct_projection<T>();
    T qrow[DIRECT ? KF1 : 1];
#pragma unroll
    for (int l = 0; l < KF; ++l) {
      T q = T(0);
      if (l < k) q = (sizeof(TQ) == 8) ? (T)__builtin_nontemporal_load(&qs[l * 64]) : (T)qs[l * 64];
      if constexpr (DIRECT) qrow[l] = q;
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        defl[c] += q * cv[c][l];
        if constexpr (!DIRECT) acc[(1 + l) * NR + c] += (double)q * (double)a[c];
      }
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      const T qn = sgn * (u[c] - defl[c]) + beta_prev[c] * qold[c];
      wnew[i * NR + c] = qn;
      acc[c] += (double)qn * (double)qn;
      if constexpr (DIRECT) {
#pragma unroll
        for (int l = 0; l < KF; ++l) acc[(1 + l) * NR + c] += (double)qrow[l] * (double)qn;
      }
      if (pend) {
        const T p = (qold[c] - pend_delta[c] * pb[i * NR + c]) * inv_pend_theta[c];
        pb[i * NR + c] = p;
        x[i * NR + c] += pend_coef[c] * p;
      }
    }
  }
  wg_reduce<NV, NT>(acc, lds, res);
  publish_partials_at<NV, NT>(partials, res, g, ng);
  if (!arrive_last(ticket, ng)) return;
  final_reduce<NV, NT>(partials, ng, lds, res);
  mrs_scalar_update<T, NR, KF>(st, res, k, tail, st_fixed, st_maxit, st_tol, t, L.sign);
  reset_ticket(ticket);
}

// Occupancy target: 4 waves per SIMD (<= 128 VGPRs), i.e. 16 waves per CU:
// 4 workgroups of 256 threads or 2 of 512.  The one-column step can run
// 512-thread workgroups (J.threads, chosen at setup): each block then takes
// half the time.  The FP32 step, latency bound, gains where its blocks fill
// whole rounds of 512 resident workgroups better than of 1,024 (the 192^3
// tiling's 2,304 blocks are 2.25 rounds of 256-thread workgroups, 4.5 of
// 512-thread ones) and loses a little where both fill them; the FP64 step
// gains a little at both 128^3 and 192^3.

template <typename T, int NR, int KF, bool STAGE, typename TQ = T, int NT = WG, bool DENSE = false>
__global__ __launch_bounds__(NT, (NR == 1 && KF <= 16) ? 4 : 1) void k_mrs_iter(MrsLaunch L, DSkew<T> J, const T* __restrict__ Q,
                                                 MrsBufs<T> buf, MrsState* st, double* partials,
                                                 unsigned* ticket) {
  // the scalar-update code strides by WG over at most NR * KMAX words, which
  // NT >= WG threads cover once
  static_assert(NT % WG == 0 && NR * KMAX <= WG, "workgroup size");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* acc_lds = reinterpret_cast<double*>(smem_raw);
  T* w_lds = reinterpret_cast<T*>(acc_lds + (size_t)J.R * NR);
  const int64_t row0 = (int64_t)xcd_block<T>() * J.R;
  const int nrow = (int)min((int64_t)J.R, L.n - row0);
  mrs_iter_block<T, NR, KF, STAGE, TQ, NT, DENSE>(L, J, buf, st, partials, ticket, row0, nrow, blockIdx.x,
                                                  gridDim.x, acc_lds, w_lds, true);
}

// The batched inner step: one launch advances the inner solves of every
// system of a batch by one step.  The systems' rows are concatenated (each
// padded to whole row blocks of the common size J.R, so no block straddles
// two systems) and the launch is persistent: a fixed number of workgroups
// take row blocks from a device work queue (an atomic counter) until none is
// left, so that uneven systems share the chip without one launch per system.
// Each system keeps its own state, partial sums and ticket; the last block of
// a system runs that system's scalar recurrence.  The workgroup that takes
// the last ticket of the queue (nblocks + workgroups - 1: every workgroup
// takes exactly one value past the blocks) puts the counter back to zero.
template <typename T, int NR, int KF, bool STAGE>
__global__ __launch_bounds__(WG, sizeof(T) == 4 ? 2 : 1) void k_mrs_iter_batched(MrsBatch B, DSkew<T> J, MrsBufs<T> buf) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* acc_lds = reinterpret_cast<double*>(smem_raw);
  T* w_lds = reinterpret_cast<T*>(acc_lds + (size_t)J.R * NR);
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)__hip_atomic_fetch_add(B.queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int b = s_item;
    __syncthreads();
    if (b >= B.nblocks) {
      if (threadIdx.x == 0 && b == B.nblocks + (int)gridDim.x - 1)
        __hip_atomic_store(B.queue, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    const MrsBatchSys& sys = B.sys[B.block_sys[b]];
    MrsLaunch L{};
    L.n = B.n;
    L.nr = NR;
    L.k = sys.k;
    L.kq = B.kq;
    L.alpha_dev = sys.alpha;
    L.sign = B.sign;
    L.Qs = B.Qs;
    L.gram = sys.gram;
    L.q32 = 0;
    const int64_t row0 = (int64_t)b * J.R;
    const int nrow = (int)min((int64_t)J.R, B.n - row0);
    mrs_iter_block<T, NR, KF, STAGE, T>(L, J, buf, sys.st, sys.partials, sys.ticket, row0, nrow,
                                        b - sys.first_block, sys.nblocks, acc_lds, w_lds);
    __syncthreads();
  }
}

// The deflation width KF is a compile-time bound (registers): the smallest of
// {0, 8, 16, 32} that holds k (32 only for single-column solves).
static inline int pick_kf(int k, int nr) {
  if (k <= 0) return 0;
  if (k <= 8) return 8;
  if (k <= 16) return 16;
  return nr == 1 ? 32 : -1;
}

template <typename T, int NR>
void mrs_init(const MrsLaunch& L, const double* rhs, int64_t ldr, const int32_t* perm, const T* Q,
              MrsBufs<T>& buf, MrsState* st, double tol, int maxit, int fixed, Reducer& red,
              hipStream_t s) {
  int groups = (int)std::min<int64_t>((L.n + WG - 1) / WG, 1024);
  groups = std::min(groups, red.max_groups);
  const int kf = pick_kf(L.k, NR);
#define ASSS_INIT(KF)                                                                              \
  hipLaunchKernelGGL((k_mrs_init<T, NR, KF>), dim3(groups), dim3(WG), 0, s, L, rhs, ldr, perm, Q,   \
                     buf, st, tol, maxit, fixed, red.partials, red.tickets + 0)
  switch (kf) {
    case 0: ASSS_INIT(0); break;
    case 8: ASSS_INIT(8); break;
    case 16: ASSS_INIT(16); break;
    default:
      if constexpr (NR == 1) ASSS_INIT(32);
      break;
  }
#undef ASSS_INIT
}

template <typename T, int NR>
void mrs_iter(const MrsLaunch& L, const DSkew<T>& J, const T* Q, MrsBufs<T>& buf, MrsState* st,
              Reducer& red, hipStream_t s) {
  constexpr bool STAGE = (NR == 1);
  size_t lds = (size_t)J.R * NR * (sizeof(double) + (STAGE ? sizeof(T) : 0));
  const int kf = pick_kf(L.k, NR);
#define ASSS_ITER(KF)                                                                                  \
  do {                                                                                                 \
    if constexpr (sizeof(T) == 8) {                                                                    \
      if (L.q32) {                                                                                     \
        hipLaunchKernelGGL((k_mrs_iter<T, NR, KF, STAGE, float>), dim3(J.nblocks), dim3(WG), lds,       \
                           s, L, J, Q, buf, st, red.partials, red.tickets + 1);                        \
        break;                                                                                         \
      }                                                                                                \
    }                                                                                                  \
    if constexpr (NR == 1) {                                                                           \
      if (J.dense) {                                                                                   \
        hipLaunchKernelGGL((k_mrs_iter<T, NR, KF, false, T, WG, true>), dim3(J.nblocks), dim3(WG),      \
                           (size_t)J.R * NR * sizeof(double), s, L, J, Q, buf, st, red.partials,         \
                           red.tickets + 1);                                                           \
        break;                                                                                         \
      }                                                                                                \
      if (J.threads == 2 * WG) {                                                                       \
        hipLaunchKernelGGL((k_mrs_iter<T, NR, KF, STAGE, T, 2 * WG>), dim3(J.nblocks), dim3(2 * WG), lds, \
                           s, L, J, Q, buf, st, red.partials, red.tickets + 1);                        \
        break;                                                                                         \
      }                                                                                                \
    }                                                                                                  \
    hipLaunchKernelGGL((k_mrs_iter<T, NR, KF, STAGE>), dim3(J.nblocks), dim3(WG), lds, s, L, J,        \
                       Q, buf, st, red.partials, red.tickets + 1);                                     \
  } while (0)
  switch (kf) {
    case 0: ASSS_ITER(0); break;
    case 8: ASSS_ITER(8); break;
    case 16: ASSS_ITER(16); break;
    default:
      if constexpr (NR == 1) ASSS_ITER(32);
      break;
  }
#undef ASSS_ITER
}

template <typename T, int NR>
void mrs_init_batched(const MrsBatch& B, const DSkew<T>& J, const double* rhs, int64_t ldr, MrsBufs<T>& buf,
                      double tol, int maxit, int fixed, int kf, int groups, hipStream_t s) {
  groups = std::max(1, std::min(groups, B.nblocks));
#define ASSS_BINIT(KF)                                                                                    \
  hipLaunchKernelGGL((k_mrs_init_batched<T, NR, KF>), dim3(groups), dim3(WG), 0, s, B, J.R, rhs, ldr, buf, \
                     tol, maxit, fixed)
  switch (kf) {
    case 0: ASSS_BINIT(0); break;
    case 8: ASSS_BINIT(8); break;
    default: ASSS_BINIT(16); break;
  }
#undef ASSS_BINIT
}

template <typename T, int NR>
void mrs_iter_batched(const MrsBatch& B, const DSkew<T>& J, MrsBufs<T>& buf, int kf, int groups, hipStream_t s) {
  constexpr bool STAGE = (NR == 1);
  const size_t lds = (size_t)J.R * NR * (sizeof(double) + (STAGE ? sizeof(T) : 0));
  groups = std::max(1, std::min(groups, B.nblocks));
#define ASSS_BITER(KF)                                                                                    \
  hipLaunchKernelGGL((k_mrs_iter_batched<T, NR, KF, STAGE>), dim3(groups), dim3(WG), lds, s, B, J, buf)
  switch (kf) {
    case 0: ASSS_BITER(0); break;
    case 8: ASSS_BITER(8); break;
    default: ASSS_BITER(16); break;
  }
#undef ASSS_BITER
}

template <typename T, int NR>
__global__ void k_mrs_output(int64_t n, int nr, MrsBufs<T> buf, const int32_t* __restrict__ perm,
                             double* __restrict__ out, int64_t ldo) {
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
    const int64_t dst = perm ? (int64_t)perm[i] : i;
    for (int c = 0; c < nr; ++c) out[(int64_t)c * ldo + dst] = (double)buf.x[i * NR + c];
  }
}
template <typename T, int NR>
void mrs_output(int64_t n, int nr, const MrsBufs<T>& buf, const int32_t* perm, double* out, int64_t ldo,
                hipStream_t s) {
  hipLaunchKernelGGL((k_mrs_output<T, NR>), grid_for(n), dim3(WG), 0, s, n, nr, buf, perm, out, ldo);
}

__global__ void k_permute_gather(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ x,
                                 double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) y[i] = x[perm[i]];
}
__global__ void k_permute_scatter(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ x,
                                  double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) y[perm[i]] = x[i];
}
// ---------------------------------------------------------------------------
// Value gradient of a linear solve: for x = A^-1 b and lambda = A^-T dL/dx,
// dL/da_ij = -lambda_i x_j on every stored entry (i, j) of A.  The caller's
// CSR arrays are checked as they are read: an entry range outside [0, nnz) or
// a column outside [0, n) is not used and raises *bad.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(WG) void k_csr_value_grad(int64_t n, int64_t nnz, const int64_t* __restrict__ ptr,
                                                       const int32_t* __restrict__ col,
                                                       const double* __restrict__ lam,
                                                       const double* __restrict__ x, double* __restrict__ g,
                                                       int* bad) {
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
    const int64_t lo = ptr[i], hi = ptr[i + 1];
    if (lo < 0 || hi < lo || hi > nnz) {
      atomicOr(bad, 1);
      continue;
    }
    const double li = lam[i];
    for (int64_t e = lo; e < hi; ++e) {
      const int32_t c = col[e];
      if (c < 0 || c >= n) {
        atomicOr(bad, 1);
        continue;
      }
      g[e] = -li * x[c];
    }
  }
}
void csr_value_grad(int64_t n, int64_t nnz, const int64_t* ptr, const int32_t* col, const double* lam,
                    const double* x, double* g, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_csr_value_grad, grid_for(n), dim3(WG), 0, s, n, nnz, ptr, col, lam, x, g, bad);
}

void permute_gather(int64_t n, const int32_t* perm, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_permute_gather, grid_for(n), dim3(WG), 0, s, n, perm, x, y);
}
void permute_scatter(int64_t n, const int32_t* perm, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_permute_scatter, grid_for(n), dim3(WG), 0, s, n, perm, x, y);
}

#define ASSS_MRS_INST(T, NR)                                                                       \
  template void mrs_init<T, NR>(const MrsLaunch&, const double*, int64_t, const int32_t*, const T*, \
                                MrsBufs<T>&, MrsState*, double, int, int, Reducer&, hipStream_t);  \
  template void mrs_iter<T, NR>(const MrsLaunch&, const DSkew<T>&, const T*, MrsBufs<T>&,          \
                                MrsState*, Reducer&, hipStream_t);                                 \
  template void mrs_output<T, NR>(int64_t, int, const MrsBufs<T>&, const int32_t*, double*, int64_t, \
                                  hipStream_t);                                                    \

ASSS_MRS_INST(double, 1)
ASSS_MRS_INST(float, 1)
ASSS_MRS_INST(double, 4)
ASSS_MRS_INST(float, 4)

#define ASSS_BATCH_INST(T, NR)                                                                             \
  template void mrs_init_batched<T, NR>(const MrsBatch&, const DSkew<T>&, const double*, int64_t,           \
                                        MrsBufs<T>&, double, int, int, int, int, hipStream_t);              \
  template void mrs_iter_batched<T, NR>(const MrsBatch&, const DSkew<T>&, MrsBufs<T>&, int, int, hipStream_t);
ASSS_BATCH_INST(double, 4)
ASSS_BATCH_INST(float, 4)

}  // namespace asss
