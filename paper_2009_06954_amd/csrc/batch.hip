// Batched solves (asss_solve_batched): many systems, up to four right-hand
// sides each, solved together by flexible GMRES with the preconditioner of
// eq. smw, every column in lockstep.
//
// The systems' rows are concatenated into one block-diagonal layout, each
// system padded to whole row blocks of kRowBlock rows, so that every row
// block belongs to one system:
//   * the inner operator (J_tilde, Q_k) of all systems is one sliced matrix,
//     and one persistent work-queue launch advances the inner solves of all
//     systems by one step (k_mrs_iter_batched); chunks of such launches are
//     captured once in a HIP graph and replayed;
//   * the outer operator, the true residual and the back-transform are
//     block-diagonal CSR products over the concatenated rows, four columns at
//     a time;
//   * Gram-Schmidt, the SMW term and the norms are segmented products: row
//     blocks accumulate partial sums, and the last block of each (system,
//     column) adds them in a fixed order.
// Each column's Hessenberg matrix, Givens rotations, residual estimate and
// stopping test are updated on the device, one wavefront per column (the
// kernels of the one-system solve, outer.hip); the host reads their flags and
// meets the device once per outer step for all columns together (twice when
// a column needs a second Gram-Schmidt pass).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "batch.hpp"
#include "handle.hpp"

namespace asss {
namespace batch {

using namespace asss::host;

constexpr int NC = NRMAX;        // columns per system
// rows per block of the batch: the inner step's LDS accumulators take
// kRowBlock x NC doubles (32 KB, two workgroups per CU), and every block pays
// one reduction of (k + 1) NC partial sums, which 512-row blocks could not
// amortise (2 rows per thread)
constexpr int kRowBlock = 1024;
constexpr int NL = 8;            // coefficients per workgroup of the segmented products

// ---------------------------------------------------------------------------
// Segmented products
// ---------------------------------------------------------------------------

__device__ __forceinline__ void seg_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double seg_load(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum over the workgroup, fixed order (wave shuffles, then the waves in order).
__device__ __forceinline__ double block_sum(double v, double* lds) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < WG / 64; ++w) s += lds[w];
  __syncthreads();
  return s;
}

// The caller's arrays of one batch, on the device.
struct Seg {
  int64_t N;                 // padded rows
  int nblocks;
  const int32_t* block_sys;  // system of each block
  const int32_t* first;      // first block of each system
  const int32_t* nb;         // blocks of each system
};

// out[(s NC + c) ldo + l] = sum over the rows of system s of
// A[l lal + c lac + i] * w[c N + i] for l < cnt[s NC + c] (grid: row block x
// coefficient group of NL x column).  Block g of a system writes its NL
// partial sums; the last block of (system, column, group) adds them in
// block order.
__global__ __launch_bounds__(WG) void k_seg_dots(Seg sg, const double* __restrict__ A, int64_t lal, int64_t lac,
                                                 const double* __restrict__ w, const int32_t* __restrict__ cnt,
                                                 double* __restrict__ out, int ldo, double* part,
                                                 unsigned* tickets, int ngy) {
  __shared__ double lds[WG / 64];
  __shared__ double res[NL];
  __shared__ unsigned s_last;
  const int b = blockIdx.x, y = blockIdx.y, c = blockIdx.z;
  const int s = sg.block_sys[b];
  const int g = b - sg.first[s], ng = sg.nb[s];
  const int sc = s * NC + c;
  const int l0 = y * NL;
  const int nl = max(0, min(NL, cnt[sc] - l0));
  const int64_t r0 = (int64_t)b * kRowBlock;
  double acc[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) acc[q] = 0.0;
  if (nl > 0) {
    for (int64_t i = r0 + threadIdx.x; i < r0 + kRowBlock; i += WG) {
      const double wi = w[(int64_t)c * sg.N + i];
#pragma unroll
      for (int q = 0; q < NL; ++q)
        if (q < nl) acc[q] += __builtin_nontemporal_load(&A[(int64_t)(l0 + q) * lal + c * lac + i]) * wi;
    }
  }
  // partials of (s, c, y): the region of system s starts at its first block
  // and holds [(c ngy + y) NL + q] ng + g.  The nl live sums are reduced
  // together: wave sums (fixed butterfly order), then waves 0..3 in order.
  double* pp = part + (int64_t)sg.first[s] * NC * ngy * NL + ((int64_t)(c * ngy + y) * NL) * ng;
  __shared__ double wsum[WG / 64][NL];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NL; ++q)
    if (q < nl) {
      double v = acc[q];
      for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) wsum[wave][q] = v;
    }
  __syncthreads();
  if (threadIdx.x < nl) {
    double v = 0.0;
    for (int w2 = 0; w2 < WG / 64; ++w2) v += wsum[w2][threadIdx.x];
    seg_store(pp + (int64_t)threadIdx.x * ng + g, v);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  unsigned* tk = tickets + (int64_t)sc * ngy + y;
  if (threadIdx.x == 0) {
    const unsigned t = __hip_atomic_fetch_add(tk, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (t == (unsigned)ng - 1) ? 1u : 0u;
  }
  __syncthreads();
  if (!s_last) return;
  if (threadIdx.x < nl) {
    double sum = 0.0;
    for (int gg = 0; gg < ng; ++gg) sum += seg_load(pp + (int64_t)threadIdx.x * ng + gg);
    res[threadIdx.x] = sum;
  }
  __syncthreads();
  if (threadIdx.x < nl) out[(int64_t)sc * ldo + l0 + threadIdx.x] = res[threadIdx.x];
  if (threadIdx.x == 0) __hip_atomic_store(tk, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// w[c N + i] += sign * sum_{l < cnt[s NC + c]} A[l lal + c lac + i] h[(s NC + c) ldh + l]
// (grid: row block x column); if nrm2, also nrm2[s NC + c] = ||w_c||^2 over
// the rows of system s (the same partial-sum scheme as k_seg_dots).
__global__ __launch_bounds__(WG) void k_seg_update(Seg sg, double* __restrict__ w, const double* __restrict__ A,
                                                   int64_t lal, int64_t lac, const double* __restrict__ h, int ldh,
                                                   const int32_t* __restrict__ cnt, double sign,
                                                   double* __restrict__ nrm2, double* part, unsigned* tickets) {
  __shared__ double lds[WG / 64];
  __shared__ double hs[256];
  __shared__ unsigned s_last;
  const int b = blockIdx.x, c = blockIdx.y;
  const int s = sg.block_sys[b];
  const int g = b - sg.first[s], ng = sg.nb[s];
  const int sc = s * NC + c;
  const int kt = min(cnt[sc], 256);
  for (int l = threadIdx.x; l < kt; l += WG) hs[l] = h[(int64_t)sc * ldh + l];
  __syncthreads();
  const int64_t r0 = (int64_t)b * kRowBlock;
  double acc = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r0 + kRowBlock; i += WG) {
    double v = w[(int64_t)c * sg.N + i];
    if (kt > 0) {
      double sum = 0.0;
      for (int l = 0; l < kt; ++l) sum += __builtin_nontemporal_load(&A[(int64_t)l * lal + c * lac + i]) * hs[l];
      v += sign * sum;
      w[(int64_t)c * sg.N + i] = v;
    }
    acc += v * v;
  }
  if (!nrm2) return;
  double* pp = part + (int64_t)sg.first[s] * NC + (int64_t)c * ng;
  const double v = block_sum(acc, lds);
  if (threadIdx.x == 0) seg_store(pp + g, v);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  unsigned* tk = tickets + sc;
  if (threadIdx.x == 0) {
    const unsigned t = __hip_atomic_fetch_add(tk, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (t == (unsigned)ng - 1) ? 1u : 0u;
  }
  __syncthreads();
  if (!s_last) return;
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int gg = 0; gg < ng; ++gg) sum += seg_load(pp + gg);
    nrm2[sc] = sum;
    __hip_atomic_store(tk, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// dst[j lj + c N + i] = f[s NC + c] * src[c N + i] for the columns with
// j = jv[s NC + c] >= 0 (the others are left alone); with gather = 1 the
// direction is reversed (dst[c N + i] = src[j lj + c N + i], 0 where j < 0).
__global__ __launch_bounds__(WG) void k_seg_move(Seg sg, double* __restrict__ dst, const double* __restrict__ src,
                                                 int64_t lj, const int32_t* __restrict__ jv,
                                                 const double* __restrict__ f, int gather) {
  const int b = blockIdx.x, c = blockIdx.y;
  const int sc = sg.block_sys[b] * NC + c;
  const int j = jv[sc];
  const int64_t r0 = (int64_t)b * kRowBlock;
  for (int64_t i = r0 + threadIdx.x; i < r0 + kRowBlock; i += WG) {
    const int64_t e = (int64_t)c * sg.N + i;
    if (gather)
      dst[e] = j >= 0 ? src[(int64_t)j * lj + e] : 0.0;
    else if (j >= 0)
      dst[(int64_t)j * lj + e] = (f ? f[sc] : 1.0) * src[e];
  }
}

// out[(s NC + c) ldo + i] = sum_l M_s[i kr + l] t[(s NC + c) ldt + l] for the
// kr_s x kr_s matrix of system s (one workgroup per (system, column)).
__global__ __launch_bounds__(WG) void k_seg_small(const double* const* __restrict__ M, const int32_t* __restrict__ kr,
                                                  const double* __restrict__ t, int ldt, double* __restrict__ out,
                                                  int ldo, const int32_t* __restrict__ cnt) {
  const int sc = blockIdx.x, s = sc / NC;
  const int k = kr[s];
  if (cnt[sc] <= 0) return;
  for (int i = threadIdx.x; i < k; i += WG) {
    double sum = 0.0;
    for (int l = 0; l < k; ++l) sum += M[s][(int64_t)i * k + l] * t[(int64_t)sc * ldt + l];
    out[(int64_t)sc * ldo + i] = sum;
  }
}

// y[c N + i] = (mode ? b[c N + i] - : ) rs[i] sum_p val[p] cs[col[p]] x[c N + col[p]]
// for the four columns, one row per thread (block-diagonal CSR of the batch).
__global__ __launch_bounds__(WG) void k_spmv4(int64_t N, const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                              const double* __restrict__ val, const double* __restrict__ x,
                                              double* __restrict__ y, const double* __restrict__ rs,
                                              const double* __restrict__ cs, int mode, const double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= N) return;
  double acc[NC] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p) {
    const int32_t j = col[p];
    const double a = val[p] * (cs ? cs[j] : 1.0);
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] += a * x[(int64_t)c * N + j];
  }
  const double r = rs ? rs[i] : 1.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double v = r * acc[c];
    y[(int64_t)c * N + i] = mode ? b[(int64_t)c * N + i] - v : v;
  }
}

// Right-hand sides of the caller (system s: column c at B[s] + c n_s) into
// the batch layout, and b_chk = Omega P D_r b (row j of system s reads row
// m_s(j) of b); zeros for padding rows and absent columns.
__global__ __launch_bounds__(WG) void k_load_rhs(Seg sg, const double* const* __restrict__ B,
                                                 const int32_t* __restrict__ nrhs, const int64_t* __restrict__ off,
                                                 const int64_t* __restrict__ nsz, double* __restrict__ bb) {
  const int b = blockIdx.x, c = blockIdx.y;
  const int s = sg.block_sys[b];
  const int64_t r0 = (int64_t)b * kRowBlock;
  for (int64_t i = r0 + threadIdx.x; i < r0 + kRowBlock; i += WG) {
    const int64_t li = i - off[s];
    bb[(int64_t)c * sg.N + i] = (c < nrhs[s] && li < nsz[s]) ? B[s][(int64_t)c * nsz[s] + li] : 0.0;
  }
}
__global__ __launch_bounds__(WG) void k_rhs_transform(int64_t N, const int32_t* __restrict__ mg,
                                                      const double* __restrict__ drp, const double* __restrict__ om,
                                                      const double* __restrict__ bb, double* __restrict__ bc) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= N) return;
#pragma unroll
  for (int c = 0; c < NC; ++c) bc[(int64_t)c * N + i] = om[i] * (drp[i] * bb[(int64_t)c * N + mg[i]]);
}
__global__ __launch_bounds__(WG) void k_store_x(Seg sg, double* const* __restrict__ X, const int32_t* __restrict__ nrhs,
                                                const int64_t* __restrict__ off, const int64_t* __restrict__ nsz,
                                                const int32_t* __restrict__ done_mask, const double* __restrict__ x) {
  const int b = blockIdx.x, c = blockIdx.y;
  const int s = sg.block_sys[b];
  if (c >= nrhs[s] || !done_mask[s * NC + c]) return;
  const int64_t r0 = (int64_t)b * kRowBlock;
  for (int64_t i = r0 + threadIdx.x; i < r0 + kRowBlock; i += WG) {
    const int64_t li = i - off[s];
    if (li < nsz[s]) X[s][(int64_t)c * nsz[s] + li] = x[(int64_t)c * sg.N + i];
  }
}

// inner solution (row-major NC columns, inner precision) to column layout
template <typename T>
__global__ __launch_bounds__(WG) void k_inner_out(int64_t N, const T* __restrict__ x, double* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= N) return;
#pragma unroll
  for (int c = 0; c < NC; ++c) z[(int64_t)c * N + i] = (double)x[i * NC + c];
}

// Concatenation of per-system arrays into the batch layout (plan building).
__global__ void k_cat_csr_rows(int64_t n, const int64_t* __restrict__ p, int64_t poff, int64_t* __restrict__ P) {
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i <= n; i += (int64_t)gridDim.x * WG) P[i] = p[i] + poff;
}
__global__ void k_cat_csr_cols(int64_t nnz, const int32_t* __restrict__ c, int32_t coff, int32_t* __restrict__ C) {
  for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * WG) C[e] = c[e] + coff;
}
__global__ void k_fill_rows(int64_t cnt, int64_t v, int64_t* __restrict__ P) {
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * WG) P[i] = v;
}
// sliced basis of one system (stride k) into the batch's (stride kq), from
// slice s0 on; columns l >= k stay zero
template <typename T>
__global__ void k_cat_slices(int64_t nslices, int k, const T* __restrict__ src, int kq, int64_t s0, T* __restrict__ dst) {
  const int64_t total = nslices * 64 * (int64_t)k;
  for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < total; e += (int64_t)gridDim.x * WG) {
    const int64_t sl = e / (64 * (int64_t)k), r = e % (64 * (int64_t)k);
    dst[(s0 + sl) * 64 * (int64_t)kq + r] = src[e];
  }
}
// column-major n x k (leading dimension n) into rows [off, off + n) of an N x kq array
__global__ void k_cat_cols(int64_t n, int k, const double* __restrict__ src, int64_t off, int64_t N,
                           double* __restrict__ dst) {
  const int64_t total = n * (int64_t)k;
  for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < total; e += (int64_t)gridDim.x * WG)
    dst[(e / n) * N + off + e % n] = src[e];
}
__global__ void k_cat_vec(int64_t n, const double* __restrict__ src, double* __restrict__ dst) {
  for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < n; e += (int64_t)gridDim.x * WG) dst[e] = src[e];
}
__global__ void k_cat_index(int64_t n, const int32_t* __restrict__ m, int32_t off, int32_t* __restrict__ dst) {
  for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < n; e += (int64_t)gridDim.x * WG) dst[e] = m[e] + off;
}

static dim3 grid_of(int64_t n) { return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + WG - 1) / WG, 65535 * 4))); }

// ---------------------------------------------------------------------------
// Plan: the concatenated data of one set of handles
// ---------------------------------------------------------------------------

struct Plan {
  std::vector<asss_handle_t> hs;
  std::vector<uint64_t> ids;
  int nsys = 0, kq = 0, krmax = 0, m = 0;
  bool fp32 = false;
  int64_t N = 0;
  int nblocks = 0;
  std::vector<int64_t> off, nsz;
  std::vector<int32_t> first, nb, kr;
  DevArena ar;
  // batch tables
  int32_t *d_block_sys = nullptr, *d_first = nullptr, *d_nb = nullptr, *d_kr = nullptr, *d_nrhs = nullptr;
  int64_t *d_off = nullptr, *d_nsz = nullptr;
  const double** d_Mf = nullptr;
  const double** d_B = nullptr;
  double** d_X = nullptr;
  // matrices and scalings (concatenated, block diagonal)
  DCsr A, Abar, S;
  int32_t* d_mg = nullptr;
  double *d_drp = nullptr, *d_om = nullptr, *d_dc = nullptr;
  DSkew<double> J64;
  DSkew<float> J32;
  void* d_Qs = nullptr;  // sliced basis of the batch (inner precision)
  double *d_Ubar = nullptr, *d_Xs = nullptr;  // N x krmax
  // inner solve
  MrsBatchSys* d_sys = nullptr;
  MrsState* d_state = nullptr;
  double* d_ipart = nullptr;
  unsigned *d_itick = nullptr, *d_queue = nullptr;
  MrsBufs<double> ib64{};
  MrsBufs<float> ib32{};
  MrsBatch MB{};
  hipGraphExec_t graph = nullptr;
  int graph_steps = 0;
  // outer workspace: V (m + 1) x NC x N, Z m x NC x N, vectors NC x N
  double *V = nullptr, *Z = nullptr, *bb = nullptr, *bc = nullptr, *xc = nullptr, *x = nullptr, *r = nullptr,
         *zc = nullptr, *wc = nullptr, *t1 = nullptr, *pin = nullptr;
  // segmented products
  double* d_part = nullptr;
  unsigned* d_tick = nullptr;
  int ngy = 0;
  double *d_h = nullptr, *d_h2 = nullptr, *d_n1 = nullptr, *d_n2 = nullptr, *d_t = nullptr, *d_t2 = nullptr,
         *d_f = nullptr, *d_y = nullptr;
  // Hessenberg workspaces of the columns (hess_slot(m) doubles each), their
  // read-back values, stopping thresholds and cycle starts
  double *d_hess = nullptr, *d_hout = nullptr, *d_thr = nullptr, *d_beta = nullptr;
  int32_t *d_jv = nullptr, *d_cnt = nullptr, *d_cnt2 = nullptr, *d_done = nullptr;
  double* h_pin = nullptr;  // pinned host scratch for read-backs
  size_t h_pin_size = 0;
  char* h_up = nullptr;     // pinned staging of uploads, reused after each synchronisation
  size_t h_up_size = 0, h_up_used = 0;
  int32_t* d_zero = nullptr;  // zero counts (norms through k_seg_update)
  int groups = 256;
  explicit Plan(const asss_allocator_t& al) : ar(al) {}
  ~Plan() {
    if (graph) (void)hipGraphExecDestroy(graph);
    if (h_pin) (void)hipHostFree(h_pin);
    if (h_up) (void)hipHostFree(h_up);
  }
  Seg seg() const { return Seg{N, nblocks, d_block_sys, d_first, d_nb}; }
  int ldh() const { return m + 2; }
};

std::mutex g_mu;
std::vector<std::unique_ptr<Plan>> g_plans;

bool eligible(asss_handle_t h, int nrhs, const asss_solve_opts_t& o) {
  return !h->il.on && h->d_perm == nullptr && h->k_eff <= 16 && h->kr <= 256 && nrhs <= NC && o.outer == ASSS_OUTER_FGMRES &&
         !o.use_x0 && o.fixed_inner_steps == 0;
}

void copy_cat_csr(Plan& P, DCsr& out, const std::vector<const DCsr*>& src, hipStream_t s) {
  int64_t nnz = 0;
  for (auto* M : src) nnz += M->nnz;
  out.nrows = out.ncols = P.N;
  out.nnz = nnz;
  out.ptr = P.ar.alloc<int64_t>(P.N + 1);
  out.col = P.ar.alloc<int32_t>(std::max<int64_t>(1, nnz));
  out.val = P.ar.alloc<double>(std::max<int64_t>(1, nnz));
  out.lanes = 0;
  int64_t poff = 0;
  for (int sidx = 0; sidx < P.nsys; ++sidx) {
    const DCsr& M = *src[sidx];
    const int64_t o = P.off[sidx], n = P.nsz[sidx];
    hipLaunchKernelGGL(k_cat_csr_rows, grid_of(n + 1), dim3(WG), 0, s, n, M.ptr, poff, out.ptr + o);
    if (M.nnz > 0) {
      hipLaunchKernelGGL(k_cat_csr_cols, grid_of(M.nnz), dim3(WG), 0, s, M.nnz, M.col, (int32_t)o, out.col + poff);
      HIPCHK(hipMemcpyAsync(out.val + poff, M.val, M.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    poff += M.nnz;
    const int64_t pad_end = (sidx + 1 < P.nsys) ? P.off[sidx + 1] : P.N;
    if (pad_end > o + n) hipLaunchKernelGGL(k_fill_rows, grid_of(pad_end - o - n), dim3(WG), 0, s, pad_end - o - n, poff, out.ptr + o + n + 1);
  }
}

Plan* build_plan(const std::vector<asss_handle_t>& hs, bool fp32, int m, hipStream_t s) {
  auto P = std::make_unique<Plan>(hs[0]->ar.al);
  P->hs = hs;
  for (auto h : hs) P->ids.push_back(h->uid);
  P->nsys = (int)hs.size();
  P->fp32 = fp32;
  P->m = m;
  P->off.resize(P->nsys);
  P->nsz.resize(P->nsys);
  P->first.resize(P->nsys);
  P->nb.resize(P->nsys);
  P->kr.resize(P->nsys);
  int64_t rows = 0;
  int blocks = 0;
  for (int s2 = 0; s2 < P->nsys; ++s2) {
    asss_handle_t h = hs[s2];
    P->off[s2] = rows;
    P->nsz[s2] = h->n;
    P->nb[s2] = (int)((h->n + kRowBlock - 1) / kRowBlock);
    P->first[s2] = blocks;
    blocks += P->nb[s2];
    rows += (int64_t)P->nb[s2] * kRowBlock;
    P->kq = std::max(P->kq, h->k_eff);
    P->kr[s2] = h->kr;
    P->krmax = std::max(P->krmax, h->kr);
  }
  if (rows > INT32_MAX) throw Error{ASSS_ERR_INVALID_ARG, "the batch has more than 2^31 rows"};
  P->N = rows;
  P->nblocks = blocks;
  const int64_t N = rows;
  DevArena& ar = P->ar;
  // tables
  std::vector<int32_t> bsys(blocks);
  for (int s2 = 0; s2 < P->nsys; ++s2)
    for (int b = 0; b < P->nb[s2]; ++b) bsys[P->first[s2] + b] = s2;
  P->d_block_sys = ar.upload(bsys, s);
  P->d_first = ar.upload(P->first, s);
  P->d_nb = ar.upload(P->nb, s);
  P->d_kr = ar.upload(P->kr, s);
  P->d_off = ar.upload(P->off, s);
  P->d_nsz = ar.upload(P->nsz, s);
  P->d_nrhs = ar.alloc<int32_t>(P->nsys);
  P->d_B = (const double**)ar.alloc<double*>(P->nsys);
  P->d_X = ar.alloc<double*>(P->nsys);
  {
    std::vector<const double*> mf(P->nsys);
    for (int s2 = 0; s2 < P->nsys; ++s2) mf[s2] = hs[s2]->d_Mf;
    P->d_Mf = (const double**)ar.alloc<double*>(P->nsys);
    HIPCHK(hipMemcpyAsync(P->d_Mf, mf.data(), P->nsys * sizeof(double*), hipMemcpyHostToDevice, s));
  }
  // matrices
  std::vector<const DCsr*> As, Abars, Ss;
  for (auto h : hs) { As.push_back(&h->dA); Abars.push_back(&h->dAbar); Ss.push_back(&h->dS); }
  copy_cat_csr(*P, P->A, As, s);
  copy_cat_csr(*P, P->Abar, Abars, s);
  copy_cat_csr(*P, P->S, Ss, s);
  // scalings and the matching (padding rows: zeros, index of the row itself)
  P->d_mg = ar.alloc<int32_t>(N);
  P->d_drp = ar.alloc<double>(N);
  P->d_om = ar.alloc<double>(N);
  P->d_dc = ar.alloc<double>(N);
  HIPCHK(hipMemsetAsync(P->d_drp, 0, N * sizeof(double), s));
  HIPCHK(hipMemsetAsync(P->d_om, 0, N * sizeof(double), s));
  HIPCHK(hipMemsetAsync(P->d_dc, 0, N * sizeof(double), s));
  {
    std::vector<int32_t> mg(N);
    for (int64_t i = 0; i < N; ++i) mg[i] = (int32_t)i;
    HIPCHK(hipMemcpyAsync(P->d_mg, mg.data(), N * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  for (int s2 = 0; s2 < P->nsys; ++s2) {
    asss_handle_t h = hs[s2];
    const int64_t o = P->off[s2], n = h->n;
    hipLaunchKernelGGL(k_cat_index, grid_of(n), dim3(WG), 0, s, n, h->d_m, (int32_t)o, P->d_mg + o);
    hipLaunchKernelGGL(k_cat_vec, grid_of(n), dim3(WG), 0, s, n, h->d_drp, P->d_drp + o);
    hipLaunchKernelGGL(k_cat_vec, grid_of(n), dim3(WG), 0, s, n, h->d_om, P->d_om + o);
    hipLaunchKernelGGL(k_cat_vec, grid_of(n), dim3(WG), 0, s, n, h->d_dc, P->d_dc + o);
  }
  // inner operator: the systems' J_tilde (upper triangles) in one block-diagonal CSR
  {
    Csr Jc;
    Jc.nrows = Jc.ncols = N;
    Jc.ptr.assign(N + 1, 0);
    int64_t nnz = 0;
    for (auto h : hs) nnz += h->U.nnz();
    Jc.col.resize(nnz);
    Jc.val.resize(nnz);
    int64_t e = 0;
    for (int s2 = 0; s2 < P->nsys; ++s2) {
      asss_handle_t h = hs[s2];
      const int64_t o = P->off[s2];
      const int64_t end = (s2 + 1 < P->nsys) ? P->off[s2 + 1] : N;
      for (int64_t i = 0; i < end - o; ++i) {
        if (i < h->n)
          for (int64_t p = h->U.ptr[i]; p < h->U.ptr[i + 1]; ++p) {
            Jc.col[e] = (int32_t)(h->U.col[p] + o);
            Jc.val[e] = h->jval[p];
            ++e;
          }
        Jc.ptr[o + i + 1] = e;
      }
    }
    SkewSell sell = pack_skew_sell(Jc, kRowBlock, SKEW_AUTO);
    SkewLayout lay = upload_layout(ar, sell, s, 0);
    P->J64 = lay.J64;
    P->J32 = lay.J32;
  }
  // sliced basis, U_bar and X of the batch
  const int kq = std::max(1, P->kq);
  const int64_t nsl = N / 64;
  if (fp32) {
    float* q = ar.alloc<float>(nsl * 64 * kq);
    HIPCHK(hipMemsetAsync(q, 0, nsl * 64 * kq * sizeof(float), s));
    for (int s2 = 0; s2 < P->nsys; ++s2)
      if (hs[s2]->k_eff > 0)
        hipLaunchKernelGGL(k_cat_slices<float>, grid_of((hs[s2]->n + 63) / 64 * 64 * hs[s2]->k_eff), dim3(WG), 0, s,
                           (int64_t)((hs[s2]->n + 63) / 64), hs[s2]->k_eff, hs[s2]->d_Qs32, kq, P->off[s2] / 64, q);
    P->d_Qs = q;
  } else {
    double* q = ar.alloc<double>(nsl * 64 * kq);
    HIPCHK(hipMemsetAsync(q, 0, nsl * 64 * kq * sizeof(double), s));
    for (int s2 = 0; s2 < P->nsys; ++s2)
      if (hs[s2]->k_eff > 0)
        hipLaunchKernelGGL(k_cat_slices<double>, grid_of((hs[s2]->n + 63) / 64 * 64 * hs[s2]->k_eff), dim3(WG), 0, s,
                           (int64_t)((hs[s2]->n + 63) / 64), hs[s2]->k_eff, hs[s2]->d_Qs64, kq, P->off[s2] / 64, q);
    P->d_Qs = q;
  }
  const int krm = std::max(1, P->krmax);
  P->d_Ubar = ar.alloc<double>(N * krm);
  P->d_Xs = ar.alloc<double>(N * krm);
  HIPCHK(hipMemsetAsync(P->d_Ubar, 0, N * krm * sizeof(double), s));
  HIPCHK(hipMemsetAsync(P->d_Xs, 0, N * krm * sizeof(double), s));
  for (int s2 = 0; s2 < P->nsys; ++s2)
    if (hs[s2]->kr > 0) {
      hipLaunchKernelGGL(k_cat_cols, grid_of(hs[s2]->n * hs[s2]->kr), dim3(WG), 0, s, hs[s2]->n, hs[s2]->kr,
                         hs[s2]->d_Ubar, P->off[s2], N, P->d_Ubar);
      hipLaunchKernelGGL(k_cat_cols, grid_of(hs[s2]->n * hs[s2]->kr), dim3(WG), 0, s, hs[s2]->n, hs[s2]->kr,
                         hs[s2]->d_X, P->off[s2], N, P->d_Xs);
    }
  // inner solve state
  P->d_state = ar.alloc<MrsState>(P->nsys);
  P->d_ipart = ar.alloc<double>((int64_t)blocks * RED_SLOTS);
  P->d_itick = ar.alloc<unsigned>(P->nsys);
  P->d_queue = ar.alloc<unsigned>(1);
  HIPCHK(hipMemsetAsync(P->d_itick, 0, P->nsys * sizeof(unsigned), s));
  HIPCHK(hipMemsetAsync(P->d_queue, 0, sizeof(unsigned), s));
  {
    std::vector<MrsBatchSys> sys(P->nsys);
    for (int s2 = 0; s2 < P->nsys; ++s2) {
      asss_handle_t h = hs[s2];
      sys[s2].st = P->d_state + s2;
      sys[s2].partials = P->d_ipart + (int64_t)P->first[s2] * RED_SLOTS;
      sys[s2].ticket = P->d_itick + s2;
      sys[s2].alpha = h->d_alpha;
      sys[s2].gram = fp32 ? h->d_G32 : h->d_G64;
      sys[s2].k = h->k_eff;
      sys[s2].nblocks = P->nb[s2];
      sys[s2].first_block = P->first[s2];
      sys[s2].pad = 0;
    }
    P->d_sys = ar.upload(sys, s);
  }
  if (fp32) {
    for (int b = 0; b < 3; ++b) P->ib32.w[b] = ar.alloc<float>(N * NC);
    for (int b = 0; b < 2; ++b) P->ib32.p[b] = ar.alloc<float>(N * NC);
    P->ib32.x = ar.alloc<float>(N * NC);
  } else {
    for (int b = 0; b < 3; ++b) P->ib64.w[b] = ar.alloc<double>(N * NC);
    for (int b = 0; b < 2; ++b) P->ib64.p[b] = ar.alloc<double>(N * NC);
    P->ib64.x = ar.alloc<double>(N * NC);
  }
  P->MB.n = N;
  P->MB.nblocks = blocks;
  P->MB.kq = kq;
  P->MB.sign = +1;
  P->MB.sys = P->d_sys;
  P->MB.block_sys = P->d_block_sys;
  P->MB.queue = P->d_queue;
  P->MB.Qs = P->d_Qs;
  {
    int dev = 0, cus = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    P->groups = std::max(1, cus) * (fp32 ? 2 : 1);
  }
  // outer workspace
  const int64_t vec = N * NC;
  P->V = ar.alloc<double>(vec * (m + 1));
  P->Z = ar.alloc<double>(vec * m);
  for (double** v : {&P->bb, &P->bc, &P->xc, &P->x, &P->r, &P->zc, &P->wc, &P->t1, &P->pin}) *v = ar.alloc<double>(vec);
  P->ngy = (m + 2 + NL - 1) / NL;
  const int64_t npart = (int64_t)blocks * NC * std::max(P->ngy, (krm + NL - 1) / NL) * NL;
  P->d_part = ar.alloc<double>(npart);
  P->d_tick = ar.alloc<unsigned>((int64_t)P->nsys * NC * std::max(P->ngy, (krm + NL - 1) / NL));
  HIPCHK(hipMemsetAsync(P->d_tick, 0, (int64_t)P->nsys * NC * std::max(P->ngy, (krm + NL - 1) / NL) * sizeof(unsigned), s));
  const int64_t ncol = (int64_t)P->nsys * NC;
  const int ldh = P->ldh();
  P->d_h = ar.alloc<double>(ncol * ldh);
  P->d_h2 = ar.alloc<double>(ncol * ldh);
  P->d_n1 = ar.alloc<double>(ncol);
  P->d_n2 = ar.alloc<double>(ncol);
  P->d_t = ar.alloc<double>(ncol * krm);
  P->d_t2 = ar.alloc<double>(ncol * krm);
  P->d_f = ar.alloc<double>(ncol);
  P->d_y = ar.alloc<double>(ncol * std::max(1, m));
  P->d_hess = ar.alloc<double>(ncol * hess_slot(std::max(1, m)));
  P->d_hout = ar.alloc<double>(ncol * HESS_OUT);
  P->d_thr = ar.alloc<double>(ncol);
  P->d_beta = ar.alloc<double>(ncol);
  P->d_jv = ar.alloc<int32_t>(ncol);
  P->d_cnt = ar.alloc<int32_t>(ncol);
  P->d_cnt2 = ar.alloc<int32_t>(ncol);
  P->d_done = ar.alloc<int32_t>(ncol);
  P->h_pin_size = (size_t)ncol * (2 * ldh + 8 + std::max(1, m)) * sizeof(double) + (size_t)P->nsys * sizeof(MrsState);
  HIPCHK(hipHostMalloc((void**)&P->h_pin, P->h_pin_size, hipHostMallocDefault));
  P->h_up_size = (size_t)ncol * (8 * sizeof(int32_t) + (4 + std::max(1, m)) * sizeof(double)) + 4096;
  HIPCHK(hipHostMalloc((void**)&P->h_up, P->h_up_size, hipHostMallocDefault));
  P->d_zero = ar.upload(std::vector<int32_t>(ncol, 0), s);
  HIPCHK(hipStreamSynchronize(s));
  Plan* raw = P.get();
  g_plans.push_back(std::move(P));
  return raw;
}

template <typename T>
MrsBufs<T>& bufs(Plan& P) {
  if constexpr (std::is_same<T, float>::value) return P.ib32;
  else return P.ib64;
}
template <typename T>
const DSkew<T>& skew(const Plan& P) {
  if constexpr (std::is_same<T, float>::value) return P.J32;
  else return P.J64;
}

int pick_kf(int kq) { return kq <= 0 ? 0 : (kq <= 8 ? 8 : 16); }

// Replays of a graph of `graph_steps` batched inner steps, captured once on a
// stream of the plan's own (the caller's stream may be the null stream, which
// cannot be captured); the kernel arguments never change, every step reads
// its position from the device state.
template <typename T>
void ensure_graph(Plan& P, int kf) {
  if (P.graph) return;
  constexpr int kSteps = 4;
  hipStream_t cap = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    MrsBufs<T>& buf = bufs<T>(P);
    const DSkew<T>& J = skew<T>(P);
    for (int i = 0; i < kSteps; ++i) mrs_iter_batched<T, NC>(P.MB, J, buf, kf, P.groups, cap);
    e = hipStreamEndCapture(cap, &g);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&P.graph, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cap);
  HIPCHK(e);
  P.graph_steps = kSteps;
}

// Batched inner solve of the four columns of every system (rhs in P.pin,
// column layout); the solution goes to P.zc.  Returns the inner steps of each
// system; the device state is checked once per graph replay.
template <typename T>
std::vector<int> inner_solve(Plan& P, double tol, int maxit, hipStream_t s, double& kern_s, int& launches) {
  MrsBufs<T>& buf = bufs<T>(P);
  const DSkew<T>& J = skew<T>(P);
  const int kf = pick_kf(P.kq);
  ensure_graph<T>(P, kf);
  mrs_init_batched<T, NC>(P.MB, J, P.pin, P.N, buf, tol, maxit, 0, kf, P.groups, s);
  MrsState* hst = reinterpret_cast<MrsState*>(P.h_pin);
  std::vector<int> its(P.nsys, 0);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (int guard = 0;; ++guard) {
    HIPCHK(hipEventRecord(e0, s));
    HIPCHK(hipGraphLaunch(P.graph, s));
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipMemcpyAsync(hst, P.d_state, P.nsys * sizeof(MrsState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    kern_s += 1e-3 * ms;
    launches += P.graph_steps;
    bool all_done = true;
    for (int s2 = 0; s2 < P.nsys; ++s2) {
      its[s2] = hst[s2].its;
      all_done &= hst[s2].status == MRS_DONE;
    }
    if (all_done) break;
    if (guard > maxit / P.graph_steps + 4) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw Error{ASSS_ERR_INTERNAL, "batched inner solve made no progress"};
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  hipLaunchKernelGGL(k_inner_out<T>, grid_of(P.N), dim3(WG), 0, s, P.N, buf.x, P.zc);
  return its;
}

// Host side of one column of flexible GMRES: its position in the cycle,
// norms, stopping threshold and counters.  The Hessenberg matrix, the Givens
// rotations, the residual estimate and its test live on the device
// (outer.hip, one workspace per column).
struct Col {
  bool active = false, done = false, implicit_ok = false, end = false;
  int j = 0, m = 1;
  double bn = 0, bcn = 0, thr = 0;
  double gabs = 0;  // |g_j|, the residual estimate after the last step
  asss_info_t inf{};
  asss_status_t status = ASSS_NOT_CONVERGED;
};

asss_status_t solve(Plan& P, const double* const* B, double* const* X, const int32_t* nrhs,
                    const asss_solve_opts_t& o, asss_info_t* infos, int maxr, hipStream_t s) {
  const double t0 = now_s();
  const int64_t N = P.N, vec = N * NC;
  const int m = P.m, ldh = P.ldh(), ns = P.nsys, ncol = ns * NC;
  const Seg sg = P.seg();
  const dim3 gb((unsigned)P.nblocks, NC);
  std::vector<Col> cols(ncol);
  double* hp = P.h_pin;  // pinned scratch (reused below)
  std::vector<int32_t> jv(ncol), cnt(ncol), cnt2(ncol), done(ncol, 0);
  // uploads go through pinned staging (an asynchronous copy may run after the
  // host vector is gone); the staging is reused after each synchronisation
  auto stage = [&](const void* src, size_t bytes) -> void* {
    const size_t at = (P.h_up_used + 255) & ~(size_t)255;
    if (at + bytes > P.h_up_size) throw Error{ASSS_ERR_INTERNAL, "batched solve: upload staging exhausted"};
    std::memcpy(P.h_up + at, src, bytes);
    P.h_up_used = at + bytes;
    return P.h_up + at;
  };
  auto sync = [&]() {
    HIPCHK(hipStreamSynchronize(s));
    P.h_up_used = 0;
  };
  auto up_i = [&](int32_t* d, const std::vector<int32_t>& v) {
    HIPCHK(hipMemcpyAsync(d, stage(v.data(), v.size() * sizeof(int32_t)), v.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, s));
  };
  auto up_d = [&](double* d, const std::vector<double>& v) {
    HIPCHK(hipMemcpyAsync(d, stage(v.data(), v.size() * sizeof(double)), v.size() * sizeof(double),
                          hipMemcpyHostToDevice, s));
  };
  // squared norms of the columns of a vector (segmented by system): the
  // update kernel with no coefficients reads the vector once and reduces
  auto norms = [&](const double* a, double* out) {
    hipLaunchKernelGGL(k_seg_update, gb, dim3(WG), 0, s, sg, const_cast<double*>(a), (const double*)nullptr,
                       (int64_t)0, (int64_t)0, (const double*)nullptr, 0, P.d_zero, 0.0, out, P.d_part, P.d_tick);
  };
  P.h_up_used = 0;
  HIPCHK(hipMemcpyAsync(P.d_B, stage(B, ns * sizeof(double*)), ns * sizeof(double*), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(P.d_X, stage(X, ns * sizeof(double*)), ns * sizeof(double*), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(P.d_nrhs, stage(nrhs, ns * sizeof(int32_t)), ns * sizeof(int32_t), hipMemcpyHostToDevice, s));
  // ---- start: b, b_chk, their norms
  hipLaunchKernelGGL(k_load_rhs, gb, dim3(WG), 0, s, sg, P.d_B, P.d_nrhs, P.d_off, P.d_nsz, P.bb);
  hipLaunchKernelGGL(k_rhs_transform, grid_of(N), dim3(WG), 0, s, N, P.d_mg, P.d_drp, P.d_om, P.bb, P.bc);
  norms(P.bb, P.d_n1);
  HIPCHK(hipMemcpyAsync(hp, P.d_n1, ncol * sizeof(double), hipMemcpyDeviceToHost, s));
  sync();
  std::vector<double> bn2(hp, hp + ncol);
  norms(P.bc, P.d_n1);
  HIPCHK(hipMemcpyAsync(hp, P.d_n1, ncol * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemsetAsync(P.xc, 0, vec * sizeof(double), s));
  HIPCHK(hipMemsetAsync(P.x, 0, vec * sizeof(double), s));
  sync();
  std::vector<double> f(ncol, 0.0), betas(ncol, -1.0);
  for (int sidx = 0; sidx < ns; ++sidx)
    for (int c = 0; c < NC; ++c) {
      Col& C = cols[sidx * NC + c];
      asss_handle_t h = P.hs[sidx];
      C.inf.k_eff = h->k_eff;
      C.inf.rank_r = h->r;
      C.inf.setup_host_s = h->setup_host_s;
      C.inf.setup_device_s = h->setup_device_s;
      jv[sidx * NC + c] = -1;
      if (c >= nrhs[sidx]) { C.done = true; continue; }
      C.bn = std::sqrt(bn2[sidx * NC + c]);
      C.bcn = std::sqrt(hp[sidx * NC + c]);
      if (C.bn == 0.0) {  // x = 0 (already zero in P.x)
        C.inf.converged = 1;
        C.status = ASSS_OK;
        C.done = true;
        done[sidx * NC + c] = 1;
        continue;
      }
      C.m = m;
      C.thr = o.tol * C.bcn;
      // first cycle: r = b_chk, beta = ||b_chk||
      C.gabs = C.bcn;
      betas[sidx * NC + c] = C.bcn;
      C.j = 0;
      C.inf.cycles = 1;
      C.implicit_ok = C.bcn <= C.thr;
      C.active = true;
      jv[sidx * NC + c] = 0;
      f[sidx * NC + c] = 1.0 / C.bcn;
    }
  up_i(P.d_jv, jv);
  up_d(P.d_f, f);
  up_d(P.d_beta, betas);
  hess_reset_batched(P.d_hess, m, ncol, P.d_beta, s);
  hipLaunchKernelGGL(k_seg_move, gb, dim3(WG), 0, s, sg, P.V, P.bc, vec, P.d_jv, P.d_f, 0);
  double kern_s = 0.0;
  int launches = 0;
  const bool fp32 = P.fp32;
  // the end of a cycle for the columns with C.end set: x_chk += Z y,
  // back-transform, true residual; then finish or restart
  auto end_cycles = [&]() {
    for (int q = 0; q < ncol; ++q) {
      Col& C = cols[q];
      cnt[q] = 0;
      if (!C.end) continue;
      cnt[q] = C.j;
      C.inf.relres_implicit = C.gabs / C.bcn;
    }
    up_i(P.d_cnt, cnt);
    hess_solve_batched(P.d_hess, m, m, ncol, P.d_cnt, P.d_y, s);
    hipLaunchKernelGGL(k_seg_update, gb, dim3(WG), 0, s, sg, P.xc, P.Z, vec, N, P.d_y, m, P.d_cnt, 1.0,
                       (double*)nullptr, P.d_part, P.d_tick);
    // x = D_c S Omega x_chk, r = b - A x
    hipLaunchKernelGGL(k_spmv4, grid_of(N), dim3(WG), 0, s, N, P.S.ptr, P.S.col, P.S.val, P.xc, P.x, P.d_dc, P.d_om, 0,
                       (const double*)nullptr);
    hipLaunchKernelGGL(k_spmv4, grid_of(N), dim3(WG), 0, s, N, P.A.ptr, P.A.col, P.A.val, P.x, P.r,
                       (const double*)nullptr, (const double*)nullptr, 1, P.bb);
    norms(P.r, P.d_n1);
    HIPCHK(hipMemcpyAsync(hp, P.d_n1, ncol * sizeof(double), hipMemcpyDeviceToHost, s));
    sync();
    bool any_restart = false;
    std::vector<int32_t> rj(ncol, -1);
    for (int q = 0; q < ncol; ++q) {
      Col& C = cols[q];
      if (!C.end) continue;
      C.end = false;
      const double relres = std::sqrt(hp[q]) / C.bn;
      C.inf.relres_true = relres;
      if (relres <= o.tol) {
        C.status = ASSS_OK;
        C.inf.converged = 1;
        C.done = true;
        C.active = false;
        done[q] = 1;
        continue;
      }
      if (C.inf.outer_its >= o.max_outer || C.j == 0) {
        C.done = true;
        C.active = false;
        done[q] = 1;
        continue;
      }
      if (C.implicit_ok) C.thr = C.thr * 0.5 * o.tol / relres;
      rj[q] = 0;
      any_restart = true;
    }
    if (!any_restart) return;
    // restart: r_chk = b_chk - A_chk x_chk, beta = ||r_chk||, V_0 = r_chk / beta
    hipLaunchKernelGGL(k_spmv4, grid_of(N), dim3(WG), 0, s, N, P.S.ptr, P.S.col, P.S.val, P.xc, P.t1,
                       (const double*)nullptr, P.d_om, 0, (const double*)nullptr);
    hipLaunchKernelGGL(k_spmv4, grid_of(N), dim3(WG), 0, s, N, P.Abar.ptr, P.Abar.col, P.Abar.val, P.t1, P.wc, P.d_om,
                       (const double*)nullptr, 1, P.bc);
    norms(P.wc, P.d_n1);
    HIPCHK(hipMemcpyAsync(hp, P.d_n1, ncol * sizeof(double), hipMemcpyDeviceToHost, s));
    sync();
    std::vector<double> ff(ncol, 0.0), rb(ncol, -1.0);
    std::vector<int32_t> mv(ncol, -1);
    for (int q = 0; q < ncol; ++q) {
      if (rj[q] < 0) continue;
      Col& C = cols[q];
      const double beta = std::sqrt(hp[q]);
      C.inf.cycles++;
      C.gabs = beta;
      rb[q] = beta;
      C.j = 0;
      C.implicit_ok = beta <= C.thr;
      if (beta > 0) {
        mv[q] = 0;
        ff[q] = 1.0 / beta;
      } else {
        C.end = true;  // handled by the next call (j = 0 ends the solve)
      }
    }
    up_i(P.d_cnt, mv);
    up_d(P.d_f, ff);
    up_d(P.d_beta, rb);
    hess_reset_batched(P.d_hess, m, ncol, P.d_beta, s);
    hipLaunchKernelGGL(k_seg_move, gb, dim3(WG), 0, s, sg, P.V, P.wc, vec, P.d_cnt, P.d_f, 0);
  };
  for (int step = 0;; ++step) {
    int nact = 0;
    for (int q = 0; q < ncol; ++q) {
      Col& C = cols[q];
      jv[q] = (C.active && !C.done) ? C.j : -1;
      nact += jv[q] >= 0;
    }
    if (nact == 0) break;
    up_i(P.d_jv, jv);
    // z_j = P^-1 v_j for every active column
    hipLaunchKernelGGL(k_seg_move, gb, dim3(WG), 0, s, sg, P.pin, P.V, vec, P.d_jv, (const double*)nullptr, 1);
    std::vector<int> its = fp32 ? inner_solve<float>(P, o.inner_tol, o.inner_maxit, s, kern_s, launches)
                                : inner_solve<double>(P, o.inner_tol, o.inner_maxit, s, kern_s, launches);
    for (int q = 0; q < ncol; ++q) {
      cnt[q] = jv[q] >= 0 ? P.kr[q / NC] : 0;
      cnt2[q] = jv[q] >= 0 ? cols[q].j + 1 : 0;
    }
    up_i(P.d_cnt, cnt);
    if (P.krmax > 0) {  // SMW: z -= X (C^-1 Sigma) (U_bar^T z)
      const int ngk = (P.krmax + NL - 1) / NL;
      hipLaunchKernelGGL(k_seg_dots, dim3((unsigned)P.nblocks, ngk, NC), dim3(WG), 0, s, sg, P.d_Ubar, N, (int64_t)0,
                         P.zc, P.d_cnt, P.d_t, P.krmax, P.d_part, P.d_tick, ngk);
      hipLaunchKernelGGL(k_seg_small, dim3(ncol), dim3(WG), 0, s, P.d_Mf, P.d_kr, P.d_t, P.krmax, P.d_t2, P.krmax,
                         P.d_cnt);
      hipLaunchKernelGGL(k_seg_update, gb, dim3(WG), 0, s, sg, P.zc, P.d_Xs, N, (int64_t)0, P.d_t2, P.krmax, P.d_cnt,
                         -1.0, (double*)nullptr, P.d_part, P.d_tick);
    }
    hipLaunchKernelGGL(k_seg_move, gb, dim3(WG), 0, s, sg, P.Z, P.zc, vec, P.d_jv, (const double*)nullptr, 0);
    // w = A_chk z (Omega Abar S Omega z)
    hipLaunchKernelGGL(k_spmv4, grid_of(N), dim3(WG), 0, s, N, P.S.ptr, P.S.col, P.S.val, P.zc, P.t1,
                       (const double*)nullptr, P.d_om, 0, (const double*)nullptr);
    hipLaunchKernelGGL(k_spmv4, grid_of(N), dim3(WG), 0, s, N, P.Abar.ptr, P.Abar.col, P.Abar.val, P.t1, P.wc, P.d_om,
                       (const double*)nullptr, 0, (const double*)nullptr);
    // classical Gram-Schmidt: h = V^T w, ||w||^2, w -= V h, ||w||^2 (as many
    // coefficient groups as the longest column needs)
    up_i(P.d_cnt2, cnt2);
    const int ngy = (*std::max_element(cnt2.begin(), cnt2.end()) + NL - 1) / NL;
    hipLaunchKernelGGL(k_seg_dots, dim3((unsigned)P.nblocks, std::max(1, ngy), NC), dim3(WG), 0, s, sg, P.V, vec, N,
                       P.wc, P.d_cnt2, P.d_h, ldh, P.d_part, P.d_tick, std::max(1, ngy));
    norms(P.wc, P.d_n1);
    hipLaunchKernelGGL(k_seg_update, gb, dim3(WG), 0, s, sg, P.wc, P.V, vec, N, P.d_h, ldh, P.d_cnt2, -1.0, P.d_n2,
                       P.d_part, P.d_tick);
    // the Hessenberg step of every active column on the device: the column
    // is taken from this pass unless its norm fell below 1/sqrt(10) of
    // ||w|| (DGKS), which only flags a second pass
    std::vector<double> thrv(ncol, 0.0);
    for (int q = 0; q < ncol; ++q) thrv[q] = cols[q].thr;
    up_d(P.d_thr, thrv);
    hess_step_batched(P.d_hess, m, m, ncol, P.d_jv, P.d_cnt2, 0, P.d_h, nullptr, ldh, P.d_n1, P.d_n2, P.d_thr,
                      P.d_hout, s);
    HIPCHK(hipMemcpyAsync(hp, P.d_hout, (size_t)ncol * HESS_OUT * sizeof(double), hipMemcpyDeviceToHost, s));
    sync();
    std::vector<int32_t> re(ncol, 0);
    bool any_re = false;
    for (int q = 0; q < ncol; ++q)
      if (jv[q] >= 0 && hp[(size_t)q * HESS_OUT + 2] != 0.0) {
        re[q] = cnt2[q];
        any_re = true;
      }
    if (any_re) {
      up_i(P.d_cnt2, re);
      const int ngr = std::max(1, (*std::max_element(re.begin(), re.end()) + NL - 1) / NL);
      hipLaunchKernelGGL(k_seg_dots, dim3((unsigned)P.nblocks, ngr, NC), dim3(WG), 0, s, sg, P.V, vec, N, P.wc,
                         P.d_cnt2, P.d_h2, ldh, P.d_part, P.d_tick, ngr);
      hipLaunchKernelGGL(k_seg_update, gb, dim3(WG), 0, s, sg, P.wc, P.V, vec, N, P.d_h2, ldh, P.d_cnt2, -1.0, P.d_n2,
                         P.d_part, P.d_tick);
      hess_step_batched(P.d_hess, m, m, ncol, P.d_jv, P.d_cnt2, 1, P.d_h, P.d_h2, ldh, P.d_n1, P.d_n2, P.d_thr,
                        P.d_hout, s);
      HIPCHK(hipMemcpyAsync(hp, P.d_hout, (size_t)ncol * HESS_OUT * sizeof(double), hipMemcpyDeviceToHost, s));
      sync();
    }
    std::vector<int32_t> nj(ncol, -1);
    std::vector<double> ff(ncol, 0.0);
    bool any_end = false;
    for (int q = 0; q < ncol; ++q) {
      if (jv[q] < 0) continue;
      Col& C = cols[q];
      const int j = C.j;
      const int sys = q / NC;
      C.inf.inner_its_total += its[sys];
      C.inf.inner_its_max = std::max(C.inf.inner_its_max, its[sys]);
      if (re[q]) C.inf.reorth++;
      const double* ho = hp + (size_t)q * HESS_OUT;
      const double hnv = ho[1];
      C.gabs = ho[0];
      C.inf.outer_its++;
      C.implicit_ok = ho[3] != 0.0;
      C.j = j + 1;
      if (hnv != 0.0) {
        nj[q] = C.j;
        ff[q] = 1.0 / hnv;
      }
      if (C.implicit_ok || hnv == 0.0 || C.inf.outer_its >= o.max_outer || C.j == m) {
        C.end = true;
        any_end = true;
      }
    }
    up_i(P.d_cnt, nj);
    up_d(P.d_f, ff);
    hipLaunchKernelGGL(k_seg_move, gb, dim3(WG), 0, s, sg, P.V, P.wc, vec, P.d_cnt, P.d_f, 0);
    while (any_end) {
      end_cycles();
      any_end = false;
      for (auto& C : cols) any_end |= C.end;  // a restart from an exactly zero residual
    }
  }
  // solutions of the finished columns to the caller
  up_i(P.d_done, done);
  hipLaunchKernelGGL(k_store_x, gb, dim3(WG), 0, s, sg, P.d_X, P.d_nrhs, P.d_off, P.d_nsz, P.d_done, P.x);
  sync();
  const double dt = now_s() - t0;
  asss_status_t worst = ASSS_OK;
  for (int sidx = 0; sidx < ns; ++sidx)
    for (int c = 0; c < nrhs[sidx]; ++c) {
      Col& C = cols[sidx * NC + c];
      C.inf.solve_s = dt;
      C.inf.inner_kernel_s = kern_s;
      C.inf.inner_launches = launches;
      if (infos) infos[(int64_t)sidx * maxr + c] = C.inf;
      worst = std::max(worst, C.status);
    }
  return worst;
}

}  // namespace batch
}  // namespace asss

namespace asss {
namespace batch {

static bool fp32_of(asss_handle_t h, const asss_solve_opts_t& o) {
  return (o.inner_fp32 < 0) ? (h->opts.inner_fp32 != 0) : (o.inner_fp32 != 0);
}

bool applies(int32_t nsys, const asss_handle_t* hs, const int32_t* nrhs, const asss_solve_opts_t& o) {
  if (nsys < 1) return false;
  const bool fp32 = fp32_of(hs[0], o);
  for (int s = 0; s < nsys; ++s) {
    if (!eligible(hs[s], nrhs[s], o)) return false;
    if (hs[s]->device != hs[0]->device || fp32_of(hs[s], o) != fp32) return false;
  }
  return true;
}

asss_status_t run(int32_t nsys, const asss_handle_t* hs, const int32_t* nrhs, const double* const* B,
                  double* const* X, const asss_solve_opts_t& o, asss_info_t* infos, int maxr, hipStream_t s) {
  Range range("asss:batch engine");
  const bool fp32 = fp32_of(hs[0], o);
  const int m = std::max(1, o.restart_m);
  std::vector<asss_handle_t> list(hs, hs + nsys);
  std::vector<uint64_t> ids;
  for (auto h : list) ids.push_back(h->uid);
  std::lock_guard<std::mutex> lock(g_mu);
  Plan* plan = nullptr;
  for (auto& p : g_plans)
    if (p->ids == ids && p->fp32 == fp32 && p->m == m) plan = p.get();
  if (!plan) {
    // one kept plan per set of handles: a new precision or restart replaces it
    g_plans.erase(std::remove_if(g_plans.begin(), g_plans.end(), [&](const std::unique_ptr<Plan>& p) { return p->ids == ids; }),
                  g_plans.end());
    Range r2("asss:batch plan");
    plan = build_plan(list, fp32, m, s);
  }
  return solve(*plan, B, X, nrhs, o, infos, maxr, s);
}

void forget(asss_handle_t h) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_plans.erase(std::remove_if(g_plans.begin(), g_plans.end(),
                               [&](const std::unique_ptr<Plan>& p) {
                                 return std::find(p->ids.begin(), p->ids.end(), h->uid) != p->ids.end();
                               }),
                g_plans.end());
}

}  // namespace batch
}  // namespace asss
