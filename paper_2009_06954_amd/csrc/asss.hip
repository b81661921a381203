// libasss driver: handle, device part of the setup (least-squares solve for S,
// skew-Lanczos, one-time SMW data), the flexible GMRES outer iteration with
// the preconditioner P^-1 of eq. smw around the inner mrs, the adjoint solve,
// and the C ABI declared in include/asss.h.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <optional>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "../../include/asss.h"
#include "batch.hpp"
#include "handle.hpp"
#include "host_setup.hpp"
#include "ildl_kernels.hpp"
#include "ildl_setup.hpp"
#include "kernels.hpp"

using namespace asss;
using namespace asss::host;

// Workspace of asss_solve_noalloc: one fixed device array per GPU, held until
// the process ends, instead of Krylov workspace the handle would allocate.
// Host code never uses the array's name as a device address: the address of
// each device's copy comes from hipGetSymbolAddress (noalloc_scratch).
constexpr size_t kNoAllocBytes = (size_t)128 << 20;  // 128 MiB
static __device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];

namespace {

thread_local std::string g_err = "";

// layout of the small device/pinned scalar buffers (doubles)
// d_small layout: [0, 2048) Arnoldi scratch, 512 doubles per lockstep column
// (the Gram-Schmidt coefficients of the first pass and the new norm at +0,
// those of a second pass at +256; restart_m <= 250), SM_T the SMW
// coefficients.  h_small: the Hessenberg step's flags of column c at
// c * SM_COL, the inner state's head at SM_HSTATE, other read-backs at 0.
constexpr int SM_COL = 512, SM_PASS2 = 256, SM_T = 2048, SM_HSTATE = 3584, SM_SIZE = 4096;
static_assert(4 * SM_COL <= SM_T, "Arnoldi scratch of four columns");

}  // namespace

namespace asss {
namespace host {

// SpMV kernel shape: one row per thread when no row has more than 32 entries
// (grid stencils, the least-squares matrices of App. A), else the smallest
// power of two of lanes per row that covers the average row.
int lanes_for(const Csr& M) {
  int64_t longest = 0;
  for (int64_t i = 0; i < M.nrows; ++i) longest = std::max(longest, M.ptr[i + 1] - M.ptr[i]);
  if (longest <= 32) return 0;
  double avg = M.nrows ? (double)M.nnz() / (double)M.nrows : 1.0;
  int l = 1;
  while (l < avg && l < 64) l <<= 1;
  return l;
}

DCsr upload_csr(DevArena& ar, const Csr& M, hipStream_t s) {
  DCsr d;
  d.nrows = M.nrows;
  d.ncols = M.ncols;
  d.nnz = M.nnz();
  d.ptr = ar.upload(M.ptr, s);
  d.col = ar.upload(M.col, s);
  d.val = ar.upload(M.val, s);
  d.lanes = lanes_for(M);
  return d;
}

// Sliced ELL copy (layout described with DSell) of the device CSR matrix M,
// built on the device; none (nrows 0) when a row is longer than SELL_MAXW, M
// is empty or device memory runs out (what was allocated for it is released).
DSell ell_from_csr(DevArena& ar, const DCsr& M, hipStream_t s) {
  const int64_t n = M.nrows, ns = (n + 63) / 64;
  if (n == 0 || M.nnz == 0) return DSell{};
  std::vector<int32_t> w((size_t)ns);
  std::vector<int64_t> o((size_t)ns);
  int32_t* dw = nullptr;
  int64_t* dof = nullptr;
  int32_t* dc = nullptr;
  double* dv = nullptr;
  auto drop = [&]() {
    HIPCHK(hipStreamSynchronize(s));
    for (void* p : {(void*)dw, (void*)dof, (void*)dc, (void*)dv})
      if (p) ar.release(p);
  };
  int64_t total = 0;
  try {
    dw = ar.alloc<int32_t>(ns);
    ell_widths(n, M.ptr, dw, s);
    HIPCHK(hipMemcpyAsync(w.data(), dw, ns * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int64_t q = 0; q < ns; ++q) {
      if (w[q] > SELL_MAXW) {
        drop();
        return DSell{};
      }
      o[q] = total;
      total += 64 * (int64_t)w[q];
    }
    dof = ar.upload(o, s);
    dc = ar.alloc<int32_t>(total);
    dv = ar.alloc<double>(total);
    ell_fill(n, M.ptr, M.col, M.val, dw, dof, dc, dv, s);
  } catch (const Error& e) {
    if (e.code != ASSS_ERR_OOM) throw;
    drop();
    return DSell{};
  }
  HIPCHK(hipStreamSynchronize(s));  // o goes out of scope
  DSell d;
  d.nrows = n;
  d.entries = total;
  d.width = dw;
  d.off = dof;
  d.col = dc;
  d.val = dv;
  return d;
}

// y = rs o (M (cs o x)), through the sliced ELL copy E when there is one
void spmv_fast(const DCsr& M, const DSell& E, const double* x, double* y, const double* rs, const double* cs,
               hipStream_t s) {
  if (E.nrows > 0) spmv_sell(E, x, y, rs, cs, s);
  else spmv(M, x, y, rs, cs, 0, nullptr, s);
}

template <typename T>
DSkew<T> upload_sell(DevArena& ar, const SkewSell& S, hipStream_t s, const int32_t* aw,
                     const int32_t* bw, const int64_t* ao, const int64_t* bo, const uint16_t* ac,
                     const int32_t* bc, const uint16_t* bcd, const int32_t* bbase, const int32_t* adoff) {
  DSkew<T> d;
  d.n = S.n;
  d.R = S.R;
  d.nblocks = S.nblocks;
  d.nslices = S.nslices;
  d.a_width = aw;
  d.b_width = bw;
  d.a_off = ao;
  d.b_off = bo;
  d.a_col = ac;
  d.b_col = bc;
  d.b_cd = bcd;
  d.b_base = bbase;
  d.b_narrow = S.b_narrow ? 1 : 0;
  d.a_doff = adoff;
  d.form = S.form;
  std::vector<T> av(S.a_val.begin(), S.a_val.end()), bv(S.b_val.begin(), S.b_val.end());
  d.a_val = ar.upload(av, s);
  d.b_val = ar.upload(bv, s);
  return d;
}

// One sliced layout of J_tilde on the device, in both precisions (the index
// arrays are shared), with the list of its buffers so that it can be replaced.

// Workgroup size of the one-column inner step for nb row blocks: the
// caller's choice; else 512 in FP64 (1-2 % faster at 128^3 and 192^3), and in
// FP32 512 when nb blocks fill whole rounds of 2 resident workgroups per
// compute unit clearly better (by more than the ~4 % a 512-thread workgroup
// costs where both fill whole rounds) than of 4.
int pick_step_threads(int opt, int nb, bool fp32) {
  if (opt == 256 || opt == 512) return opt;
  if (!fp32) return 2 * WG;
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (cus <= 0 || nb <= 0) return WG;
  auto fill = [&](int slots) {
    const double r = (double)nb / slots;
    return r / std::ceil(r);
  };
  return fill(2 * cus) > fill(4 * cus) + 0.05 ? 2 * WG : WG;
}

SkewLayout upload_layout(DevArena& ar, const SkewSell& sell, hipStream_t s, int step_threads) {
  SkewLayout L;
  auto keep = [&](const void* p) { if (p) L.bufs.push_back(p); };
  const int32_t* aw = ar.upload(sell.a_width, s);
  const int32_t* bw = ar.upload(sell.b_width, s);
  const int64_t* ao = ar.upload(sell.a_off, s);
  const int64_t* bo = ar.upload(sell.b_off, s);
  // per-entry columns: part a 16-bit local; part b 16-bit deltas from per-slot
  // bases when every slot fits (2 bytes per entry instead of 4), else global
  // 32-bit columns.  Offset slots store no per-entry columns, only one offset
  // per slot (part a) and one base per slot (part b).
  const bool slots = sell.form == SKEW_SLOTS;
  const uint16_t* ac = slots ? nullptr : ar.upload(sell.a_col, s);
  const int32_t* bc = (sell.form == SKEW_WIDE) ? ar.upload(sell.b_col, s) : nullptr;
  const uint16_t* bcd = (sell.form == SKEW_NARROW) ? ar.upload(sell.b_cd, s) : nullptr;
  const int32_t* bbase = (sell.form != SKEW_WIDE) ? ar.upload(sell.b_base, s) : nullptr;
  const int32_t* adoff = slots ? ar.upload(sell.a_doff, s) : nullptr;
  for (const void* p : {(const void*)aw, (const void*)bw, (const void*)ao, (const void*)bo, (const void*)ac,
                        (const void*)bc, (const void*)bcd, (const void*)bbase, (const void*)adoff})
    keep(p);
  L.J64 = upload_sell<double>(ar, sell, s, aw, bw, ao, bo, ac, bc, bcd, bbase, adoff);
  L.J32 = upload_sell<float>(ar, sell, s, aw, bw, ao, bo, ac, bc, bcd, bbase, adoff);
  L.J64.threads = pick_step_threads(step_threads, L.J64.nblocks, false);
  L.J32.threads = pick_step_threads(step_threads, L.J32.nblocks, true);
  for (const void* p : {(const void*)L.J64.a_val, (const void*)L.J64.b_val, (const void*)L.J32.a_val,
                        (const void*)L.J32.b_val})
    keep(p);
  L.a_entries = sell.a_entries;
  L.b_entries = sell.b_entries;
  L.narrow = sell.b_narrow ? 1 : 0;
  L.form = sell.form;
  return L;
}

void release_layout(DevArena& ar, SkewLayout& L, hipStream_t s) {
  HIPCHK(hipStreamSynchronize(s));  // no kernel may still read it
  for (const void* p : L.bufs) ar.release(const_cast<void*>(p));
  L = SkewLayout{};
}

}  // namespace host
}  // namespace asss

namespace {

// ---------------------------------------------------------------------------
// small helpers on the handle
// ---------------------------------------------------------------------------

double dot_host(asss_handle_s* h, int64_t n, const double* a, const double* b, hipStream_t s) {
  gemm_tn<double, double>(n, 1, a, n, b, 1, h->d_small, nullptr, h->red, 2, s);
  HIPCHK(hipMemcpyAsync(h->h_small, h->d_small, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return h->h_small[0];
}

// w = Omega Abar S Omega z   (t1 scratch); with the incomplete LDL^T
// preconditioner w = Lcal^-1 A_hat Lcal^-T z in the factorization's positions
void outer_op(asss_handle_s* h, const double* z, double* w, hipStream_t s) {
  if (h->il.on) {
    auto& il = h->il;
    if (il.A_rows) dense_rows(h->n, il.A_rows, z, w, s);
    else ildl_sandwich<double>(il.Lb64, il.Ap, il.Lf64, z, w, il.t64[0], il.t64[1], il.t64[2], il.t64[3], s);
    return;
  }
  spmv_fast(h->dS, h->eS, z, h->t1, nullptr, h->d_om, s);
  spmv_fast(h->dAbar, h->eAbar, h->t1, w, h->d_om, nullptr, s);
}
// w = (Omega Abar S Omega)^T z = Omega S^T Abar^T Omega z
void outer_op_T(asss_handle_s* h, const double* z, double* w, hipStream_t s) {
  if (h->il.on) {
    auto& il = h->il;
    if (il.AT_rows) dense_rows(h->n, il.AT_rows, z, w, s);
    else ildl_sandwich<double>(il.Lb64, il.ApT, il.Lf64, z, w, il.t64[0], il.t64[1], il.t64[2], il.t64[3], s);
    return;
  }
  spmv_fast(h->dAbarT, h->eAbarT, z, h->t1, nullptr, h->d_om, s);
  spmv_fast(h->dSt, h->eSt, h->t1, w, h->d_om, nullptr, s);
}

// Right-hand side of the scaled system: b_chk = Omega P Dr b, or for the
// adjoint g_chk = Omega S^T Dc g; with the incomplete LDL^T, Lcal^-1 applied
// to (P Dr b)[perm] and to (S^T Dc g)[perm] (t1, tmp scratch).
void rhs_transform(asss_handle_s* h, bool adjoint, const double* b, double* bchk, hipStream_t s) {
  const int64_t n = h->n;
  if (h->il.on) {
    auto& il = h->il;
    if (!adjoint) {
      gather_scale(n, il.d_mp, il.d_drp, il.d_ones, b, h->tmp, s);
    } else {
      spmv(h->dSt, b, h->t1, nullptr, h->d_dc, 0, nullptr, s);
      permute_gather(n, il.d_perm, h->t1, h->tmp, s);
    }
    ildl_trsv(il.Lf64, h->tmp, bchk, il.t64[3], s);
    return;
  }
  if (!adjoint) gather_scale(n, h->d_m, h->d_drp, h->d_om, b, bchk, s);
  else spmv_fast(h->dSt, h->eSt, b, bchk, h->d_om, h->d_dc, s);  // g_chk = Omega S^T (Dc o g)
}

// Solution from the scaled one: x = Dc S Omega x_chk, or for the adjoint
// lambda = Dr P^T Omega l_chk; with the incomplete LDL^T the positions are
// mapped back after Lcal^-T (t1, tmp scratch).
void back_transform(asss_handle_s* h, bool adjoint, const double* xchk, double* x, hipStream_t s) {
  const int64_t n = h->n;
  if (h->il.on) {
    auto& il = h->il;
    ildl_trsv(il.Lb64, xchk, h->t1, il.t64[3], s);
    permute_scatter(n, il.d_perm, h->t1, h->tmp, s);
    if (!adjoint) spmv(h->dS, h->tmp, x, h->d_dc, nullptr, 0, nullptr, s);
    else scatter_scale(n, h->d_m, h->d_drp, il.d_ones, h->tmp, x, s);
    return;
  }
  if (!adjoint) spmv_fast(h->dS, h->eS, xchk, x, h->d_dc, h->d_om, s);
  else scatter_scale(n, h->d_m, h->d_drp, h->d_om, xchk, x, s);
}

// J_tilde v in FP64 (skew-Lanczos, operator export)
void jtilde_apply(asss_handle_s* h, const double* in, double* out, hipStream_t s) {
  if (h->il.on) {
    auto& il = h->il;
    ildl_sandwich<double>(il.Lb64, il.J64, il.Lf64, in, out, il.t64[0], il.t64[1], il.t64[2], il.t64[3], s);
  } else {
    skew_spmv<double>(h->J64, in, out, s);
  }
}

// ---------------------------------------------------------------------------
// inner mrs driver (single right-hand side, NR = 1)
// ---------------------------------------------------------------------------

template <typename T>
MrsLaunch make_launch(asss_handle_s* h, int nr, int sign, bool one_col) {
  MrsLaunch L{};
  L.n = h->n;
  L.nr = nr;
  L.k = h->k_eff;
  L.alpha_dev = h->d_alpha;
  L.sign = sign;
  // deflation = 3: the basis holds FP32 values, and the one-column FP64 step
  // reads the FP32 copy (the 4-column step reads the FP64 copy of the same values,
  // which it streams faster)
  L.q32 = (!std::is_same<T, float>::value && one_col && h->opts.deflation == 3 && h->k_eff > 0) ? 1 : 0;
  L.Qs = (std::is_same<T, float>::value || L.q32) ? (const void*)h->d_Qs32 : (const void*)h->d_Qs64;
  L.kq = h->k_eff;
  L.gram = std::is_same<T, float>::value ? h->d_G32 : h->d_G64;
  return L;
}

// Inner mrs solve of nc <= NR right-hand sides (columns of rhs / out with
// leading dimension n; NR = 4: App. B's simultaneous form, one matrix pass per
// step for all columns, shared stop rule), in three parts so that a caller can
// put more work on the stream before it waits: start() enqueues the start and
// a chunk of steps sized from the previous solve (steps after the end return
// at once) and copies the state's head to host scratch; settle(), after the
// caller's synchronization, reads it and returns true when the solve was done,
// else enqueues more steps (sized from the observed contraction rate) and a
// new copy; finish() enqueues the output.
template <typename T, int NR = 1>
struct MrsJob {
  asss_handle_s* h;
  const DSkew<T>* J;
  const T* Q;
  MrsBufs<T>* mb;
  double* out;
  int nc;
  double tol;
  int maxit, fixed;
  hipStream_t s;
  MrsLaunch L{};
  int its = 0, chunk = 0, prev_its = 0, polls = 0;
  double prev_rel = 1.0;

  // expect >= 0: the caller's estimate of the steps; the chunk then takes a
  // margin (a step launched after the end costs a few microseconds, a chunk
  // that falls short costs the caller a second round trip)
  void start(const double* rhs, int sign, int expect = -1) {
    L = make_launch<T>(h, nc, sign, NR == 1);
    if (J->nblocks <= 0) throw Error{ASSS_ERR_INTERNAL, "the sliced inner operator is not built for this handle"};
    if (J->nblocks > h->red.max_groups) throw Error{ASSS_ERR_INTERNAL, "more row blocks than reduction slots"};
    mrs_init<T, NR>(L, rhs, h->n, h->d_perm, Q, *mb, h->d_state, tol, maxit, fixed, h->red, s);
    if (fixed > 0) chunk = fixed + 1;
    else if (expect >= 0) chunk = std::max(4, expect + 5 + expect / 4);
    else chunk = std::max(4, h->last_inner + 1);
    launch_chunk();
  }
  void launch_chunk() {
    HIPCHK(hipEventRecord(h->ev0, s));
    for (int c = 0; c < chunk; ++c) mrs_iter<T, NR>(L, *J, Q, *mb, h->d_state, h->red, s);
    HIPCHK(hipEventRecord(h->ev1, s));
    HIPCHK(hipMemcpyAsync(h->h_small + SM_HSTATE, h->d_state, kStateHead, hipMemcpyDeviceToHost, s));
  }
  bool settle() {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    h->prof_s += 1e-3 * ms;
    h->prof_launches += chunk;
    const char* hs = (const char*)(h->h_small + SM_HSTATE);
    int32_t st_its, st_status;
    double rel;
    std::memcpy(&st_its, hs + offsetof(MrsState, its), 4);
    std::memcpy(&st_status, hs + offsetof(MrsState, status), 4);
    std::memcpy(&rel, hs + offsetof(MrsState, relres_max), 8);
    if (st_status == MRS_RUNNING && st_its <= its && polls > 0)
      throw Error{ASSS_ERR_INTERNAL, "inner mrs made no progress"};
    if (++polls > 100000) throw Error{ASSS_ERR_INTERNAL, "inner mrs did not finish"};
    its = st_its;
    if (st_status == MRS_DONE) {
      h->last_inner = its;
      return true;
    }
    if (st_status == MRS_CONVERGED) {
      chunk = 1;  // the final deferred update
    } else {
      // estimate the remaining steps from the observed contraction rate
      int est = 8;
      if (its > prev_its && rel > 0 && prev_rel > 0 && rel < prev_rel) {
        const double rate = std::log(rel / prev_rel) / (double)(its - prev_its);
        const double need = std::log(tol / rel) / rate;
        est = (int)std::ceil(need) + 1;
      }
      const int left = (fixed > 0 ? fixed : maxit) - its + 1;
      chunk = std::max(2, std::min({est, 64, left}));
      prev_rel = rel;
      prev_its = its;
    }
    launch_chunk();
    return false;
  }
  void finish() { mrs_output<T, NR>(h->n, nc, *mb, h->d_perm, out, h->n, s); }
};

template <typename T, int NR = 1>
int run_mrs(asss_handle_s* h, const DSkew<T>& J, const T* Q, MrsBufs<T>& mb,
            const double* rhs, double* out, int sign, double tol, int maxit, int fixed, hipStream_t s,
            int nc = 1) {
  Range range(NR == 1 ? "asss:inner mrs" : "asss:inner mrs (4 columns)");
  MrsJob<T, NR> job{h, &J, Q, &mb, out, nc, tol, maxit, fixed, s};
  job.start(rhs, sign);
  do {
    HIPCHK(hipStreamSynchronize(s));
  } while (!job.settle());
  job.finish();
  return job.its;
}

template <typename T>
int run_mrs1(asss_handle_s* h, const DSkew<T>& J, const T* Q, MrsBufs<T>& mb,
             const double* rhs, double* out, int sign, double tol, int maxit, int fixed, hipStream_t s) {
  return run_mrs<T, 1>(h, J, Q, mb, rhs, out, sign, tol, maxit, fixed, s);
}

// The inner solve with the incomplete LDL^T preconditioner: one launch of the
// persistent one-workgroup kernel (start, all steps, final update, output),
// its state's head copied to host scratch; ildl_settle reads it after the
// caller's synchronization.
template <typename T>
void ildl_launch(asss_handle_s* h, const double* rhs, double* out, int sign, double tol, int maxit, int fixed,
                 hipStream_t s) {
  auto& il = h->il;
  constexpr bool f32 = std::is_same<T, float>::value;
  IldlMrsArgs<T> a;
  a.n = (int32_t)h->n;
  a.k = h->k_eff;
  a.sign = sign;
  a.alpha = h->d_alpha;
  if constexpr (f32) {
    a.Q = h->d_Q32; a.gram = h->d_G32; a.Lb = il.Lb32; a.Lf = il.Lf32; a.J = il.J32;
    a.buf = h->mb32; a.y = il.y32; a.z = il.z32; a.u = il.u32; a.bs = il.t32[3];
  } else {
    a.Q = h->d_Q64; a.gram = h->d_G64; a.Lb = il.Lb64; a.Lf = il.Lf64; a.J = il.J64;
    a.buf = h->mb64; a.y = il.y64; a.z = il.z64; a.u = il.u64; a.bs = il.t64[3];
  }
  a.rhs = rhs;
  a.out = out;
  a.st = h->d_state;
  a.tol = tol;
  a.maxit = maxit;
  a.fixed = fixed;
  HIPCHK(hipEventRecord(h->ev0, s));
  ildl_mrs<T>(a, s);
  HIPCHK(hipEventRecord(h->ev1, s));
  HIPCHK(hipMemcpyAsync(h->h_small + SM_HSTATE, h->d_state, kStateHead, hipMemcpyDeviceToHost, s));
}

int ildl_settle(asss_handle_s* h) {
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  h->prof_s += 1e-3 * ms;
  h->prof_launches += 1;
  const char* hs = (const char*)(h->h_small + SM_HSTATE);
  int32_t st_its, st_status;
  std::memcpy(&st_its, hs + offsetof(MrsState, its), 4);
  std::memcpy(&st_status, hs + offsetof(MrsState, status), 4);
  if (st_status != MRS_DONE) throw Error{ASSS_ERR_INTERNAL, "inner mrs (incomplete LDL^T) did not finish"};
  h->last_inner = st_its;
  return st_its;
}

template <typename T>
int run_ildl_mrs(asss_handle_s* h, const double* rhs, double* out, int sign, double tol, int maxit, int fixed,
                 hipStream_t s) {
  Range range("asss:inner mrs (incomplete LDL^T)");
  ildl_launch<T>(h, rhs, out, sign, tol, maxit, fixed, s);
  HIPCHK(hipStreamSynchronize(s));
  return ildl_settle(h);
}

// The preconditioner's inner solve (sliced mrs in FP64 or FP32, or the
// incomplete LDL^T kernel, which finishes in its one launch) as a job in the
// three parts of MrsJob.
struct InnerJob {
  int mode = 0;  // 0 / 1: sliced FP64 / FP32; 2 / 3: incomplete LDL^T FP64 / FP32
  asss_handle_s* h = nullptr;
  MrsJob<double> d{};
  MrsJob<float> f{};
  int ildl_its = 0;

  void start(asss_handle_s* h_, bool fp32, const double* rhs, double* out, int sign, double tol, int maxit,
             int fixed, hipStream_t s, int expect = -1) {
    h = h_;
    if (h->il.on && !h->il.explicit_j) {
      mode = fp32 ? 3 : 2;
      if (fp32) ildl_launch<float>(h, rhs, out, sign, tol, maxit, fixed, s);
      else ildl_launch<double>(h, rhs, out, sign, tol, maxit, fixed, s);
    } else if (fp32) {
      mode = 1;
      f = MrsJob<float>{h, &h->J32, h->d_Q32, &h->mb32, out, 1, tol, maxit, fixed, s};
      f.start(rhs, sign, expect);
    } else {
      mode = 0;
      d = MrsJob<double>{h, &h->J64, h->d_Q64, &h->mb64, out, 1, tol, maxit, fixed, s};
      d.start(rhs, sign, expect);
    }
  }
  bool settle() {
    if (mode >= 2) {
      ildl_its = ildl_settle(h);
      return true;
    }
    return mode == 1 ? f.settle() : d.settle();
  }
  void finish() {
    if (mode == 1) f.finish();
    else if (mode == 0) d.finish();
  }
  int its() const { return mode >= 2 ? ildl_its : (mode == 1 ? f.its : d.its); }
};

int inner_solve(asss_handle_s* h, bool fp32, const double* rhs, double* out, int sign, double tol,
                int maxit, int fixed, hipStream_t s) {
  Range range(h->il.on && !h->il.explicit_j ? "asss:inner mrs (incomplete LDL^T)" : "asss:inner mrs");
  InnerJob job;
  job.start(h, fp32, rhs, out, sign, tol, maxit, fixed, s);
  do {
    HIPCHK(hipStreamSynchronize(s));
  } while (!job.settle());
  job.finish();
  return job.its();
}

// z <- z - X (C^-1 Sigma) (U_bar^T z): the low-rank part of eq. smw (inverse-free form)
void smw_correct(asss_handle_s* h, double* z, hipStream_t s) {
  if (h->kr > 0) {
    double* t = h->d_small + SM_T;
    gemm_tn<double, double>(h->n, h->kr, h->d_Ubar, h->n, z, 1, t, h->d_Mf, h->red, 3, s);
    gemv_acc(h->n, h->kr, h->d_X, h->n, t, -1.0, z, s);
  }
}

// z = P^-1 v (eq. smw in the inverse-free form)
int prec_apply(asss_handle_s* h, bool fp32, const double* v, double* z, const asss_solve_opts_t& o,
               hipStream_t s) {
  int its = inner_solve(h, fp32, v, z, +1, o.inner_tol, o.inner_maxit, o.fixed_inner_steps, s);
  smw_correct(h, z, s);
  return its;
}

// Buffers of the 4-column inner solve and of up to 4 lockstep outer columns.
void ensure_multi(asss_handle_s* h, int m, bool fp32) {
  const int64_t n = h->n;
  if (fp32 && !h->mb4_32.x) {
    for (int b = 0; b < 3; ++b) h->mb4_32.w[b] = h->ar.alloc<float>(n * NRMAX);
    for (int b = 0; b < 2; ++b) h->mb4_32.p[b] = h->ar.alloc<float>(n * NRMAX);
    h->mb4_32.x = h->ar.alloc<float>(n * NRMAX);
  }
  if (!fp32 && !h->mb4_64.x) {
    for (int b = 0; b < 3; ++b) h->mb4_64.w[b] = h->ar.alloc<double>(n * NRMAX);
    for (int b = 0; b < 2; ++b) h->mb4_64.p[b] = h->ar.alloc<double>(n * NRMAX);
    h->mb4_64.x = h->ar.alloc<double>(n * NRMAX);
  }
  if (!h->pin) {
    h->pin = h->ar.alloc<double>(n * NRMAX);
    h->pout = h->ar.alloc<double>(n * NRMAX);
    for (int c = 0; c < NRMAX; ++c) {
      h->mcol[c].bchk = h->ar.alloc<double>(n);
      h->mcol[c].xchk = h->ar.alloc<double>(n);
      h->mcol[c].rv = h->ar.alloc<double>(n);
    }
  }
  if (h->m_alloc_multi < m) {
    for (int c = 0; c < NRMAX; ++c) {
      if (h->mcol[c].V) { h->ar.release(h->mcol[c].V); h->ar.release(h->mcol[c].Z); }
      h->mcol[c].V = h->ar.alloc<double>(n * (int64_t)(m + 1));
      h->mcol[c].Z = h->ar.alloc<double>(n * (int64_t)m);
    }
    h->m_alloc_multi = m;
  }
}

// The low-rank part of z = P^-T v = S_bar^-T (v - U_bar Sigma^T C^-T X^T v),
// ahead of the inner solve: returns the inner system's right-hand side.
const double* prec_pre_T(asss_handle_s* h, const double* v, hipStream_t s) {
  if (h->kr == 0) return v;
  double* t = h->d_small + SM_T;
  gemm_tn<double, double>(h->n, h->kr, h->d_X, h->n, v, 1, t, h->d_Ma, h->red, 3, s);
  axpby(h->n, 1.0, v, 0.0, h->tmp, s);
  gemv_acc(h->n, h->kr, h->d_Ubar, h->n, t, -1.0, h->tmp, s);
  return h->tmp;
}

int prec_apply_T(asss_handle_s* h, bool fp32, const double* v, double* z, const asss_solve_opts_t& o,
                 hipStream_t s) {
  return inner_solve(h, fp32, prec_pre_T(h, v, s), z, -1, o.inner_tol, o.inner_maxit, o.fixed_inner_steps, s);
}

// ---------------------------------------------------------------------------
// row-block autotuner
// ---------------------------------------------------------------------------

// Average duration of one fused inner step (k_mrs_iter, the handle's
// deflation, one column) on layout J, timed with HIP events over a fixed
// number of steps from the right-hand side in h->tmp.  Leaves no trace in
// the handle's counters.
template <typename T>
double time_inner_step(asss_handle_s* h, const DSkew<T>& J, const T* Q, MrsBufs<T>& mb,
                       int steps, hipStream_t s) {
  const double ps = h->prof_s;
  const int pl = h->prof_launches, li = h->last_inner;
  h->prof_s = 0.0;
  h->prof_launches = 0;
  run_mrs1<T>(h, J, Q, mb, h->tmp, h->w, +1, 1e-300, steps, steps, s);
  const double t = h->prof_launches > 0 ? h->prof_s / h->prof_launches : 0.0;
  h->prof_s = ps;
  h->prof_launches = pl;
  h->last_inner = li;
  return t;
}

double time_layout(asss_handle_s* h, const SkewLayout& L, bool fp32, hipStream_t s) {
  auto run = [&](int steps) {
    return fp32 ? time_inner_step<float>(h, L.J32, h->d_Q32, h->mb32, steps, s)
                : time_inner_step<double>(h, L.J64, h->d_Q64, h->mb64, steps, s);
  };
  const double warm = run(4);
  // about 4 ms of timed steps per repeat, best of two repeats
  const int steps = (int)std::min(256.0, std::max(8.0, 4e-3 / std::max(warm, 1e-7)));
  return std::min(run(steps), run(steps));
}

// Packs the sliced layout of J_tilde (strict upper part Jup, in the order of
// the inner system) for every candidate row-block size, times the inner step on each in the
// handle's default inner precision and keeps the fastest in the handle.  All
// layouts hold the same operator, so the deflation and SMW data stay valid.
void tune_row_block(asss_handle_s* h, const Csr& Jup, const std::vector<int>& cands, hipStream_t s) {
  const int64_t n = h->n;
  {  // a fixed pseudo-random right-hand side in (-1, 1)
    std::vector<double> r(n);
    uint64_t x = 0x9e3779b97f4a7c15ull;
    for (int64_t i = 0; i < n; ++i) {
      x ^= x << 13; x ^= x >> 7; x ^= x << 17;  // xorshift64
      r[i] = (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
    HIPCHK(hipMemcpyAsync(h->tmp, r.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  const bool fp32 = h->opts.inner_fp32 != 0;
  SkewLayout best;
  best.J64 = h->J64;
  best.J32 = h->J32;
  best.bufs = h->lay_bufs;
  best.a_entries = h->sell_a;
  best.b_entries = h->sell_b;
  best.narrow = h->narrow_b;
  best.form = h->skew_form;
  double t_best = time_layout(h, best, fp32, s);
  h->tuned.assign(1, {h->J64.R, 1e6 * t_best});
  for (int R : cands) {
    if (R == best.J64.R) continue;
    SkewSell sell;
    try {
      sell = pack_skew_sell(Jup, R, h->opts.skew_form);
    } catch (const HostError&) {
      continue;  // a forced column form that does not fit this row-block size
    }
    SkewLayout cand = upload_layout(h->ar, sell, s, h->opts.step_threads);
    HIPCHK(hipStreamSynchronize(s));
    const double t = time_layout(h, cand, fp32, s);
    h->tuned.push_back({R, 1e6 * t});
    if (t < t_best) {
      release_layout(h->ar, best, s);
      best = std::move(cand);
      t_best = t;
    } else {
      release_layout(h->ar, cand, s);
    }
  }
  std::sort(h->tuned.begin(), h->tuned.end());
  h->J64 = best.J64;
  h->J32 = best.J32;
  h->lay_bufs = best.bufs;
  h->sell_a = best.a_entries;
  h->sell_b = best.b_entries;
  h->narrow_b = best.narrow;
  h->skew_form = best.form;
  h->cross_natural = count_cross_pairs(h->U, h->J64.R);
  h->cross_used = count_cross_pairs(Jup, h->J64.R);
}

// ---------------------------------------------------------------------------
// setup: least squares for S on the device (LSQR, Paige & Saunders 1982)
// ---------------------------------------------------------------------------

std::vector<double> lsqr_device(asss_handle_s* h, const LlsSystem& L, double tol, int maxit,
                                hipStream_t s) {
  DevArena tmp(h->ar.al);
  const int64_t m = L.B.nrows, nu = L.B.ncols;
  DCsr B = upload_csr(tmp, L.B, s), Bt = upload_csr(tmp, L.Bt, s);
  const DSell eB = ell_from_csr(tmp, B, s), eBt = ell_from_csr(tmp, Bt, s);
  // The bidiagonalization vectors are kept unnormalized: u holds beta u_i and
  // v holds alpha v_i, and each 1/beta, 1/alpha rides on the next product or
  // update instead of a pass of its own.
  double* u = tmp.upload(L.rhs, s);
  double* v = tmp.alloc<double>(nu);
  double* w = tmp.alloc<double>(nu);
  double* x = tmp.alloc<double>(nu);
  double* y = tmp.alloc<double>(std::max(m, nu));
  double* part = tmp.alloc<double>((std::max(m, nu) + 255) / 256 + 256);
  HIPCHK(hipMemsetAsync(x, 0, nu * sizeof(double), s));
  auto nrm = [&](int64_t len, const double* a) { return std::sqrt(dot_host(h, len, a, a, s)); };
  // io = sa (M in) + sb io; returns ||io|| (from the product's epilogue when
  // it reads the sliced copy)
  auto prod = [&](const DCsr& M, const DSell& E, const double* in, double* io, double sa, double sb) {
    if (E.nrows > 0) {
      spmv_sell_acc(E, in, io, sa, sb, part, s);
      sum_parts((E.nrows + 255) / 256, part, h->d_small, s);
      HIPCHK(hipMemcpyAsync(h->h_small, h->d_small, sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      return std::sqrt(h->h_small[0]);
    }
    spmv(M, in, y, nullptr, nullptr, 0, nullptr, s);
    axpby(M.nrows, sa, y, sb, io, s);
    return nrm(M.nrows, io);
  };
  double beta = nrm(m, u);
  const double bnorm = beta;
  std::vector<double> out(nu, 0.0);
  if (beta == 0.0) return out;
  double alpha = prod(Bt, eBt, u, v, 1.0 / beta, 0.0);  // alpha_1 v_1 = B^T u_1
  if (alpha == 0.0) return out;
  axpby(nu, 1.0 / alpha, v, 0.0, w, s);  // w_1 = v_1
  double phibar = beta, rhobar = alpha, anorm2 = 0.0;
  int it = 0;
  double test1 = 1.0, test2 = 1.0;
  for (it = 1; it <= maxit; ++it) {
    beta = prod(B, eB, v, u, 1.0 / alpha, -alpha / beta);  // beta_{i+1} u_{i+1} = B v_i - alpha_i u_i
    anorm2 += alpha * alpha + beta * beta;
    if (beta > 0) {
      alpha = prod(Bt, eBt, u, v, 1.0 / beta, -beta / alpha);  // alpha_{i+1} v_{i+1} = B^T u_{i+1} - beta_{i+1} v_i
    } else {
      alpha = 0.0;  // u_{i+1} = 0: the next v is zero and the iteration ends below
    }
    const double rho = std::hypot(rhobar, beta);
    const double c = rhobar / rho, sn = beta / rho;
    const double theta = sn * alpha;
    rhobar = -c * alpha;
    const double phi = c * phibar;
    phibar = sn * phibar;
    axpby(nu, phi / rho, w, 1.0, x, s);
    if (alpha > 0) axpby(nu, 1.0 / alpha, v, -theta / rho, w, s);  // w = v_{i+1} - (theta / rho) w
    const double anorm = std::sqrt(anorm2);
    const double rnorm = phibar;
    const double arnorm = phibar * alpha * std::fabs(c);
    test1 = rnorm / bnorm;
    test2 = (anorm > 0 && rnorm > 0) ? arnorm / (anorm * rnorm) : 0.0;
    if (test1 <= tol || test2 <= std::max(tol, 1.1e-16) || alpha == 0.0) break;
  }
  h->lls_its = std::min(it, maxit);
  h->lls_relres = test1;
  h->lls_kkt = test2;
  HIPCHK(hipMemcpyAsync(out.data(), x, nu * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (double vv : out)
    if (!std::isfinite(vv)) throw Error{ASSS_ERR_LLS, "least-squares solution is not finite"};
  return out;
}

// LU with partial pivoting of a small dense matrix (row-major), and solves.
struct SmallLU {
  int n = 0;
  std::vector<double> a;
  std::vector<int> piv;
  void factor(const std::vector<double>& m, int nn) {
    n = nn;
    a = m;
    piv.resize(n);
    for (int k = 0; k < n; ++k) {
      int p = k;
      for (int i = k + 1; i < n; ++i)
        if (std::fabs(a[i * n + k]) > std::fabs(a[p * n + k])) p = i;
      piv[k] = p;
      if (p != k)
        for (int j = 0; j < n; ++j) std::swap(a[k * n + j], a[p * n + j]);
      if (a[k * n + k] == 0.0) throw Error{ASSS_ERR_INTERNAL, "SMW matrix C is singular"};
      for (int i = k + 1; i < n; ++i) {
        a[i * n + k] /= a[k * n + k];
        for (int j = k + 1; j < n; ++j) a[i * n + j] -= a[i * n + k] * a[k * n + j];
      }
    }
  }
  // solve C x = b (trans = false) or C^T x = b (trans = true)
  std::vector<double> solve(std::vector<double> b, bool trans) const {
    if (!trans) {
      for (int k = 0; k < n; ++k) std::swap(b[k], b[piv[k]]);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) b[i] -= a[i * n + j] * b[j];
      for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) b[i] -= a[i * n + j] * b[j];
        b[i] /= a[i * n + i];
      }
    } else {
      for (int i = 0; i < n; ++i) {
        for (int j = 0; j < i; ++j) b[i] -= a[j * n + i] * b[j];
        b[i] /= a[i * n + i];
      }
      for (int i = n - 1; i >= 0; --i)
        for (int j = i + 1; j < n; ++j) b[i] -= a[j * n + i] * b[j];
      for (int k = n - 1; k >= 0; --k) std::swap(b[k], b[piv[k]]);
    }
    return b;
  }
};

void device_setup(asss_handle_s* h, hipStream_t s) {
  const int64_t n = h->n;
  const int k = h->opts.k;
  // ---- skew-Lanczos (Fig. 2) in FP64
  std::vector<double> alpha;
  int keff = 0;
  if (k > 0 && h->q_given.size() == (size_t)n * k) {  // the caller's basis (original order)
    h->d_Q64 = h->ar.alloc<double>(n * (int64_t)k);
    double* z = h->ar.alloc<double>(n * (int64_t)k);
    HIPCHK(hipMemcpyAsync(z, h->q_given.data(), (size_t)n * k * sizeof(double), hipMemcpyHostToDevice, s));
    for (int c = 0; c < k; ++c) {
      if (h->d_perm)
        permute_gather(n, h->d_perm, z + (int64_t)c * n, h->d_Q64 + (int64_t)c * n, s);
      else
        HIPCHK(hipMemcpyAsync(h->d_Q64 + (int64_t)c * n, z + (int64_t)c * n, n * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    h->ar.release(z);
    std::vector<double>().swap(h->q_given);
    alpha = h->alpha_given;
    keff = k;
  } else if (k > 0) {
    h->d_Q64 = h->ar.alloc<double>(n * (int64_t)k);
    double* z = h->ar.alloc<double>(n);
    double* q0 = h->d_Q64;
    if (h->d_perm) {  // the start vector is defined in the original order
      splitmix_vector(n, h->opts.lanczos_seed, z, s);
      permute_gather(n, h->d_perm, z, q0, s);
    } else {
      splitmix_vector(n, h->opts.lanczos_seed, q0, s);
    }
    double nq = std::sqrt(dot_host(h, n, q0, q0, s));
    scale(n, 1.0 / nq, q0, q0, s);
    keff = 1;
    if (k >= 2) {
      jtilde_apply(h, q0, z, s);
      double a1 = std::sqrt(dot_host(h, n, z, z, s));
      if (a1 != 0.0) {
        alpha.push_back(a1);
        scale(n, -1.0 / a1, z, h->d_Q64 + n, s);
        keff = 2;
        for (int i = 2; i < k; ++i) {
          jtilde_apply(h, h->d_Q64 + (int64_t)(i - 1) * n, z, s);
          axpby(n, -alpha[i - 2], h->d_Q64 + (int64_t)(i - 2) * n, 1.0, z, s);
          double ai = std::sqrt(dot_host(h, n, z, z, s));
          if (ai <= 1e-14 * a1) break;
          alpha.push_back(ai);
          scale(n, -1.0 / ai, z, h->d_Q64 + (int64_t)i * n, s);
          keff = i + 1;
        }
      }
    }
    h->ar.release(z);
  }
  h->k_eff = keff;
  h->alpha = alpha;
  if (keff > 0) {
    h->d_Q32 = h->ar.alloc<float>(n * (int64_t)keff);
    cast_d2f(n * (int64_t)keff, h->d_Q64, h->d_Q32, s);
    // deflation = 3: Q_k rounded to FP32 values and used so everywhere (the
    // deflated operator, U_bar, X, G): eq. smw gives back the same P for any
    // basis used consistently, and the FP64 inner step reads half the bytes
    if (h->opts.deflation == 3) cast_f2d(n * (int64_t)keff, h->d_Q32, h->d_Q64, s);
  }
  if (keff > 0 && h->d_perm) {
    h->d_Qorig = h->ar.alloc<double>(n * (int64_t)keff);
    for (int c = 0; c < keff; ++c)
      permute_scatter(n, h->d_perm, h->d_Q64 + (int64_t)c * n, h->d_Qorig + (int64_t)c * n, s);
  } else {
    h->d_Qorig = h->d_Q64;
  }
  h->d_alpha = h->ar.upload(alpha.empty() ? std::vector<double>{0.0} : alpha, s);
  if (keff > 0) {
    const int64_t npad = ((n + 63) / 64) * 64;
    h->d_Qs64 = h->ar.alloc<double>(npad * keff);
    h->d_Qs32 = h->ar.alloc<float>(npad * keff);
    slice_columns<double>(n, keff, h->d_Q64, h->d_Qs64, s);
    slice_columns<float>(n, keff, h->d_Q32, h->d_Qs32, s);
    // Gram matrices G = Q_k^T Q_k of both stored copies (column c of G at
    // G + c k; G is symmetric bit for bit, the products and their order being
    // the same); the FP64 one's distance from I is reported
    h->d_G64 = h->ar.alloc<double>((int64_t)keff * keff);
    h->d_G32 = h->ar.alloc<double>((int64_t)keff * keff);
    for (int c = 0; c < keff; ++c) {
      gemm_tn<double, double>(n, keff, h->d_Q64, n, h->d_Q64 + (int64_t)c * n, 1, h->d_G64 + (int64_t)c * keff,
                              nullptr, h->red, 2, s);
      gemm_tn<float, float>(n, keff, h->d_Q32, n, h->d_Q32 + (int64_t)c * n, 1, h->d_G32 + (int64_t)c * keff,
                            nullptr, h->red, 2, s);
    }
    std::vector<double> g64((size_t)keff * keff);
    HIPCHK(hipMemcpyAsync(g64.data(), h->d_G64, g64.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double err = 0.0;
    for (int c = 0; c < keff; ++c)
      for (int l = 0; l < keff; ++l) err = std::max(err, std::fabs(g64[(size_t)c * keff + l] - (l == c ? 1.0 : 0.0)));
    h->orth_err = err;
  }
  // ---- one-time SMW data (Sec. 4.1): U_bar, X = S_bar^-1 U_bar, G, C
  // U_r: unit vectors at the negative entries of D (diagonal reading), or the
  // columns of the low-rank term of the scaled incomplete factor (Fig. 1)
  h->r = h->il.on ? (int)h->il.Sc.sigma.size() : (int)h->neg.size();
  const int kr = keff + h->r;
  if (kr > 512) throw Error{ASSS_ERR_INTERNAL, "rank of the low-rank term k + r exceeds 512"};
  h->kr = kr;
  if (kr == 0) return;
  h->d_Ubar = h->ar.alloc<double>(n * (int64_t)kr);
  HIPCHK(hipMemsetAsync(h->d_Ubar, 0, n * (int64_t)kr * sizeof(double), s));
  if (keff > 0)
    HIPCHK(hipMemcpyAsync(h->d_Ubar, h->d_Qorig, n * (int64_t)keff * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (h->il.on) {
    const auto& Sc = h->il.Sc;
    for (int j = 0; j < h->r; ++j)
      for (int t = 0; t < 2; ++t)
        if (Sc.ur_pos[2 * j + t] >= 0)
          HIPCHK(hipMemcpyAsync(h->d_Ubar + (int64_t)(keff + j) * n + Sc.ur_pos[2 * j + t], &Sc.ur_val[2 * j + t],
                                sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  } else {
    std::vector<double> one(1, 1.0);
    for (int j = 0; j < h->r; ++j)
      HIPCHK(hipMemcpyAsync(h->d_Ubar + (int64_t)(keff + j) * n + h->neg[j], one.data(), sizeof(double),
                            hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  h->d_X = h->ar.alloc<double>(n * (int64_t)kr);
  if (h->il.on && !h->il.explicit_j) {  // X = S_bar^-1 U_bar column by column (one-workgroup inner solves)
    int xits = 0;
    for (int c = 0; c < kr; ++c)
      xits = std::max(xits, run_ildl_mrs<double>(h, h->d_Ubar + (int64_t)c * n, h->d_X + (int64_t)c * n, +1,
                                                 h->opts.x_tol, h->opts.x_maxit, 0, s));
    h->x_its = xits;
  } else {  // simultaneous mrs (App. B) on groups of NRMAX columns in FP64
    DevArena tmp(h->ar.al);
    MrsBufs<double> mb4;
    for (int b = 0; b < 3; ++b) mb4.w[b] = tmp.alloc<double>(n * NRMAX);
    for (int b = 0; b < 2; ++b) mb4.p[b] = tmp.alloc<double>(n * NRMAX);
    mb4.x = tmp.alloc<double>(n * NRMAX);
    const bool use4 = keff <= 16 && !h->J64.dense;  // the 4-column step has no explicit form
    int xits = 0;
    for (int c0 = 0; c0 < kr; c0 += (use4 ? NRMAX : 1)) {
      const int nc = use4 ? std::min(NRMAX, kr - c0) : 1;
      if (use4) {
        MrsLaunch L = make_launch<double>(h, nc, +1, false);
        mrs_init<double, NRMAX>(L, h->d_Ubar + (int64_t)c0 * n, n, h->d_perm, h->d_Q64, mb4, h->d_state,
                                h->opts.x_tol, h->opts.x_maxit, 0, h->red, s);
        int group_its = -1;
        for (int guard = 0; guard < 1000000; ++guard) {
          for (int c = 0; c < 16; ++c) mrs_iter<double, NRMAX>(L, h->J64, h->d_Q64, mb4, h->d_state, h->red, s);
          HIPCHK(hipMemcpyAsync(h->h_small, h->d_state, kStateHead, hipMemcpyDeviceToHost, s));
          HIPCHK(hipStreamSynchronize(s));
          int32_t st_its, st_status;
          std::memcpy(&st_its, (char*)h->h_small + offsetof(MrsState, its), 4);
          std::memcpy(&st_status, (char*)h->h_small + offsetof(MrsState, status), 4);
          if (st_status == MRS_RUNNING && st_its <= group_its)
            throw Error{ASSS_ERR_INTERNAL, "setup mrs made no progress"};
          group_its = st_its;
          xits = std::max(xits, (int)st_its);
          if (st_status == MRS_DONE) break;
          if (st_status == MRS_CONVERGED) {
            mrs_iter<double, NRMAX>(L, h->J64, h->d_Q64, mb4, h->d_state, h->red, s);
            break;
          }
        }
        mrs_output<double, NRMAX>(n, nc, mb4, h->d_perm, h->d_X + (int64_t)c0 * n, n, s);
      } else {
        int it = run_mrs1<double>(h, h->J64, h->d_Q64, h->mb64, h->d_Ubar + (int64_t)c0 * n,
                                  h->d_X + (int64_t)c0 * n, +1, h->opts.x_tol, h->opts.x_maxit, 0, s);
        xits = std::max(xits, it);
      }
    }
    HIPCHK(hipStreamSynchronize(s));
    h->x_its = xits;
  }
  // G = U_bar^T X (kr x kr), C = I + Sigma G
  std::vector<double> G((size_t)kr * kr);
  for (int c = 0; c < kr; ++c) {
    gemm_tn<double, double>(n, kr, h->d_Ubar, n, h->d_X + (int64_t)c * n, 1, h->d_small, nullptr, h->red, 2, s);
    HIPCHK(hipMemcpyAsync(h->h_small, h->d_small, kr * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int l = 0; l < kr; ++l) G[(size_t)l * kr + c] = h->h_small[l];
  }
  std::vector<double> Sig((size_t)kr * kr, 0.0);
  for (int i = 0; i + 1 < keff; ++i) {
    Sig[(size_t)i * kr + i + 1] = alpha[i];
    Sig[(size_t)(i + 1) * kr + i] = -alpha[i];
  }
  for (int j = 0; j < h->r; ++j)
    Sig[(size_t)(keff + j) * kr + keff + j] = h->il.on ? h->il.Sc.sigma[j] : -2.0;
  std::vector<double> C((size_t)kr * kr, 0.0);
  for (int i = 0; i < kr; ++i)
    for (int j = 0; j < kr; ++j) {
      double acc = (i == j) ? 1.0 : 0.0;
      for (int l = 0; l < kr; ++l) acc += Sig[(size_t)i * kr + l] * G[(size_t)l * kr + j];
      C[(size_t)i * kr + j] = acc;
    }
  SmallLU lu;
  lu.factor(C, kr);
  // Mf = C^-1 Sigma (columns: C^-1 Sigma e_j), Ma = Sigma^T C^-T
  std::vector<double> Mf((size_t)kr * kr), CinvT((size_t)kr * kr), Ma((size_t)kr * kr);
  for (int j = 0; j < kr; ++j) {
    std::vector<double> col(kr), e(kr, 0.0);
    for (int i = 0; i < kr; ++i) col[i] = Sig[(size_t)i * kr + j];
    col = lu.solve(col, false);
    for (int i = 0; i < kr; ++i) Mf[(size_t)i * kr + j] = col[i];
    e[j] = 1.0;
    e = lu.solve(e, true);  // column j of C^-T
    for (int i = 0; i < kr; ++i) CinvT[(size_t)i * kr + j] = e[i];
  }
  for (int i = 0; i < kr; ++i)
    for (int j = 0; j < kr; ++j) {
      double acc = 0.0;
      for (int l = 0; l < kr; ++l) acc += Sig[(size_t)l * kr + i] * CinvT[(size_t)l * kr + j];
      Ma[(size_t)i * kr + j] = acc;
    }
  h->d_Mf = h->ar.upload(Mf, s);
  h->d_Ma = h->ar.upload(Ma, s);
  HIPCHK(hipStreamSynchronize(s));
}

void ensure_outer(asss_handle_s* h, int m) {
  if (h->m_alloc >= m) return;
  if (h->no_alloc) throw Error{ASSS_ERR_INTERNAL, "the fixed workspace is smaller than the solve needs"};
  if (h->V) { h->ar.release(h->V); h->ar.release(h->Z); }
  h->V = h->ar.alloc<double>(h->n * (int64_t)(m + 1));
  h->Z = h->ar.alloc<double>(h->n * (int64_t)m);
  h->m_alloc = m;
}

// [a, a + la) and [b, b + lb) share an element
bool overlaps(const double* a, int64_t la, const double* b, int64_t lb) {
  const uintptr_t a0 = (uintptr_t)a, a1 = a0 + (uintptr_t)la * sizeof(double);
  const uintptr_t b0 = (uintptr_t)b, b1 = b0 + (uintptr_t)lb * sizeof(double);
  return a0 < b1 && b0 < a1;
}

bool b_is_finite(asss_handle_s* h, const double* b, hipStream_t s) {
  HIPCHK(hipMemsetAsync(h->d_flag, 0, sizeof(int), s));
  check_finite(h->n, b, h->d_flag, s);
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, h->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return flag == 0;
}

// One column of flexible GMRES(m) on the scaled system, with the stopping rule
// of the oracle, as a state machine: step() runs one outer step of a single
// column; lockstep columns instead apply the preconditioner to v_next() into
// z_next() together, then each calls count_inner() and arnoldi_enqueue(),
// and after one shared wait arnoldi_finish().  A column restarts and finishes
// by itself.  The Hessenberg matrix, its Givens rotations, the
// residual estimate and the stopping test live on the device (outer.hip, one
// workspace per column); the host reads back a few flags per Arnoldi step.
struct FgmresCol {
  asss_handle_s* h = nullptr;
  bool adjoint = false;
  const double* b = nullptr;
  double* x = nullptr;
  asss_solve_opts_t o{};
  hipStream_t s = nullptr;
  int64_t n = 0;
  int m = 1;
  double *V = nullptr, *Z = nullptr, *bchk = nullptr, *xchk = nullptr, *rv = nullptr;
  double* W = nullptr;        // Hessenberg workspace (device)
  double bn = 0.0, bcn = 0.0, thr = 0.0, t0 = 0.0;
  double gabs = 0.0;          // |g_j|, the residual estimate after the last step
  int slot = 0;  // Arnoldi scratch: d_small + slot * SM_COL; flags: h_small + slot * SM_COL
  int last_its = 0;
  int recent[4] = {0, 0, 0, 0};  // inner steps of the last four outer steps
  int nrecent = 0;
  int j = 0;
  bool first = true, done = false, implicit_ok = false;
  asss_info_t inf{};
  asss_status_t status = ASSS_NOT_CONVERGED;

  void op(const double* in, double* out) {
    if (!adjoint) outer_op(h, in, out, s);
    else outer_op_T(h, in, out, s);
  }
  const double* v_next() const { return V + (int64_t)j * n; }
  double* z_next() { return Z + (int64_t)j * n; }
  const double* flags() const { return h->h_small + slot * SM_COL; }

  void begin(asss_handle_s* h_, bool adj, const double* b_, double* x_, const asss_solve_opts_t& o_,
             double* V_, double* Z_, double* bchk_, double* xchk_, double* rv_, hipStream_t s_) {
    h = h_; adjoint = adj; b = b_; x = x_; o = o_; s = s_;
    V = V_; Z = Z_; bchk = bchk_; xchk = xchk_; rv = rv_;
    W = h->d_hess + (int64_t)slot * HESS_SLOT;
    t0 = now_s();
    n = h->n;
    m = std::max(1, o.restart_m);
    if (m > HESS_MMAX) throw Error{ASSS_ERR_INVALID_ARG, "restart_m above 250"};
    inf = asss_info_t{};
    inf.k_eff = h->k_eff;
    inf.rank_r = h->r;
    inf.setup_host_s = h->setup_host_s;
    inf.setup_device_s = h->setup_device_s;
    bn = std::sqrt(dot_host(h, n, b, b, s));
    if (bn == 0.0) {
      HIPCHK(hipMemsetAsync(x, 0, n * sizeof(double), s));
      inf.converged = 1;
      status = ASSS_OK;
      done = true;
      return;
    }
    rhs_transform(h, adjoint, b, bchk, s);
    bcn = std::sqrt(dot_host(h, n, bchk, bchk, s));
    thr = o.tol * bcn;
    HIPCHK(hipMemsetAsync(xchk, 0, n * sizeof(double), s));
    first = true;
    start_cycle();
  }

  void start_cycle() {
    if (first) {
      axpby(n, 1.0, bchk, 0.0, rv, s);
    } else {
      op(xchk, h->w);
      axpby(n, 1.0, bchk, 0.0, rv, s);
      axpby(n, -1.0, h->w, 1.0, rv, s);
    }
    first = false;
    const double beta = std::sqrt(dot_host(h, n, rv, rv, s));
    inf.cycles++;
    j = 0;
    gabs = beta;
    implicit_ok = beta <= thr;
    if (beta > 0) {
      hess_reset(W, beta, s);
      scale(n, 1.0 / beta, rv, V, s);
    } else {
      end_cycle();
    }
  }

  void count_inner(int its) {
    recent[nrecent++ & 3] = its;
    last_its = its;
    inf.inner_its_total += its;
    inf.inner_its_max = std::max(inf.inner_its_max, its);
  }

  // Arnoldi step j after the preconditioner application z_j, in two halves so
  // that lockstep columns share one host round trip: arnoldi_enqueue puts
  // w = A_chk z_j (straight into V[:, j+1]), the classical Gram-Schmidt
  // coefficients V^T w with the updated norm, and the Hessenberg step on the
  // stream, and copies the step's flags to this column's host scratch;
  // arnoldi_finish (stream synchronized) reads them, runs a second
  // Gram-Schmidt pass when the norm dropped below 1/sqrt(10) of its value
  // (DGKS), normalizes the new vector and ends the cycle when the residual
  // estimate passed the test.  Enqueueing again recomputes the same step.
  void arnoldi_enqueue() {
    double* hbuf = h->d_small + slot * SM_COL;
    double* vn = V + (int64_t)(j + 1) * n;
    op(Z + (int64_t)j * n, vn);
    gemm_tn<double, double>(n, j + 2, V, n, vn, 1, hbuf, nullptr, h->red, 4, s);
    gemv_acc_norm(n, j + 1, V, n, hbuf, -1.0, vn, hbuf + j + 2, h->red, 5, s);
    hess_step(W, hbuf, nullptr, j, m, 0, thr, s);
    HIPCHK(hipMemcpyAsync(h->h_small + slot * SM_COL, hess_out(W), HESS_OUT * sizeof(double),
                          hipMemcpyDeviceToHost, s));
  }

  // One outer step of a single column with one host synchronization in the
  // usual case: the inner solve (a chunk of steps sized from the previous
  // solve), its output, the low-rank correction and the Arnoldi step go on
  // the stream together; only when the inner solve needed more steps than
  // the chunk does the host wait for it and enqueue the rest of the step
  // again.
  void step(bool fp32) {
    Range range("asss:outer step (inner solve, Arnoldi step, Hessenberg update)");
    const double* v = v_next();
    double* z = z_next();
    int expect = h->last_inner;
    if (nrecent > 0) expect = *std::max_element(recent, recent + std::min(nrecent, 4));
    InnerJob in;
    in.start(h, fp32, adjoint ? prec_pre_T(h, v, s) : v, z, adjoint ? -1 : +1, o.inner_tol, o.inner_maxit,
             o.fixed_inner_steps, s, expect);
    in.finish();
    if (!adjoint) smw_correct(h, z, s);
    arnoldi_enqueue();
    HIPCHK(hipStreamSynchronize(s));
    if (!in.settle()) {
      do {
        HIPCHK(hipStreamSynchronize(s));
      } while (!in.settle());
      in.finish();
      if (!adjoint) smw_correct(h, z, s);
      arnoldi_enqueue();
      HIPCHK(hipStreamSynchronize(s));
    }
    count_inner(in.its());
    arnoldi_finish();
  }

  void arnoldi_finish() {
    double* hbuf = h->d_small + slot * SM_COL;
    double* vn = V + (int64_t)(j + 1) * n;
    if (flags()[2] != 0.0) {
      double* h2 = hbuf + SM_PASS2;
      gemm_tn<double, double>(n, j + 1, V, n, vn, 1, h2, nullptr, h->red, 4, s);
      gemv_acc_norm(n, j + 1, V, n, h2, -1.0, vn, h2 + j + 1, h->red, 5, s);
      hess_step(W, hbuf, h2, j, m, 1, thr, s);
      HIPCHK(hipMemcpyAsync(h->h_small + slot * SM_COL, hess_out(W), HESS_OUT * sizeof(double),
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      inf.reorth++;
    }
    const double hn = flags()[1];
    gabs = flags()[0];
    implicit_ok = flags()[3] != 0.0;
    if (hn != 0.0) scale(n, 1.0 / hn, vn, vn, s);
    inf.outer_its++;
    if (h->opts.verbose)
      std::fprintf(stderr, "[asss] outer %d inner %d implicit %.3e\n", inf.outer_its, last_its, gabs / bcn);
    ++j;
    if (implicit_ok || hn == 0.0 || inf.outer_its >= o.max_outer || j == m) end_cycle();
  }

  // x_chk += Z y, back-transform, true residual; then finish or restart.
  void end_cycle() {
    const int j_used = j;
    if (j_used > 0) {
      hess_solve(W, j_used, m, s);
      gemv_acc(n, j_used, Z, n, hess_y(W), 1.0, xchk, s);
    }
    inf.relres_implicit = gabs / bcn;
    back_transform(h, adjoint, xchk, x, s);
    if (!adjoint) spmv(h->dA, x, rv, nullptr, nullptr, 1, b, s);   // r = b - A x
    else spmv(h->dAt, x, rv, nullptr, nullptr, 1, b, s);           // r = g - A^T lambda
    const double relres = std::sqrt(dot_host(h, n, rv, rv, s)) / bn;
    inf.relres_true = relres;
    if (relres <= o.tol) {
      status = ASSS_OK;
      inf.converged = 1;
      done = true;
      return;
    }
    if (inf.outer_its >= o.max_outer || j_used == 0) {
      // j_used == 0: the scaled residual was exactly zero while the true one is
      // not below tol; a restart would start from the same point
      done = true;
      return;
    }
    if (implicit_ok) thr = thr * 0.5 * o.tol / relres;
    start_cycle();
  }

  asss_status_t finish(asss_info_t* info) {
    HIPCHK(hipStreamSynchronize(s));
    inf.solve_s = now_s() - t0;
    inf.inner_kernel_s = h->prof_s;
    inf.inner_launches = h->prof_launches;
    if (info) *info = inf;
    return status;
  }
};

asss_status_t fgmres(asss_handle_s* h, bool adjoint, const double* b, double* x,
                     const asss_solve_opts_t& o, asss_info_t* info, hipStream_t s) {
  const bool fp32 = (o.inner_fp32 < 0) ? (h->opts.inner_fp32 != 0) : (o.inner_fp32 != 0);
  ensure_outer(h, std::max(1, o.restart_m));
  h->last_inner = 0;
  h->prof_s = 0.0;
  h->prof_launches = 0;
  FgmresCol c;
  c.begin(h, adjoint, b, x, o, h->V, h->Z, h->bchk, h->xchk, h->rv, s);
  while (!c.done) c.step(fp32);
  return c.finish(info);
}

// Up to NRMAX right-hand sides of one system (columns of B and X, leading
// dimension n) as FGMRES columns in lockstep: each step gathers the active
// columns' v_j into one block, solves the inner system for all of them with
// the simultaneous mrs of App. B (one pass over J_tilde and Q_k per inner
// step; the stop rule is the maximum over the block, so a column may iterate
// past its own tolerance), applies the SMW correction per column and lets each
// column take its Arnoldi step.  Columns restart and finish independently.
asss_status_t fgmres_block(asss_handle_s* h, int nc, const double* const* B, double* const* X,
                           const asss_solve_opts_t& o, asss_info_t* infos, hipStream_t s) {
  const int64_t n = h->n;
  const bool fp32 = (o.inner_fp32 < 0) ? (h->opts.inner_fp32 != 0) : (o.inner_fp32 != 0);
  const int m = std::max(1, o.restart_m);
  ensure_multi(h, m, fp32);
  h->last_inner = 0;
  h->prof_s = 0.0;
  h->prof_launches = 0;
  FgmresCol cols[NRMAX];
  for (int c = 0; c < nc; ++c) {
    cols[c].slot = c;
    cols[c].begin(h, false, B[c], X[c], o, h->mcol[c].V, h->mcol[c].Z, h->mcol[c].bchk, h->mcol[c].xchk,
                  h->mcol[c].rv, s);
  }
  for (;;) {
    int act[NRMAX], na = 0;
    for (int c = 0; c < nc; ++c)
      if (!cols[c].done) act[na++] = c;
    if (na == 0) break;
    for (int i = 0; i < na; ++i)
      HIPCHK(hipMemcpyAsync(h->pin + (int64_t)i * n, cols[act[i]].v_next(), n * sizeof(double),
                            hipMemcpyDeviceToDevice, s));
    int its;
    if (fp32)
      its = run_mrs<float, NRMAX>(h, h->J32, h->d_Q32, h->mb4_32, h->pin, h->pout, +1, o.inner_tol,
                                  o.inner_maxit, o.fixed_inner_steps, s, na);
    else
      its = run_mrs<double, NRMAX>(h, h->J64, h->d_Q64, h->mb4_64, h->pin, h->pout, +1, o.inner_tol,
                                   o.inner_maxit, o.fixed_inner_steps, s, na);
    // every active column's Arnoldi step goes on the stream, then one host
    // round trip serves them all
    Range range("asss:outer steps (lockstep columns, with their SMW terms)");
    for (int i = 0; i < na; ++i) {
      FgmresCol& c = cols[act[i]];
      double* z = c.z_next();
      HIPCHK(hipMemcpyAsync(z, h->pout + (int64_t)i * n, n * sizeof(double), hipMemcpyDeviceToDevice, s));
      smw_correct(h, z, s);
      c.count_inner(its);
      c.arnoldi_enqueue();
    }
    HIPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < na; ++i) cols[act[i]].arnoldi_finish();
  }
  asss_status_t worst = ASSS_OK;
  for (int c = 0; c < nc; ++c) {
    asss_status_t st = cols[c].finish(infos ? &infos[c] : nullptr);
    if (st > worst) worst = st;
  }
  return worst;
}

// Transpose-free QMR (Freund) on A_chk P^-1 y = b_chk with the iterate kept as
// x_chk = P^-1 y: every vector u that enters a product gets z = P^-1 u once,
// the product is A_chk z, and the direction is carried as P^-1 d built from
// the same z's (consistent with the products even though the inner solve is
// inexact).  Half steps m = 0, 1, ...: even m takes alpha = rho / (v, r*) and
// u_{m+1} = u_m - alpha v_m; odd m takes beta from rho = (w, r*) and forms
// u_{m+1} = w_{m+1} + beta u_m, v_{m+1} = A u_{m+1} + beta (A u_m + beta v_m).
// The quasi-residual bound tau sqrt(m + 2) triggers the true-residual check;
// a failed check or a breakdown restarts from x_chk (threshold as in fgmres).
asss_status_t tfqmr(asss_handle_s* h, bool adjoint, const double* b, double* x,
                    const asss_solve_opts_t& o, asss_info_t* info, hipStream_t s) {
  const double t0 = now_s();
  const int64_t n = h->n;
  const bool fp32 = (o.inner_fp32 < 0) ? (h->opts.inner_fp32 != 0) : (o.inner_fp32 != 0);
  asss_info_t inf{};
  inf.k_eff = h->k_eff;
  inf.rank_r = h->r;
  inf.setup_host_s = h->setup_host_s;
  inf.setup_device_s = h->setup_device_s;
  const double bn = std::sqrt(dot_host(h, n, b, b, s));
  if (bn == 0.0) {
    HIPCHK(hipMemsetAsync(x, 0, n * sizeof(double), s));
    HIPCHK(hipStreamSynchronize(s));
    inf.converged = 1;
    inf.solve_s = now_s() - t0;
    if (info) *info = inf;
    return ASSS_OK;
  }
  ensure_outer(h, 6);  // 7 + 6 work vectors
  double* w = h->V;
  double* u = h->V + n;
  double* un = h->V + 2 * n;
  double* v = h->V + 3 * n;
  double* Au = h->V + 4 * n;
  double* Aum_buf = h->V + 5 * n;
  double* rstar = h->V + 6 * n;
  double* z = h->Z;
  double* zm_buf = h->Z + n;
  double* dz = h->Z + 2 * n;
  rhs_transform(h, adjoint, b, h->bchk, s);
  const double bcn = std::sqrt(dot_host(h, n, h->bchk, h->bchk, s));
  double thr = o.tol * bcn;
  HIPCHK(hipMemsetAsync(h->xchk, 0, n * sizeof(double), s));
  auto op = [&](const double* in, double* out) {
    if (!adjoint) outer_op(h, in, out, s);
    else outer_op_T(h, in, out, s);
  };
  auto pre = [&](const double* in, double* out) {
    const int its = adjoint ? prec_apply_T(h, fp32, in, out, o, s) : prec_apply(h, fp32, in, out, o, s);
    inf.inner_its_total += its;
    inf.inner_its_max = std::max(inf.inner_its_max, its);
  };
  asss_status_t status = ASSS_NOT_CONVERGED;
  h->last_inner = 0;
  h->prof_s = 0.0;
  h->prof_launches = 0;
  bool first = true;
  for (;;) {
    axpby(n, 1.0, h->bchk, 0.0, w, s);  // w = r = b_chk - A_chk x_chk
    if (!first) {
      op(h->xchk, h->rv);
      axpby(n, -1.0, h->rv, 1.0, w, s);
    }
    first = false;
    inf.cycles++;
    double tau = std::sqrt(dot_host(h, n, w, w, s));
    double bound = tau;
    bool implicit_ok = tau <= thr;
    int cycle_steps = tau > 0.0 ? 1 : 0;  // 0: nothing to iterate on
    if (!implicit_ok) {
      axpby(n, 1.0, w, 0.0, rstar, s);
      axpby(n, 1.0, w, 0.0, u, s);
      double rho = tau * tau;
      pre(u, z);
      op(z, Au);
      axpby(n, 1.0, Au, 0.0, v, s);
      HIPCHK(hipMemsetAsync(dz, 0, n * sizeof(double), s));
      double theta = 0.0, eta = 0.0, alpha = 0.0;
      for (int m = 0;; ++m) {
        const double* zm;
        const double* Aum;
        if (m % 2 == 0) {
          const double sigma = dot_host(h, n, v, rstar, s);
          if (sigma == 0.0 || rho == 0.0) break;  // breakdown: restart
          alpha = rho / sigma;
          axpby(n, 1.0, u, 0.0, un, s);
          axpby(n, -alpha, v, 1.0, un, s);  // u_{m+1} = u_m - alpha v_m
          zm = z;
          Aum = Au;
        } else {
          pre(u, zm_buf);
          op(zm_buf, Aum_buf);
          zm = zm_buf;
          Aum = Aum_buf;
        }
        axpby(n, -alpha, Aum, 1.0, w, s);                                   // w -= alpha A u_m
        axpby(n, 1.0, zm, (theta * theta / alpha) * eta, dz, s);            // P^-1 d
        theta = std::sqrt(dot_host(h, n, w, w, s)) / tau;
        const double c = 1.0 / std::sqrt(1.0 + theta * theta);
        tau = tau * theta * c;
        eta = c * c * alpha;
        axpby(n, eta, dz, 1.0, h->xchk, s);
        inf.outer_its++;
        bound = tau * std::sqrt(m + 2.0);
        implicit_ok = bound <= thr;
        if (h->opts.verbose)
          std::fprintf(stderr, "[asss] tfqmr half step %d bound %.3e\n", inf.outer_its, bound / bcn);
        if (implicit_ok || inf.outer_its >= o.max_outer) break;
        if (m % 2 == 1) {
          const double rho_new = dot_host(h, n, w, rstar, s);
          if (rho_new == 0.0) break;  // breakdown: restart
          const double beta = rho_new / rho;
          rho = rho_new;
          axpby(n, 1.0, w, 0.0, un, s);
          axpby(n, beta, u, 1.0, un, s);  // u_{m+1} = w_{m+1} + beta u_m
          pre(un, z);
          op(z, Au);                      // A u_{m+1}
          axpby(n, 1.0, Aum, beta, v, s);  // v = A u_m + beta v_m
          axpby(n, 1.0, Au, beta, v, s);   // v = A u_{m+1} + beta (A u_m + beta v_m)
        }
        std::swap(u, un);
      }
    }
    inf.relres_implicit = bound / bcn;
    double relres;
    back_transform(h, adjoint, h->xchk, x, s);
    if (!adjoint) spmv(h->dA, x, h->rv, nullptr, nullptr, 1, b, s);
    else spmv(h->dAt, x, h->rv, nullptr, nullptr, 1, b, s);
    relres = std::sqrt(dot_host(h, n, h->rv, h->rv, s)) / bn;
    inf.relres_true = relres;
    if (relres <= o.tol) {
      status = ASSS_OK;
      inf.converged = 1;
      break;
    }
    // a zero scaled residual with the true one above tol: no step can be taken
    if (inf.outer_its >= o.max_outer || cycle_steps == 0) break;
    if (implicit_ok) thr = thr * 0.5 * o.tol / relres;
  }
  HIPCHK(hipStreamSynchronize(s));
  inf.solve_s = now_s() - t0;
  inf.inner_kernel_s = h->prof_s;
  inf.inner_launches = h->prof_launches;
  if (info) *info = inf;
  return status;
}

asss_status_t outer_from_zero(asss_handle_s* h, bool adjoint, const double* b, double* x,
                              const asss_solve_opts_t& o, asss_info_t* info, hipStream_t s) {
  if (o.outer == ASSS_OUTER_TFQMR) return tfqmr(h, adjoint, b, x, o, info, s);
  return fgmres(h, adjoint, b, x, o, info, s);
}

// With use_x0 the iteration starts from the caller's x: the outer method
// solves for the correction d of the residual r0 = b - A x0 (A^T for the
// adjoint) to the relative tolerance tol ||b|| / ||r0||, and x = x0 + d.  In
// exact arithmetic this is the iteration started at the transformed x0 (the
// right-preconditioned residual of x0 is the transformed r0) without having
// to apply S^-1 to x0.  The reported true residual is that of x0 + d against b.
asss_status_t outer_solve(asss_handle_s* h, bool adjoint, const double* b, double* x,
                          const asss_solve_opts_t& o, asss_info_t* info, hipStream_t s) {
  if (!o.use_x0) return outer_from_zero(h, adjoint, b, x, o, info, s);
  const int64_t n = h->n;
  if (!b_is_finite(h, x, s)) throw Error{ASSS_ERR_NONFINITE, "x0 has a non-finite entry"};
  if (!h->x0r) {
    if (h->no_alloc) throw Error{ASSS_ERR_INTERNAL, "no workspace for a solve from x0"};
    h->x0r = h->ar.alloc<double>(n);
    h->x0d = h->ar.alloc<double>(n);
  }
  const DCsr& M = adjoint ? h->dAt : h->dA;
  auto residual = [&]() {  // x0r = b - M x
    spmv(M, x, h->x0r, nullptr, nullptr, 0, nullptr, s);
    axpby(n, 1.0, b, -1.0, h->x0r, s);
    return std::sqrt(dot_host(h, n, h->x0r, h->x0r, s));
  };
  const double t0 = now_s();
  const double bn = std::sqrt(dot_host(h, n, b, b, s));
  const double rn = residual();
  asss_solve_opts_t oo = o;
  oo.use_x0 = 0;
  if (bn == 0.0 || rn <= o.tol * bn) {  // b = 0 gives x = 0, as from zero
    if (bn == 0.0) HIPCHK(hipMemsetAsync(x, 0, n * sizeof(double), s));
    asss_info_t inf{};
    inf.converged = 1;
    inf.k_eff = h->k_eff;
    inf.rank_r = h->r;
    inf.relres_true = bn == 0.0 ? 0.0 : rn / bn;
    inf.setup_host_s = h->setup_host_s;
    inf.setup_device_s = h->setup_device_s;
    HIPCHK(hipStreamSynchronize(s));
    inf.solve_s = now_s() - t0;
    if (info) *info = inf;
    return ASSS_OK;
  }
  oo.tol = o.tol * bn / rn;
  asss_info_t inf{};
  outer_from_zero(h, adjoint, h->x0r, h->x0d, oo, &inf, s);
  axpby(n, 1.0, h->x0d, 1.0, x, s);
  const double rel = residual() / bn;
  inf.relres_true = rel;
  inf.converged = rel <= o.tol ? 1 : 0;
  HIPCHK(hipStreamSynchronize(s));
  inf.solve_s = now_s() - t0;
  if (info) *info = inf;
  return inf.converged ? ASSS_OK : ASSS_NOT_CONVERGED;
}

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current and kept.
double* noalloc_scratch(int device) {
  static std::mutex mu;
  static std::map<int, double*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it != addr.end()) return it->second;
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  if (cur != device) HIPCHK(hipSetDevice(device));
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) HIPCHK(hipSetDevice(cur));
  HIPCHK(e);
  if (!p) throw Error{ASSS_ERR_HIP, "hipGetSymbolAddress gave no address for the fixed workspace"};
  addr[device] = (double*)p;
  return (double*)p;
}

// Points the handle's Krylov workspace (m columns) and the buffers of a
// solve from x0 into the fixed scratch for one call, forbids allocation, and
// puts the handle's own workspace back afterwards (also when the call throws).
struct ScratchWorkspace {
  asss_handle_s* h;
  double *V, *Z, *x0r, *x0d;
  int m_alloc;
  ScratchWorkspace(asss_handle_s* h_, double* base, int m)
      : h(h_), V(h_->V), Z(h_->Z), x0r(h_->x0r), x0d(h_->x0d), m_alloc(h_->m_alloc) {
    const int64_t n = h->n;
    h->V = base;
    h->Z = base + n * (int64_t)(m + 1);
    h->x0r = h->Z + n * (int64_t)m;
    h->x0d = h->x0r + n;
    h->m_alloc = m;
    h->no_alloc = true;
  }
  ~ScratchWorkspace() {
    h->V = V; h->Z = Z; h->x0r = x0r; h->x0d = x0d;
    h->m_alloc = m_alloc;
    h->no_alloc = false;
  }
};

void check_handle(asss_handle_s* h) {
  if (!h) throw Error{ASSS_ERR_INVALID_ARG, "null handle"};
  HIPCHK(hipSetDevice(h->device));
}

asss_solve_opts_t opts_or_default(const asss_solve_opts_t* o) {
  asss_solve_opts_t d;
  asss_default_solve_opts(&d);
  return o ? *o : d;
}

template <class F>
asss_status_t guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    g_err = e.msg;
    return e.code;
  } catch (const HostError& e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host out of memory";
    return ASSS_ERR_OOM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return ASSS_ERR_INTERNAL;
  }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

// Matching, scalings and S of a saved setup (asss_load).
struct Preset {
  std::vector<int32_t> m;
  std::vector<double> Dr, Dc;
  Csr S;
};

// Setup; `pre` (from asss_load) supplies the matching, the scalings and S
// (pattern and values), which are then neither recomputed nor solved for.
static asss_status_t setup_impl(const asss_csr_t* A, const asss_setup_opts_t* opts, void* hip_stream,
                                asss_handle_t* out, const Preset* pre) {
  Range range("asss_setup");
  return guarded([&]() -> asss_status_t {
    if (!A || !out) throw Error{ASSS_ERR_INVALID_ARG, "null argument"};
    *out = nullptr;
    asss_setup_opts_t o;
    asss_default_setup_opts(&o);
    if (opts) o = *opts;
    if (o.k < 0 || o.k > KMAX) throw Error{ASSS_ERR_INVALID_ARG, "k must be in [0, 32]"};
    if (!(o.gamma > 0)) throw Error{ASSS_ERR_INVALID_ARG, "gamma must be positive"};
    if (o.deflation < 0 || o.deflation > 3 || o.deflation == 2)
      throw Error{ASSS_ERR_INVALID_ARG, "deflation must be 0, 1 or 3 (2, a recurrence form of the projector, "
                                        "loses orthogonality and is not provided)"};
    if (o.reorder < 0 || o.reorder > 4 || o.reorder == 2)
      throw Error{ASSS_ERR_INVALID_ARG, "reorder must be 0, 1, 3 or 4 (2, a BFS block partition, is not provided)"};
    if (o.reorder == 3 && !o.inner_perm) throw Error{ASSS_ERR_INVALID_ARG, "reorder 3 needs inner_perm"};
    if (o.row_block != 0 && (o.row_block % 64 != 0 || o.row_block > 4096))
      throw Error{ASSS_ERR_INVALID_ARG, "row_block must be a multiple of 64 and <= 4096"};
    if (o.autotune < 0 || o.autotune > 1) throw Error{ASSS_ERR_INVALID_ARG, "autotune must be 0 or 1"};
    if (o.skew_form < 0 || o.skew_form > 3) throw Error{ASSS_ERR_INVALID_ARG, "skew_form must be 0, 1, 2 or 3"};
    if (o.step_threads != 0 && o.step_threads != 256 && o.step_threads != 512)
      throw Error{ASSS_ERR_INVALID_ARG, "step_threads must be 0, 256 or 512"};
    if (o.ildl_explicit < -1 || o.ildl_explicit > 1)
      throw Error{ASSS_ERR_INVALID_ARG, "ildl_explicit must be -1, 0 or 1"};
    if (o.precond != ASSS_PRECOND_DIAG && o.precond != ASSS_PRECOND_ILDL)
      throw Error{ASSS_ERR_INVALID_ARG, "precond must be ASSS_PRECOND_DIAG or ASSS_PRECOND_ILDL"};
    if (o.precond == ASSS_PRECOND_ILDL) {
      if (o.reorder > 1)
        throw Error{ASSS_ERR_INVALID_ARG, "the incomplete LDL^T preconditioner runs in its factorization's order "
                                          "(reorder must be 0)"};
      if (o.deflation == 3 || o.autotune)
        throw Error{ASSS_ERR_INVALID_ARG, "the incomplete LDL^T preconditioner takes neither the FP32-valued "
                                          "deflation basis nor the row-block autotuner"};
      if (!(o.ildl_droptol >= 0.0) || !(o.ildl_fill > 0.0))
        throw Error{ASSS_ERR_INVALID_ARG, "ildl_droptol must be >= 0 and ildl_fill > 0"};
    }
    hipStream_t s = (hipStream_t)hip_stream;
    std::unique_ptr<asss_handle_s> h(new asss_handle_s());
    static std::atomic<uint64_t> next_uid{1};
    h->uid = next_uid++;
    HIPCHK(hipGetDevice(&h->device));
    if (o.allocator) {
      if (!o.allocator->alloc || !o.allocator->free)
        throw Error{ASSS_ERR_INVALID_ARG, "allocator needs both alloc and free"};
      h->ar.al = *o.allocator;  // copied: the caller's structure may go away
    }
    h->opts = o;
    h->opts.allocator = nullptr;
    h->opts.s_val = nullptr;  // caller arrays are read during setup only
    h->opts.q_basis = h->opts.q_alpha = nullptr;
    std::optional<Range> phase;
    phase.emplace("asss_setup:host preprocessing");
    const double t0 = now_s();
    // ---- host preprocessing
    Csr Ah = validate_and_copy(A->n, A->nnz, A->rowptr, A->colind, A->val);
    h->n = Ah.nrows;
    h->nnz_a = Ah.nnz();
    const int64_t n = h->n;
    if (o.q_basis && o.k > 0) {
      if (o.k > 1 && !o.q_alpha) throw Error{ASSS_ERR_INVALID_ARG, "q_basis needs q_alpha (k - 1 values)"};
      h->q_given.assign(o.q_basis, o.q_basis + (size_t)n * o.k);
      if (o.k > 1) h->alpha_given.assign(o.q_alpha, o.q_alpha + (o.k - 1));
      for (double v : h->q_given)
        if (!std::isfinite(v)) throw Error{ASSS_ERR_NONFINITE, "q_basis holds a NaN or Inf"};
      for (double v : h->alpha_given)
        if (!std::isfinite(v)) throw Error{ASSS_ERR_NONFINITE, "q_alpha holds a NaN or Inf"};
    }
    if (pre) {
      if ((int64_t)pre->m.size() != n || (int64_t)pre->Dr.size() != n || (int64_t)pre->Dc.size() != n ||
          pre->S.nrows != n)
        throw Error{ASSS_ERR_INVALID_ARG, "saved setup does not match the matrix size"};
      h->m = pre->m;
      h->Dr = pre->Dr;
      h->Dc = pre->Dc;
    } else {
      h->m = max_product_matching(Ah);
      canonical_scaling(Ah, h->m, h->Dr, h->Dc);
    }
    Csr Abar = permute_scale(Ah, h->m, h->Dr, h->Dc);
    Csr Spat;
    if (pre) {
      Spat = pre->S;
      Spat.val.clear();
    } else {
      Spat = s_pattern(Abar, o.s_pattern, o.s_rowptr, o.s_colind);
    }
    LlsSystem L;
    build_lls(Abar, Spat, o.gamma, L);
    h->lls_rows = L.B.nrows;
    h->lls_nnz = L.B.nnz();
    const double t1 = now_s();
    phase.reset();
    phase.emplace("asss_setup:LSQR for S");
    // ---- device: reducer and scalar buffers first (LSQR uses them)
    int R = o.row_block;
    int auto_R = 64;
    while (auto_R < 2048 && (int64_t)auto_R * 2 * 1024 <= n) auto_R *= 2;
    // reorder 4: tiles of whole grid lines when Abar is a lexicographic 3D grid,
    // up to 1.5x the automatic block: tiles of 4 x 4 lines at 128^3 (R = 2048)
    // and at 192^3 (R = 3072; 4 x 2 lines within 2048 gave 430 against 408 us
    // per FP64 step)
    std::vector<int32_t> grid_perm;
    int32_t grid_R = 0;
    if (o.reorder == 4) grid_perm = grid_line_order(Abar, R ? R : 3 * auto_R / 2, grid_R);
    if (R == 0) R = grid_perm.empty() ? auto_R : grid_R;
    // autotuner candidates: the automatic size and up to two doublings and
    // halvings of it within [64, 4096]
    std::vector<int> cands;
    if (o.autotune && o.row_block == 0)
      for (int c = std::max(64, R / 4); c <= std::min(4096, R * 4); c *= 2) cands.push_back(c);
    const int Rmin = cands.empty() ? R : cands.front();
    const int64_t nblocks = (n + Rmin - 1) / Rmin;
    h->red.max_groups = (int)std::max<int64_t>(nblocks, 1024);
    h->red.partials = h->ar.alloc<double>((int64_t)h->red.max_groups * RED_SLOTS);
    h->red.tickets = h->ar.alloc<unsigned>(16);
    HIPCHK(hipMemsetAsync(h->red.tickets, 0, 16 * sizeof(unsigned), s));
    h->d_small = h->ar.alloc<double>(SM_SIZE);
    h->d_hess = h->ar.alloc<double>((int64_t)NRMAX * HESS_SLOT);
    h->d_flag = h->ar.alloc<int>(1);
    HIPCHK(hipHostMalloc((void**)&h->h_small, SM_SIZE * sizeof(double), hipHostMallocDefault));
    h->d_state = h->ar.alloc<MrsState>(1);
    HIPCHK(hipEventCreate(&h->ev0));
    HIPCHK(hipEventCreate(&h->ev1));
    std::vector<double> svals;
    if (pre) {
      svals = pre->S.val;
    } else if (o.s_val) {  // S given by the caller: no least-squares solve
      svals.assign(o.s_val, o.s_val + Spat.nnz());
      for (double v : svals)
        if (!std::isfinite(v)) throw Error{ASSS_ERR_NONFINITE, "s_val holds a NaN or Inf"};
    } else {
      svals = lsqr_device(h.get(), L, o.lls_tol, o.lls_maxit, s);
    }
    const double t2 = now_s();
    phase.reset();
    phase.emplace("asss_setup:split and pack");
    h->S = Spat;
    h->S.val = svals;
    Csr Ahat = spgemm_on_pattern(Abar, h->S, L.P);
    h->nnz_ahat = Ahat.nnz();
    h->U = L.U;
    const bool ildl = o.precond == ASSS_PRECOND_ILDL;
    h->neg.clear();
    Csr Jup;
    bool reordered = false;
    SkewSell sell;
    if (ildl) {
      // D = diag(A_hat) and J_hat = (A_hat - A_hat^T) / 2 on U, unscaled: the
      // scaling is inside the factor Lcal (ildl_setup)
      h->D.assign(n, 0.0);
      h->Omega.assign(n, 1.0);
      Csr Ms, Js;
      symmetric_skew_split(Ahat, Ms, Js);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t e = Ahat.ptr[i]; e < Ahat.ptr[i + 1]; ++e)
          if (Ahat.col[e] == i) h->D[i] = Ahat.val[e];
      h->jval.clear();
      for (int64_t i = 0; i < n; ++i)
        for (int64_t e = Js.ptr[i]; e < Js.ptr[i + 1]; ++e)
          if (Js.col[e] > i) h->jval.push_back(Js.val[e]);
      if ((int64_t)h->jval.size() != h->U.nnz()) throw Error{ASSS_ERR_INTERNAL, "pattern of J_hat differs from U"};
    } else {
    split_ahat(Ahat, h->U, h->D, h->Omega, h->jval);
    for (int64_t i = 0; i < n; ++i)
      if (h->D[i] < 0) h->neg.push_back((int32_t)i);
    Jup = h->U;
    Jup.val = h->jval;
    // block order of the inner system (fewer pairs stored twice in the sliced layout)
    h->cross_natural = count_cross_pairs(Jup, R);
    h->cross_used = h->cross_natural;
    if (o.reorder == 4 && !grid_perm.empty()) {  // line tiles of a detected grid
      Jup = permute_skew_upper(Jup, grid_perm);
      h->cross_used = count_cross_pairs(Jup, R);
      h->perm = std::move(grid_perm);
      reordered = true;
    } else if (o.reorder == 3) {  // the caller's order, validated as a permutation
      std::vector<int32_t> perm(o.inner_perm, o.inner_perm + n);
      std::vector<char> seen(n, 0);
      for (int64_t i = 0; i < n; ++i) {
        if (perm[i] < 0 || perm[i] >= n || seen[perm[i]])
          throw Error{ASSS_ERR_INVALID_ARG, "inner_perm is not a permutation of 0..n-1"};
        seen[perm[i]] = 1;
      }
      Jup = permute_skew_upper(Jup, perm);
      h->cross_used = count_cross_pairs(Jup, R);
      h->perm = std::move(perm);
      reordered = true;
    }
    sell = pack_skew_sell(Jup, R, o.skew_form);
    h->sell_a = sell.a_entries;
    h->sell_b = sell.b_entries;
    }
    { LlsSystem dummy; std::swap(L, dummy); }
    // ---- device uploads
    h->Apat.nrows = h->Apat.ncols = n;
    h->Apat.ptr = Ah.ptr;
    h->Apat.col = Ah.col;
    h->dA = upload_csr(h->ar, Ah, s);
    h->dAt = upload_csr(h->ar, transpose(Ah), s);
    h->dAbar = upload_csr(h->ar, Abar, s);
    h->dAbarT = upload_csr(h->ar, transpose(Abar), s);
    h->dS = upload_csr(h->ar, h->S, s);
    h->dSt = upload_csr(h->ar, transpose(h->S), s);
    if (!ildl) {
      h->eAbar = ell_from_csr(h->ar, h->dAbar, s);
      h->eAbarT = ell_from_csr(h->ar, h->dAbarT, s);
      h->eS = ell_from_csr(h->ar, h->dS, s);
      h->eSt = ell_from_csr(h->ar, h->dSt, s);
    }
    h->d_m = h->ar.upload(h->m, s);
    if (reordered) h->d_perm = h->ar.upload(h->perm, s);
    std::vector<double> drp(n);
    for (int64_t j = 0; j < n; ++j) drp[j] = h->Dr[h->m[j]];
    h->d_drp = h->ar.upload(drp, s);
    h->d_om = h->ar.upload(h->Omega, s);
    h->d_dc = h->ar.upload(h->Dc, s);
    if (!ildl) {
      SkewLayout lay = upload_layout(h->ar, sell, s, h->opts.step_threads);
      h->narrow_b = lay.narrow;
      h->skew_form = lay.form;
      h->J64 = lay.J64;
      h->J32 = lay.J32;
      h->lay_bufs = std::move(lay.bufs);
    }
    for (int b = 0; b < 3; ++b) { h->mb64.w[b] = h->ar.alloc<double>(n); h->mb32.w[b] = h->ar.alloc<float>(n); }
    for (int b = 0; b < 2; ++b) { h->mb64.p[b] = h->ar.alloc<double>(n); h->mb32.p[b] = h->ar.alloc<float>(n); }
    h->mb64.x = h->ar.alloc<double>(n);
    h->mb32.x = h->ar.alloc<float>(n);
    h->w = h->ar.alloc<double>(n);
    h->t1 = h->ar.alloc<double>(n);
    h->xchk = h->ar.alloc<double>(n);
    h->bchk = h->ar.alloc<double>(n);
    h->rv = h->ar.alloc<double>(n);
    h->tmp = h->ar.alloc<double>(n);
    HIPCHK(hipStreamSynchronize(s));
    if (ildl) {
      Range r3("asss_setup:incomplete LDL^T");
      h->il.opts.droptol = o.ildl_droptol;
      h->il.opts.fill = o.ildl_fill;
      h->il.opts.pivoting = o.ildl_pivoting != 0;
      ildl_setup(h.get(), Ahat, s);
      if (o.ildl_explicit == 1) {
        ildl_explicit_jtilde(h.get(), s);
      } else if (o.ildl_explicit < 0 && n <= 12288) {
        try {  // by default: the triangular solves per product when the dense operators do not fit
          ildl_explicit_jtilde(h.get(), s);
        } catch (const Error& e) {
          if (e.code != ASSS_ERR_OOM) throw;
          (void)hipGetLastError();
        }
      }
    }
    const double t3 = now_s();
    phase.reset();
    phase.emplace("asss_setup:Lanczos, X, C");
    device_setup(h.get(), s);
    const double t4 = now_s();
    phase.reset();
    if (cands.size() > 1) {
      Range tune("asss_setup:row-block autotune");
      tune_row_block(h.get(), Jup, cands, s);
      h->tune_s = now_s() - t4;
      if (o.verbose) {
        std::fprintf(stderr, "[asss] row-block autotune %.3fs:", h->tune_s);
        for (auto& c : h->tuned) std::fprintf(stderr, " %d:%.1fus", c.first, c.second);
        std::fprintf(stderr, " -> %d\n", h->J64.R);
      }
    }
    h->setup_host_s = (t1 - t0) + (t3 - t2);
    h->setup_device_s = (t2 - t1) + (t4 - t3);
    if (o.verbose)
      std::fprintf(stderr,
                   "[asss] setup n=%lld host %.3fs (pre %.3f, split/pack %.3f) lsqr %.3fs (%d its, kkt %.2e) "
                   "device %.3fs (k_eff %d, r %d, X its %d, orth %.1e, deflation %s)\n",
                   (long long)n, h->setup_host_s, t1 - t0, t3 - t2, t2 - t1, h->lls_its, h->lls_kkt,
                   t4 - t3, h->k_eff, h->r, h->x_its, h->orth_err,
                   h->opts.deflation == 3 ? "explicit, FP32 basis" : "explicit");
    *out = h.release();
    return ASSS_OK;
  });
}

struct asss_ildl_s {
  IldlFactor F;
  IldlScaled S;
};

extern "C" {

void asss_default_setup_opts(asss_setup_opts_t* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->gamma = 1.0;
  o->s_pattern = ASSS_S_TRIDIAG;
  o->k = 20;
  o->lanczos_seed = 0x2009069540ull;
  o->inner_fp32 = 0;
  o->x_tol = 1e-10;
  o->x_maxit = 2000;
  o->lls_tol = 1e-15;
  o->lls_maxit = 20000;
  o->row_block = 0;
  o->verbose = 0;
  o->deflation = 0;
  o->reorder = 0;
  o->autotune = 0;
  o->inner_perm = nullptr;
  o->skew_form = 0;
  o->precond = ASSS_PRECOND_DIAG;
  o->ildl_droptol = 0.0;
  o->ildl_fill = HUGE_VAL;
  o->ildl_pivoting = 1;
  o->ildl_explicit = -1;
  o->step_threads = 0;
}

void asss_default_solve_opts(asss_solve_opts_t* o) {
  if (!o) return;
  o->tol = 1e-8;
  o->restart_m = 64;
  o->max_outer = 2000;
  o->inner_tol = 1e-5;
  o->inner_maxit = 1000;
  o->fixed_inner_steps = 0;
  o->inner_fp32 = -1;
  o->outer = ASSS_OUTER_FGMRES;
  o->batch_streams = 0;
  o->use_x0 = 0;
  o->batch_engine = 0;
}

const char* asss_last_error(void) { return g_err.c_str(); }

asss_status_t asss_setup(const asss_csr_t* A, const asss_setup_opts_t* opts, void* hip_stream,
                         asss_handle_t* out) {
  return setup_impl(A, opts, hip_stream, out, nullptr);
}

asss_status_t asss_solve(asss_handle_t h, const double* b_dev, double* x_dev, const asss_solve_opts_t* o,
                         asss_info_t* info, void* hip_stream) {
  Range range("asss_solve");
  return guarded([&]() -> asss_status_t {
    check_handle(h);
    if (!b_dev || !x_dev) throw Error{ASSS_ERR_INVALID_ARG, "null vector"};
    if (overlaps(b_dev, h->n, x_dev, h->n)) throw Error{ASSS_ERR_INVALID_ARG, "b and x overlap"};
    hipStream_t s = (hipStream_t)hip_stream;
    asss_solve_opts_t oo = opts_or_default(o);
    if (oo.restart_m < 1 || oo.restart_m > 250) throw Error{ASSS_ERR_INVALID_ARG, "restart_m must be in [1, 250]"};
    if (oo.outer != ASSS_OUTER_FGMRES && oo.outer != ASSS_OUTER_TFQMR)
      throw Error{ASSS_ERR_INVALID_ARG, "outer must be ASSS_OUTER_FGMRES or ASSS_OUTER_TFQMR"};
    if (!b_is_finite(h, b_dev, s)) throw Error{ASSS_ERR_NONFINITE, "b has a non-finite entry"};
    return outer_solve(h, false, b_dev, x_dev, oo, info, s);
  });
}

asss_status_t asss_solve_noalloc(asss_handle_t h, const double* b_dev, double* x_dev, const asss_solve_opts_t* o,
                                 asss_info_t* info, void* hip_stream) {
  Range range("asss_solve_noalloc");
  return guarded([&]() -> asss_status_t {
    check_handle(h);
    if (!b_dev || !x_dev) throw Error{ASSS_ERR_INVALID_ARG, "null vector"};
    if (overlaps(b_dev, h->n, x_dev, h->n)) throw Error{ASSS_ERR_INVALID_ARG, "b and x overlap"};
    hipStream_t s = (hipStream_t)hip_stream;
    asss_solve_opts_t oo = opts_or_default(o);
    if (oo.restart_m < 1 || oo.restart_m > 250) throw Error{ASSS_ERR_INVALID_ARG, "restart_m must be in [1, 250]"};
    if (oo.outer != ASSS_OUTER_FGMRES && oo.outer != ASSS_OUTER_TFQMR)
      throw Error{ASSS_ERR_INVALID_ARG, "outer must be ASSS_OUTER_FGMRES or ASSS_OUTER_TFQMR"};
    // FGMRES(m): V (m + 1 vectors) and Z (m); TFQMR: 7 + 6 vectors; x0: 2 more
    const int m = oo.outer == ASSS_OUTER_TFQMR ? 6 : oo.restart_m;
    const uint64_t need = (uint64_t)h->n * (uint64_t)(2 * m + 3) * sizeof(double);
    if (need > kNoAllocBytes) {
      char msg[200];
      std::snprintf(msg, sizeof msg,
                    "asss_solve_noalloc needs n (2 m + 3) 8 = %llu bytes of workspace (n = %lld, m = %d); "
                    "its fixed workspace holds %llu",
                    (unsigned long long)need, (long long)h->n, m, (unsigned long long)kNoAllocBytes);
      throw Error{ASSS_ERR_INVALID_ARG, msg};
    }
    double* base = noalloc_scratch(h->device);
    if (!b_is_finite(h, b_dev, s)) throw Error{ASSS_ERR_NONFINITE, "b has a non-finite entry"};
    ScratchWorkspace ws(h, base, m);
    return outer_solve(h, false, b_dev, x_dev, oo, info, s);
  });
}

asss_status_t asss_solve_adjoint(asss_handle_t h, const double* g_dev, double* lambda_dev,
                                 const asss_solve_opts_t* o, asss_info_t* info, void* hip_stream) {
  Range range("asss_solve_adjoint");
  return guarded([&]() -> asss_status_t {
    check_handle(h);
    if (!g_dev || !lambda_dev) throw Error{ASSS_ERR_INVALID_ARG, "null vector"};
    if (overlaps(g_dev, h->n, lambda_dev, h->n)) throw Error{ASSS_ERR_INVALID_ARG, "g and lambda overlap"};
    hipStream_t s = (hipStream_t)hip_stream;
    asss_solve_opts_t oo = opts_or_default(o);
    if (oo.restart_m < 1 || oo.restart_m > 250) throw Error{ASSS_ERR_INVALID_ARG, "restart_m must be in [1, 250]"};
    if (oo.outer != ASSS_OUTER_FGMRES && oo.outer != ASSS_OUTER_TFQMR)
      throw Error{ASSS_ERR_INVALID_ARG, "outer must be ASSS_OUTER_FGMRES or ASSS_OUTER_TFQMR"};
    if (!b_is_finite(h, g_dev, s)) throw Error{ASSS_ERR_NONFINITE, "g has a non-finite entry"};
    return outer_solve(h, true, g_dev, lambda_dev, oo, info, s);
  });
}

asss_status_t asss_update_values(asss_handle_t h, const asss_csr_t* A, void* hip_stream) {
  return guarded([&]() -> asss_status_t {
    check_handle(h);
    if (!A) throw Error{ASSS_ERR_INVALID_ARG, "null argument"};
    if (h->il.on)
      throw Error{ASSS_ERR_INVALID_ARG, "value updates are not provided for the incomplete LDL^T preconditioner "
                                        "(its outer operator holds A_hat itself)"};
    hipStream_t s = (hipStream_t)hip_stream;
    Csr Ah = map_values_onto(h->Apat, A->n, A->nnz, A->rowptr, A->colind, A->val);
    Csr Abar = permute_scale(Ah, h->m, h->Dr, h->Dc);
    Csr At = transpose(Ah), AbarT = transpose(Abar);
    const DCsr* dst[4] = {&h->dA, &h->dAt, &h->dAbar, &h->dAbarT};
    const Csr* src[4] = {&Ah, &At, &Abar, &AbarT};
    for (int q = 0; q < 4; ++q) {
      if (src[q]->nnz() != dst[q]->nnz) throw Error{ASSS_ERR_INTERNAL, "stored pattern changed"};
      HIPCHK(hipMemcpyAsync(dst[q]->val, src[q]->val.data(), src[q]->nnz() * sizeof(double),
                            hipMemcpyHostToDevice, s));
    }
    // the sliced copies from the new CSR values, after their copies on s
    const DSell* edst[2] = {&h->eAbar, &h->eAbarT};
    for (int q = 0; q < 2; ++q) {
      const DSell& E = *edst[q];
      const DCsr& M = *dst[2 + q];
      if (E.nrows > 0) ell_fill(M.nrows, M.ptr, M.col, M.val, E.width, E.off, E.col, E.val, s);
    }
    HIPCHK(hipStreamSynchronize(s));  // the host arrays go out of scope
    return ASSS_OK;
  });
}

asss_status_t asss_value_gradient(asss_handle_t h, int64_t nnz, const int64_t* rowptr_dev,
                                  const int32_t* colind_dev, const double* lambda_dev, const double* x_dev,
                                  double* grad_dev, void* hip_stream) {
  return guarded([&]() -> asss_status_t {
    check_handle(h);
    if (nnz < 0) throw Error{ASSS_ERR_INVALID_ARG, "nnz must be >= 0"};
    if (!rowptr_dev || !lambda_dev || !x_dev || (nnz > 0 && (!colind_dev || !grad_dev)))
      throw Error{ASSS_ERR_INVALID_ARG, "null argument"};
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(hipMemsetAsync(h->d_flag, 0, sizeof(int), s));
    csr_value_grad(h->n, nnz, rowptr_dev, colind_dev, lambda_dev, x_dev, grad_dev, h->d_flag, s);
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, h->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (bad) throw Error{ASSS_ERR_INVALID_CSR, "invalid row pointer or column index in the gradient pattern"};
    return ASSS_OK;
  });
}

asss_status_t asss_solve_batched(int32_t nsys, const asss_handle_t* hs, const int32_t* nrhs,
                                 const double* const* B_dev, double* const* X_dev,
                                 const asss_solve_opts_t* o, asss_info_t* infos, void* hip_stream) {
  Range range("asss_solve_batched");
  return guarded([&]() -> asss_status_t {
    if (nsys < 0 || (nsys > 0 && (!hs || !nrhs || !B_dev || !X_dev)))
      throw Error{ASSS_ERR_INVALID_ARG, "null argument"};
    hipStream_t s = (hipStream_t)hip_stream;
    asss_solve_opts_t oo = opts_or_default(o);
    if (oo.restart_m < 1 || oo.restart_m > 250) throw Error{ASSS_ERR_INVALID_ARG, "restart_m must be in [1, 250]"};
    if (oo.outer != ASSS_OUTER_FGMRES && oo.outer != ASSS_OUTER_TFQMR)
      throw Error{ASSS_ERR_INVALID_ARG, "outer must be ASSS_OUTER_FGMRES or ASSS_OUTER_TFQMR"};
    int maxr = 0;
    for (int sidx = 0; sidx < nsys; ++sidx) {
      if (!hs[sidx]) throw Error{ASSS_ERR_INVALID_ARG, "null handle"};
      if (nrhs[sidx] < 0 || (nrhs[sidx] > 0 && (!B_dev[sidx] || !X_dev[sidx])))
        throw Error{ASSS_ERR_INVALID_ARG, "bad nrhs or null block"};
      if (nrhs[sidx] > 0 && overlaps(B_dev[sidx], hs[sidx]->n * (int64_t)nrhs[sidx], X_dev[sidx],
                                     hs[sidx]->n * (int64_t)nrhs[sidx]))
        throw Error{ASSS_ERR_INVALID_ARG, "a right-hand side block and its solution block overlap"};
      maxr = std::max(maxr, (int)nrhs[sidx]);
    }
    // every right-hand side is checked before any is solved
    for (int sidx = 0; sidx < nsys; ++sidx) {
      check_handle(hs[sidx]);
      for (int j = 0; j < nrhs[sidx]; ++j)
        if (!b_is_finite(hs[sidx], B_dev[sidx] + (int64_t)j * hs[sidx]->n, s))
          throw Error{ASSS_ERR_NONFINITE, "a right-hand side has a non-finite entry"};
    }
    if (oo.batch_streams < 0 || oo.batch_streams > 16)
      throw Error{ASSS_ERR_INVALID_ARG, "batch_streams must be in [0, 16]"};
    if (oo.batch_engine < 0 || oo.batch_engine > 2)
      throw Error{ASSS_ERR_INVALID_ARG, "batch_engine must be 0, 1 or 2"};
    if (oo.batch_engine != 2 && batch::applies(nsys, hs, nrhs, oo))
      return batch::run(nsys, hs, nrhs, B_dev, X_dev, oo, infos, maxr, s);
    if (oo.batch_engine == 1)
      throw Error{ASSS_ERR_INVALID_ARG, "the batch engine does not take these systems (it needs FGMRES from zero, no "
                                        "fixed inner steps, at most 4 right-hand sides, 16 deflation vectors and "
                                        "256 low-rank columns per system, the natural inner order, one device and "
                                        "one inner precision)"};
    // Work list: systems (all right-hand sides of one handle stay together, a
    // handle is not used from two threads), largest first, dealt to up to
    // batch_streams workers -- one host thread and one stream each -- so that
    // small, latency-bound systems run side by side on the GPU.
    std::map<asss_handle_t, std::vector<int>> by_handle;
    for (int sidx = 0; sidx < nsys; ++sidx)
      if (nrhs[sidx] > 0) by_handle[hs[sidx]].push_back(sidx);
    std::vector<std::pair<int64_t, std::vector<int>>> groups;
    for (auto& kv : by_handle) {
      int64_t work = 0;
      for (int sidx : kv.second) work += kv.first->n * (int64_t)nrhs[sidx];
      groups.push_back({work, kv.second});
    }
    std::sort(groups.begin(), groups.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    bool one_device = true;
    for (int sidx = 0; sidx < nsys; ++sidx) one_device &= hs[sidx]->device == hs[0]->device;
    // 16 by default: the systems' host round trips (Givens, stop checks) leave
    // gaps on each stream that the other streams fill (64 uneven systems:
    // 1 / 4 / 8 / 16 streams 0.62 / 0.32 / 0.26 / 0.22 s)
    const int want = oo.batch_streams > 0 ? oo.batch_streams : 16;
    const int nworkers = one_device ? std::min<int>(want, (int)groups.size()) : 1;
    std::vector<std::vector<int>> assign(std::max(1, nworkers));
    std::vector<int64_t> load(std::max(1, nworkers), 0);
    for (auto& g : groups) {
      const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[w] += g.first;
      assign[w].insert(assign[w].end(), g.second.begin(), g.second.end());
    }
    auto solve_system = [&](int sidx, hipStream_t st) -> asss_status_t {
      asss_handle_t h = hs[sidx];
      const int64_t n = h->n;
      asss_status_t worst_s = ASSS_OK;
      for (int j0 = 0; j0 < nrhs[sidx]; j0 += NRMAX) {
        const int nc = std::min(NRMAX, (int)nrhs[sidx] - j0);
        asss_info_t inf[NRMAX] = {};
        asss_status_t stt;
        // the 4-column inner kernels hold at most 16 deflation vectors and act
        // on the sliced J_tilde (the incomplete LDL^T solves one column at a time)
        if (nc >= 2 && oo.outer == ASSS_OUTER_FGMRES && h->k_eff <= 16 && !oo.use_x0 && !h->il.on) {
          const double* bs[NRMAX];
          double* xs[NRMAX];
          for (int c = 0; c < nc; ++c) {
            bs[c] = B_dev[sidx] + (int64_t)(j0 + c) * n;
            xs[c] = X_dev[sidx] + (int64_t)(j0 + c) * n;
          }
          stt = fgmres_block(h, nc, bs, xs, oo, inf, st);
        } else {
          stt = ASSS_OK;
          for (int c = 0; c < nc; ++c) {
            asss_status_t sc = outer_solve(h, false, B_dev[sidx] + (int64_t)(j0 + c) * n,
                                           X_dev[sidx] + (int64_t)(j0 + c) * n, oo, &inf[c], st);
            if (sc > stt) stt = sc;
          }
        }
        if (infos)
          for (int c = 0; c < nc; ++c) infos[(int64_t)sidx * maxr + j0 + c] = inf[c];
        if (stt > worst_s) worst_s = stt;
      }
      return worst_s;
    };
    if (nworkers <= 1) {
      asss_status_t worst = ASSS_OK;
      for (auto& list : assign)
        for (int sidx : list) {
          check_handle(hs[sidx]);
          worst = std::max(worst, solve_system(sidx, s));
        }
      return worst;
    }
    // worker streams (default priority) start after the caller's stream; the
    // caller's current device is restored on the way out
    struct DeviceRestore {
      int prev = -1;
      ~DeviceRestore() { if (prev >= 0) (void)hipSetDevice(prev); }
    } restore;
    HIPCHK(hipGetDevice(&restore.prev));
    HIPCHK(hipSetDevice(hs[0]->device));
    hipEvent_t ready = nullptr;
    HIPCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    std::vector<hipStream_t> streams(nworkers, nullptr);
    struct Outcome { asss_status_t status = ASSS_OK; int code = 0; std::string msg; };
    std::vector<Outcome> out(nworkers);
    try {
      HIPCHK(hipEventRecord(ready, s));
      for (int w = 0; w < nworkers; ++w) {
        HIPCHK(hipStreamCreateWithFlags(&streams[w], hipStreamNonBlocking));
        HIPCHK(hipStreamWaitEvent(streams[w], ready, 0));
      }
      std::vector<std::thread> threads;
      // a thread that cannot be started must not leave the started ones
      // unjoined: they are joined before the error goes on
      struct JoinAll {
        std::vector<std::thread>& t;
        ~JoinAll() { for (auto& x : t) if (x.joinable()) x.join(); }
      } join_all{threads};
      for (int w = 0; w < nworkers; ++w)
        threads.emplace_back([&, w]() {
          try {
            HIPCHK(hipSetDevice(hs[0]->device));
            for (int sidx : assign[w]) out[w].status = std::max(out[w].status, solve_system(sidx, streams[w]));
            HIPCHK(hipStreamSynchronize(streams[w]));
          } catch (const Error& e) {
            out[w].code = e.code;
            out[w].msg = e.msg;
          } catch (const HostError& e) {
            out[w].code = e.code;
            out[w].msg = e.msg;
          } catch (const std::bad_alloc&) {
            out[w].code = ASSS_ERR_OOM;
            out[w].msg = "host out of memory";
          } catch (const std::exception& e) {
            out[w].code = ASSS_ERR_INTERNAL;
            out[w].msg = e.what();
          } catch (...) {
            out[w].code = ASSS_ERR_INTERNAL;
            out[w].msg = "unknown error in a batched-solve worker";
          }
        });
      for (auto& t : threads) t.join();
    } catch (...) {
      for (hipStream_t st : streams)
        if (st) { (void)hipStreamSynchronize(st); (void)hipStreamDestroy(st); }
      (void)hipEventDestroy(ready);
      throw;
    }
    for (hipStream_t st : streams) (void)hipStreamDestroy(st);
    (void)hipEventDestroy(ready);
    asss_status_t worst = ASSS_OK;
    for (auto& r : out) {
      if (r.code != 0) throw Error{r.code, r.msg};
      worst = std::max(worst, r.status);
    }
    return worst;
  });
}

// ---- saved setups ---------------------------------------------------------
// File: "ASSSSAV1", then every array as an int64 count and its elements:
// A (rowptr, colind, values), the matching, D_r, D_c, S (rowptr, colind,
// values), the inner order (empty = natural) and the setup options
// (8-byte numbers: gamma, k, seed, inner_fp32, x_tol, x_maxit, lls_tol,
// lls_maxit, row_block, deflation, column form, S pattern kind).
static const char kSaveMagic[8] = {'A', 'S', 'S', 'S', 'S', 'A', 'V', '1'};

asss_status_t asss_save(asss_handle_t h, const char* path) {
  return guarded([&]() -> asss_status_t {
    check_handle(h);
    if (!path) throw Error{ASSS_ERR_INVALID_ARG, "null path"};
    if (h->il.on) throw Error{ASSS_ERR_INVALID_ARG, "saved setups are not provided for the incomplete LDL^T preconditioner"};
    std::vector<double> aval(h->dA.nnz);
    if (h->dA.nnz)
      HIPCHK(hipMemcpy(aval.data(), h->dA.val, h->dA.nnz * sizeof(double), hipMemcpyDeviceToHost));
    FILE* f = std::fopen(path, "wb");
    if (!f) throw Error{ASSS_ERR_INVALID_ARG, std::string("cannot write ") + path};
    bool ok = std::fwrite(kSaveMagic, 1, 8, f) == 8;
    auto put = [&](const void* p, int64_t cnt, size_t esz) {
      ok = ok && std::fwrite(&cnt, 8, 1, f) == 1;
      if (cnt > 0) ok = ok && std::fwrite(p, esz, (size_t)cnt, f) == (size_t)cnt;
    };
    put(h->Apat.ptr.data(), (int64_t)h->Apat.ptr.size(), 8);
    put(h->Apat.col.data(), (int64_t)h->Apat.col.size(), 4);
    put(aval.data(), (int64_t)aval.size(), 8);
    put(h->m.data(), (int64_t)h->m.size(), 4);
    put(h->Dr.data(), (int64_t)h->Dr.size(), 8);
    put(h->Dc.data(), (int64_t)h->Dc.size(), 8);
    put(h->S.ptr.data(), (int64_t)h->S.ptr.size(), 8);
    put(h->S.col.data(), (int64_t)h->S.col.size(), 4);
    put(h->S.val.data(), (int64_t)h->S.val.size(), 8);
    put(h->perm.data(), (int64_t)h->perm.size(), 4);
    const asss_setup_opts_t& o = h->opts;
    const double opt[12] = {o.gamma, (double)o.k, 0.0, (double)o.inner_fp32, o.x_tol, (double)o.x_maxit,
                            o.lls_tol, (double)o.lls_maxit, (double)h->J64.R, (double)o.deflation,
                            (double)h->skew_form, (double)o.s_pattern};
    put(opt, 12, 8);
    const uint64_t seed = o.lanczos_seed;  // exact, not through a double
    put(&seed, 1, 8);
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) throw Error{ASSS_ERR_INVALID_ARG, std::string("write failed: ") + path};
    return ASSS_OK;
  });
}

asss_status_t asss_load(const char* path, const asss_setup_opts_t* opts, void* hip_stream, asss_handle_t* out) {
  // the file is read and checked before any HIP call
  std::vector<int64_t> arp, srp;
  std::vector<int32_t> aci, sci, perm;
  std::vector<double> ava, sva, opt;
  std::vector<uint64_t> seed;
  Preset pre;
  asss_status_t st = guarded([&]() -> asss_status_t {
    if (!path || !out) throw Error{ASSS_ERR_INVALID_ARG, "null argument"};
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) throw Error{ASSS_ERR_INVALID_ARG, std::string("cannot open ") + path};
    char magic[8] = {};
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kSaveMagic, 8) == 0;
    auto get = [&](auto& v) {
      int64_t cnt = -1;
      ok = ok && std::fread(&cnt, 8, 1, f) == 1 && cnt >= 0 && cnt < ((int64_t)1 << 40);
      if (!ok) return;
      v.resize((size_t)cnt);
      if (cnt > 0) ok = std::fread(v.data(), sizeof(v[0]), (size_t)cnt, f) == (size_t)cnt;
    };
    get(arp); get(aci); get(ava); get(pre.m); get(pre.Dr); get(pre.Dc);
    get(srp); get(sci); get(sva); get(perm); get(opt); get(seed);
    std::fclose(f);
    if (!ok) throw Error{ASSS_ERR_INVALID_ARG, std::string("not a saved setup (or truncated): ") + path};
    const int64_t n = (int64_t)arp.size() - 1;
    bool sane = n >= 1 && opt.size() == 12 && seed.size() == 1 && aci.size() == ava.size() &&
                arp.back() == (int64_t)aci.size() && (int64_t)pre.m.size() == n && (int64_t)pre.Dr.size() == n &&
                (int64_t)pre.Dc.size() == n && (int64_t)srp.size() == n + 1 && srp[0] == 0 &&
                srp[n] == (int64_t)sci.size() && sci.size() == sva.size() && (perm.empty() || (int64_t)perm.size() == n);
    for (int64_t i = 0; sane && i < n; ++i) {  // S pattern: sorted, in range
      if (srp[i + 1] < srp[i]) { sane = false; break; }
      for (int64_t p = srp[i]; p < srp[i + 1]; ++p)
        if (sci[p] < 0 || sci[p] >= n || (p > srp[i] && sci[p] <= sci[p - 1])) { sane = false; break; }
    }
    for (int64_t j = 0; sane && j < n; ++j) sane = pre.m[j] >= 0 && pre.m[j] < n;
    if (!sane) throw Error{ASSS_ERR_INVALID_ARG, std::string("inconsistent saved setup: ") + path};
    pre.S.nrows = pre.S.ncols = n;
    pre.S.ptr = srp;
    pre.S.col = sci;
    pre.S.val = sva;
    return ASSS_OK;
  });
  if (st != ASSS_OK) return st;
  asss_setup_opts_t o;
  asss_default_setup_opts(&o);
  o.gamma = opt[0];
  o.k = (int32_t)opt[1];
  o.lanczos_seed = seed[0];
  o.inner_fp32 = (int32_t)opt[3];
  o.x_tol = opt[4];
  o.x_maxit = (int32_t)opt[5];
  o.lls_tol = opt[6];
  o.lls_maxit = (int32_t)opt[7];
  o.row_block = (int32_t)opt[8];
  o.deflation = (int32_t)opt[9];
  o.skew_form = (int32_t)opt[10];
  o.s_pattern = (int32_t)opt[11];
  if (!perm.empty()) {
    o.reorder = 3;
    o.inner_perm = perm.data();
  }
  if (opts) {  // from the caller: where the memory comes from and the log level
    o.allocator = opts->allocator;
    o.verbose = opts->verbose;
  }
  const asss_csr_t A{(int64_t)arp.size() - 1, (int64_t)aci.size(), arp.data(), aci.data(), ava.data()};
  return setup_impl(&A, &o, hip_stream, out, &pre);
}

asss_status_t asss_destroy(asss_handle_t h) {
  return guarded([&]() -> asss_status_t {
    if (!h) return ASSS_OK;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    batch::forget(h);
    delete h;
    return ASSS_OK;
  });
}

asss_status_t asss_ildl_factor(const asss_csr_t* M, double droptol, double fill, int32_t pivoting,
                               asss_ildl_t* out) {
  return guarded([&]() -> asss_status_t {
    if (!M || !out) throw Error{ASSS_ERR_INVALID_ARG, "null argument"};
    *out = nullptr;
    if (!(droptol >= 0.0) || !(fill > 0.0)) throw Error{ASSS_ERR_INVALID_ARG, "droptol must be >= 0 and fill > 0"};
    Csr Mh = validate_and_copy(M->n, M->nnz, M->rowptr, M->colind, M->val);
    std::unique_ptr<asss_ildl_s> f(new asss_ildl_s());
    IldlOpts o;
    o.droptol = droptol;
    o.fill = fill;
    o.pivoting = pivoting != 0;
    f->F = ildl_bunch_kaufman(Mh, o);
    f->S = ildl_scale(f->F);
    *out = f.release();
    return ASSS_OK;
  });
}

asss_status_t asss_ildl_get(asss_ildl_t f, int32_t which, void* dst, int64_t* count) {
  return guarded([&]() -> asss_status_t {
    if (!f || !count) throw Error{ASSS_ERR_INVALID_ARG, "null argument"};
    std::vector<unsigned char> bytes;
    int64_t cnt = 0;
    if (!ildl_export(f->F, f->S, which, bytes, cnt)) throw Error{ASSS_ERR_INVALID_ARG, "unknown array id"};
    *count = cnt;
    if (dst && !bytes.empty()) std::memcpy(dst, bytes.data(), bytes.size());
    return ASSS_OK;
  });
}

asss_status_t asss_ildl_destroy(asss_ildl_t f) {
  delete f;
  return ASSS_OK;
}

asss_status_t asss_get_handle_info(asss_handle_t h, asss_handle_info_t* out) {
  return guarded([&]() -> asss_status_t {
    if (!h || !out) throw Error{ASSS_ERR_INVALID_ARG, "null argument"};
    asss_handle_info_t i{};
    i.n = h->n;
    i.nnz_a = h->nnz_a;
    i.nnz_s = h->S.nnz();
    i.nnz_ahat = h->nnz_ahat;
    i.nh = h->U.nnz();
    i.lls_rows = h->lls_rows;
    i.lls_nnz = h->lls_nnz;
    i.k_eff = h->k_eff;
    i.rank_r = h->r;
    i.lls_its = h->lls_its;
    i.x_its = h->x_its;
    i.row_block = h->J64.R;
    i.nblocks = h->J64.nblocks;
    i.sell_entries_a = h->sell_a;
    i.sell_entries_b = h->sell_b;
    i.lls_relres = h->lls_relres;
    i.lls_kkt = h->lls_kkt;
    i.lanczos_orth_err = h->orth_err;
    i.narrow_b_columns = h->narrow_b;
    i.skew_form = h->skew_form;
    i.deflation_mode = h->k_eff == 0 ? 0 : (h->opts.deflation == 3 ? 3 : 1);
    i.reordered = h->d_perm ? 1 : 0;
    i.cross_pairs_natural = h->cross_natural;
    i.cross_pairs_used = h->cross_used;
    i.tune_n = (int32_t)std::min<size_t>(h->tuned.size(), 8);
    for (int c = 0; c < i.tune_n; ++c) {
      i.tune_rows[c] = h->tuned[c].first;
      i.tune_us[c] = h->tuned[c].second;
    }
    i.tune_s = h->tune_s;
    i.precond = h->il.on ? ASSS_PRECOND_ILDL : ASSS_PRECOND_DIAG;
    if (h->il.on) {
      i.ildl_n2x2 = h->il.F.n2x2;
      i.ildl_levels_lower = h->il.nlev_f;
      i.ildl_levels_upper = h->il.nlev_b;
      i.ildl_nnz_l = h->il.F.L.nnz();
      i.ildl_dropped = h->il.F.dropped;
    }
    i.step_threads = h->J32.threads > 0 ? h->J32.threads : WG;
    i.step_threads_fp64 = h->J64.threads > 0 ? h->J64.threads : WG;
    i.ildl_explicit = h->il.explicit_j ? 1 : 0;
    i.outer_ell = h->eAbar.nrows > 0 ? 1 : 0;
    *out = i;
    return ASSS_OK;
  });
}

asss_status_t asss_get_array(asss_handle_t h, int32_t which, void* dst, int64_t* count) {
  return guarded([&]() -> asss_status_t {
    if (!h || !count) throw Error{ASSS_ERR_INVALID_ARG, "null argument"};
    check_handle(h);
    const int64_t n = h->n;
    auto give = [&](const void* src, int64_t cnt, size_t esz) {
      *count = cnt;
      if (dst && cnt > 0) std::memcpy(dst, src, (size_t)cnt * esz);
    };
    auto give_dev = [&](const void* src, int64_t cnt, size_t esz) {
      *count = cnt;
      if (dst && cnt > 0) {
        HIPCHK(hipMemcpy(dst, src, (size_t)cnt * esz, hipMemcpyDeviceToHost));
      }
    };
    switch (which) {
      case ASSS_ARR_MATCH: give(h->m.data(), n, 4); break;
      case ASSS_ARR_DR: give(h->Dr.data(), n, 8); break;
      case ASSS_ARR_DC: give(h->Dc.data(), n, 8); break;
      case ASSS_ARR_S_ROWPTR: give(h->S.ptr.data(), n + 1, 8); break;
      case ASSS_ARR_S_COLIND: give(h->S.col.data(), h->S.nnz(), 4); break;
      case ASSS_ARR_S_VAL: give(h->S.val.data(), h->S.nnz(), 8); break;
      case ASSS_ARR_D: give(h->D.data(), n, 8); break;
      case ASSS_ARR_J_ROWPTR: give(h->U.ptr.data(), n + 1, 8); break;
      case ASSS_ARR_J_COLIND: give(h->U.col.data(), h->U.nnz(), 4); break;
      case ASSS_ARR_J_VAL: give(h->jval.data(), (int64_t)h->jval.size(), 8); break;
      case ASSS_ARR_Q: give_dev(h->d_Qorig, n * (int64_t)h->k_eff, 8); break;
      case ASSS_ARR_ALPHA: give(h->alpha.data(), (int64_t)h->alpha.size(), 8); break;
      case ASSS_ARR_X: give_dev(h->d_X, n * (int64_t)h->kr, 8); break;
      case ASSS_ARR_NEG: give(h->neg.data(), (int64_t)h->neg.size(), 4); break;
      default: {
        std::vector<unsigned char> bytes;
        int64_t cnt = 0;
        if (which < ASSS_ARR_ILDL_PERM || which > ASSS_ARR_SIGMA_R)
          throw Error{ASSS_ERR_INVALID_ARG, "unknown array id"};
        if (!h->il.on) {
          *count = 0;
          break;
        }
        ildl_export(h->il.F, h->il.Sc, which, bytes, cnt);
        *count = cnt;
        if (dst && !bytes.empty()) std::memcpy(dst, bytes.data(), bytes.size());
        break;
      }
    }
    return ASSS_OK;
  });
}

asss_status_t asss_apply(asss_handle_t h, int32_t op, const double* in, double* out,
                         const asss_solve_opts_t* o, int32_t* inner_its, void* hip_stream) {
  return guarded([&]() -> asss_status_t {
    check_handle(h);
    if (!in || !out) throw Error{ASSS_ERR_INVALID_ARG, "null vector"};
    hipStream_t s = (hipStream_t)hip_stream;
    asss_solve_opts_t oo = opts_or_default(o);
    const bool fp32 = (oo.inner_fp32 < 0) ? (h->opts.inner_fp32 != 0) : (oo.inner_fp32 != 0);
    const int64_t n = h->n;
    int its = 0;
    switch (op) {
      case ASSS_OP_SKEW:
      case ASSS_OP_DEFLATED: {
        // the operators act in the inner (block) order: gather, apply, scatter
        const double* vin = in;
        double* vout = out;
        if (h->d_perm) {
          permute_gather(n, h->d_perm, in, h->tmp, s);
          vin = h->tmp;
          vout = h->w;
        }
        if (h->il.on) {
          auto& il = h->il;
          if (fp32) ildl_sandwich<float>(il.Lb32, il.J32, il.Lf32, vin, vout, il.t32[0], il.t32[1], il.t32[2], il.t32[3], s);
          else ildl_sandwich<double>(il.Lb64, il.J64, il.Lf64, vin, vout, il.t64[0], il.t64[1], il.t64[2], il.t64[3], s);
        } else if (fp32) {
          cast_d2f(n, vin, h->mb32.w[0], s);
          skew_spmv<float>(h->J32, h->mb32.w[0], h->mb32.w[1], s);
          cast_f2d(n, h->mb32.w[1], vout, s);
        } else {
          skew_spmv<double>(h->J64, vin, vout, s);
        }
        if (op == ASSS_OP_DEFLATED && h->k_eff > 0) {
          // out -= Q (S_k (Q^T in))
          double* d = h->d_small + SM_T;
          gemm_tn<double, double>(n, h->k_eff, h->d_Q64, n, vin, 1, d, nullptr, h->red, 3, s);
          HIPCHK(hipMemcpyAsync(h->h_small, d, h->k_eff * sizeof(double), hipMemcpyDeviceToHost, s));
          HIPCHK(hipStreamSynchronize(s));
          std::vector<double> c(h->k_eff, 0.0);
          for (int l = 0; l < h->k_eff; ++l) {
            if (l + 1 < h->k_eff) c[l] += h->alpha[l] * h->h_small[l + 1];
            if (l >= 1) c[l] -= h->alpha[l - 1] * h->h_small[l - 1];
          }
          HIPCHK(hipMemcpyAsync(d, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice, s));
          gemv_acc(n, h->k_eff, h->d_Q64, n, d, -1.0, vout, s);
        }
        if (h->d_perm) permute_scatter(n, h->d_perm, vout, out, s);
        break;
      }
      case ASSS_OP_OUTER: outer_op(h, in, out, s); break;
      case ASSS_OP_OUTER_T: outer_op_T(h, in, out, s); break;
      case ASSS_OP_MRS:
        its = inner_solve(h, fp32, in, out, +1, oo.inner_tol, oo.inner_maxit, oo.fixed_inner_steps, s);
        break;
      case ASSS_OP_PREC: its = prec_apply(h, fp32, in, out, oo, s); break;
      case ASSS_OP_PREC_T: its = prec_apply_T(h, fp32, in, out, oo, s); break;
      case ASSS_OP_A: spmv(h->dA, in, out, nullptr, nullptr, 0, nullptr, s); break;
      case ASSS_OP_AT: spmv(h->dAt, in, out, nullptr, nullptr, 0, nullptr, s); break;
      default: throw Error{ASSS_ERR_INVALID_ARG, "unknown operator id"};
    }
    HIPCHK(hipStreamSynchronize(s));
    if (inner_its) *inner_its = its;
    return ASSS_OK;
  });
}

}  // extern "C"
