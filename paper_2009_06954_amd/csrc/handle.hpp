// Host-side internals shared by the library's sources: error type, roctx
// ranges, the device arena and the handle (the opaque asss_handle_s of
// include/asss.h).
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cstddef>
#include <string>
#include <utility>
#include <vector>

#include "../../include/asss.h"
#include "host_setup.hpp"
#include "ildl_host.hpp"
#include "ildl_kernels.hpp"
#include "kernels.hpp"
#include "outer_kernels.hpp"

namespace asss {
namespace host {

// roctx range around a phase (setup stages, a solve, an outer step, an inner
// solve): visible in a rocprofv3 --marker-trace, a no-op call otherwise.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

struct Error {
  int code;
  std::string msg;
};

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw Error{e_ == hipErrorOutOfMemory ? ASSS_ERR_OOM : ASSS_ERR_HIP,                  \
                  std::string(#expr) + ": " + hipGetErrorString(e_)};                       \
  } while (0)

// leading part of MrsState read back by the host: its, status, ..., relres_max
constexpr size_t kStateHead = offsetof(MrsState, relres_max) + sizeof(double);
inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Device allocations owned by a handle.
struct DevArena {
  std::vector<void*> ptrs;
  asss_allocator_t al{};  // al.alloc == nullptr: hipMalloc / hipFree
  DevArena() = default;
  explicit DevArena(const asss_allocator_t& a) : al(a) {}
  DevArena(const DevArena&) = delete;
  DevArena& operator=(const DevArena&) = delete;
  template <typename T>
  T* alloc(int64_t count) {
    if (count <= 0) count = 1;
    const size_t bytes = (size_t)count * sizeof(T);
    void* p = nullptr;
    if (al.alloc) {
      p = al.alloc(bytes, al.ctx);
      if (!p) throw Error{ASSS_ERR_OOM, "the caller's allocator returned no memory"};
    } else {
      const hipError_t e = hipMalloc(&p, bytes);
      if (e == hipErrorOutOfMemory) throw Error{ASSS_ERR_OOM, "hipMalloc: out of device memory"};
      HIPCHK(e);
    }
    ptrs.push_back(p);
    return (T*)p;
  }
  template <typename T>
  T* upload(const std::vector<T>& v, hipStream_t s) {
    T* p = alloc<T>((int64_t)v.size());
    if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return p;
  }
  void give_back(void* p) {
    if (al.alloc) al.free(p, al.ctx);
    else (void)hipFree(p);
  }
  void release(void* p) {
    auto it = std::find(ptrs.begin(), ptrs.end(), p);
    if (it != ptrs.end()) {
      give_back(*it);
      ptrs.erase(it);
    }
  }
  ~DevArena() {
    for (void* p : ptrs) give_back(p);
  }
};


// Device copies of the host structures (definitions in asss.hip).
int lanes_for(const Csr& M);
DCsr upload_csr(DevArena& ar, const Csr& M, hipStream_t s);
struct SkewLayout {
  DSkew<double> J64;
  DSkew<float> J32;
  std::vector<const void*> bufs;
  int64_t a_entries = 0, b_entries = 0;
  int narrow = 0;
  int form = SKEW_WIDE;
};
SkewLayout upload_layout(DevArena& ar, const SkewSell& sell, hipStream_t s, int step_threads);

}  // namespace host
}  // namespace asss

struct asss_handle_s {
  using DevArena = asss::host::DevArena;
  using Csr = asss::Csr;
  using DCsr = asss::DCsr;
  template <typename T>
  using DSkew = asss::DSkew<T>;
  template <typename T>
  using MrsBufs = asss::MrsBufs<T>;
  using MrsState = asss::MrsState;
  using Reducer = asss::Reducer;
  static constexpr int NRMAX = asss::NRMAX;
  uint64_t uid = 0;  // unique per handle of the process (keys of kept batch data)
  int device = 0;
  int64_t n = 0;
  asss_setup_opts_t opts{};
  DevArena ar;  // every device buffer of the handle (caller's allocator if given)
  // host data kept for inspection
  std::vector<int32_t> m;
  std::vector<double> Dr, Dc, D, Omega, alpha;
  Csr S, U;
  std::vector<double> jval;
  std::vector<int32_t> neg;
  int64_t nnz_a = 0, nnz_ahat = 0, lls_rows = 0, lls_nnz = 0;
  int lls_its = 0, x_its = 0;
  double lls_relres = 0, lls_kkt = 0;
  int64_t sell_a = 0, sell_b = 0;
  int k_eff = 0, r = 0, kr = 0;
  double setup_host_s = 0, setup_device_s = 0;
  // device data
  DCsr dA, dAt, dAbar, dAbarT, dS, dSt;
  // sliced ELL copies of the outer operator's factors (nrows 0: CSR only)
  asss::DSell eAbar, eAbarT, eS, eSt;
  Csr Apat;  // pattern of A as stored (explicit zeros dropped), for value updates
  int32_t* d_m = nullptr;
  double *d_drp = nullptr, *d_om = nullptr, *d_dc = nullptr;
  DSkew<double> J64;
  DSkew<float> J32;
  std::vector<const void*> lay_bufs;  // buffers of the J64 / J32 layout
  // row-block autotuner: candidates timed at setup (row_block, us per inner step)
  std::vector<std::pair<int, double>> tuned;
  double tune_s = 0.0;
  // a deflation basis given by the caller (setup option q_basis), until device_setup
  std::vector<double> q_given, alpha_given;
  // inner system in block order: row i of the inner system is row perm[i]
  std::vector<int32_t> perm;
  int32_t* d_perm = nullptr;  // null when the natural order is kept
  int64_t cross_natural = 0, cross_used = 0;
  int narrow_b = 0;  // part-b columns stored as 16-bit deltas
  int skew_form = 0; // column form of the sliced J_tilde (SKEW_*)
  double* d_Qorig = nullptr;  // Q_k in the original order (U_bar, export)
  double* d_Q64 = nullptr;    // Q_k in the inner (block) order
  float* d_Q32 = nullptr;
  double* d_Qs64 = nullptr;   // sliced copies for the inner iteration kernel
  float* d_Qs32 = nullptr;
  double* d_G64 = nullptr;    // Q_k^T Q_k of the FP64 and of the FP32 copy (k x k)
  double* d_G32 = nullptr;
  double* d_alpha = nullptr;
  double orth_err = 0.0;      // max |Q_k^T Q_k - I|
  double* d_Ubar = nullptr;   // n x kr column-major
  double* d_X = nullptr;      // n x kr column-major
  double* d_Mf = nullptr;     // C^-1 Sigma (kr x kr row-major)
  double* d_Ma = nullptr;     // Sigma^T C^-T (kr x kr row-major)
  MrsBufs<double> mb64{};
  MrsBufs<float> mb32{};
  MrsState* d_state = nullptr;
  Reducer red;
  double* d_small = nullptr;  // SM_SIZE doubles of scalars (layout above)
  double* d_hess = nullptr;   // NRMAX Hessenberg workspaces of HESS_SLOT doubles
  int* d_flag = nullptr;
  double* h_small = nullptr;  // pinned
  // outer workspace
  int m_alloc = 0;
  double *V = nullptr, *Z = nullptr;
  // lockstep columns of a batched solve (up to NRMAX) and the 4-column inner buffers
  struct MultiCol {
    double *V = nullptr, *Z = nullptr, *bchk = nullptr, *xchk = nullptr, *rv = nullptr;
  } mcol[NRMAX];
  int m_alloc_multi = 0;
  double *pin = nullptr, *pout = nullptr;
  MrsBufs<double> mb4_64{};
  MrsBufs<float> mb4_32{};
  double *w = nullptr, *t1 = nullptr, *xchk = nullptr, *bchk = nullptr, *rv = nullptr, *tmp = nullptr;
  double *x0r = nullptr, *x0d = nullptr;  // residual and correction of a solve from x0
  bool no_alloc = false;  // a call of asss_solve_noalloc is running: never allocate
  int last_inner = 0;
  // HIP events bracketing each chunk of back-to-back mrs iteration kernels
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double prof_s = 0.0;
  int prof_launches = 0;

  // The general incomplete LDL^T preconditioner (setup option precond = 1,
  // paper Sec. 3): the scaled system lives in the factorization's positions.
  struct Ildl {
    bool on = false;
    bool explicit_j = false;  // J_tilde formed at setup: the inner solve runs the sliced kernels
    double* A_rows = nullptr;   // with explicit_j: A_chk = Lcal^-1 A_hat_p Lcal^-T row-major
    double* AT_rows = nullptr;  // and A_chk^T row-major (A_chk column-major)
    asss::IldlOpts opts;
    asss::IldlFactor F;     // perm, L, pivot blocks (host copy, for inspection)
    asss::IldlScaled Sc;    // Lcal, U_r, Sigma_r
    int32_t nlev_f = 0, nlev_b = 0;
    asss::DTri<double> Lf64, Lb64;  // Lcal (forward solves) and Lcal^T (backward)
    asss::DTri<float> Lf32, Lb32;
    asss::DCsr32<double> J64, Ap, ApT;  // J_hat, A_hat and A_hat^T in positions
    asss::DCsr32<float> J32;
    int32_t* d_perm = nullptr;  // position p -> index perm[p] of Abar
    int32_t* d_mp = nullptr;    // m[perm[p]]: row of A behind position p
    double* d_drp = nullptr;    // Dr[m[perm[p]]]
    double* d_ones = nullptr;
    double* t64[4] = {nullptr, nullptr, nullptr, nullptr};
    float* t32[4] = {nullptr, nullptr, nullptr, nullptr};
    double *y64 = nullptr, *z64 = nullptr, *u64 = nullptr;
    float *y32 = nullptr, *z32 = nullptr, *u32 = nullptr;
  } il;

  ~asss_handle_s() {
    if (h_small) (void)hipHostFree(h_small);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }
};

