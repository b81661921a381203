// Setup of the general incomplete LDL^T preconditioner (paper Sec. 3): the
// symmetric and skew parts of A_hat, the Bunch-Kaufman factorization of
// M_hat on the host, the scaled factor and low-rank term, and the device
// copies that the triangular-solve kernels read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "handle.hpp"
#include "ildl_host.hpp"
#include "ildl_kernels.hpp"
#include "ildl_setup.hpp"

namespace asss {
namespace host {

namespace {

// Lanes per row for rows of at most `longest` entries, `rows` rows solved
// side by side: about four entries per lane, fewer lanes when the rows would
// not fit the workgroup in one pass.
int lanes_per_row(int64_t longest, int64_t rows, int64_t width) {
  int lpr = 1;
  while (lpr < 64 && (int64_t)lpr * 4 < longest) lpr *= 2;
  while (lpr > 1 && rows * lpr > width) lpr /= 2;
  return lpr;
}

// A triangular CSR (rows over positions, diagonal stored in each row) in
// schedule order: the rows level by level with their inverse diagonals, and
// each level's off-diagonal entries as one padded block (slot-major within an
// entry index, see DTri), the lanes per row chosen per level.  Uploaded in
// FP64 and FP32 (index arrays shared).
void upload_tri(DevArena& ar, const Csr& T, bool lower, DTri<double>& d64, DTri<float>& d32, int32_t& nlev,
                hipStream_t s) {
  const int64_t n = T.nrows;
  LevelSchedule L = level_schedule(T, lower);
  nlev = L.nlevels();
  // one wave takes the whole solve when every level fits its 64 lanes in one
  // pass with at most four entries per lane (a level then costs one round of
  // LDS gathers); else the workgroup, with lanes per row chosen for it
  std::vector<int32_t> lpr(nlev), lw(nlev), lbase(nlev);
  std::vector<int64_t> longest(nlev, 0);
  int wave = 1;
  for (int32_t l = 0; l < nlev; ++l) {
    for (int32_t e = L.ptr[l]; e < L.ptr[l + 1]; ++e) {
      const int32_t i = L.rows[e];
      longest[l] = std::max<int64_t>(longest[l], T.ptr[i + 1] - T.ptr[i] - 1);  // off-diagonal entries
    }
    int lw1 = 1;
    while (lw1 < 64 && (int64_t)lw1 * 4 < longest[l]) lw1 *= 2;
    if ((int64_t)(L.ptr[l + 1] - L.ptr[l]) * lw1 > 64 || (int64_t)lw1 * 4 < longest[l]) wave = 0;
  }
  std::vector<double> dinv(n, 0.0);
  int64_t total = 0;
  for (int32_t l = 0; l < nlev; ++l) {
    const int64_t rows = L.ptr[l + 1] - L.ptr[l];
    lpr[l] = lanes_per_row(longest[l], rows, wave ? 64 : TRI_WG);
    lw[l] = (int32_t)((longest[l] + lpr[l] - 1) / lpr[l]);
    lbase[l] = (int32_t)total;
    total += (int64_t)lw[l] * rows * lpr[l];
    if (total >= (int64_t)INT32_MAX - TRI_WG)
      throw Error{ASSS_ERR_INVALID_ARG, "the padded incomplete factor has 2^31 entries or more"};
  }
  const int32_t pad_col = L.rows[0];  // a row of level 0: solved before any level reads it
  std::vector<int32_t> ecol(total + TRI_WG, pad_col);
  std::vector<double> eval(total + TRI_WG, 0.0);
  for (int32_t l = 0; l < nlev; ++l) {
    const int64_t nslots = (int64_t)(L.ptr[l + 1] - L.ptr[l]) * lpr[l];
    for (int32_t e = L.ptr[l]; e < L.ptr[l + 1]; ++e) {
      const int32_t i = L.rows[e];
      const int64_t r_local = e - L.ptr[l];
      int64_t k = 0;
      for (int64_t q = T.ptr[i]; q < T.ptr[i + 1]; ++q) {
        if (T.col[q] == i) {
          dinv[e] = T.val[q];
          continue;
        }
        const int64_t j = k % lpr[l], t = k / lpr[l];
        const int64_t idx = lbase[l] + t * nslots + r_local * lpr[l] + j;
        ecol[idx] = T.col[q];
        eval[idx] = T.val[q];
        ++k;
      }
      if (dinv[e] == 0.0) throw Error{ASSS_ERR_INTERNAL, "the scaled incomplete factor has a zero diagonal entry"};
    }
  }
  // the diagonal is stored inverted (FP64, rounded once; the FP32 copy is the
  // FP32 inverse of the FP32 diagonal)
  std::vector<float> eval32(eval.begin(), eval.end()), dinv32(n);
  for (int64_t e = 0; e < n; ++e) {
    dinv32[e] = 1.0f / (float)dinv[e];
    dinv[e] = 1.0 / dinv[e];
  }
  const int32_t* dlp = ar.upload(L.ptr, s);
  const int32_t* dlpr = ar.upload(lpr, s);
  const int32_t* dlw = ar.upload(lw, s);
  const int32_t* dlb = ar.upload(lbase, s);
  const int32_t* drow = ar.upload(L.rows, s);
  const int32_t* dcol = ar.upload(ecol, s);
  d64.n = d32.n = (int32_t)n;
  d64.nlev = d32.nlev = nlev;
  d64.wave = d32.wave = wave;
  d64.lev_ptr = d32.lev_ptr = dlp;
  d64.lev_lpr = d32.lev_lpr = dlpr;
  d64.lev_w = d32.lev_w = dlw;
  d64.lev_base = d32.lev_base = dlb;
  d64.row = d32.row = drow;
  d64.ecol = d32.ecol = dcol;
  d64.eval = ar.upload(eval, s);
  d64.dinv = ar.upload(dinv, s);
  d32.eval = ar.upload(eval32, s);
  d32.dinv = ar.upload(dinv32, s);
}

template <typename T>
DCsr32<T> upload_csr32(DevArena& ar, const Csr& M, const int32_t** shared_ptr_col, hipStream_t s) {
  if (M.nnz() >= (int64_t)INT32_MAX) throw Error{ASSS_ERR_INVALID_ARG, "an operator has 2^31 entries or more"};
  DCsr32<T> d;
  d.n = (int32_t)M.nrows;
  int64_t longest = 0;
  for (int64_t i = 0; i < M.nrows; ++i) longest = std::max<int64_t>(longest, M.ptr[i + 1] - M.ptr[i]);
  // up to two passes of the workgroup over the rows
  d.lpr = lanes_per_row(longest, M.nrows, 2 * TRI_WG);
  if (shared_ptr_col && shared_ptr_col[0]) {
    d.ptr = shared_ptr_col[0];
    d.col = shared_ptr_col[1];
  } else {
    std::vector<int32_t> ptr(M.ptr.begin(), M.ptr.end());
    d.ptr = ar.upload(ptr, s);
    d.col = ar.upload(M.col, s);
    if (shared_ptr_col) {
      shared_ptr_col[0] = d.ptr;
      shared_ptr_col[1] = d.col;
    }
  }
  std::vector<T> v(M.val.begin(), M.val.end());
  d.val = ar.upload(v, s);
  return d;
}

}  // namespace

void ildl_setup(asss_handle_s* h, const Csr& Ahat, hipStream_t s) {
  auto& il = h->il;
  const int64_t n = h->n;
  Csr M, J;
  symmetric_skew_split(Ahat, M, J);
  il.F = ildl_bunch_kaufman(M, il.opts);
  il.Sc = ildl_scale(il.F);
  il.on = true;
  // the positions of the factorization are the order of the scaled system
  const std::vector<int32_t>& perm = il.F.perm;
  Csr Ap = permute_symmetric(Ahat, perm);
  Csr Jp = permute_symmetric(J, perm);
  upload_tri(h->ar, il.Sc.Lc, true, il.Lf64, il.Lf32, il.nlev_f, s);
  upload_tri(h->ar, il.Sc.LcT, false, il.Lb64, il.Lb32, il.nlev_b, s);
  const int32_t* jpc[2] = {nullptr, nullptr};
  il.J64 = upload_csr32<double>(h->ar, Jp, jpc, s);
  il.J32 = upload_csr32<float>(h->ar, Jp, jpc, s);
  il.Ap = upload_csr32<double>(h->ar, Ap, nullptr, s);
  il.ApT = upload_csr32<double>(h->ar, transpose(Ap), nullptr, s);
  std::vector<int32_t> mp(n);
  std::vector<double> drp(n);
  for (int64_t p = 0; p < n; ++p) {
    mp[p] = h->m[perm[p]];
    drp[p] = h->Dr[h->m[perm[p]]];
  }
  il.d_perm = h->ar.upload(perm, s);
  il.d_mp = h->ar.upload(mp, s);
  il.d_drp = h->ar.upload(drp, s);
  il.d_ones = h->ar.upload(std::vector<double>(n, 1.0), s);
  for (int b = 0; b < 4; ++b) {
    il.t64[b] = h->ar.alloc<double>(n);
    il.t32[b] = h->ar.alloc<float>(n);
  }
  il.y64 = h->ar.alloc<double>(n);
  il.z64 = h->ar.alloc<double>(n);
  il.u64 = h->ar.alloc<double>(n);
  il.y32 = h->ar.alloc<float>(n);
  il.z32 = h->ar.alloc<float>(n);
  il.u32 = h->ar.alloc<float>(n);
  HIPCHK(hipStreamSynchronize(s));
}

namespace {

// D[i n + j] = (C[j n + i] - C[i n + j]) / 2 for column-major C (n x n):
// row-major and exactly skew (fl(a - b) = -fl(b - a)).  Tiles of 32 x 32
// through LDS so that both the reads and the writes are coalesced.
// D = C^T (both n x n): tiles of 32 x 32 through LDS.
__global__ void k_transpose(int64_t n, const double* __restrict__ C, double* __restrict__ D) {
  __shared__ double tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.y * 32, j0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int a = ty; a < 32; a += 8) {
    const int64_t j = j0 + a, i = i0 + tx;
    tile[a][tx] = (j < n && i < n) ? C[j * n + i] : 0.0;
  }
  __syncthreads();
  for (int a = ty; a < 32; a += 8) {
    const int64_t i = i0 + a, j = j0 + tx;
    if (i < n && j < n) D[i * n + j] = tile[tx][a];
  }
}

__global__ void k_skew_part_rowmajor(int64_t n, const double* __restrict__ C, double* __restrict__ D) {
  __shared__ double tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.y * 32, j0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows of 32
  // tile[a][b] = C[(j0 + a) n + i0 + b] = J[i0 + b][j0 + a]
  for (int a = ty; a < 32; a += 8) {
    const int64_t j = j0 + a, i = i0 + tx;
    tile[a][tx] = (j < n && i < n) ? C[j * n + i] : 0.0;
  }
  __syncthreads();
  // row i = i0 + a, column j = j0 + tx: (C[j n + i] - C[i n + j]) / 2
  for (int a = ty; a < 32; a += 8) {
    const int64_t i = i0 + a, j = j0 + tx;
    if (i < n && j < n) D[i * n + j] = 0.5 * (tile[tx][a] - C[i * n + j]);
  }
}

}  // namespace

void ildl_explicit_jtilde(asss_handle_s* h, hipStream_t s) {
  auto& il = h->il;
  const int64_t n = h->n;
  // up to 512 columns at a time, one workgroup each
  const int64_t B = std::min<int64_t>(n, 512);
  // every buffer first, so that a failed allocation leaves nothing behind
  double *C = nullptr, *scratch = nullptr, *D64 = nullptr, *CA = nullptr;
  float* D32 = nullptr;
  try {
    C = h->ar.alloc<double>(n * n);
    scratch = h->ar.alloc<double>(4 * n * B);
    D64 = h->ar.alloc<double>(n * n);
    D32 = h->ar.alloc<float>(n * n);
    CA = h->ar.alloc<double>(n * n);
  } catch (...) {
    for (void* p : {(void*)C, (void*)scratch, (void*)D64, (void*)D32, (void*)CA})
      if (p) h->ar.release(p);
    throw;
  }
  for (int64_t j0 = 0; j0 < n; j0 += B)
    ildl_columns(il.Lb64, il.J64, il.Lf64, j0, (int)std::min<int64_t>(B, n - j0), C, scratch, s);
  const unsigned gt = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(k_skew_part_rowmajor, dim3(gt, gt), dim3(256), 0, s, n, C, D64);
  cast_d2f(n * n, D64, D32, s);
  HIPCHK(hipStreamSynchronize(s));
  // the outer operator the same way: A_chk column-major from the columns
  // (which is A_chk^T row-major) and its transpose (A_chk row-major)
  for (int64_t j0 = 0; j0 < n; j0 += B)
    ildl_columns(il.Lb64, il.Ap, il.Lf64, j0, (int)std::min<int64_t>(B, n - j0), CA, scratch, s);
  double* RA = C;  // the columns of J_tilde are no longer needed
  hipLaunchKernelGGL(k_transpose, dim3(gt, gt), dim3(256), 0, s, n, CA, RA);
  HIPCHK(hipStreamSynchronize(s));
  il.A_rows = RA;
  il.AT_rows = CA;
  h->ar.release(scratch);
  // row blocks of R rows (a multiple of 8), at most about 512 blocks, one
  // wave per row within a block
  const int64_t R = std::max<int64_t>(8, 8 * ((n + 8 * 512 - 1) / (8 * 512)));
  const int32_t nb = (int32_t)((n + R - 1) / R);
  if (nb > h->red.max_groups) throw Error{ASSS_ERR_INTERNAL, "more row blocks than reduction slots"};
  DSkew<double> J64;
  DSkew<float> J32;
  J64.n = J32.n = (int32_t)n;
  J64.R = J32.R = (int32_t)R;
  J64.nblocks = J32.nblocks = nb;
  J64.dense = D64;
  J32.dense = D32;
  J64.dense_ld = J32.dense_ld = n;
  h->J64 = J64;
  h->J32 = J32;
  h->lay_bufs = {D64, D32};
  il.explicit_j = true;
}

}  // namespace host
}  // namespace asss
