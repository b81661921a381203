// Host-side preprocessing of the ASSS scheme: validation, maximum product
// matching and scaling (paper Sec. 2, eq. mc64), the least-squares system for
// the skew-symmetrizer (Sec. 2 eqs. 1-2, App. A), A_hat = Abar S and its
// splitting (Sec. 3), and the sliced layout of J_tilde used by the kernels.
#include "host_setup.hpp"

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <limits>
#include <numeric>
#include <queue>
#include <thread>

#include "../../include/asss.h"

namespace asss {

int num_threads() {
  unsigned h = std::thread::hardware_concurrency();
  if (h == 0) h = 4;
  return (int)std::min<unsigned>(h, 16);
}

static void parallel_chunks(int64_t n, int64_t min_parallel, const std::function<void(int64_t, int64_t)>& f) {
  if (n <= 0) return;
  int nt = num_threads();
  if (n < min_parallel || nt <= 1) {
    f(0, n);
    return;
  }
  int64_t chunks = std::min<int64_t>(n, (int64_t)nt * 8);
  std::atomic<int64_t> next(0);
  auto worker = [&]() {
    for (;;) {
      int64_t c = next.fetch_add(1);
      if (c >= chunks) break;
      int64_t lo = n * c / chunks, hi = n * (c + 1) / chunks;
      f(lo, hi);
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(worker);
  worker();
  for (auto& t : th) t.join();
}

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& f) { parallel_chunks(n, 4096, f); }

// one task per index (coarse tasks such as graph parts)
static void parallel_tasks(int64_t n, const std::function<void(int64_t, int64_t)>& f) { parallel_chunks(n, 2, f); }

static void fail(int code, const std::string& msg) { throw HostError{code, msg}; }

Csr validate_and_copy(int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colind,
                      const double* val) {
  if (n < 1 || n > (int64_t)std::numeric_limits<int32_t>::max() - 1)
    fail(ASSS_ERR_INVALID_ARG, "n must be in [1, 2^31-2]");
  if (!rowptr || (nnz > 0 && (!colind || !val))) fail(ASSS_ERR_INVALID_ARG, "null CSR array");
  if (rowptr[0] != 0 || rowptr[n] != nnz) fail(ASSS_ERR_INVALID_CSR, "rowptr[0] != 0 or rowptr[n] != nnz");
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) fail(ASSS_ERR_INVALID_CSR, "rowptr decreases");
  std::atomic<int> bad(0);
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        int32_t c = colind[p];
        if (c < 0 || c >= n) { bad = 1; return; }
        if (p > rowptr[i] && colind[p - 1] >= c) { bad = 2; return; }
        if (!std::isfinite(val[p])) { bad = 3; return; }
      }
    }
  });
  if (bad == 1) fail(ASSS_ERR_INVALID_CSR, "column index out of range");
  if (bad == 2) fail(ASSS_ERR_INVALID_CSR, "columns not strictly increasing within a row");
  if (bad == 3) fail(ASSS_ERR_NONFINITE, "A has a non-finite value");
  Csr A;
  A.nrows = A.ncols = n;
  A.ptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    int64_t c = 0;
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) c += (val[p] != 0.0);
    A.ptr[i + 1] = A.ptr[i] + c;
  }
  A.col.resize(A.ptr[n]);
  A.val.resize(A.ptr[n]);
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      int64_t q = A.ptr[i];
      for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
        if (val[p] != 0.0) { A.col[q] = colind[p]; A.val[q] = val[p]; ++q; }
    }
  });
  return A;
}

Csr map_values_onto(const Csr& pat, int64_t n, int64_t nnz, const int64_t* rowptr,
                    const int32_t* colind, const double* val) {
  if (n != pat.nrows) fail(ASSS_ERR_INVALID_ARG, "n differs from the matrix given at setup");
  if (!rowptr || (nnz > 0 && (!colind || !val))) fail(ASSS_ERR_INVALID_ARG, "null CSR array");
  if (rowptr[0] != 0 || rowptr[n] != nnz) fail(ASSS_ERR_INVALID_CSR, "rowptr[0] != 0 or rowptr[n] != nnz");
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) fail(ASSS_ERR_INVALID_CSR, "rowptr decreases");
  Csr A;
  A.nrows = A.ncols = n;
  A.ptr = pat.ptr;
  A.col = pat.col;
  A.val.assign(pat.col.size(), 0.0);
  std::atomic<int> bad(0);
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi && !bad; ++i) {
      int64_t q = pat.ptr[i];
      const int64_t qe = pat.ptr[i + 1];
      for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        const int32_t c = colind[p];
        if (c < 0 || c >= n) { bad = 1; return; }
        if (p > rowptr[i] && colind[p - 1] >= c) { bad = 2; return; }
        if (!std::isfinite(val[p])) { bad = 3; return; }
        while (q < qe && pat.col[q] < c) ++q;
        if (q < qe && pat.col[q] == c) {
          A.val[q] = val[p];
        } else if (val[p] != 0.0) {
          bad = 4;
          return;
        }
      }
    }
  });
  if (bad == 1) fail(ASSS_ERR_INVALID_CSR, "column index out of range");
  if (bad == 2) fail(ASSS_ERR_INVALID_CSR, "columns not strictly increasing within a row");
  if (bad == 3) fail(ASSS_ERR_NONFINITE, "A has a non-finite value");
  if (bad == 4) fail(ASSS_ERR_INVALID_ARG, "a nonzero outside the pattern given at setup");
  return A;
}

Csr transpose(const Csr& A) {
  Csr T;
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.ptr.assign(T.nrows + 1, 0);
  for (int32_t c : A.col) T.ptr[c + 1]++;
  for (int64_t i = 0; i < T.nrows; ++i) T.ptr[i + 1] += T.ptr[i];
  T.col.resize(A.nnz());
  bool has_val = !A.val.empty();
  if (has_val) T.val.resize(A.nnz());
  std::vector<int64_t> cur(T.ptr.begin(), T.ptr.end() - 1);
  for (int64_t i = 0; i < A.nrows; ++i)       // row order keeps columns of T sorted
    for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
      int64_t q = cur[A.col[p]]++;
      T.col[q] = (int32_t)i;
      if (has_val) T.val[q] = A.val[p];
    }
  return T;
}

// ---------------------------------------------------------------------------
// Matching (Sec. 2, eq. mc64)
// ---------------------------------------------------------------------------

std::vector<int32_t> max_product_matching(const Csr& A) {
  const int64_t n = A.nrows;
  Csr C = transpose(A);  // row j of C = column j of A
  // column-normalised costs c_ij = log(colmax_j) - log|a_ij| >= 0
  std::vector<double> cost(C.nnz());
  for (int64_t j = 0; j < n; ++j) {
    double cm = 0.0;
    for (int64_t p = C.ptr[j]; p < C.ptr[j + 1]; ++p) cm = std::max(cm, std::fabs(C.val[p]));
    if (C.ptr[j] == C.ptr[j + 1]) fail(ASSS_ERR_STRUCTURALLY_SINGULAR, "empty column");
    double lcm = std::log(cm);
    for (int64_t p = C.ptr[j]; p < C.ptr[j + 1]; ++p) cost[p] = lcm - std::log(std::fabs(C.val[p]));
  }
  const double INF = std::numeric_limits<double>::infinity();
  std::vector<double> u(n, INF), v(n, 0.0);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t p = C.ptr[j]; p < C.ptr[j + 1]; ++p) u[C.col[p]] = std::min(u[C.col[p]], cost[p]);
  for (int64_t i = 0; i < n; ++i)
    if (u[i] == INF) fail(ASSS_ERR_STRUCTURALLY_SINGULAR, "empty row");
  std::vector<int32_t> row_mate(n, -1), col_mate(n, -1);
  // greedy matching on tight edges
  for (int64_t j = 0; j < n; ++j)
    for (int64_t p = C.ptr[j]; p < C.ptr[j + 1]; ++p) {
      int32_t i = C.col[p];
      if (row_mate[i] < 0 && cost[p] - u[i] - v[j] == 0.0) {
        row_mate[i] = (int32_t)j;
        col_mate[j] = i;
        break;
      }
    }
  // shortest augmenting paths for the remaining columns
  std::vector<double> dist(n, INF);
  std::vector<char> done(n, 0);
  std::vector<int32_t> pred(n, -1);
  std::vector<double> dcol(n, 0.0);
  std::vector<int32_t> touched, finalized, tree_cols;
  typedef std::pair<double, int32_t> Item;
  for (int64_t j0 = 0; j0 < n; ++j0) {
    if (col_mate[j0] >= 0) continue;
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
    auto relax_from = [&](int32_t j, double dj) {
      for (int64_t p = C.ptr[j]; p < C.ptr[j + 1]; ++p) {
        int32_t i = C.col[p];
        if (done[i]) continue;
        double nd = dj + (cost[p] - u[i] - v[j]);
        if (nd < dist[i]) {
          if (dist[i] == INF) touched.push_back(i);
          dist[i] = nd;
          pred[i] = j;
          heap.push(Item(nd, i));
        }
      }
    };
    dcol[j0] = 0.0;
    tree_cols.push_back((int32_t)j0);
    relax_from((int32_t)j0, 0.0);
    int32_t final_row = -1;
    double L = 0.0;
    while (!heap.empty()) {
      Item it = heap.top();
      heap.pop();
      int32_t i = it.second;
      if (done[i] || it.first > dist[i]) continue;
      done[i] = 1;
      finalized.push_back(i);
      if (row_mate[i] < 0) {
        final_row = i;
        L = it.first;
        break;
      }
      int32_t j = row_mate[i];
      dcol[j] = it.first;
      tree_cols.push_back(j);
      relax_from(j, it.first);
    }
    if (final_row < 0) fail(ASSS_ERR_STRUCTURALLY_SINGULAR, "no perfect matching (structurally singular)");
    for (int32_t i : finalized)
      if (dist[i] < L) u[i] -= (L - dist[i]);
    for (int32_t j : tree_cols)
      if (dcol[j] < L) v[j] += (L - dcol[j]);
    for (int32_t i = final_row;;) {
      int32_t j = pred[i];
      int32_t old = col_mate[j];
      col_mate[j] = i;
      row_mate[i] = j;
      if (j == j0) break;
      i = old;
    }
    for (int32_t i : touched) { dist[i] = INF; done[i] = 0; pred[i] = -1; }
    touched.clear();
    finalized.clear();
    tree_cols.clear();
  }
  return col_mate;
}

void canonical_scaling(const Csr& A, const std::vector<int32_t>& m, std::vector<double>& Dr,
                       std::vector<double>& Dc) {
  const int64_t n = A.nrows;
  // At = P A: row i of At is row m[i] of A
  std::vector<double> dg(n);
  for (int64_t i = 0; i < n; ++i) {
    int64_t r = m[i];
    const int32_t* b = A.col.data() + A.ptr[r];
    const int32_t* e = A.col.data() + A.ptr[r + 1];
    const int32_t* f = std::lower_bound(b, e, (int32_t)i);
    if (f == e || *f != i) fail(ASSS_ERR_STRUCTURALLY_SINGULAR, "matched entry missing");
    dg[i] = std::fabs(A.val[A.ptr[r] + (f - b)]);
  }
  // Bellman-Ford (queue based) from gamma = 0: gamma_j <= gamma_i + w_ij
  std::vector<double> gamma(n, 0.0);
  std::vector<char> inq(n, 1);
  std::deque<int32_t> q;
  for (int64_t i = 0; i < n; ++i) q.push_back((int32_t)i);
  int64_t relax = 0, limit = 64 * (A.nnz() + n) + 1000000;
  while (!q.empty()) {
    int32_t i = q.front();
    q.pop_front();
    inq[i] = 0;
    int64_t r = m[i];
    double li = std::log(dg[i]);
    for (int64_t p = A.ptr[r]; p < A.ptr[r + 1]; ++p) {
      int32_t j = A.col[p];
      if (j == i) continue;
      double w = li - std::log(std::fabs(A.val[p]));
      double cand = gamma[i] + w;
      if (cand < gamma[j]) {
        gamma[j] = cand;
        if (!inq[j]) { inq[j] = 1; q.push_back(j); }
      }
    }
    if (++relax > limit) fail(ASSS_ERR_INTERNAL, "scaling relaxation did not settle");
  }
  Dc.resize(n);
  Dr.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    Dc[i] = std::exp(gamma[i]);
    Dr[m[i]] = std::exp(-gamma[i]) / dg[i];
  }
}

Csr permute_scale(const Csr& A, const std::vector<int32_t>& m, const std::vector<double>& Dr,
                  const std::vector<double>& Dc) {
  const int64_t n = A.nrows;
  Csr B;
  B.nrows = B.ncols = n;
  B.ptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) B.ptr[i + 1] = B.ptr[i] + (A.ptr[m[i] + 1] - A.ptr[m[i]]);
  B.col.resize(B.ptr[n]);
  B.val.resize(B.ptr[n]);
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      int64_t r = m[i], q = B.ptr[i];
      double dr = Dr[r];
      for (int64_t p = A.ptr[r]; p < A.ptr[r + 1]; ++p, ++q) {
        B.col[q] = A.col[p];
        B.val[q] = (dr * A.val[p]) * Dc[A.col[p]];
      }
    }
  });
  return B;
}

Csr s_pattern(const Csr& Abar, int kind, const int64_t* urow, const int32_t* ucol) {
  const int64_t n = Abar.nrows;
  Csr S;
  S.nrows = S.ncols = n;
  S.ptr.assign(n + 1, 0);
  if (kind == ASSS_S_DIAG) {
    for (int64_t i = 0; i < n; ++i) { S.ptr[i + 1] = i + 1; S.col.push_back((int32_t)i); }
  } else if (kind == ASSS_S_TRIDIAG) {
    for (int64_t i = 0; i < n; ++i) {
      for (int64_t j = std::max<int64_t>(0, i - 1); j <= std::min<int64_t>(n - 1, i + 1); ++j)
        S.col.push_back((int32_t)j);
      S.ptr[i + 1] = (int64_t)S.col.size();
    }
  } else if (kind == ASSS_S_PATTERN_OF_ABAR) {
    S.ptr = Abar.ptr;
    S.col = Abar.col;
  } else if (kind == ASSS_S_USER) {
    if (!urow || !ucol) fail(ASSS_ERR_INVALID_ARG, "user S pattern missing");
    if (urow[0] != 0) fail(ASSS_ERR_INVALID_CSR, "S pattern rowptr[0] != 0");
    for (int64_t i = 0; i < n; ++i) {
      if (urow[i + 1] < urow[i]) fail(ASSS_ERR_INVALID_CSR, "S pattern rowptr decreases");
      for (int64_t p = urow[i]; p < urow[i + 1]; ++p) {
        if (ucol[p] < 0 || ucol[p] >= n) fail(ASSS_ERR_INVALID_CSR, "S pattern column out of range");
        if (p > urow[i] && ucol[p - 1] >= ucol[p]) fail(ASSS_ERR_INVALID_CSR, "S pattern columns not increasing");
      }
    }
    S.ptr.assign(urow, urow + n + 1);
    S.col.assign(ucol, ucol + urow[n]);
  } else {
    fail(ASSS_ERR_INVALID_ARG, "unknown S pattern kind");
  }
  return S;
}

// ---------------------------------------------------------------------------
// Least-squares system (App. A)
// ---------------------------------------------------------------------------

static int64_t find_in_row(const Csr& M, int64_t row, int32_t c) {
  const int32_t* b = M.col.data() + M.ptr[row];
  const int32_t* e = M.col.data() + M.ptr[row + 1];
  const int32_t* f = std::lower_bound(b, e, c);
  if (f == e || *f != c) return -1;
  return M.ptr[row] + (f - b);
}

void build_lls(const Csr& Abar, const Csr& Spat, double gamma, LlsSystem& out) {
  const int64_t n = Abar.nrows;
  // Terms of A_hat = Abar S grouped by row: for row i, entries (j, unknown, coef)
  // with coef = abar_ik and unknown = position of s_kj, sorted by (j, unknown).
  Csr& P = out.P;
  P.nrows = P.ncols = n;
  P.ptr.assign(n + 1, 0);
  std::vector<int64_t> tptr(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    int64_t c = 0;
    for (int64_t p = Abar.ptr[i]; p < Abar.ptr[i + 1]; ++p) {
      int32_t k = Abar.col[p];
      c += Spat.ptr[k + 1] - Spat.ptr[k];
    }
    tptr[i + 1] = tptr[i] + c;
  }
  const int64_t nterms = tptr[n];
  std::vector<int32_t> tcol(nterms), tunk(nterms);
  std::vector<double> tcoef(nterms);
  std::vector<int64_t> pcount(n, 0);
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    std::vector<int64_t> idx;
    std::vector<int32_t> c2;
    std::vector<int32_t> u2;
    std::vector<double> v2;
    for (int64_t i = lo; i < hi; ++i) {
      int64_t b = tptr[i], q = b;
      for (int64_t p = Abar.ptr[i]; p < Abar.ptr[i + 1]; ++p) {
        int32_t k = Abar.col[p];
        for (int64_t s = Spat.ptr[k]; s < Spat.ptr[k + 1]; ++s, ++q) {
          tcol[q] = Spat.col[s];
          tunk[q] = (int32_t)s;
          tcoef[q] = Abar.val[p];
        }
      }
      int64_t len = q - b;
      idx.resize(len);
      std::iota(idx.begin(), idx.end(), 0);
      std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
        if (tcol[b + x] != tcol[b + y]) return tcol[b + x] < tcol[b + y];
        return tunk[b + x] < tunk[b + y];
      });
      c2.resize(len); u2.resize(len); v2.resize(len);
      for (int64_t t = 0; t < len; ++t) { c2[t] = tcol[b + idx[t]]; u2[t] = tunk[b + idx[t]]; v2[t] = tcoef[b + idx[t]]; }
      int64_t distinct = 0;
      for (int64_t t = 0; t < len; ++t) {
        tcol[b + t] = c2[t]; tunk[b + t] = u2[t]; tcoef[b + t] = v2[t];
        if (t == 0 || c2[t] != c2[t - 1]) ++distinct;
      }
      pcount[i] = distinct;
    }
  });
  for (int64_t i = 0; i < n; ++i) P.ptr[i + 1] = P.ptr[i] + pcount[i];
  P.col.resize(P.ptr[n]);
  // segment starts of each distinct column within a row's terms
  std::vector<int64_t> pseg(P.ptr[n] + 1);
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      int64_t q = P.ptr[i];
      for (int64_t t = tptr[i]; t < tptr[i + 1]; ++t)
        if (t == tptr[i] || tcol[t] != tcol[t - 1]) { P.col[q] = tcol[t]; pseg[q] = t; ++q; }
    }
  });
  pseg[P.ptr[n]] = nterms;
  // U = strictly upper pattern of P + P^T
  Csr Pt = transpose(P);
  Csr& U = out.U;
  U.nrows = U.ncols = n;
  U.ptr.assign(n + 1, 0);
  std::vector<int64_t> ucount(n);
  auto merge_row = [&](int64_t i, int32_t* dst) -> int64_t {
    const int32_t* a = P.col.data() + P.ptr[i];
    const int32_t* ae = P.col.data() + P.ptr[i + 1];
    const int32_t* b = Pt.col.data() + Pt.ptr[i];
    const int32_t* be = Pt.col.data() + Pt.ptr[i + 1];
    a = std::upper_bound(a, ae, (int32_t)i);
    b = std::upper_bound(b, be, (int32_t)i);
    int64_t c = 0;
    while (a < ae || b < be) {
      int32_t x;
      if (b >= be || (a < ae && *a < *b)) x = *a++;
      else if (a >= ae || *b < *a) x = *b++;
      else { x = *a; ++a; ++b; }
      if (dst) dst[c] = x;
      ++c;
    }
    return c;
  };
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) ucount[i] = merge_row(i, nullptr);
  });
  for (int64_t i = 0; i < n; ++i) U.ptr[i + 1] = U.ptr[i] + ucount[i];
  U.col.resize(U.ptr[n]);
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) merge_row(i, U.col.data() + U.ptr[i]);
  });
  const int64_t nz = U.ptr[n];
  // B rows: pair (i,j), i<j: terms of row i with column j, then terms of row j
  // with column i; diagonal row i: sqrt(gamma) * terms of row i with column i.
  auto seg = [&](int64_t row, int32_t c, int64_t& b, int64_t& e) {
    int64_t q = find_in_row(P, row, c);
    if (q < 0) { b = e = 0; return; }
    b = pseg[q];
    e = pseg[q + 1];
  };
  Csr& B = out.B;
  B.nrows = nz + n;
  B.ncols = Spat.nnz();
  B.ptr.assign(nz + n + 1, 0);
  std::vector<int64_t> rlen(nz + n, 0);
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      for (int64_t e = U.ptr[i]; e < U.ptr[i + 1]; ++e) {
        int32_t j = U.col[e];
        int64_t b1, e1, b2, e2;
        seg(i, j, b1, e1);
        seg(j, (int32_t)i, b2, e2);
        rlen[e] = (e1 - b1) + (e2 - b2);
      }
      int64_t b1, e1;
      seg(i, (int32_t)i, b1, e1);
      rlen[nz + i] = e1 - b1;
    }
  });
  for (int64_t r = 0; r < nz + n; ++r) B.ptr[r + 1] = B.ptr[r] + rlen[r];
  B.col.resize(B.ptr[nz + n]);
  B.val.resize(B.ptr[nz + n]);
  const double sg = std::sqrt(gamma);
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t i = lo; i < hi; ++i) {
      for (int64_t e = U.ptr[i]; e < U.ptr[i + 1]; ++e) {
        int32_t j = U.col[e];
        int64_t b1, e1, b2, e2;
        seg(i, j, b1, e1);
        seg(j, (int32_t)i, b2, e2);
        row.clear();
        for (int64_t t = b1; t < e1; ++t) row.emplace_back(tunk[t], tcoef[t]);
        for (int64_t t = b2; t < e2; ++t) row.emplace_back(tunk[t], tcoef[t]);
        std::sort(row.begin(), row.end(),
                  [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) { return x.first < y.first; });
        int64_t q = B.ptr[e];
        for (auto& pr : row) { B.col[q] = pr.first; B.val[q] = pr.second; ++q; }
      }
      int64_t b1, e1;
      seg(i, (int32_t)i, b1, e1);
      int64_t q = B.ptr[nz + i];
      for (int64_t t = b1; t < e1; ++t) { B.col[q] = tunk[t]; B.val[q] = sg * tcoef[t]; ++q; }
    }
  });
  out.rhs.assign(nz + n, 0.0);
  for (int64_t i = 0; i < n; ++i) out.rhs[nz + i] = sg;
  out.Bt = transpose(B);
  P.val.clear();
}

Csr spgemm_on_pattern(const Csr& Abar, const Csr& S, const Csr& P) {
  const int64_t n = Abar.nrows;
  Csr Y;
  Y.nrows = Y.ncols = n;
  Y.ptr = P.ptr;
  Y.col = P.col;
  Y.val.assign(P.nnz(), 0.0);
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      for (int64_t p = Abar.ptr[i]; p < Abar.ptr[i + 1]; ++p) {
        int32_t k = Abar.col[p];
        double a = Abar.val[p];
        for (int64_t s = S.ptr[k]; s < S.ptr[k + 1]; ++s) {
          int64_t q = find_in_row(P, i, S.col[s]);
          Y.val[q] += a * S.val[s];
        }
      }
    }
  });
  return Y;
}

void split_ahat(const Csr& Ahat, const Csr& U, std::vector<double>& D, std::vector<double>& Omega,
                std::vector<double>& jval) {
  const int64_t n = Ahat.nrows;
  D.assign(n, 0.0);
  Omega.assign(n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    int64_t q = find_in_row(Ahat, i, (int32_t)i);
    D[i] = q >= 0 ? Ahat.val[q] : 0.0;
    if (D[i] == 0.0) fail(ASSS_ERR_ZERO_DIAGONAL, "diag(Abar S) has a zero entry");
    Omega[i] = 1.0 / std::sqrt(std::fabs(D[i]));
  }
  jval.assign(U.nnz(), 0.0);
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i)
      for (int64_t e = U.ptr[i]; e < U.ptr[i + 1]; ++e) {
        int32_t j = U.col[e];
        int64_t q1 = find_in_row(Ahat, i, j), q2 = find_in_row(Ahat, j, (int32_t)i);
        double aij = q1 >= 0 ? Ahat.val[q1] : 0.0;
        double aji = q2 >= 0 ? Ahat.val[q2] : 0.0;
        jval[e] = Omega[i] * Omega[j] * (aij - aji) / 2.0;
      }
  });
}

// ---------------------------------------------------------------------------
// Sliced layout of J_tilde
// ---------------------------------------------------------------------------

// Slot form: per slice, the sorted distinct offsets d = j - i of its rows'
// in-block upper entries (part a) and of its off-block entries of both
// triangles (part b); one slot per offset.
static SkewSell pack_skew_slots(const Csr& Jup, const Csr& Lo, int32_t R,
                                const std::vector<std::vector<int32_t>>& aoffs,
                                const std::vector<std::vector<int32_t>>& boffs) {
  SkewSell S;
  const int64_t n = Jup.nrows;
  S.n = (int32_t)n;
  S.R = R;
  S.nblocks = (int32_t)((n + R - 1) / R);
  S.nslices = (int32_t)((n + 63) / 64);
  S.form = SKEW_SLOTS;
  S.a_width.assign(S.nslices, 0);
  S.b_width.assign(S.nslices, 0);
  S.a_off.assign(S.nslices + 1, 0);
  S.b_off.assign(S.nslices + 1, 0);
  for (int64_t s = 0; s < S.nslices; ++s) {
    S.a_width[s] = (int32_t)aoffs[s].size();
    S.b_width[s] = (int32_t)boffs[s].size();
    S.a_off[s + 1] = S.a_off[s] + (int64_t)S.a_width[s] * 64;
    S.b_off[s + 1] = S.b_off[s] + (int64_t)S.b_width[s] * 64;
  }
  S.a_val.assign(S.a_off[S.nslices], 0.0);
  S.b_val.assign(S.b_off[S.nslices], 0.0);
  S.a_doff.assign(S.a_off[S.nslices] / 64, 0);
  S.b_base.assign(S.b_off[S.nslices] / 64, 0);
  std::vector<int64_t> na(S.nslices, 0), nb(S.nslices, 0);
  parallel_for(S.nslices, [&](int64_t lo, int64_t hi) {
    for (int64_t s = lo; s < hi; ++s) {
      const auto& ao = aoffs[s];
      const auto& bo = boffs[s];
      for (size_t t = 0; t < ao.size(); ++t) S.a_doff[S.a_off[s] / 64 + t] = ao[t];
      for (size_t t = 0; t < bo.size(); ++t) S.b_base[S.b_off[s] / 64 + t] = (int32_t)(s * 64 + bo[t]);
      auto slot = [](const std::vector<int32_t>& v, int64_t d) {
        return (int64_t)(std::lower_bound(v.begin(), v.end(), (int32_t)d) - v.begin());
      };
      for (int lane = 0; lane < 64; ++lane) {
        const int64_t i = s * 64 + lane;
        if (i >= n) break;
        const int64_t blk = i / R;
        for (int64_t p = Lo.ptr[i]; p < Lo.ptr[i + 1]; ++p)
          if (Lo.col[p] / R != blk) {
            S.b_val[S.b_off[s] + slot(bo, Lo.col[p] - i) * 64 + lane] = -Lo.val[p];
            ++nb[s];
          }
        for (int64_t p = Jup.ptr[i]; p < Jup.ptr[i + 1]; ++p) {
          const int64_t j = Jup.col[p];
          if (j / R == blk) {
            S.a_val[S.a_off[s] + slot(ao, j - i) * 64 + lane] = Jup.val[p];
            ++na[s];
          } else {
            S.b_val[S.b_off[s] + slot(bo, j - i) * 64 + lane] = Jup.val[p];
            ++nb[s];
          }
        }
      }
    }
  });
  for (int64_t s = 0; s < S.nslices; ++s) {
    S.a_entries += na[s];
    S.b_entries += nb[s];
  }
  return S;
}

SkewSell pack_skew_sell(const Csr& Jup, int32_t R, int32_t form) {
  const int64_t n = Jup.nrows;
  const int64_t nslices = (n + 63) / 64;
  // lower part: for row i, entries (i, j) with j < i come from upper row j
  Csr Lo = transpose(Jup);  // row i of Lo: columns j < i with value u_ji
  if (form == SKEW_AUTO || form == SKEW_SLOTS) {
    std::vector<std::vector<int32_t>> aoffs(nslices), boffs(nslices);
    std::vector<int64_t> per_std(nslices, 0), per_slots(nslices, 0);
    parallel_for(nslices, [&](int64_t lo, int64_t hi) {
      for (int64_t s = lo; s < hi; ++s) {
        auto& ao = aoffs[s];
        auto& bo = boffs[s];
        int32_t wa = 0, wl = 0, wu = 0;
        for (int64_t i = s * 64; i < std::min<int64_t>(n, s * 64 + 64); ++i) {
          const int64_t blk = i / R;
          int32_t ra = 0, rl = 0, ru = 0;
          for (int64_t p = Lo.ptr[i]; p < Lo.ptr[i + 1]; ++p)
            if (Lo.col[p] / R != blk) { bo.push_back((int32_t)(Lo.col[p] - i)); ++rl; }
          for (int64_t p = Jup.ptr[i]; p < Jup.ptr[i + 1]; ++p) {
            if (Jup.col[p] / R == blk) { ao.push_back((int32_t)(Jup.col[p] - i)); ++ra; }
            else { bo.push_back((int32_t)(Jup.col[p] - i)); ++ru; }
          }
          wa = std::max(wa, ra);
          wl = std::max(wl, rl);
          wu = std::max(wu, ru);
        }
        std::sort(ao.begin(), ao.end());
        ao.erase(std::unique(ao.begin(), ao.end()), ao.end());
        std::sort(bo.begin(), bo.end());
        bo.erase(std::unique(bo.begin(), bo.end()), bo.end());
        per_std[s] = (int64_t)wa + wl + wu;
        per_slots[s] = (int64_t)ao.size() + bo.size();
      }
    });
    int64_t tot_std = 0, tot_slots = 0;
    for (int64_t s = 0; s < nslices; ++s) { tot_std += per_std[s]; tot_slots += per_slots[s]; }
    if (form == SKEW_SLOTS && tot_slots > 16 * std::max<int64_t>(tot_std, 1))
      fail(ASSS_ERR_INVALID_ARG, "the slot form of this matrix would store more than 16x the entries");
    if (form == SKEW_SLOTS || tot_slots * 10 <= tot_std * 12)
      return pack_skew_slots(Jup, Lo, R, aoffs, boffs);
  }
  SkewSell S;
  S.n = (int32_t)n;
  S.R = R;
  S.nblocks = (int32_t)((n + R - 1) / R);
  S.nslices = (int32_t)nslices;
  // part b of a row: nbl entries in earlier blocks, then nbu in later blocks;
  // each group gets its own slot range in the slice (below), so that one slot
  // never mixes a neighbour before the block with one after it
  std::vector<int32_t> na(n, 0), nb(n, 0), nbl(n, 0);
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      int64_t blk = i / R;
      for (int64_t p = Jup.ptr[i]; p < Jup.ptr[i + 1]; ++p) {
        if (Jup.col[p] / R == blk) na[i]++;
        else nb[i]++;
      }
      for (int64_t p = Lo.ptr[i]; p < Lo.ptr[i + 1]; ++p)
        if (Lo.col[p] / R != blk) { nb[i]++; nbl[i]++; }
    }
  });
  S.a_width.assign(S.nslices, 0);
  S.b_width.assign(S.nslices, 0);
  S.a_off.assign(S.nslices + 1, 0);
  S.b_off.assign(S.nslices + 1, 0);
  std::vector<int32_t> wlo(S.nslices, 0);
  for (int64_t s = 0; s < S.nslices; ++s) {
    int32_t wa = 0, wl = 0, wu = 0;
    for (int64_t i = s * 64; i < std::min<int64_t>(n, s * 64 + 64); ++i) {
      wa = std::max(wa, na[i]);
      wl = std::max(wl, nbl[i]);
      wu = std::max(wu, nb[i] - nbl[i]);
    }
    const int32_t wb = wl + wu;
    wlo[s] = wl;
    S.a_width[s] = wa;
    S.b_width[s] = wb;
    S.a_off[s + 1] = S.a_off[s] + (int64_t)wa * 64;
    S.b_off[s + 1] = S.b_off[s] + (int64_t)wb * 64;
  }
  S.a_col.assign(S.a_off[S.nslices], 0);
  S.a_val.assign(S.a_off[S.nslices], 0.0);
  S.b_col.assign(S.b_off[S.nslices], 0);
  S.b_val.assign(S.b_off[S.nslices], 0.0);
  parallel_for(S.nslices, [&](int64_t lo, int64_t hi) {
    for (int64_t s = lo; s < hi; ++s) {
      for (int lane = 0; lane < 64; ++lane) {
        int64_t i = s * 64 + lane;
        int64_t blk = i / R, b0 = blk * R;
        int32_t la = 0, lb = 0;
        if (i < n) {
          // part b: entries before the block in slots [0, wlo), entries after
          // it from slot wlo on (ascending columns within each group)
          for (int64_t p = Lo.ptr[i]; p < Lo.ptr[i + 1]; ++p)
            if (Lo.col[p] / R != blk) {
              int64_t q = S.b_off[s] + (int64_t)lb * 64 + lane;
              S.b_col[q] = Lo.col[p];
              S.b_val[q] = -Lo.val[p];
              ++lb;
            }
          for (; lb < wlo[s]; ++lb) {  // padding up to the upper group
            int64_t q = S.b_off[s] + (int64_t)lb * 64 + lane;
            S.b_col[q] = -1;  // placeholder: set to the slot's base below
            S.b_val[q] = 0.0;
          }
          for (int64_t p = Jup.ptr[i]; p < Jup.ptr[i + 1]; ++p) {
            int32_t j = Jup.col[p];
            if (j / R == blk) {
              int64_t q = S.a_off[s] + (int64_t)la * 64 + lane;
              S.a_col[q] = (uint16_t)(j - b0);
              S.a_val[q] = Jup.val[p];
              ++la;
            } else {
              int64_t q = S.b_off[s] + (int64_t)lb * 64 + lane;
              S.b_col[q] = j;
              S.b_val[q] = Jup.val[p];
              ++lb;
            }
          }
        }
        int64_t self = i < n ? i : (n - 1);
        int64_t selfb0 = (self / R) * R;
        for (; la < S.a_width[s]; ++la) {
          int64_t q = S.a_off[s] + (int64_t)la * 64 + lane;
          S.a_col[q] = (uint16_t)(self - selfb0);
          S.a_val[q] = 0.0;
        }
        for (; lb < S.b_width[s]; ++lb) {
          int64_t q = S.b_off[s] + (int64_t)lb * 64 + lane;
          S.b_col[q] = (int32_t)self;
          S.b_val[q] = 0.0;
        }
      }
    }
  });
  int64_t ta = 0, tb = 0;
  for (int64_t i = 0; i < n; ++i) { ta += na[i]; tb += nb[i]; }
  S.a_entries = ta;
  S.b_entries = tb;
  // narrow part-b columns: per slot, base = smallest real column; padding
  // entries (value 0) take the base so that they do not widen the span
  const int64_t nslots = S.b_off[S.nslices] / 64;
  S.b_base.assign(nslots, 0);
  std::atomic<int> wide(0);
  parallel_for(S.nslices, [&](int64_t lo, int64_t hi) {
    for (int64_t s = lo; s < hi; ++s) {
      for (int32_t l = 0; l < S.b_width[s]; ++l) {
        const int64_t q0 = S.b_off[s] + (int64_t)l * 64;
        int64_t mn = INT64_MAX, mx = INT64_MIN;
        auto real = [&](int lane) {
          const int64_t i = s * 64 + lane;
          if (i >= n) return false;
          return l < nbl[i] || (l >= wlo[s] && l - wlo[s] < nb[i] - nbl[i]);
        };
        for (int lane = 0; lane < 64; ++lane) {
          if (real(lane)) {
            mn = std::min<int64_t>(mn, S.b_col[q0 + lane]);
            mx = std::max<int64_t>(mx, S.b_col[q0 + lane]);
          }
        }
        if (mn == INT64_MAX) mn = mx = S.b_col[q0];  // cannot happen: l < width
        for (int lane = 0; lane < 64; ++lane)
          if (!real(lane)) S.b_col[q0 + lane] = (int32_t)mn;
        S.b_base[q0 / 64] = (int32_t)mn;
        if (mx - mn > 65535) wide = 1;
      }
    }
  });
  if (form == SKEW_NARROW && wide != 0)
    fail(ASSS_ERR_INVALID_ARG, "16-bit off-block columns do not fit this matrix");
  S.b_narrow = (wide == 0) && form != SKEW_WIDE;
  S.form = S.b_narrow ? SKEW_NARROW : SKEW_WIDE;
  if (S.b_narrow) {
    S.b_cd.resize(S.b_col.size());
    parallel_for(nslots, [&](int64_t lo, int64_t hi) {
      for (int64_t t = lo; t < hi; ++t)
        for (int lane = 0; lane < 64; ++lane)
          S.b_cd[t * 64 + lane] = (uint16_t)(S.b_col[t * 64 + lane] - S.b_base[t]);
    });
  }
  return S;
}

// ---------------------------------------------------------------------------
// Block reordering of the inner system
// ---------------------------------------------------------------------------

int64_t count_cross_pairs(const Csr& U, int32_t R) {
  int64_t c = 0;
  for (int64_t i = 0; i < U.nrows; ++i)
    for (int64_t p = U.ptr[i]; p < U.ptr[i + 1]; ++p) c += (U.col[p] / R != i / R);
  return c;
}

namespace {

// BFS restricted to vertices with part[v] == pid, from `src`; fills dist for
// the visited vertices and returns the last vertex reached (a farthest one).
int32_t bfs_part(const Csr& G, const std::vector<int32_t>& part, int32_t pid, int32_t src,
                 std::vector<int32_t>& dist, std::vector<int32_t>& queue) {
  queue.clear();
  queue.push_back(src);
  dist[src] = 0;
  size_t head = 0;
  int32_t last = src;
  while (head < queue.size()) {
    int32_t v = queue[head++];
    last = v;
    for (int64_t p = G.ptr[v]; p < G.ptr[v + 1]; ++p) {
      int32_t w = G.col[p];
      if (part[w] == pid && dist[w] < 0) {
        dist[w] = dist[v] + 1;
        queue.push_back(w);
      }
    }
  }
  return last;
}

}  // namespace

std::vector<int32_t> grid_line_order(const Csr& Abar, int32_t target_R, int32_t& R_out) {
  const int64_t n = Abar.nrows;
  R_out = 0;
  // distinct positive column offsets (a grid stencil has a handful)
  std::vector<int64_t> offs;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = Abar.ptr[i]; p < Abar.ptr[i + 1]; ++p) {
      const int64_t d = (int64_t)Abar.col[p] - i;
      if (d <= 0 || std::find(offs.begin(), offs.end(), d) != offs.end()) continue;
      offs.push_back(d);
      if (offs.size() > 3) return {};
    }
  std::sort(offs.begin(), offs.end());
  if (offs.size() != 3 || offs[0] != 1) return {};
  const int64_t m1 = offs[1], plane = offs[2];
  if (m1 < 2 || plane % m1 != 0 || n % plane != 0) return {};
  const int64_t m2 = plane / m1, m3 = n / plane;
  if (m2 < 2 || m3 < 2) return {};
  // lines per tile: the largest power of two <= target_R / m1 with a split
  // ty x tz (powers of two, ty | m2, tz | m3, as square as possible) and
  // m1 ty tz a multiple of 64 within 4096
  int64_t best_ty = 0, best_tz = 0;
  int64_t T0 = 1;
  while (T0 * 2 <= target_R / m1) T0 *= 2;
  for (int64_t T = T0; T >= 1 && !best_ty; T /= 2) {
    if ((m1 * T) % 64 != 0 || m1 * T > 4096) continue;
    int64_t gap = -1;
    for (int64_t ty = 1; ty <= T; ty *= 2) {
      const int64_t tz = T / ty;
      if (ty * tz != T || m2 % ty != 0 || m3 % tz != 0) continue;
      const int64_t g = std::max(ty, tz) / std::min(ty, tz);
      if (gap < 0 || g < gap) { gap = g; best_ty = ty; best_tz = tz; }
    }
  }
  if (!best_ty) return {};
  const int64_t ty = best_ty, tz = best_tz;
  std::vector<int32_t> perm((size_t)n);
  int64_t k = 0;
  for (int64_t TZ = 0; TZ < m3 / tz; ++TZ)
    for (int64_t TY = 0; TY < m2 / ty; ++TY)
      for (int64_t z = 0; z < tz; ++z)
        for (int64_t y = 0; y < ty; ++y)
          for (int64_t x = 0; x < m1; ++x)
            perm[(size_t)k++] = (int32_t)(x + m1 * ((TY * ty + y) + m2 * (TZ * tz + z)));
  R_out = (int32_t)(m1 * ty * tz);
  return perm;
}

Csr permute_skew_upper(const Csr& U, const std::vector<int32_t>& perm) {
  const int64_t n = U.nrows;
  std::vector<int32_t> iperm(n);
  for (int64_t i = 0; i < n; ++i) iperm[perm[i]] = (int32_t)i;
  std::vector<int64_t> cnt(n + 1, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = U.ptr[i]; p < U.ptr[i + 1]; ++p) {
      int32_t a = iperm[i], b = iperm[U.col[p]];
      cnt[std::min(a, b) + 1]++;
    }
  Csr P;
  P.nrows = P.ncols = n;
  P.ptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) P.ptr[i + 1] = P.ptr[i] + cnt[i + 1];
  P.col.resize(U.nnz());
  P.val.resize(U.nnz());
  std::vector<int64_t> cur(P.ptr.begin(), P.ptr.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = U.ptr[i]; p < U.ptr[i + 1]; ++p) {
      int32_t a = iperm[i], b = iperm[U.col[p]];
      int64_t q = cur[std::min(a, b)]++;
      P.col[q] = std::max(a, b);
      P.val[q] = a < b ? U.val[p] : -U.val[p];
    }
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t i = lo; i < hi; ++i) {
      row.clear();
      for (int64_t p = P.ptr[i]; p < P.ptr[i + 1]; ++p) row.emplace_back(P.col[p], P.val[p]);
      std::sort(row.begin(), row.end(),
                [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) { return x.first < y.first; });
      int64_t q = P.ptr[i];
      for (auto& e : row) { P.col[q] = e.first; P.val[q] = e.second; ++q; }
    }
  });
  return P;
}

}  // namespace asss
