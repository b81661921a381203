// Incomplete LDL^T with Bunch-Kaufman pivoting, scaled factor, low-rank term
// and level schedules (paper Sec. 3: the factorization of M_hat, eq. absfac,
// eq. preconditioner, Fig. 1).
//
// The factorization is left-looking: when position j is reached, the columns
// of the current Schur complement that the pivot test needs are formed from
// the original M and the finished columns of L,
//
//   W[:, c] = M[:, c] - sum over finished blocks b of L_b P_b L_b[c, :]^T,
//
// restricted to the rows not yet eliminated.  Each finished column was
// thinned by the dropping rules before it was stored, so W is the Schur
// complement of the right-looking elimination that drops entries of a column
// before the column updates the rest of the matrix.  Entries of L are kept by
// original index, so a symmetric interchange of two positions only swaps two
// entries of perm and of its inverse.
#include "ildl_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "../../include/asss.h"

namespace asss {

namespace {

[[noreturn]] void fail(int code, const char* msg) { throw HostError{code, msg}; }

// Bunch and Kaufman's constant (1 + sqrt 17) / 8: it bounds the growth of the
// entries of the Schur complements.
const double kAlpha = (1.0 + std::sqrt(17.0)) / 8.0;

// Sparse accumulator of one Schur column, indexed by original index.
struct Spa {
  std::vector<double> w;
  std::vector<char> mark;
  std::vector<int32_t> list;
  explicit Spa(int64_t n) : w(n, 0.0), mark(n, 0) {}
  void add(int32_t i, double v) {
    if (!mark[i]) {
      mark[i] = 1;
      w[i] = 0.0;
      list.push_back(i);
    }
    w[i] += v;
  }
  double get(int32_t i) const { return mark[i] ? w[i] : 0.0; }
  void clear() {
    for (int32_t i : list) mark[i] = 0;
    list.clear();
  }
};

struct Entry {
  int32_t idx;  // original row index (column lists) or column position (row lists)
  double v;
};

// Symmetric 2x2 eigendecomposition by one Jacobi rotation (Golub and Van
// Loan, the symmetric Schur decomposition of a 2x2 block): B = V diag(l) V^T,
// V = [[c, s], [-s, c]].
void sym2_eig(double a, double b, double d, double l[2], double V[2][2]) {
  if (b == 0.0) {
    l[0] = a; l[1] = d;
    V[0][0] = 1.0; V[0][1] = 0.0; V[1][0] = 0.0; V[1][1] = 1.0;
    return;
  }
  const double tau = (d - a) / (2.0 * b);
  const double t = (tau >= 0.0) ? 1.0 / (tau + std::sqrt(1.0 + tau * tau))
                                : -1.0 / (-tau + std::sqrt(1.0 + tau * tau));
  const double c = 1.0 / std::sqrt(1.0 + t * t);
  const double s = t * c;
  l[0] = a - t * b;
  l[1] = d + t * b;
  V[0][0] = c; V[0][1] = s;
  V[1][0] = -s; V[1][1] = c;
}

}  // namespace

void symmetric_skew_split(const Csr& A, Csr& M, Csr& J) {
  const int64_t n = A.nrows;
  Csr At = transpose(A);
  M = Csr{};
  J = Csr{};
  M.nrows = M.ncols = J.nrows = J.ncols = n;
  M.ptr.assign(n + 1, 0);
  J.ptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    int64_t p = A.ptr[i], q = At.ptr[i];
    const int64_t pe = A.ptr[i + 1], qe = At.ptr[i + 1];
    while (p < pe || q < qe) {
      int32_t c;
      double a = 0.0, at = 0.0;
      if (q >= qe || (p < pe && A.col[p] < At.col[q])) {
        c = A.col[p]; a = A.val[p]; ++p;
      } else if (p >= pe || At.col[q] < A.col[p]) {
        c = At.col[q]; at = At.val[q]; ++q;
      } else {
        c = A.col[p]; a = A.val[p]; at = At.val[q]; ++p; ++q;
      }
      const double m = (a + at) / 2.0;
      if (m != 0.0) { M.col.push_back(c); M.val.push_back(m); }
      if ((int64_t)c != i) {
        // exact skew symmetry: the entry below the diagonal is the negation
        // of the one above it
        const double u = (int64_t)c > i ? (a - at) / 2.0 : -((at - a) / 2.0);
        J.col.push_back(c);
        J.val.push_back(u);
      }
    }
    M.ptr[i + 1] = (int64_t)M.col.size();
    J.ptr[i + 1] = (int64_t)J.col.size();
  }
}

Csr permute_symmetric(const Csr& A, const std::vector<int32_t>& perm) {
  const int64_t n = A.nrows;
  std::vector<int32_t> pos(n);
  for (int64_t p = 0; p < n; ++p) pos[perm[p]] = (int32_t)p;
  Csr B;
  B.nrows = B.ncols = n;
  B.ptr.assign(n + 1, 0);
  B.col.reserve(A.nnz());
  B.val.reserve(A.nnz());
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t p = 0; p < n; ++p) {
    const int32_t i = perm[p];
    row.clear();
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) row.push_back({pos[A.col[e]], A.val[e]});
    std::sort(row.begin(), row.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    for (auto& e : row) { B.col.push_back(e.first); B.val.push_back(e.second); }
    B.ptr[p + 1] = (int64_t)B.col.size();
  }
  return B;
}

IldlFactor ildl_bunch_kaufman(const Csr& M, const IldlOpts& o) {
  const int64_t n = M.nrows;
  if (M.ncols != n) fail(ASSS_ERR_INVALID_ARG, "M is not square");
  {  // symmetric in pattern and values
    Csr Mt = transpose(M);
    if (Mt.ptr != M.ptr || Mt.col != M.col || Mt.val != M.val) fail(ASSS_ERR_INVALID_ARG, "M is not symmetric");
  }
  IldlFactor F;
  F.n = n;
  F.perm.resize(n);
  std::vector<int32_t> pos(n);
  for (int64_t i = 0; i < n; ++i) F.perm[i] = pos[i] = (int32_t)i;
  std::vector<std::vector<Entry>> Lcol(n);  // by column position: (original row, value)
  std::vector<std::vector<Entry>> Lrow(n);  // by original row: (column position, value)
  std::vector<int32_t> blk_of(n, -1);
  Spa s1(n), s2(n);

  // Column c (original index) of the Schur complement at step j, rows with
  // position >= j.
  auto schur = [&](int32_t c, int64_t j, Spa& sp) {
    sp.clear();
    for (int64_t e = M.ptr[c]; e < M.ptr[c + 1]; ++e)
      if (pos[M.col[e]] >= j) sp.add(M.col[e], M.val[e]);
    const std::vector<Entry>& rl = Lrow[c];
    for (size_t t = 0; t < rl.size();) {
      const int32_t b = blk_of[rl[t].idx];
      const int32_t p = F.bstart[b];
      double a0 = 0.0, a1 = 0.0;
      while (t < rl.size() && blk_of[rl[t].idx] == b) {
        (rl[t].idx == p ? a0 : a1) = rl[t].v;
        ++t;
      }
      const double* B = &F.bval[3 * (size_t)b];
      double v0, v1 = 0.0;
      if (F.bsize[b] == 1) {
        v0 = B[0] * a0;
      } else {
        v0 = B[0] * a0 + B[1] * a1;
        v1 = B[1] * a0 + B[2] * a1;
      }
      for (const Entry& e : Lcol[p])
        if (pos[e.idx] >= j) sp.add(e.idx, -e.v * v0);
      if (F.bsize[b] == 2)
        for (const Entry& e : Lcol[p + 1])
          if (pos[e.idx] >= j) sp.add(e.idx, -e.v * v1);
    }
  };
  auto swap_pos = [&](int64_t a, int64_t b) {
    if (a == b) return;
    std::swap(F.perm[a], F.perm[b]);
    pos[F.perm[a]] = (int32_t)a;
    pos[F.perm[b]] = (int32_t)b;
  };

  std::vector<std::pair<int32_t, double>> col;  // a computed column: (original row, value)
  std::vector<int32_t> order;
  for (int64_t j = 0; j < n;) {
    const int32_t c = F.perm[j];
    schur(c, j, s1);
    int s = 1;
    int32_t piv2 = -1;  // original index of the second row of a 2x2 pivot
    bool use_r = false;
    if (o.pivoting && j < n - 1) {
      const double akk = std::fabs(s1.get(c));
      double lam = 0.0;
      int32_t r = -1;
      for (int32_t i : s1.list) {
        if (i == c) continue;
        const double v = std::fabs(s1.w[i]);
        if (v > lam || (v == lam && v > 0.0 && pos[i] < pos[r])) { lam = v; r = i; }
      }
      if (!(std::max(akk, lam) == 0.0 || akk >= kAlpha * lam)) {
        schur(r, j, s2);
        double sigma = 0.0;
        for (int32_t i : s2.list)
          if (i != r) sigma = std::max(sigma, std::fabs(s2.w[i]));
        if (akk >= kAlpha * lam * (lam / sigma)) {
          // 1x1 pivot at j
        } else if (std::fabs(s2.get(r)) >= kAlpha * sigma) {
          use_r = true;
          swap_pos(j, pos[r]);
        } else {
          s = 2;
          piv2 = r;
          swap_pos(j + 1, pos[r]);
        }
      }
    }
    const int32_t b = (int32_t)F.bstart.size();
    F.bstart.push_back((int32_t)j);
    F.bsize.push_back(s);
    double B0, B1 = 0.0, B2 = 0.0;
    const Spa& sp0 = use_r ? s2 : s1;  // Schur column of the pivot
    const int32_t c0 = F.perm[j];
    col.clear();
    if (s == 1) {
      B0 = sp0.get(c0);
      if (B0 == 0.0) {
        bool zero_col = true;
        for (int32_t i : sp0.list)
          if (i != c0 && sp0.w[i] != 0.0) zero_col = false;
        if (!(o.pivoting && zero_col)) fail(ASSS_ERR_ZERO_DIAGONAL, "zero pivot in the incomplete LDL^T of M_hat");
        B0 = 1.0;  // a zero row of the Schur complement: pivot 1
      }
      for (int32_t i : sp0.list)
        if (pos[i] > j && sp0.w[i] != 0.0) col.push_back({i, sp0.w[i] / B0});
    } else {
      const int32_t c1 = piv2;
      B0 = s1.get(c0);
      B1 = s1.get(c1);
      B2 = s2.get(c1);
      // rows below the block: union of the two Schur columns; each row's
      // 2-vector solved against the block by LU with partial pivoting
      const bool sw = std::fabs(B1) > std::fabs(B0);
      const double p00 = sw ? B1 : B0, p01 = sw ? B2 : B1;  // pivot row
      const double q00 = sw ? B0 : B1, q01 = sw ? B1 : B2;  // other row
      const double l10 = q00 / p00;
      const double u11 = q01 - l10 * p01;
      std::vector<int32_t> rows;
      for (int32_t i : s1.list)
        if (pos[i] >= j + 2) rows.push_back(i);
      for (int32_t i : s2.list)
        if (pos[i] >= j + 2 && !s1.mark[i]) rows.push_back(i);
      for (int32_t i : rows) {
        const double r0 = s1.get(i), r1 = s2.get(i);
        const double y0 = sw ? r1 : r0, y1 = sw ? r0 : r1;
        const double z1 = (y1 - l10 * y0) / u11;
        const double z0 = (y0 - p01 * z1) / p00;
        col.push_back({i, z0});
        col.push_back({i, z1});  // interleaved: entry 2t is column j, 2t+1 column j+1
      }
    }
    F.bval.push_back(B0);
    F.bval.push_back(B1);
    F.bval.push_back(B2);
    // dropping, one column of the block at a time
    for (int q = 0; q < s; ++q) {
      std::vector<std::pair<int32_t, double>> cq;
      if (s == 1) {
        cq = col;
      } else {
        for (size_t t = q; t < col.size(); t += 2)
          if (col[t].second != 0.0) cq.push_back(col[t]);
      }
      const size_t before = cq.size();
      double nrm2 = 0.0;
      for (auto& e : cq) nrm2 += e.second * e.second;
      const double nrm = std::sqrt(nrm2);
      if (o.droptol > 0.0 && nrm > 0.0) {
        size_t w = 0;
        for (auto& e : cq)
          if (!(std::fabs(e.second) < o.droptol * nrm)) cq[w++] = e;
        cq.resize(w);
      }
      if (std::isfinite(o.fill)) {
        const int32_t cc = F.perm[j + q];
        int64_t cnt = 0;
        for (int64_t e = M.ptr[cc]; e < M.ptr[cc + 1]; ++e)
          if (pos[M.col[e]] >= j + s && M.val[e] != 0.0) ++cnt;
        const size_t cap = (size_t)std::ceil(o.fill * (double)cnt);
        if (cq.size() > cap) {
          std::sort(cq.begin(), cq.end(), [&](const auto& x, const auto& y) {
            const double ax = std::fabs(x.second), ay = std::fabs(y.second);
            return ax > ay || (ax == ay && pos[x.first] < pos[y.first]);
          });
          cq.resize(cap);
        }
      }
      F.dropped += (int64_t)(before - cq.size());
      std::sort(cq.begin(), cq.end(), [&](const auto& x, const auto& y) { return pos[x.first] < pos[y.first]; });
      const int32_t kpos = (int32_t)(j + q);
      blk_of[kpos] = b;
      for (auto& e : cq) {
        Lcol[kpos].push_back({e.first, e.second});
        Lrow[e.first].push_back({kpos, e.second});
      }
    }
    if (s == 2) F.n2x2++;
    j += s;
  }
  // L over positions (rows of the original indices in their final positions)
  F.L.nrows = F.L.ncols = n;
  F.L.ptr.assign(n + 1, 0);
  for (int64_t p = 0; p < n; ++p) {
    for (const Entry& e : Lrow[F.perm[p]]) {
      F.L.col.push_back(e.idx);
      F.L.val.push_back(e.v);
    }
    F.L.ptr[p + 1] = (int64_t)F.L.col.size();
  }
  return F;
}

IldlScaled ildl_scale(const IldlFactor& F) {
  const int64_t n = F.n;
  const int64_t nb = (int64_t)F.bstart.size();
  IldlScaled R;
  // per position: the 2x2 factor entries of its block's column(s)
  std::vector<double> c00(nb), c10(nb), c11(nb);
  R.mr.assign(3 * nb, 0.0);
  for (int64_t b = 0; b < nb; ++b) {
    const double* B = &F.bval[3 * b];
    const int32_t p = F.bstart[b];
    if (F.bsize[b] == 1) {
      c00[b] = std::sqrt(std::fabs(B[0]));
      const double m = (B[0] < 0.0 ? -1.0 : 1.0) - 1.0;
      R.mr[3 * b] = m;
      if (m != 0.0) {
        R.ur_pos.push_back(p); R.ur_pos.push_back(-1);
        R.ur_val.push_back(1.0); R.ur_val.push_back(0.0);
        R.sigma.push_back(m);
      }
      continue;
    }
    // |B| = V |Lambda| V^T, symmetrized, and its lower Cholesky factor
    double l[2], V[2][2];
    sym2_eig(B[0], B[1], B[2], l, V);
    double ab[2][2];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) ab[r][c] = V[r][0] * std::fabs(l[0]) * V[c][0] + V[r][1] * std::fabs(l[1]) * V[c][1];
    const double off = (ab[0][1] + ab[1][0]) / 2.0;
    const double a = std::sqrt(ab[0][0]);
    const double cb = off / a;
    const double d = std::sqrt(ab[1][1] - cb * cb);
    c00[b] = a; c10[b] = cb; c11[b] = d;
    // M_r block = C^-1 B C^-T - I (symmetrized)
    // T = C^-1 B (forward substitution on each column of B)
    const double Bm[2][2] = {{B[0], B[1]}, {B[1], B[2]}};
    double T[2][2];
    for (int c = 0; c < 2; ++c) {
      T[0][c] = Bm[0][c] / a;
      T[1][c] = (Bm[1][c] - cb * T[0][c]) / d;
    }
    // Mb = C^-1 T^T, transposed: Mb^T = (C^-1 T^T)^T
    double U2[2][2];  // U2 = C^-1 T^T
    for (int c = 0; c < 2; ++c) {
      U2[0][c] = T[c][0] / a;
      U2[1][c] = (T[c][1] - cb * U2[0][c]) / d;
    }
    double Mb[2][2];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) Mb[r][c] = U2[c][r] - (r == c ? 1.0 : 0.0);
    const double moff = (Mb[0][1] + Mb[1][0]) / 2.0;
    R.mr[3 * b] = Mb[0][0];
    R.mr[3 * b + 1] = moff;
    R.mr[3 * b + 2] = Mb[1][1];
    double ml[2], MV[2][2];
    sym2_eig(Mb[0][0], moff, Mb[1][1], ml, MV);
    for (int t = 0; t < 2; ++t)
      if (ml[t] < -1.0) {
        R.ur_pos.push_back(p); R.ur_pos.push_back(p + 1);
        R.ur_val.push_back(MV[0][t]); R.ur_val.push_back(MV[1][t]);
        R.sigma.push_back(ml[t]);
      }
  }
  // Lcal = L C by columns (positions), then the rows
  std::vector<int32_t> blk(n);
  for (int64_t b = 0; b < nb; ++b)
    for (int q = 0; q < F.bsize[b]; ++q) blk[F.bstart[b] + q] = (int32_t)b;
  Csr Lt = transpose(F.L);  // row k of Lt = column k of L (rows increasing)
  std::vector<std::vector<std::pair<int32_t, double>>> cols(n);
  for (int64_t b = 0; b < nb; ++b) {
    const int32_t p = F.bstart[b];
    if (F.bsize[b] == 1) {
      cols[p].push_back({p, c00[b]});
      for (int64_t e = Lt.ptr[p]; e < Lt.ptr[p + 1]; ++e) {
        const double v = Lt.val[e] * c00[b];
        if (v != 0.0) cols[p].push_back({Lt.col[e], v});
      }
      continue;
    }
    // column p: L_p c00 + L_{p+1} c10 (merge of two sorted lists); column p+1: L_{p+1} c11
    cols[p].push_back({p, c00[b]});
    if (c10[b] != 0.0) cols[p].push_back({p + 1, c10[b]});
    cols[p + 1].push_back({p + 1, c11[b]});
    int64_t e0 = Lt.ptr[p], e1 = Lt.ptr[p + 1];
    const int64_t f0 = Lt.ptr[p + 1], f1 = Lt.ptr[p + 2];
    int64_t u = e0, w = f0;
    (void)e1;
    while (u < f0 || w < f1) {
      int32_t r;
      double v0 = 0.0, v1 = 0.0;
      if (w >= f1 || (u < f0 && Lt.col[u] < Lt.col[w])) {
        r = Lt.col[u]; v0 = Lt.val[u]; ++u;
      } else if (u >= f0 || Lt.col[w] < Lt.col[u]) {
        r = Lt.col[w]; v1 = Lt.val[w]; ++w;
      } else {
        r = Lt.col[u]; v0 = Lt.val[u]; v1 = Lt.val[w]; ++u; ++w;
      }
      const double a = v0 * c00[b] + v1 * c10[b];
      if (a != 0.0) cols[p].push_back({r, a});
      const double d = v1 * c11[b];
      if (d != 0.0) cols[p + 1].push_back({r, d});
    }
  }
  // LcT: row k = column k of Lcal (diagonal first, rows increasing)
  R.LcT.nrows = R.LcT.ncols = n;
  R.LcT.ptr.assign(n + 1, 0);
  for (int64_t k = 0; k < n; ++k) {
    for (auto& e : cols[k]) { R.LcT.col.push_back(e.first); R.LcT.val.push_back(e.second); }
    R.LcT.ptr[k + 1] = (int64_t)R.LcT.col.size();
  }
  R.Lc = transpose(R.LcT);  // rows with columns increasing: the diagonal is last
  return R;
}

bool ildl_export(const IldlFactor& F, const IldlScaled& S, int which, std::vector<unsigned char>& out,
                 int64_t& count) {
  const int64_t n = F.n;
  auto put = [&](const void* src, int64_t cnt, size_t esz) {
    count = cnt;
    out.resize((size_t)cnt * esz);
    if (cnt > 0) std::memcpy(out.data(), src, (size_t)cnt * esz);
  };
  switch (which) {
    case ASSS_ARR_ILDL_PERM: put(F.perm.data(), n, 4); return true;
    case ASSS_ARR_ILDL_L_ROWPTR: put(F.L.ptr.data(), n + 1, 8); return true;
    case ASSS_ARR_ILDL_L_COLIND: put(F.L.col.data(), F.L.nnz(), 4); return true;
    case ASSS_ARR_ILDL_L_VAL: put(F.L.val.data(), F.L.nnz(), 8); return true;
    case ASSS_ARR_ILDL_BSIZE:
    case ASSS_ARR_ILDL_D: {
      std::vector<int32_t> bs(n, 0);
      std::vector<double> d(3 * n, 0.0);
      for (size_t b = 0; b < F.bstart.size(); ++b) {
        const int32_t p = F.bstart[b];
        bs[p] = F.bsize[b];
        for (int t = 0; t < 3; ++t) d[3 * (size_t)p + t] = F.bval[3 * b + t];
      }
      if (which == ASSS_ARR_ILDL_BSIZE) put(bs.data(), n, 4);
      else put(d.data(), 3 * n, 8);
      return true;
    }
    case ASSS_ARR_LCAL_ROWPTR: put(S.Lc.ptr.data(), n + 1, 8); return true;
    case ASSS_ARR_LCAL_COLIND: put(S.Lc.col.data(), S.Lc.nnz(), 4); return true;
    case ASSS_ARR_LCAL_VAL: put(S.Lc.val.data(), S.Lc.nnz(), 8); return true;
    case ASSS_ARR_UR: {
      const int64_t r = (int64_t)S.sigma.size();
      std::vector<double> U((size_t)(n * r), 0.0);
      for (int64_t c = 0; c < r; ++c)
        for (int t = 0; t < 2; ++t)
          if (S.ur_pos[2 * c + t] >= 0) U[(size_t)(c * n + S.ur_pos[2 * c + t])] = S.ur_val[2 * c + t];
      put(U.data(), n * r, 8);
      return true;
    }
    case ASSS_ARR_SIGMA_R: put(S.sigma.data(), (int64_t)S.sigma.size(), 8); return true;
    default: return false;
  }
}

LevelSchedule level_schedule(const Csr& T, bool lower) {
  const int64_t n = T.nrows;
  std::vector<int32_t> lev(n, 0);
  int32_t nl = 0;
  auto visit = [&](int64_t i) {
    int32_t l = 0;
    for (int64_t e = T.ptr[i]; e < T.ptr[i + 1]; ++e) {
      const int32_t c = T.col[e];
      if (c != i) l = std::max(l, lev[c] + 1);
    }
    lev[i] = l;
    nl = std::max(nl, l + 1);
  };
  if (lower)
    for (int64_t i = 0; i < n; ++i) visit(i);
  else
    for (int64_t i = n - 1; i >= 0; --i) visit(i);
  LevelSchedule S;
  S.ptr.assign(nl + 1, 0);
  for (int64_t i = 0; i < n; ++i) S.ptr[lev[i] + 1]++;
  for (int32_t l = 0; l < nl; ++l) {
    S.max_width = std::max(S.max_width, S.ptr[l + 1]);
    S.ptr[l + 1] += S.ptr[l];
  }
  S.rows.resize(n);
  std::vector<int32_t> cur(S.ptr.begin(), S.ptr.end() - 1);
  for (int64_t i = 0; i < n; ++i) S.rows[cur[lev[i]]++] = (int32_t)i;
  return S;
}

}  // namespace asss
