// Host check of the sliced skew storage: packs the strict upper triangle of a
// 25-point grid pattern (random values) and applies the skew matrix through the
// packed form and through the CSR; exits 0 when they agree to rounding.
// Usage: host_pack_check m R  (prints whether the 16-bit column form was chosen)
#include "host_setup.hpp"
#include <cstdio>
#include <random>
#include <map>
using namespace asss;
int main(int argc, char** argv) {
  int m = argc > 1 ? atoi(argv[1]) : 64;
  int R = argc > 2 ? atoi(argv[2]) : 2048;
  int64_t n = (int64_t)m * m * m;
  // strict upper triangle of the 25-point pattern (offsets = sums of two 7-point offsets)
  std::vector<std::array<int,3>> offs;
  int e[7][3] = {{0,0,0},{1,0,0},{-1,0,0},{0,1,0},{0,-1,0},{0,0,1},{0,0,-1}};
  std::map<std::array<int,3>, int> seen;
  for (auto& a : e) for (auto& b : e) { std::array<int,3> o{a[0]+b[0], a[1]+b[1], a[2]+b[2]}; seen[o] = 1; }
  std::mt19937_64 rng(7); std::uniform_real_distribution<double> U(-1, 1);
  Csr J; J.nrows = J.ncols = n; J.ptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    int x = i % m, y = (i / m) % m, z = i / ((int64_t)m * m);
    std::vector<int64_t> cols;
    for (auto& kv : seen) {
      auto o = kv.first; int xx = x + o[0], yy = y + o[1], zz = z + o[2];
      if (xx < 0 || yy < 0 || zz < 0 || xx >= m || yy >= m || zz >= m) continue;
      int64_t j = xx + (int64_t)m * (yy + (int64_t)m * zz);
      if (j > i) cols.push_back(j);
    }
    std::sort(cols.begin(), cols.end());
    for (auto c : cols) { J.col.push_back((int32_t)c); J.val.push_back(U(rng)); }
    J.ptr[i + 1] = J.col.size();
  }
  SkewSell S = pack_skew_sell(J, R);
  printf("n=%lld nh=%lld narrow=%d a=%lld b=%lld stored_b=%lld\n", (long long)n, (long long)J.nnz(), (int)S.b_narrow,
         (long long)S.a_entries, (long long)S.b_entries, (long long)S.b_off[S.nslices]);
  // rebuild: y = J_full v through the sliced storage vs through the CSR (both triangles)
  std::vector<double> v(n), y1(n, 0.0), y2(n, 0.0);
  for (auto& t : v) t = U(rng);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = J.ptr[i]; p < J.ptr[i + 1]; ++p) { y1[i] += J.val[p] * v[J.col[p]]; y1[J.col[p]] -= J.val[p] * v[i]; }
  for (int64_t s = 0; s < S.nslices; ++s)
    for (int lane = 0; lane < 64; ++lane) {
      int64_t i = s * 64 + lane; if (i >= n) continue;
      int64_t b0 = (i / R) * R;
      for (int l = 0; l < S.a_width[s]; ++l) {
        int64_t q = S.a_off[s] + (int64_t)l * 64 + lane;
        int64_t j = b0 + S.a_col[q];
        y2[i] += S.a_val[q] * v[j]; y2[j] -= S.a_val[q] * v[i];
      }
      for (int l = 0; l < S.b_width[s]; ++l) {
        int64_t q = S.b_off[s] + (int64_t)l * 64 + lane;
        int64_t j = S.b_narrow ? (int64_t)S.b_base[q / 64] + S.b_cd[q] : S.b_col[q];
        if (j < 0 || j >= n) { printf("BAD col %lld\n", (long long)j); return 1; }
        y2[i] += S.b_val[q] * v[j];
      }
    }
  double md = 0, mx = 0;
  for (int64_t i = 0; i < n; ++i) { md = std::max(md, std::fabs(y1[i] - y2[i])); mx = std::max(mx, std::fabs(y1[i])); }
  printf("max |diff| %.3e (max |y| %.3e)\n", md, mx);
  return md <= 1e-12 * mx ? 0 : 2;
}
