// Host check of the sliced skew storage: packs the strict upper triangle of a
// 25-point grid pattern (random values) and applies the skew matrix through the
// packed form and through the CSR; exits 0 when they agree to rounding.
// Usage: host_pack_check m R [form [random]]  (form 0 automatic, 1 wide,
// 2 narrow, 3 offset slots; prints the form used; "random": m^3 rows with 12
// random upper entries each instead of the grid pattern; a rejected form
// exits with 3).  The slot form is read the way the
// kernels read it: columns from the slot offsets, clamped into the block
// (part a) or into [0, n) (part b); every real entry must need no clamping.
#include "host_setup.hpp"
#include <cstdio>
#include <random>
#include <map>
#include <string>
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
  const bool random = argc > 4 && std::string(argv[4]) == "random";
  std::uniform_int_distribution<int64_t> C(0, n - 1);
  for (int64_t i = 0; i < n; ++i) {
    int x = i % m, y = (i / m) % m, z = i / ((int64_t)m * m);
    std::vector<int64_t> cols;
    if (random) {
      for (int t = 0; t < 12; ++t) { int64_t j = C(rng); if (j > i) cols.push_back(j); }
      std::sort(cols.begin(), cols.end());
      cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    }
    for (auto& kv : seen) {
      if (random) break;
      auto o = kv.first; int xx = x + o[0], yy = y + o[1], zz = z + o[2];
      if (xx < 0 || yy < 0 || zz < 0 || xx >= m || yy >= m || zz >= m) continue;
      int64_t j = xx + (int64_t)m * (yy + (int64_t)m * zz);
      if (j > i) cols.push_back(j);
    }
    std::sort(cols.begin(), cols.end());
    for (auto c : cols) { J.col.push_back((int32_t)c); J.val.push_back(U(rng)); }
    J.ptr[i + 1] = J.col.size();
  }
  int form = argc > 3 ? atoi(argv[3]) : 0;
  SkewSell S;
  try {
    S = pack_skew_sell(J, R, form);
  } catch (const HostError& e) {
    printf("rejected: %s\n", e.msg.c_str());
    return 3;
  }
  printf("n=%lld nh=%lld form=%d narrow=%d a=%lld b=%lld stored_a=%lld stored_b=%lld\n", (long long)n,
         (long long)J.nnz(), (int)S.form, (int)S.b_narrow, (long long)S.a_entries, (long long)S.b_entries,
         (long long)S.a_off[S.nslices], (long long)S.b_off[S.nslices]);
  const bool slots = S.form == SKEW_SLOTS;
  // rebuild: y = J_full v through the sliced storage vs through the CSR (both triangles)
  std::vector<double> v(n), y1(n, 0.0), y2(n, 0.0);
  for (auto& t : v) t = U(rng);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = J.ptr[i]; p < J.ptr[i + 1]; ++p) { y1[i] += J.val[p] * v[J.col[p]]; y1[J.col[p]] -= J.val[p] * v[i]; }
  int64_t real_a = 0, real_b = 0;
  for (int64_t s = 0; s < S.nslices; ++s)
    for (int lane = 0; lane < 64; ++lane) {
      int64_t i = s * 64 + lane;
      int64_t b0 = ((s * 64) / R) * R;
      int64_t nrow = std::min<int64_t>(R, n - b0);
      int64_t il = i - b0;
      for (int l = 0; l < S.a_width[s]; ++l) {
        int64_t q = S.a_off[s] + (int64_t)l * 64 + lane;
        int64_t jl;
        if (slots) {
          int64_t d = S.a_doff[q / 64];
          if (d <= 0) { printf("BAD part-a offset %lld\n", (long long)d); return 1; }
          jl = std::min(il + d, nrow - 1);
          if (S.a_val[q] != 0.0 && (il + d >= nrow || i >= n)) { printf("BAD clamped real entry\n"); return 1; }
        } else {
          jl = S.a_col[q];
        }
        if (jl < 0 || jl >= nrow) { printf("BAD local col %lld\n", (long long)jl); return 1; }
        if (S.a_val[q] != 0.0) ++real_a;
        if (i >= n) continue;  // rows past n are not rows of the matrix
        int64_t j = b0 + jl;
        y2[i] += S.a_val[q] * v[j]; y2[j] -= S.a_val[q] * v[i];
      }
      for (int l = 0; l < S.b_width[s]; ++l) {
        int64_t q = S.b_off[s] + (int64_t)l * 64 + lane;
        int64_t j;
        if (slots) {
          int64_t raw = (int64_t)S.b_base[q / 64] + lane;
          j = std::min<int64_t>(std::max<int64_t>(raw, 0), n - 1);
          if (S.b_val[q] != 0.0 && (raw != j || i >= n || raw / R == i / R)) { printf("BAD real part-b entry\n"); return 1; }
        } else {
          j = S.b_narrow ? (int64_t)S.b_base[q / 64] + S.b_cd[q] : S.b_col[q];
        }
        if (j < 0 || j >= n) { printf("BAD col %lld\n", (long long)j); return 1; }
        if (S.b_val[q] != 0.0) ++real_b;
        if (i >= n) continue;
        y2[i] += S.b_val[q] * v[j];
      }
    }
  if (real_a != S.a_entries || real_b != S.b_entries) {
    printf("BAD entry counts %lld %lld\n", (long long)real_a, (long long)real_b);
    return 1;
  }
  double md = 0, mx = 0;
  for (int64_t i = 0; i < n; ++i) { md = std::max(md, std::fabs(y1[i] - y2[i])); mx = std::max(mx, std::fabs(y1[i])); }
  printf("max |diff| %.3e (max |y| %.3e)\n", md, mx);
  return md <= 1e-12 * mx ? 0 : 2;
}
