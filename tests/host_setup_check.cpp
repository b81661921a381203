// Host check of the setup stages that run on the CPU (Sec. 2 and Sec. 3):
// matching, canonical scaling, Abar, the pattern of S, the least-squares
// system of App. A, and, for S values given from outside, A_hat = Abar S,
// D, Omega and J_tilde.  Reads a binary input file, writes a binary output
// file; the test compares both with the oracle.
//
// Input  (native endianness): int64 n, int64 nnz, int32 s_kind, rowptr[n+1]
//        int64, colind[nnz] int32, val[nnz] f64, int64 nS, S values[nS] f64
//        (CSR order of the S pattern; nS = 0 skips the split).
// Output: m[n] i32, Dr[n], Dc[n], Abar ptr/col/val, S ptr/col, B nrows ncols
//         nnz, B ptr/col/val, rhs, then (if nS > 0) D[n], Omega[n], J upper
//         ptr/col/val -- every array preceded by its int64 length.
#include "host_setup.hpp"
#include <cstdio>
#include <vector>
using namespace asss;

template <typename T>
static bool rd(FILE* f, std::vector<T>& v, int64_t n) {
  v.resize(n);
  return n == 0 || fread(v.data(), sizeof(T), n, f) == (size_t)n;
}
template <typename T>
static void wr(FILE* f, const std::vector<T>& v) {
  int64_t n = (int64_t)v.size();
  fwrite(&n, 8, 1, f);
  if (n) fwrite(v.data(), sizeof(T), n, f);
}

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t n = 0, nnz = 0, nS = 0;
  int32_t kind = 1;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> va, sv;
  if (fread(&n, 8, 1, f) != 1 || fread(&nnz, 8, 1, f) != 1 || fread(&kind, 4, 1, f) != 1) return 2;
  if (!rd(f, rp, n + 1) || !rd(f, ci, nnz) || !rd(f, va, nnz)) return 2;
  if (fread(&nS, 8, 1, f) != 1 || !rd(f, sv, nS)) return 2;
  fclose(f);
  try {
    Csr A = validate_and_copy(n, nnz, rp.data(), ci.data(), va.data());
    std::vector<int32_t> m = max_product_matching(A);
    std::vector<double> Dr, Dc;
    canonical_scaling(A, m, Dr, Dc);
    Csr Abar = permute_scale(A, m, Dr, Dc);
    Csr Spat = s_pattern(Abar, kind, nullptr, nullptr);
    LlsSystem L;
    build_lls(Abar, Spat, 1.0, L);
    FILE* o = fopen(argv[2], "wb");
    if (!o) return 2;
    wr(o, m); wr(o, Dr); wr(o, Dc);
    wr(o, Abar.ptr); wr(o, Abar.col); wr(o, Abar.val);
    wr(o, Spat.ptr); wr(o, Spat.col);
    std::vector<int64_t> shape{L.B.nrows, L.B.ncols, L.B.nnz()};
    wr(o, shape);
    wr(o, L.B.ptr); wr(o, L.B.col); wr(o, L.B.val); wr(o, L.rhs);
    if (nS > 0) {
      if (nS != Spat.nnz()) return 3;
      Csr S = Spat;
      S.val = sv;
      Csr Ahat = spgemm_on_pattern(Abar, S, L.P);
      std::vector<double> D, Om, jv;
      split_ahat(Ahat, L.U, D, Om, jv);
      wr(o, D); wr(o, Om); wr(o, L.U.ptr); wr(o, L.U.col); wr(o, jv);
    }
    fclose(o);
  } catch (const HostError& e) {
    printf("error %d: %s\n", e.code, e.msg.c_str());
    return 4;
  }
  return 0;
}
