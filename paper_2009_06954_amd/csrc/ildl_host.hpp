// Host part of the general preconditioner of paper Sec. 3: the incomplete
// LDL^T factorization of M_hat = (A_hat + A_hat^T) / 2 with Bunch-Kaufman
// pivoting, the scaled factor of eq. absfac, the low-rank term of Fig. 1, and
// the level schedules of the two triangular solves that every application of
// J_tilde = Lcal^-1 J_hat Lcal^-T performs on the device.  Pure C++17.
#pragma once

#include <cmath>
#include <cstdint>
#include <vector>

#include "host_setup.hpp"

namespace asss {

struct IldlOpts {
  double droptol = 0.0;       // drop l_ij when |l_ij| < droptol ||l_j||_2 (0: none)
  double fill = INFINITY;     // keep at most ceil(fill c_j) entries per column (inf: all)
  bool pivoting = true;       // Bunch-Kaufman; false: 1x1 pivots in the natural order
};

// M[perm][:, perm] = L D L^T + E.  Positions p = 0..n-1; position p holds the
// original index perm[p].  L: strictly lower part of the unit lower factor,
// CSR over positions (columns increasing).  Pivot blocks b: first position
// bstart[b], size bsize[b] (1 or 2), values bval[3 b .. 3 b + 2] = (d11, d21,
// d22) of the symmetric block (d21 = d22 = 0 for a 1x1 block).
struct IldlFactor {
  int64_t n = 0;
  std::vector<int32_t> perm;
  Csr L;
  std::vector<int32_t> bstart;
  std::vector<int32_t> bsize;
  std::vector<double> bval;
  int64_t dropped = 0;
  int32_t n2x2 = 0;
};

// Throws HostError(ASSS_ERR_ZERO_DIAGONAL) on a zero pivot that pivoting
// cannot avoid, HostError(ASSS_ERR_INVALID_ARG) if M is not symmetric.
IldlFactor ildl_bunch_kaufman(const Csr& M, const IldlOpts& o);

// Scaled factor and low-rank term.  C = blockdiag(C_b), C_b the lower
// Cholesky factor of |B_b| = V |Lambda| V^T; Lcal = L C (lower triangular,
// CSR over positions with the diagonal as the last entry of each row) and
// its transpose (upper, diagonal first).  M_r = C^-1 D C^-T - I is block
// diagonal with eigenvalues 0 or -2; U_r holds one column per eigenpair of a
// block with eigenvalue below -1 (Fig. 1 walked block by block over all
// blocks): column c has ur_val[2c], ur_val[2c+1] at positions ur_pos[2c],
// ur_pos[2c+1] (ur_pos[2c+1] = -1 for a column of a 1x1 block), sigma[c] its
// eigenvalue.
struct IldlScaled {
  Csr Lc, LcT;
  std::vector<int32_t> ur_pos;
  std::vector<double> ur_val;
  std::vector<double> sigma;
  std::vector<double> mr;  // 3 values per block: (m11, m21, m22) of M_r's block
};
IldlScaled ildl_scale(const IldlFactor& F);

// Level schedule of a triangular solve with the CSR T (rows over positions,
// the diagonal stored in each row): level(i) = 1 + max level(j) over the
// off-diagonal entries (i, j) of row i, which all lie before i (lower) or all
// after it (upper).  rows: the rows level by level (increasing row index within
// a level), ptr: nlevels + 1 offsets into rows.
struct LevelSchedule {
  std::vector<int32_t> rows;
  std::vector<int32_t> ptr;
  int32_t max_width = 0;
  int32_t nlevels() const { return (int32_t)ptr.size() - 1; }
};
LevelSchedule level_schedule(const Csr& T, bool lower);

// Symmetric and skew parts of A_hat on the union of its pattern and its
// transpose's: M = (A + A^T) / 2 (entries that are exactly zero dropped) and
// J = (A - A^T) / 2 (both triangles, exactly skew: the lower entry is the
// negation of the upper one).
void symmetric_skew_split(const Csr& A, Csr& M, Csr& J);

// P A P^T for perm (new -> old): row p of the result is row perm[p] with
// columns mapped to positions (sorted).
Csr permute_symmetric(const Csr& A, const std::vector<int32_t>& perm);

// Array `which` (ASSS_ARR_ILDL_* / LCAL_* / UR / SIGMA_R of include/asss.h)
// as raw bytes and its element count; false for another id.
bool ildl_export(const IldlFactor& F, const IldlScaled& S, int which, std::vector<unsigned char>& out,
                 int64_t& count);

}  // namespace asss
