// Host-side preprocessing of the ASSS scheme (paper Sec. 2 and Sec. 3).
// Pure C++17; parallel loops use std::thread.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace asss {

struct Csr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> ptr;  // nrows + 1
  std::vector<int32_t> col;  // sorted within a row
  std::vector<double> val;   // may be empty for a pattern
  int64_t nnz() const { return (int64_t)col.size(); }
};

struct HostError {
  int code;
  std::string msg;
};

int num_threads();

// f(lo, hi) over contiguous chunks of [0, n), run on num_threads() threads.
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& f);

// Validate a caller CSR and copy it, dropping stored zeros (Sec. 1: a general
// sparse matrix; a stored zero is no nonzero).  Throws HostError.
Csr validate_and_copy(int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colind,
                      const double* val);

// New values for the stored pattern `pat` (the pattern kept at setup, explicit
// zeros dropped) from a caller CSR with the same checks as validate_and_copy:
// an entry of the caller inside the pattern sets that value, a zero outside it
// is ignored, a nonzero outside it is an INVALID_ARG error, and pattern entries
// the caller does not list become zero.
Csr map_values_onto(const Csr& pat, int64_t n, int64_t nnz, const int64_t* rowptr,
                    const int32_t* colind, const double* val);

Csr transpose(const Csr& A);

// Maximum product perfect matching (Sec. 2, eq. mc64): m[j] = row matched to
// column j.  Successive shortest augmenting paths (Dijkstra with dual
// potentials) on the costs c_ij = log(max_k |a_kj|) - log|a_ij|.
std::vector<int32_t> max_product_matching(const Csr& A);

// Scalings for the matching (largest gamma <= 0 with gamma_j <= gamma_i + w_ij,
// w_ij = log|at_ii| - log|at_ij| for At = P A).  Dr indexed by rows of A.
void canonical_scaling(const Csr& A, const std::vector<int32_t>& m, std::vector<double>& Dr,
                       std::vector<double>& Dc);

// Abar = P Dr A Dc with (P y)_j = y_{m[j]}.
Csr permute_scale(const Csr& A, const std::vector<int32_t>& m, const std::vector<double>& Dr,
                  const std::vector<double>& Dc);

// Pattern of S (values unset).  kind: 0 diag, 1 tridiag, 2 pattern of Abar, 3 user.
Csr s_pattern(const Csr& Abar, int kind, const int64_t* urow, const int32_t* ucol);

// Least-squares system of App. A for the pattern Spat.  Unknowns are the
// pattern entries of S in CSR (row-major) order; equations are the strictly
// upper pairs of pattern(Abar S) + its transpose in row-major order, then the
// n diagonal equations weighted by sqrt(gamma).
struct LlsSystem {
  Csr B, Bt;                 // B: equations x unknowns; Bt its transpose
  std::vector<double> rhs;   // 0 for pair equations, sqrt(gamma) for diagonal ones
  Csr P;                     // pattern of Abar S
  Csr U;                     // strictly upper pattern of P + P^T (pattern of J_tilde)
};
void build_lls(const Csr& Abar, const Csr& Spat, double gamma, LlsSystem& out);

// Numeric A_hat = Abar S on the structural pattern P.
Csr spgemm_on_pattern(const Csr& Abar, const Csr& S, const Csr& P);

// D = diag(A_hat), Omega = |D|^-1/2, J_tilde strict upper values on U
// (u_ij = Omega_i Omega_j (ahat_ij - ahat_ji) / 2).  Throws on a zero D_i.
void split_ahat(const Csr& Ahat, const Csr& U, std::vector<double>& D, std::vector<double>& Omega,
                std::vector<double>& jval);

// Sliced storage of the skew operator for the GPU kernels.  Rows are cut into
// blocks of R rows (a multiple of 64) and each block into slices of 64 rows
// (one wavefront, one row per lane).  For a row i:
//   part a: upper entries (i, j), j > i, with j in i's block, local column
//           j - block_start (uint16) -- used for a gather from and a scatter
//           into the block's LDS window;
//   part b: every entry whose column lies in another block, both triangles,
//           with the signed value of J_tilde (lower entries are -u_ji).
// Each part of a slice is stored column-major in (width x 64) with padding
// entries (local/global column = the row itself, value 0).
//
// Column forms (form):
//   SKEW_WIDE    part a: 16-bit local columns; part b: 32-bit global columns;
//   SKEW_NARROW  part b as a 16-bit delta from a per-(slice, slot) base, when
//                every slot spans fewer than 2^16 columns;
//   SKEW_SLOTS   no per-entry columns: each slot of a slice holds one offset d
//                (column = row + d) for all 64 lanes, lanes without that entry
//                hold value 0.  Part a keeps d per slot (a_doff, d > 0), part b
//                the column of lane 0 (b_base = first row of the slice + d); the
//                reader clamps a padding lane's column into the block (part a)
//                or into [0, n) (part b).  Slots are the sorted distinct offsets
//                of the slice's entries in each part, so a grid pattern needs
//                about as many slots as it has entries per row.
enum { SKEW_AUTO = 0, SKEW_WIDE = 1, SKEW_NARROW = 2, SKEW_SLOTS = 3 };
struct SkewSell {
  int32_t n = 0, R = 0, nblocks = 0, nslices = 0;
  std::vector<int32_t> a_width, b_width;  // per slice
  std::vector<int64_t> a_off, b_off;      // per slice, offset in entries
  std::vector<uint16_t> a_col;
  std::vector<int32_t> b_col;             // global column (wide form)
  // narrow form of the part-b columns, used when every (slice, slot) of part
  // b spans fewer than 2^16 columns (grid-like matrices): column = base of the
  // slot + 16-bit delta; b_base has one entry per slot (b_off[s] / 64 + l)
  bool b_narrow = false;
  std::vector<int32_t> b_base;
  std::vector<uint16_t> b_cd;
  std::vector<int32_t> a_doff;            // SKEW_SLOTS: offset d per part-a slot
  std::vector<double> a_val, b_val;
  int64_t a_entries = 0, b_entries = 0;   // real (unpadded) entries
  int32_t form = SKEW_WIDE;
};
// form: SKEW_AUTO picks SKEW_SLOTS when it stores at most 1.2 times the
// entries (padding included) of the per-entry-column forms, else SKEW_NARROW
// when it fits, else SKEW_WIDE.  A forced SKEW_NARROW that does not fit, or a
// forced SKEW_SLOTS that would store more than 16 times as many entries,
// throws HostError(ASSS_ERR_INVALID_ARG).
SkewSell pack_skew_sell(const Csr& Jup, int32_t R, int32_t form = SKEW_AUTO);

// Order of the inner system for a lexicographic 3D grid (node x + m1 y +
// m1 m2 z): detected from the pattern of Abar, whose positive column offsets
// must be exactly {1, m1, m1 m2} with m1 m2 dividing n.  Rows are then grouped
// into tiles of ty x tz whole x-lines (tiles in lexicographic (y, z) order,
// lines y-fastest inside a tile), ty tz a power of two as close to
// target_R / m1 as fits, ty | m2, tz | m3, ty and tz as equal as possible, and
// m1 ty tz a multiple of 64 (at most 4096): one tile per row block of that
// size, returned in R_out.  Returns perm (new -> old), or an empty vector
// when the pattern is not such a grid or no tile fits.
std::vector<int32_t> grid_line_order(const Csr& Abar, int32_t target_R, int32_t& R_out);

// Strict upper triangle of P J P^T for the permutation perm (new -> old) of
// the skew matrix whose strict upper triangle is U (values u_ij, lower -u_ij).
Csr permute_skew_upper(const Csr& U, const std::vector<int32_t>& perm);

// Number of upper pairs (i, j) of U with i and j in different R-blocks.
int64_t count_cross_pairs(const Csr& U, int32_t R);

}  // namespace asss
