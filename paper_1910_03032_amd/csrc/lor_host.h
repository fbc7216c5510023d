// Host side of the low-order-refined preconditioner (Section 5.2): the sparse LOR matrix
// and its smoothed-aggregation multigrid hierarchy (plain C++ on the host threads, no
// device code; every sum in a fixed order, so the results do not depend on the number of
// threads).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace sfem {

// Host CSR matrix (sorted column indices per row, no duplicates).
struct HostCsr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  int64_t nnz() const { return (int64_t)col.size(); }
};

// A_LOR = alpha M_LOR + beta nu_e K_LOR on the refined mesh that splits every element
// into the p^3 sub-hexahedra between its GLL points (gll: the p + 1 points on [-1, 1]),
// each the trilinear element through its 8 corner nodes, integrated with 2 x 2 x 2 Gauss
// points; nu_e (per element, may be null: 1) scales the stiffness of element e's
// sub-elements; rows and columns of essential DoFs (ess[g] != 0) are constrained
// (identity rows, zero columns).  xyz [nelem][8][3], dofs [nelem][(p+1)^3] (unflagged).
void lor_assemble(int p, const double *gll, int64_t nelem, const double *xyz, const int32_t *dofs,
                  int64_t ndof, const uint8_t *ess, double alpha, double beta, const double *nu_e,
                  HostCsr &A);

// Multigrid hierarchy on the host: A[0] = A_LOR, A[l + 1] = P[l]^T A[l] P[l], the spectral
// radius estimates rho[l] of D^-1 A[l], and the dense pseudo-inverse of the last A.
struct HostAmg {
  std::vector<HostCsr> A, P;
  std::vector<double> rho;
  std::vector<double> coarse;
};

// T = A^T (sorted columns).
void csr_transpose(const HostCsr &A, HostCsr &T);

// Sliced ELL form of a matrix (rows in slices of kSellRows; see DevSell in lor.h for the
// layout): value array, per-slice offsets and column forms, explicit columns, patterns.
constexpr int kSellRows = 64;
struct HostSell {
  int64_t nrows = 0, ncols = 0, pattern_slices = 0;
  std::vector<int32_t> off, pinfo, col, pat;
  std::vector<double> val;
};
// Build S from H.  With patterns (square H only), a slice whose rows' column offsets
// (col - row) number at most 1/8 more than its longest row stores that union of offsets
// once (shared by every slice that has the same one) instead of a column index per entry.
// Returns an empty string or an error message.
std::string sell_build(const HostCsr &H, bool patterns, HostSell &S);

// Smoothed-aggregation setup of A0 (strength threshold theta; stop at <= coarse_size
// rows or max_levels levels).  Returns an empty string or an error message.
std::string amg_build_host(const HostCsr &A0, double theta, int64_t coarse_size, int max_levels,
                           HostAmg &H);

}  // namespace sfem
