// Low-order-refined (LOR) preconditioner of Section 5.2: the Q1 operator on the
// GLL-refined mesh, assembled as a sparse matrix on the host, and a smoothed-aggregation
// algebraic multigrid hierarchy for it whose V-cycle runs on the GPU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lor_host.h"

namespace sfem {

// Device copy of a CSR matrix (int32 row offsets: nnz < 2^31); val32 is the FP32 copy of
// the values (made with the FP32 V-cycle's data, else null).
struct DevCsr {
  int64_t nrows = 0, ncols = 0, nnz = 0;
  int32_t *ptr = nullptr, *col = nullptr;
  double *val = nullptr;
  float *val32 = nullptr;
};
template <typename T>
inline const T *csr_vals(const DevCsr &A) {
  if constexpr (sizeof(T) == 8) return A.val;
  else return A.val32;
}

// Device copy of a matrix in sliced ELL form: rows in slices of kSellRows (one
// wave); slice s holds len_s = (off[s+1] - off[s]) / kSellRows values per row, stored
// entry-major (entry k of the slice's row r at off[s] + k kSellRows + r), so that a thread
// per row reads the values of its slice in contiguous runs.  The columns of a slice come
// in one of two forms (pinfo[s]):
//   pinfo[s] >= 0: explicit, entry k of row r in column col[pinfo[s] + k kSellRows + r],
//     rows shorter than len_s padded with (their last column, 0);
//   pinfo[s] < 0: a column-offset pattern shared by the slice's rows, entry k of row i in
//     column i + pat[-pinfo[s] - 1 + k] (clamped to [0, ncols)), value 0 where the row
//     has no entry there.  The rows of a square operator on a structured numbering (the
//     27-point couplings of a Q1 operator) share their offsets, so such slices read no
//     column indices at all.
// (kSellRows and the host-side construction, sell_build, are in lor_host.h.)
struct DevSell {
  int64_t nrows = 0, ncols = 0, nnz = 0, padded = 0;  // padded: stored values
  int64_t pattern_slices = 0;
  int32_t *off = nullptr, *pinfo = nullptr;  // [nslices + 1], [nslices]
  int32_t *col = nullptr, *pat = nullptr;    // explicit columns, offset patterns
  double *val = nullptr;
  float *val32 = nullptr;
};
template <typename T>
inline const T *sell_vals(const DevSell &A) {
  if constexpr (sizeof(T) == 8) return A.val;
  else return A.val32;
}

// A matrix of the hierarchy in one of the two forms: sliced ELL for many short rows of
// similar length (a thread per row), CSR otherwise (a group of lanes per row: few or long
// rows, where a thread per row would leave the GPU idle or pad much).
struct DevMat {
  bool sell = false;
  DevSell S;
  DevCsr C;
  int64_t nrows() const { return sell ? S.nrows : C.nrows; }
};

// Per-level data in the precision T of a V-cycle.
template <typename T>
struct LevelVecs {
  T *dinv = nullptr;                           // 1 / diag(A)
  T *b = nullptr, *x = nullptr, *t = nullptr;  // work vectors (nrows)
};

struct AmgLevel {
  DevMat A, P, R;              // operator, prolongator (to this level from the next), P^T
  double omega = 0.0;          // Jacobi damping 4 / (3 rho(D^-1 A))
  LevelVecs<double> d;         // FP64 V-cycle
  LevelVecs<float> f;          // FP32 V-cycle (after amg_make_f32)
  template <typename T>
  const LevelVecs<T> &vecs() const {
    if constexpr (sizeof(T) == 8) return d;
    else return f;
  }
};

// Smoothed-aggregation hierarchy (setup on the host, data on the device).
struct Amg {
  std::vector<AmgLevel> lv;
  double *coarse = nullptr;    // dense pseudo-inverse of the coarsest operator [n][n]
  float *coarse32 = nullptr;   // its FP32 copy (after amg_make_f32)
  bool has32 = false;
  int64_t ncoarse = 0;
  int nu = 2;                  // Jacobi sweeps before and after the coarse correction
  std::vector<int64_t> rows, nnzs;
  std::vector<int32_t> sliced;  // per level: bit 0 A, bit 1 P, bit 2 R in sliced ELL,
                               // bit 3 slices of A with a column-offset pattern
  std::vector<void *> bufs;    // every device allocation
  double setup_ms = 0.0;
};

// Build the hierarchy of A (strength threshold theta, stop at <= coarse_size rows or
// max_levels levels) and upload it.  Returns an empty string or an error message.
std::string amg_setup(const HostCsr &A, double theta, int64_t coarse_size, int max_levels, int nu,
                      Amg &out);
void amg_free(Amg &amg);
// FP32 copies of the hierarchy's values, diagonals and coarse inverse, and FP32 work
// vectors, for amg_vcycle<float> (the FP64 data stays).  Empty string or an error message.
std::string amg_make_f32(Amg &amg, hipStream_t s);
// x = V-cycle(b) on the finest level in precision T (b, x: device [n], distinct; T = float
// after amg_make_f32).
template <typename T>
hipError_t amg_vcycle(const Amg &amg, const T *b, T *x, hipStream_t s);
// y = A_0 x (the finest operator).
hipError_t amg_apply_fine(const Amg &amg, const double *x, double *y, hipStream_t s);

// Kernel launchers (k_lor.hip); T = double or float (the matrix values of that precision).
// x_out = x_in + omega dinv (b - A x_in); x_in == null: x_out = omega dinv b
template <typename T>
hipError_t launch_mat_jacobi(const DevMat &A, const T *dinv, T omega, const T *b, const T *x_in,
                             T *x_out, hipStream_t s);
// r = b - A x
template <typename T>
hipError_t launch_mat_residual(const DevMat &A, const T *b, const T *x, T *r, hipStream_t s);
// y = M x (accumulate: y += M x)
template <typename T>
hipError_t launch_mat_spmv(const DevMat &M, const T *x, T *y, bool accumulate, hipStream_t s);
// out = (TO) in
template <typename TI, typename TO>
hipError_t launch_convert(const TI *in, TO *out, int64_t n, hipStream_t s);
// out = a x + b y (out may alias x or y)
hipError_t launch_axpby(int64_t n, double a, const double *x, double b, const double *y, double *out,
                        hipStream_t s);
// y = C x for a dense row-major [n][n] C
template <typename T>
hipError_t launch_dense_matvec(const T *C, int64_t n, const T *x, T *y, hipStream_t s);

}  // namespace sfem
