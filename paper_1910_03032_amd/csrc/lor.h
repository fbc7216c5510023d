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

// Device copy of a CSR matrix (int32 row offsets: nnz < 2^31).
struct DevCsr {
  int64_t nrows = 0, ncols = 0, nnz = 0;
  int32_t *ptr = nullptr, *col = nullptr;
  double *val = nullptr;
};

struct AmgLevel {
  DevCsr A, P, R;              // operator, prolongator (to this level from the next), P^T
  double *dinv = nullptr;      // 1 / diag(A)
  double omega = 0.0;          // Jacobi damping 4 / (3 rho(D^-1 A))
  double *b = nullptr, *x = nullptr, *t = nullptr;  // work vectors (nrows)
};

// Smoothed-aggregation hierarchy (setup on the host, data on the device).
struct Amg {
  std::vector<AmgLevel> lv;
  double *coarse = nullptr;    // dense pseudo-inverse of the coarsest operator [n][n]
  int64_t ncoarse = 0;
  int nu = 2;                  // Jacobi sweeps before and after the coarse correction
  std::vector<int64_t> rows, nnzs;
  std::vector<void *> bufs;    // every device allocation
  double setup_ms = 0.0;
};

// Build the hierarchy of A (strength threshold theta, stop at <= coarse_size rows or
// max_levels levels) and upload it.  Returns an empty string or an error message.
std::string amg_setup(const HostCsr &A, double theta, int64_t coarse_size, int max_levels, int nu,
                      Amg &out);
void amg_free(Amg &amg);
// x = V-cycle(b) on the finest level (b, x: device [n], distinct).
hipError_t amg_vcycle(const Amg &amg, const double *b, double *x, hipStream_t s);
// y = A_0 x (the finest operator).
hipError_t amg_apply_fine(const Amg &amg, const double *x, double *y, hipStream_t s);

// Kernel launchers (k_lor.hip).
// x_out = x_in + omega dinv (b - A x_in); x_in == null: x_out = omega dinv b
hipError_t launch_csr_jacobi(const DevCsr &A, const double *dinv, double omega, const double *b,
                             const double *x_in, double *x_out, hipStream_t s);
// r = b - A x
hipError_t launch_csr_residual(const DevCsr &A, const double *b, const double *x, double *r,
                               hipStream_t s);
// y = M x (accumulate: y += M x)
hipError_t launch_csr_spmv(const DevCsr &M, const double *x, double *y, bool accumulate, hipStream_t s);
// out = a x + b y (out may alias x or y)
hipError_t launch_axpby(int64_t n, double a, const double *x, double b, const double *y, double *out,
                        hipStream_t s);
// CG vector steps: x += a p, r -= a w; block partials of r.r and r.z ([2][nblk])
hipError_t launch_cg_update(int64_t n, double a, const double *p, const double *w, double *x, double *r,
                            hipStream_t s);
hipError_t launch_dot2(int64_t n, const double *r, const double *z, double *part, int nblk, hipStream_t s);
// y = C x for a dense row-major [n][n] C
hipError_t launch_dense_matvec(const double *C, int64_t n, const double *x, double *y, hipStream_t s);

}  // namespace sfem
