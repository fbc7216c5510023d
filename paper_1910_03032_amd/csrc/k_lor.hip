// Kernels of the LOR multigrid V-cycle: CSR products with a group of LPR lanes per row (the
// lanes read consecutive entries of the row, so a wave's loads of values and column
// indices are contiguous; a fixed shuffle tree sums the group, so results are
// reproducible), with the residual and the damped-Jacobi update fused into the product,
// and the dense coarsest-level product.  LPR is picked from the average row length.
#include <hip/hip_runtime.h>

#include "lor.h"

namespace sfem {

namespace {

constexpr int kRowBlock = 256;

enum CsrMode { kSpmv = 0, kSpmvAdd = 1, kResidual = 2, kJacobi = 3 };

// y_i = (A x)_i combined per MODE:
//   kSpmv      out = A x            kSpmvAdd  out += A x
//   kResidual  out = b - A x        kJacobi   out = x + omega dinv (b - A x)
template <int LPR, int MODE>
__global__ void __launch_bounds__(kRowBlock)
csr_kernel(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
           const double *__restrict__ val, const double *__restrict__ x, const double *__restrict__ b,
           const double *__restrict__ dinv, double omega, double *__restrict__ out, int64_t n) {
  const int lane = threadIdx.x % LPR;
  const int64_t groups = (int64_t)gridDim.x * (kRowBlock / LPR);
  for (int64_t i = ((int64_t)blockIdx.x * kRowBlock + threadIdx.x) / LPR; i < n; i += groups) {
    double s = 0.0;
    const int32_t k1 = ptr[i + 1];
    for (int32_t k = ptr[i] + lane; k < k1; k += LPR) s += val[k] * x[col[k]];
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) s += __shfl_down(s, off, LPR);
    if (lane == 0) {
      if constexpr (MODE == kSpmv) out[i] = s;
      else if constexpr (MODE == kSpmvAdd) out[i] += s;
      else if constexpr (MODE == kResidual) out[i] = b[i] - s;
      else out[i] = x[i] + omega * dinv[i] * (b[i] - s);
    }
  }
}

// out = omega dinv b (a Jacobi sweep from x = 0)
__global__ void __launch_bounds__(kRowBlock)
scaled_copy_kernel(const double *__restrict__ dinv, double omega, const double *__restrict__ b,
                   double *__restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRowBlock)
    out[i] = omega * dinv[i] * b[i];
}

__global__ void __launch_bounds__(kRowBlock)
axpby_kernel(int64_t n, double a, const double *x, double b, const double *y, double *out) {
  for (int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRowBlock)
    out[i] = a * x[i] + b * y[i];
}

// x += a p, r -= a w
__global__ void __launch_bounds__(kRowBlock)
cg_update_kernel(int64_t n, double a, const double *__restrict__ p, const double *__restrict__ w,
                 double *__restrict__ x, double *__restrict__ r) {
  for (int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRowBlock) {
    x[i] += a * p[i];
    r[i] -= a * w[i];
  }
}

// block partials of r.r (part[blk]) and r.z (part[nblk + blk]); fixed order within a block
__global__ void __launch_bounds__(kRowBlock)
dot2_kernel(int64_t n, const double *__restrict__ r, const double *__restrict__ z,
            double *__restrict__ part, int nblk) {
  __shared__ double sh[2][kRowBlock];
  double rr = 0.0, rz = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; i < n; i += (int64_t)nblk * kRowBlock) {
    const double ri = r[i];
    rr += ri * ri;
    rz += ri * z[i];
  }
  sh[0][threadIdx.x] = rr;
  sh[1][threadIdx.x] = rz;
  __syncthreads();
  for (int off = kRowBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + off];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sh[0][0];
    part[nblk + blockIdx.x] = sh[1][0];
  }
}

// y = C x, one wave per row of the dense [n][n] C
__global__ void __launch_bounds__(kRowBlock)
dense_matvec_kernel(const double *__restrict__ C, int64_t n, const double *__restrict__ x,
                    double *__restrict__ y) {
  const int lane = threadIdx.x % 64;
  const int64_t waves = (int64_t)gridDim.x * (kRowBlock / 64);
  for (int64_t i = ((int64_t)blockIdx.x * kRowBlock + threadIdx.x) / 64; i < n; i += waves) {
    double s = 0.0;
    for (int64_t j = lane; j < n; j += 64) s += C[i * n + j] * x[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) y[i] = s;
  }
}

unsigned grid_for_rows(int64_t n, int lpr) {
  int64_t b = (n * lpr + kRowBlock - 1) / kRowBlock;
  if (b < 1) b = 1;
  if (b > 65535) b = 65535;
  return (unsigned)b;
}

template <int MODE>
hipError_t launch_csr(const DevCsr &A, const double *x, const double *b, const double *dinv,
                      double omega, double *out, hipStream_t s) {
  if (A.nrows <= 0) return hipSuccess;
  const double avg = A.nrows > 0 ? (double)A.nnz / (double)A.nrows : 0.0;
#define SFEM_CSR(L)                                                                          \
  hipLaunchKernelGGL((csr_kernel<L, MODE>), dim3(grid_for_rows(A.nrows, L)), dim3(kRowBlock), 0, s, \
                     A.ptr, A.col, A.val, x, b, dinv, omega, out, A.nrows)
  if (avg <= 6.0) SFEM_CSR(4);
  else if (avg <= 16.0) SFEM_CSR(8);
  else if (avg <= 40.0) SFEM_CSR(16);
  else if (avg <= 128.0) SFEM_CSR(32);
  else SFEM_CSR(64);
#undef SFEM_CSR
  return hipGetLastError();
}

}  // namespace

hipError_t launch_csr_jacobi(const DevCsr &A, const double *dinv, double omega, const double *b,
                             const double *x_in, double *x_out, hipStream_t s) {
  if (A.nrows <= 0) return hipSuccess;
  if (!x_in) {
    hipLaunchKernelGGL(scaled_copy_kernel, dim3(grid_for_rows(A.nrows, 1)), dim3(kRowBlock), 0, s, dinv,
                       omega, b, x_out, A.nrows);
    return hipGetLastError();
  }
  return launch_csr<kJacobi>(A, x_in, b, dinv, omega, x_out, s);
}

hipError_t launch_csr_residual(const DevCsr &A, const double *b, const double *x, double *r,
                               hipStream_t s) {
  return launch_csr<kResidual>(A, x, b, nullptr, 0.0, r, s);
}

hipError_t launch_csr_spmv(const DevCsr &M, const double *x, double *y, bool accumulate, hipStream_t s) {
  return accumulate ? launch_csr<kSpmvAdd>(M, x, nullptr, nullptr, 0.0, y, s)
                    : launch_csr<kSpmv>(M, x, nullptr, nullptr, 0.0, y, s);
}

hipError_t launch_axpby(int64_t n, double a, const double *x, double b, const double *y, double *out,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for_rows(n, 1)), dim3(kRowBlock), 0, s, n, a, x, b, y, out);
  return hipGetLastError();
}

hipError_t launch_cg_update(int64_t n, double a, const double *p, const double *w, double *x, double *r,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(cg_update_kernel, dim3(grid_for_rows(n, 1)), dim3(kRowBlock), 0, s, n, a, p, w, x, r);
  return hipGetLastError();
}

hipError_t launch_dot2(int64_t n, const double *r, const double *z, double *part, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(dot2_kernel, dim3(nblk), dim3(kRowBlock), 0, s, n, r, z, part, nblk);
  return hipGetLastError();
}

hipError_t launch_dense_matvec(const double *C, int64_t n, const double *x, double *y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dense_matvec_kernel, dim3(grid_for_rows(n, 64)), dim3(kRowBlock), 0, s, C, n, x, y);
  return hipGetLastError();
}

}  // namespace sfem
