// Kernels of the LOR multigrid V-cycle: products with the level operators and the
// prolongators in sliced ELL form (a thread per row; explicit columns or a column-offset
// pattern per slice), with the residual and the damped-Jacobi update fused in; products
// with the restrictions (long rows) in CSR form with a group of LPR lanes per row (the
// lanes read consecutive entries of the row, so a wave's loads of values and column
// indices are contiguous; a fixed shuffle tree sums the group, so results are
// reproducible; LPR is picked from the average row length); the dense coarsest-level
// product.  The V-cycle kernels exist in FP64 and in FP32 (values and vectors of one type
// T; the FP32 V-cycle reads half the bytes and serves as a preconditioner inside FP64 CG).
#include <hip/hip_runtime.h>

#include "lor.h"

namespace sfem {

namespace {

constexpr int kRowBlock = 256;
static_assert(kRowBlock % kSellRows == 0 && kSellRows == 64, "a wave per slice");

enum CsrMode { kSpmv = 0, kSpmvAdd = 1, kResidual = 2, kJacobi = 3 };

// Block index remapped so that each of the 8 XCDs (workgroups are dispatched to them in
// turn) takes one contiguous range of the grid's blocks, i.e. of the rows: the rows of a
// range gather their x values mostly from one region, which then stays in that XCD's L2
// instead of being fetched from HBM by several XCDs.  A bijection of [0, gridDim.x).
// Used by the CSR products (the restriction's gathers: 1.6x -> 1.0x the algorithmic
// HBM bytes); the sliced ELL products keep the dispatch order, which is faster for them
// although it fetches about 10 % more.
__device__ __forceinline__ int64_t row_block() {
  const unsigned nblk = gridDim.x, b = blockIdx.x;
  const unsigned xcd = b & 7u, k = b >> 3;
  const unsigned q8 = nblk >> 3, r8 = nblk & 7u;
  return (int64_t)(xcd * q8 + (xcd < r8 ? xcd : r8) + k);
}

// y_i = (A x)_i combined per MODE:
//   kSpmv      out = A x            kSpmvAdd  out += A x
//   kResidual  out = b - A x        kJacobi   out = x + omega dinv (b - A x)
template <int LPR, int MODE, typename T>
__global__ void __launch_bounds__(kRowBlock)
csr_kernel(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
           const T *__restrict__ val, const T *__restrict__ x, const T *__restrict__ b,
           const T *__restrict__ dinv, T omega, T *__restrict__ out, int64_t n) {
  const int lane = threadIdx.x % LPR;
  const int64_t groups = (int64_t)gridDim.x * (kRowBlock / LPR);
  for (int64_t i = (row_block() * kRowBlock + threadIdx.x) / LPR; i < n; i += groups) {
    T s = T(0);
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

// The same products with the operator in sliced ELL form (DevSell): one thread per row,
// the slice's values read entry-major, so a wave's loads of values (and explicit column
// indices) are contiguous; in a slice with a column-offset pattern the wave reads the
// pattern through scalar loads and forms the columns itself.  The row's terms are summed
// in column order.
template <int MODE, typename T>
__global__ void __launch_bounds__(kRowBlock)
sell_kernel(const int32_t *__restrict__ off, const int32_t *__restrict__ pinfo,
            const int32_t *__restrict__ col, const int32_t *__restrict__ pat, const T *__restrict__ val,
            const T *__restrict__ x, const T *__restrict__ b, const T *__restrict__ dinv, T omega,
            T *__restrict__ out, int64_t n, int64_t ncols) {
  const int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
  if (i >= n) return;
  // the wave's 64 rows form one slice (kRowBlock is a multiple of kSellRows)
  const int sl = __builtin_amdgcn_readfirstlane((int)(i / kSellRows));
  const int lane = (int)(i - (int64_t)sl * kSellRows);
  const int32_t k0 = off[sl];
  const int len = (off[sl + 1] - k0) / kSellRows;
  const int32_t pi = pinfo[sl];
  const T *v = val + k0 + lane;
  T s = T(0);
  if (pi >= 0) {
    const int32_t *c = col + pi + lane;
#pragma unroll 4
    for (int k = 0; k < len; ++k) s += v[(int64_t)k * kSellRows] * x[c[(int64_t)k * kSellRows]];
  } else {
    const int32_t *po = pat + (-1 - pi);
#pragma unroll 4
    for (int k = 0; k < len; ++k) {
      int64_t c = i + po[k];
      c = c < 0 ? 0 : (c >= ncols ? ncols - 1 : c);  // absent entries (value 0) of edge rows
      s += v[(int64_t)k * kSellRows] * x[c];
    }
  }
  if constexpr (MODE == kSpmv) out[i] = s;
  else if constexpr (MODE == kSpmvAdd) out[i] += s;
  else if constexpr (MODE == kResidual) out[i] = b[i] - s;
  else out[i] = x[i] + omega * dinv[i] * (b[i] - s);
}

// out = omega dinv b (a Jacobi sweep from x = 0)
template <typename T>
__global__ void __launch_bounds__(kRowBlock)
scaled_copy_kernel(const T *__restrict__ dinv, T omega, const T *__restrict__ b, T *__restrict__ out,
                   int64_t n) {
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

// y = C x, one wave per row of the dense [n][n] C
template <typename T>
__global__ void __launch_bounds__(kRowBlock)
dense_matvec_kernel(const T *__restrict__ C, int64_t n, const T *__restrict__ x, T *__restrict__ y) {
  const int lane = threadIdx.x % 64;
  const int64_t waves = (int64_t)gridDim.x * (kRowBlock / 64);
  for (int64_t i = ((int64_t)blockIdx.x * kRowBlock + threadIdx.x) / 64; i < n; i += waves) {
    T s = T(0);
    for (int64_t j = lane; j < n; j += 64) s += C[i * n + j] * x[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) y[i] = s;
  }
}

// out = (TO) in, elementwise
template <typename TI, typename TO>
__global__ void __launch_bounds__(kRowBlock)
convert_kernel(const TI *__restrict__ in, TO *__restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRowBlock)
    out[i] = (TO)in[i];
}

unsigned grid_for_rows(int64_t n, int lpr) {
  int64_t b = (n * lpr + kRowBlock - 1) / kRowBlock;
  if (b < 1) b = 1;
  if (b > 65535) b = 65535;
  return (unsigned)b;
}

template <int MODE, typename T>
hipError_t launch_csr(const DevCsr &A, const T *x, const T *b, const T *dinv, T omega, T *out,
                      hipStream_t s) {
  if (A.nrows <= 0) return hipSuccess;
  const T *val = csr_vals<T>(A);
  if (!val) return hipErrorInvalidValue;
  const double avg = A.nrows > 0 ? (double)A.nnz / (double)A.nrows : 0.0;
#define SFEM_CSR(L)                                                                          \
  hipLaunchKernelGGL((csr_kernel<L, MODE, T>), dim3(grid_for_rows(A.nrows, L)), dim3(kRowBlock), 0, s, \
                     A.ptr, A.col, val, x, b, dinv, omega, out, A.nrows)
  if (avg <= 6.0) SFEM_CSR(4);
  else if (avg <= 16.0) SFEM_CSR(8);
  else if (avg <= 40.0) SFEM_CSR(16);
  else if (avg <= 128.0) SFEM_CSR(32);
  else SFEM_CSR(64);
#undef SFEM_CSR
  return hipGetLastError();
}

template <int MODE, typename T>
hipError_t launch_sell(const DevSell &A, const T *x, const T *b, const T *dinv, T omega, T *out,
                       hipStream_t s) {
  if (A.nrows <= 0) return hipSuccess;
  const T *val = sell_vals<T>(A);
  if (!val) return hipErrorInvalidValue;
  const int64_t nblk = (A.nrows + kRowBlock - 1) / kRowBlock;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((sell_kernel<MODE, T>), dim3((unsigned)nblk), dim3(kRowBlock), 0, s, A.off, A.pinfo,
                     A.col, A.pat, val, x, b, dinv, omega, out, A.nrows, A.ncols);
  return hipGetLastError();
}

template <int MODE, typename T>
hipError_t launch_mat(const DevMat &A, const T *x, const T *b, const T *dinv, T omega, T *out,
                      hipStream_t s) {
  return A.sell ? launch_sell<MODE, T>(A.S, x, b, dinv, omega, out, s)
                : launch_csr<MODE, T>(A.C, x, b, dinv, omega, out, s);
}

}  // namespace

template <typename T>
hipError_t launch_mat_jacobi(const DevMat &A, const T *dinv, T omega, const T *b, const T *x_in,
                             T *x_out, hipStream_t s) {
  const int64_t n = A.nrows();
  if (n <= 0) return hipSuccess;
  if (!x_in) {
    hipLaunchKernelGGL((scaled_copy_kernel<T>), dim3(grid_for_rows(n, 1)), dim3(kRowBlock), 0, s, dinv,
                       omega, b, x_out, n);
    return hipGetLastError();
  }
  return launch_mat<kJacobi, T>(A, x_in, b, dinv, omega, x_out, s);
}

template <typename T>
hipError_t launch_mat_residual(const DevMat &A, const T *b, const T *x, T *r, hipStream_t s) {
  return launch_mat<kResidual, T>(A, x, b, nullptr, T(0), r, s);
}

template <typename T>
hipError_t launch_mat_spmv(const DevMat &M, const T *x, T *y, bool accumulate, hipStream_t s) {
  return accumulate ? launch_mat<kSpmvAdd, T>(M, x, nullptr, nullptr, T(0), y, s)
                    : launch_mat<kSpmv, T>(M, x, nullptr, nullptr, T(0), y, s);
}

template <typename T>
hipError_t launch_dense_matvec(const T *C, int64_t n, const T *x, T *y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((dense_matvec_kernel<T>), dim3(grid_for_rows(n, 64)), dim3(kRowBlock), 0, s, C, n, x,
                     y);
  return hipGetLastError();
}

template <typename TI, typename TO>
hipError_t launch_convert(const TI *in, TO *out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((convert_kernel<TI, TO>), dim3(grid_for_rows(n, 1)), dim3(kRowBlock), 0, s, in, out,
                     n);
  return hipGetLastError();
}

#define SFEM_LOR_INST(T)                                                                              \
  template hipError_t launch_mat_jacobi<T>(const DevMat &, const T *, T, const T *, const T *, T *,  \
                                           hipStream_t);                                            \
  template hipError_t launch_mat_residual<T>(const DevMat &, const T *, const T *, T *, hipStream_t); \
  template hipError_t launch_mat_spmv<T>(const DevMat &, const T *, T *, bool, hipStream_t);          \
  template hipError_t launch_dense_matvec<T>(const T *, int64_t, const T *, T *, hipStream_t);
SFEM_LOR_INST(double)
SFEM_LOR_INST(float)
#undef SFEM_LOR_INST
template hipError_t launch_convert<double, float>(const double *, float *, int64_t, hipStream_t);
template hipError_t launch_convert<float, double>(const float *, double *, int64_t, hipStream_t);

hipError_t launch_axpby(int64_t n, double a, const double *x, double b, const double *y, double *out,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for_rows(n, 1)), dim3(kRowBlock), 0, s, n, a, x, b, y, out);
  return hipGetLastError();
}

}  // namespace sfem
