// Device side of the low-order-refined preconditioner (Section 5.2): upload of the
// multigrid hierarchy built on the host, and the V-cycle driver whose every step is a
// kernel of k_lor.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "lor.h"

namespace sfem {

namespace {

int64_t diag_pos(const HostCsr &A, int64_t row) {
  const int32_t *b = A.col.data() + A.ptr[row], *e = A.col.data() + A.ptr[row + 1];
  const int32_t *it = std::lower_bound(b, e, (int32_t)row);
  return (it != e && *it == (int32_t)row) ? (int64_t)(it - A.col.data()) : -1;
}

template <typename T>
std::string upload(Amg &amg, T **dst, const T *src, int64_t count) {
  *dst = nullptr;
  if (count <= 0) return "";
  void *p = nullptr;
  if (hipMalloc(&p, (size_t)count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return "LOR multigrid: device allocation failed";
  }
  amg.bufs.push_back(p);
  if (src && hipMemcpy(p, src, (size_t)count * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return "LOR multigrid: upload failed";
  *dst = (T *)p;
  return "";
}

std::string upload_csr(Amg &amg, const HostCsr &H, DevCsr &D) {
  D.nrows = H.nrows;
  D.ncols = H.ncols;
  D.nnz = H.nnz();
  if (D.nnz >= (int64_t)INT32_MAX) return "LOR multigrid: matrix too large (nnz >= 2^31)";
  std::vector<int32_t> p32(H.ptr.begin(), H.ptr.end());
  std::string e;
  if (!(e = upload(amg, &D.ptr, p32.data(), (int64_t)p32.size())).empty()) return e;
  if (!(e = upload(amg, &D.col, H.col.data(), D.nnz)).empty()) return e;
  return upload(amg, &D.val, H.val.data(), D.nnz);
}

}  // namespace


std::string amg_setup(const HostCsr &A0, double theta, int64_t coarse_size, int max_levels, int nu,
                      Amg &out) {
  const auto t0 = std::chrono::steady_clock::now();
  amg_free(out);
  out.nu = nu;
  HostAmg H;
  std::string e = amg_build_host(A0, theta, coarse_size, max_levels, H);
  if (!e.empty()) return e;
  const std::vector<HostCsr> &As = H.A, &Ps = H.P;
  const std::vector<double> &rhos = H.rho;
  // upload
  const size_t L = As.size();
  out.lv.assign(L, AmgLevel{});
  for (size_t l = 0; l < L; ++l) {
    AmgLevel &v = out.lv[l];
    out.rows.push_back(As[l].nrows);
    out.nnzs.push_back(As[l].nnz());
    v.omega = 4.0 / (3.0 * rhos[l]);
    if (l + 1 < L) {
      if (!(e = upload_csr(out, As[l], v.A)).empty()) return e;
      std::vector<double> dinv((size_t)As[l].nrows);
      for (int64_t i = 0; i < As[l].nrows; ++i) dinv[i] = 1.0 / As[l].val[diag_pos(As[l], i)];
      if (!(e = upload(out, &v.dinv, dinv.data(), (int64_t)dinv.size())).empty()) return e;
      HostCsr R;
      csr_transpose(Ps[l], R);
      if (!(e = upload_csr(out, Ps[l], v.P)).empty()) return e;
      if (!(e = upload_csr(out, R, v.R)).empty()) return e;
    } else if (l == 0) {
      if (!(e = upload_csr(out, As[l], v.A)).empty()) return e;
    }
    const int64_t n = As[l].nrows;
    if (l > 0) {
      if (!(e = upload<double>(out, &v.b, nullptr, n)).empty()) return e;
      if (!(e = upload<double>(out, &v.x, nullptr, n)).empty()) return e;
    }
    if (!(e = upload<double>(out, &v.t, nullptr, n)).empty()) return e;
  }
  out.ncoarse = As.back().nrows;
  if (!(e = upload(out, &out.coarse, H.coarse.data(), (int64_t)H.coarse.size())).empty()) return e;
  out.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return "";
}

void amg_free(Amg &amg) {
  for (void *p : amg.bufs) (void)hipFree(p);
  amg.bufs.clear();
  amg.lv.clear();
  amg.rows.clear();
  amg.nnzs.clear();
  amg.coarse = nullptr;
  amg.ncoarse = 0;
}

namespace {

hipError_t vcycle_level(const Amg &amg, size_t l, const double *b, double *x, hipStream_t s) {
  const AmgLevel &v = amg.lv[l];
  if (l + 1 == amg.lv.size()) return launch_dense_matvec(amg.coarse, amg.ncoarse, b, x, s);
  hipError_t e;
  // pre-smoothing from x = 0: the first sweep is omega D^-1 b
  if ((e = launch_csr_jacobi(v.A, v.dinv, v.omega, b, nullptr, x, s)) != hipSuccess) return e;
  double *cur = x, *oth = v.t;
  for (int it = 1; it < amg.nu; ++it) {
    if ((e = launch_csr_jacobi(v.A, v.dinv, v.omega, b, cur, oth, s)) != hipSuccess) return e;
    std::swap(cur, oth);
  }
  // residual, restriction, coarse correction, prolongation
  if ((e = launch_csr_residual(v.A, b, cur, oth, s)) != hipSuccess) return e;
  const AmgLevel &c = amg.lv[l + 1];
  if ((e = launch_csr_spmv(v.R, oth, c.b, false, s)) != hipSuccess) return e;
  if ((e = vcycle_level(amg, l + 1, c.b, c.x, s)) != hipSuccess) return e;
  if ((e = launch_csr_spmv(v.P, c.x, cur, true, s)) != hipSuccess) return e;
  for (int it = 0; it < amg.nu; ++it) {
    if ((e = launch_csr_jacobi(v.A, v.dinv, v.omega, b, cur, oth, s)) != hipSuccess) return e;
    std::swap(cur, oth);
  }
  if (cur != x)
    e = hipMemcpyAsync(x, cur, (size_t)v.A.nrows * sizeof(double), hipMemcpyDeviceToDevice, s);
  return e;
}

}  // namespace

hipError_t amg_vcycle(const Amg &amg, const double *b, double *x, hipStream_t s) {
  if (amg.lv.empty()) return hipErrorInvalidValue;
  return vcycle_level(amg, 0, b, x, s);
}

hipError_t amg_apply_fine(const Amg &amg, const double *x, double *y, hipStream_t s) {
  if (amg.lv.empty()) return hipErrorInvalidValue;
  return launch_csr_spmv(amg.lv[0].A, x, y, false, s);
}

}  // namespace sfem
