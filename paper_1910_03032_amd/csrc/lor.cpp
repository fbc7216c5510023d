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

// Sliced ELL copy of H (see DevSell), built on the host by sell_build.
std::string upload_sell(Amg &amg, const HostCsr &H, DevSell &D, bool patterns) {
  HostSell S;
  std::string e = sell_build(H, patterns, S);
  if (!e.empty()) return e;
  D.nrows = H.nrows;
  D.ncols = H.ncols;
  D.nnz = H.nnz();
  D.padded = (int64_t)S.val.size();
  D.pattern_slices = S.pattern_slices;
  if (!(e = upload(amg, &D.off, S.off.data(), (int64_t)S.off.size())).empty()) return e;
  if (!(e = upload(amg, &D.pinfo, S.pinfo.data(), (int64_t)S.pinfo.size())).empty()) return e;
  if (!(e = upload(amg, &D.col, S.col.data(), (int64_t)S.col.size())).empty()) return e;
  if (!(e = upload(amg, &D.pat, S.pat.data(), (int64_t)S.pat.size())).empty()) return e;
  return upload(amg, &D.val, S.val.data(), D.padded);
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

// The form of H on the device: sliced ELL for at least 16384 rows of at most 48 entries
// on average, padded by at most half (the level operators and prolongators of the fine
// levels; column-offset patterns for the square operators), CSR otherwise (the
// restrictions' long rows, the small coarse levels).
std::string upload_mat(Amg &amg, const HostCsr &H, DevMat &D) {
  int64_t padded = 0;
  const int64_t nsl = (H.nrows + kSellRows - 1) / kSellRows;
  for (int64_t s = 0; s < nsl; ++s) {
    int64_t len = 0;
    for (int64_t r = s * kSellRows; r < std::min(H.nrows, (s + 1) * kSellRows); ++r)
      len = std::max(len, H.ptr[r + 1] - H.ptr[r]);
    padded += len * kSellRows;
  }
  D.sell = H.nrows >= 16384 && H.nnz() <= 48 * H.nrows && 2 * padded <= 3 * H.nnz();
  return D.sell ? upload_sell(amg, H, D.S, H.nrows == H.ncols) : upload_csr(amg, H, D.C);
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
      if (!(e = upload_mat(out, As[l], v.A)).empty()) return e;
      std::vector<double> dinv((size_t)As[l].nrows);
      for (int64_t i = 0; i < As[l].nrows; ++i) dinv[i] = 1.0 / As[l].val[diag_pos(As[l], i)];
      if (!(e = upload(out, &v.d.dinv, dinv.data(), (int64_t)dinv.size())).empty()) return e;
      HostCsr R;
      csr_transpose(Ps[l], R);
      if (!(e = upload_mat(out, Ps[l], v.P)).empty()) return e;
      if (!(e = upload_mat(out, R, v.R)).empty()) return e;
    } else if (l == 0) {
      if (!(e = upload_mat(out, As[l], v.A)).empty()) return e;
    }
    const int64_t n = As[l].nrows;
    if (l > 0) {
      if (!(e = upload<double>(out, &v.d.b, nullptr, n)).empty()) return e;
      if (!(e = upload<double>(out, &v.d.x, nullptr, n)).empty()) return e;
    }
    if (!(e = upload<double>(out, &v.d.t, nullptr, n)).empty()) return e;
  }
  for (const AmgLevel &v : out.lv)
    out.sliced.push_back((v.A.sell ? 1 : 0) | (v.P.sell ? 2 : 0) | (v.R.sell ? 4 : 0) |
                         (v.A.sell && v.A.S.pattern_slices > 0 ? 8 : 0));
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
  amg.sliced.clear();
  amg.coarse = nullptr;
  amg.coarse32 = nullptr;
  amg.has32 = false;
  amg.ncoarse = 0;
}

namespace {

// FP32 copy of count device values src (allocated into amg.bufs).
std::string to_f32(Amg &amg, float **dst, const double *src, int64_t count, hipStream_t s) {
  *dst = nullptr;
  if (count <= 0 || !src) return "";
  std::string e = upload<float>(amg, dst, nullptr, count);
  if (!e.empty()) return e;
  if (launch_convert<double, float>(src, *dst, count, s) != hipSuccess) {
    (void)hipGetLastError();
    return "LOR multigrid: FP32 conversion launch failed";
  }
  return "";
}

}  // namespace

std::string amg_make_f32(Amg &amg, hipStream_t s) {
  if (amg.has32) return "";
  if (amg.lv.empty()) return "LOR multigrid: no hierarchy";
  std::string e;
  const size_t L = amg.lv.size();
  for (size_t l = 0; l < L; ++l) {
    AmgLevel &v = amg.lv[l];
    const int64_t n = amg.rows[l];
    if (l + 1 < L) {
      for (DevMat *M : {&v.A, &v.P, &v.R}) {
        e = M->sell ? to_f32(amg, &M->S.val32, M->S.val, M->S.padded, s)
                    : to_f32(amg, &M->C.val32, M->C.val, M->C.nnz, s);
        if (!e.empty()) return e;
      }
      if (!(e = to_f32(amg, &v.f.dinv, v.d.dinv, n, s)).empty()) return e;
    }
    if (l > 0) {
      if (!(e = upload<float>(amg, &v.f.b, nullptr, n)).empty()) return e;
      if (!(e = upload<float>(amg, &v.f.x, nullptr, n)).empty()) return e;
    }
    if (!(e = upload<float>(amg, &v.f.t, nullptr, n)).empty()) return e;
  }
  if (!(e = to_f32(amg, &amg.coarse32, amg.coarse, amg.ncoarse * amg.ncoarse, s)).empty()) return e;
  amg.has32 = true;
  return "";
}

namespace {

template <typename T>
hipError_t vcycle_level(const Amg &amg, size_t l, const T *b, T *x, hipStream_t s) {
  const AmgLevel &v = amg.lv[l];
  if (l + 1 == amg.lv.size()) {
    const T *C;
    if constexpr (sizeof(T) == 8) C = amg.coarse;
    else C = amg.coarse32;
    return launch_dense_matvec<T>(C, amg.ncoarse, b, x, s);
  }
  const LevelVecs<T> &w = v.vecs<T>();
  const T omega = (T)v.omega;
  hipError_t e;
  // pre-smoothing from x = 0: the first sweep is omega D^-1 b.  It goes to the work
  // vector, so that after the 2 nu - 1 alternations between the two vectors the last
  // post-smoothing sweep lands in x (x serves as scratch until then).
  if ((e = launch_mat_jacobi<T>(v.A, w.dinv, omega, b, nullptr, w.t, s)) != hipSuccess) return e;
  T *cur = w.t, *oth = x;
  for (int it = 1; it < amg.nu; ++it) {
    if ((e = launch_mat_jacobi<T>(v.A, w.dinv, omega, b, cur, oth, s)) != hipSuccess) return e;
    std::swap(cur, oth);
  }
  // residual, restriction, coarse correction, prolongation
  if ((e = launch_mat_residual<T>(v.A, b, cur, oth, s)) != hipSuccess) return e;
  const LevelVecs<T> &c = amg.lv[l + 1].vecs<T>();
  if ((e = launch_mat_spmv<T>(v.R, oth, c.b, false, s)) != hipSuccess) return e;
  if ((e = vcycle_level<T>(amg, l + 1, c.b, c.x, s)) != hipSuccess) return e;
  if ((e = launch_mat_spmv<T>(v.P, c.x, cur, true, s)) != hipSuccess) return e;
  for (int it = 0; it < amg.nu; ++it) {
    if ((e = launch_mat_jacobi<T>(v.A, w.dinv, omega, b, cur, oth, s)) != hipSuccess) return e;
    std::swap(cur, oth);
  }
  if (cur != x) e = hipMemcpyAsync(x, cur, (size_t)v.A.nrows() * sizeof(T), hipMemcpyDeviceToDevice, s);
  return e;
}

}  // namespace

template <typename T>
hipError_t amg_vcycle(const Amg &amg, const T *b, T *x, hipStream_t s) {
  if (amg.lv.empty()) return hipErrorInvalidValue;
  if (sizeof(T) == 4 && !amg.has32) return hipErrorInvalidValue;
  return vcycle_level<T>(amg, 0, b, x, s);
}
template hipError_t amg_vcycle<double>(const Amg &, const double *, double *, hipStream_t);
template hipError_t amg_vcycle<float>(const Amg &, const float *, float *, hipStream_t);

hipError_t amg_apply_fine(const Amg &amg, const double *x, double *y, hipStream_t s) {
  if (amg.lv.empty()) return hipErrorInvalidValue;
  return launch_mat_spmv<double>(amg.lv[0].A, x, y, false, s);
}

}  // namespace sfem
