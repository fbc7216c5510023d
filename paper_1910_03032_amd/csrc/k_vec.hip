// Vector kernels of the Jacobi-preconditioned CG (Section 5, Section 5.3) and of the
// FP64 iterative refinement around an FP32 inner CG.
//
// All dot products accumulate in float64, also for float32 vectors.  Reductions are
// two-level and in a fixed order (per-block partial sums, then one block per batch
// member), so every result is bitwise reproducible for a given size.  The CG scalars
// (rho, alpha, beta, ...) stay on the device; the host only reads them at its
// convergence checks.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace sfem {
namespace {

constexpr int VB = 256;

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double sh[NV][VB];
#pragma unroll
  for (int k = 0; k < NV; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
#pragma unroll
  for (int s = VB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int k = 0; k < NV; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = sh[k][0];
}

template <int NV>
__device__ __forceinline__ void write_part(double (&v)[NV], double *part, int nblk) {
  block_sum<NV>(v);
  if (threadIdx.x == 0) {
    const int m = blockIdx.y;
#pragma unroll
    for (int k = 0; k < NV; ++k) part[((int64_t)m * NV + k) * nblk + blockIdx.x] = v[k];
  }
}

// Sum of the nblk partials of quantity k (NV quantities per member, part[(m NV + k) nblk
// + i]) of member m by a block of NT threads: each thread sums a fixed strided subset
// (4 independent loads per step), then a wave64 butterfly and the waves in order.  The
// order depends only on nblk and NT.  Result broadcast to all threads.
template <int NV, int NT>
__device__ __forceinline__ void reduce_parts_m(const double *part, int nblk, int m, double (&v)[NV]) {
  __shared__ double sh[NV][NT / 64];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double *pk = part + ((int64_t)m * NV + k) * nblk;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * NT < nblk; i += 4 * NT) {
      s0 += pk[i];
      s1 += pk[i + NT];
      s2 += pk[i + 2 * NT];
      s3 += pk[i + 3 * NT];
    }
    for (; i < nblk; i += NT) s0 += pk[i];
    double s = (s0 + s1) + (s2 + s3);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += sh[k][w];
    v[k] = s;
  }
}

// One block of RB threads per member (blockIdx.x = member).
constexpr int RB = 1024;
template <int NV>
__device__ __forceinline__ void reduce_parts(const double *part, int nblk, double (&v)[NV]) {
  reduce_parts_m<NV, RB>(part, nblk, blockIdx.x, v);
}

// CG step length from p.Ap (or the failure state).
__device__ __forceinline__ void set_alpha(PcgScalars &s, double pw) {
  s.pw = pw;
  s.alpha = 0.0;
  if (s.active) {
    if (!isfinite(pw)) {
      s.status = SFEM_E_NAN;
      s.active = 0;
    } else if (!(pw > 0.0)) {
      s.status = SFEM_E_BREAKDOWN;
      s.active = 0;
    } else {
      s.alpha = s.rho / pw;
    }
  }
}

// New direction coefficient from r.z and r.r, and the stopping test.
__device__ __forceinline__ void set_beta(PcgScalars &s, double rz, double rr) {
  s.beta = 0.0;
  if (s.active) {
    s.iters += 1;
    if (!isfinite(rz) || !isfinite(rr)) {
      s.status = SFEM_E_NAN;
      s.active = 0;
    } else {
      s.beta = rz / s.rho;
      s.rho = rz;
      s.rr = rr;
      if (rr <= s.tol2) s.active = 0;
    }
  }
}

// r = b - w (w may be null: r = b); x = 0 if xzero; p = dinv r;
// partials: r.p (rho), r.r, b.b, sum p, sum r
template <typename T>
__global__ void start_kernel(const T *__restrict__ b, const T *__restrict__ w, T *__restrict__ x,
                             T *__restrict__ r, const T *__restrict__ dinv, int64_t dinv_mstride,
                             T *__restrict__ p, double *__restrict__ part, int nblk, int64_t n) {
  const int64_t off = (int64_t)blockIdx.y * n;
  const T *dm = dinv + (int64_t)blockIdx.y * dinv_mstride;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)nblk * VB) {
    const T bi = b[off + i];
    const T ri = w ? (T)(bi - w[off + i]) : bi;
    const T pi = dm[i] * ri;
    r[off + i] = ri;
    p[off + i] = pi;
    if (x) x[off + i] = T(0);
    v[0] += (double)ri * (double)pi;
    v[1] += (double)ri * (double)ri;
    v[2] += (double)bi * (double)bi;
    v[3] += (double)pi;
    v[4] += (double)ri;
  }
  write_part<5>(v, part, nblk);
}

template <typename T>
__global__ void dot_kernel(const T *__restrict__ a, const T *__restrict__ c, int64_t c_mstride,
                           double *__restrict__ part, int nblk, int64_t n) {
  const int64_t off = (int64_t)blockIdx.y * n;
  const T *cm = c ? c + (int64_t)blockIdx.y * c_mstride : nullptr;
  double v[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)nblk * VB)
    v[0] += (double)a[off + i] * (cm ? (double)cm[i] : 1.0);
  write_part<1>(v, part, nblk);
}

// The step length of the current iteration from the scalars sc (rho, active) and the
// apply's partial sums of p.Ap (member m: dpart[m * dmstride + i], i < dcount), summed
// in a fixed order by every block that needs it -- the same value in each.
__device__ __forceinline__ double step_alpha(const PcgScalars &s, double pw) {
  return (s.active && isfinite(pw) && pw > 0.0) ? s.rho / pw : 0.0;
}

// x += alpha p; r -= alpha w; partials: r.z, r.r, sum z, sum r (z = dinv r).  alpha is
// formed by every block from the apply's partials.
template <typename T>
__global__ void update_kernel(T *__restrict__ x, const T *__restrict__ p, T *__restrict__ r,
                              const T *__restrict__ w, const T *__restrict__ dinv,
                              int64_t dinv_mstride, const PcgScalars *__restrict__ sc,
                              const double *__restrict__ dpart, int64_t dmstride, int dcount,
                              double *__restrict__ part, int nblk, int64_t n) {
  const int m = blockIdx.y;
  const int64_t off = (int64_t)m * n;
  const T *dm = dinv + (int64_t)m * dinv_mstride;
  // the operands of the first entry are requested before the partial sums are read
  const int64_t i0 = (int64_t)blockIdx.x * VB + threadIdx.x, stride = (int64_t)nblk * VB;
  const bool has0 = i0 < n;
  const int64_t j0 = has0 ? i0 : 0;
  const T x0 = x[off + j0], p0 = p[off + j0], r0 = r[off + j0], w0 = w[off + j0], d0 = dm[j0];
  double pw[1];
  reduce_parts_m<1, VB>(dpart + (int64_t)m * dmstride, dcount, 0, pw);
  const T alpha = (T)step_alpha(sc[m], pw[0]);
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  auto step = [&](int64_t i, T xi, T pi, T ri, T wi, T di) {
    x[off + i] = xi + alpha * pi;
    ri = ri - alpha * wi;
    r[off + i] = ri;
    const T zi = di * ri;
    v[0] += (double)ri * (double)zi;
    v[1] += (double)ri * (double)ri;
    v[2] += (double)zi;
    v[3] += (double)ri;
  };
  if (has0) step(i0, x0, p0, r0, w0, d0);
  for (int64_t i = i0 + stride; i < n; i += stride)
    step(i, x[off + i], p[off + i], r[off + i], w[off + i], dm[i]);
  write_part<4>(v, part, nblk);
}

// New direction p = (dinv r - zshift) + beta p, with beta (and the null-space shift)
// formed by every block from the update's partials.  Block 0 of each member also
// writes the next iteration's scalars to sc_next (the scalars are double-buffered, so
// no block reads a value another block of the same launch writes).
template <typename T>
__global__ void newdir_kernel(const T *__restrict__ r, const T *__restrict__ dinv,
                              int64_t dinv_mstride, T *__restrict__ p,
                              const PcgScalars *__restrict__ sc, PcgScalars *__restrict__ sc_next,
                              const double *__restrict__ dpart, int64_t dmstride, int dcount,
                              const double *__restrict__ upart, int unblk, int nullspace,
                              int64_t n) {
  const int m = blockIdx.y;
  const int64_t off = (int64_t)m * n;
  const T *dm = dinv + (int64_t)m * dinv_mstride;
  // the operands of the first entry are requested before the partial sums are read
  const int64_t i0 = (int64_t)blockIdx.x * VB + threadIdx.x, stride = (int64_t)gridDim.x * VB;
  const bool has0 = i0 < n;
  const int64_t j0 = has0 ? i0 : 0;
  const T r0 = r[off + j0], d0 = dm[j0], p0 = p[off + j0];
  double pw[1], u[4];
  reduce_parts_m<1, VB>(dpart + (int64_t)m * dmstride, dcount, 0, pw);
  reduce_parts_m<4, VB>(upart, unblk, m, u);
  PcgScalars s = sc[m];
  set_alpha(s, pw[0]);
  const double zs = nullspace ? u[2] / (double)n : 0.0;
  if (s.active) s.zshift = zs;
  set_beta(s, u[0] - zs * u[3], u[1]);
  if (blockIdx.x == 0 && threadIdx.x == 0) sc_next[m] = s;
  const T beta = (T)s.beta;
  const T zst = (T)s.zshift;
  if (has0) p[off + i0] = (d0 * r0 - zst) + beta * p0;
  for (int64_t i = i0 + stride; i < n; i += stride)
    p[off + i] = (dm[i] * r[off + i] - zst) + beta * p[off + i];
}

// ---- CG steps around a preconditioner applied between the launches (z given), one member:
// the step length, the next direction and the next scalars come from device-side partial
// sums, as in the Jacobi CG, so that the host only reads the scalars to stop.

// x += alpha p; r -= alpha w, alpha formed by every block from the scalars and the apply's
// partials of p.Ap; with r32 also r32 = (float) r (the input of an FP32 preconditioner).
__global__ void gpcg_update_kernel(double *__restrict__ x, const double *__restrict__ p,
                                   double *__restrict__ r, const double *__restrict__ w,
                                   float *__restrict__ r32, const PcgScalars *__restrict__ sc,
                                   const double *__restrict__ dpart, int dcount, int64_t n) {
  double pw[1];
  reduce_parts_m<1, VB>(dpart, dcount, 0, pw);
  const double alpha = step_alpha(sc[0], pw[0]);
  for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * w[i];
    r[i] = ri;
    if (r32) r32[i] = (float)ri;
  }
}

// Partials of r.z and r.r, then by NV: 4, sum z and sum r (for the null-space shift);
// 5, b.b and two zeros (the five quantities the scalar initialization reads).
template <int NV, typename TZ>
__global__ void gpcg_dots_kernel(const double *__restrict__ r, const TZ *__restrict__ z,
                                 const double *__restrict__ b, double *__restrict__ part, int nblk,
                                 int64_t n) {
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)nblk * VB) {
    const double ri = r[i], zi = (double)z[i];
    v[0] += ri * zi;
    v[1] += ri * ri;
    if constexpr (NV == 4) {
      v[2] += zi;
      v[3] += ri;
    }
    if constexpr (NV == 5) v[2] += b[i] * b[i];
  }
  write_part<NV>(v, part, nblk);
}

// p = (z - zs) + beta p, with alpha (for the failure state), beta and the stopping test
// formed by every block from the scalars and the partials of p.Ap and of r.z, r.r (and,
// with NS, sum z and sum r: zs = mean(z), the preconditioned residual orthogonalized
// against the constants, whose r.(z - zs) = r.z - zs sum r); block 0 writes the next
// scalars to sc_next (double-buffered).
template <typename TZ, bool NS>
__global__ void gpcg_newdir_kernel(const TZ *__restrict__ z, double *__restrict__ p,
                                   const PcgScalars *__restrict__ sc, PcgScalars *__restrict__ sc_next,
                                   const double *__restrict__ dpart, int dcount,
                                   const double *__restrict__ upart, int unblk, int64_t n) {
  constexpr int NU = NS ? 4 : 2;
  double pw[1], u[NU];
  reduce_parts_m<1, VB>(dpart, dcount, 0, pw);
  reduce_parts_m<NU, VB>(upart, unblk, 0, u);
  PcgScalars s = sc[0];
  set_alpha(s, pw[0]);
  double zs = 0.0, rz = u[0];
  if constexpr (NS) {
    zs = u[2] / (double)n;
    rz = u[0] - zs * u[3];
  }
  set_beta(s, rz, u[1]);
  if (blockIdx.x == 0 && threadIdx.x == 0) sc_next[0] = s;
  const double beta = s.beta;
  for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB)
    p[i] = ((double)z[i] - zs) + beta * p[i];
}

// r = b - w with partial r.r (w may be null: r = b); r may be null (norm only)
__global__ void sub_norm_kernel(const double *__restrict__ b, const double *__restrict__ w,
                                double *__restrict__ r, double *__restrict__ part, int nblk,
                                int64_t n) {
  const int64_t off = (int64_t)blockIdx.y * n;
  double v[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)nblk * VB) {
    const double ri = w ? b[off + i] - w[off + i] : b[off + i];
    if (r) r[off + i] = ri;
    v[0] += ri * ri;
  }
  write_part<1>(v, part, nblk);
}

__global__ void __launch_bounds__(RB) init_scalars_kernel(const double *__restrict__ part, int nblk, double rtol,
                                    PcgScalars *__restrict__ sc, int nullspace, int64_t n) {
  double v[5];
  reduce_parts<5>(part, nblk, v);
  if (threadIdx.x == 0) {
    PcgScalars &s = sc[blockIdx.x];
    s.zshift = nullspace ? v[3] / (double)n : 0.0;
    s.rho = v[0] - s.zshift * v[4];
    s.rr = v[1];
    s.bb = v[2];
    s.pw = 0.0;
    s.alpha = 0.0;
    s.beta = 0.0;
    s.tol2 = rtol * rtol * v[2];
    s.iters = 0;
    const bool finite = isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
    s.status = finite ? 0 : SFEM_E_NAN;
    s.active = (finite && v[2] > 0.0 && v[1] > s.tol2) ? 1 : 0;
  }
}

// v[m][i] -= sc[m].zshift
template <typename T>
__global__ void zshift_kernel(T *__restrict__ v, const PcgScalars *__restrict__ sc, int64_t n) {
  const int m = blockIdx.y;
  const T zs = (T)sc[m].zshift;
  for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB)
    v[(int64_t)m * n + i] -= zs;
}

// v[m][i] -= c[m] * scale
__global__ void shift_kernel(double *__restrict__ v, const double *__restrict__ c, double scale,
                             int64_t n) {
  const int m = blockIdx.y;
  const double d = c[m] * scale;
  for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB)
    v[(int64_t)m * n + i] -= d;
}

// out[m * nv + k] = sum of partials
template <int NV>
__global__ void __launch_bounds__(RB) reduce_out_kernel(const double *__restrict__ part, int nblk,
                                  double *__restrict__ out) {
  double v[NV];
  reduce_parts<NV>(part, nblk, v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) out[(int64_t)blockIdx.x * NV + k] = v[k];
  }
}

// IR state per member: [0] = ||r||^2, [1] = ||b||^2, [2] = scale (||r|| while refining, else 0)
__global__ void __launch_bounds__(RB) ir_norm_kernel(const double *__restrict__ part, int nblk, int set_bb, double rtol,
                               double *__restrict__ ir) {
  double v[1];
  reduce_parts<1>(part, nblk, v);
  if (threadIdx.x == 0) {
    double *s = ir + 3 * (int64_t)blockIdx.x;
    s[0] = v[0];
    if (set_bb) s[1] = v[0];
    s[2] = (v[0] > rtol * rtol * s[1]) ? sqrt(v[0]) : 0.0;
  }
}

__global__ void ir_cast_kernel(const double *__restrict__ r, const double *__restrict__ ir,
                               float *__restrict__ r32, int64_t n) {
  const int m = blockIdx.y;
  const double sc = ir[3 * m + 2];
  const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
  const int64_t off = (int64_t)m * n;
  for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * VB)
    r32[off + i] = (float)(r[off + i] * inv);
}

__global__ void ir_accum_kernel(double *__restrict__ x, const float *__restrict__ d,
                                const double *__restrict__ ir, int64_t n) {
  const int m = blockIdx.y;
  const double sc = ir[3 * m + 2];
  if (sc == 0.0) return;
  const int64_t off = (int64_t)m * n;
  for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * VB)
    x[off + i] += sc * (double)d[off + i];
}

// Assembly over the list of shared and essential DoFs: y[g] = sum of the E-vector
// entries of list entry i in element order -- [aoff[i], aoff[i+1]) for the DoF-ordered
// E-vector (consecutive threads then read consecutive runs), slot[aoff[i]..aoff[i+1])
// for the element-ordered one; essential DoFs (no entries) get x[g], 1 or 0 (kEssAdd:
// y[g] += the sum at the other DoFs, essential entries untouched).  DOT: also
// the per-block sums of x_g y_g.  Each thread takes AU list entries per pass (stride
// VB); the first KS entries of each are loaded together, longer lists fall back to a
// loop.  Index arithmetic is 32-bit (entries below 2^30, checked at set-up).
constexpr int AU = 1;
constexpr int KS = 8;

template <typename T, bool DOT>
__global__ void __launch_bounds__(VB)
assemble_kernel(AsmPlan pl, const T *__restrict__ Y, int64_t estride, const T *__restrict__ x,
                T *__restrict__ y, int64_t n, int ess_kind, double *__restrict__ part,
                int64_t part_mstride, int nblk, const double *__restrict__ epart, int ne) {
  const int mb = blockIdx.y;
  const T *Ym = Y + (int64_t)mb * estride;
  const T *xm = x ? x + (int64_t)mb * n : nullptr;
  T *ym = y + (int64_t)mb * n;
  const int na = (int)pl.na;
  double v[1] = {0.0};
  for (int base = (int)blockIdx.x * (VB * AU) + (int)threadIdx.x; base < na; base += nblk * (VB * AU)) {
    int32_t g[AU], a[AU], d[AU];
#pragma unroll
    for (int k = 0; k < AU; ++k) {
      const int i = base + k * VB;
      const bool in = i < na;
      g[k] = in ? pl.alist[i] : 0;
      a[k] = in ? pl.aoff[i] : 0;
      d[k] = in ? pl.aoff[i + 1] - a[k] : -1;
    }
    int32_t sl[AU][KS];
#pragma unroll
    for (int k = 0; k < AU; ++k)
#pragma unroll
      for (int j = 0; j < KS; ++j) sl[k][j] = (j < d[k]) ? (pl.slot ? pl.slot[a[k] + j] : a[k] + j) : 0;
    T val[AU][KS];
#pragma unroll
    for (int k = 0; k < AU; ++k)
#pragma unroll
      for (int j = 0; j < KS; ++j) val[k][j] = (j < d[k]) ? Ym[sl[k][j]] : T(0);
#pragma unroll
    for (int k = 0; k < AU; ++k) {
      if (d[k] < 0) continue;
      T acc = val[k][0];
#pragma unroll
      for (int j = 1; j < KS; ++j)
        if (j < d[k]) acc += val[k][j];
      for (int j = KS; j < d[k]; ++j) acc += Ym[pl.slot ? pl.slot[a[k] + j] : a[k] + j];
      const T xg = (DOT || (d[k] == 0 && ess_kind == kEssCopyX)) ? xm[g[k]] : T(0);
      if (ess_kind == kEssAdd) {
        if (d[k] > 0) ym[g[k]] += acc;
        continue;
      }
      if (d[k] == 0) acc = (ess_kind == kEssCopyX) ? xg : (ess_kind == kEssOne ? T(1) : T(0));
      ym[g[k]] = acc;
      if constexpr (DOT) v[0] += (double)xg * (double)acc;
    }
  }
  if constexpr (DOT) {
    // this block's share of the element kernel's partial sums (a fixed range), so that
    // the apply leaves one partial per assembly block
    const double *ep = epart + (int64_t)mb * part_mstride;
    const int lo = (int)((int64_t)ne * blockIdx.x / nblk);
    const int hi = (int)((int64_t)ne * (blockIdx.x + 1) / nblk);
    for (int i = lo + (int)threadIdx.x; i < hi; i += VB) v[0] += ep[i];
    block_sum<1>(v);
    if (threadIdx.x == 0) part[(int64_t)mb * part_mstride + blockIdx.x] = v[0];
  }
}

template <typename T>
__global__ void fill_kernel(T *__restrict__ p, T v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * VB)
    p[i] = v;
}

template <typename T>
__global__ void recip_kernel(const double *__restrict__ d, T *__restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * VB)
    out[i] = (T)(1.0 / d[i]);
}

unsigned grid_for(int64_t n) {
  int64_t b = (n + VB * 4 - 1) / (VB * 4);
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (unsigned)b;
}

}  // namespace

int assemble_nblk(int64_t na) {
  int64_t b = (na + VB * AU - 1) / (VB * AU);
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return (int)b;
}


int assemble_nblk_dot(int64_t na) {
  const int b = assemble_nblk(na);
  return b < kMaxParts ? b : kMaxParts;
}

int vec_nblk(int64_t n) {
  int64_t b = (n + VB * 2 - 1) / (VB * 2);
  if (b < 1) b = 1;
  if (b > kMaxParts) b = kMaxParts;
  return (int)b;
}

template <typename T>
hipError_t VecOps<T>::start(const T *b, const T *w, T *x, T *r, const T *dinv, int64_t dms, T *p,
                            double *part, int nblk, int64_t n, int nb, hipStream_t s) {
  hipLaunchKernelGGL((start_kernel<T>), dim3(nblk, nb), dim3(VB), 0, s, b, w, x, r, dinv, dms, p,
                     part, nblk, n);
  return hipGetLastError();
}

template <typename T>
hipError_t VecOps<T>::dot(const T *a, const T *c, int64_t c_mstride, double *part, int nblk,
                          int64_t n, int nb, hipStream_t s) {
  hipLaunchKernelGGL((dot_kernel<T>), dim3(nblk, nb), dim3(VB), 0, s, a, c, c_mstride, part, nblk, n);
  return hipGetLastError();
}

template <typename T>
hipError_t VecOps<T>::update(T *x, const T *p, T *r, const T *w, const T *dinv, int64_t dms,
                             const PcgScalars *sc, const double *dpart, int64_t dmstride,
                             int dcount, double *part, int nblk, int64_t n, int nb,
                             hipStream_t s) {
  hipLaunchKernelGGL((update_kernel<T>), dim3(nblk, nb), dim3(VB), 0, s, x, p, r, w, dinv, dms, sc,
                     dpart, dmstride, dcount, part, nblk, n);
  return hipGetLastError();
}

template <typename T>
hipError_t VecOps<T>::newdir(const T *r, const T *dinv, int64_t dms, T *p, const PcgScalars *sc,
                             PcgScalars *sc_next, const double *dpart, int64_t dmstride,
                             int dcount, const double *upart, int unblk, int nullspace, int64_t n,
                             int nb, hipStream_t s) {
  hipLaunchKernelGGL((newdir_kernel<T>), dim3(vec_nblk(n), nb), dim3(VB), 0, s, r, dinv, dms, p, sc,
                     sc_next, dpart, dmstride, dcount, upart, unblk, nullspace, n);
  return hipGetLastError();
}

template <typename T>
hipError_t VecOps<T>::fill(T *p, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((fill_kernel<T>), dim3(grid_for(n)), dim3(VB), 0, s, p, v, n);
  return hipGetLastError();
}

template <typename T>
hipError_t VecOps<T>::recip(const double *d, T *out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((recip_kernel<T>), dim3(grid_for(n)), dim3(VB), 0, s, d, out, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_assemble(const AsmPlan &pl, const T *evec, int64_t estride, const T *x, T *y,
                           int64_t n, int nb, int ess_kind, double *part, int64_t part_mstride,
                           hipStream_t s, const double *epart, int ne) {
  if (pl.na <= 0 || nb <= 0) return hipSuccess;
  const int nblk = part ? assemble_nblk_dot(pl.na) : assemble_nblk(pl.na);
  if (part)
    hipLaunchKernelGGL((assemble_kernel<T, true>), dim3(nblk, nb), dim3(VB), 0, s, pl, evec, estride,
                       x, y, n, ess_kind, part, part_mstride, nblk, epart, ne);
  else
    hipLaunchKernelGGL((assemble_kernel<T, false>), dim3(nblk, nb), dim3(VB), 0, s, pl, evec, estride,
                       x, y, n, ess_kind, part, part_mstride, nblk, epart, ne);
  return hipGetLastError();
}
template hipError_t launch_assemble<double>(const AsmPlan &, const double *, int64_t, const double *,
                                            double *, int64_t, int, int, double *, int64_t,
                                            hipStream_t, const double *, int);
template hipError_t launch_assemble<float>(const AsmPlan &, const float *, int64_t, const float *,
                                           float *, int64_t, int, int, double *, int64_t, hipStream_t,
                                           const double *, int);

template struct VecOps<double>;
template struct VecOps<float>;

hipError_t launch_gpcg_update(double *x, const double *p, double *r, const double *w, float *r32,
                              const PcgScalars *sc, const double *dpart, int dcount, int64_t n,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gpcg_update_kernel, dim3(vec_nblk(n)), dim3(VB), 0, s, x, p, r, w, r32, sc, dpart,
                     dcount, n);
  return hipGetLastError();
}

template <typename TZ>
hipError_t launch_gpcg_dots(const double *r, const TZ *z, const double *b, int nullspace, double *part,
                            int nblk, int64_t n, hipStream_t s) {
  if (b)
    hipLaunchKernelGGL((gpcg_dots_kernel<5, TZ>), dim3(nblk), dim3(VB), 0, s, r, z, b, part, nblk, n);
  else if (nullspace)
    hipLaunchKernelGGL((gpcg_dots_kernel<4, TZ>), dim3(nblk), dim3(VB), 0, s, r, z, b, part, nblk, n);
  else
    hipLaunchKernelGGL((gpcg_dots_kernel<2, TZ>), dim3(nblk), dim3(VB), 0, s, r, z, b, part, nblk, n);
  return hipGetLastError();
}

template <typename TZ>
hipError_t launch_gpcg_newdir(const TZ *z, double *p, const PcgScalars *sc, PcgScalars *sc_next,
                              const double *dpart, int dcount, const double *upart, int unblk,
                              int nullspace, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (nullspace)
    hipLaunchKernelGGL((gpcg_newdir_kernel<TZ, true>), dim3(vec_nblk(n)), dim3(VB), 0, s, z, p, sc, sc_next,
                       dpart, dcount, upart, unblk, n);
  else
    hipLaunchKernelGGL((gpcg_newdir_kernel<TZ, false>), dim3(vec_nblk(n)), dim3(VB), 0, s, z, p, sc,
                       sc_next, dpart, dcount, upart, unblk, n);
  return hipGetLastError();
}
template hipError_t launch_gpcg_dots<double>(const double *, const double *, const double *, int, double *,
                                             int, int64_t, hipStream_t);
template hipError_t launch_gpcg_dots<float>(const double *, const float *, const double *, int, double *,
                                            int, int64_t, hipStream_t);
template hipError_t launch_gpcg_newdir<double>(const double *, double *, const PcgScalars *, PcgScalars *,
                                               const double *, int, const double *, int, int, int64_t,
                                               hipStream_t);
template hipError_t launch_gpcg_newdir<float>(const float *, double *, const PcgScalars *, PcgScalars *,
                                              const double *, int, const double *, int, int, int64_t,
                                              hipStream_t);

hipError_t launch_sub_norm(const double *b, const double *w, double *r, double *part, int nblk,
                           int64_t n, int nb, hipStream_t s) {
  hipLaunchKernelGGL(sub_norm_kernel, dim3(nblk, nb), dim3(VB), 0, s, b, w, r, part, nblk, n);
  return hipGetLastError();
}

hipError_t launch_pcg_init(const double *part, int nblk, int nb, double rtol, PcgScalars *sc,
                           hipStream_t s, int nullspace, int64_t n) {
  hipLaunchKernelGGL(init_scalars_kernel, dim3(nb), dim3(RB), 0, s, part, nblk, rtol, sc, nullspace, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zshift(T *v, const PcgScalars *sc, int64_t n, int nb, hipStream_t s) {
  if (n <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((zshift_kernel<T>), dim3(grid_for(n), nb), dim3(VB), 0, s, v, sc, n);
  return hipGetLastError();
}
template hipError_t launch_zshift<double>(double *, const PcgScalars *, int64_t, int, hipStream_t);
template hipError_t launch_zshift<float>(float *, const PcgScalars *, int64_t, int, hipStream_t);

hipError_t launch_shift(double *v, const double *c, double scale, int64_t n, int nb, hipStream_t s) {
  if (n <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(shift_kernel, dim3(grid_for(n), nb), dim3(VB), 0, s, v, c, scale, n);
  return hipGetLastError();
}

hipError_t launch_reduce1(const double *part, int nblk, int nb, double *out, hipStream_t s) {
  hipLaunchKernelGGL((reduce_out_kernel<1>), dim3(nb), dim3(RB), 0, s, part, nblk, out);
  return hipGetLastError();
}

hipError_t launch_ir_norm(const double *part, int nblk, int nb, int set_bb, double rtol, double *ir,
                          hipStream_t s) {
  hipLaunchKernelGGL(ir_norm_kernel, dim3(nb), dim3(RB), 0, s, part, nblk, set_bb, rtol, ir);
  return hipGetLastError();
}

hipError_t launch_ir_cast(const double *r, const double *ir, float *r32, int64_t n, int nb,
                          hipStream_t s) {
  hipLaunchKernelGGL(ir_cast_kernel, dim3(grid_for(n), nb), dim3(VB), 0, s, r, ir, r32, n);
  return hipGetLastError();
}

hipError_t launch_ir_accum(double *x, const float *d, const double *ir, int64_t n, int nb,
                           hipStream_t s) {
  hipLaunchKernelGGL(ir_accum_kernel, dim3(grid_for(n), nb), dim3(VB), 0, s, x, d, ir, n);
  return hipGetLastError();
}

}  // namespace sfem
