// Setup kernels: quadrature data (Section 3.1: w|J| and w|J| J^-1 J^-T stored at the
// quadrature points), physical quadrature-point coordinates, folding of the
// Helmholtz coefficients into the stored factors, precision casts.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "flow.h"

namespace sfem {
namespace {

struct GaussArg {
  double x[SFEM_MAX_P + 2];
  double w[SFEM_MAX_P + 2];
};

// Trilinear map through the 8 vertices (vertex v = i + 2j + 4k at reference corner
// (2i-1, 2j-1, 2k-1)): position and Jacobian J[r][d] = dx_r / dxi_d.
__device__ inline void trilinear(const double *X, const double xi[3], double pos[3],
                                 double J[3][3]) {
  for (int r = 0; r < 3; ++r) {
    pos[r] = 0.0;
    for (int d = 0; d < 3; ++d) J[r][d] = 0.0;
  }
  for (int v = 0; v < 8; ++v) {
    double s[3], f[3];
    for (int d = 0; d < 3; ++d) {
      s[d] = ((v >> d) & 1) ? 1.0 : -1.0;
      f[d] = 0.5 * (1.0 + s[d] * xi[d]);
    }
    const double Nv = f[0] * f[1] * f[2];
    const double dN0 = 0.5 * s[0] * f[1] * f[2];
    const double dN1 = 0.5 * s[1] * f[0] * f[2];
    const double dN2 = 0.5 * s[2] * f[0] * f[1];
    for (int r = 0; r < 3; ++r) {
      const double Xr = X[v * 3 + r];
      pos[r] += Xr * Nv;
      J[r][0] += Xr * dN0;
      J[r][1] += Xr * dN1;
      J[r][2] += Xr * dN2;
    }
  }
}

// Rank of local node l among the surface nodes of an order-p element (same order as the
// host plan and the element kernels), -1 for an interior node.
__device__ inline int surface_rank_rt(int p, int l) {
  const int n = p + 1;
  const int i = l % n, j = (l / n) % n, k = l / (n * n);
  if (k == 0) return i + n * j;
  if (k == p) return n * n + i + n * j;
  const int base = 2 * n * n + (k - 1) * 4 * p;
  if (j == 0) return base + i;
  if (j == p) return base + n + i;
  if (i == 0 || i == p) return base + 2 * n + 2 * (j - 1) + (i == 0 ? 0 : 1);
  return -1;
}

// Collocated mass (Section 5.1): integrating the mass matrix with the GLL rule at the
// nodes themselves makes it diagonal; element node l contributes w_l |J(xi_l)| (tensor
// GLL weight times the Jacobian determinant at the node).  Written like an element
// output: sole DoFs directly into diag, shared nodes into their E-vector entry,
// essential DoFs not at all (the assembly sets them).
__global__ void colloc_mass_kernel(GaussArg g, int p, const double *__restrict__ xyz,
                                   const int32_t *__restrict__ map, const int32_t *__restrict__ pos,
                                   int compact, int64_t nelem, double *__restrict__ diag,
                                   double *__restrict__ Y) {
  const int n = p + 1, n3 = n * n * n;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nelem * n3) return;
  const int64_t e = gid / n3;
  const int l = (int)(gid - e * n3);
  const int i = l % n, j = (l / n) % n, k = l / (n * n);
  const int32_t c = map[gid];
  if (c < 0) return;
  const double xi[3] = {g.x[i], g.x[j], g.x[k]};
  double x3[3], J[3][3];
  trilinear(xyz + e * 24, xi, x3, J);
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  const double v = g.w[i] * g.w[j] * g.w[k] * det;
  if (c & kSoleBit) {
    diag[c & kDofMask] = v;
  } else {
    const int S = p == 1 ? 8 : 2 * n * n + (n - 2) * 4 * p;
    const int64_t q = compact ? e * S + surface_rank_rt(p, l) : gid;
    Y[pos ? pos[q] : q] = v;
  }
}

__global__ void qdata_setup_kernel(GaussArg g, int q, const double *__restrict__ xyz, int64_t nei,
                                   double *__restrict__ qd, int *__restrict__ bad) {
  const int64_t q3 = (int64_t)q * q * q;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nei * q3) return;
  const int64_t e = gid / q3;
  const int qi = (int)(gid - e * q3);
  const int a = qi % q, b = (qi / q) % q, c = qi / (q * q);
  const double xi[3] = {g.x[a], g.x[b], g.x[c]};
  const double w = g.w[a] * g.w[b] * g.w[c];
  double pos[3], J[3][3];
  trilinear(xyz + e * 24, xi, pos, J);
  // adjugate: adj = det * J^{-1}
  double A[3][3];
  A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
  if (!(det > 0.0)) *bad = 1;
  // w|J| J^{-1} J^{-T} = (w / det) adj adj^T
  const double s = w / det;
  double Gm[3][3];
  for (int d = 0; d < 3; ++d)
    for (int f = 0; f < 3; ++f)
      Gm[d][f] = s * (A[d][0] * A[f][0] + A[d][1] * A[f][1] + A[d][2] * A[f][2]);
  double *o = qd + e * (int64_t)(kQdSlots * q3) + qi;
  o[0 * q3] = w * det;
  o[1 * q3] = Gm[0][0];
  o[2 * q3] = Gm[1][1];
  o[3 * q3] = Gm[2][2];
  o[4 * q3] = Gm[0][1];
  o[5 * q3] = Gm[0][2];
  o[6 * q3] = Gm[1][2];
}

// Coupling factors of the Stokes blocks: C = w |J| J^{-T} = w adj(J)^T, slot 3c + d
// holds C_cd = w adj(J)_dc; per element stored like the folded Helmholtz factors, in the
// order of the kernels' xi_3 loops: slice pairs (k, q-1-k) in turn, within a pair the two
// slices, within a slice the 9 slots of its q^2 points.
__global__ void coupling_setup_kernel(GaussArg g, int q, const double *__restrict__ xyz,
                                      int64_t nei, double *__restrict__ cq) {
  const int64_t q3 = (int64_t)q * q * q;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nei * q3) return;
  const int64_t e = gid / q3;
  const int qi = (int)(gid - e * q3);
  const int a = qi % q, b = (qi / q) % q, c = qi / (q * q);
  const double xi[3] = {g.x[a], g.x[b], g.x[c]};
  const double w = g.w[a] * g.w[b] * g.w[c];
  double pos[3], J[3][3];
  trilinear(xyz + e * 24, xi, pos, J);
  double A[3][3];  // adj(J) = det(J) J^{-1}
  A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const int q2 = q * q, t = qi - c * q2;
  const int pc = c <= q - 1 - c ? c : q - 1 - c;
  double *o = cq + e * (int64_t)(9 * q3) + (int64_t)(2 * pc + (c > q - 1 - c ? 1 : 0)) * 9 * q2 + t;
  for (int r = 0; r < 3; ++r)
    for (int d = 0; d < 3; ++d) o[(3 * r + d) * q2] = w * A[d][r];
}

__global__ void qpoint_coords_kernel(GaussArg g, int q, const double *__restrict__ xyz,
                                     int64_t nei, double *__restrict__ xq) {
  const int64_t q3 = (int64_t)q * q * q;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nei * q3) return;
  const int64_t e = gid / q3;
  const int qi = (int)(gid - e * q3);
  const int a = qi % q, b = (qi / q) % q, c = qi / (q * q);
  const double xi[3] = {g.x[a], g.x[b], g.x[c]};
  double pos[3], J[3][3];
  trilinear(xyz + e * 24, xi, pos, J);
  const int64_t o = e * q3 + qi;
  const int64_t plane = nei * q3;
  xq[o] = pos[0];
  xq[plane + o] = pos[1];
  xq[2 * plane + o] = pos[2];
}

// Folded Helmholtz factors, slot s = 0: alpha w|J|; s = 1..6: beta nu_f w|J| J^-1 J^-T, stored
// per element in the order the element kernel reads them: slice pairs (c, q-1-c) in turn,
// within a pair slice c then slice q-1-c (the middle slice of an odd q alone), within a
// slice the 7 slots, each the q^2 points of the slice:
//   fold[f][e][(2 min(c, q-1-c) + [c > q-1-c]) 7 q^2 + s q^2 + a + q b]   (point (a, b, c))
__global__ void fold_kernel(int q, int q3, const double *__restrict__ qd,
                            const double *__restrict__ nu_user, int64_t nei, int nfield,
                            double alpha, double beta,
                            double *__restrict__ fold64, float *__restrict__ fold32,
                            double *__restrict__ nu64, float *__restrict__ nu32) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per_field = nei * q3;
  if (gid >= per_field * nfield) return;
  const int64_t f = gid / per_field;
  const int64_t r = gid - f * per_field;
  const int64_t e = r / q3;
  const int qi = (int)(r - e * q3);
  const double nv = nu_user ? nu_user[f * per_field + r] : 1.0;
  const double *src = qd + e * (int64_t)(kQdSlots * q3) + qi;
  const int q2 = q * q, c = qi / q2, t = qi - c * q2;
  const int pc = c <= q - 1 - c ? c : q - 1 - c;
  const int64_t o = (f * nei + e) * (int64_t)(kQdSlots * q3) +
                    (int64_t)(2 * pc + (c > q - 1 - c ? 1 : 0)) * kQdSlots * q2 + t;
  for (int s = 0; s < kQdSlots; ++s) {
    const double v = (s == 0) ? alpha * src[0] : beta * nv * src[(int64_t)s * q3];
    fold64[o + (int64_t)s * q2] = v;
    fold32[o + (int64_t)s * q2] = (float)v;
  }
  nu64[f * per_field + r] = nv;
  nu32[f * per_field + r] = (float)nv;
}

__global__ void cast_kernel(const double *__restrict__ src, float *__restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

GaussArg gauss_arg(const double *rules_x, const double *rules_w, int q) {
  GaussArg g{};
  for (int i = 0; i < q; ++i) {
    g.x[i] = rules_x[i];
    g.w[i] = rules_w[i];
  }
  return g;
}

unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_qdata_setup(int q, const double *gx, const double *gw, const double *xyz,
                              int64_t nei, double *qd, int *bad, hipStream_t s) {
  const int64_t n = nei * (int64_t)q * q * q;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(qdata_setup_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s,
                     gauss_arg(gx, gw, q), q, xyz, nei, qd, bad);
  return hipGetLastError();
}

hipError_t launch_coupling_setup(int q, const double *gx, const double *gw, const double *xyz,
                                 int64_t nei, double *cq, hipStream_t s) {
  const int64_t n = nei * (int64_t)q * q * q;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(coupling_setup_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s,
                     gauss_arg(gx, gw, q), q, xyz, nei, cq);
  return hipGetLastError();
}

hipError_t launch_qpoint_coords(int q, const double *gx, const double *gw, const double *xyz,
                                int64_t nei, double *xq, hipStream_t s) {
  const int64_t n = nei * (int64_t)q * q * q;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(qpoint_coords_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s,
                     gauss_arg(gx, gw, q), q, xyz, nei, xq);
  return hipGetLastError();
}

hipError_t launch_fold(int q, const double *qd, const double *nu_user, int64_t nei, int nfield,
                       double alpha, double beta, double *fold64, float *fold32, double *nu64,
                       float *nu32, hipStream_t s) {
  const int q3 = q * q * q;
  const int64_t n = nei * (int64_t)q3 * nfield;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fold_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, q, q3, qd, nu_user,
                     nei, nfield, alpha, beta, fold64, fold32, nu64, nu32);
  return hipGetLastError();
}

hipError_t launch_colloc_mass(int p, const double *gll_x, const double *gll_w, const double *xyz,
                              const int32_t *map, const int32_t *pos, int compact, int64_t nelem,
                              double *diag, double *evec, hipStream_t s) {
  const int64_t n = nelem * (int64_t)(p + 1) * (p + 1) * (p + 1);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(colloc_mass_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s,
                     gauss_arg(gll_x, gll_w, p + 1), p, xyz, map, pos, compact, nelem, diag, evec);
  return hipGetLastError();
}

hipError_t launch_cast_f32(const double *src, float *dst, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(cast_kernel, dim3((unsigned)(nb < 65536 ? nb : 65536)), dim3(256), 0, s, src,
                     dst, n);
  return hipGetLastError();
}

}  // namespace sfem
