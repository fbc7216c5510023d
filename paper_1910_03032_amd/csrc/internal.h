// Internal declarations of the sfem library (host side + kernel launchers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "plan.h"
#include "sfem.h"

namespace sfem {

// How the assembly sets essential DoFs: copy x (operator apply), 1 (diagonal), 0 (load)
// What the assembly kernel writes at the essential DoFs (kEssAdd: it adds the assembled
// sums to y at the other listed DoFs and leaves the essential entries as they are).
enum EssKind { kEssCopyX = 0, kEssOne = 1, kEssZero = 2, kEssAdd = 3 };

// Quadrature-data slots per point, layout [elem][kQdSlots][q^3]:
//   0: w|J|      1..6: w|J| (J^-1 J^-T) as (11, 22, 33, 12, 13, 23)
constexpr int kQdSlots = 7;

// 1D tables for order P (n = P + 1 GLL nodes, q = P + 2 Gauss points), row-major
// [q][n]: B(a, i) = phi_i(xi_a), G(a, i) = phi_i'(xi_a).
struct Rules1D {
  int p = 0, q = 0;
  std::vector<double> gll_x, gll_w, gauss_x, gauss_w;
  std::vector<double> B, G;
};
// Host computation of the rules (Newton iterations on Legendre recurrences,
// barycentric Lagrange weights).  Returns false if a Newton iteration fails.
bool make_rules(int p, int q, Rules1D &out);

// Per-member PCG scalars kept on the device.
struct PcgScalars {
  double rho;     // r^T z
  double rr;      // r^T r
  double bb;      // b^T b
  double pw;      // p^T A p
  double alpha, beta;
  double tol2;    // (rtol ||b||)^2
  int active;     // 1 while iterating
  int status;     // 0 ok, SFEM_E_BREAKDOWN, SFEM_E_NAN
  int iters;      // completed iterations
  int pad;
  double zshift;  // null-space solves: mean of dinv r, removed from the preconditioned residual
};

// ---------------------------------------------------------------------------
// Kernel launchers (implemented in the .hip files).  Every launcher enqueues on
// `s` and returns the hipError_t of the launch.  The 1D tables are compile-time
// constants of the kernels (rules.h).
// ---------------------------------------------------------------------------
struct ApplyArgs {
  int p;
  int op;                   // SFEM_MASS / SFEM_DIFFUSION / SFEM_HELMHOLTZ
  const int32_t *map;       // [nei][n^3] flagged map, internal element order
  const void *qd;           // quadrature data, [nei][7][q^3] (slot layout above)
  int64_t qd_mstride;       // elements of qd between batch members (0 = shared)
  const void *nu;           // DIFFUSION only: [nei][q^3] or null
  int64_t nu_mstride;
  int64_t ndof;
  int nbatch;
  int64_t nelem;
  const void *x;
  void *y;                  // output at the sole DoFs
  void *evec;               // E-vector of the shared nodes, [nbatch][estride]
  int64_t estride;          // E-vector entries per member (contributions to shared DoFs)
  const int32_t *pos;       // DoF-ordered E-vector: [nelem][epe] entry of each element
                            // node; null: element-ordered, node r of element e -> e*epe + r
  int compact;              // nodes indexed by surface rank (1, epe = S) or local node (0)
  double *part;             // per-block dot partials (or null)
  int64_t part_mstride;
};
// Element phase of the apply over all elements (writes the E-vector).
hipError_t launch_apply_f64(const ApplyArgs &a, hipStream_t s);
hipError_t launch_apply_f32(const ApplyArgs &a, hipStream_t s);
// elements per workgroup of the apply kernel (one dot partial per workgroup)
int apply_group_elems_f64(int p);
int apply_group_elems_f32(int p);
// Assembly list on the device (see HostPlan): the assembled DoFs, ascending, the CSR
// offsets of their contributions, and for the element-ordered E-vector the entries of
// those contributions (slot == null: DoF-ordered, the entries are [aoff[i], aoff[i+1])).
struct AsmPlan {
  const int32_t *alist;
  const int32_t *aoff;
  const int32_t *slot;
  int64_t na;
};
// Assembly phase over the list: y[g] = sum of g's E-vector entries in element order;
// essential DoFs get x[g], 1 or 0 per ess_kind.  With part != null also the per-block
// sums of x_g y_g (part[m * part_mstride + block], assemble_nblk_dot blocks), each
// including a fixed range of the ne element-kernel partials epart[m * part_mstride + i]:
// the partials the assembly leaves are then the whole apply's.
constexpr int kMaxParts = 1024;  // cap of the partial-sum count of a reduction
int assemble_nblk(int64_t na);
int assemble_nblk_dot(int64_t na);
template <typename T>
hipError_t launch_assemble(const AsmPlan &pl, const T *evec, int64_t estride, const T *x, T *y,
                           int64_t n, int nb, int ess_kind, double *part, int64_t part_mstride,
                           hipStream_t s, const double *epart = nullptr, int ne = 0);

struct DiagArgs {
  int p;
  const int32_t *map;
  const double *qd;         // base quadrature data (FP64)
  const double *nu;         // [nelem][q^3] or null
  double alpha, beta;       // coefficients of the mass and diffusion terms
  int64_t nelem;
  double *diag;             // [ndof], written at the sole DoFs
  double *evec;             // E-vector of the shared nodes
  const int32_t *pos;       // E-vector entry of each element node, or null (see ApplyArgs)
  int compact;
};
hipError_t launch_diag(const DiagArgs &a, hipStream_t s);

hipError_t launch_qdata_setup(int q, const double *gx, const double *gw, const double *xyz,
                              int64_t nei, double *qd, int *bad, hipStream_t s);
// Collocated (GLL-integrated) mass contributions of every element node: sole DoFs into
// diag, shared nodes into their E-vector entry (then assembled with ess rows = 1).
hipError_t launch_colloc_mass(int p, const double *gll_x, const double *gll_w, const double *xyz,
                              const int32_t *map, const int32_t *pos, int compact, int64_t nelem,
                              double *diag, double *evec, hipStream_t s);
hipError_t launch_qpoint_coords(int q, const double *gx, const double *gw, const double *xyz,
                                int64_t nei, double *xq, hipStream_t s);
hipError_t launch_fold(int q, const double *qd, const double *nu_user, int64_t nei, int nfield,
                       double alpha, double beta, double *fold64, float *fold32, double *nu64,
                       float *nu32, hipStream_t s);
hipError_t launch_cast_f32(const double *src, float *dst, int64_t n, hipStream_t s);

struct GradArgs {
  int p;
  const int32_t *map;
  const double *qd;
  double beta;
  int64_t ndof, nei;
  int nbatch;
  const double *u, *lam;
  double *g;                // [nbatch][nelem][q^3] caller order
};
hipError_t launch_grad(const GradArgs &a, hipStream_t s);

struct LoadArgs {
  int p;
  const int32_t *map;
  const double *qd;
  int64_t ndof, nei;
  int nbatch;
  const double *f;          // [nbatch][nelem][q^3]
  double *b;                // written at the sole DoFs
  double *evec;             // E-vector of the shared nodes, [nbatch][estride]
  int64_t estride;
  const int32_t *pos;       // E-vector entry of each element node, or null (see ApplyArgs)
  int compact;
};
hipError_t launch_load(const LoadArgs &a, hipStream_t s);

// Vector kernels of the PCG (T = double or float).  Partial-sum buffers hold
// [nb][nv][nblk] doubles.  dinv may be shared by all members (dms = 0) or per member
// (dms = n).
template <typename T>
struct VecOps {
  static hipError_t start(const T *b, const T *w, T *x, T *r, const T *dinv, int64_t dms, T *p,
                          double *part, int nblk, int64_t n, int nb, hipStream_t s);
  // per-member partial sums of a[m] . c[m] (a: [nb][n]; c: member stride c_mstride, 0 for
  // one vector shared by all members, or null for the all-ones vector)
  static hipError_t dot(const T *a, const T *c, int64_t c_mstride, double *part, int nblk,
                        int64_t n, int nb, hipStream_t s);
  // One CG step after the apply w = A p, whose partial sums of p.Ap are dpart[m * dmstride
  // + i], i < dcount: update forms alpha and updates x and r, leaving the partials of
  // r.z, r.r, sum z, sum r in part ([nb][4][nblk]); newdir forms beta from them, updates
  // p and writes the next scalars to sc_next (the scalars are double-buffered).
  static hipError_t update(T *x, const T *p, T *r, const T *w, const T *dinv, int64_t dms,
                           const PcgScalars *sc, const double *dpart, int64_t dmstride,
                           int dcount, double *part, int nblk, int64_t n, int nb, hipStream_t s);
  static hipError_t newdir(const T *r, const T *dinv, int64_t dms, T *p, const PcgScalars *sc,
                           PcgScalars *sc_next, const double *dpart, int64_t dmstride, int dcount,
                           const double *upart, int unblk, int nullspace, int64_t n, int nb,
                           hipStream_t s);
  static hipError_t fill(T *p, T v, int64_t n, hipStream_t s);
  static hipError_t recip(const double *d, T *out, int64_t n, hipStream_t s);
};
int vec_nblk(int64_t n);
hipError_t launch_sub_norm(const double *b, const double *w, double *r, double *part, int nblk,
                           int64_t n, int nb, hipStream_t s);
// Scalar steps of the CG.  With nullspace != 0 (constants in the operator's null space,
// n unknowns per member) the preconditioned residual z = dinv r is orthogonalized,
// z - mean(z) 1, and rho = r^T z of that vector (Section 5.3).
hipError_t launch_pcg_init(const double *part, int nblk, int nb, double rtol, PcgScalars *sc,
                           hipStream_t s, int nullspace = 0, int64_t n = 0);
// v[m][i] -= sc[m].zshift (the initial direction of a null-space solve)
template <typename T>
hipError_t launch_zshift(T *v, const PcgScalars *sc, int64_t n, int nb, hipStream_t s);
// v[m][i] -= c[m] * scale (member-wise constant shift)
hipError_t launch_shift(double *v, const double *c, double scale, int64_t n, int nb, hipStream_t s);
hipError_t launch_reduce1(const double *part, int nblk, int nb, double *out, hipStream_t s);
// CG around a preconditioner applied between the launches (one member, z given in FP64
// or FP32):
//   update  x += alpha p, r -= alpha w (alpha from sc and the apply's partials dpart[0..dcount));
//           r32 != null: also r32 = (float) r
//   dots    partials of r.z, r.r ([2][nblk]); nullspace: also sum z, sum r ([4][nblk]); with
//           b != null of r.z, r.r, b.b, 0, 0 ([5][nblk], the input of launch_pcg_init)
//   newdir  p = (z - zs) + beta p with zs = mean(z) when nullspace (else 0); scalars of the
//           next iteration to sc_next
hipError_t launch_gpcg_update(double *x, const double *p, double *r, const double *w, float *r32,
                              const PcgScalars *sc, const double *dpart, int dcount, int64_t n,
                              hipStream_t s);
template <typename TZ>
hipError_t launch_gpcg_dots(const double *r, const TZ *z, const double *b, int nullspace, double *part,
                            int nblk, int64_t n, hipStream_t s);
template <typename TZ>
hipError_t launch_gpcg_newdir(const TZ *z, double *p, const PcgScalars *sc, PcgScalars *sc_next,
                              const double *dpart, int dcount, const double *upart, int unblk,
                              int nullspace, int64_t n, hipStream_t s);
hipError_t launch_ir_norm(const double *part, int nblk, int nb, int set_bb, double rtol, double *ir,
                          hipStream_t s);
hipError_t launch_ir_cast(const double *r, const double *ir, float *r32, int64_t n, int nb,
                          hipStream_t s);
hipError_t launch_ir_accum(double *x, const float *d, const double *ir, int64_t n, int nb,
                           hipStream_t s);

}  // namespace sfem
