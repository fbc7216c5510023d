// Internal interfaces of the flow-solver operators (not part of the C ABI): the
// Taylor-Hood coupling blocks of the Stokes operator and the convection term, with the
// coupling factors they read.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfem {

// Coupling blocks of the Taylor-Hood Stokes operator (velocity order p, pressure p - 1),
// one pass over the elements: G p added into the velocity vector yv ([3][nv]; sole DoFs
// directly, shared nodes through the velocity E-vector Yv, members at stride vestride:
// with the DoF-ordered E-vector added into the entries of the Helmholtz element kernel's
// output, assembled once with kEssCopyX, else stored and assembled with kEssAdd) and
// -D P u into the pressure space (sole DoFs of yp, shared nodes into the element-ordered
// pressure E-vector Yp).
struct StokesArgs {
  int p;
  int64_t nelem;
  const int32_t *vmap;      // velocity flagged map [nelem][(p+1)^3]
  const int32_t *vpos;      // velocity position table (DoF-ordered E-vector) or null
  int vcompact;
  const int32_t *pmap;      // pressure flagged map [nelem][p^3]
  int pcompact;
  const double *cq;         // coupling factors [nelem][9][q^3]
  const double *u;          // [3][nv]
  const double *pres;       // [np]
  int64_t nv;
  double *Yv;               // [3][vestride]
  int64_t vestride;
  double *yv;               // [3][nv], added into
  double *Yp;               // [nelem * epe_p]
  double *yp;               // [np]
};
hipError_t launch_stokes(const StokesArgs &a, hipStream_t s);
// Convection term N(u) on the velocity space (three members), or one of the equal-order
// weak vector operators of the projection step (gradient: one input member, three
// outputs; curl: three and three; divergence: three inputs, one output): sole DoFs of y
// directly, shared nodes into the E-vector (assembled with kEssZero).
enum WeakKind { kWeakConvection = 0, kWeakGradient = 1, kWeakCurl = 2, kWeakDivergence = 3 };
struct ConvArgs {
  int kind;                 // WeakKind (the convection term or a weak vector operator)
  int p;
  int64_t nelem;
  const int32_t *vmap;
  const int32_t *vpos;
  int vcompact;
  const double *cq;         // coupling factors [nelem][9][q^3]
  const double *u;          // [3][nv]
  int64_t nv;
  double *Yv;               // [3][vestride]
  int64_t vestride;
  double *yv;               // [3][nv]
};
hipError_t launch_convection(const ConvArgs &a, hipStream_t s);
// y[m][i] = (sum_j c_j x_j[m][i]) / scale[i] (scale optional), 0 where mask[i] != 0
// (mask optional), for nb members of length n; y may be one of the x_j.
constexpr int kMaxLinTerms = 8;
struct LinComb {
  int nterm;
  double c[kMaxLinTerms];
  const double *x[kMaxLinTerms];
};
hipError_t launch_lincomb(const LinComb &lc, const double *scale, const uint8_t *mask, double *y,
                          int64_t n, int nb, hipStream_t s);
// coupling factors C = w |J| J^{-T} at the q^3 Gauss points, [nelem][9][q^3], slot 3c + d
hipError_t launch_coupling_setup(int q, const double *gx, const double *gw, const double *xyz,
                                 int64_t nei, double *cq, hipStream_t s);

}  // namespace sfem
