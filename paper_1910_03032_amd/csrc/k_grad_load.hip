// Adjoint-gradient integrand and load vector, built from the same sum-factorized
// stages as the apply.
//
// Gradient: K depends on nu only through the stored factor W = nu w|J| J^-1 J^-T
// (Section 3.1), so dJ/dnu_q = -lam^T (dA/dnu_q) u = -beta (Gq grad_ref lam).grad_ref u
// at each quadrature point.  Reference gradients of u and lam are interpolated with
// the forward stages; the result goes to the caller's element order.
//
// Load vector: b_i = sum_q w|J| f_q phi_i, i.e. the transposed stages with the
// mass weight only (B^T in each direction), assembled like the apply (the assembly
// kernel sets the essential entries to 0).
#include <hip/hip_runtime.h>

#include "apply_impl.h"

namespace sfem {
namespace {

// Reference gradient (d/dxi_1, d/dxi_2, d/dxi_3) of a nodal field at the q points of
// this thread's xi_3 line.
template <int P, typename T>
__device__ __forceinline__ void ref_grad_line(T *buf, int t, bool active, const int32_t *emap,
                                              const T *__restrict__ v,
                                              T (&gx)[P + 2], T (&gy)[P + 2], T (&gz)[P + 2]) {
  constexpr int N = P + 1, Q = P + 2;
  using TB = Tab<P, T>;
  gather_e<P, T>(buf, t, active, emap, v);
  fwd_x<P, T, true>(buf, t);
  fwd_y<P, T, true>(buf, t);
  T zbb[N], zgb[N], zbg[N];
  load_z<P, T, true>(buf, t, zbb, zgb, zbg);
#pragma unroll
  for (int c = 0; c < Q; ++c) {
    T dx = 0, dy = 0, dz = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      dz += TB::G(c, k) * zbb[k];
      dy += TB::B(c, k) * zgb[k];
      dx += TB::B(c, k) * zbg[k];
    }
    gx[c] = dx;
    gy[c] = dy;
    gz[c] = dz;
  }
  __syncthreads();  // buf is reused by the next gather
}

template <int P>
__global__ void __launch_bounds__(Dims<P>::THREADS)
grad_kernel(const int32_t *__restrict__ map, const double *__restrict__ qd, double beta,
            int64_t nei, int nbatch, int64_t ndof, const double *__restrict__ u,
            const double *__restrict__ lam, double *__restrict__ g) {
  using D = Dims<P>;
  constexpr int Q = D::Q, Q2 = D::Q2, Q3 = D::Q3, TPE = D::TPE, E = D::E;
  __shared__ double smem[E * D::BUF];
  const int le = threadIdx.x / TPE;
  const int t = threadIdx.x - le * TPE;
  const int64_t e = (int64_t)blockIdx.x * E + le;
  const bool active = e < nei;
  const int64_t es = active ? e : 0;
  double *buf = smem + le * D::BUF;
  const int32_t *emap = map + es * (int64_t)D::N3;
  const double *qe = qd + es * (int64_t)(kQdSlots * Q3);
  for (int m = 0; m < nbatch; ++m) {
    double lx[Q], ly[Q], lz[Q], ux[Q], uy[Q], uz[Q];
    ref_grad_line<P, double>(buf, t, active, emap, lam + (int64_t)m * ndof, lx, ly, lz);
    ref_grad_line<P, double>(buf, t, active, emap, u + (int64_t)m * ndof, ux, uy, uz);
    if (active) {
      double *go = g + ((int64_t)m * nei + e) * Q3;
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        const int qi = c * Q2 + t;
        const double G11 = qe[1 * Q3 + qi], G22 = qe[2 * Q3 + qi], G33 = qe[3 * Q3 + qi];
        const double G12 = qe[4 * Q3 + qi], G13 = qe[5 * Q3 + qi], G23 = qe[6 * Q3 + qi];
        const double f1 = G11 * ux[c] + G12 * uy[c] + G13 * uz[c];
        const double f2 = G12 * ux[c] + G22 * uy[c] + G23 * uz[c];
        const double f3 = G13 * ux[c] + G23 * uy[c] + G33 * uz[c];
        go[qi] = -beta * (lx[c] * f1 + ly[c] * f2 + lz[c] * f3);
      }
    }
  }
}

template <int P>
__global__ void __launch_bounds__(Dims<P>::THREADS)
load_kernel(const int32_t *__restrict__ map, const double *__restrict__ qd, int64_t nei,
            int nbatch, int64_t ndof, const double *__restrict__ f, double *__restrict__ b,
            double *__restrict__ Y, int64_t estride, const int32_t *__restrict__ pos, int compact) {
  using D = Dims<P>;
  using TB = Tab<P, double>;
  constexpr int N = D::N, Q = D::Q, Q2 = D::Q2, Q3 = D::Q3, TPE = D::TPE, E = D::E;
  __shared__ double smem[E * D::BUF];
  const int le = threadIdx.x / TPE;
  const int t = threadIdx.x - le * TPE;
  const int64_t e = (int64_t)blockIdx.x * E + le;
  const bool active = e < nei;
  const int64_t es = active ? e : 0;
  double *buf = smem + le * D::BUF;
  const int32_t *emap = map + es * (int64_t)D::N3;
  const double *qe = qd + es * (int64_t)(kQdSlots * Q3);
  for (int m = 0; m < nbatch; ++m) {
    double p1[N];
#pragma unroll
    for (int k = 0; k < N; ++k) p1[k] = 0.0;
    if (active) {
      const double *fe = f + ((int64_t)m * nei + e) * Q3;
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        const int qi = c * Q2 + t;
        const double v = qe[qi] * fe[qi];
#pragma unroll
        for (int k = 0; k < N; ++k) p1[k] += TB::B(c, k) * v;
      }
    }
#pragma unroll
    for (int k = 0; k < N; ++k) buf[k * Q2 + t] = p1[k];
    __syncthreads();
    bwd_y<P, double, false>(buf, t);
    bwd_x<P, double, false>(buf, t);
    if (active) {
      double *bm = b + (int64_t)m * ndof;
      double *Ym = Y + (int64_t)m * estride;
      for (int l = t; l < D::N3; l += TPE) {
        const int32_t c = emap[l];
        if (c < 0) continue;
        if (c & kSoleBit) {
          bm[c & kDofMask] = buf[l];
        } else {
          const int64_t q = compact ? e * surf_count<P>() + surf_rank<P>(l) : e * D::N3 + l;
          Ym[pos ? pos[q] : q] = buf[l];
        }
      }
    }
    __syncthreads();
  }
}

template <int P>
hipError_t launch_grad_p(const GradArgs &a, hipStream_t s) {
  using D = Dims<P>;
  if (a.nei <= 0 || a.nbatch <= 0) return hipSuccess;
  hipLaunchKernelGGL((grad_kernel<P>), dim3((unsigned)((a.nei + D::E - 1) / D::E)),
                     dim3(D::THREADS), 0, s, a.map, a.qd, a.beta, a.nei, a.nbatch,
                     a.ndof, a.u, a.lam, a.g);
  return hipGetLastError();
}

template <int P>
hipError_t launch_load_p(const LoadArgs &a, hipStream_t s) {
  using D = Dims<P>;
  const int64_t ne = a.nei;
  if (ne <= 0 || a.nbatch <= 0) return hipSuccess;
  hipLaunchKernelGGL((load_kernel<P>), dim3((unsigned)((ne + D::E - 1) / D::E)), dim3(D::THREADS),
                     0, s, a.map, a.qd, a.nei, a.nbatch, a.ndof, a.f, a.b, a.evec, a.estride,
                     a.pos, a.compact);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_grad(const GradArgs &a, hipStream_t s) {
#define SFEM_CALL(P) launch_grad_p<P>(a, s)
  SFEM_DISPATCH_P(a.p, SFEM_CALL)
#undef SFEM_CALL
}

hipError_t launch_load(const LoadArgs &a, hipStream_t s) {
#define SFEM_CALL(P) launch_load_p<P>(a, s)
  SFEM_DISPATCH_P(a.p, SFEM_CALL)
#undef SFEM_CALL
}

}  // namespace sfem
