// Coupling blocks of the Taylor-Hood Stokes operator (Section 3, eq. gradient and
// eq. divergence): velocity in (Q_p)^3, pressure in Q_{p-1}, both nodal on the GLL
// points, on the same elements and the same q = p + 2 Gauss points.  With the stored
// coupling factor C = w |J| J^{-T} at each point (C_cd = w adj(J)_dc), the physical
// gradient of a scalar f integrated against w|J| is C grad_ref f, so
//
//   (G p)_{l, c} = sum_Q phi_l(Q) (C_Q grad_ref p(Q))_c
//   (D u)_m      = sum_Q psi_m(Q) sum_c (C_Q grad_ref u_c(Q))_c
//
// Both are sum-factorized like the scalar operators (Section 3.1): the reference
// gradient by B/G contractions direction by direction, the test functions by the
// transposed B contractions.  One element per q^2 threads, the workgroups of the apply
// kernel (same LDS buffers, same thread-per-1D-line stages).  Outputs go through the
// same conflict-free assembly as the apply: values of DoFs owned by one element are
// written directly, those of shared DoFs to the E-vector of their space.
#include <hip/hip_runtime.h>

#include "apply_impl.h"

namespace sfem {
namespace {

// 1D tables of an order-PO space at the q points of order P (q = P + 2).
template <int PO, int Q>
struct Tab2 {
  static constexpr rules::Tables<PO, Q> c = rules::tables<PO, Q>();
  static constexpr double B(int a, int i) { return c.B[a][i]; }
  static constexpr double G(int a, int i) { return c.G[a][i]; }
};

// Forward reference gradient of a nodal field with NI nodes per direction (in buf,
// [k][j][i]) for the q x q threads of an element: stage xi_1 and xi_2 through LDS, the
// xi_3 contraction is done by the caller from the three lines this returns.
template <int NI, int Q, typename TB>
__device__ __forceinline__ void fwd_grad_xy(double *buf, int t) {
  constexpr int N2 = NI * NI, QN2 = Q * N2, NQ2 = NI * Q * Q;
  {  // xi_1: [k][j][i] -> [k][j][a] (B and G)
    const bool w = t < N2;
    const int j = t % NI, k = t / NI;
    double ob[Q], og[Q];
    if (w) {
      double in[NI];
#pragma unroll
      for (int i = 0; i < NI; ++i) in[i] = buf[(k * NI + j) * NI + i];
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        double sb = 0.0, sg = 0.0;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          sb += TB::B(a, i) * in[i];
          sg += TB::G(a, i) * in[i];
        }
        ob[a] = sb;
        og[a] = sg;
      }
    }
    __syncthreads();
    if (w) {
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        buf[(k * NI + j) * Q + a] = ob[a];
        buf[QN2 + (k * NI + j) * Q + a] = og[a];
      }
    }
    __syncthreads();
  }
  {  // xi_2: [k][j][a] -> [k][b][a]: B(Bx), G(Bx), B(Gx)
    const bool w = t < Q * NI;
    const int a = t % Q, k = t / Q;
    double obb[Q], ogb[Q], obg[Q];
    if (w) {
      double ib[NI], ig[NI];
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        ib[j] = buf[(k * NI + j) * Q + a];
        ig[j] = buf[QN2 + (k * NI + j) * Q + a];
      }
#pragma unroll
      for (int b = 0; b < Q; ++b) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int j = 0; j < NI; ++j) {
          s0 += TB::B(b, j) * ib[j];
          s1 += TB::G(b, j) * ib[j];
          s2 += TB::B(b, j) * ig[j];
        }
        obb[b] = s0;
        ogb[b] = s1;
        obg[b] = s2;
      }
    }
    __syncthreads();
    if (w) {
#pragma unroll
      for (int b = 0; b < Q; ++b) {
        buf[(k * Q + b) * Q + a] = obb[b];
        buf[NQ2 + (k * Q + b) * Q + a] = ogb[b];
        buf[2 * NQ2 + (k * Q + b) * Q + a] = obg[b];
      }
    }
    __syncthreads();
  }
}

// Transposed mass-type contractions of NF fields given at the q^3 points (each thread
// holds its xi_3 line v[f][c]) down to nodal fields with NO nodes per direction, field f
// at buf + f * NO^3 ([k][j][i]).  Ends with a barrier.
template <int NO, int Q, int NF, typename TB>
__device__ __forceinline__ void bwd_mass(double *buf, int t, const double (&v)[NF][Q]) {
  constexpr int NQ2 = NO * Q * Q, N2Q = NO * NO * Q, N3 = NO * NO * NO;
  {  // xi_3: [c] -> [k][b][a]
    double r[NF][NO];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int k = 0; k < NO; ++k) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < Q; ++c) s += TB::B(c, k) * v[f][c];
        r[f][k] = s;
      }
    __syncthreads();
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int k = 0; k < NO; ++k) buf[f * NQ2 + k * Q * Q + t] = r[f][k];
    __syncthreads();
  }
  {  // xi_2: [k][b][a] -> [k][j][a]
    const bool w = t < Q * NO;
    const int a = t % Q, k = t / Q;
    double r[NF][NO];
    if (w) {
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        double in[Q];
#pragma unroll
        for (int b = 0; b < Q; ++b) in[b] = buf[f * NQ2 + (k * Q + b) * Q + a];
#pragma unroll
        for (int j = 0; j < NO; ++j) {
          double s = 0.0;
#pragma unroll
          for (int b = 0; b < Q; ++b) s += TB::B(b, j) * in[b];
          r[f][j] = s;
        }
      }
    }
    __syncthreads();
    if (w) {
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int j = 0; j < NO; ++j) buf[f * N2Q + (k * NO + j) * Q + a] = r[f][j];
    }
    __syncthreads();
  }
  {  // xi_1: [k][j][a] -> [k][j][i]
    const bool w = t < NO * NO;
    const int j = t % NO, k = t / NO;
    double r[NF][NO];
    if (w) {
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        double in[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) in[a] = buf[f * N2Q + (k * NO + j) * Q + a];
#pragma unroll
        for (int i = 0; i < NO; ++i) {
          double s = 0.0;
#pragma unroll
          for (int a = 0; a < Q; ++a) s += TB::B(a, i) * in[a];
          r[f][i] = s;
        }
      }
    }
    __syncthreads();
    if (w) {
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int i = 0; i < NO; ++i) buf[f * N3 + (k * NO + j) * NO + i] = r[f][i];
    }
    __syncthreads();
  }
}

// Gather of a pressure-space element (order P - 1, no essential DoFs) into buf and its
// map entries into smap, for the q^2 threads of the element (TPE = (P + 2)^2).
template <int P>
__device__ __forceinline__ void gather_pres(double *buf, int t, bool active, const int32_t *emap,
                                            const double *__restrict__ x, int32_t *smap) {
  constexpr int NP3 = P * P * P, TPE = (P + 2) * (P + 2);
  constexpr int NL = (NP3 + TPE - 1) / TPE;
  int32_t c[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int l0 = t + k * TPE;
    c[k] = emap[l0 < NP3 ? l0 : NP3 - 1];
  }
  double v[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) v[k] = x[c[k] & kDofMask];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int l = t + k * TPE;
    if (l < NP3) {
      buf[l] = active ? v[k] : 0.0;
      smap[l] = c[k];
    }
  }
  __syncthreads();
}

// Output of a pressure-space element vector (element-ordered E-vector, surface ranks of
// order P - 1 when compact): sole DoFs -> y, shared nodes -> Y[e * epe + r].
template <int P>
__device__ __forceinline__ void emit_pres(const double *buf, int t, bool active,
                                          const int32_t *smap, int64_t e, bool compact,
                                          double *__restrict__ Y, double *__restrict__ y) {
  constexpr int NP3 = P * P * P, TPE = (P + 2) * (P + 2);
  constexpr int NL = (NP3 + TPE - 1) / TPE;
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int l0 = t + k * TPE;
    const int l = l0 < NP3 ? l0 : NP3 - 1;
    const int32_t c = smap[l];
    const double v = buf[l];
    const bool ok = active && l0 < NP3;
    const bool sole = (c & kSoleBit) != 0;
    const int64_t ye = compact ? e * surf_count<P - 1>() + surf_rank<P - 1>(l) : e * NP3 + l;
    double *dst = sole ? y + (c & kDofMask) : Y + ye;
    if (ok) *dst = v;
  }
}

// The velocity element's map entries into smap (as the apply's gather keeps them: with
// POS the E-vector entry of each shared node, from the position table row epos).
template <int P, bool POS>
__device__ __forceinline__ void vel_entries(int t, const int32_t *emap, int32_t *smap,
                                            const int32_t *epos, bool compact) {
  using D = Dims<P>;
  constexpr int NL = Per<P>::NL;
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int l0 = t + k * D::TPE;
    const int l = l0 < D::N3 ? l0 : D::N3 - 1;
    const int32_t c = emap[l];
    int32_t v = c;
    if constexpr (POS) {
      const int r = compact ? surf_rank<P>(l) : l;
      const int32_t q = epos[r >= 0 ? r : 0];
      v = (c >= 0 && !(c & kSoleBit)) ? q : c;
    }
    if (l0 < D::N3) smap[l] = v;
  }
  __syncthreads();
}

template <int P>
struct SDims {
  using D = Dims<P>;
  static constexpr int N = P + 1, NP = P, Q = P + 2, Q2 = Q * Q, Q3 = Q * Q * Q;
  static constexpr int TPE = D::TPE, E = D::E, THREADS = D::THREADS;
  static_assert(D::BUF >= 3 * N * Q * Q && D::BUF >= 3 * Q * Q * NP && D::BUF >= 2 * Q * N * N,
                "element buffer");
};

// Output of a velocity element vector that adds into y: sole DoFs y[g] += v (each has
// exactly one writer), shared nodes -> their E-vector entry (as the apply), essential ->
// nothing.
template <int P, bool POS>
__device__ __forceinline__ void emit_add_vel(const double *buf, int t, bool active,
                                             const int32_t *smap, int64_t e, bool compact,
                                             double *__restrict__ Y, double *__restrict__ y) {
  using D = Dims<P>;
  constexpr int NL = Per<P>::NL;
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int l0 = t + k * D::TPE;
    const int l = l0 < D::N3 ? l0 : D::N3 - 1;
    const int32_t c = smap[l];
    const double v = buf[l];
    if (!(active && l0 < D::N3 && c >= 0)) continue;
    if (c & kSoleBit) {
      y[c & kDofMask] += v;
    } else if constexpr (POS) {
      Y[c] = v;
    } else {
      Y[compact ? e * surf_count<P>() + surf_rank<P>(l) : e * D::N3 + l] = v;
    }
  }
}

// Both coupling blocks in one pass over the elements, so that the coupling factors are
// read once: G p added into the three velocity components (their E-vector for the shared
// nodes, members at stride vestride; the sole DoFs of yv directly) and -D P u into the
// pressure space (element-ordered E-vector Yp, sole DoFs of yp).  cq: [nelem][9][q^3],
// slot 3c + d holds C_cd.
template <int P, bool POS>
__global__ void __launch_bounds__(Dims<P>::THREADS)
coupling_kernel(const int32_t *__restrict__ vmap, const int32_t *__restrict__ vpos, int vcompact,
                const int32_t *__restrict__ pmap, int pcompact, const double *__restrict__ cq,
                int64_t nelem, const double *__restrict__ u, const double *__restrict__ pres,
                int64_t nv, double *__restrict__ Yv, int64_t vestride, double *__restrict__ yv,
                double *__restrict__ Yp, double *__restrict__ yp) {
  using S = SDims<P>;
  using D = Dims<P>;
  constexpr int N = S::N, NP = S::NP, Q = S::Q, Q2 = S::Q2, Q3 = S::Q3, TPE = S::TPE, E = S::E;
  constexpr int N3 = N * N * N, NP3 = NP * NP * NP;
  using TP = Tab2<P - 1, Q>;
  using TV = Tab2<P, Q>;
  __shared__ __align__(16) double smem[E * D::BUF];
  __shared__ int32_t smap_all[E * N3];
  const int le = threadIdx.x / TPE;
  const int t0 = threadIdx.x - le * TPE;
  const int t = t0;
  const int e = xcd_block() * E + le;
  const bool active = e < nelem;
  const int es = active ? e : 0;
  double *buf = smem + le * D::BUF;
  int32_t *smap = smap_all + le * N3;
  // pressure element: the xi_3 lines of its reference gradient
  gather_pres<P>(buf, t, active, pmap + (int64_t)es * NP3, pres, smap);
  fwd_grad_xy<NP, Q, TP>(buf, t);
  double pbb[NP], pgb[NP], pbg[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    pbb[k] = buf[k * Q2 + t];
    pgb[k] = buf[NP * Q2 + k * Q2 + t];
    pbg[k] = buf[2 * NP * Q2 + k * Q2 + t];
  }
  // the velocity element's map entries for the output
  const int64_t vepe = vcompact ? surf_count<P>() : N3;
  vel_entries<P, POS>(t, vmap + (int64_t)es * N3, smap, POS ? vpos + (int64_t)es * vepe : nullptr,
                      vcompact != 0);
  const double *ce = cq + (int64_t)es * (9 * Q3) + t;
  double s[1][Q];
#pragma unroll
  for (int c = 0; c < Q; ++c) s[0][c] = 0.0;
  // (one component at a time, not unrolled: fewer live registers)
#pragma unroll 1
  for (int r = 0; r < 3; ++r) {
    // indices derived from the thread are recomputed per component rather than kept live
    int t = t0;
    asm volatile("" : "+v"(t));
    // velocity component r (essential DoFs read as 0)
    gather_e<P, double, false>(buf, t, active, vmap + (int64_t)es * N3, u + r * nv);
    fwd_grad_xy<N, Q, TV>(buf, t);
    double zbb[N], zgb[N], zbg[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      zbb[k] = buf[k * Q2 + t];
      zgb[k] = buf[N * Q2 + k * Q2 + t];
      zbg[k] = buf[2 * N * Q2 + k * Q2 + t];
    }
    const double *cr = ce + (int64_t)(3 * r) * Q3;
    double v[1][Q];
#pragma unroll
    for (int c = 0; c < Q; ++c) {
      double ux = 0.0, uy = 0.0, uz = 0.0, px = 0.0, py = 0.0, pz = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        uz += TV::G(c, k) * zbb[k];
        uy += TV::B(c, k) * zgb[k];
        ux += TV::B(c, k) * zbg[k];
      }
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        pz += TP::G(c, k) * pbb[k];
        py += TP::B(c, k) * pgb[k];
        px += TP::B(c, k) * pbg[k];
      }
      // row r of C times grad_ref p (G) and times grad_ref u_r (D)
      const double c0 = cr[c * Q2], c1 = cr[Q3 + c * Q2], c2 = cr[2 * Q3 + c * Q2];
      v[0][c] = c0 * px + c1 * py + c2 * pz;
      s[0][c] -= c0 * ux + c1 * uy + c2 * uz;
    }
    // G p, component r: added into yv / the velocity E-vector
    bwd_mass<N, Q, 1, TV>(buf, t, v);
    emit_add_vel<P, POS>(buf, t, active, smap, es, vcompact != 0, Yv + r * vestride, yv + r * nv);
    __syncthreads();  // buf is reused by the next gather
  }
  // -D P u: one pressure field
  bwd_mass<NP, Q, 1, TP>(buf, t, s);
  {
    constexpr int NL = (NP3 + TPE - 1) / TPE;
    const int32_t *em = pmap + (int64_t)es * NP3;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int l = t + k * TPE;
      if (l < NP3) smap[l] = em[l];
    }
    __syncthreads();
  }
  emit_pres<P>(buf, t, active, smap, es, pcompact != 0, Yp, yp);
}

template <int P>
hipError_t launch_stokes_pt(const StokesArgs &a, hipStream_t s) {
  if constexpr (P < 2) {
    return hipErrorInvalidValue;
  } else {
    using D = Dims<P>;
    if (a.nelem <= 0) return hipSuccess;
    constexpr bool POS = evec_dof_ordered(P);
    if ((a.vpos != nullptr) != POS) return hipErrorInvalidValue;
    dim3 grid((unsigned)((a.nelem + D::E - 1) / D::E));
    dim3 block(D::THREADS);
    hipLaunchKernelGGL((coupling_kernel<P, POS>), grid, block, 0, s, a.vmap, a.vpos, a.vcompact,
                       a.pmap, a.pcompact, a.cq, a.nelem, a.u, a.pres, a.nv, a.Yv, a.vestride,
                       a.yv, a.Yp, a.yp);
    return hipGetLastError();
  }
}

}  // namespace

hipError_t launch_stokes(const StokesArgs &a, hipStream_t s) {
#define SFEM_CALL(P) launch_stokes_pt<P>(a, s)
  SFEM_DISPATCH_P(a.p, SFEM_CALL)
#undef SFEM_CALL
}

}  // namespace sfem
