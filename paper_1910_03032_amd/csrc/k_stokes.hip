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
#include "flow.h"

namespace sfem {
namespace {

// 1D tables of an order-PO space at the q points of order P (q = P + 2).
template <int PO, int Q>
struct Tab2 {
  static constexpr rules::Tables<PO, Q> c = rules::tables<PO, Q>();
  static constexpr double B(int a, int i) { return c.B[a][i]; }
  static constexpr double G(int a, int i) { return c.G[a][i]; }
};
// The same tables in the accessor form of the even-odd helpers (WHICH 0 = B, 1 = G): the
// GLL nodes of any order and the Gauss points are symmetric about 0, so B is
// centro-symmetric and G centro-antisymmetric for every (order, q) pair.
template <int PO, int Q, int WHICH>
struct TabEO {
  static constexpr int NO = Q, NI = PO + 1;
  static constexpr int S = WHICH == 0 ? 1 : -1;
  static constexpr double t(int a, int i) { return WHICH == 0 ? Tab2<PO, Q>::B(a, i) : Tab2<PO, Q>::G(a, i); }
  static constexpr double e(int a, int i) { return 0.5 * (t(a, i) + t(a, NI - 1 - i)); }
  static constexpr double o(int a, int i) { return 0.5 * (t(a, i) - t(a, NI - 1 - i)); }
};

// Outputs (a, q-1-a) of a 1D contraction from the even-odd split x of its input line.
template <typename TB>
__device__ __forceinline__ void row_pair(const eo::Split<TB::NI, double> &x, int a, double &lo,
                                         double &hi) {
  double Ev = 0.0, Od = 0.0;
#pragma unroll
  for (int i = 0; i < TB::NI / 2; ++i) {
    Ev += TB::e(a, i) * x.e[i];
    Od += TB::o(a, i) * x.o[i];
  }
  if constexpr (TB::NI % 2 == 1) Ev += TB::t(a, TB::NI / 2) * x.e[TB::NI / 2];
  lo = Ev + Od;
  hi = (TB::S > 0) ? (Ev - Od) : (Od - Ev);
}
// The middle output (a = q/2) of an odd q.
template <typename TB>
__device__ __forceinline__ double row_mid(const eo::Split<TB::NI, double> &x) {
  constexpr int M = TB::NO / 2;
  double v = 0.0;
#pragma unroll
  for (int i = 0; i < TB::NI / 2; ++i) v += TB::t(M, i) * (TB::S > 0 ? x.e[i] : x.o[i]);
  if constexpr (TB::NI % 2 == 1 && TB::S > 0) v += TB::t(M, TB::NI / 2) * x.e[TB::NI / 2];
  return v;
}

// Forward reference gradient of a nodal field of order PO (NI = PO + 1 nodes per
// direction, in buf as [k][j][i]) for the q x q threads of an element: stages xi_1 and
// xi_2 through LDS (even-odd contractions); the xi_3 contraction is the caller's.
template <int PO, int Q>
__device__ __forceinline__ void fwd_grad_xy(double *buf, int t) {
  constexpr int NI = PO + 1;
  constexpr int N2 = NI * NI, QN2 = Q * N2, NQ2 = NI * Q * Q;
  using BT = TabEO<PO, Q, 0>;
  using GT = TabEO<PO, Q, 1>;
  {  // xi_1: [k][j][i] -> [k][j][a] (B and G)
    const bool w = t < N2;
    const int j = t % NI, k = t / NI;
    double ob[Q], og[Q];
    if (w) {
      double in[NI];
#pragma unroll
      for (int i = 0; i < NI; ++i) in[i] = buf[(k * NI + j) * NI + i];
      const auto sp = eo::split(in);
      eo::apply<BT>(sp, ob);
      eo::apply<GT>(sp, og);
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
      const auto sb = eo::split(ib);
      eo::apply<BT>(sb, obb);
      eo::apply<GT>(sb, ogb);
      eo::apply<BT>(eo::split(ig), obg);
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
// holds its xi_3 line v[f][c]) down to nodal fields of order PO (NO = PO + 1 nodes per
// direction), field f at buf + f * NO^3 ([k][j][i]); even-odd form.  Ends with a barrier.
template <int PO, int Q, int NF>
__device__ __forceinline__ void bwd_mass(double *buf, int t, const double (&v)[NF][Q]) {
  constexpr int NO = PO + 1;
  constexpr int NQ2 = NO * Q * Q, N2Q = NO * NO * Q, N3 = NO * NO * NO;
  using BT = TabEO<PO, Q, 0>;
  auto line = [](const double (&in)[Q], double (&out)[NO]) {
    eo::Acc<NO, double> A;
    A.zero();
#pragma unroll
    for (int c = 0; c < Q / 2; ++c) A.template add_pair<BT>(c, in[c], in[Q - 1 - c]);
    if constexpr (Q % 2 == 1) A.template add_mid<BT>(in[Q / 2]);
    A.finish(out);
  };
  {  // xi_3: [c] -> [k][b][a]
    double r[NF][NO];
#pragma unroll
    for (int f = 0; f < NF; ++f) line(v[f], r[f]);
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
        line(in, r[f]);
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
        line(in, r[f]);
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

// Offset of slot z at slice c (points a + q b follow) within an element's coupling
// factors, stored by slice pair (c, q-1-c), then slice, then slot.
template <int Q>
__device__ __forceinline__ int cq_at(int c, int z) {
  const int pc = c <= Q - 1 - c ? c : Q - 1 - c;
  return ((2 * pc + (c > Q - 1 - c ? 1 : 0)) * 9 + z) * Q * Q;
}

template <int P>
struct SDims {
  using D = Dims<P>;
  static constexpr int N = P + 1, NP = P, Q = P + 2, Q2 = Q * Q, Q3 = Q * Q * Q;
  static constexpr int TPE = D::TPE, E = D::E, THREADS = D::THREADS;
  static_assert(D::BUF >= 3 * N * Q * Q && D::BUF >= 3 * Q * Q * NP && D::BUF >= 2 * Q * N * N,
                "element buffer");
  // minimum waves per SIMD the kernels below are compiled for: 2 (at most 256 registers)
  // up to p = 7, where the second wave outweighs a small spill (convection at 28^3 p = 5:
  // 338 -> 302 us, 24^3 p = 7: 577 -> 472 us); at p = 8 the spill is large and one wave
  // with more registers is faster
  static constexpr int OCC = P <= 7 ? 2 : 1;
};

// Output of a velocity element vector that adds into an apply's output: sole DoFs
// y[g] += v (each has exactly one writer), shared nodes -> their E-vector entry, essential
// -> nothing.  With the DoF-ordered E-vector (POS) the value is added into the entry the
// Helmholtz element kernel wrote, and one assembly sums both; with the element-ordered
// one (p >= 5) it is stored into an E-vector of its own, assembled into y afterwards
// (adding into the element-ordered entries measured 1-2 % slower than the second
// assembly).
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
      Y[c] += v;
    } else {
      Y[compact ? e * surf_count<P>() + surf_rank<P>(l) : e * D::N3 + l] = v;
    }
  }
}

// Both coupling blocks in one pass over the elements, so that the coupling factors are
// read once: G p added into the three velocity components (the sole DoFs of yv directly,
// the shared nodes through the E-vector, members at stride vestride, as emit_add_vel
// describes) and -D P u into the pressure space (element-ordered E-vector Yp, sole DoFs
// of yp).  cq: [nelem][9 q^3]
// (cq_at order), slot 3c + d holds C_cd.
template <int P, bool POS>
__global__ void __launch_bounds__(Dims<P>::THREADS, SDims<P>::OCC)
coupling_kernel(const int32_t *__restrict__ vmap, const int32_t *__restrict__ vpos, int vcompact,
                const int32_t *__restrict__ pmap, int pcompact, const double *__restrict__ cq,
                int64_t nelem, const double *__restrict__ u, const double *__restrict__ pres,
                int64_t nv, double *__restrict__ Yv, int64_t vestride, double *__restrict__ yv,
                double *__restrict__ Yp, double *__restrict__ yp) {
  using S = SDims<P>;
  using D = Dims<P>;
  constexpr int N = S::N, NP = S::NP, Q = S::Q, Q2 = S::Q2, Q3 = S::Q3, TPE = S::TPE, E = S::E;
  constexpr int N3 = N * N * N, NP3 = NP * NP * NP;
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
  fwd_grad_xy<P - 1, Q>(buf, t);
  eo::Split<NP, double> pbb, pgb, pbg;  // xi_3 lines of the pressure, even-odd split
  {
    double zb[NP], zg[NP], zx[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      zb[k] = buf[k * Q2 + t];
      zg[k] = buf[NP * Q2 + k * Q2 + t];
      zx[k] = buf[2 * NP * Q2 + k * Q2 + t];
    }
    pbb = eo::split(zb);
    pgb = eo::split(zg);
    pbg = eo::split(zx);
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
    fwd_grad_xy<P, Q>(buf, t);
    eo::Split<N, double> ubb, ugb, ubg;
    {
      double zb[N], zg[N], zx[N];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        zb[k] = buf[k * Q2 + t];
        zg[k] = buf[N * Q2 + k * Q2 + t];
        zx[k] = buf[2 * N * Q2 + k * Q2 + t];
      }
      ubb = eo::split(zb);
      ugb = eo::split(zg);
      ubg = eo::split(zx);
    }
    double v[1][Q];
    // row r of C times grad_ref p (G) and times grad_ref u_r (D) at slice c
    auto point = [&](int c, double ux, double uy, double uz, double px, double py, double pz) {
      const double *cr = ce + cq_at<Q>(c, 3 * r);
      const double c0 = cr[0], c1 = cr[Q2], c2 = cr[2 * Q2];
      v[0][c] = c0 * px + c1 * py + c2 * pz;
      s[0][c] -= c0 * ux + c1 * uy + c2 * uz;
    };
    using VB = TabEO<P, Q, 0>;
    using VG = TabEO<P, Q, 1>;
    using PB = TabEO<P - 1, Q, 0>;
    using PG = TabEO<P - 1, Q, 1>;
#pragma unroll
    for (int c = 0; c < Q / 2; ++c) {
      double uz0, uz1, uy0, uy1, ux0, ux1, pz0, pz1, py0, py1, px0, px1;
      row_pair<VG>(ubb, c, uz0, uz1);
      row_pair<VB>(ugb, c, uy0, uy1);
      row_pair<VB>(ubg, c, ux0, ux1);
      row_pair<PG>(pbb, c, pz0, pz1);
      row_pair<PB>(pgb, c, py0, py1);
      row_pair<PB>(pbg, c, px0, px1);
      point(c, ux0, uy0, uz0, px0, py0, pz0);
      point(Q - 1 - c, ux1, uy1, uz1, px1, py1, pz1);
    }
    if constexpr (Q % 2 == 1)
      point(Q / 2, row_mid<VB>(ubg), row_mid<VB>(ugb), row_mid<VG>(ubb), row_mid<PB>(pbg),
            row_mid<PB>(pgb), row_mid<PG>(pbb));
    // G p, component r: added into yv / the velocity E-vector
    bwd_mass<P, Q, 1>(buf, t, v);
    emit_add_vel<P, POS>(buf, t, active, smap, es, vcompact != 0, Yv + r * vestride, yv + r * nv);
    __syncthreads();  // buf is reused by the next gather
  }
  // -D P u: one pressure field
  bwd_mass<P - 1, Q, 1>(buf, t, s);
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

// Gather of a velocity component with the values of every DoF, essential ones included
// (the convection term takes u as it is).
template <int P>
__device__ __forceinline__ void gather_all(double *buf, int t, bool active, const int32_t *emap,
                                           const double *__restrict__ x) {
  using D = Dims<P>;
  constexpr int NL = Per<P>::NL;
  int32_t c[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int l0 = t + k * D::TPE;
    c[k] = emap[l0 < D::N3 ? l0 : D::N3 - 1];
  }
  double v[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) v[k] = x[c[k] & kDofMask];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int l = t + k * D::TPE;
    if (l < D::N3) buf[l] = active ? v[k] : 0.0;
  }
  __syncthreads();
}

// Interpolation of a nodal field of order P to the points, stages xi_1 and xi_2 (B only):
// afterwards buf holds [k][b][a] and each thread reads its xi_3 line.
template <int P, int Q>
__device__ __forceinline__ void fwd_val_xy(double *buf, int t) {
  constexpr int NI = P + 1, N2 = NI * NI;
  using BT = TabEO<P, Q, 0>;
  {
    const bool w = t < N2;
    const int j = t % NI, k = t / NI;
    double ob[Q];
    if (w) {
      double in[NI];
#pragma unroll
      for (int i = 0; i < NI; ++i) in[i] = buf[(k * NI + j) * NI + i];
      eo::apply<BT>(eo::split(in), ob);
    }
    __syncthreads();
    if (w) {
#pragma unroll
      for (int a = 0; a < Q; ++a) buf[(k * NI + j) * Q + a] = ob[a];
    }
    __syncthreads();
  }
  {
    const bool w = t < Q * NI;
    const int a = t % Q, k = t / Q;
    double ob[Q];
    if (w) {
      double in[NI];
#pragma unroll
      for (int j = 0; j < NI; ++j) in[j] = buf[(k * NI + j) * Q + a];
      eo::apply<BT>(eo::split(in), ob);
    }
    __syncthreads();
    if (w) {
#pragma unroll
      for (int b = 0; b < Q; ++b) buf[(k * Q + b) * Q + a] = ob[b];
    }
    __syncthreads();
  }
}

// Pointwise products of the element kernels below that test against the basis values
// (the three outputs are tested against phi): with the coupling factor C = w |J| J^{-T}
// and Gamma_dr = sum_k C_dk d_ref_k u_r = w |J| d u_r / d x_d,
//   kConvection:   n_c = sum_d u_d Gamma_dc               (eq. nonlinear)
//   kCurl:         n_c = eps_cde Gamma_de                  (w |J| (curl u)_c)
//   kGradient:     n_c = Gamma_c0 (one input field s)      (w |J| (grad s)_c)
enum PointMode { kConvection = 0, kCurl = 1, kGradient = 2 };

// Convection term N(u) (eq. nonlinear) on the velocity space, and the equal-order weak
// curl and gradient of the projection step (Section 4.2), which share its stages: one
// gather and forward pass per input component (value and reference gradient from the
// same xi_1/xi_2 stages), the components' xi_3 lines held per thread, C read once per
// point, then the three outputs (member c of the velocity E-vector and of y; essential
// rows get nothing).  (For the convection term, two passes, values first and then per
// component its gradient, hold fewer registers but measured 441 vs 264 us at 32^3 p = 4
// and 620 vs 576 us at 24^3 p = 7.)
template <int P, bool POS, int MODE>
__device__ __forceinline__ void phi_test_body(const int32_t *__restrict__ vmap,
                                              const int32_t *__restrict__ vpos, int vcompact,
                                              const double *__restrict__ cq, int64_t nelem,
                                              const double *__restrict__ u, int64_t nv,
                                              double *__restrict__ Yv, int64_t vestride,
                                              double *__restrict__ yv) {
  using S = SDims<P>;
  using D = Dims<P>;
  constexpr int N = S::N, Q = S::Q, Q2 = S::Q2, Q3 = S::Q3, TPE = S::TPE, E = S::E;
  constexpr int N3 = N * N * N;
  constexpr int NIN = MODE == kGradient ? 1 : 3;
  using VB = TabEO<P, Q, 0>;
  using VG = TabEO<P, Q, 1>;
  __shared__ __align__(16) double smem[E * D::BUF];
  __shared__ int32_t smap_all[E * N3];
  const int le = threadIdx.x / TPE;
  const int t0 = threadIdx.x - le * TPE;
  const int e = xcd_block() * E + le;
  const bool active = e < nelem;
  const int es = active ? e : 0;
  double *buf = smem + le * D::BUF;
  int32_t *smap = smap_all + le * N3;
  const int32_t *emap = vmap + (int64_t)es * N3;
  // the input components' xi_3 lines (value and reference-gradient fields, even-odd
  // split), one gather and one forward pass each
  eo::Split<N, double> sbb[NIN], sgb[NIN], sbg[NIN];
#pragma unroll
  for (int r = 0; r < NIN; ++r) {
    gather_all<P>(buf, t0, active, emap, u + r * nv);
    fwd_grad_xy<P, Q>(buf, t0);
    double zb[N], zg[N], zx[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      zb[k] = buf[k * Q2 + t0];
      zg[k] = buf[N * Q2 + k * Q2 + t0];
      zx[k] = buf[2 * N * Q2 + k * Q2 + t0];
    }
    sbb[r] = eo::split(zb);
    sgb[r] = eo::split(zg);
    sbg[r] = eo::split(zx);
    __syncthreads();  // buf is reused by the next gather
  }
  const int64_t vepe = vcompact ? surf_count<P>() : N3;
  vel_entries<P, POS>(t0, emap, smap, POS ? vpos + (int64_t)es * vepe : nullptr, vcompact != 0);
  const double *ce = cq + (int64_t)es * (9 * Q3) + t0;
  // the three outputs at the points of the line
  double n[3][Q];
  auto point = [&](int c, const double (&uv)[NIN], const double (&g)[NIN][3]) {
    const double *cp = ce + cq_at<Q>(c, 0);
    double cm[9];
#pragma unroll
    for (int z = 0; z < 9; ++z) cm[z] = cp[z * Q2];
    // Gamma_dr = (C grad_ref u_r)_d
    auto gam = [&](int d, int r) {
      return cm[3 * d] * g[r][0] + cm[3 * d + 1] * g[r][1] + cm[3 * d + 2] * g[r][2];
    };
    if constexpr (MODE == kConvection) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) acc += uv[d] * gam(d, r);
        n[r][c] = acc;
      }
    } else if constexpr (MODE == kCurl) {
      n[0][c] = gam(1, 2) - gam(2, 1);
      n[1][c] = gam(2, 0) - gam(0, 2);
      n[2][c] = gam(0, 1) - gam(1, 0);
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) n[d][c] = gam(d, 0);
    }
  };
#pragma unroll
  for (int c = 0; c < Q / 2; ++c) {
    double u0[NIN], u1[NIN], g0[NIN][3], g1[NIN][3];
#pragma unroll
    for (int r = 0; r < NIN; ++r) {
      row_pair<VB>(sbb[r], c, u0[r], u1[r]);
      row_pair<VB>(sbg[r], c, g0[r][0], g1[r][0]);
      row_pair<VB>(sgb[r], c, g0[r][1], g1[r][1]);
      row_pair<VG>(sbb[r], c, g0[r][2], g1[r][2]);
    }
    point(c, u0, g0);
    point(Q - 1 - c, u1, g1);
  }
  if constexpr (Q % 2 == 1) {
    double um[NIN], gm[NIN][3];
#pragma unroll
    for (int r = 0; r < NIN; ++r) {
      um[r] = row_mid<VB>(sbb[r]);
      gm[r][0] = row_mid<VB>(sbg[r]);
      gm[r][1] = row_mid<VB>(sgb[r]);
      gm[r][2] = row_mid<VG>(sbb[r]);
    }
    point(Q / 2, um, gm);
  }
  // the three outputs
  bwd_mass<P, Q, 3>(buf, t0, n);
#pragma unroll
  for (int r = 0; r < 3; ++r)
    emit_e<P, double, false, POS>(buf + r * N3, t0, active, smap, u, es, vcompact != 0,
                                  Yv + r * vestride, yv + r * nv);
}

template <int P, bool POS>
__global__ void __launch_bounds__(Dims<P>::THREADS, SDims<P>::OCC)
convection_kernel(const int32_t *__restrict__ vmap, const int32_t *__restrict__ vpos,
                  int vcompact, const double *__restrict__ cq, int64_t nelem,
                  const double *__restrict__ u, int64_t nv, double *__restrict__ Yv,
                  int64_t vestride, double *__restrict__ yv) {
  phi_test_body<P, POS, kConvection>(vmap, vpos, vcompact, cq, nelem, u, nv, Yv, vestride, yv);
}

// Weak curl (MODE = kCurl) or weak gradient (MODE = kGradient) of the projection step.
template <int P, bool POS, int MODE>
__global__ void __launch_bounds__(Dims<P>::THREADS, SDims<P>::OCC)
weak_phi_kernel(const int32_t *__restrict__ vmap, const int32_t *__restrict__ vpos,
                int vcompact, const double *__restrict__ cq, int64_t nelem,
                const double *__restrict__ u, int64_t nv, double *__restrict__ Yv,
                int64_t vestride, double *__restrict__ yv) {
  phi_test_body<P, POS, MODE>(vmap, vpos, vcompact, cq, nelem, u, nv, Yv, vestride, yv);
}

// Transposed reference-gradient contraction: from the three channels v_k at the points
// of the thread's xi_3 line (the components of the field to be tested against the
// reference gradient d_ref_k phi), the element vector sum_Q sum_k d_ref_k phi_l(Q) v_k(Q)
// in buf[0 .. n^3).  Channel k carries G along xi_k and B along the other two directions.
template <int PO, int Q>
__device__ __forceinline__ void bwd_grad(double *buf, int t, const double (&v)[3][Q]) {
  constexpr int NO = PO + 1;
  constexpr int NQ2 = NO * Q * Q, N2Q = NO * NO * Q;
  using BT = TabEO<PO, Q, 0>;
  using GT = TabEO<PO, Q, 1>;
  // out[i] += sum_c T(c, i) in[c] for c over the q points (T = B or G)
  auto line = [](auto tag, const double (&in)[Q], eo::Acc<NO, double> &A) {
    using TB = decltype(tag);
#pragma unroll
    for (int c = 0; c < Q / 2; ++c) A.template add_pair<TB>(c, in[c], in[Q - 1 - c]);
    if constexpr (Q % 2 == 1) A.template add_mid<TB>(in[Q / 2]);
  };
  {  // xi_3: channels 0, 1 with B, channel 2 with G: [c] -> [k][b][a]
    double r[3][NO];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      eo::Acc<NO, double> A;
      A.zero();
      if (f == 2) line(GT{}, v[f], A);
      else line(BT{}, v[f], A);
      A.finish(r[f]);
    }
    __syncthreads();
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
      for (int k = 0; k < NO; ++k) buf[f * NQ2 + k * Q * Q + t] = r[f][k];
    __syncthreads();
  }
  {  // xi_2: [k][b][a] -> [k][j][a]; s0 = B^T ch0 (G along xi_1 pending), s1 = G^T ch1 + B^T ch2
    const bool w = t < Q * NO;
    const int a = t % Q, k = t / Q;
    double r[2][NO];
    if (w) {
      double in0[Q], in1[Q], in2[Q];
#pragma unroll
      for (int b = 0; b < Q; ++b) {
        in0[b] = buf[(k * Q + b) * Q + a];
        in1[b] = buf[NQ2 + (k * Q + b) * Q + a];
        in2[b] = buf[2 * NQ2 + (k * Q + b) * Q + a];
      }
      eo::Acc<NO, double> A0, A1;
      A0.zero();
      A1.zero();
      line(BT{}, in0, A0);
      line(GT{}, in1, A1);
      line(BT{}, in2, A1);
      A0.finish(r[0]);
      A1.finish(r[1]);
    }
    __syncthreads();
    if (w) {
#pragma unroll
      for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int j = 0; j < NO; ++j) buf[f * N2Q + (k * NO + j) * Q + a] = r[f][j];
    }
    __syncthreads();
  }
  {  // xi_1: [k][j][a] -> [k][j][i]; out = G^T s0 + B^T s1
    const bool w = t < NO * NO;
    const int j = t % NO, k = t / NO;
    double r[NO];
    if (w) {
      double in0[Q], in1[Q];
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        in0[a] = buf[(k * NO + j) * Q + a];
        in1[a] = buf[N2Q + (k * NO + j) * Q + a];
      }
      eo::Acc<NO, double> A;
      A.zero();
      line(GT{}, in0, A);
      line(BT{}, in1, A);
      A.finish(r);
    }
    __syncthreads();
    if (w) {
#pragma unroll
      for (int i = 0; i < NO; ++i) buf[(k * NO + j) * NO + i] = r[i];
    }
    __syncthreads();
  }
}

// Weak divergence of a nodal vector field V (the pressure right-hand side of the
// projection step, Section 4.2): r_l = sum_Q w |J| grad phi_l . V = sum_Q
// grad_ref phi_l . (C^T V) with C = w |J| J^{-T}.  The three components are gathered
// and interpolated (values only), C^T V is formed per point, and one backward
// reference-gradient pass gives the single output (member 0 of the E-vector and of y).
template <int P, bool POS>
__global__ void __launch_bounds__(Dims<P>::THREADS, SDims<P>::OCC)
weak_div_kernel(const int32_t *__restrict__ vmap, const int32_t *__restrict__ vpos,
                int vcompact, const double *__restrict__ cq, int64_t nelem,
                const double *__restrict__ u, int64_t nv, double *__restrict__ Yv,
                double *__restrict__ yv) {
  using S = SDims<P>;
  using D = Dims<P>;
  constexpr int N = S::N, Q = S::Q, Q2 = S::Q2, Q3 = S::Q3, TPE = S::TPE, E = S::E;
  constexpr int N3 = N * N * N;
  using VB = TabEO<P, Q, 0>;
  __shared__ __align__(16) double smem[E * D::BUF];
  __shared__ int32_t smap_all[E * N3];
  const int le = threadIdx.x / TPE;
  const int t0 = threadIdx.x - le * TPE;
  const int e = xcd_block() * E + le;
  const bool active = e < nelem;
  const int es = active ? e : 0;
  double *buf = smem + le * D::BUF;
  int32_t *smap = smap_all + le * N3;
  const int32_t *emap = vmap + (int64_t)es * N3;
  eo::Split<N, double> sv[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    gather_all<P>(buf, t0, active, emap, u + r * nv);
    fwd_val_xy<P, Q>(buf, t0);
    double z[N];
#pragma unroll
    for (int k = 0; k < N; ++k) z[k] = buf[k * Q2 + t0];
    sv[r] = eo::split(z);
    __syncthreads();
  }
  const int64_t vepe = vcompact ? surf_count<P>() : N3;
  vel_entries<P, POS>(t0, emap, smap, POS ? vpos + (int64_t)es * vepe : nullptr, vcompact != 0);
  const double *ce = cq + (int64_t)es * (9 * Q3) + t0;
  double h[3][Q];  // (C^T V)_k at the points of the line
  auto point = [&](int c, const double (&vv)[3]) {
    const double *cp = ce + cq_at<Q>(c, 0);
    double cm[9];
#pragma unroll
    for (int z = 0; z < 9; ++z) cm[z] = cp[z * Q2];
#pragma unroll
    for (int k = 0; k < 3; ++k) h[k][c] = cm[k] * vv[0] + cm[3 + k] * vv[1] + cm[6 + k] * vv[2];
  };
#pragma unroll
  for (int c = 0; c < Q / 2; ++c) {
    double v0[3], v1[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) row_pair<VB>(sv[r], c, v0[r], v1[r]);
    point(c, v0);
    point(Q - 1 - c, v1);
  }
  if constexpr (Q % 2 == 1) {
    double vm[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) vm[r] = row_mid<VB>(sv[r]);
    point(Q / 2, vm);
  }
  bwd_grad<P, Q>(buf, t0, h);
  emit_e<P, double, false, POS>(buf, t0, active, smap, u, es, vcompact != 0, Yv, yv);
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

template <int P>
hipError_t launch_convection_pt(const ConvArgs &a, hipStream_t s) {
  using D = Dims<P>;
  if (a.nelem <= 0) return hipSuccess;
  constexpr bool POS = evec_dof_ordered(P);
  if ((a.vpos != nullptr) != POS) return hipErrorInvalidValue;
  dim3 grid((unsigned)((a.nelem + D::E - 1) / D::E));
  dim3 block(D::THREADS);
  switch (a.kind) {
    case kWeakConvection:
      hipLaunchKernelGGL((convection_kernel<P, POS>), grid, block, 0, s, a.vmap, a.vpos,
                         a.vcompact, a.cq, a.nelem, a.u, a.nv, a.Yv, a.vestride, a.yv);
      break;
    case kWeakCurl:
      hipLaunchKernelGGL((weak_phi_kernel<P, POS, kCurl>), grid, block, 0, s, a.vmap, a.vpos,
                         a.vcompact, a.cq, a.nelem, a.u, a.nv, a.Yv, a.vestride, a.yv);
      break;
    case kWeakGradient:
      hipLaunchKernelGGL((weak_phi_kernel<P, POS, kGradient>), grid, block, 0, s, a.vmap, a.vpos,
                         a.vcompact, a.cq, a.nelem, a.u, a.nv, a.Yv, a.vestride, a.yv);
      break;
    case kWeakDivergence:
      hipLaunchKernelGGL((weak_div_kernel<P, POS>), grid, block, 0, s, a.vmap, a.vpos, a.vcompact,
                         a.cq, a.nelem, a.u, a.nv, a.Yv, a.yv);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
lincomb_kernel(LinComb lc, const double *__restrict__ scale, const uint8_t *__restrict__ mask,
               double *y, int64_t n, int64_t total) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256) {
    double v = 0.0;
    for (int j = 0; j < lc.nterm; ++j) v += lc.c[j] * lc.x[j][i];
    const int64_t g = i % n;
    if (scale) v /= scale[g];
    if (mask && mask[g]) v = 0.0;
    y[i] = v;
  }
}

}  // namespace

hipError_t launch_stokes(const StokesArgs &a, hipStream_t s) {
#define SFEM_CALL(P) launch_stokes_pt<P>(a, s)
  SFEM_DISPATCH_P(a.p, SFEM_CALL)
#undef SFEM_CALL
}

hipError_t launch_convection(const ConvArgs &a, hipStream_t s) {
#define SFEM_CALL(P) launch_convection_pt<P>(a, s)
  SFEM_DISPATCH_P(a.p, SFEM_CALL)
#undef SFEM_CALL
}

hipError_t launch_lincomb(const LinComb &lc, const double *scale, const uint8_t *mask, double *y,
                          int64_t n, int nb, hipStream_t s) {
  const int64_t total = n * nb;
  if (total <= 0) return hipSuccess;
  if (lc.nterm < 1 || lc.nterm > kMaxLinTerms) return hipErrorInvalidValue;
  int64_t blocks = (total + 1023) / 1024;
  if (blocks > 65535) blocks = 65535;
  hipLaunchKernelGGL(lincomb_kernel, dim3((unsigned)blocks), dim3(256), 0, s, lc, scale, mask, y, n,
                     total);
  return hipGetLastError();
}

}  // namespace sfem
