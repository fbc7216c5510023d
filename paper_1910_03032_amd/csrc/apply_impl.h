// Sum-factorized element kernels for Q_p hexahedra on gfx950.
//
// Per element (Section 3.1, eq. sumFactorized and L^K = G^T W G):
//   gather x_e -> contract xi_1 with B, G -> contract xi_2 -> contract xi_3
//   -> pointwise quadrature function with the stored factors
//      (v = m u,  g = Gq grad_ref u)
//   -> transposed contractions xi_3 -> xi_2 -> xi_1 -> scatter into y.
//
// Work decomposition: one element is owned by q^2 threads; in every stage a thread
// owns one 1D line of the tensor along the direction being contracted, holds the
// n (or q) inputs of that line in registers and produces the whole output line, so
// LDS is read once per input value.  The 1D tables are compile-time constants and
// every contraction uses their symmetry (even-odd form: the nodes and the Gauss
// points are symmetric about 0, so B is centro-symmetric and G centro-antisymmetric),
// which halves the multiply-adds; the xi_3 stage walks the quadrature slices in
// symmetric pairs (c, q-1-c).  Intermediates between stages live in LDS, one buffer
// per element.  Several (element, batch member) pairs share a workgroup (E = 256 / q^2),
// the members of an element next to each other, so that a batched apply reads each
// element's quadrature data from HBM once for all members.
//
// Assembly (no atomics, deterministic): one launch of the element kernel covers every
// element.  A DoF that belongs to this element only (the element-interior nodes of a
// conforming mesh) is written straight to y.  The value of a shared node (element
// surface) goes to its own entry of the E-vector, which is ordered by destination DoF
// (the entry comes from a position table read with the map); an assembly kernel then
// gives each shared DoF to one thread, which sums its contiguous E-vector entries in
// element order (owner computes) -- and sets the essential DoFs.
// Workgroups are mapped to elements so that each of the 8 XCDs works on one
// contiguous range of elements, which keeps the x values shared by neighbouring
// elements in that XCD's L2.
//
// LDS layouts inside an element buffer (a, b, c: quadrature indices along
// xi_1..3; i, j, k: node indices):
//   nodal         [k][j][i]
//   after xi_1    [k][j][a]      (two fields: B- and G-contracted)
//   after xi_2    [k][b][a]      (three fields)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eo.h"
#include "internal.h"
#include "rules.h"

namespace sfem {

template <int P>
struct Dims {
  static constexpr int N = P + 1, Q = P + 2;
  static constexpr int N2 = N * N, N3 = N * N * N, Q2 = Q * Q, Q3 = Q * Q * Q;
  static constexpr int QN2 = Q * N2, NQ2 = N * Q2;
  static constexpr int TPE = Q2;  // threads per element
  static constexpr int E = (256 / TPE) > 0 ? (256 / TPE) : 1;
  static constexpr int mx(int a, int b) { return a > b ? a : b; }
  static constexpr int BUF = mx(N3, mx(2 * Q * N2, 3 * Q2 * N));
  static constexpr int THREADS = E * TPE;
  // minimum waves per SIMD the element kernels are compiled for: the largest that
  // the Helmholtz kernels reach without spilling registers (p = 8 spills slightly)
  static constexpr int OCC = P <= 2 ? 4 : (P <= 4 ? 3 : 2);
};

// The 1D tables as compile-time constants of the order P (q = P + 2): after loop
// unrolling every table entry is a literal, so no table lives in registers or memory.
template <int P, typename T>
struct Tab {
  static constexpr rules::Tables<P, P + 2> c = rules::tables<P, P + 2>();
  __host__ __device__ static constexpr T B(int a, int i) { return (T)c.B[a][i]; }
  __host__ __device__ static constexpr T G(int a, int i) { return (T)c.G[a][i]; }
};

// Local nodes one thread handles in the gather and output loops (l = t + k TPE).
template <int P>
struct Per {
  static constexpr int NL = (Dims<P>::N3 + Dims<P>::TPE - 1) / Dims<P>::TPE;
};

// Rank of local node l among the element's surface nodes (a node with i, j or k in
// {0, p}): face k = 0, face k = p, then for each interior k the ring of the (i, j)
// square; -1 for an interior node.  The ranks of all local nodes of order P form a
// table in constant memory: one 2-byte load per node instead of index arithmetic.
template <int P>
struct RankTable {
  int16_t r[(P + 1) * (P + 1) * (P + 1)];
};
template <int P>
constexpr RankTable<P> make_rank_table() {
  RankTable<P> t{};
  constexpr int N = P + 1;
  for (int l = 0; l < N * N * N; ++l) {
    const int i = l % N, j = (l / N) % N, k = l / (N * N);
    int r = -1;
    if (k == 0) {
      r = i + N * j;
    } else if (k == P) {
      r = N * N + i + N * j;
    } else {
      const int base = 2 * N * N + (k - 1) * 4 * P;
      if (j == 0)
        r = base + i;
      else if (j == P)
        r = base + N + i;
      else if (i == 0 || i == P)
        r = base + 2 * N + 2 * (j - 1) + (i == 0 ? 0 : 1);
    }
    t.r[l] = (int16_t)r;
  }
  return t;
}
template <int P>
__constant__ RankTable<P> kRankTable = make_rank_table<P>();
template <int P>
__device__ __forceinline__ int surf_rank(int l) {
  return kRankTable<P>.r[l];
}
template <int P>
__host__ __device__ constexpr int surf_count() {
  return 2 * (P + 1) * (P + 1) + (P - 1) * 4 * P;
}

// Gather the element's nodal values (essential DoFs as 0) into buf[k][j][i].  All map
// loads of the thread are issued together, then all value loads.  Loads are
// unconditional (an inactive slot reads a valid element's entries and discards them)
// so that the compiler can batch them.  If smap is given (LDS), it receives each
// node's map entry -- except, with POS (DoF-ordered E-vector), that a shared node gets
// its E-vector entry from the element's row epos of the position table, read together
// with the map.
template <int P, typename T, bool POS = false>
__device__ __forceinline__ void gather_e(T *buf, int t, bool active, const int32_t *emap,
                                         const T *__restrict__ xm, int32_t *smap = nullptr,
                                         const int32_t *epos = nullptr, bool compact = true) {
  using D = Dims<P>;
  constexpr int NL = Per<P>::NL;
  int32_t c[NL], q[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int l0 = t + k * D::TPE;
    const int l = l0 < D::N3 ? l0 : D::N3 - 1;
    c[k] = emap[l];
    if constexpr (POS) {
      const int r = compact ? surf_rank<P>(l) : l;
      q[k] = epos[r >= 0 ? r : 0];
    }
  }
  T v[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) v[k] = xm[c[k] & kDofMask];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int l = t + k * D::TPE;
    if (l < D::N3) {
      buf[l] = (active && c[k] >= 0) ? v[k] : T(0);
      if (smap) {
        if constexpr (POS)
          smap[l] = (c[k] >= 0 && !(c[k] & kSoleBit)) ? q[k] : c[k];
        else
          smap[l] = c[k];
      }
    }
  }
  __syncthreads();
}

// Output of the element vector buf[l] of element e: sole DoFs -> y, shared nodes ->
// their E-vector entry (POS: the entry kept in smap by the gather; otherwise e * S + the
// node's surface rank, or e * n^3 + l for the general layout), essential -> nothing.
// The map entries come from LDS, kept by the gather.  With DOT, returns this thread's
// part of sum x_g y_g over the sole DoFs (x read again from xm).
template <int P, typename T, bool DOT, bool POS>
__device__ __forceinline__ double emit_e(const T *buf, int t, bool active, const int32_t *smap,
                                         const T *__restrict__ xm, int64_t e, bool compact,
                                         T *__restrict__ Y, T *__restrict__ y) {
  using D = Dims<P>;
  constexpr int NL = Per<P>::NL;
  double dot = 0.0;
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int l0 = t + k * D::TPE;
    const int l = l0 < D::N3 ? l0 : D::N3 - 1;
    const int32_t c = smap[l];
    const T v = buf[l];
    // one predicated store per node: the destination is selected, not branched to
    const bool ok = active && l0 < D::N3 && c >= 0;
    const bool sole = (c & kSoleBit) != 0;
    const int32_t g = c & kDofMask;
    int64_t ye;
    if constexpr (POS)
      ye = c;
    else
      ye = compact ? e * surf_count<P>() + surf_rank<P>(l) : e * D::N3 + l;
    T *dst = sole ? y + g : Y + ye;
    if (ok) *dst = v;
    if constexpr (DOT) {
      const T xv = xm[sole ? g : 0];  // in range for every entry
      if (ok && sole) dot += (double)xv * (double)v;
    }
  }
  return dot;
}

// Deterministic block sum, result on thread 0.  Every thread stores its value in LDS
// (sh holds blockDim.x entries); the lanes of wave 0 each add a fixed strided subset,
// then a wave64 butterfly.  Only values of existing threads are read, so a block whose
// size is not a multiple of 64 needs no special case.
__device__ __forceinline__ double block_sum_d(double v, double *sh) {
  __syncthreads();
  sh[threadIdx.x] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < 64) {
    for (int i = threadIdx.x; i < (int)blockDim.x; i += 64) s += sh[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  }
  return s;
}

// xi_1 contraction: [k][j][i] -> [k][j][a] with B (field 0) and, if DIFF, G (field 1).
template <int P, typename T, bool DIFF>
__device__ __forceinline__ void fwd_x(T *buf, int t) {
  using D = Dims<P>;
  constexpr int N = D::N, Q = D::Q;
  const bool w = t < D::N2;
  const int j = t % N, k = t / N;
  T ob[Q], og[Q];
  if (w) {
    T in[N];
#pragma unroll
    for (int i = 0; i < N; ++i) in[i] = buf[(k * N + j) * N + i];
    const auto sp = eo::split(in);
    eo::apply<eo::Tab1<P, 0>>(sp, ob);
    if constexpr (DIFF) eo::apply<eo::Tab1<P, 1>>(sp, og);
  }
  __syncthreads();
  if (w) {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      buf[(k * N + j) * Q + a] = ob[a];
      if constexpr (DIFF) buf[D::QN2 + (k * N + j) * Q + a] = og[a];
    }
  }
  __syncthreads();
}

// xi_2 contraction: [k][j][a] -> [k][b][a]: field 0 = B(B x), and if DIFF
// field 1 = G_y(B_x x) (for d/dxi_2), field 2 = B_y(G_x x) (for d/dxi_1).
template <int P, typename T, bool DIFF>
__device__ __forceinline__ void fwd_y(T *buf, int t) {
  using D = Dims<P>;
  constexpr int N = D::N, Q = D::Q;
  const bool w = t < Q * N;
  const int a = t % Q, k = t / Q;
  T obb[Q], ogb[Q], obg[Q];
  if (w) {
    T ib[N], ig[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      ib[j] = buf[(k * N + j) * Q + a];
      if constexpr (DIFF) ig[j] = buf[D::QN2 + (k * N + j) * Q + a];
    }
    const auto sb = eo::split(ib);
    eo::apply<eo::Tab1<P, 0>>(sb, obb);
    if constexpr (DIFF) {
      eo::apply<eo::Tab1<P, 1>>(sb, ogb);
      eo::apply<eo::Tab1<P, 0>>(eo::split(ig), obg);
    }
  }
  __syncthreads();
  if (w) {
#pragma unroll
    for (int b = 0; b < Q; ++b) {
      buf[(k * Q + b) * Q + a] = obb[b];
      if constexpr (DIFF) {
        buf[D::NQ2 + (k * Q + b) * Q + a] = ogb[b];
        buf[2 * D::NQ2 + (k * Q + b) * Q + a] = obg[b];
      }
    }
  }
  __syncthreads();
}

// Read the xi_3 lines of thread t = a + q b (no barrier).
template <int P, typename T, bool DIFF>
__device__ __forceinline__ void load_z(const T *buf, int t, T (&zbb)[P + 1], T (&zgb)[P + 1],
                                       T (&zbg)[P + 1]) {
  using D = Dims<P>;
#pragma unroll
  for (int k = 0; k < D::N; ++k) {
    zbb[k] = buf[k * D::Q2 + t];
    if constexpr (DIFF) {
      zgb[k] = buf[D::NQ2 + k * D::Q2 + t];
      zbg[k] = buf[2 * D::NQ2 + k * D::Q2 + t];
    }
  }
}

// Transposed xi_2: [k][b][a] (fields p1, p2, p3) -> [k][j][a] (fields r1, r2) with
// r1 = B^T p1 + G^T p2 and r2 = B^T p3.
template <int P, typename T, bool DIFF>
__device__ __forceinline__ void bwd_y(T *buf, int t) {
  using D = Dims<P>;
  using BT = eo::Tab1<P, 0>;
  using GT = eo::Tab1<P, 1>;
  constexpr int N = D::N, Q = D::Q;
  const bool w = t < Q * N;
  const int a = t % Q, k = t / Q;
  T r1[N], r2[N];
  if (w) {
    T i1[Q], i2[Q], i3[Q];
#pragma unroll
    for (int b = 0; b < Q; ++b) {
      i1[b] = buf[(k * Q + b) * Q + a];
      if constexpr (DIFF) {
        i2[b] = buf[D::NQ2 + (k * Q + b) * Q + a];
        i3[b] = buf[2 * D::NQ2 + (k * Q + b) * Q + a];
      }
    }
    eo::Acc<N, T> A1, A2;
    A1.zero();
    A2.zero();
#pragma unroll
    for (int b = 0; b < Q / 2; ++b) {
      A1.template add_pair<BT>(b, i1[b], i1[Q - 1 - b]);
      if constexpr (DIFF) {
        A1.template add_pair<GT>(b, i2[b], i2[Q - 1 - b]);
        A2.template add_pair<BT>(b, i3[b], i3[Q - 1 - b]);
      }
    }
    if constexpr (Q % 2 == 1) {
      A1.template add_mid<BT>(i1[Q / 2]);
      if constexpr (DIFF) {
        A1.template add_mid<GT>(i2[Q / 2]);
        A2.template add_mid<BT>(i3[Q / 2]);
      }
    }
    A1.finish(r1);
    if constexpr (DIFF) A2.finish(r2);
  }
  __syncthreads();
  if (w) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      buf[(k * N + j) * Q + a] = r1[j];
      if constexpr (DIFF) buf[D::QN2 + (k * N + j) * Q + a] = r2[j];
    }
  }
  __syncthreads();
}

// Transposed xi_1: [k][j][a] (r1, r2) -> nodal [k][j][i] = B^T r1 + G^T r2.
template <int P, typename T, bool DIFF>
__device__ __forceinline__ void bwd_x(T *buf, int t) {
  using D = Dims<P>;
  using BT = eo::Tab1<P, 0>;
  using GT = eo::Tab1<P, 1>;
  constexpr int N = D::N, Q = D::Q;
  const bool w = t < D::N2;
  const int j = t % N, k = t / N;
  T yo[N];
  if (w) {
    T i1[Q], i2[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      i1[a] = buf[(k * N + j) * Q + a];
      if constexpr (DIFF) i2[a] = buf[D::QN2 + (k * N + j) * Q + a];
    }
    eo::Acc<N, T> A;
    A.zero();
#pragma unroll
    for (int a = 0; a < Q / 2; ++a) {
      A.template add_pair<BT>(a, i1[a], i1[Q - 1 - a]);
      if constexpr (DIFF) A.template add_pair<GT>(a, i2[a], i2[Q - 1 - a]);
    }
    if constexpr (Q % 2 == 1) {
      A.template add_mid<BT>(i1[Q / 2]);
      if constexpr (DIFF) A.template add_mid<GT>(i2[Q / 2]);
    }
    A.finish(yo);
  }
  __syncthreads();
  if (w) {
#pragma unroll
    for (int i = 0; i < N; ++i) buf[(k * N + j) * N + i] = yo[i];
  }
  __syncthreads();
}

// Index of the element batch of this workgroup such that XCD k (workgroups are
// dispatched round-robin over the 8 XCDs) gets one contiguous range of batches.
__device__ __forceinline__ int xcd_block() {
  const unsigned nblk = gridDim.x, b = blockIdx.x;
  const unsigned xcd = b & 7u, k = b >> 3;
  const unsigned q8 = nblk >> 3, r8 = nblk & 7u;
  return (int)(xcd * q8 + (xcd < r8 ? xcd : r8) + k);
}

// How the element kernel of order P and precision T feeds its xi_3 stage (chosen by
// measurement on MI355X, see the design notes):
//   ZLDS   the stage's input lines are read from LDS again for every slice pair instead
//          of being held in registers for the whole stage (fewer registers);
//   PRE_X, PRE_Y  slice pairs [0, PRE_X) of quadrature data are requested before the
//          xi_1 contraction and [PRE_X, PRE_Y) before the xi_2 contraction;
//   LA     in the xi_3 loop, pair c + LA is requested when pair c starts;
//   OCC    minimum waves per SIMD the kernel is compiled for (launch bound);
//   E      elements per workgroup (q^2 threads each).
template <int P, typename T>
struct ApplyCfg {
  static constexpr bool F64 = sizeof(T) == 8;
  // (p = 8 with 5 elements per workgroup, 500 of 512 lanes busy instead of 200 of 256,
  // measured 4 % slower in FP64: one workgroup per CU at its register count)
  static constexpr int E = Dims<P>::E;
  static constexpr int THREADS = E * Dims<P>::TPE;
  static constexpr bool ZLDS = F64 ? (P >= 5) : (P == 6 || P == 8);
  // (p = 4, FP64: slice pair 0 requested before the xi_1 stage, pair 1 before xi_2, pair 2
  // when the xi_3 loop starts; 2 % faster than one pair ahead with the factors stored by
  // slice pair)
  static constexpr bool AHEAD = F64 ? (P == 8 || P == 4) : (P == 6 || P == 8);
  static constexpr int PRE_X = AHEAD ? 1 : 0, PRE_Y = (P == 4) ? 2 : 1, LA = AHEAD ? 1 : 0;
  static constexpr int OCC = Dims<P>::OCC;
};

// OP: 0 mass, 1 diffusion, 2 helmholtz (matches sfem_op).  Writes y at the sole DoFs
// and the E-vector Y[m] at the shared nodes; with part != null also the per-block sums
// of x_g y_g over the sole DoFs (part[m * part_mstride + block], 0 for a member with no
// element in the block).
//
// Work items are (element, member) pairs, pair v = e * nbatch + m, E per workgroup: the
// members of one element run side by side (in the same workgroup or in neighbouring
// ones, on one XCD) and read the element's quadrature data, which all members share
// unless qd_mstride != 0, from the same cache lines, so that it comes from HBM once for
// all members.
template <int P, typename T, int OP>
__global__ void __launch_bounds__((ApplyCfg<P, T>::THREADS), (ApplyCfg<P, T>::OCC))
apply_kernel(const int32_t *__restrict__ map, const T *__restrict__ qd,
             int64_t qd_mstride, const T *__restrict__ nu, int64_t nu_mstride, int64_t nelem,
             int nbatch, int64_t ndof, const T *__restrict__ x, T *__restrict__ Y,
             int64_t estride, const int32_t *__restrict__ pos, int compact, T *__restrict__ y,
             double *__restrict__ part,
             int64_t part_mstride) {
  using D = Dims<P>;
  constexpr int N = D::N, Q = D::Q, Q2 = D::Q2, Q3 = D::Q3, N3 = D::N3;
  constexpr int TPE = D::TPE, E = ApplyCfg<P, T>::E, THREADS = ApplyCfg<P, T>::THREADS;
  constexpr bool MASS = (OP == 0) || (OP == 2);
  constexpr bool DIFF = (OP == 1) || (OP == 2);

  constexpr bool POS = evec_dof_ordered(P);
  // element buffers; after the output step also the block sum of the fused dot product
  // (E * BUF * sizeof(T) >= THREADS * 8 bytes)
  static_assert(E * D::BUF * sizeof(T) >= THREADS * sizeof(double), "block sum space");
  __shared__ __align__(16) T smem[E * D::BUF];
  __shared__ int32_t smap_all[E * N3];  // the elements' map entries, kept for the output
  const int le = threadIdx.x / TPE;
  const int t = threadIdx.x - le * TPE;
  // the grid has one workgroup per E (element, member) pairs (nelem * nbatch pairs)
  const int64_t npair = nelem * (int64_t)nbatch;
  const int64_t v = (int64_t)xcd_block() * E + le;
  const bool active = v < npair;
  const int64_t vs = active ? v : 0;
  const int es = (int)(vs / nbatch);
  const int m = (int)(vs - (int64_t)es * nbatch);
  T *buf = smem + le * D::BUF;

  // Quadrature values one thread needs per slice c: w|J| (mass), the 6 entries of
  // w|J| J^-1 J^-T (diffusion), and nu for the diffusion operator.
  constexpr int NS = (OP == 0) ? 1 : (OP == 2 ? 7 : 7);
  {
    const T *xm = x + (int64_t)m * ndof;
    const T *qe = qd + (int64_t)m * qd_mstride + es * (int64_t)(kQdSlots * Q3);
    const T *ne = nullptr;
    if constexpr (OP == 1) ne = nu + (int64_t)m * nu_mstride + es * (int64_t)Q3;
    // (inactive slots read element 0's data, which is discarded)
    auto load_slice = [&](T (&dst)[NS], int c) {
      const int qi = c * Q2 + t;
      if constexpr (OP == 0) {
        dst[0] = qe[qi];
      } else if constexpr (OP == 2) {
        // the folded factors are stored by slice pair, then slice, then slot
        const int pc = c <= Q - 1 - c ? c : Q - 1 - c;
        const int base = (2 * pc + (c > Q - 1 - c ? 1 : 0)) * 7 * Q2 + t;
#pragma unroll
        for (int s = 0; s < 7; ++s) dst[s] = qe[base + s * Q2];
      } else {
#pragma unroll
        for (int s = 0; s < 6; ++s) dst[s] = qe[(s + 1) * Q3 + qi];
        dst[6] = ne[qi];
      }
    };

    int32_t *smap = smap_all + le * N3;
    const int64_t moff = (int64_t)es * N3;
    const int64_t epe = compact ? surf_count<P>() : N3;
    gather_e<P, T, POS>(buf, t, active, map + moff, xm, smap,
                        POS ? pos + (int64_t)es * epe : nullptr, compact != 0);
    // quadrature data of slice pair c (slices c and q-1-c; the middle slice of an odd q
    // alone), requested ahead of use as ApplyCfg sets
    using C = ApplyCfg<P, T>;
    constexpr int NPR = (Q + 1) / 2;
    constexpr int PRE_X = C::PRE_X < NPR ? C::PRE_X : NPR;
    constexpr int PRE_Y = C::PRE_Y < NPR ? C::PRE_Y : NPR;
    T qlo[NPR][NS], qhi[NPR][NS];
    auto load_pair = [&](int c) {
      load_slice(qlo[c], c);
      if (c != Q - 1 - c) load_slice(qhi[c], Q - 1 - c);
    };
#pragma unroll
    for (int c = 0; c < PRE_X; ++c) load_pair(c);
    fwd_x<P, T, DIFF>(buf, t);
#pragma unroll
    for (int c = PRE_X; c < PRE_Y; ++c) load_pair(c);
    fwd_y<P, T, DIFF>(buf, t);

    // xi_3 contraction, quadrature function, transposed xi_3: thread = line (a, b),
    // processed by symmetric slice pairs (c, q-1-c).
    {
      using BT = eo::Tab1<P, 0>;
      using GT = eo::Tab1<P, 1>;
      // the stage's input lines (split into even and odd parts), held in registers or,
      // with ZLDS, read from LDS again for every slice pair
      eo::Split<N, T> rbb{}, rgb{}, rbg{};
      auto read_lines = [&](eo::Split<N, T> &sbb, eo::Split<N, T> &sgb, eo::Split<N, T> &sbg) {
        T zbb[N], zgb[N], zbg[N];
        load_z<P, T, DIFF>(buf, t, zbb, zgb, zbg);
        sbb = eo::split(zbb);
        if constexpr (DIFF) {
          sgb = eo::split(zgb);
          sbg = eo::split(zbg);
        }
      };
      if constexpr (!C::ZLDS) read_lines(rbb, rgb, rbg);
      auto zlines = [&](eo::Split<N, T> &sbb, eo::Split<N, T> &sgb, eo::Split<N, T> &sbg) {
        if constexpr (C::ZLDS) {
          asm volatile("" ::: "memory");  // a fresh LDS read, not a reuse of the last one
          read_lines(sbb, sgb, sbg);
        } else {
          sbb = rbb;
          sgb = rgb;
          sbg = rbg;
        }
      };
      eo::Acc<N, T> A1, A2, A3;
      A1.zero();
      A2.zero();
      A3.zero();
      auto row_pair = [](auto tb, const eo::Split<N, T> &x, int c, T &lo, T &hi) {
        using TT = decltype(tb);
        T Ev = 0, Od = 0;
#pragma unroll
        for (int i = 0; i < N / 2; ++i) {
          Ev += (T)TT::e(c, i) * x.e[i];
          Od += (T)TT::o(c, i) * x.o[i];
        }
        if constexpr (N % 2 == 1) Ev += (T)TT::t(c, N / 2) * x.e[N / 2];
        lo = Ev + Od;
        hi = (TT::S > 0) ? (Ev - Od) : (Od - Ev);
      };
      auto row_mid = [](auto tb, const eo::Split<N, T> &x) -> T {
        using TT = decltype(tb);
        T M = 0;
#pragma unroll
        for (int i = 0; i < N / 2; ++i) M += (T)TT::t(Q / 2, i) * (TT::S > 0 ? x.e[i] : x.o[i]);
        if constexpr (N % 2 == 1 && TT::S > 0) M += (T)TT::t(Q / 2, N / 2) * x.e[N / 2];
        return M;
      };
      auto qfun = [&](int c, T u, T dx, T dy, T dz, T &v, T &g1, T &g2, T &g3) {
        T cur[NS];
        const int pc = c <= Q - 1 - c ? c : Q - 1 - c;  // the slice's pair
        if (C::LA == 0 && pc >= PRE_Y) {
          load_slice(cur, c);  // not requested ahead: load at its use
        } else {
#pragma unroll
          for (int z = 0; z < NS; ++z) cur[z] = (c == pc) ? qlo[pc][z] : qhi[pc][z];
        }
        v = g1 = g2 = g3 = T(0);
        if constexpr (MASS) v = cur[0] * u;
        if constexpr (DIFF) {
          constexpr int o = MASS ? 1 : 0;
          const T G11 = cur[o + 0], G22 = cur[o + 1], G33 = cur[o + 2];
          const T G12 = cur[o + 3], G13 = cur[o + 4], G23 = cur[o + 5];
          g1 = G11 * dx + G12 * dy + G13 * dz;
          g2 = G12 * dx + G22 * dy + G23 * dz;
          g3 = G13 * dx + G23 * dy + G33 * dz;
          if constexpr (OP == 1) {
            g1 *= cur[NS - 1];
            g2 *= cur[NS - 1];
            g3 *= cur[NS - 1];
          }
        }
      };
#pragma unroll
      for (int c = 0; c < Q / 2; ++c) {
        if (C::LA > 0 && c + C::LA >= PRE_Y && c + C::LA < NPR) load_pair(c + C::LA);
        T u0 = 0, u1 = 0, dx0 = 0, dx1 = 0, dy0 = 0, dy1 = 0, dz0 = 0, dz1 = 0;
        eo::Split<N, T> sbb, sgb, sbg;
        zlines(sbb, sgb, sbg);
        if constexpr (MASS) row_pair(BT{}, sbb, c, u0, u1);
        if constexpr (DIFF) {
          row_pair(GT{}, sbb, c, dz0, dz1);
          row_pair(BT{}, sgb, c, dy0, dy1);
          row_pair(BT{}, sbg, c, dx0, dx1);
        }
        T v0, g10, g20, g30, v1, g11, g21, g31;
        qfun(c, u0, dx0, dy0, dz0, v0, g10, g20, g30);
        qfun(Q - 1 - c, u1, dx1, dy1, dz1, v1, g11, g21, g31);
        if constexpr (MASS) A1.template add_pair<BT>(c, v0, v1);
        if constexpr (DIFF) {
          A1.template add_pair<GT>(c, g30, g31);
          A2.template add_pair<BT>(c, g20, g21);
          A3.template add_pair<BT>(c, g10, g11);
        }
      }
      if constexpr (Q % 2 == 1) {
        T u = 0, dx = 0, dy = 0, dz = 0;
        eo::Split<N, T> sbb, sgb, sbg;
        zlines(sbb, sgb, sbg);
        if constexpr (MASS) u = row_mid(BT{}, sbb);
        if constexpr (DIFF) {
          dz = row_mid(GT{}, sbb);
          dy = row_mid(BT{}, sgb);
          dx = row_mid(BT{}, sbg);
        }
        T v, g1, g2, g3;
        qfun(Q / 2, u, dx, dy, dz, v, g1, g2, g3);
        if constexpr (MASS) A1.template add_mid<BT>(v);
        if constexpr (DIFF) {
          A1.template add_mid<GT>(g3);
          A2.template add_mid<BT>(g2);
          A3.template add_mid<BT>(g1);
        }
      }
      T p1[N], p2[N], p3[N];
      A1.finish(p1);
      if constexpr (DIFF) {
        A2.finish(p2);
        A3.finish(p3);
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < N; ++k) {
        buf[k * Q2 + t] = p1[k];
        if constexpr (DIFF) {
          buf[D::NQ2 + k * Q2 + t] = p2[k];
          buf[2 * D::NQ2 + k * Q2 + t] = p3[k];
        }
      }
      __syncthreads();
    }

    bwd_y<P, T, DIFF>(buf, t);
    bwd_x<P, T, DIFF>(buf, t);
    if (part) {
      const double dot = emit_e<P, T, true, POS>(buf, t, active, smap, xm, es, compact != 0,
                                                 Y + (int64_t)m * estride, y + (int64_t)m * ndof);
      // one sum per member; the block's pairs v_lo.. hold members (v_lo + k) mod nbatch,
      // k < count (a uniform test: members without a pair here get 0 without a sum)
      const int64_t v_lo = (int64_t)xcd_block() * E;
      const int64_t count = (npair - v_lo) < E ? (npair - v_lo) : E;
      const int r_lo = (int)(v_lo % nbatch);
      for (int mm = 0; mm < nbatch; ++mm) {
        const bool here = ((mm - r_lo + nbatch) % nbatch) < count;
        double sum = 0.0;
        if (here) sum = block_sum_d((active && m == mm) ? dot : 0.0, reinterpret_cast<double *>(smem));
        if (threadIdx.x == 0) part[(int64_t)mm * part_mstride + blockIdx.x] = sum;
      }
    } else {
      emit_e<P, T, false, POS>(buf, t, active, smap, xm, es, compact != 0,
                               Y + (int64_t)m * estride, y + (int64_t)m * ndof);
    }
  }
}

template <int P, typename T>
hipError_t launch_apply_pt(const ApplyArgs &a, hipStream_t s) {
  using D = Dims<P>;
  if (a.nelem <= 0 || a.nbatch <= 0) return hipSuccess;
  if ((a.pos != nullptr) != evec_dof_ordered(P)) return hipErrorInvalidValue;
  using C = ApplyCfg<P, T>;
  dim3 grid((unsigned)((a.nelem * a.nbatch + C::E - 1) / C::E));
  dim3 block(C::THREADS);
  const T *qd = (const T *)a.qd;
  const T *nu = (const T *)a.nu;
  const T *x = (const T *)a.x;
  T *Y = (T *)a.evec;
  T *y = (T *)a.y;
#define SFEM_APPLY_ARGS                                                                    \
  a.map, qd, a.qd_mstride, nu, a.nu_mstride, a.nelem, a.nbatch, a.ndof, x, Y, a.estride, \
      a.pos, a.compact, y, a.part, a.part_mstride
  switch (a.op) {
    case SFEM_MASS:
      hipLaunchKernelGGL((apply_kernel<P, T, 0>), grid, block, 0, s, SFEM_APPLY_ARGS);
      break;
    case SFEM_DIFFUSION:
      hipLaunchKernelGGL((apply_kernel<P, T, 1>), grid, block, 0, s, SFEM_APPLY_ARGS);
      break;
    default:
      hipLaunchKernelGGL((apply_kernel<P, T, 2>), grid, block, 0, s, SFEM_APPLY_ARGS);
      break;
  }
#undef SFEM_APPLY_ARGS
  return hipGetLastError();
}

// Elements per workgroup of the apply kernel for order P and precision T.
template <int P, typename T>
int apply_group_elems_pt() {
  return ApplyCfg<P, T>::E;
}

#define SFEM_DISPATCH_P(p, CALL) \
  switch (p) {                   \
    case 1: return CALL(1);      \
    case 2: return CALL(2);      \
    case 3: return CALL(3);      \
    case 4: return CALL(4);      \
    case 5: return CALL(5);      \
    case 6: return CALL(6);      \
    case 7: return CALL(7);      \
    case 8: return CALL(8);      \
    default: return hipErrorInvalidValue; \
  }

}  // namespace sfem
