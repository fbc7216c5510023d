// Exact diagonal of the assembled operator alpha M + beta K(nu), sum-factorized.
//
// With the stored factors m = w|J| and Gq = w|J| J^-1 J^-T (symmetric, 6 entries),
// the diagonal entry of node (i, j, k) of an element is
//   alpha sum_abc m B2(a,i) B2(b,j) B2(c,k)
// + beta  sum_abc nu sum_{r,s} Gq_rs t_r t_s
// where t_1 = G(a,i) B(b,j) B(c,k), t_2 = B G B, t_3 = B B G (the rows of the tensor
// gradient of eq. tensorGradient evaluated on the node's own basis function).  Each
// of the 7 distinct (r, s) products factors per direction into a Hadamard product
// of 1D tables: B2 = B.B, G2 = G.G, BG = B.G, with the off-diagonal pairs doubled.
// Every term is then a three-stage contraction q^3 -> n^3.  The element
// contributions are assembled like the apply's (sole DoFs directly, shared nodes via
// the E-vector and the assembly kernel, which sets the essential rows to 1).
#include <hip/hip_runtime.h>

#include "apply_impl.h"

namespace sfem {
namespace {

// Hadamard products of the compile-time 1D tables: 0: B.B, 1: G.G, 2: B.G
template <int P>
__device__ __forceinline__ constexpr double dtab(int which, int a, int i) {
  using TB = Tab<P, double>;
  return which == 0 ? TB::B(a, i) * TB::B(a, i)
                    : (which == 1 ? TB::G(a, i) * TB::G(a, i) : TB::B(a, i) * TB::G(a, i));
}

// (x, y, z) table of each term; term 0 = mass, 1..6 = G11, G22, G33, G12, G13, G23
__device__ constexpr int kTermTab[7][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                                           {2, 2, 0}, {2, 0, 2}, {0, 2, 2}};

template <int P>
__global__ void __launch_bounds__(Dims<P>::Q2 < 64 ? 64 : Dims<P>::Q2)
diag_kernel(const int32_t *__restrict__ map, const double *__restrict__ qd,
            const double *__restrict__ nu, double alpha, double beta, int64_t nelem,
            double *__restrict__ diag, double *__restrict__ Y, const int32_t *__restrict__ pos,
            int compact) {
  using D = Dims<P>;
  constexpr int N = D::N, Q = D::Q, N2 = D::N2, N3 = D::N3, Q2 = D::Q2, Q3 = D::Q3;
  __shared__ double s0[Q3];
  __shared__ double s1[Q2 * N];
  __shared__ double s2[Q * N2];
  const int t = threadIdx.x;
  const int nt = blockDim.x;
  const int64_t e = blockIdx.x;
  if (e >= nelem) return;  // whole block exits together (one element per block)
  const double *qe = qd + e * (int64_t)(kQdSlots * Q3);
  const double *ne = nu ? nu + e * (int64_t)Q3 : nullptr;
  double acc[N];
#pragma unroll
  for (int k = 0; k < N; ++k) acc[k] = 0.0;

#pragma unroll
  for (int term = 0; term < 7; ++term) {
    const double coef = (term == 0) ? alpha : ((term <= 3) ? beta : 2.0 * beta);
    if (coef == 0.0) continue;  // uniform across the block
    for (int qi = t; qi < Q3; qi += nt) {
      double v = coef * qe[(int64_t)term * Q3 + qi];
      if (term > 0 && ne) v *= ne[qi];
      s0[qi] = v;
    }
    __syncthreads();
    const int tx = kTermTab[term][0], ty = kTermTab[term][1], tz = kTermTab[term][2];
    if (t < Q2) {  // contract a: lines (b, c)
      const int b = t % Q, c = t / Q;
      double in[Q];
#pragma unroll
      for (int a = 0; a < Q; ++a) in[a] = s0[c * Q2 + b * Q + a];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < Q; ++a) s += dtab<P>(tx, a, i) * in[a];
        s1[(c * Q + b) * N + i] = s;
      }
    }
    __syncthreads();
    if (t < Q * N) {  // contract b: lines (i, c)
      const int i = t % N, c = t / N;
      double in[Q];
#pragma unroll
      for (int b = 0; b < Q; ++b) in[b] = s1[(c * Q + b) * N + i];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < Q; ++b) s += dtab<P>(ty, b, j) * in[b];
        s2[(c * N + j) * N + i] = s;
      }
    }
    __syncthreads();
    if (t < N2) {  // contract c: lines (i, j)
      const int i = t % N, j = t / N;
      double in[Q];
#pragma unroll
      for (int c = 0; c < Q; ++c) in[c] = s2[(c * N + j) * N + i];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < Q; ++c) s += dtab<P>(tz, c, k) * in[c];
        acc[k] += s;
      }
    }
    __syncthreads();
  }
  // nodal values into s0 as [k][j][i]
  if (t < N2) {
    const int i = t % N, j = t / N;
#pragma unroll
    for (int k = 0; k < N; ++k) s0[(k * N + j) * N + i] = acc[k];
  }
  __syncthreads();
  const int32_t *emap = map + e * (int64_t)N3;
  for (int l = t; l < N3; l += nt) {
    const int32_t c = emap[l];
    if (c < 0) continue;
    if (c & kSoleBit)
      diag[c & kDofMask] = s0[l];
    else {
      const int64_t q = compact ? e * surf_count<P>() + surf_rank<P>(l) : e * N3 + l;
      Y[pos ? pos[q] : q] = s0[l];
    }
  }
}

template <int P>
hipError_t launch_diag_p(const DiagArgs &a, hipStream_t s) {
  using D = Dims<P>;
  const int64_t ne = a.nelem;
  if (ne <= 0) return hipSuccess;
  const int threads = D::Q2 < 64 ? 64 : D::Q2;
  hipLaunchKernelGGL((diag_kernel<P>), dim3((unsigned)ne), dim3(threads), 0, s, a.map, a.qd,
                     a.nu, a.alpha, a.beta, a.nelem, a.diag, a.evec, a.pos, a.compact);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_diag(const DiagArgs &a, hipStream_t s) {
#define SFEM_CALL(P) launch_diag_p<P>(a, s)
  SFEM_DISPATCH_P(a.p, SFEM_CALL)
#undef SFEM_CALL
}

}  // namespace sfem
