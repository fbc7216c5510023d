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
// contributions are added with the same colored, atomic-free scatter as the apply;
// essential rows are set to 1.
#include <hip/hip_runtime.h>

#include "apply_impl.h"

namespace sfem {
namespace {

template <int P>
struct DiagTab {
  double T[3][P + 2][P + 1];  // 0: B2, 1: G2, 2: BG
};

// (x, y, z) table of each term; term 0 = mass, 1..6 = G11, G22, G33, G12, G13, G23
__device__ constexpr int kTermTab[7][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                                           {2, 2, 0}, {2, 0, 2}, {0, 2, 2}};

template <int P>
__global__ void __launch_bounds__(Dims<P>::Q2 < 64 ? 64 : Dims<P>::Q2)
diag_kernel(const DiagTab<P> tb, const int32_t *__restrict__ map, const double *__restrict__ qd,
            const double *__restrict__ nu, double alpha, double beta, int64_t e_begin,
            int64_t e_end, double *__restrict__ diag) {
  using D = Dims<P>;
  constexpr int N = D::N, Q = D::Q, N2 = D::N2, N3 = D::N3, Q2 = D::Q2, Q3 = D::Q3;
  __shared__ double s0[Q3];
  __shared__ double s1[Q2 * N];
  __shared__ double s2[Q * N2];
  const int t = threadIdx.x;
  const int nt = blockDim.x;
  const int64_t e = e_begin + blockIdx.x;
  if (e >= e_end) return;  // whole block exits together (one element per block)
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
        for (int a = 0; a < Q; ++a) s += tb.T[tx][a][i] * in[a];
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
        for (int b = 0; b < Q; ++b) s += tb.T[ty][b][j] * in[b];
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
        for (int c = 0; c < Q; ++c) s += tb.T[tz][c][k] * in[c];
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
    const int64_t g = c & kDofMask;
    if (c < 0) {
      if (c & kFirstBit) diag[g] = 1.0;
    } else if (c & kFirstBit) {
      diag[g] = s0[l];
    } else {
      diag[g] += s0[l];
    }
  }
}

template <int P>
hipError_t launch_diag_p(const DiagArgs &a, int64_t e_begin, int64_t e_end, hipStream_t s) {
  using D = Dims<P>;
  const int64_t ne = e_end - e_begin;
  if (ne <= 0) return hipSuccess;
  DiagTab<P> tb;
  for (int x = 0; x < P + 2; ++x)
    for (int i = 0; i < P + 1; ++i) {
      const double b = a.B[x * (P + 1) + i], g = a.G[x * (P + 1) + i];
      tb.T[0][x][i] = b * b;
      tb.T[1][x][i] = g * g;
      tb.T[2][x][i] = b * g;
    }
  const int threads = D::Q2 < 64 ? 64 : D::Q2;
  hipLaunchKernelGGL((diag_kernel<P>), dim3((unsigned)ne), dim3(threads), 0, s, tb, a.map, a.qd,
                     a.nu, a.alpha, a.beta, e_begin, e_end, a.diag);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_diag(const DiagArgs &a, int64_t e_begin, int64_t e_end, hipStream_t s) {
#define SFEM_CALL(P) launch_diag_p<P>(a, e_begin, e_end, s)
  SFEM_DISPATCH_P(a.p, SFEM_CALL)
#undef SFEM_CALL
}

}  // namespace sfem
