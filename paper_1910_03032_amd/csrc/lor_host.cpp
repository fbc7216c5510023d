// Host side of the low-order-refined preconditioner (Section 5.2): assembly of A_LOR on the
// GLL-refined mesh and the smoothed-aggregation multigrid setup (strength, aggregation,
// Jacobi-smoothed prolongator, Galerkin products, coarse pseudo-inverse) and the sliced
// ELL forms.  Plain C++ on the host threads (no device code), also compiled by the host
// tests; the parallel parts combine their results in a fixed order.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <map>
#include <thread>
#include <string>
#include <vector>

#include "lor_host.h"

namespace sfem {

namespace {

// Host threads of the set-up: SFEM_HOST_THREADS if set (1..16), else the hardware's, at
// most 16.
int host_threads() {
  if (const char *env = std::getenv("SFEM_HOST_THREADS")) {
    const int v = std::atoi(env);
    if (v >= 1) return std::min(v, 16);
  }
  const unsigned h = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(h, 16u));
}

// f(lo, hi, c) for the chunks [c chunk, min(n, (c + 1) chunk)) of [0, n), spread over the
// host threads.  Results that f keeps per chunk and combines in chunk order do not depend
// on the number of threads.
template <class F>
void for_chunks(int64_t n, int64_t chunk, F &&f) {
  const int64_t nc = n > 0 ? (n + chunk - 1) / chunk : 0;
  const int nt = (int)std::min<int64_t>(host_threads(), nc);
  std::atomic<int64_t> next{0};
  auto work = [&]() {
    for (int64_t c = next++; c < nc; c = next++) f(c * chunk, std::min(n, (c + 1) * chunk), c);
  };
  if (nt <= 1) {
    work();
    return;
  }
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(work);
  work();
  for (std::thread &t : th) t.join();
}

// Trilinear vertex functions and their reference derivatives at eta (vertex v = a + 2b + 4c
// at corner (2a-1, 2b-1, 2c-1)).
void trilinear(const double eta[3], double N[8], double dN[8][3]) {
  for (int v = 0; v < 8; ++v) {
    double f[3], s[3];
    for (int d = 0; d < 3; ++d) {
      s[d] = ((v >> d) & 1) ? 1.0 : -1.0;
      f[d] = 0.5 * (1.0 + s[d] * eta[d]);
    }
    N[v] = f[0] * f[1] * f[2];
    dN[v][0] = 0.5 * s[0] * f[1] * f[2];
    dN[v][1] = 0.5 * s[1] * f[0] * f[2];
    dN[v][2] = 0.5 * s[2] * f[0] * f[1];
  }
}

// Q1 mass and stiffness of the trilinear hexahedron through Y[8][3], 2 x 2 x 2 Gauss points.
void q1_element(const double Y[8][3], double M[8][8], double K[8][8]) {
  std::memset(M, 0, sizeof(double) * 64);
  std::memset(K, 0, sizeof(double) * 64);
  const double g = 1.0 / std::sqrt(3.0);
  for (int qp = 0; qp < 8; ++qp) {
    const double eta[3] = {(qp & 1) ? g : -g, (qp & 2) ? g : -g, (qp & 4) ? g : -g};
    double N[8], dN[8][3];
    trilinear(eta, N, dN);
    double J[3][3] = {};  // J[r][d] = dx_r / d eta_d
    for (int v = 0; v < 8; ++v)
      for (int r = 0; r < 3; ++r)
        for (int d = 0; d < 3; ++d) J[r][d] += Y[v][r] * dN[v][d];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double inv[3][3];  // inv = J^{-1}: inv[d][r]
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    double G[8][3];  // physical gradients: G[v][r] = sum_d inv[d][r] dN[v][d]
    for (int v = 0; v < 8; ++v)
      for (int r = 0; r < 3; ++r) G[v][r] = inv[0][r] * dN[v][0] + inv[1][r] * dN[v][1] + inv[2][r] * dN[v][2];
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b) {
        M[a][b] += det * N[a] * N[b];
        K[a][b] += det * (G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2]);
      }
  }
}

int64_t find_col(const HostCsr &A, int64_t row, int32_t c) {
  const int32_t *b = A.col.data() + A.ptr[row], *e = A.col.data() + A.ptr[row + 1];
  const int32_t *it = std::lower_bound(b, e, c);
  return (it != e && *it == c) ? (int64_t)(it - A.col.data()) : -1;
}

// C = A B (both CSR with sorted columns); dense accumulator over B's columns.  Rows in
// chunks over the host threads, each chunk's rows kept apart and concatenated in order.
void spgemm(const HostCsr &A, const HostCsr &B, HostCsr &C) {
  C.nrows = A.nrows;
  C.ncols = B.ncols;
  C.ptr.assign((size_t)C.nrows + 1, 0);
  constexpr int64_t kChunk = 8192;
  const int64_t nc = (A.nrows + kChunk - 1) / kChunk;
  std::vector<std::vector<int32_t>> ccol((size_t)nc);
  std::vector<std::vector<double>> cval((size_t)nc);
  for_chunks(A.nrows, kChunk, [&](int64_t lo, int64_t hi, int64_t ch) {
    std::vector<int64_t> mark((size_t)B.ncols, -1);
    std::vector<double> acc((size_t)B.ncols, 0.0);
    std::vector<int32_t> cols;
    std::vector<int32_t> &oc = ccol[(size_t)ch];
    std::vector<double> &ov = cval[(size_t)ch];
    for (int64_t i = lo; i < hi; ++i) {
      cols.clear();
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        const int32_t j = A.col[k];
        const double a = A.val[k];
        for (int64_t m = B.ptr[j]; m < B.ptr[j + 1]; ++m) {
          const int32_t c = B.col[m];
          if (mark[c] != i) {
            mark[c] = i;
            acc[c] = 0.0;
            cols.push_back(c);
          }
          acc[c] += a * B.val[m];
        }
      }
      std::sort(cols.begin(), cols.end());
      for (int32_t c : cols) {
        oc.push_back(c);
        ov.push_back(acc[c]);
      }
      C.ptr[(size_t)i + 1] = (int64_t)cols.size();
    }
  });
  for (int64_t i = 0; i < C.nrows; ++i) C.ptr[(size_t)i + 1] += C.ptr[(size_t)i];
  C.col.resize((size_t)C.ptr[(size_t)C.nrows]);
  C.val.resize(C.col.size());
  for_chunks(nc, 1, [&](int64_t ch, int64_t, int64_t) {
    const int64_t at = C.ptr[(size_t)(ch * kChunk)];
    std::copy(ccol[(size_t)ch].begin(), ccol[(size_t)ch].end(), C.col.begin() + at);
    std::copy(cval[(size_t)ch].begin(), cval[(size_t)ch].end(), C.val.begin() + at);
  });
}

void transpose(const HostCsr &A, HostCsr &T) {
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.ptr.assign((size_t)T.nrows + 1, 0);
  for (int32_t c : A.col) T.ptr[(size_t)c + 1]++;
  for (int64_t i = 0; i < T.nrows; ++i) T.ptr[i + 1] += T.ptr[i];
  T.col.resize(A.col.size());
  T.val.resize(A.val.size());
  std::vector<int64_t> pos(T.ptr.begin(), T.ptr.end() - 1);
  for (int64_t i = 0; i < A.nrows; ++i)  // rows in order: each column of T stays sorted
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const int64_t q = pos[A.col[k]]++;
      T.col[q] = (int32_t)i;
      T.val[q] = A.val[k];
    }
}

// rho(D^-1 A) by npower power iterations from v_i = 1 + (i mod 7) / 7.
double spectral_radius(const HostCsr &A, const std::vector<double> &dinv, int npower) {
  const int64_t n = A.nrows;
  std::vector<double> v((size_t)n), w((size_t)n);
  for (int64_t i = 0; i < n; ++i) v[i] = 1.0 + (double)(i % 7) / 7.0;
  double rho = 0.0;
  constexpr int64_t kChunk = 16384;
  const int64_t nc = (n + kChunk - 1) / kChunk;
  std::vector<double> pv((size_t)nc), pw((size_t)nc);
  for (int it = 0; it < npower; ++it) {
    for_chunks(n, kChunk, [&](int64_t lo, int64_t hi, int64_t ch) {
      double sv = 0.0, sw = 0.0;
      for (int64_t i = lo; i < hi; ++i) {
        double s = 0.0;
        for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) s += A.val[k] * v[A.col[k]];
        w[i] = dinv[i] * s;
        sv += v[i] * v[i];
        sw += w[i] * w[i];
      }
      pv[(size_t)ch] = sv;
      pw[(size_t)ch] = sw;
    });
    double nv = 0.0, nw = 0.0;
    for (int64_t ch = 0; ch < nc; ++ch) {
      nv += pv[(size_t)ch];
      nw += pw[(size_t)ch];
    }
    rho = std::sqrt(nw) / std::sqrt(nv);
    const double inw = 1.0 / std::sqrt(nw);
    for (int64_t i = 0; i < n; ++i) v[i] = w[i] * inw;
  }
  return rho;
}

// Aggregates of the rows of A (-1: isolated row: no nonzero off-diagonal entry).  Strong
// connection: j != i, a_ij != 0, |a_ij| >= theta sqrt(|a_ii a_jj|).  Three passes over the
// rows in index order: (a) a row whose strong neighbours are all unaggregated starts an
// aggregate with them; (b) a remaining row joins the aggregate that pass (a) gave its first
// strong neighbour (column order) if any; (c) a row still left starts an aggregate with
// its unaggregated strong neighbours.
int64_t aggregate(const HostCsr &A, double theta, std::vector<int64_t> &agg) {
  const int64_t n = A.nrows;
  std::vector<double> d((size_t)n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t k = find_col(A, i, (int32_t)i);
    d[i] = k >= 0 ? std::fabs(A.val[k]) : 0.0;
  }
  std::vector<int64_t> sptr((size_t)n + 1, 0);
  std::vector<int32_t> scol;
  std::vector<char> isolated((size_t)n, 1);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const int32_t j = A.col[k];
      if (j == i || A.val[k] == 0.0) continue;
      isolated[i] = 0;
      if (std::fabs(A.val[k]) >= theta * std::sqrt(d[i] * d[j])) scol.push_back(j);
    }
    sptr[i + 1] = (int64_t)scol.size();
  }
  agg.assign((size_t)n, -1);
  int64_t nagg = 0;
  for (int64_t i = 0; i < n; ++i) {  // pass (a)
    if (isolated[i] || agg[i] >= 0) continue;
    bool free_nbhd = true;
    for (int64_t k = sptr[i]; k < sptr[i + 1] && free_nbhd; ++k) free_nbhd = agg[scol[k]] < 0;
    if (!free_nbhd) continue;
    agg[i] = nagg;
    for (int64_t k = sptr[i]; k < sptr[i + 1]; ++k) agg[scol[k]] = nagg;
    ++nagg;
  }
  const std::vector<int64_t> first = agg;
  for (int64_t i = 0; i < n; ++i) {  // pass (b)
    if (isolated[i] || agg[i] >= 0) continue;
    for (int64_t k = sptr[i]; k < sptr[i + 1]; ++k)
      if (first[scol[k]] >= 0) {
        agg[i] = first[scol[k]];
        break;
      }
  }
  for (int64_t i = 0; i < n; ++i) {  // pass (c)
    if (isolated[i] || agg[i] >= 0) continue;
    agg[i] = nagg;
    for (int64_t k = sptr[i]; k < sptr[i + 1]; ++k)
      if (agg[scol[k]] < 0) agg[scol[k]] = nagg;
    ++nagg;
  }
  return nagg;
}

// Pseudo-inverse of the symmetric n x n matrix C (row-major) by cyclic Jacobi rotations:
// eigenvalues below 1e-12 of the largest magnitude are dropped.
void pseudo_inverse(int64_t n, std::vector<double> &C) {
  std::vector<double> V((size_t)(n * n), 0.0);
  for (int64_t i = 0; i < n; ++i) V[i * n + i] = 1.0;
  auto a = [&](int64_t i, int64_t j) -> double & { return C[i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < n; ++j) {
        tot += a(i, j) * a(i, j);
        if (i != j) off += a(i, j) * a(i, j);
      }
    if (off <= 1e-30 * tot) break;
    for (int64_t p = 0; p < n - 1; ++p)
      for (int64_t q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (apq == 0.0) continue;
        const double th = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int64_t k = 0; k < n; ++k) {  // columns p, q
          const double akp = a(k, p), akq = a(k, q);
          a(k, p) = c * akp - s * akq;
          a(k, q) = s * akp + c * akq;
        }
        for (int64_t k = 0; k < n; ++k) {  // rows p, q
          const double apk = a(p, k), aqk = a(q, k);
          a(p, k) = c * apk - s * aqk;
          a(q, k) = s * apk + c * aqk;
        }
        for (int64_t k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  std::vector<double> lam((size_t)n);
  double lmax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    lam[i] = a(i, i);
    lmax = std::max(lmax, std::fabs(lam[i]));
  }
  std::vector<double> out((size_t)(n * n), 0.0);
  for (int64_t k = 0; k < n; ++k) {
    if (!(lam[k] > 1e-12 * lmax)) continue;
    const double il = 1.0 / lam[k];
    for (int64_t i = 0; i < n; ++i) {
      const double vi = V[i * n + k] * il;
      for (int64_t j = 0; j < n; ++j) out[i * n + j] += vi * V[j * n + k];
    }
  }
  C.swap(out);
}

}  // namespace

void lor_assemble(int p, const double *gll, int64_t nelem, const double *xyz, const int32_t *dofs,
                  int64_t ndof, const uint8_t *ess, double alpha, double beta, const double *nu_e,
                  HostCsr &A) {
  const int n = p + 1;
  const int64_t n3 = (int64_t)n * n * n;
  // corner local nodes of every sub-element
  std::vector<int32_t> corner((size_t)p * p * p * 8);
  for (int k = 0; k < p; ++k)
    for (int j = 0; j < p; ++j)
      for (int i = 0; i < p; ++i)
        for (int v = 0; v < 8; ++v) {
          const int a = v & 1, b = (v >> 1) & 1, c = (v >> 2) & 1;
          corner[((size_t)(i + p * (j + p * k))) * 8 + v] = (i + a) + n * ((j + b) + n * (k + c));
        }
  const int64_t nsub = (int64_t)p * p * p;
  auto is_ess = [&](int32_t g) { return ess && ess[g] != 0; };
  // pattern: candidate columns per free row (free-free pairs), then sort + unique
  std::vector<int64_t> cnt((size_t)ndof + 1, 0);
  for (int64_t e = 0; e < nelem; ++e)
    for (int64_t s = 0; s < nsub; ++s)
      for (int v = 0; v < 8; ++v) {
        const int32_t g = dofs[e * n3 + corner[s * 8 + v]];
        if (!is_ess(g)) cnt[(size_t)g + 1] += 8;
      }
  for (int64_t g = 0; g < ndof; ++g) cnt[g + 1] += cnt[g];
  std::vector<int32_t> cand((size_t)cnt[ndof]);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t e = 0; e < nelem; ++e)
    for (int64_t s = 0; s < nsub; ++s) {
      int32_t g[8];
      for (int v = 0; v < 8; ++v) g[v] = dofs[e * n3 + corner[s * 8 + v]];
      for (int a = 0; a < 8; ++a) {
        if (is_ess(g[a])) continue;
        for (int b = 0; b < 8; ++b)
          cand[fill[g[a]]++] = is_ess(g[b]) ? g[a] : g[b];  // essential columns dropped
      }
    }
  A.nrows = A.ncols = ndof;
  A.ptr.assign((size_t)ndof + 1, 0);
  // each row's candidates sorted and made unique in place (rows over the host threads);
  // an essential (or unused) row keeps the diagonal alone
  constexpr int64_t kRows = 16384;
  auto lone = [&](int64_t g) { return is_ess((int32_t)g) || cnt[g] == cnt[g + 1]; };
  for_chunks(ndof, kRows, [&](int64_t lo, int64_t hi, int64_t) {
    for (int64_t g = lo; g < hi; ++g) {
      if (lone(g)) {
        A.ptr[g + 1] = 1;
        continue;
      }
      auto b = cand.begin() + cnt[g], e = cand.begin() + cnt[g + 1];
      std::sort(b, e);
      A.ptr[g + 1] = (int64_t)(std::unique(b, e) - b);
    }
  });
  for (int64_t g = 0; g < ndof; ++g) A.ptr[g + 1] += A.ptr[g];
  A.col.resize((size_t)A.ptr[ndof]);
  for_chunks(ndof, kRows, [&](int64_t lo, int64_t hi, int64_t) {
    for (int64_t g = lo; g < hi; ++g) {
      if (lone(g))
        A.col[(size_t)A.ptr[g]] = (int32_t)g;
      else
        std::copy(cand.begin() + cnt[g], cand.begin() + cnt[g] + (A.ptr[g + 1] - A.ptr[g]),
                  A.col.begin() + A.ptr[g]);
    }
  });
  std::vector<int32_t>().swap(cand);
  A.val.assign(A.col.size(), 0.0);
  // values: element by element, sub-element by sub-element.  The elements are colored
  // greedily in index order so that no two of one color share a DoF; the colors run one
  // after another and the elements of a color over the host threads, so every entry gets
  // its terms in one fixed order whatever the number of threads (a mesh that needs more
  // than 32 colors runs its elements one after another).
  std::vector<uint32_t> dmask((size_t)ndof, 0u);
  std::vector<std::vector<int64_t>> byc;
  for (int64_t e = 0; e < nelem; ++e) {
    uint32_t forb = 0;
    for (int64_t l = 0; l < n3; ++l) forb |= dmask[(size_t)dofs[e * n3 + l]];
    if (forb == 0xffffffffu) {
      byc.assign(1, std::vector<int64_t>());
      break;
    }
    int c = 0;
    while (forb & (1u << c)) ++c;
    for (int64_t l = 0; l < n3; ++l) dmask[(size_t)dofs[e * n3 + l]] |= 1u << c;
    if ((int)byc.size() <= c) byc.resize((size_t)c + 1);
    byc[(size_t)c].push_back(e);
  }
  const bool serial = byc.size() == 1 && (int64_t)byc[0].size() != nelem;
  std::vector<uint32_t>().swap(dmask);
  const double *x1 = gll;
  auto element_values = [&](int64_t e) {
    const double *X = xyz + e * 24;
    const double nu = nu_e ? nu_e[e] : 1.0;
    for (int64_t s = 0; s < nsub; ++s) {
      double Y[8][3];
      int32_t g[8];
      for (int v = 0; v < 8; ++v) {
        const int l = corner[s * 8 + v];
        g[v] = dofs[e * n3 + l];
        const double eta[3] = {x1[l % n], x1[(l / n) % n], x1[l / (n * n)]};
        double N[8], dN[8][3];
        trilinear(eta, N, dN);
        for (int r = 0; r < 3; ++r) {
          double acc = 0.0;
          for (int w = 0; w < 8; ++w) acc += N[w] * X[w * 3 + r];
          Y[v][r] = acc;
        }
      }
      double M[8][8], K[8][8];
      q1_element(Y, M, K);
      for (int a = 0; a < 8; ++a) {
        if (is_ess(g[a])) continue;
        for (int b = 0; b < 8; ++b) {
          if (is_ess(g[b])) continue;
          const int64_t k = find_col(A, g[a], g[b]);
          A.val[k] += alpha * M[a][b] + beta * nu * K[a][b];
        }
      }
    }
  };
  if (serial) {
    for (int64_t e = 0; e < nelem; ++e) element_values(e);
  } else {
    for (const std::vector<int64_t> &els : byc)
      for_chunks((int64_t)els.size(), 64, [&](int64_t lo, int64_t hi, int64_t) {
        for (int64_t i = lo; i < hi; ++i) element_values(els[(size_t)i]);
      });
  }
  for (int64_t g = 0; g < ndof; ++g)
    if (is_ess((int32_t)g)) A.val[A.ptr[g]] = 1.0;  // constrained row: the identity
}

void csr_transpose(const HostCsr &A, HostCsr &T) { transpose(A, T); }

namespace {

// Column offsets (col - row) of the rows of slice s of H, sorted and unique.  Fast path:
// when every row's offsets are among those of the slice's longest row (rows are sorted,
// so a merge per row checks it), that row's offsets are the union.
std::vector<int32_t> slice_offsets(const HostCsr &H, int64_t s) {
  const int64_t r0 = s * kSellRows, r1 = std::min(H.nrows, (s + 1) * kSellRows);
  int64_t longest = r0;
  for (int64_t r = r0; r < r1; ++r)
    if (H.ptr[(size_t)r + 1] - H.ptr[(size_t)r] > H.ptr[(size_t)longest + 1] - H.ptr[(size_t)longest]) longest = r;
  std::vector<int32_t> u;
  for (int64_t k = H.ptr[(size_t)longest]; k < H.ptr[(size_t)longest + 1]; ++k)
    u.push_back((int32_t)(H.col[(size_t)k] - longest));
  bool subset = true;
  for (int64_t r = r0; r < r1 && subset; ++r) {
    size_t j = 0;
    for (int64_t k = H.ptr[(size_t)r]; k < H.ptr[(size_t)r + 1] && subset; ++k) {
      const int32_t o = (int32_t)(H.col[(size_t)k] - r);
      while (j < u.size() && u[j] < o) ++j;
      subset = j < u.size() && u[j] == o;
    }
  }
  if (subset) return u;
  u.clear();
  for (int64_t r = r0; r < r1; ++r)
    for (int64_t k = H.ptr[(size_t)r]; k < H.ptr[(size_t)r + 1]; ++k)
      u.push_back((int32_t)(H.col[(size_t)k] - r));
  std::sort(u.begin(), u.end());
  u.erase(std::unique(u.begin(), u.end()), u.end());
  return u;
}

}  // namespace

std::string sell_build(const HostCsr &H, bool patterns, HostSell &S) {
  S = HostSell{};
  S.nrows = H.nrows;
  S.ncols = H.ncols;
  patterns = patterns && H.nrows == H.ncols;
  const int64_t nsl = (H.nrows + kSellRows - 1) / kSellRows;
  std::vector<int64_t> off((size_t)nsl + 1, 0), len((size_t)nsl, 0);
  S.pinfo.assign((size_t)nsl, 0);
  std::vector<std::vector<int32_t>> sofs((size_t)nsl);
  std::map<std::vector<int32_t>, int32_t> known;  // pattern -> its start in S.pat
  int64_t ncol = 0;
  for (int64_t s = 0; s < nsl; ++s) {
    int64_t l = 0;
    for (int64_t r = s * kSellRows; r < std::min(H.nrows, (s + 1) * kSellRows); ++r)
      l = std::max(l, H.ptr[(size_t)r + 1] - H.ptr[(size_t)r]);
    bool use_pat = false;
    if (patterns && l > 0) {
      sofs[(size_t)s] = slice_offsets(H, s);
      use_pat = (int64_t)sofs[(size_t)s].size() <= l + l / 8;
    }
    if (use_pat) {
      auto it = known.find(sofs[(size_t)s]);
      if (it == known.end()) {
        if ((int64_t)S.pat.size() + (int64_t)sofs[(size_t)s].size() >= (int64_t)INT32_MAX)
          return "sliced ELL: too many column-offset patterns";
        it = known.emplace(sofs[(size_t)s], (int32_t)S.pat.size()).first;
        S.pat.insert(S.pat.end(), sofs[(size_t)s].begin(), sofs[(size_t)s].end());
      }
      S.pinfo[(size_t)s] = -1 - it->second;
      len[(size_t)s] = (int64_t)sofs[(size_t)s].size();
      ++S.pattern_slices;
    } else {
      sofs[(size_t)s].clear();
      if (ncol + l * kSellRows >= (int64_t)INT32_MAX) return "sliced ELL: matrix too large (padded nnz >= 2^31)";
      S.pinfo[(size_t)s] = (int32_t)ncol;
      len[(size_t)s] = l;
      ncol += l * kSellRows;
    }
    off[(size_t)s + 1] = off[(size_t)s] + len[(size_t)s] * kSellRows;
    if (off[(size_t)s + 1] >= (int64_t)INT32_MAX) return "sliced ELL: matrix too large (padded nnz >= 2^31)";
  }
  S.off.assign(off.begin(), off.end());
  S.col.assign((size_t)ncol, 0);
  S.val.assign((size_t)off[(size_t)nsl], 0.0);
  for (int64_t s = 0; s < nsl; ++s) {
    const int64_t o = off[(size_t)s];
    const int32_t pi = S.pinfo[(size_t)s];
    const std::vector<int32_t> &u = sofs[(size_t)s];
    for (int64_t r = s * kSellRows; r < (s + 1) * kSellRows; ++r) {
      const int64_t lane = r - s * kSellRows;
      const int64_t b = r < H.nrows ? H.ptr[(size_t)r] : 0, e = r < H.nrows ? H.ptr[(size_t)r + 1] : 0;
      if (pi < 0) {
        // each entry of the row at its offset's place in the pattern (both sorted)
        size_t k = 0;
        for (int64_t q = b; q < e; ++q) {
          const int32_t d = (int32_t)(H.col[(size_t)q] - r);
          while (u[k] != d) ++k;
          S.val[(size_t)(o + (int64_t)k * kSellRows + lane)] = H.val[(size_t)q];
        }
        continue;
      }
      // padding: the row's last column (a valid index near its others) with value 0
      const int32_t last = e > b ? H.col[(size_t)(e - 1)] : 0;
      for (int64_t k = 0; k < len[(size_t)s]; ++k) {
        const bool in = b + k < e;
        S.col[(size_t)(pi + k * kSellRows + lane)] = in ? H.col[(size_t)(b + k)] : last;
        S.val[(size_t)(o + k * kSellRows + lane)] = in ? H.val[(size_t)(b + k)] : 0.0;
      }
    }
  }
  return "";
}


std::string amg_build_host(const HostCsr &A0, double theta, int64_t coarse_size, int max_levels,
                           HostAmg &H) {
  std::vector<HostCsr> &As = H.A, &Ps = H.P;
  std::vector<double> &rhos = H.rho;
  As.clear();
  Ps.clear();
  rhos.clear();
  As.push_back(A0);
  for (;;) {
    const HostCsr &A = As.back();
    std::vector<double> dinv((size_t)A.nrows);
    for (int64_t i = 0; i < A.nrows; ++i) {
      const int64_t k = find_col(A, i, (int32_t)i);
      if (k < 0 || A.val[k] == 0.0) return "LOR multigrid: zero diagonal entry";
      dinv[i] = 1.0 / A.val[k];
    }
    rhos.push_back(spectral_radius(A, dinv, 15));
    if (A.nrows <= coarse_size || (int)As.size() == max_levels) break;
    std::vector<int64_t> agg;
    const int64_t nagg = aggregate(A, theta, agg);
    if (nagg == 0 || nagg >= A.nrows) break;
    // smoothed prolongator P = (I - omega D^-1 A) P0, P0 the aggregate indicator
    const double omega = 4.0 / (3.0 * rhos.back());
    HostCsr P;
    P.nrows = A.nrows;
    P.ncols = nagg;
    P.ptr.assign((size_t)A.nrows + 1, 0);
    std::vector<int64_t> mark((size_t)nagg, -1);
    std::vector<double> acc((size_t)nagg, 0.0);
    std::vector<int32_t> cols;
    for (int64_t i = 0; i < A.nrows; ++i) {
      cols.clear();
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        const int64_t J = agg[A.col[k]];
        if (J < 0) continue;
        if (mark[J] != i) {
          mark[J] = i;
          acc[J] = 0.0;
          cols.push_back((int32_t)J);
        }
        acc[J] += A.val[k];
      }
      std::sort(cols.begin(), cols.end());
      for (int32_t J : cols) {
        const double v = (agg[i] == J ? 1.0 : 0.0) - omega * dinv[i] * acc[J];
        P.col.push_back(J);
        P.val.push_back(v);
      }
      P.ptr[i + 1] = (int64_t)P.col.size();
    }
    HostCsr R, AP, Ac;
    transpose(P, R);
    spgemm(A, P, AP);
    spgemm(R, AP, Ac);
    Ps.push_back(std::move(P));
    As.push_back(std::move(Ac));
  }
  // coarsest level: dense pseudo-inverse
  const HostCsr &C = As.back();
  H.coarse.assign((size_t)(C.nrows * C.nrows), 0.0);
  for (int64_t i = 0; i < C.nrows; ++i)
    for (int64_t k = C.ptr[i]; k < C.ptr[i + 1]; ++k) H.coarse[(size_t)(i * C.nrows + C.col[k])] = C.val[k];
  pseudo_inverse(C.nrows, H.coarse);
  return "";
}

}  // namespace sfem
