// Host replay of the library's LOR assembly and multigrid setup (lor_host.cpp) for the
// comparison with the oracle: reads a mesh and coefficients from a binary file, writes the
// LOR matrix and every level of the hierarchy to another.  It also builds the sliced ELL
// form of every level operator (with column-offset patterns) and prolongator, replays the
// device kernel's product on it and requires the CSR product's result exactly (exit 3
// otherwise); it prints the number of pattern slices per level.
//   lor_check IN OUT
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lor_host.h"

using namespace sfem;

template <typename T>
static void rd(FILE *f, T *p, size_t n) {
  if (n && fread(p, sizeof(T), n, f) != n) {
    fprintf(stderr, "short read\n");
    exit(2);
  }
}
template <typename T>
static void wr(FILE *f, const T *p, size_t n) {
  if (n) fwrite(p, sizeof(T), n, f);
}
static void write_csr(FILE *f, const HostCsr &A) {
  const int64_t hdr[3] = {A.nrows, A.ncols, A.nnz()};
  wr(f, hdr, 3);
  wr(f, A.ptr.data(), A.ptr.size());
  wr(f, A.col.data(), A.col.size());
  wr(f, A.val.data(), A.val.size());
}

// y = M x through the sliced ELL form, term by term as the device kernel forms it.
static std::vector<double> sell_product(const HostSell &S, const std::vector<double> &x) {
  std::vector<double> y((size_t)S.nrows, 0.0);
  const int64_t nsl = (int64_t)S.pinfo.size();
  for (int64_t s = 0; s < nsl; ++s) {
    const int64_t k0 = S.off.at((size_t)s), len = (S.off.at((size_t)s + 1) - k0) / kSellRows;
    const int32_t pi = S.pinfo.at((size_t)s);
    for (int64_t lane = 0; lane < kSellRows; ++lane) {
      const int64_t i = s * kSellRows + lane;
      if (i >= S.nrows) break;
      double acc = 0.0;
      for (int64_t k = 0; k < len; ++k) {
        int64_t c;
        if (pi >= 0) {
          c = S.col.at((size_t)(pi + k * kSellRows + lane));
        } else {
          c = i + S.pat.at((size_t)(-1 - pi + k));
          c = c < 0 ? 0 : (c >= S.ncols ? S.ncols - 1 : c);
        }
        acc += S.val.at((size_t)(k0 + k * kSellRows + lane)) * x.at((size_t)c);
      }
      y[(size_t)i] = acc;
    }
  }
  return y;
}

// The sliced ELL product of M equals its CSR product on two vectors; returns the number of
// pattern slices (and the stored values in *stored), or -1.
static int64_t check_sell(const HostCsr &M, bool patterns, int64_t *stored = nullptr) {
  HostSell S;
  if (!sell_build(M, patterns, S).empty()) return -1;
  if (S.val.size() != (size_t)S.off.back()) return -1;
  for (int t = 0; t < 2; ++t) {
    std::vector<double> x((size_t)M.ncols);
    for (size_t j = 0; j < x.size(); ++j) x[j] = std::sin(1.0 + (double)j * (t ? 0.37 : 1.13));
    const std::vector<double> y = sell_product(S, x);
    for (int64_t i = 0; i < M.nrows; ++i) {
      double acc = 0.0;
      for (int64_t q = M.ptr[(size_t)i]; q < M.ptr[(size_t)i + 1]; ++q) acc += M.val[(size_t)q] * x[(size_t)M.col[(size_t)q]];
      if (acc != y[(size_t)i]) {
        fprintf(stderr, "sliced ELL product differs in row %lld\n", (long long)i);
        return -1;
      }
    }
  }
  if (stored) *stored = (int64_t)S.val.size();
  return S.pattern_slices;
}

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  FILE *in = fopen(argv[1], "rb");
  if (!in) return 2;
  int64_t hdr[5];  // p, nelem, ndof, coarse_size, max_levels
  double coef[3];  // alpha, beta, theta
  int32_t has_nu = 0;
  rd(in, hdr, 5);
  rd(in, coef, 3);
  rd(in, &has_nu, 1);
  const int p = (int)hdr[0];
  const int64_t nelem = hdr[1], ndof = hdr[2], n3 = (int64_t)(p + 1) * (p + 1) * (p + 1);
  std::vector<double> gll((size_t)p + 1), xyz((size_t)nelem * 24), nu((size_t)(has_nu ? nelem : 0));
  std::vector<int32_t> dofs((size_t)(nelem * n3));
  std::vector<uint8_t> ess((size_t)ndof);
  rd(in, gll.data(), gll.size());
  rd(in, xyz.data(), xyz.size());
  rd(in, dofs.data(), dofs.size());
  rd(in, ess.data(), ess.size());
  rd(in, nu.data(), nu.size());
  fclose(in);
  HostCsr A;
  lor_assemble(p, gll.data(), nelem, xyz.data(), dofs.data(), ndof, ess.data(), coef[0], coef[1],
               has_nu ? nu.data() : nullptr, A);
  HostAmg H;
  const std::string e = amg_build_host(A, coef[2], hdr[3], (int)hdr[4], H);
  if (!e.empty()) {
    fprintf(stderr, "%s\n", e.c_str());
    return 1;
  }
  for (size_t l = 0; l < H.A.size(); ++l) {
    int64_t stored = 0;
    const int64_t np = check_sell(H.A[l], true, &stored);
    if (np < 0 || (l < H.P.size() && check_sell(H.P[l], true) < 0)) return 3;
    printf("pattern slices %zu %lld of %lld, values %lld stored for %lld nonzeros\n", l, (long long)np,
           (long long)((H.A[l].nrows + kSellRows - 1) / kSellRows), (long long)stored,
           (long long)H.A[l].nnz());
  }
  FILE *out = fopen(argv[2], "wb");
  const int64_t L = (int64_t)H.A.size();
  wr(out, &L, 1);
  for (int64_t l = 0; l < L; ++l) {
    write_csr(out, H.A[(size_t)l]);
    wr(out, &H.rho[(size_t)l], 1);
  }
  for (int64_t l = 0; l + 1 < L; ++l) write_csr(out, H.P[(size_t)l]);
  wr(out, H.coarse.data(), H.coarse.size());
  fclose(out);
  printf("levels %lld\n", (long long)L);
  return 0;
}
