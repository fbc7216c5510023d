// Host replay of the library's LOR assembly and multigrid setup (lor_host.cpp) for the
// comparison with the oracle: reads a mesh and coefficients from a binary file, writes the
// LOR matrix and every level of the hierarchy to another.
//   lor_check IN OUT
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
