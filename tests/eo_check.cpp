// Host check of the even-odd contraction helpers against direct sums, p = 1..8.
#include <cmath>
#include <cstdio>
#include <random>

#include "eo.h"

using namespace sfem;

static double worst = 0.0;

template <int P, int W>
void check_table() {
  using TB = eo::Tab1<P, W>;
  constexpr int NO = TB::NO, NI = TB::NI;
  std::mt19937_64 rng(1234 + 17 * P + W);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  // the symmetry the decomposition relies on
  for (int a = 0; a < NO; ++a)
    for (int i = 0; i < NI; ++i) {
      const double d = std::fabs(TB::t(NO - 1 - a, NI - 1 - i) - TB::S * TB::t(a, i));
      if (d > 1e-13) std::printf("FAIL symmetry P=%d W=%d a=%d i=%d d=%g\n", P, W, a, i, d);
    }
  for (int rep = 0; rep < 20; ++rep) {
    double v[NI], out[NO];
    for (auto &x : v) x = U(rng);
    eo::apply<TB>(eo::split(v), out);
    for (int a = 0; a < NO; ++a) {
      double ref = 0.0, scale = 0.0;
      for (int i = 0; i < NI; ++i) {
        ref += TB::t(a, i) * v[i];
        scale += std::fabs(TB::t(a, i) * v[i]);
      }
      worst = std::fmax(worst, std::fabs(out[a] - ref) / (scale + 1e-300));
    }
    // transposed, accumulated by input pairs
    double in[NO], tout[NI];
    for (auto &x : in) x = U(rng);
    eo::Acc<NI, double> acc;
    acc.zero();
    for (int a = 0; a < NO / 2; ++a) acc.template add_pair<TB>(a, in[a], in[NO - 1 - a]);
    if (NO % 2 == 1) acc.template add_mid<TB>(in[NO / 2]);
    acc.finish(tout);
    for (int i = 0; i < NI; ++i) {
      double ref = 0.0, scale = 0.0;
      for (int a = 0; a < NO; ++a) {
        ref += TB::t(a, i) * in[a];
        scale += std::fabs(TB::t(a, i) * in[a]);
      }
      worst = std::fmax(worst, std::fabs(tout[i] - ref) / (scale + 1e-300));
    }
  }
}

template <int P>
void check_mixed() {
  // one accumulator fed by a symmetric and an antisymmetric table (B^T v + G^T g)
  using TBB = eo::Tab1<P, 0>;
  using TBG = eo::Tab1<P, 1>;
  constexpr int NO = TBB::NO, NI = TBB::NI;
  std::mt19937_64 rng(99 + P);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  double v[NO], g[NO], out[NI];
  for (auto &x : v) x = U(rng);
  for (auto &x : g) x = U(rng);
  eo::Acc<NI, double> acc;
  acc.zero();
  for (int a = 0; a < NO / 2; ++a) {
    acc.template add_pair<TBB>(a, v[a], v[NO - 1 - a]);
    acc.template add_pair<TBG>(a, g[a], g[NO - 1 - a]);
  }
  if (NO % 2 == 1) {
    acc.template add_mid<TBB>(v[NO / 2]);
    acc.template add_mid<TBG>(g[NO / 2]);
  }
  acc.finish(out);
  for (int i = 0; i < NI; ++i) {
    double ref = 0.0, scale = 0.0;
    for (int a = 0; a < NO; ++a) {
      ref += TBB::t(a, i) * v[a] + TBG::t(a, i) * g[a];
      scale += std::fabs(TBB::t(a, i) * v[a]) + std::fabs(TBG::t(a, i) * g[a]);
    }
    worst = std::fmax(worst, std::fabs(out[i] - ref) / (scale + 1e-300));
  }
}

template <int P>
void check_p() {
  check_table<P, 0>();
  check_table<P, 1>();
  check_mixed<P>();
}

int main() {
  check_p<1>();
  check_p<2>();
  check_p<3>();
  check_p<4>();
  check_p<5>();
  check_p<6>();
  check_p<7>();
  check_p<8>();
  std::printf("worst %.3e\n", worst);
  return worst < 1e-13 ? 0 : 1;
}
