// Even-odd (symmetry) form of the 1D contractions.
//
// The GLL nodes and the Gauss points are symmetric about 0, so the tables satisfy
// B(q-1-a, n-1-i) = B(a, i) and G(q-1-a, n-1-i) = -G(a, i) (Section 6 remarks that
// these symmetries can be exploited).  Splitting an input line v into
// e_i = v_i + v_{n-1-i} and o_i = v_i - v_{n-1-i} turns each pair of outputs (a, q-1-a)
// into E +- O with E = sum_i Te(a,i) e_i, O = sum_i To(a,i) o_i, where
// Te(a,i) = (T(a,i) + T(a,n-1-i)) / 2 and To(a,i) = (T(a,i) - T(a,n-1-i)) / 2:
// half the multiply-adds and half the distinct table constants.
//
// The same half tables serve the transposed contraction out_i = sum_a T(a,i) in_a,
// accumulated one input pair (a, q-1-a) at a time (EoAcc).
#pragma once

#include "rules.h"

#if defined(__HIPCC__)
#define SFEM_HD __host__ __device__ __forceinline__
#else
#define SFEM_HD inline
#endif

namespace sfem {
namespace eo {

// Table accessors for order P (q = P + 2): WHICH 0 = B (symmetric), 1 = G (antisymmetric).
template <int P, int WHICH>
struct Tab1 {
  static constexpr int NO = P + 2, NI = P + 1;
  static constexpr int S = WHICH == 0 ? 1 : -1;
  static constexpr rules::Tables<P, P + 2> c = rules::tables<P, P + 2>();
  static constexpr double t(int a, int i) { return WHICH == 0 ? c.B[a][i] : c.G[a][i]; }
  static constexpr double e(int a, int i) { return 0.5 * (t(a, i) + t(a, NI - 1 - i)); }
  static constexpr double o(int a, int i) { return 0.5 * (t(a, i) - t(a, NI - 1 - i)); }
};

// Split of a line of length L: e[i] = v[i] + v[L-1-i], o[i] = v[i] - v[L-1-i] (i < L/2);
// for odd L, e[L/2] = v[L/2] (the middle entry).
template <int L, typename T>
struct Split {
  T e[(L + 1) / 2];
  T o[L / 2 > 0 ? L / 2 : 1];
};

template <int L, typename T>
SFEM_HD Split<L, T> split(const T (&v)[L]) {
  Split<L, T> s;
#pragma unroll
  for (int i = 0; i < L / 2; ++i) {
    s.e[i] = v[i] + v[L - 1 - i];
    s.o[i] = v[i] - v[L - 1 - i];
  }
  if constexpr (L % 2 == 1) s.e[L / 2] = v[L / 2];
  return s;
}

// out[a] = sum_i T(a, i) v[i] for the table TB (NO x NI), from the split of v.
template <typename TB, typename T, int NO = TB::NO, int NI = TB::NI>
SFEM_HD void apply(const Split<NI, T> &x, T (&out)[NO]) {
  constexpr int HI = NI / 2, HO = NO / 2;
#pragma unroll
  for (int a = 0; a < HO; ++a) {
    T E = 0, O = 0;
#pragma unroll
    for (int i = 0; i < HI; ++i) {
      E += (T)TB::e(a, i) * x.e[i];
      O += (T)TB::o(a, i) * x.o[i];
    }
    if constexpr (NI % 2 == 1) E += (T)TB::t(a, HI) * x.e[HI];
    out[a] = E + O;
    out[NO - 1 - a] = (TB::S > 0) ? (E - O) : (O - E);
  }
  if constexpr (NO % 2 == 1) {
    T M = 0;
#pragma unroll
    for (int i = 0; i < HI; ++i) M += (T)TB::t(HO, i) * (TB::S > 0 ? x.e[i] : x.o[i]);
    if constexpr (NI % 2 == 1 && TB::S > 0) M += (T)TB::t(HO, HI) * x.e[HI];
    out[HO] = M;
  }
}

// Transposed contraction out[i] = sum_a T(a, i) in[a] (NI outputs), accumulated one input
// pair (a, NO-1-a) -- or the middle input -- at a time.
template <int NI, typename T>
struct Acc {
  T E[(NI + 1) / 2];
  T O[NI / 2 > 0 ? NI / 2 : 1];
  SFEM_HD void zero() {
#pragma unroll
    for (int i = 0; i < (NI + 1) / 2; ++i) E[i] = T(0);
#pragma unroll
    for (int i = 0; i < NI / 2; ++i) O[i] = T(0);
  }
  // add T(a, .) in_a + T(NO-1-a, .) in_b for a < NO/2 (in_a at a, in_b at NO-1-a)
  template <typename TB>
  SFEM_HD void add_pair(int a, T in_a, T in_b) {
    const T sp = in_a + in_b, sm = in_a - in_b;
    const T ue = TB::S > 0 ? sp : sm, uo = TB::S > 0 ? sm : sp;
#pragma unroll
    for (int i = 0; i < NI / 2; ++i) {
      E[i] += (T)TB::e(a, i) * ue;
      O[i] += (T)TB::o(a, i) * uo;
    }
    if constexpr (NI % 2 == 1) E[NI / 2] += (T)TB::t(a, NI / 2) * ue;
  }
  // add T(m, .) in_m for the middle input m = NO/2 of an odd NO
  template <typename TB>
  SFEM_HD void add_mid(T in_m) {
    constexpr int m = TB::NO / 2;
#pragma unroll
    for (int i = 0; i < NI / 2; ++i) {
      E[i] += (T)TB::e(m, i) * in_m;
      O[i] += (T)TB::o(m, i) * in_m;
    }
    if constexpr (NI % 2 == 1) E[NI / 2] += (T)TB::t(m, NI / 2) * in_m;
  }
  SFEM_HD void finish(T (&out)[NI]) const {
#pragma unroll
    for (int i = 0; i < NI / 2; ++i) {
      out[i] = E[i] + O[i];
      out[NI - 1 - i] = E[i] - O[i];
    }
    if constexpr (NI % 2 == 1) out[NI / 2] = E[NI / 2];
  }
};

}  // namespace eo
}  // namespace sfem
