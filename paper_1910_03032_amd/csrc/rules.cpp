// Host copies of the compile-time 1D rules and tables (see rules.h): the arrays the
// set-up kernels receive are bit-identical to the constants compiled into the
// operator kernels.
#include "rules.h"

#include "internal.h"

namespace sfem {
namespace {

template <int P>
void copy_rules(Rules1D &r) {
  using C = rules::Const<P>;
  constexpr int N = P + 1, Q = P + 2;
  r.p = P;
  r.q = Q;
  r.gll_x.assign(C::gll_rule.x, C::gll_rule.x + N);
  r.gll_w.assign(C::gll_rule.w, C::gll_rule.w + N);
  r.gauss_x.assign(C::gauss_rule.x, C::gauss_rule.x + Q);
  r.gauss_w.assign(C::gauss_rule.w, C::gauss_rule.w + Q);
  r.B.assign(&C::tab.B[0][0], &C::tab.B[0][0] + Q * N);
  r.G.assign(&C::tab.G[0][0], &C::tab.G[0][0] + Q * N);
}

}  // namespace

bool make_rules(int p, int q, Rules1D &r) {
  if (q != p + 2) return false;
  switch (p) {
    case 1: copy_rules<1>(r); return true;
    case 2: copy_rules<2>(r); return true;
    case 3: copy_rules<3>(r); return true;
    case 4: copy_rules<4>(r); return true;
    case 5: copy_rules<5>(r); return true;
    case 6: copy_rules<6>(r); return true;
    case 7: copy_rules<7>(r); return true;
    case 8: copy_rules<8>(r); return true;
    default: return false;
  }
}

}  // namespace sfem
