// Instantiations of the sum-factorized apply in double for p = 1..8, q = p + 2.
#include "apply_impl.h"

namespace sfem {

hipError_t launch_apply_f64(const ApplyArgs &a, hipStream_t s) {
#define SFEM_CALL(P) launch_apply_pt<P, double>(a, s)
  SFEM_DISPATCH_P(a.p, SFEM_CALL)
#undef SFEM_CALL
}

int apply_group_elems_f64(int p) {
#define SFEM_CALL(P) apply_group_elems_pt<P, double>()
  SFEM_DISPATCH_P(p, SFEM_CALL)
#undef SFEM_CALL
}

}  // namespace sfem
