// Instantiations of the sum-factorized apply in double for p = 1..8, q = p + 2.
#include "apply_impl.h"

namespace sfem {

hipError_t launch_apply_f64(const ApplyArgs &a, int64_t e_begin, int64_t e_end, hipStream_t s) {
#define SFEM_CALL(P) launch_apply_pt<P, double>(a, e_begin, e_end, s)
  SFEM_DISPATCH_P(a.p, SFEM_CALL)
#undef SFEM_CALL
}

}  // namespace sfem
