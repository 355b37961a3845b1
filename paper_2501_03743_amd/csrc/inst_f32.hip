// FP32 instantiations of the outer iteration (inner solves of mixed-precision
// refinement; monomial and Chebyshev bases), s = 1..8.
#include "engine.hpp"

namespace ssp {

namespace {
template <int... Ss>
struct Table {
  static iter_fn<float> iter(int s) {
    iter_fn<float> f = nullptr;
    ((s == Ss ? (f = &sstep_iteration<Ss, float>, 0) : 0), ...);
    return f;
  }
  static iter_fn<float> cheb(int s) {
    iter_fn<float> f = nullptr;
    ((s == Ss ? (f = &sstep_cheb_iteration<Ss, float>, 0) : 0), ...);
    return f;
  }
};
using T32 = Table<1, 2, 3, 4, 5, 6, 7, 8>;
}  // namespace

iter_fn<float> iteration_f32(int s) { return T32::iter(s); }
iter_fn<float> cheb_iteration_f32(int s) { return T32::cheb(s); }

}  // namespace ssp
