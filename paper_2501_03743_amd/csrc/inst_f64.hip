// FP64 instantiations of the outer iteration (monomial and Chebyshev bases),
// s = 1..16.
#include "engine.hpp"

namespace ssp {

namespace {
template <int... Ss>
struct Table {
  static iter_fn<double> iter(int s) {
    iter_fn<double> f = nullptr;
    ((s == Ss ? (f = &sstep_iteration<Ss, double>, 0) : 0), ...);
    return f;
  }
  static iter_fn<double> cheb(int s) {
    iter_fn<double> f = nullptr;
    ((s == Ss ? (f = &sstep_cheb_iteration<Ss, double>, 0) : 0), ...);
    return f;
  }
  static cheb_basis_fn chebb(int s) {
    cheb_basis_fn f = nullptr;
    ((s == Ss ? (f = &cheb_basis_only<Ss>, 0) : 0), ...);
    return f;
  }
  static mpk_fn mpk(int s) {
    mpk_fn f = nullptr;
    ((s == Ss ? (f = &mpk_only<Ss>, 0) : 0), ...);
    return f;
  }
};
using T64 = Table<1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16>;
}  // namespace

iter_fn<double> iteration_f64(int s) { return T64::iter(s); }
iter_fn<double> cheb_iteration_f64(int s) { return T64::cheb(s); }
mpk_fn mpk_f64(int s) { return T64::mpk(s); }
cheb_basis_fn cheb_basis_f64(int s) { return T64::chebb(s); }

}  // namespace ssp
