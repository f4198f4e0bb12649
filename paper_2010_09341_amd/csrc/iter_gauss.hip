// Iteration kernels of one integrand (see vegas_iterate.hpp).
#include "vegas_iterate.hpp"

namespace vegas {

const void* iterate_kernel_gauss(int prec, int dim, bool dump) {
  return pick_integrand<kGauss>(prec, dim, dump);
}

const void* iterate_kernel_gauss8_rg() {
  return (const void*)k_iterate<8, kGauss, kFp32Eval, false, true>;
}

}  // namespace vegas
