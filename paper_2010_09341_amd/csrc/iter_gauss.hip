// Iteration kernels of one integrand (see vegas_iterate.hpp).
#include "vegas_iterate.hpp"

namespace vegas {

const void* iterate_kernel_gauss(int prec, int dim, bool dump) {
  return pick_integrand<kGauss>(prec, dim, dump);
}

}  // namespace vegas
