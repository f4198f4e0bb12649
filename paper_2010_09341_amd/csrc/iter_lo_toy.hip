// Iteration kernels of one integrand (see vegas_iterate.hpp).
#include "vegas_iterate.hpp"

namespace vegas {

const void* iterate_kernel_lo_toy(int prec, int dim, bool dump) {
  return pick_integrand<kLoToy>(prec, dim, dump);
}

}  // namespace vegas
