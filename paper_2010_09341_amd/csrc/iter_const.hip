// Iteration kernels of one integrand (see vegas_iterate.hpp).
#include "vegas_iterate.hpp"

namespace vegas {

const void* iterate_kernel_const(int prec, int dim, bool dump) {
  return pick_integrand<kConst>(prec, dim, dump);
}

}  // namespace vegas
