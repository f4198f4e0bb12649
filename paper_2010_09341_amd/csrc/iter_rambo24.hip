// Iteration kernels of one integrand (see vegas_iterate.hpp).
#include "vegas_iterate.hpp"

namespace vegas {

const void* iterate_kernel_rambo24(int prec, int dim, bool dump) {
  return pick_integrand<kRambo24>(prec, dim, dump);
}

}  // namespace vegas
