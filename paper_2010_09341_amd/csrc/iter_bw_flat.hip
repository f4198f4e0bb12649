// Iteration kernels of one integrand (see vegas_iterate.hpp).
#include "vegas_iterate.hpp"

namespace vegas {

const void* iterate_kernel_bw_flat(int prec, int dim, bool dump) {
  return pick_integrand<kBwFlat>(prec, dim, dump);
}

}  // namespace vegas
