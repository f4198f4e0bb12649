// vegas_common.hpp — host-side helpers shared by the handle API and the
// serving scheduler (workspace layout, parameter preparation, combination).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "vegas.h"
#include "vegas_launch.hpp"
#include "vegas_types.hpp"

namespace vegas {

// Byte offsets of one integral's device state inside its workspace.
struct Layout {
  size_t t, edges, hist, copies, rec64, rec32, partials, results, total;
};

const char* status_name(int s);
bool shape_ok(int dim, int nb);
// max_partials workgroup/chunk partial slots, ring result entries.
Layout layout(int dim, int nb, int max_partials = kMaxBlocks, int ring = kRing);
DevGrid bind_grid(void* ws, int dim, int nb, int max_partials = kMaxBlocks, int ring = kRing);
// Derived integrand constants; VEGAS_OK or VEGAS_EINVAL. out may be NULL.
int build_integrand_args(int fid, int dim, const double* p, int np, IntegrandArgs* out);
// Workgroups for the iteration kernel: enough to fill the GPU at its
// occupancy, no more than the events need, at most cap. -1 on HIP error.
int default_blocks(const IterKernel& kernel, int threads, size_t lds, int64_t n_events, int cap);
// Threads per workgroup for the iteration kernel: of 1024, 512, 256, 128 and
// 64, up to the largest the kernel was built for, the one that keeps the most
// waves resident per CU (the larger on a tie). -1 on HIP error.
int default_threads(const IterKernel& kernel, size_t lds);
// Largest workgroup the kernel was built for; -1 on HIP error.
int kernel_max_threads(const IterKernel& kernel);
// Whether fid names a built-in integrand or the range of run-time ones.
inline bool integrand_id_ok(int fid) {
  return (fid >= 0 && fid < VEGAS_N_INTEGRANDS) ||
         (fid >= VEGAS_F_USER && fid < VEGAS_F_USER + VEGAS_MAX_USER);
}
// Inverse-variance combination of iteration results and chi^2 per dof.
void combine(const std::vector<double>& I_t, const std::vector<double>& s_t, double* I,
             double* sigma, double* chi2);

}  // namespace vegas
