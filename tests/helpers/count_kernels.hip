// The iteration kernels whose event loops tests/test_valu_count.py counts:
// the 8-D Gaussian and the LO toy in both precisions, RAMBO 2->4 in FP32-eval.
#include "vegas_iterate.hpp"

namespace vegas {
template __global__ void k_iterate<8, kGauss, kFp32Eval, false, NoUser>(IterArgsDev, IntegrandArgs);
template __global__ void k_iterate<8, kGauss, kFp64, false, NoUser>(IterArgsDev, IntegrandArgs);
template __global__ void k_iterate<4, kLoToy, kFp32Eval, false, NoUser>(IterArgsDev, IntegrandArgs);
template __global__ void k_iterate<4, kLoToy, kFp64, false, NoUser>(IterArgsDev, IntegrandArgs);
template __global__ void k_iterate<16, kRambo24, kFp32Eval, false, NoUser>(IterArgsDev, IntegrandArgs);
}  // namespace vegas
