// vegas_types.hpp — plain data types shared by the kernels and the host
// runtime of the Vegas library (no device code).
#pragma once

#include <stdint.h>

namespace vegas {

// Integrand identifiers (the VEGAS_F_* values of the C interface).
enum : int { kConst = 0, kSum = 1, kGauss = 2, kLoToy = 3, kRambo24 = 4, kBwFlat = 5 };
enum : int { kFp64 = 0, kFp32Eval = 1 };

constexpr int kMaxDim = 32;
// Global histogram copies: workgroup b flushes its LDS histogram into copy
// b % kHistCopies, one per XCD under round-robin workgroup dispatch, so the
// flush atomics of different XCDs never meet on one address.
constexpr int kHistCopies = 8;

// Derived integrand constants, filled on the host from the user's parameters.
struct IntegrandArgs {
  double d[8];
  double c64[kMaxDim];  // Gaussian centres
  float f[8];
  float c32[kMaxDim];
  int mode;
  int pad[3];
};

// Grid record of bin k in dimension d.
//   FP64: {e_k, e_{k+1} - e_k}
//   FP32: {e_k, delta_k, log2(nb * delta_k), 0} with e_k rounded to binary32
//         and delta_k the binary32 difference of the rounded edges, so that
//         e_k + delta_k lands on the rounded e_{k+1}.
struct Rec64 {
  double e, w;
};
struct alignas(16) Rec32 {
  float e, w, l2j, pad;
};

// Workgroup partial slots and result-ring entries per integral.
constexpr int kMaxBlocks = 4096;
constexpr int kRing = 1024;

}  // namespace vegas
