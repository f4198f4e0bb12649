// vegas_types.hpp — plain data types shared by the kernels and the host
// runtime of the Vegas library (no device code).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace vegas {

// Integrand identifiers (the VEGAS_F_* values of the C interface).
enum : int { kConst = 0, kSum = 1, kGauss = 2, kLoToy = 3, kRambo24 = 4, kBwFlat = 5 };
// Integrands compiled at run time (the VEGAS_F_USER range of the C interface).
constexpr int kUser = 64;
constexpr int kMaxUser = 64;
constexpr int kUserParams = 32;  // parameters of a run-time integrand (IntegrandArgs::c64/c32)
enum : int { kFp64 = 0, kFp32Eval = 1 };

constexpr int kMaxDim = 32;
// Global histogram copies: workgroup b flushes its LDS histogram into copy
// b % kHistCopies, one per XCD under round-robin workgroup dispatch, so the
// flush atomics of different XCDs never meet on one address.
constexpr int kHistCopies = 8;

// Derived integrand constants, filled on the host from the user's parameters.
struct IntegrandArgs {
  double d[8];
  double c64[kMaxDim];  // Gaussian centres; a run-time integrand's parameters
  float f[8];
  float c32[kMaxDim];
  int mode;
  int pad[3];
};

// Grid record of bin k in dimension d.
//   FP64: {e_k, e_{k+1} - e_k}
//   FP32: {e_k, delta_k} with e_k rounded to binary32 and delta_k the
//         binary32 difference of the rounded edges, so that e_k + delta_k
//         lands on the rounded e_{k+1}.
struct Rec64 {
  double e, w;
};
struct alignas(8) Rec32 {
  float e, w;
};

// LDS of the iteration kernels' workgroups: `copies` histograms of w^2
// (binary64) for the cells (d, k) = d * nb + k, copy stride cstride entries;
// lane l adds into copy l % copies, which splits the lanes of a wave that hit
// the same bin. The grid records are read through the vector cache, so every
// LDS access is a binary64 atomic at an 8-byte stride. At most 64 KiB.
struct LdsLayout {
  uint32_t cells;
  uint32_t cstride;  // histogram copy stride in entries
  uint32_t copies;   // 1, 2 or 4
};

__host__ __device__ inline LdsLayout lds_layout(int dim, int nb) {
  LdsLayout L;
  L.cells = (uint32_t)(dim * nb);
  L.cstride = L.cells + 4u;
  L.copies = 4u;
  while (L.copies > 1u && 8u * L.cstride * L.copies > 65536u) L.copies >>= 1;
  return L;
}

__host__ __device__ inline uint32_t lds_bytes(const LdsLayout& L) {
  return 8u * L.cstride * L.copies;
}

// Workgroup partial slots and result-ring entries per integral.
constexpr int kMaxBlocks = 4096;
constexpr int kRing = 1024;

}  // namespace vegas
