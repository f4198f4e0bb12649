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

// Grid record of bin k in dimension d, whose edges are lo = e_k and
// hi = e_{k+1} (binary64) and whose width is Delta = hi - lo.
//   FP64: {e, w} with w = Delta 2^-32 (exact) and e = lo + 2^-33 Delta
//         (rounded once), so that the point at fraction (l + 1/2) 2^-32 of
//         the bin, lo + that fraction times Delta, is one fma l w + e of the
//         remainder l converted exactly. e is within half an ulp of a number
//         no larger than the point, so the point keeps a relative error of a
//         few ulps wherever it lies in the bin (an origin shifted below lo
//         instead would cancel against l w near the lower edge of a bin
//         whose lower edge is small against its width, bin 0 above all).
//         Widths below 2^-990 lose bits in w (the weight is then below
//         that times the integrand).
//   FP32: {e, w} with w = Delta rounded to binary32 (the bin's own width,
//         not the difference of its rounded edges, so that a bin narrower
//         than the binary32 spacing at its position keeps its width), e =
//         lo - (1 - 2^-24) w rounded to binary32 (kRec32Shift: the point at
//         fraction (l' + 1/2) 2^-23 is e + (1 + l' 2^-23) w). Eight bytes:
//         one aligned 64-bit load per dimension and event.
constexpr double kRec64Half = 0x1p-33;
constexpr double kRec64Scale = 0x1p-32;
constexpr float kRec32Shift = 1.0f - 0x1p-24f;
struct Rec64 {
  double e, w;
};
struct alignas(8) Rec32 {
  float e, w;
};
static_assert(sizeof(Rec32) == 8, "binary32 grid record is two words");

// LDS of the iteration kernels' workgroups: `copies` histograms of w^2
// (binary64), interleaved per cell: the entry of cell (d, k) = d * nb + k in
// copy c is at index cell * copies + c, and lane l adds into copy
// l % copies. With 16 copies the 16 lanes that the LDS serves together hit 16
// distinct bank pairs whatever their bins, so the atomics never conflict
// (fewer copies for the largest grids, within the kernel's LDS budget; one
// copy of the largest grid, 8192 cells, takes 64 KiB, the single-integral
// kernel's budget; the serving kernel's budget is a target for its copies,
// and a grid above 4096 cells still gets its one copy there).
struct LdsLayout {
  uint32_t cells;
  uint32_t copies;  // 1, 2, 4, 8 or 16
  uint32_t cshift;  // log2(8 * copies): bytes per cell as a shift
};

// Copies and LDS budget of the single-integral iteration kernel (up to two
// 1024-thread workgroups per CU) and of the serving kernel (256-thread
// workgroups, four or more per CU; smaller chunks flush more often).
constexpr uint32_t kIterCopies = 16;
constexpr uint32_t kIterLdsBudget = 65536;
constexpr uint32_t kServeCopies = 8;
constexpr uint32_t kServeLdsBudget = 32768;

__host__ __device__ inline LdsLayout lds_layout(int dim, int nb, uint32_t max_copies,
                                                uint32_t budget) {
  LdsLayout L;
  L.cells = (uint32_t)(dim * nb);
  L.copies = max_copies;
  while (L.copies > 1u && 8u * L.cells * L.copies > budget) L.copies >>= 1;
  L.cshift = 3u;
  while ((1u << (L.cshift - 3u)) < L.copies) ++L.cshift;
  return L;
}

__host__ __device__ inline uint32_t lds_bytes(const LdsLayout& L) {
  return 8u * L.cells * L.copies;
}

// Workgroup partial slots and result-ring entries per integral.
constexpr int kMaxBlocks = 4096;
// Largest workgroup of the iteration kernel (any multiple of 64 up to it).
constexpr int kIterThreadsMax = 1024;
constexpr int kRing = 1024;

}  // namespace vegas
