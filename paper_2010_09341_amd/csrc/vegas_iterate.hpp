// vegas_iterate.hpp — the iteration kernel template: draw (Philox4x32-10 in
// registers) -> grid map (records through the vector cache) -> integrand -> sum w, sum w^2
// (binary64, DPP wave sums + LDS) -> w^2 histogram (LDS-private binary64
// atomics, flushed with global binary64 atomics into one of 8 copies chosen by
// workgroup index, i.e. by XCD under round-robin dispatch).
//
// Each integrand's instantiations live in their own translation unit
// (iter_*.hip) so they compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "vegas_device.hpp"

namespace vegas {

struct IterArgsDev {
  const uint32_t* t;
  const void* rec;
  double* copies;
  double* partials;
  double* w_out;
  uint64_t n_events;  // events of this launch (dump: number of events to dump)
  uint64_t first;     // index of the launch's first event
  int accumulate;     // add to the workgroup partials of earlier launches
  LdsLayout lds;
  uint32_t seed_lo, seed_hi;
  int dim;
  uint32_t nb;
  // CUs of the device when the grid is a whole number of workgroups per CU of
  // whole groups of four waves, else 0 (the order of the event slots)
  uint32_t slot_cus;
};

// Largest workgroup of an iteration kernel. A 1024-thread workgroup keeps 4
// waves on every SIMD, which caps a thread at 128 VGPRs; kernels that need
// more (binary64 RAMBO, binary64 above 12 dimensions and at 11, the run-time
// dimension classes) are built for 256-thread workgroups instead, so that
// they do not spill. (The 11-dimension binary64 kernel exceeds 128 VGPRs by a
// few where the 12-dimension one, scheduled differently, does not.)
template <int D_T, int FID, int PREC>
constexpr int iter_threads_max() {
  if (FID == kRambo24) return PREC == kFp64 ? 256 : 1024;
  if (D_T < 0) return 256;
  if (PREC == kFp32Eval) return 1024;
  return (D_T <= 10 || D_T == 12) ? 1024 : 256;
}

// Waves per SIMD a kernel is built to keep resident (the register budget):
// 8 (64 VGPRs, two 1024-thread workgroups per CU) for the binary32 kernels of
// up to 9 dimensions, 4 (128 VGPRs) for the binary64 kernels of 9 to 13
// dimensions, whose event loops fit in that many registers without spilling;
// otherwise no bound beyond the workgroup size.
template <int D_T, int FID, int PREC>
constexpr int iter_min_waves() {
  if (FID == kRambo24 || D_T < 0) return 1;
  if (PREC == kFp32Eval) return D_T <= 9 ? 8 : 1;
  return (D_T >= 9 && D_T <= 13) ? 4 : 1;
}

template <int D_T, int FID, int PREC, bool DUMP, class U = NoUser>
__global__ __launch_bounds__((iter_threads_max<D_T, FID, PREC>()))
__attribute__((amdgpu_waves_per_eu(iter_min_waves<D_T, FID, PREC>()))) void k_iterate(
    IterArgsDev a, IntegrandArgs P) {
  extern __shared__ __align__(16) unsigned char smem[];
  using Dm = Dims<D_T>;
  const LdsLayout L = a.lds;
  // the iteration counter (written by the previous finalize) is read first,
  // so that its memory latency overlaps the clearing of the LDS histogram
  const uint32_t t = *a.t;
  if constexpr (!DUMP) {
    zero_hist(L, smem);
    __syncthreads();
  }

  // per-dimension LDS bases held in registers, except where registers are
  // short (the kernels built for 256-thread workgroups)
  constexpr bool kHoist = D_T > 0 && iter_threads_max<D_T, FID, PREC>() == 1024;
  const uint32_t lane_off = lane_hist_offset(L);
  uint32_t hb[Dm::kMax];
  if constexpr (kHoist) lane_hist_bases<Dm::kMax>(L, (int)a.nb, hb);
  // Grid stride over events, 64 events per wave slot; the order of the slots
  // decides where a partial last stride runs. With slot_cus = C (the grid is
  // k workgroups per CU, workgroup b on the CU of b mod C, and four waves in a
  // row of a workgroup on four different SIMDs) slot s goes to CU s mod C and,
  // within the CU, runs through the waves four at a time (0-3 of each of its
  // k workgroups, then 4-7, ...), so that any number of leading slots loads
  // the SIMDs of all CUs evenly. Otherwise slot s = v * gridDim.x + b, which
  // spreads over workgroups first.
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t n;
  {
    const uint32_t v = threadIdx.x >> 6, b = blockIdx.x;
    uint32_t s;
    if (a.slot_cus) {
      const uint32_t j = b / a.slot_cus, c = b - j * a.slot_cus, k = gridDim.x / a.slot_cus;
      s = ((((v >> 2) * k + j) << 2) | (v & 3)) * a.slot_cus + c;
    } else {
      s = v * gridDim.x + b;
    }
    n = (uint64_t)s * 64 + (threadIdx.x & 63);
  }
  uint32_t hist[Dm::kMax];

  if constexpr (DUMP) {
    for (; n < a.n_events; n += stride)
      a.w_out[n] = event_weight<D_T, FID, PREC, U, kHoist>(a.first + n, t, a.seed_lo, a.seed_hi, a.dim,
                                                a.nb, a.rec, hb,
                                                lane_off, L.cshift, P, hist);
    return;
  } else {
    double s1 = 0.0, s2 = 0.0;
    uint32_t bad = 0;
    for (; n < a.n_events; n += stride) {
      double w = event_weight<D_T, FID, PREC, U, kHoist>(a.first + n, t, a.seed_lo, a.seed_hi, a.dim, a.nb,
                                              a.rec, hb, lane_off,
                                              L.cshift, P, hist);
      if (!__builtin_isfinite(w)) {
        ++bad;
        w = 0.0;
      }
      const double w2 = w * w;
      s1 += w;
      s2 += w2;
#pragma unroll
      for (int d = 0; d < Dm::kMax; ++d)
        if (Dm::on(d, a.dim))
          __hip_atomic_fetch_add(static_cast<double*>(__builtin_assume_aligned(smem + hist[d], 8)),
                                 w2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }

    __shared__ double red[3][kIterThreadsMax / 64];
    s1 = wave_total(s1);
    s2 = wave_total(s2);
    bad = wave_total_u32(bad);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
      red[0][wid] = s1;
      red[1][wid] = s2;
      red[2][wid] = (double)bad;
    }
    __syncthreads();  // also orders every LDS histogram update before the flush
    if (threadIdx.x == 0) {
      double a1 = 0.0, a2 = 0.0, ab = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        a1 += red[0][w];
        a2 += red[1][w];
        ab += red[2][w];
      }
      double* p = a.partials + 4 * (size_t)blockIdx.x;
      if (a.accumulate) {
        p[0] += a1;
        p[1] += a2;
        p[2] += ab;
      } else {
        p[0] = a1;
        p[1] = a2;
        p[2] = ab;
        p[3] = 0.0;
      }
    }
    flush_hist(L, smem, a.copies + (size_t)(blockIdx.x % kHistCopies) * L.cells);
  }
}

// Kernel of one integrand for `dim` dimensions: exact dimension counts up to
// 16, and 20/24/28/32 with the count given at run time above that.
template <int FID, int PREC, bool DUMP>
const void* pick_dims(int dim) {
  if constexpr (FID == kLoToy) {
    return dim == 4 ? (const void*)k_iterate<4, FID, PREC, DUMP> : nullptr;
  } else if constexpr (FID == kRambo24) {
    return dim == 16 ? (const void*)k_iterate<16, FID, PREC, DUMP> : nullptr;
  } else {
    switch (dim) {
      case 1: return (const void*)k_iterate<1, FID, PREC, DUMP>;
      case 2: return (const void*)k_iterate<2, FID, PREC, DUMP>;
      case 3: return (const void*)k_iterate<3, FID, PREC, DUMP>;
      case 4: return (const void*)k_iterate<4, FID, PREC, DUMP>;
      case 5: return (const void*)k_iterate<5, FID, PREC, DUMP>;
      case 6: return (const void*)k_iterate<6, FID, PREC, DUMP>;
      case 7: return (const void*)k_iterate<7, FID, PREC, DUMP>;
      case 8: return (const void*)k_iterate<8, FID, PREC, DUMP>;
      case 9: return (const void*)k_iterate<9, FID, PREC, DUMP>;
      case 10: return (const void*)k_iterate<10, FID, PREC, DUMP>;
      case 11: return (const void*)k_iterate<11, FID, PREC, DUMP>;
      case 12: return (const void*)k_iterate<12, FID, PREC, DUMP>;
      case 13: return (const void*)k_iterate<13, FID, PREC, DUMP>;
      case 14: return (const void*)k_iterate<14, FID, PREC, DUMP>;
      case 15: return (const void*)k_iterate<15, FID, PREC, DUMP>;
      case 16: return (const void*)k_iterate<16, FID, PREC, DUMP>;
      default: break;
    }
    if (dim >= 17 && dim <= 20) return (const void*)k_iterate<-20, FID, PREC, DUMP>;
    if (dim >= 21 && dim <= 24) return (const void*)k_iterate<-24, FID, PREC, DUMP>;
    if (dim >= 25 && dim <= 28) return (const void*)k_iterate<-28, FID, PREC, DUMP>;
    if (dim >= 29 && dim <= 32) return (const void*)k_iterate<-32, FID, PREC, DUMP>;
    return nullptr;
  }
}

template <int FID>
const void* pick_integrand(int prec, int dim, bool dump) {
  if (prec == kFp64) return dump ? pick_dims<FID, kFp64, true>(dim) : pick_dims<FID, kFp64, false>(dim);
  return dump ? pick_dims<FID, kFp32Eval, true>(dim) : pick_dims<FID, kFp32Eval, false>(dim);
}

// One per translation unit iter_*.hip.
const void* iterate_kernel_const(int prec, int dim, bool dump);
const void* iterate_kernel_sum(int prec, int dim, bool dump);
const void* iterate_kernel_gauss(int prec, int dim, bool dump);
const void* iterate_kernel_lo_toy(int prec, int dim, bool dump);
const void* iterate_kernel_rambo24(int prec, int dim, bool dump);
const void* iterate_kernel_bw_flat(int prec, int dim, bool dump);

}  // namespace vegas
