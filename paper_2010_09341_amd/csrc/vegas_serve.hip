// vegas_serve.hip — kernels of the serving loop: many integrals of different
// dimension, bin count, integrand and event count advance together, one
// iteration each per tick.
//
//   k_serve_init      uniform grid of newly admitted integrals (one wave per
//                     (integral, dimension))
//   k_serve_iterate   one workgroup per (integral, event chunk): the same
//                     draw / map / integrand / moments / histogram steps as
//                     the single-integral iteration kernel, with the chunk's
//                     partial sums written to the integral's chunk slot (so
//                     the estimate does not depend on what else runs)
//   k_serve_finalize  one wave per (integral, role): the moments of the
//                     iteration, or one dimension's histogram reduction and
//                     refinement
#include <hip/hip_runtime.h>

#include "vegas_device.hpp"
#include "vegas_finalize.hpp"
#include "vegas_serve.hpp"

namespace vegas {

template <int D_T, int FID, int PREC>
__device__ void serve_chunk(const SlotDev& S, uint32_t chunk, unsigned char* smem) {
  using Dm = Dims<D_T>;
  const LdsLayout L = lds_layout(S.dim, (int)S.nb, kServeCopies, kServeLdsBudget);
  const uint32_t t = *S.t;  // issued before the LDS clearing it can overlap
  zero_hist(L, smem);
  __syncthreads();
  const void* rec = PREC == kFp64 ? (const void*)S.rec64 : (const void*)S.rec32;
  const uint32_t lane_off = lane_hist_offset(L);
  const uint64_t begin = (uint64_t)chunk * S.chunk_events;
  uint64_t end = begin + S.chunk_events;
  if (end > S.n_events) end = S.n_events;
  double s1 = 0.0, s2 = 0.0;
  uint32_t bad = 0;
  uint32_t hist[Dm::kMax];
  for (uint64_t n = begin + threadIdx.x; n < end; n += blockDim.x) {
    double w = event_weight<D_T, FID, PREC>(n, t, S.seed_lo, S.seed_hi, S.dim, S.nb, rec,
                                            nullptr, lane_off, L.cshift, S.P, hist);
    if (!__builtin_isfinite(w)) {
      ++bad;
      w = 0.0;
    }
    const double w2 = w * w;
    s1 += w;
    s2 += w2;
#pragma unroll
    for (int d = 0; d < Dm::kMax; ++d)
      if (Dm::on(d, S.dim))
        __hip_atomic_fetch_add(static_cast<double*>(__builtin_assume_aligned(smem + hist[d], 8)),
                               w2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __shared__ double red[3][kServeThreads / 64];
  s1 = wave_total(s1);
  s2 = wave_total(s2);
  bad = wave_total_u32(bad);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wid] = s1;
    red[1][wid] = s2;
    red[2][wid] = (double)bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a1 = 0.0, a2 = 0.0, ab = 0.0;
    for (int w = 0; w < kServeThreads / 64; ++w) {
      a1 += red[0][w];
      a2 += red[1][w];
      ab += red[2][w];
    }
    double* p = S.partials + 4 * (size_t)chunk;
    p[0] = a1;
    p[1] = a2;
    p[2] = ab;
    p[3] = 0.0;
  }
  flush_hist(L, smem, S.copies + (size_t)(chunk % kHistCopies) * L.cells);
  __syncthreads();  // the LDS is reused by the next work item
}

// Work items of one precision and dimension class (at most -D_T dimensions).
template <int D_T, int PREC>
__global__ __launch_bounds__(kServeThreads) void k_serve_iterate(const SlotDev* slots,
                                                                 const WorkItem* items,
                                                                 int n_items) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const WorkItem w = items[it];
    const SlotDev& S = slots[w.slot];
    switch (S.fid) {
      case kConst: serve_chunk<D_T, kConst, PREC>(S, w.chunk, smem); break;
      case kSum: serve_chunk<D_T, kSum, PREC>(S, w.chunk, smem); break;
      case kGauss: serve_chunk<D_T, kGauss, PREC>(S, w.chunk, smem); break;
      case kLoToy: serve_chunk<D_T, kLoToy, PREC>(S, w.chunk, smem); break;
      case kRambo24: serve_chunk<D_T, kRambo24, PREC>(S, w.chunk, smem); break;
      case kBwFlat: serve_chunk<D_T, kBwFlat, PREC>(S, w.chunk, smem); break;
      default: break;
    }
  }
}

__global__ __launch_bounds__(64) void k_serve_finalize(const SlotDev* slots, const FinItem* items,
                                                       int n_items, double* out) {
  extern __shared__ __align__(16) double fsm[];
  if ((int)blockIdx.x >= n_items) return;
  const FinItem f = items[blockIdx.x];
  const SlotDev& S = slots[f.slot];
  const int nb = (int)S.nb;
  if (f.role < 0) {
    wg_moments(S.partials, (int)S.n_chunks, (double)S.n_events, S.t, S.results, S.ring,
               out + 4 * (size_t)f.out);
    return;
  }
  const int d = f.role;
  double* erow = S.edges + (size_t)d * (nb + 1);
  wg_reduce_hist(S.copies, S.hist + (size_t)d * nb, S.dim * nb, d, nb, fsm, erow,
                 f.refine ? fsm + nb : nullptr);
  if (f.refine)
    wg_refine_dim(nb, S.alpha, erow, fsm, S.rec64 + (size_t)d * nb, S.rec32 + (size_t)d * nb,
                  fsm + nb, true);
}

// New integrals: f.out indexes their descriptor in `fresh` (the tick's input
// buffer); the wave of dimension 0 also installs it in slots[f.slot], which
// the later kernels of the tick read.
__global__ __launch_bounds__(64) void k_serve_init(SlotDev* slots, const FinItem* items,
                                                   int n_items, const SlotDev* fresh) {
  extern __shared__ __align__(16) double ism[];
  if ((int)blockIdx.x >= n_items) return;
  const FinItem f = items[blockIdx.x];
  const SlotDev& S = fresh[f.out];
  const int nb = (int)S.nb;
  const int d = f.role;
  if (d == 0) {
    static_assert(sizeof(SlotDev) % 4 == 0, "descriptor copied in 32-bit words");
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&S);
    uint32_t* dst = reinterpret_cast<uint32_t*>(slots + f.slot);
    for (int i = threadIdx.x; i < (int)(sizeof(SlotDev) / 4); i += 64) dst[i] = src[i];
  }
  wg_uniform_dim(nb, S.edges + (size_t)d * (nb + 1), S.copies, S.dim * nb, d,
                 S.rec64 + (size_t)d * nb, S.rec32 + (size_t)d * nb, ism);
  if (d == 0 && threadIdx.x == 0) *S.t = 0;
}

hipError_t launch_serve_iterate(int dmax, int prec, const SlotDev* slots, const WorkItem* items,
                                int n_items, int max_lds, hipStream_t s) {
  if (n_items < 1) return hipSuccess;
  const size_t lds = (size_t)max_lds;
  const int blocks = n_items < kServeMaxBlocks ? n_items : kServeMaxBlocks;
  void* args[] = {&slots, &items, &n_items};
  const void* k = nullptr;
  if (dmax == 16)
    k = prec == kFp64 ? (const void*)k_serve_iterate<-16, kFp64>
                      : (const void*)k_serve_iterate<-16, kFp32Eval>;
  else if (dmax == 32)
    k = prec == kFp64 ? (const void*)k_serve_iterate<-32, kFp64>
                      : (const void*)k_serve_iterate<-32, kFp32Eval>;
  if (!k) return hipErrorInvalidValue;
  return hipLaunchKernel(k, dim3(blocks), dim3(kServeThreads), args, lds, s);
}

hipError_t launch_serve_finalize(const SlotDev* slots, const FinItem* items, int n_items,
                                 int max_nb, double* out, hipStream_t s) {
  if (n_items < 1) return hipSuccess;
  const size_t lds = sizeof(double) * (max_nb + refine_lds_doubles(max_nb));
  hipLaunchKernelGGL(k_serve_finalize, dim3(n_items), dim3(64), lds, s, slots, items, n_items, out);
  return hipGetLastError();
}

// A tick's packed inputs, 16 bytes per thread, from pinned host memory
// mapped into the device's address space into device memory.
__global__ __launch_bounds__(256) void k_serve_stage(const uint4* src, uint4* dst, uint32_t n16) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < n16) dst[i] = src[i];
}

hipError_t launch_serve_stage(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t n16 = (bytes + 15) / 16;
  if (n16 == 0) return hipSuccess;
  if (!src || !dst || n16 > 0xFFFFFFFFu) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_serve_stage, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, s,
                     static_cast<const uint4*>(src), static_cast<uint4*>(dst), (uint32_t)n16);
  return hipGetLastError();
}

hipError_t launch_serve_init(SlotDev* slots, const FinItem* items, int n_items, int max_nb,
                             const SlotDev* fresh, hipStream_t s) {
  if (n_items < 1) return hipSuccess;
  hipLaunchKernelGGL(k_serve_init, dim3(n_items), dim3(64), sizeof(double) * (max_nb + 1), s,
                     slots, items, n_items, fresh);
  return hipGetLastError();
}

}  // namespace vegas
