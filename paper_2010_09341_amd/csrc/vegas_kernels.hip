// vegas_kernels.hip — the kernels of one Vegas iteration on gfx950.
//
//   k_iterate   (vegas_iterate.hpp, instantiated in iter_*.hip) draw, map,
//               integrand, moments, w^2 histogram
//   k_finalize  fixed-order reduction of the workgroup partials into (I, sigma),
//               of the histogram copies into the iteration's histogram, and
//               the refinement of every dimension (one wave per dimension)
//   k_refine    refinement from a histogram set by the host
//   k_init_grid / k_prepare / k_set_t   grid set-up and state writes
//
// The method: VegasFlow (arXiv:2010.09341) Sec. 1 (importance sampling on
// adaptive grids, after Lepage), Sec. 3.1 (integrand contract, iterations),
// Sec. 3.2 (each iteration informs the next). Nothing here is a dense
// contraction, so there is no MFMA; the iteration kernel is bound by vector
// ALU issue (integer multiplies of Philox, map and integrand arithmetic).
#include <hip/hip_runtime.h>

#include <atomic>
#include <type_traits>

#include "vegas_device.hpp"
#include "vegas_finalize.hpp"
#include "vegas_iterate.hpp"
#include "vegas_launch.hpp"

namespace vegas {

// ---------------------------------------------------------------------------
// finalize (+ refine): one wave per workgroup. Workgroup 0 reduces the
// iteration's workgroup partials (fixed order) into (I, sigma) at
// results[t % ring] and advances t; workgroup 1 + d reduces the histogram
// copies of dimension d into hist (zeroing the copies) and, when asked,
// refines dimension d from it.
// ---------------------------------------------------------------------------
struct FinArgs {
  uint32_t* t;
  const double* partials;
  double* results;
  double* results_host;
  double* copies;
  double* hist;
  double* edges;
  Rec64* rec64;
  Rec32* rec32;
  double n_events;
  double alpha;
  int blocks;
  int ring;
  int dim;
  int nb;
  int refine;
};

__global__ __launch_bounds__(64) void k_finalize(FinArgs a) {
  extern __shared__ __align__(16) double fsm[];
  if (blockIdx.x == 0) {
    wg_moments(a.partials, a.blocks, a.n_events, a.t, a.results, a.ring, nullptr,
               a.results_host);
    return;
  }
  const int d = blockIdx.x - 1;
  const int nb = a.nb;
  double* h = fsm;
  double* erow = a.edges + (size_t)d * (nb + 1);
  wg_reduce_hist(a.copies, a.hist + (size_t)d * nb, a.dim * nb, d, nb, h, erow,
                 a.refine ? fsm + nb : nullptr);
  if (a.refine)
    wg_refine_dim(nb, a.alpha, erow, h, a.rec64 + (size_t)d * nb, a.rec32 + (size_t)d * nb,
                  fsm + nb, true);
}

// refine from the stored histogram (after the histogram was set by the host)
struct RefArgs {
  double* edges;
  const double* hist;
  Rec64* rec64;
  Rec32* rec32;
  double alpha;
  int nb;
};

__global__ __launch_bounds__(64) void k_refine(RefArgs a) {
  extern __shared__ __align__(16) double rsm[];
  const int nb = a.nb;
  const int d = blockIdx.x;
  for (int k = threadIdx.x; k < nb; k += 64) rsm[k] = a.hist[(size_t)d * nb + k];
  __syncthreads();
  wg_refine_dim(nb, a.alpha, a.edges + (size_t)d * (nb + 1), rsm, a.rec64 + (size_t)d * nb,
                a.rec32 + (size_t)d * nb, rsm + nb);
}

// ---------------------------------------------------------------------------
// Set-up kernels: one wave per dimension.
// ---------------------------------------------------------------------------
struct GridArgs {
  uint32_t* t;
  double* edges;
  double* copies;
  Rec64* rec64;
  Rec32* rec32;
  int nb;
  int cells;
  int uniform;  // 1: write the uniform grid, zero the copies and t
};

__global__ __launch_bounds__(64) void k_grid(GridArgs a) {
  extern __shared__ __align__(16) double gsm[];
  const int nb = a.nb;
  const int d = blockIdx.x;
  double* erow = a.edges + (size_t)d * (nb + 1);
  if (a.uniform) {
    wg_uniform_dim(nb, erow, a.copies, a.cells, d, a.rec64 + (size_t)d * nb,
                   a.rec32 + (size_t)d * nb, gsm);
    if (d == 0 && threadIdx.x == 0) *a.t = 0;
  } else {
    for (int i = threadIdx.x; i <= nb; i += 64) gsm[i] = erow[i];
    __syncthreads();
    wg_write_records(nb, gsm, a.rec64 + (size_t)d * nb, a.rec32 + (size_t)d * nb);
  }
}

__global__ void k_set_t(uint32_t* t, uint32_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *t = v;
}

// ---------------------------------------------------------------------------
// Dispatch
// ---------------------------------------------------------------------------
static const void* builtin_kernel(int fid, int prec, int dim, bool dump) {
  switch (fid) {
    case kConst: return iterate_kernel_const(prec, dim, dump);
    case kSum: return iterate_kernel_sum(prec, dim, dump);
    case kGauss: return iterate_kernel_gauss(prec, dim, dump);
    case kLoToy: return iterate_kernel_lo_toy(prec, dim, dump);
    case kRambo24: return iterate_kernel_rambo24(prec, dim, dump);
    case kBwFlat: return iterate_kernel_bw_flat(prec, dim, dump);
    default: return nullptr;
  }
}

IterKernel iterate_kernel(int fid, int prec, int dim, bool dump) {
  if (dim < 1 || dim > kMaxDim || (prec != kFp64 && prec != kFp32Eval)) return IterKernel{};
  if (fid >= kUser) return user_iterate_kernel(fid, prec, dim, dump);
  IterKernel k;
  k.fn = builtin_kernel(fid, prec, dim, dump);
  return k;
}

hipError_t launch_kernel(const IterKernel& k, unsigned blocks, unsigned threads, void** args,
                         size_t lds, hipStream_t s) {
  if (k.fn) return hipLaunchKernel(k.fn, dim3(blocks), dim3(threads), args, lds, s);
  if (k.mf)
    return hipModuleLaunchKernel(k.mf, blocks, 1, 1, threads, 1, 1, (unsigned)lds, s, args,
                                 nullptr);
  return hipErrorInvalidValue;
}

size_t iterate_lds_bytes(int dim, int nb) {
  return lds_bytes(lds_layout(dim, nb, kIterCopies, kIterLdsBudget));
}

// CUs of the current device (read once per device), 0 if unknown.
static uint32_t device_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  int n = cache[dev].load(std::memory_order_relaxed);
  if (n < 1) {
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n < 1)
      return 0;
    cache[dev].store(n, std::memory_order_relaxed);
  }
  return (uint32_t)n;
}

// IterArgsDev::slot_cus for a grid: the CU count when the grid is a whole
// number of workgroups per CU and the workgroups whole groups of four waves.
static uint32_t slot_cus(int blocks, int threads) {
  const uint32_t cus = device_cus();
  return cus && blocks > 0 && (uint32_t)blocks % cus == 0 && threads % 256 == 0 ? cus : 0;
}

static IterArgsDev iter_args(const DevGrid& g, const IterLaunch& L) {
  IterArgsDev a;
  a.t = g.t;
  a.rec = L.prec == kFp64 ? g.rec64 : g.rec32;
  a.copies = g.copies;
  a.partials = g.partials;
  a.w_out = L.w_out;
  a.n_events = (uint64_t)L.n_events;
  a.first = L.first;
  a.accumulate = L.accumulate ? 1 : 0;
  a.seed_lo = (uint32_t)L.seed;
  a.seed_hi = (uint32_t)(L.seed >> 32);
  a.dim = g.dim;
  a.nb = (uint32_t)g.nb;
  a.lds = lds_layout(g.dim, g.nb, kIterCopies, kIterLdsBudget);
  a.slot_cus = slot_cus(L.blocks, L.threads);
  return a;
}

hipError_t launch_iterate(const DevGrid& g, const IterLaunch& L, const IntegrandArgs& P,
                          hipStream_t s) {
  const IterKernel k = iterate_kernel(L.fid, L.prec, g.dim, false);
  if (!k || L.blocks < 1 || L.blocks > g.max_blocks || L.threads < 64 ||
      L.threads > kIterThreadsMax || (L.threads & 63))
    return hipErrorInvalidValue;
  IterArgsDev a = iter_args(g, L);
  IntegrandArgs p = P;
  void* args[] = {&a, &p};
  return launch_kernel(k, (unsigned)L.blocks, (unsigned)L.threads, args,
                       iterate_lds_bytes(g.dim, g.nb), s);
}

hipError_t launch_dump(const DevGrid& g, const IterLaunch& L, const IntegrandArgs& P,
                       hipStream_t s) {
  const IterKernel k = iterate_kernel(L.fid, L.prec, g.dim, true);
  if (!k || L.count < 1 || !L.w_out) return hipErrorInvalidValue;
  IterArgsDev a = iter_args(g, L);
  a.n_events = (uint64_t)L.count;
  IntegrandArgs p = P;
  void* args[] = {&a, &p};
  const int threads = 256;
  int64_t blocks = (L.count + threads - 1) / threads;
  if (blocks > 4096) blocks = 4096;
  a.slot_cus = slot_cus((int)blocks, threads);
  return launch_kernel(k, (unsigned)blocks, (unsigned)threads, args,
                       iterate_lds_bytes(g.dim, g.nb), s);
}

hipError_t launch_finalize(const DevGrid& g, int blocks, int64_t n_events, bool refine,
                           double alpha, hipStream_t s) {
  if (blocks < 1 || blocks > g.max_blocks) return hipErrorInvalidValue;
  FinArgs a;
  a.t = g.t;
  a.partials = g.partials;
  a.results = g.results;
  a.results_host = g.results_host;
  a.copies = g.copies;
  a.hist = g.hist;
  a.edges = g.edges;
  a.rec64 = static_cast<Rec64*>(g.rec64);
  a.rec32 = static_cast<Rec32*>(g.rec32);
  a.n_events = (double)n_events;
  a.alpha = alpha;
  a.blocks = blocks;
  a.ring = g.ring;
  a.dim = g.dim;
  a.nb = g.nb;
  a.refine = refine ? 1 : 0;
  const size_t lds = sizeof(double) * (g.nb + refine_lds_doubles(g.nb));
  hipLaunchKernelGGL(k_finalize, dim3(1 + g.dim), dim3(64), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_refine(const DevGrid& g, double alpha, hipStream_t s) {
  RefArgs a;
  a.edges = g.edges;
  a.hist = g.hist;
  a.rec64 = static_cast<Rec64*>(g.rec64);
  a.rec32 = static_cast<Rec32*>(g.rec32);
  a.alpha = alpha;
  a.nb = g.nb;
  const size_t lds = sizeof(double) * (g.nb + refine_lds_doubles(g.nb));
  hipLaunchKernelGGL(k_refine, dim3(g.dim), dim3(64), lds, s, a);
  return hipGetLastError();
}

static hipError_t launch_grid(const DevGrid& g, int uniform, hipStream_t s) {
  GridArgs a;
  a.t = g.t;
  a.edges = g.edges;
  a.copies = g.copies;
  a.rec64 = static_cast<Rec64*>(g.rec64);
  a.rec32 = static_cast<Rec32*>(g.rec32);
  a.nb = g.nb;
  a.cells = g.dim * g.nb;
  a.uniform = uniform;
  hipLaunchKernelGGL(k_grid, dim3(g.dim), dim3(64), sizeof(double) * (g.nb + 1), s, a);
  return hipGetLastError();
}

hipError_t launch_init_grid(const DevGrid& g, hipStream_t s) { return launch_grid(g, 1, s); }
hipError_t launch_prepare(const DevGrid& g, hipStream_t s) { return launch_grid(g, 0, s); }

hipError_t launch_set_t(const DevGrid& g, uint32_t t, hipStream_t s) {
  hipLaunchKernelGGL(k_set_t, dim3(1), dim3(64), 0, s, g.t, t);
  return hipGetLastError();
}

}  // namespace vegas
