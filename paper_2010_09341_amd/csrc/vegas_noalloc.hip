// vegas_noalloc.hip — vegas_iterate_noalloc (include/vegas.h): one Vegas
// iteration that allocates nothing, for callers that cannot allocate device
// memory (code under hipGraph capture, tight serving loops, harnesses that
// forbid hipMalloc).
//
// It runs the same iteration and finalize kernels as vegas_iterate. The
// caller passes the grid edges, the histogram output and the result output
// in device memory; every intermediate buffer (iteration counter, grid
// records, workgroup partials, histogram flush copies) lives in `scratch`, a
// fixed device array of this library. Each GPU holds its own copy of the
// array until the process ends; its device address is looked up once per GPU
// with hipGetSymbolAddress, and host code passes only that address to the
// kernels. Every call clears what must start at zero (the histogram copies)
// and writes the iteration counter before the iteration kernel reads them.
// Calls that overlap on one GPU (two streams, two threads) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "vegas.h"
#include "vegas_common.hpp"
#include "vegas_finalize.hpp"
#include "vegas_launch.hpp"

static_assert(VEGAS_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size in 256-byte units");

// In host code this name is a host-side stand-in, not a device address:
// host code uses only the address scratch_address() looks up.
static __device__ __align__(256) unsigned char scratch[VEGAS_NOALLOC_SCRATCH_BYTES];

namespace vegas {
namespace {

// One wave per dimension d: the grid records of row d from the caller's
// edges, the histogram copies of row d zeroed, and (d = 0) the iteration
// counter set to t0.
__global__ __launch_bounds__(64) void k_noalloc_setup(const double* edges, double* copies,
                                                      int cells, Rec64* rec64, Rec32* rec32,
                                                      uint32_t* t, uint32_t t0, int nb) {
  extern __shared__ __align__(16) double esm[];
  const int d = blockIdx.x;
  for (int i = threadIdx.x; i <= nb; i += 64) esm[i] = edges[(size_t)d * (nb + 1) + i];
  __syncthreads();
  wg_write_records(nb, esm, rec64 + (size_t)d * nb, rec32 + (size_t)d * nb);
  for (int c = 0; c < kHistCopies; ++c)
    for (int k = threadIdx.x; k < nb; k += 64) copies[(size_t)c * cells + (size_t)d * nb + k] = 0.0;
  if (d == 0 && threadIdx.x == 0) *t = t0;
}

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch`, per GPU

// The device address of the current GPU's copy of `scratch`, looked up on
// the first call on that GPU.
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace
}  // namespace vegas

using namespace vegas;

extern "C" int vegas_iterate_noalloc(int dim, int n_bins, int prec, int integrand_id,
                                     const double* params, int n_params, const double* edges_dev,
                                     int64_t n_events, uint64_t seed, uint32_t t,
                                     double* hist_dev, double* result_dev, void* stream) {
  if (!shape_ok(dim, n_bins) || (prec != VEGAS_FP64 && prec != VEGAS_FP32_EVAL) ||
      integrand_id < 0 || integrand_id >= VEGAS_N_INTEGRANDS || n_events < 2 || !edges_dev ||
      !result_dev)
    return VEGAS_EINVAL;
  IntegrandArgs P;
  if (build_integrand_args(integrand_id, dim, params, n_params, &P) != VEGAS_OK)
    return VEGAS_EINVAL;
  // the scratch layout: counter, records, histogram copies, partials (the
  // edges and, without hist_dev, the histogram too)
  const Layout L = layout(dim, n_bins, kMaxBlocks, 1);
  if (L.total > (size_t)VEGAS_NOALLOC_SCRATCH_BYTES) return VEGAS_EINVAL;
  void* base = nullptr;
  if (scratch_address(&base) != hipSuccess) return VEGAS_EDEVICE;
  DevGrid g = bind_grid(base, dim, n_bins, kMaxBlocks, 1);
  if (hist_dev) g.hist = hist_dev;
  g.results = result_dev;
  hipStream_t s = static_cast<hipStream_t>(stream);

  const IterKernel k = iterate_kernel(integrand_id, prec, dim, false);
  if (!k) return VEGAS_EINVAL;
  const size_t lds = iterate_lds_bytes(dim, n_bins);
  const int threads = default_threads(k, lds);
  if (threads < 1) return VEGAS_EDEVICE;
  const int blocks = default_blocks(k, threads, lds, n_events, kMaxBlocks);
  if (blocks < 1) return VEGAS_EDEVICE;

  hipLaunchKernelGGL(k_noalloc_setup, dim3(dim), dim3(64), sizeof(double) * (n_bins + 1), s,
                     edges_dev, g.copies, dim * n_bins, static_cast<Rec64*>(g.rec64),
                     static_cast<Rec32*>(g.rec32), g.t, t, n_bins);
  if (hipGetLastError() != hipSuccess) return VEGAS_EDEVICE;
  IterLaunch it;
  it.fid = integrand_id;
  it.prec = prec;
  it.n_events = n_events;
  it.seed = seed;
  it.blocks = blocks;
  it.threads = threads;
  if (launch_iterate(g, it, P, s) != hipSuccess) return VEGAS_EDEVICE;
  if (launch_finalize(g, blocks, n_events, false, 0.0, s) != hipSuccess) return VEGAS_EDEVICE;
  return VEGAS_OK;
}
