// vegas_launch.hpp — host-side launch interface of the Vegas kernels.
// Plain C++ types only, so the runtime (vegas_runtime.cpp) needs no device code.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace vegas {

struct IntegrandArgs;

// Device buffers of one integral (one handle, or one serving slot).
struct DevGrid {
  int dim = 0;
  int nb = 0;
  uint32_t* t = nullptr;       // iteration counter
  double* edges = nullptr;     // [dim][nb+1]
  double* hist = nullptr;      // [dim][nb], reduced histogram of the last iteration
  double* copies = nullptr;    // [kHistCopies][dim][nb], flush targets (zero between iterations)
  void* rec64 = nullptr;       // [dim][nb] Rec64
  void* rec32 = nullptr;       // [dim][nb] Rec32
  double* partials = nullptr;  // [max_blocks][4]: sum w, sum w^2, non-finite count, 0
  double* results = nullptr;   // [ring][4]: I, sigma, non-finite count, t
  // optional host-mapped mirror of results (pinned host memory, written by
  // the finalize kernel so that no copy is needed to read a result)
  double* results_host = nullptr;
  int max_blocks = 0;
  int ring = 0;
};

struct IterLaunch {
  int fid = 0;
  int prec = 0;
  int64_t n_events = 0;
  uint64_t seed = 0;
  int blocks = 0;
  int threads = 256;
  // a launch covering events first .. first+n_events-1 of the iteration, adding
  // to the workgroup partials of earlier launches when accumulate is set
  uint64_t first = 0;
  bool accumulate = false;
  // dump mode only
  double* w_out = nullptr;
  int64_t count = 0;
};

// An iteration kernel: compiled into the library (fn) or loaded from the
// code object of a run-time integrand (mf).
struct IterKernel {
  const void* fn = nullptr;
  hipFunction_t mf = nullptr;
  explicit operator bool() const { return fn || mf; }
  const void* key() const { return fn ? fn : (const void*)mf; }
};

// Iteration kernel (draw, map, evaluate, moments, histogram) for the given
// integrand/precision/dimension; empty if the combination does not exist (or
// a run-time integrand's code could not be loaded on the current GPU).
IterKernel iterate_kernel(int fid, int prec, int dim, bool dump);
hipError_t launch_kernel(const IterKernel& k, unsigned blocks, unsigned threads, void** args,
                         size_t lds, hipStream_t s);
// Run-time integrands (vegas_rtc.cpp): whether id fid exists and serves
// `dim` dimensions, and its kernel, loaded on the current GPU on first use.
int user_integrand_fits(int fid, int dim);
IterKernel user_iterate_kernel(int fid, int prec, int dim, bool dump);
size_t iterate_lds_bytes(int dim, int nb);

hipError_t launch_iterate(const DevGrid& g, const IterLaunch& L, const IntegrandArgs& P,
                          hipStream_t s);
hipError_t launch_dump(const DevGrid& g, const IterLaunch& L, const IntegrandArgs& P,
                       hipStream_t s);
// Reduce block partials to (I, sigma) in results[t % ring], advance t,
// reduce the histogram copies into hist (zeroing the copies) and, if refine,
// refine the grid with exponent alpha.
hipError_t launch_finalize(const DevGrid& g, int blocks, int64_t n_events, bool refine,
                           double alpha, hipStream_t s);
hipError_t launch_refine(const DevGrid& g, double alpha, hipStream_t s);
// Uniform grid, t = 0, zero histogram copies, grid records.
hipError_t launch_init_grid(const DevGrid& g, hipStream_t s);
// Grid records from the edges (after the edges were written from the host).
hipError_t launch_prepare(const DevGrid& g, hipStream_t s);
// Set t on the device.
hipError_t launch_set_t(const DevGrid& g, uint32_t t, hipStream_t s);

}  // namespace vegas
