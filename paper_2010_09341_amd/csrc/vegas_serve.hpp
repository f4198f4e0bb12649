// vegas_serve.hpp — device-side descriptors and launchers of the serving
// kernels (plain types; included by host and device code).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include "vegas_types.hpp"

namespace vegas {

constexpr int kServeThreads = 256;
constexpr int kServeMaxBlocks = 8192;

// One admitted integral: its shape, integrand and pointers to its state in
// the server's device arena.
struct SlotDev {
  uint32_t* t;
  double* edges;     // [dim][nb+1]
  double* hist;      // [dim][nb]
  double* copies;    // [kHistCopies][dim][nb]
  Rec64* rec64;      // [dim][nb]
  Rec32* rec32;      // [dim][nb]
  double* partials;  // [n_chunks][4]
  double* results;   // [ring][4]
  uint64_t n_events;
  uint64_t chunk_events;
  uint32_t n_chunks;
  uint32_t seed_lo, seed_hi;
  int dim;
  uint32_t nb;
  int fid;
  int prec;
  int ring;
  double alpha;
  IntegrandArgs P;
};

struct WorkItem {
  uint32_t slot;
  uint32_t chunk;
};

// role < 0: the moments of the slot's iteration (written to out[4*out]);
// role = d >= 0: histogram reduction of dimension d, then refinement if
// refine != 0. For k_serve_init, role = d is the dimension to initialise and
// out the index of the integral's descriptor among the tick's new ones.
struct FinItem {
  uint32_t slot;
  int32_t role;
  uint32_t out;
  uint32_t refine;
};

hipError_t launch_serve_iterate(int dmax, int prec, const SlotDev* slots, const WorkItem* items,
                                int n_items, int max_lds, hipStream_t s);
hipError_t launch_serve_finalize(const SlotDev* slots, const FinItem* items, int n_items,
                                 int max_nb, double* out, hipStream_t s);
hipError_t launch_serve_init(SlotDev* slots, const FinItem* items, int n_items, int max_nb,
                             const SlotDev* fresh, hipStream_t s);
// bytes (rounded up to 16; both buffers must hold that many) from src, host
// memory mapped into the device's address space, to dst in device memory.
hipError_t launch_serve_stage(const void* src, void* dst, size_t bytes, hipStream_t s);

}  // namespace vegas
