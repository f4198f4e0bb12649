// vegas_kernels.hip — the kernels of one Vegas iteration on gfx950.
//
//   k_iterate   (vegas_iterate.hpp, instantiated in iter_*.hip) draw, map,
//               integrand, moments, w^2 histogram
//   k_finalize  fixed-order reduction of the workgroup partials into (I, sigma),
//               and of the histogram copies into the iteration's histogram
//   k_refine    smoothing, normalisation, compression, equal-share re-binning
//   k_init_grid / k_prepare / k_set_t   grid set-up and state writes
//
// The method: VegasFlow (arXiv:2010.09341) Sec. 1 (importance sampling on
// adaptive grids, after Lepage), Sec. 3.1 (integrand contract, iterations),
// Sec. 3.2 (each iteration informs the next). Nothing here is a dense
// contraction, so there is no MFMA; the iteration kernel is bound by vector
// ALU issue (integer multiplies of Philox, map and integrand arithmetic).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "vegas_device.hpp"
#include "vegas_iterate.hpp"
#include "vegas_launch.hpp"

namespace vegas {

// ---------------------------------------------------------------------------
// finalize: workgroup 0 reduces the partials in a fixed order and writes
// (I, sigma, non-finite count, t) to results[t % ring], then advances t;
// workgroup 1 + d reduces the histogram copies of dimension d (fixed copy
// order) into hist and zeroes the copies for the next iteration.
// ---------------------------------------------------------------------------
struct FinArgs {
  uint32_t* t;
  const double* partials;
  double* results;
  double* copies;
  double* hist;
  double n_events;
  int blocks;
  int ring;
  int dim;
  int nb;
};

__global__ __launch_bounds__(256) void k_finalize(FinArgs a) {
  const int cells = a.dim * a.nb;
  if (blockIdx.x == 0) {
    double s1 = 0.0, s2 = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < a.blocks; i += blockDim.x) {
      s1 += a.partials[4 * i];
      s2 += a.partials[4 * i + 1];
      b += a.partials[4 * i + 2];
    }
    __shared__ double red[3][4];
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
      red[0][wid] = s1;
      red[1][wid] = s2;
      red[2][wid] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double S1 = 0.0, S2 = 0.0, B = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        S1 += red[0][w];
        S2 += red[1][w];
        B += red[2][w];
      }
      const double N = a.n_events;
      const double I = S1 / N;
      const double var = (S2 / N - I * I) / (N - 1.0);
      const uint32_t t = *a.t;
      double* r = a.results + 4 * (size_t)(t % (uint32_t)a.ring);
      r[0] = I;
      r[1] = sqrt(var > 0.0 ? var : 0.0);
      r[2] = B;
      r[3] = (double)t;
      *a.t = t + 1;
    }
  } else {
    const int d = blockIdx.x - 1;
    for (int k = threadIdx.x; k < a.nb; k += blockDim.x) {
      const int idx = d * a.nb + k;
      double v = 0.0;
#pragma unroll
      for (int c = 0; c < kHistCopies; ++c) {
        v += a.copies[(size_t)c * cells + idx];
        a.copies[(size_t)c * cells + idx] = 0.0;
      }
      a.hist[idx] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Grid records of one dimension from its edges in LDS (one wave).
// ---------------------------------------------------------------------------
__device__ void write_records(int d, int nb, const double* e, Rec64* rec64, Rec32* rec32) {
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    const double lo = e[k], hi = e[k + 1];
    rec64[d * nb + k] = Rec64{lo, hi - lo};
    const float lo32 = (float)lo, hi32 = (float)hi;
    const double w32 = (double)hi32 - (double)lo32;  // exact
    const double jac = (double)nb * w32;
    Rec32 r;
    r.e = lo32;
    r.w = (float)w32;
    // a bin narrower than binary32 resolution carries a vanishing Jacobian
    r.l2j = (float)log2(jac > 0x1p-1000 ? jac : 0x1p-1000);
    r.pad = 0.f;
    rec32[d * nb + k] = r;
  }
}

// ---------------------------------------------------------------------------
// refine: one wave per dimension.
//  1. smooth: s_i = (h_{i-1} + h_i + h_{i+1})/3, (h_0+h_1)/2 and
//     (h_{nb-2}+h_{nb-1})/2 at the ends;
//  2. p_i = s_i / sum s (a dimension with sum 0 keeps its edges);
//  3. r_i = ((1 - p_i)/(-ln p_i))^alpha (0 for p_i = 0, 1 for p_i = 1);
//  4. running sums C_k of r (per-lane contiguous segments, then a wave scan);
//  5. new edge j at the point where the piecewise-uniform r density reaches
//     j C_nb / nb: the old bin k is the smallest with C_{k+1} >= j C_nb/nb
//     (binary search), the position linear inside it;
//  6. e_0 = 0, e_nb = 1; records rebuilt.
// ---------------------------------------------------------------------------
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
  const int lane = threadIdx.x;
  double* eo = rsm;            // nb + 1
  double* en = eo + (nb + 1);  // nb + 1
  double* C = en + (nb + 1);   // nb + 1
  double* s = C + (nb + 1);    // nb
  double* r = s + nb;          // nb
  const double* h = a.hist + (size_t)d * nb;
  double* erow = a.edges + (size_t)d * (nb + 1);
  for (int i = lane; i <= nb; i += 64) eo[i] = erow[i];
  for (int i = lane; i < nb; i += 64) r[i] = h[i];
  __syncthreads();
  for (int i = lane; i < nb; i += 64) {
    double v;
    if (i == 0)
      v = (r[0] + r[1]) / 2.0;
    else if (i == nb - 1)
      v = (r[nb - 2] + r[nb - 1]) / 2.0;
    else
      v = (r[i - 1] + r[i] + r[i + 1]) / 3.0;
    s[i] = v;
  }
  __syncthreads();
  double part = 0.0;
  for (int i = lane; i < nb; i += 64) part += s[i];
  const double S = wave_sum(part);
  if (!(S > 0.0)) {
    for (int i = lane; i <= nb; i += 64) en[i] = eo[i];
  } else {
    for (int i = lane; i < nb; i += 64) {
      const double p = s[i] / S;
      double v;
      if (p <= 0.0)
        v = 0.0;
      else if (p >= 1.0)
        v = 1.0;
      else
        v = pow((1.0 - p) / (-log(p)), a.alpha);
      r[i] = v;
    }
    __syncthreads();
    const int seg = (nb + 63) / 64;
    const int lo = lane * seg;
    const int hi = lo + seg < nb ? lo + seg : nb;
    double local = 0.0;
    for (int i = lo; i < hi; ++i) local += r[i];
    double incl = local;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    double excl = __shfl_up(incl, 1, 64);
    if (lane == 0) excl = 0.0;
    if (lo < nb) {
      double c = excl;
      C[lo] = c;
      for (int i = lo; i < hi; ++i) {
        c += r[i];
        C[i + 1] = c;
      }
    }
    if (lane == 0) C[0] = 0.0;
    __syncthreads();
    const double delta = C[nb] / nb;
    for (int j = lane + 1; j < nb; j += 64) {
      const double target = j * delta;
      int lo_k = 0, hi_k = nb - 1;
      while (lo_k < hi_k) {
        const int mid = (lo_k + hi_k) >> 1;
        if (C[mid + 1] >= target)
          hi_k = mid;
        else
          lo_k = mid + 1;
      }
      const int k = lo_k;
      en[j] = eo[k] + (target - C[k]) / r[k] * (eo[k + 1] - eo[k]);
    }
    if (lane == 0) {
      en[0] = 0.0;
      en[nb] = 1.0;
    }
  }
  __syncthreads();
  for (int i = lane; i <= nb; i += 64) erow[i] = en[i];
  write_records(d, nb, en, a.rec64, a.rec32);
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
  for (int i = threadIdx.x; i <= nb; i += 64) {
    if (a.uniform) {
      gsm[i] = (double)i / nb;
      erow[i] = gsm[i];
    } else {
      gsm[i] = erow[i];
    }
  }
  if (a.uniform) {
    for (int c = 0; c < kHistCopies; ++c)
      for (int k = threadIdx.x; k < nb; k += 64) a.copies[(size_t)c * a.cells + d * nb + k] = 0.0;
    if (d == 0 && threadIdx.x == 0) *a.t = 0;
  }
  __syncthreads();
  write_records(d, nb, gsm, a.rec64, a.rec32);
}

__global__ void k_set_t(uint32_t* t, uint32_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *t = v;
}

// ---------------------------------------------------------------------------
// Dispatch
// ---------------------------------------------------------------------------
const void* iterate_kernel(int fid, int prec, int dim, bool dump) {
  if (dim < 1 || dim > kMaxDim || (prec != kFp64 && prec != kFp32Eval)) return nullptr;
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

size_t iterate_lds_bytes(int dim, int nb) { return (size_t)dim * nb * kCellBytes; }

static IterArgsDev iter_args(const DevGrid& g, const IterLaunch& L) {
  IterArgsDev a;
  a.t = g.t;
  a.rec = L.prec == kFp64 ? g.rec64 : g.rec32;
  a.copies = g.copies;
  a.partials = g.partials;
  a.w_out = L.w_out;
  a.n_events = (uint64_t)L.n_events;
  a.first = L.first;
  a.seed_lo = (uint32_t)L.seed;
  a.seed_hi = (uint32_t)(L.seed >> 32);
  a.dim = g.dim;
  a.nb = (uint32_t)g.nb;
  a.nb_pow_d = pow((double)g.nb, (double)g.dim);
  return a;
}

hipError_t launch_iterate(const DevGrid& g, const IterLaunch& L, const IntegrandArgs& P,
                          hipStream_t s) {
  const void* k = iterate_kernel(L.fid, L.prec, g.dim, false);
  if (!k || L.blocks < 1 || L.blocks > g.max_blocks || L.threads < 64 ||
      L.threads > kIterThreadsMax || (L.threads & 63))
    return hipErrorInvalidValue;
  IterArgsDev a = iter_args(g, L);
  IntegrandArgs p = P;
  void* args[] = {&a, &p};
  return hipLaunchKernel(k, dim3(L.blocks), dim3(L.threads), args,
                         iterate_lds_bytes(g.dim, g.nb), s);
}

hipError_t launch_dump(const DevGrid& g, const IterLaunch& L, const IntegrandArgs& P,
                       hipStream_t s) {
  const void* k = iterate_kernel(L.fid, L.prec, g.dim, true);
  if (!k || L.count < 1 || !L.w_out) return hipErrorInvalidValue;
  IterArgsDev a = iter_args(g, L);
  a.n_events = (uint64_t)L.count;
  IntegrandArgs p = P;
  void* args[] = {&a, &p};
  const int threads = 256;
  int64_t blocks = (L.count + threads - 1) / threads;
  if (blocks > 4096) blocks = 4096;
  return hipLaunchKernel(k, dim3((unsigned)blocks), dim3(threads), args,
                         iterate_lds_bytes(g.dim, g.nb), s);
}

hipError_t launch_finalize(const DevGrid& g, int blocks, int64_t n_events, hipStream_t s) {
  if (blocks < 1 || blocks > g.max_blocks) return hipErrorInvalidValue;
  FinArgs a;
  a.t = g.t;
  a.partials = g.partials;
  a.results = g.results;
  a.copies = g.copies;
  a.hist = g.hist;
  a.n_events = (double)n_events;
  a.blocks = blocks;
  a.ring = g.ring;
  a.dim = g.dim;
  a.nb = g.nb;
  hipLaunchKernelGGL(k_finalize, dim3(1 + g.dim), dim3(256), 0, s, a);
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
  const size_t lds = sizeof(double) * (3 * (size_t)(g.nb + 1) + 2 * (size_t)g.nb);
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
