// vegas_finalize.hpp — per-workgroup steps that close an iteration, for
// workgroups of exactly one wave (64 threads), shared by the single-integral
// kernels and the serving kernels:
//   wg_moments        fixed-order reduction of the chunk/workgroup partials
//                     into (I, sigma) = (S1/N, sqrt((S2/N - I^2)/(N-1)))
//   wg_reduce_hist    the histogram copies of one dimension summed in a fixed
//                     copy order, copies zeroed for the next iteration
//   wg_refine_dim     smoothing, normalisation, compression, equal-share
//                     re-binning of one dimension; grid records rebuilt
//   wg_uniform_dim    the uniform grid of one dimension
#pragma once

#include <hip/hip_runtime.h>

#include "vegas_device.hpp"

namespace vegas {

// Grid records of bin k = lane, lane+64, ... of dimension row `d` from its
// edges e[0..nb] (the layouts are those of Rec64 and Rec32).
__device__ inline void wg_write_records(int nb, const double* e, Rec64* rec64, Rec32* rec32) {
  for (int k = threadIdx.x; k < nb; k += 64) {
    const double lo = e[k], hi = e[k + 1];
    const double delta = hi - lo;
    rec64[k] = Rec64{fma(delta, kRec64Half, lo), delta * kRec64Scale};
    Rec32 r;
    r.w = (float)delta;
    r.e = (float)(lo - (double)r.w * (double)kRec32Shift);
    rec32[k] = r;
  }
}

// (I, sigma, non-finite count, t) of the iteration into results[t % ring]
// (and into mirror[t % ring] and out[0..3] where those are not null), then
// t += 1.
__device__ inline void wg_moments(const double* partials, int n_partials, double N, uint32_t* t,
                                  double* results, int ring, double* out,
                                  double* mirror = nullptr) {
  const uint32_t tt = *t;  // issued together with the partial loads
  // The partials were written by workgroups on every XCD, so each load goes
  // to memory: issue 8 independent 32-byte loads per lane before adding.
  const double4* p4 = reinterpret_cast<const double4*>(partials);
  double s1 = 0.0, s2 = 0.0, b = 0.0;
  for (int base = 0; base < n_partials; base += 8 * 64) {
    double4 v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = base + j * 64 + (int)threadIdx.x;
      v[j] = i < n_partials ? p4[i] : make_double4(0.0, 0.0, 0.0, 0.0);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      s1 += v[j].x;
      s2 += v[j].y;
      b += v[j].z;
    }
  }
  s1 = wave_total(s1);
  s2 = wave_total(s2);
  b = wave_total(b);
  if (threadIdx.x == 0) {
    const double I = s1 / N;
    const double var = (s2 / N - I * I) / (N - 1.0);
    const double sig = sqrt(var > 0.0 ? var : 0.0);
    double* r = results + 4 * (size_t)(tt % (uint32_t)ring);
    r[0] = I;
    r[1] = sig;
    r[2] = b;
    r[3] = (double)tt;
    if (out) {
      out[0] = I;
      out[1] = sig;
      out[2] = b;
      out[3] = (double)tt;
    }
    if (mirror) {
      double* m = mirror + 4 * (size_t)(tt % (uint32_t)ring);
      m[0] = I;
      m[1] = sig;
      m[2] = b;
      m[3] = (double)tt;
    }
    *t = tt + 1;
  }
}

// hist_row[k] = sum over copies c of copies[c][d][k] (fixed order); copies
// zeroed; the row is also left in h_lds[0..nb). When eo_lds is not null the
// dimension's edges erow[0..nb] are loaded into it in the same pass, so that
// both sets of global loads are in flight together.
__device__ inline void wg_reduce_hist(double* copies, double* hist_row, int cells, int d, int nb,
                                      double* h_lds, const double* erow = nullptr,
                                      double* eo_lds = nullptr) {
  for (int k = threadIdx.x; k <= nb; k += 64) {
    if (eo_lds) eo_lds[k] = erow[k];
    if (k == nb) break;
    const size_t idx = (size_t)d * nb + k;
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < kHistCopies; ++c) {
      v += copies[(size_t)c * cells + idx];
      copies[(size_t)c * cells + idx] = 0.0;
    }
    hist_row[k] = v;
    h_lds[k] = v;
  }
  __syncthreads();
}

// LDS doubles wg_refine_dim needs for nb bins (besides the histogram row).
__host__ __device__ constexpr int refine_lds_doubles(int nb) { return 3 * (nb + 1) + 2 * nb; }

// Refine one dimension from its histogram row h (LDS, nb entries).
//  1. smooth: s_i = (h_{i-1} + h_i + h_{i+1})/3, (h_0+h_1)/2 and
//     (h_{nb-2}+h_{nb-1})/2 at the ends;
//  2. p_i = s_i / sum s (a dimension with sum 0 keeps its edges);
//  3. r_i = ((1 - p_i)/(-ln p_i))^alpha (0 for p_i = 0, 1 for p_i = 1);
//  4. running sums C_k of r (per-lane contiguous segments, then a wave scan by
//     DPP moves);
//  5. new edge j where the piecewise-uniform r density reaches j C_nb / nb:
//     the old bin k is the smallest with C_{k+1} >= j C_nb/nb (binary
//     search), the position linear inside it;
//  6. e_0 = 0, e_nb = 1; the records are rebuilt.
// lds[0..nb] must already hold the old edges when edges_loaded is true.
__device__ inline void wg_refine_dim(int nb, double alpha, double* erow, const double* h,
                                     Rec64* rec64, Rec32* rec32, double* lds,
                                     bool edges_loaded = false) {
  const int lane = threadIdx.x;
  double* eo = lds;            // nb + 1
  double* en = eo + (nb + 1);  // nb + 1
  double* C = en + (nb + 1);   // nb + 1
  double* s = C + (nb + 1);    // nb
  double* r = s + nb;          // nb
  if (!edges_loaded)
    for (int i = lane; i <= nb; i += 64) eo[i] = erow[i];
  for (int i = lane; i < nb; i += 64) {
    double v;
    if (i == 0)
      v = (h[0] + h[1]) / 2.0;
    else if (i == nb - 1)
      v = (h[nb - 2] + h[nb - 1]) / 2.0;
    else
      v = (h[i - 1] + h[i] + h[i + 1]) / 3.0;
    s[i] = v;
  }
  __syncthreads();
  double part = 0.0;
  for (int i = lane; i < nb; i += 64) part += s[i];
  const double S = wave_total(part);  // bitwise equal in every lane
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
        v = pow_pos((1.0 - p) / (-log_f64(p)), alpha);
      r[i] = v;
    }
    __syncthreads();
    const int seg = (nb + 63) / 64;
    const int lo = lane * seg;
    const int hi = lo + seg < nb ? lo + seg : nb;
    double local = 0.0;
    for (int i = lo; i < hi; ++i) local += r[i];
    const double excl = wave_scan_excl(local);  // S > 0 in every lane: the whole wave is here
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
  wg_write_records(nb, en, rec64, rec32);
}

// The uniform grid e_i = i/nb of one dimension, its records, and zeroed
// histogram copies of that dimension.
__device__ inline void wg_uniform_dim(int nb, double* erow, double* copies, int cells, int d,
                                      Rec64* rec64, Rec32* rec32, double* lds) {
  for (int i = threadIdx.x; i <= nb; i += 64) {
    lds[i] = (double)i / nb;
    erow[i] = lds[i];
  }
  for (int c = 0; c < kHistCopies; ++c)
    for (int k = threadIdx.x; k < nb; k += 64) copies[(size_t)c * cells + (size_t)d * nb + k] = 0.0;
  __syncthreads();
  wg_write_records(nb, lds, rec64, rec32);
}

}  // namespace vegas
