// vegas_device.hpp — device building blocks of one Vegas iteration on gfx950.
//
// The method (VegasFlow, arXiv:2010.09341, Sec. 1 and Sec. 3.1): points of the
// unit hypercube are drawn through a per-dimension adaptive grid, the integrand
// is evaluated on them, and the weights w = f(x) * J feed the estimate and the
// grid's next refinement. Everything here runs per event in registers; the
// grid records are read through the vector cache and the w^2 histogram sits
// in LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vegas_math.hpp"
#include "vegas_types.hpp"

namespace vegas {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// -> 64-bit products of counter words 0 and 2 by fixed odd multipliers, the
// high halves mixed into words 1 and 3 with the round key, the key advanced by
// two Weyl increments between rounds. The key and the iteration word are
// wave-uniform, so the compiler keeps them (and the first products that depend
// only on them) on the scalar unit.
// ---------------------------------------------------------------------------
struct Words4 {
  uint32_t v[4];
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t pa = (uint64_t)c0 * 0xD2511F53u;
    const uint64_t pb = (uint64_t)c2 * 0xCD9E8D57u;
    // three-input xor (truth table 0x96) in one gfx950 v_bitop3_b32
    const uint32_t next0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb >> 32), c1, k0, 0x96);
    const uint32_t next2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa >> 32), c3, k1, 0x96);
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = next0;
    c2 = next2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Words4 out;
  out.v[0] = c0;
  out.v[1] = c1;
  out.v[2] = c2;
  out.v[3] = c3;
  return out;
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
// Sum over the 64 lanes of a whole wave (every lane active), returned
// wave-uniform: within each row of 16 lanes a butterfly of DPP moves (lane
// xor 1 and xor 2 by quad permutes, then the half-row and row mirrors, which
// pair the quads and the halves), so every lane of a row holds the row's sum;
// then the four row sums read from lanes 0, 16, 32, 48 and added in that
// order. Register moves only, no LDS round trips.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t lo = dpp_u32<CTRL>((uint32_t)u), hi = dpp_u32<CTRL>((uint32_t)(u >> 32));
  return __longlong_as_double((long long)((hi << 32) | lo));
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return __longlong_as_double((long long)((hi << 32) | lo));
}

constexpr int kDppXor1 = 0xB1;        // quad_perm(1,0,3,2)
constexpr int kDppXor2 = 0x4E;        // quad_perm(2,3,0,1)
constexpr int kDppHalfMirror = 0x141;  // lane i <- 7 - i within each half row
constexpr int kDppMirror = 0x140;      // lane i <- 15 - i within each row

__device__ __forceinline__ double wave_total(double v) {
  v += dpp_f64<kDppXor1>(v);
  v += dpp_f64<kDppXor2>(v);
  v += dpp_f64<kDppHalfMirror>(v);
  v += dpp_f64<kDppMirror>(v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

__device__ __forceinline__ uint32_t wave_total_u32(uint32_t v) {
  v += dpp_u32<kDppXor1>(v);
  v += dpp_u32<kDppXor2>(v);
  v += dpp_u32<kDppHalfMirror>(v);
  v += dpp_u32<kDppMirror>(v);
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
         (uint32_t)__builtin_amdgcn_readlane((int)v, 32) + (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

// Exclusive prefix sum over the 64 lanes of a whole wave (every lane active):
// inclusive sums within each row of 16 lanes by DPP row shifts of 1, 2, 4 and
// 8 (a lane shifted in from outside the row reads 0), then every row offset by
// the totals of the rows before it (read from lanes 15, 31, 47); the exclusive
// value is the inclusive one of the lane before in the row, or the offset
// itself in the row's first lane.
template <int CTRL>
__device__ __forceinline__ double dpp_f64_zero(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t lo =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const uint64_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)((hi << 32) | lo));
}

constexpr int kDppRowShr1 = 0x111;  // lane i <- i - 1 within each row
constexpr int kDppRowShr2 = 0x112;
constexpr int kDppRowShr4 = 0x114;
constexpr int kDppRowShr8 = 0x118;

__device__ __forceinline__ double wave_scan_excl(double v) {
  double incl = v;
  incl += dpp_f64_zero<kDppRowShr1>(incl);
  incl += dpp_f64_zero<kDppRowShr2>(incl);
  incl += dpp_f64_zero<kDppRowShr4>(incl);
  incl += dpp_f64_zero<kDppRowShr8>(incl);
  const double t0 = readlane_f64(incl, 15), t1 = readlane_f64(incl, 31), t2 = readlane_f64(incl, 47);
  const double p2 = t0 + t1, p3 = p2 + t2;
  const uint32_t lane = __lane_id(), row = lane >> 4;
  const double off = row == 0 ? 0.0 : row == 1 ? t0 : row == 2 ? p2 : p3;
  incl += off;
  const double prev = dpp_f64_zero<kDppRowShr1>(incl);
  return (lane & 15u) ? prev : off;
}

// ---------------------------------------------------------------------------
// Integrands in binary64. x[0..D) in the unit hypercube.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rambo24_f64(const double* x, const IntegrandArgs& P) {
  const double W = P.d[1];
  if (P.mode == 1) return W;
  // As in binary32, the final scaling x = sqrt(s)/M is not applied: the cut
  // on s_ij = (2 s / M^2) d_ij reads d_ij > (c / 2s) M^2 and the weight is
  // (W / 16 s^4) M^8 / prod d_ij (P.d[4] = c / 2s, P.d[5] = W / 16 s^4).
  const double cut_d = P.d[4], w_d = P.d[5];
  double q[4][4];
  double Q0 = 0.0, Qx = 0.0, Qy = 0.0, Qz = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double ct = 2.0 * x[4 * i] - 1.0;
    const double st = sqrt(1.0 - ct * ct);
    double sp, cp;
    sincos_turns_f64(x[4 * i + 1], &sp, &cp);  // sin, cos of 2 pi u
    const double en = -log_f64(x[4 * i + 2] * x[4 * i + 3]);
    q[i][0] = en;
    q[i][1] = en * st * cp;
    q[i][2] = en * st * sp;
    q[i][3] = en * ct;
    Q0 += q[i][0];
    Qx += q[i][1];
    Qy += q[i][2];
    Qz += q[i][3];
  }
  const double M2 = Q0 * Q0 - Qx * Qx - Qy * Qy - Qz * Qz;
  const double iM = 1.0 / sqrt(M2);
  const double bx = -Qx * iM, by = -Qy * iM, bz = -Qz * iM;
  const double gam = Q0 * iM;
  const double a = 1.0 / (1.0 + gam);
  double p[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double bq = bx * q[i][1] + by * q[i][2] + bz * q[i][3];
    const double e = q[i][0] + a * bq;
    p[i][0] = gam * q[i][0] + bq;
    p[i][1] = q[i][1] + bx * e;
    p[i][2] = q[i][2] + by * e;
    p[i][3] = q[i][3] + bz * e;
  }
  const double thr = cut_d * M2;
  double prod = 1.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = (i + 1) & 3;
    const double dij = p[i][0] * p[j][0] - p[i][1] * p[j][1] - p[i][2] * p[j][2] - p[i][3] * p[j][3];
    if (!(dij > thr)) return 0.0;
    prod *= dij;
  }
  const double m4 = M2 * M2;
  return w_d * (m4 * m4) / prod;
}

// The integrand of a kernel compiled at run time: U::f64 / U::f32 wrap the
// user's device functions.
struct NoUser {};

template <int FID, class U = NoUser>
__device__ __forceinline__ double integrand_f64(const double* x, int DMAX, int D,
                                                const IntegrandArgs& P) {
  if constexpr (FID == kUser) {
    return U::f64(x, D, P.c64);
  } else if constexpr (FID == kConst) {
    return 1.0;
  } else if constexpr (FID == kSum) {
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < kMaxDim; ++d)
      if (d < DMAX && d < D) s += x[d];
    return s;
  } else if constexpr (FID == kGauss) {
    // prod_d exp(-z_d^2/a^2)/(a sqrt(pi)) = exp(-sum z_d^2 / a^2 - D ln(a sqrt(pi)))
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < kMaxDim; ++d)
      if (d < DMAX && d < D) {
        const double z = x[d] - P.c64[d];
        acc += z * z;
      }
    return exp_f64(P.d[1] - acc * P.d[0]);
  } else if constexpr (FID == kLoToy) {
    const double S = P.d[0], m2 = P.d[1], mG = P.d[2], norm = P.d[3], cut = P.d[4];
    const double x1 = x[0], x2 = x[1];
    const double c = 2.0 * x[2] - 1.0;
    const double x12 = x1 * x2;
    const double shat = x12 * S;
    if (!(sqrt(shat) > cut)) return 0.0;
    // g(x1) g(x2) (1 + c^2) BW / s^ with g(x) = (1 - x)^3 / sqrt(x) and
    // BW = norm / ((s^ - m^2)^2 + (m G)^2), norm = (m G / pi) 2 2 pi: one
    // square root and one division
    const double y12 = (1.0 - x1) * (1.0 - x2);
    const double dm = shat - m2;
    const double num = y12 * y12 * y12 * (1.0 + c * c) * norm;
    return num / (sqrt(x12) * (dm * dm + mG * mG) * shat);
  } else if constexpr (FID == kRambo24) {
    return rambo24_f64(x, P);
  } else {  // kBwFlat
    const double z = x[0] - P.d[0];
    return P.d[2] / (z * z + P.d[1]);
  }
}

// ---------------------------------------------------------------------------
// Integrands in binary32. Each returns f as a binary32 factor and, for the
// Gaussian, its log2 (the factor is then 1), so that tails far below the
// binary32 range still produce a binary64 weight.
// ---------------------------------------------------------------------------
struct F32Val {
  float f;
  float log2f;
};

__device__ __forceinline__ float rambo24_f32(const float* x, const IntegrandArgs& P) {
  const float W = P.f[1];
  if (P.mode == 1) return W;
  // RAMBO's final scaling x = sqrt(s)/M is never applied: with p = x p' the
  // invariants are s_ij = 2 x^2 (p'_i.p'_j) = (2 s / M^2) d_ij, so the cut
  // s_ij > c reads d_ij > (c / 2s) M^2 and the weight W / prod s_ij reads
  // (W / 16 s^4) M^8 / prod d_ij (P.f[3] = c / 2s, P.f[4] = W / 16 s^4)
  const float cut_d = P.f[3], w_d = P.f[4];
  float q[4][4];
  float Q0 = 0.f, Qx = 0.f, Qy = 0.f, Qz = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float ct = fminf(fmaf(2.f, x[4 * i], -1.f), 1.f);
    // the hardware square root (within an ulp, one instruction; the correctly
    // rounded one costs a dozen)
    const float st = __builtin_amdgcn_sqrtf(fmaxf(fmaf(-ct, ct, 1.f), 0.f));
    // v_sin_f32 / v_cos_f32 take their argument in turns: sin(2 pi u) = sin_turns(u)
    const float sp = __builtin_amdgcn_sinf(x[4 * i + 1]);
    const float cp = __builtin_amdgcn_cosf(x[4 * i + 1]);
    // -ln(u u') = -log2(u u') * ln 2
    const float en = fmaxf(-__builtin_amdgcn_logf(x[4 * i + 2] * x[4 * i + 3]) * 0.69314718f, 0.f);
    q[i][0] = en;
    q[i][1] = en * st * cp;
    q[i][2] = en * st * sp;
    q[i][3] = en * ct;
    Q0 += q[i][0];
    Qx += q[i][1];
    Qy += q[i][2];
    Qz += q[i][3];
  }
  const float M2 = Q0 * Q0 - Qx * Qx - Qy * Qy - Qz * Qz;
  const float iM = __builtin_amdgcn_rsqf(M2);
  const float bx = -Qx * iM, by = -Qy * iM, bz = -Qz * iM;
  const float gam = Q0 * iM;
  const float a = __builtin_amdgcn_rcpf(1.f + gam);
  // the boosted momenta before the scaling
  float p[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float bq = bx * q[i][1] + by * q[i][2] + bz * q[i][3];
    const float e = q[i][0] + a * bq;
    p[i][0] = gam * q[i][0] + bq;
    p[i][1] = q[i][1] + bx * e;
    p[i][2] = q[i][2] + by * e;
    p[i][3] = q[i][3] + bz * e;
  }
  const float thr = cut_d * M2;
  float prod = 1.f;
  bool pass = true;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = (i + 1) & 3;
    const float dij = p[i][0] * p[j][0] - p[i][1] * p[j][1] - p[i][2] * p[j][2] - p[i][3] * p[j][3];
    pass = pass && (dij > thr);
    prod *= dij;
  }
  const float m4 = M2 * M2;
  return pass ? w_d * (m4 * m4) * __builtin_amdgcn_rcpf(prod) : 0.f;
}

template <int FID, class U = NoUser>
__device__ __forceinline__ F32Val integrand_f32(const float* x, int DMAX, int D,
                                                const IntegrandArgs& P) {
  F32Val r{1.f, 0.f};
  if constexpr (FID == kUser) {
    r.f = U::f32(x, D, P.c32);
  } else if constexpr (FID == kConst) {
  } else if constexpr (FID == kSum) {
    float s = 0.f;
#pragma unroll
    for (int d = 0; d < kMaxDim; ++d)
      if (d < DMAX && d < D) s += x[d];
    r.f = s;
  } else if constexpr (FID == kGauss) {
    // log2 f = -(log2 e / a^2) sum z^2 - D log2(a sqrt(pi))
    float acc = 0.f;
#pragma unroll
    for (int d = 0; d < kMaxDim; ++d)
      if (d < DMAX && d < D) {
        const float z = x[d] - P.c32[d];
        acc = fmaf(z, z, acc);
      }
    r.log2f = fmaf(-P.f[0], acc, P.f[1]);
  } else if constexpr (FID == kLoToy) {
    const float S = P.f[0], m2 = P.f[1], mG = P.f[2], norm = P.f[3], cut2 = P.f[4];
    const float x1 = x[0], x2 = x[1];
    const float c = fmaf(2.f, x[2], -1.f);
    const float shat = x1 * x2 * S;
    // g(x1) g(x2) = ((1 - x1)(1 - x2))^3 / sqrt(x1 x2)
    const float y12 = (1.f - x1) * (1.f - x2);
    const float g12 = (y12 * y12 * y12) * __builtin_amdgcn_rsqf(x1 * x2);
    const float dm = shat - m2;
    const float den = fmaf(dm, dm, mG * mG) * shat;
    const float v = g12 * fmaf(c, c, 1.f) * norm * __builtin_amdgcn_rcpf(den);
    r.f = (shat > cut2) ? v : 0.f;
  } else if constexpr (FID == kRambo24) {
    r.f = rambo24_f32(x, P);
  } else {  // kBwFlat
    const float z = x[0] - P.f[0];
    r.f = P.f[2] * __builtin_amdgcn_rcpf(fmaf(z, z, P.f[1]));
  }
  return r;
}

// Dimension count: D_T > 0 is the exact count known at compile time; D_T < 0
// means at most -D_T dimensions with the actual count D given at run time.
template <int D_T>
struct Dims {
  static constexpr int kMax = D_T > 0 ? D_T : -D_T;
  static constexpr int kBlocks = (kMax + 3) / 4;
  __device__ static constexpr bool on(int d, int D) { return D_T > 0 ? d < D_T : d < D; }
};

// Zero the workgroup's LDS histograms.
__device__ inline void zero_hist(const LdsLayout& L, unsigned char* smem) {
  double* h = reinterpret_cast<double*>(smem);
  const int nh = (int)(L.cells * L.copies);
  for (int i = threadIdx.x; i < nh; i += blockDim.x) h[i] = 0.0;
}

// hb[d]: LDS byte address of this lane's copy of cell (d, 0); bin k of
// dimension d is at hb[d] + (k << L.cshift).
// Byte offset of this lane's copy within a cell.
__device__ inline uint32_t lane_hist_offset(const LdsLayout& L) {
  return 8u * (threadIdx.x & (L.copies - 1u));
}

// hb[d]: LDS byte address of this lane's copy of cell (d, 0), so that bin k
// of dimension d is at hb[d] + (k << L.cshift) — one instruction per
// dimension in the event loop, for KMAX registers held across it (used by
// the kernels for an exact dimension count that are not short of
// registers). The bases pass through an
// identity DPP move, which the compiler cannot see through: otherwise it
// folds them back into (d*nb + k) << cshift, two instructions per dimension.
template <int KMAX>
__device__ inline void lane_hist_bases(const LdsLayout& L, int nb, uint32_t* hb) {
  const uint32_t lane_off = lane_hist_offset(L);
#pragma unroll
  for (int d = 0; d < KMAX; ++d) {
    const uint32_t v = lane_off + (((uint32_t)d * (uint32_t)nb) << L.cshift);
    // quad_perm(0,1,2,3): every lane reads its own value
    hb[d] = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xE4, 0xF, 0xF, false);
  }
}

// Add the LDS histogram copies of cell i (in copy order) and flush non-zero
// sums into dst (global binary64 atomics). Needs a barrier before it.
__device__ inline void flush_hist(const LdsLayout& L, const unsigned char* smem, double* dst) {
  const double* h = reinterpret_cast<const double*>(smem);
  for (int i = threadIdx.x; i < (int)L.cells; i += blockDim.x) {
    const double* hc = h + (size_t)i * L.copies;
    double v = hc[0];
    for (uint32_t c = 1; c < L.copies; ++c) v += hc[c];
    if (v != 0.0) __hip_atomic_fetch_add(&dst[i], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// One event: draw, map, evaluate. The grid records come from global memory
// through the vector cache (a few KiB, resident after the first events).
// Returns w = f(x) * J in binary64 and, in hist[d], the LDS byte address of
// the histogram entry that dimension d fell into (in this lane's copy: from
// hb, set by lane_hist_bases, when HOIST, else from lane_off).
// ---------------------------------------------------------------------------
// Grid records are read with structured buffer loads: one resource for the
// whole record table (workgroup-uniform, in scalar registers) whose stride is
// the record size, the bin as the vector index and the dimension's first
// record as the scalar byte offset, so the address costs no vector
// instruction. The range check (index below the table size) always passes:
// k < nb.
typedef uint32_t rec_u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t rec_u32x4 __attribute__((ext_vector_type(4)));
__device__ rec_u32x2 rec_buffer_load_b64(__amdgpu_buffer_rsrc_t rsrc, int index, int voffset,
                                         int soffset, int aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.v2i32");
__device__ rec_u32x4 rec_buffer_load_b128(__amdgpu_buffer_rsrc_t rsrc, int index, int voffset,
                                          int soffset, int aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.v4i32");

template <class R>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rec_rsrc(const void* rec,
                                                                 uint32_t rec_bytes) {
  // the fourth descriptor word of gfx9-family GPUs (no format conversion)
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(rec), (short)sizeof(R),
                                           (int)rec_bytes, 0x00020000);
}

__device__ __forceinline__ Rec32 load_rec32(__amdgpu_buffer_rsrc_t r, uint32_t k,
                                            uint32_t soff) {
  const rec_u32x2 v = rec_buffer_load_b64(r, (int)k, 0, (int)soff, 0);
  Rec32 g;
  g.e = __uint_as_float(v[0]);
  g.w = __uint_as_float(v[1]);
  return g;
}

__device__ __forceinline__ Rec64 load_rec64(__amdgpu_buffer_rsrc_t r, uint32_t k,
                                            uint32_t soff) {
  const rec_u32x4 v = rec_buffer_load_b128(r, (int)k, 0, (int)soff, 0);
  Rec64 g;
  g.e = __hiloint2double((int)v[1], (int)v[0]);
  g.w = __hiloint2double((int)v[3], (int)v[2]);
  return g;
}

template <int PREC>
struct std_conditional_rec {
  using type = Rec32;
};
template <>
struct std_conditional_rec<kFp64> {
  using type = Rec64;
};

template <int D_T, int FID, int PREC, class U = NoUser, bool HOIST = false>
__device__ __forceinline__ double event_weight(uint64_t n, uint32_t t, uint32_t k0, uint32_t k1,
                                               int D, uint32_t nb, const void* rec,
                                               const uint32_t* hb, uint32_t lane_off,
                                               uint32_t cshift, const IntegrandArgs& P,
                                               uint32_t* hist) {
  using Dm = Dims<D_T>;
  const uint32_t n_lo = (uint32_t)n, n_hi = (uint32_t)(n >> 32);
  const uint32_t rec_bytes =
      (uint32_t)(D_T > 0 ? D_T : D) * nb * (PREC == kFp64 ? sizeof(Rec64) : sizeof(Rec32));
  const __amdgpu_buffer_rsrc_t rsrc =
      make_rec_rsrc<typename std_conditional_rec<PREC>::type>(rec, rec_bytes);
  if constexpr (PREC == kFp64) {
    // Up to 8 dimensions every grid record of the event is requested before
    // any is used, so that the loads overlap each other and the later
    // blocks' Philox rounds; above that the records of each 4-dimension
    // block are used within the block (holding all of them would cost more
    // registers than the overlap gains).
    constexpr bool kLoadsFirst = Dm::kMax <= 8;
    uint32_t rem[Dm::kMax];
    Rec64 g[Dm::kMax];
    double x[Dm::kMax];
    // J = prod_d (nb Delta_d), the factors taken in dimension order; the
    // record holds Delta 2^-32, and nb 2^32 is exact
    const double nbd = (double)nb * 0x1p32;
    double jac = 1.0;
#pragma unroll
    for (int j = 0; j < Dm::kBlocks; ++j) {
      if (Dm::on(4 * j, D)) {
        const Words4 r = philox4x32_10(n_lo, n_hi, t, (uint32_t)j, k0, k1);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int d = 4 * j + i;
          if (d < Dm::kMax && Dm::on(d, D)) {
            const uint64_t prod = (uint64_t)r.v[i] * nb;
            const uint32_t k = (uint32_t)(prod >> 32);
            // the point at fraction (rem + 1/2) 2^-32 of the bin: rem
            // converts exactly, and the record's e carries the half
            rem[d] = (uint32_t)prod;
            g[d] = load_rec64(rsrc, k, (uint32_t)d * nb * (uint32_t)sizeof(Rec64));
            hist[d] = HOIST ? hb[d] + (k << cshift)
                              : ((((uint32_t)d * nb) + k) << cshift) + lane_off;
            if constexpr (!kLoadsFirst) {
              x[d] = fma((double)rem[d], g[d].w, g[d].e);
              jac *= nbd * g[d].w;
            }
          }
        }
      }
    }
    if constexpr (kLoadsFirst) {
      // keeps the scheduler from moving any load below this point
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int d = 0; d < Dm::kMax; ++d)
        if (Dm::on(d, D)) {
          x[d] = fma((double)rem[d], g[d].w, g[d].e);
          jac *= nbd * g[d].w;
        }
    }
    return integrand_f64<FID, U>(x, Dm::kMax, D_T > 0 ? D_T : D, P) * jac;
  } else {
    float x[Dm::kMax];
    // log2 J = sum over pairs of dimensions (2i, 2i+1) of log2(nb^2 Delta_2i
    // Delta_2i+1), and log2(nb Delta) of a last unpaired dimension: binary32
    // products (nb^2 <= 2^18 is exact) and one hardware log2 per pair, in the
    // normal binary32 range wherever a pair's nb^2 Delta Delta >= 2^-126
    // (bins wider than about 1e-19 / nb), and no constant D log2(nb) whose
    // rounding would bias every weight alike
    const float nbf = (float)nb, nb2 = (float)(nb * nb);
    const int Dn = D_T > 0 ? D_T : D;
    float l2j = 0.f, pw = 1.f;
#pragma unroll
    for (int j = 0; j < Dm::kBlocks; ++j) {
      if (Dm::on(4 * j, D)) {
        const Words4 r = philox4x32_10(n_lo, n_hi, t, (uint32_t)j, k0, k1);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int d = 4 * j + i;
          if (d < Dm::kMax && Dm::on(d, D)) {
            const uint64_t prod = (uint64_t)r.v[i] * nb;
            const uint32_t k = (uint32_t)(prod >> 32);
            const uint32_t rem = (uint32_t)prod;
            // 1 + (rem >> 9) 2^-23, exact: the bits under the exponent of
            // 1.0; with the record's shifted origin the point is at the
            // centre ((rem >> 9) + 1/2) 2^-23 of a 2^-23 cell of the bin
            const float y = __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, rem, 9u));
            const Rec32 g = load_rec32(rsrc, k, (uint32_t)d * nb * (uint32_t)sizeof(Rec32));
            x[d] = fmaf(y, g.w, g.e);
            if ((d & 1) == 0) {
              pw = g.w * (d + 1 < Dn ? nb2 : nbf);
            } else {
              pw *= g.w;
              l2j += __builtin_amdgcn_logf(pw);
            }
            hist[d] = HOIST ? hb[d] + (k << cshift)
                              : ((((uint32_t)d * nb) + k) << cshift) + lane_off;
          }
        }
      }
    }
    if (Dn & 1) l2j += __builtin_amdgcn_logf(pw);
    const F32Val v = integrand_f32<FID, U>(x, Dm::kMax, D_T > 0 ? D_T : D, P);
    // w = f * 2^(log2 J + log2 f), the power split into a binary32 mantissa
    // in [1, 2) and an integer exponent applied in binary64.
    const float l2 = l2j + v.log2f;
    const float fl = __builtin_floorf(l2);
    const double m = (double)__builtin_amdgcn_exp2f(l2 - fl);
    return (double)v.f * __builtin_ldexp(m, (int)fl);
  }
}

}  // namespace vegas
