// Device-side building blocks for the Householder Dice kernels (gfx950).
//
//  * counter-based normal draws: Philox4x32-10 (Salmon et al., SC'11) feeding
//    Box-Muller (1958) in FP64, keyed exactly as the library documents
//    (key = (seed, trial), counter = (lo32(i/4), step, tag, hi32(i/4)));
//  * 64-lane wavefront reductions, including a reduce-scatter that sums CG
//    per-lane partials over the wave with CG - 1 + log2(64/CG) exchanges
//    instead of CG full reductions, on permlane swaps and DPP moves (no LDS);
//  * panel row loads (four consecutive rows: one 16-byte load for FP32, two
//    for FP64), optionally non-temporal.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hd_internal.hpp"

namespace hd {

// ------------------------------------------------------------------ RNG ---

struct PhiloxKey {
  uint32_t k0, k1;
};

__device__ __forceinline__ void philox10(uint32_t& c0, uint32_t& c1,
                                         uint32_t& c2, uint32_t& c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ double open_unit(uint32_t w) {
  return ((double)w + 0.5) * 2.3283064365386963e-10;  // 2^-32
}

// The four normals with indices 4*blk .. 4*blk+3 of stream (key, step, tag).
__device__ __forceinline__ void normals4(PhiloxKey key, uint32_t step,
                                         uint32_t tag, uint64_t blk,
                                         double out[4]) {
  uint32_t c0 = (uint32_t)blk, c1 = step, c2 = tag, c3 = (uint32_t)(blk >> 32);
  philox10(c0, c1, c2, c3, key.k0, key.k1);
  const uint32_t w[4] = {c0, c1, c2, c3};
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const double rad = sqrt(-2.0 * log(open_unit(w[2 * p])));
    const double ang = 6.283185307179586 * open_unit(w[2 * p + 1]);
    double s, c;
    sincos(ang, &s, &c);
    out[2 * p] = rad * c;
    out[2 * p + 1] = rad * s;
  }
}

// A single normal (index i) of the stream.
__device__ __forceinline__ double normal_at(PhiloxKey key, uint32_t step,
                                            uint32_t tag, uint64_t i) {
  double v[4];
  normals4(key, step, tag, i >> 2, v);
  return v[i & 3];
}

// ----------------------------------------------------------- reductions ---

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of v over the workgroup; every thread gets the result.  `scratch`
// holds kWaves doubles.  Contains two barriers.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) r += scratch[w];
  __syncthreads();
  return r;
}

// ------------------------------------------- cross-lane exchanges ------
//
// The reduce-scatter below pairs lane l with a partner whose lane bit OFF
// differs and whose higher bits agree: OFF = 32 and 16 use the gfx950
// permlane swaps (one instruction exchanges the halves of two registers),
// OFF = 8, 4, 2, 1 use DPP moves (row_ror:8, row_half_mirror, and two quad
// permutations).  Partners are l ^ OFF except at OFF = 4, where row_half_mirror
// pairs l with the lane 7 - (l & 7) of the same group of eight; that lane also
// differs in bit 4 and agrees above it, which is all the reduction needs.

__device__ __forceinline__ uint32_t lo_word(double v) {
  return (uint32_t)__builtin_bit_cast(uint64_t, v);
}
__device__ __forceinline__ uint32_t hi_word(double v) {
  return (uint32_t)(__builtin_bit_cast(uint64_t, v) >> 32);
}
__device__ __forceinline__ double from_words(uint32_t lo, uint32_t hi) {
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <int OFF>
constexpr int dpp_ctrl() {
  return OFF == 8 ? 0x128 : OFF == 4 ? 0x141 : OFF == 2 ? 0x4E : 0xB1;
}

// v from the partner lane (OFF = 8, 4, 2, 1).
template <int OFF>
__device__ __forceinline__ double dpp_partner(double v) {
  static_assert(OFF == 8 || OFF == 4 || OFF == 2 || OFF == 1, "OFF");
  const int lo = __builtin_amdgcn_update_dpp(0, (int)lo_word(v), dpp_ctrl<OFF>(),
                                             0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)hi_word(v), dpp_ctrl<OFF>(),
                                             0xF, 0xF, true);
  return from_words((uint32_t)lo, (uint32_t)hi);
}

// Sum of v and the partner lane's v.
template <int OFF>
__device__ __forceinline__ double add_partner(double v) {
  if constexpr (OFF >= 16)
    return v + __shfl_xor(v, OFF, 64);
  else
    return v + dpp_partner<OFF>(v);
}

// One level of the wave reduce-scatter: lanes with the OFF bit set keep the
// upper H partial sums, the others the lower H, and each adds its partner's
// copy of the half it keeps.  Levels are compile-time so that every array
// index is a constant.
template <int H, int OFF, int CG>
__device__ __forceinline__ void rs_level(double (&v)[CG], bool upper) {
#pragma unroll
  for (int q = 0; q < H; ++q) {
    if constexpr (OFF == 32 || OFF == 16) {
      // permlane{32,16}_swap exchange the odd rows (of OFF lanes) of the
      // first operand with the even rows of the second: afterwards lanes
      // of even rows hold (own v[q], partner v[q]) and lanes of odd rows
      // (partner v[q+H], own v[q+H]).
      const double a = v[q], b = v[q + H];
      uint32_t l0, l1, h0, h1;
      if constexpr (OFF == 32) {
        const auto L = __builtin_amdgcn_permlane32_swap(lo_word(a), lo_word(b),
                                                        false, false);
        const auto U = __builtin_amdgcn_permlane32_swap(hi_word(a), hi_word(b),
                                                        false, false);
        l0 = L[0]; l1 = L[1]; h0 = U[0]; h1 = U[1];
      } else {
        const auto L = __builtin_amdgcn_permlane16_swap(lo_word(a), lo_word(b),
                                                        false, false);
        const auto U = __builtin_amdgcn_permlane16_swap(hi_word(a), hi_word(b),
                                                        false, false);
        l0 = L[0]; l1 = L[1]; h0 = U[0]; h1 = U[1];
      }
      // even rows: own + partner; odd rows: partner + own (the same sum)
      const double x = from_words(l0, h0), y = from_words(l1, h1);
      v[q] = x + y;
    } else {
      const double send = upper ? v[q] : v[q + H];
      const double keep = upper ? v[q + H] : v[q];
      v[q] = keep + dpp_partner<OFF>(send);
    }
  }
}

template <int H, int OFF, int CG>
__device__ __forceinline__ void rs_levels(double (&v)[CG], int lane) {
  if constexpr (H >= 1) {
    rs_level<H, OFF, CG>(v, (lane & OFF) != 0);
    rs_levels<H / 2, OFF / 2, CG>(v, lane);
  }
}

template <int OFF>
__device__ __forceinline__ double rs_tail(double r) {
  if constexpr (OFF >= 1)
    return rs_tail<OFF / 2>(add_partner<OFF>(r));
  else
    return r;
}

// Reduce-scatter over one wave: each lane holds CG partial sums v[0..CG-1]
// (one per column).  On return, lanes with lane % (64/CG) == 0 hold in the
// result the wave total of column lane / (64/CG).  CG must be a power of two
// no larger than 64.  v is clobbered.
template <int CG>
__device__ __forceinline__ double wave_reduce_scatter(double (&v)[CG]) {
  static_assert(CG >= 1 && CG <= 64 && (CG & (CG - 1)) == 0, "CG");
  const int lane = threadIdx.x & 63;
  rs_levels<CG / 2, 32, CG>(v, lane);
  return rs_tail<32 / CG>(v[0]);
}

// ---------------------------------------------------------------- loads ---

// NT: non-temporal loads, for panel streams that nothing re-reads (they
// then do not displace reusable lines from the caches).
typedef float hd_f4 __attribute__((ext_vector_type(4)));
typedef double hd_d2 __attribute__((ext_vector_type(2)));

template <bool NT>
__device__ __forceinline__ void load4(const float* __restrict__ p,
                                      double out[4]) {
  hd_f4 v;
  if constexpr (NT)
    v = __builtin_nontemporal_load((const hd_f4*)p);
  else
    v = *(const hd_f4*)p;
  out[0] = v.x;
  out[1] = v.y;
  out[2] = v.z;
  out[3] = v.w;
}

template <bool NT>
__device__ __forceinline__ void load4(const double* __restrict__ p,
                                      double out[4]) {
  hd_d2 a, b;
  if constexpr (NT) {
    a = __builtin_nontemporal_load((const hd_d2*)p);
    b = __builtin_nontemporal_load((const hd_d2*)(p + 2));
  } else {
    a = *(const hd_d2*)p;
    b = *(const hd_d2*)(p + 2);
  }
  out[0] = a.x;
  out[1] = a.y;
  out[2] = b.x;
  out[3] = b.y;
}

}  // namespace hd
