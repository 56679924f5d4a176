// Device-side building blocks for the Householder Dice kernels (gfx950).
//
//  * counter-based normal draws: Philox4x32-10 (Salmon et al., SC'11) feeding
//    Box-Muller (1958) in FP64, keyed exactly as the library documents
//    (key = (seed, trial), counter = (lo32(i/4), step, tag, hi32(i/4)));
//  * 64-lane wavefront reductions, including a reduce-scatter that sums CG
//    per-lane partials over the wave with CG - 1 + log2(64/CG) shuffles
//    instead of CG full reductions;
//  * panel row loads (one 16-byte load per column for four FP32 rows).
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

// Reduce-scatter over one wave: each lane holds CG partial sums v[0..CG-1]
// (one per column).  On return, lanes with lane % (64/CG) == 0 hold in the
// result the wave total of column lane / (64/CG).  CG must be a power of two
// no larger than 64.  v is clobbered.
template <int CG>
__device__ __forceinline__ double wave_reduce_scatter(double (&v)[CG]) {
  const int lane = threadIdx.x & 63;
  int off = 32;
#pragma unroll
  for (int h = CG / 2; h >= 1; h >>= 1) {
    const bool upper = (lane & off) != 0;
#pragma unroll
    for (int q = 0; q < h; ++q) {
      const double send = upper ? v[q] : v[q + h];
      const double keep = upper ? v[q + h] : v[q];
      v[q] = keep + __shfl_xor(send, off, 64);
    }
    off >>= 1;
  }
  double r = v[0];
#pragma unroll
  for (int o = 32 / CG; o >= 1; o >>= 1) r += __shfl_xor(r, o, 64);
  return r;
}

// out[slot] = sum_{w0 <= w < w1} P[w * pstride + slot] in increasing w, one
// thread per slot; loads are issued eight rows at a time.  Ends with a
// barrier.
__device__ __forceinline__ void reduce_rows(const double* P, int pstride,
                                            int w0, int w1, SlotRanges rg,
                                            double* out) {
  const int total = rg.count[0] + rg.count[1] + rg.count[2];
  for (int s = threadIdx.x; s < total; s += kWG) {
    int slot;
    if (s < rg.count[0])
      slot = rg.start[0] + s;
    else if (s - rg.count[0] < rg.count[1])
      slot = rg.start[1] + (s - rg.count[0]);
    else
      slot = rg.start[2] + (s - rg.count[0] - rg.count[1]);
    const double* col = P + slot;
    double acc = 0.0;
    int w = w0;
    for (; w + 8 <= w1; w += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = col[(int64_t)(w + q) * pstride];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc += v[q];
    }
    for (; w < w1; ++w) acc += col[(int64_t)w * pstride];
    out[slot] = acc;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- loads ---

__device__ __forceinline__ void load4(const float* __restrict__ p,
                                      double out[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  out[0] = v.x;
  out[1] = v.y;
  out[2] = v.z;
  out[3] = v.w;
}

__device__ __forceinline__ void load4(const double* __restrict__ p,
                                      double out[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  out[0] = a.x;
  out[1] = a.y;
  out[2] = b.x;
  out[3] = b.y;
}

// RPL consecutive panel entries of one lane (RPL = 4: one 16-byte load for
// FP32, two for FP64; RPL = 1: one element).
template <int RPL, typename T>
__device__ __forceinline__ void load_rows(const T* __restrict__ p,
                                          double (&out)[RPL]) {
  if constexpr (RPL == 4) {
    load4(p, out);
  } else {
#pragma unroll
    for (int e = 0; e < RPL; ++e) out[e] = (double)p[e];
  }
}

}  // namespace hd
