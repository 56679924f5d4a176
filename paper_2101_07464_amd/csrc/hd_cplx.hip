// hd_cplx.hip -- complex Householder Dice (Sec. 3.4): the complex Ginibre
// ensemble, the Haar ensemble on the unitary group U(n) and, as two queries,
// the Gaussian unitary ensemble.  Kernels and the C-ABI runtime of complex
// handles (hd_c*).
//
// Reflectors are the unitary ones of eq. (Householder_c).  With
// v_1 / ||v|| = r e^{i theta},
//   H(v) = c (I - tau u u^H),  u = v + e^{i theta} ||v|| e_1,
//   c = -e^{-i theta},  tau = 1 / (||v||^2 (1 + r)) = 2 / ||u||^2,
// and H_k(p) acts on entries k.. as in eq. (Householder_e).  The phase c_j of
// reflector j acts on entries >= j, so it commutes with every later
// reflector, and a product of the first K reflectors of a side factors as
//   H_K .. H_1 = Delta (I - U T^H U^H),   H_1^H .. H_K^H = (I - U T U^H) Delta^*,
// with U the panel of u's (column j zero above row j), T the upper
// triangular compact-WY factor of (I - tau_1 u_1 u_1^H)..(I - tau_K u_K u_K^H)
// and Delta = diag(delta_min(i, K-1)), delta_j = c_0 .. c_j (a phase prefix,
// the complex form of the real path's sign prefix).
//
// One query (data side D: the side whose reflector is built from the query
// vector; random side G), in launches:
//   L1  dots: w = U_D^H x (and d = B_D^H x on Ginibre) | random side: the dots
//       of U_G with the fresh draw g (and, on Haar, g written into the new
//       column of U_G with its norm and pivot); the panel whose last column
//       came from the previous query's data pass also dots its earlier
//       columns with that column, in the same sweep;
//   S1  that pending T column, then z = T_D^H w;
//   L2  data pass: p = Delta_D (x - U_D z); rows below the new reflector's
//       index k are kept (head), row k is its pivot, rows > k its column
//       (its T column waits for the next L1, which streams the panel anyway);
//   S2  the new reflectors' scalars (and, on Haar, the draw side's T column),
//       then the coefficients of the output;
//   L3  output pass over the random side: Haar y = (I - U_G T_G U_G^H)
//       Delta_G^* (p_head, ||p_tail||, 0..); Ginibre (Alg. 1 with ^H)
//       y = sigma (B_G a + nu u_t + Delta^* b - U_G c_b) and the new explicit
//       basis column u_t = Delta^* Z g - U_G c'.
// Every panel kernel is row-split: a thread owns four rows (strided by 64, so
// each load instruction of a wave covers 64 consecutive complex entries);
// dots are summed over the wave with the reduce-scatter of hd_device.hpp and
// written as per-wave partial rows, which k_cx_reduce1/2 sum in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include <hip/hip_ext.h>

#include "hd.h"
#include "hd_device.hpp"

namespace hd {
namespace cx {

constexpr int kRPT = 4;                 // rows per thread
constexpr int kRowsWave = 64 * kRPT;    // 256
constexpr int kRowsWG = kWG * kRPT;     // 1024 rows per workgroup
constexpr int kMaxT = 1024;             // queries per handle
constexpr double kRs2 = 0.70710678118654752440;  // 1 / sqrt(2)

// Layout of the reduced FP64 values (and of every partial row): complex
// values as (re, im) pairs.
struct RedLay {
  int w, d, e, t, s, end;
};
inline RedLay red_lay(int kmax) {
  RedLay r;
  r.w = 0;             // U_D^H x
  r.d = 2 * kmax;      // B_D^H x (Ginibre)
  r.e = 4 * kmax;      // random-side dots with the draw
  r.t = 6 * kmax;      // pending column: earlier columns with it
  r.s = 8 * kmax;      // [0] ssq of the data tail, [1] ssq of the draw tail
  r.end = 8 * kmax + 8;
  return r;
}

// Coefficient vectors read by the passes (complex pairs).
struct CoefLay {
  int z, c1, c2, c3, s, end;
};
inline CoefLay coef_lay(int kmax) {
  CoefLay c;
  c.z = 0;
  c.c1 = 2 * (kmax + 1);
  c.c2 = 4 * (kmax + 1);
  c.c3 = 6 * (kmax + 1);
  c.s = 8 * (kmax + 1);
  c.end = 10 * (kmax + 1);
  return c;
}

// Per-reflector FP64 scalars.
enum {
  kRefNu = 0, kRefR, kRefCos, kRefSin, kRefTau, kRefIdent,
  kRefUp = 6,  // pivot entry of u (complex, FP64)
  kRefStride = 8
};
// Scalars.
enum {
  kScPivD = 0,   // pivot of the data tail (complex)
  kScPivG = 2,   // pivot of the draw tail (complex, Haar)
  kScNuD = 4,    // ||data tail||
  kScPh = 6,     // phase of the fresh basis column (complex, Ginibre)
  kScCount = 8
};

struct cd {
  double re, im;
};
__device__ __forceinline__ cd cmul(cd a, cd b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cd cjmul(cd a, cd b) {  // conj(a) * b
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cscale(double s, cd a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cd cconj(cd a) { return {a.re, -a.im}; }
__device__ __forceinline__ cd ld2(const double* p) { return {p[0], p[1]}; }
__device__ __forceinline__ void st2(double* p, cd v) {
  p[0] = v.re;
  p[1] = v.im;
}

template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
  using V = float2;
};
template <>
struct Vec2<double> {
  using V = double2;
};

// Complex entry i of a panel column / vector in storage type T.
template <typename T>
__device__ __forceinline__ cd ldc(const T* __restrict__ p, int64_t i) {
  const typename Vec2<T>::V v = *(const typename Vec2<T>::V*)(p + 2 * i);
  return {(double)v.x, (double)v.y};
}
template <typename T>
__device__ __forceinline__ void stc(T* p, int64_t i, cd v) {
  typename Vec2<T>::V w;
  w.x = (T)v.re;
  w.y = (T)v.im;
  *(typename Vec2<T>::V*)(p + 2 * i) = w;
}
template <typename T>
__device__ __forceinline__ cd roundc(cd v) {
  return {(double)(T)v.re, (double)(T)v.im};
}

// Complex normal i of the stream (key, step, tag 0): real normals 2i and
// 2i + 1 of the documented real stream, i.e. the two halves of one
// Box-Muller pair of Philox block i / 2, scaled by 1/sqrt(2).
__device__ __forceinline__ cd cdraw(PhiloxKey key, uint32_t step, int64_t i) {
  const uint64_t blk = (uint64_t)i >> 1;
  uint32_t c0 = (uint32_t)blk, c1 = step, c2 = 0u, c3 = (uint32_t)(blk >> 32);
  philox10(c0, c1, c2, c3, key.k0, key.k1);
  const bool hi = (i & 1) != 0;
  const double rad = sqrt(-2.0 * log(open_unit(hi ? c2 : c0)));
  const double ang = 6.283185307179586 * open_unit(hi ? c3 : c1);
  double s, c;
  sincos(ang, &s, &c);
  return {rad * c * kRs2, rad * s * kRs2};
}

__device__ __forceinline__ int64_t row_of(int64_t blk, int e) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return blk * kRowsWG + wave * kRowsWave + e * 64 + lane;
}

// Partial dots over this wave's rows: out0[2 j] + i out0[2 j + 1] =
// sum_i conj(P[i, j]) b0_i for j < nc and, with NR = 2, likewise b1 into
// out1 for j < nc1 (out: this wave's partial row), each panel entry loaded
// once.  Every panel row up to ld is allocated and zero beyond the dimension.
template <typename T, int NR>
__device__ __forceinline__ void cdots(const T* __restrict__ P, int64_t ld,
                                      int nc, const int64_t (&row)[kRPT],
                                      const cd (&b0)[kRPT],
                                      const cd (&b1)[kRPT], int nc1,
                                      double* out0, double* out1) {
  constexpr int CG = 4 / NR;
  constexpr int NV = 2 * CG * NR;
  constexpr int kStep = 64 / NV;
  using V2 = typename Vec2<T>::V;
  const int lane = threadIdx.x & 63;
  // four complex columns per group (two with two right-hand sides); the raw
  // entries of the next group are loaded before the current group's
  // products and reduction, so two groups of loads are in flight (138 VGPRs,
  // three waves per SIMD in complex64: 2% faster than one group at 104 VGPRs
  // and four waves)
  V2 cur[CG][kRPT], nxt[CG][kRPT];
  auto load = [&](int j0, V2 (&buf)[CG][kRPT]) {
#pragma unroll
    for (int c = 0; c < CG; ++c) {
      const int j = min(j0 + c, nc - 1);
      const T* __restrict__ col = P + 2 * (int64_t)j * ld;
#pragma unroll
      for (int e = 0; e < kRPT; ++e)
        buf[c][e] = *(const V2*)(col + 2 * row[e]);
    }
  };
  if (nc > 0) load(0, cur);
  for (int j0 = 0; j0 < nc; j0 += CG) {
    if (j0 + CG < nc) load(j0 + CG, nxt);
    double v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = 0.0;
#pragma unroll
    for (int c = 0; c < CG; ++c) {
      if (j0 + c < nc) {
#pragma unroll
        for (int e = 0; e < kRPT; ++e) {
          const cd u{(double)cur[c][e].x, (double)cur[c][e].y};
          v[2 * c] += u.re * b0[e].re + u.im * b0[e].im;
          v[2 * c + 1] += u.re * b0[e].im - u.im * b0[e].re;
          if (NR == 2) {
            v[2 * CG + 2 * c] += u.re * b1[e].re + u.im * b1[e].im;
            v[2 * CG + 2 * c + 1] += u.re * b1[e].im - u.im * b1[e].re;
          }
        }
      }
    }
    const double r = wave_reduce_scatter<NV>(v);
    if (lane % kStep == 0) {
      const int q = lane / kStep;
      if (q < 2 * CG) {
        if (j0 + q / 2 < nc) out0[2 * j0 + q] = r;
      } else if (NR == 2) {
        const int q1 = q - 2 * CG;
        if (j0 + q1 / 2 < nc1) out1[2 * j0 + q1] = r;
      }
    }
    if (j0 + CG < nc) {
#pragma unroll
      for (int c = 0; c < CG; ++c)
#pragma unroll
        for (int e = 0; e < kRPT; ++e) cur[c][e] = nxt[c][e];
    }
  }
}

// acc[e] -= sum_{j < nc} P[row_e, j] coef_j  (coef: complex FP64 pairs)
template <typename T>
__device__ __forceinline__ void cgemv(const T* __restrict__ P, int64_t ld,
                                      int nc, const int64_t (&row)[kRPT],
                                      const double* __restrict__ coef,
                                      cd (&acc)[kRPT]) {
  int j = 0;
  for (; j + 4 <= nc; j += 4) {
    cd u[4][kRPT];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int e = 0; e < kRPT; ++e)
        u[c][e] = ldc<T>(P + 2 * (int64_t)(j + c) * ld, row[e]);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const cd z = ld2(coef + 2 * (j + c));
#pragma unroll
      for (int e = 0; e < kRPT; ++e) acc[e] = csub(acc[e], cmul(u[c][e], z));
    }
  }
  for (; j < nc; ++j) {
    const cd z = ld2(coef + 2 * j);
#pragma unroll
    for (int e = 0; e < kRPT; ++e)
      acc[e] = csub(acc[e], cmul(ldc<T>(P + 2 * (int64_t)j * ld, row[e]), z));
  }
}

// acc[e] -= sum_{j < nc} P[row_e, j] coef_j and, in the same sweep, the
// partial dots out[2 j] + i out[2 j + 1] = sum over the wave's rows of
// conj(P[i, j]) b_i (each panel entry loaded once).
template <typename T>
__device__ __forceinline__ void cgemv_dots(const T* __restrict__ P,
                                           int64_t ld, int nc,
                                           const int64_t (&row)[kRPT],
                                           const double* __restrict__ coef,
                                           cd (&acc)[kRPT],
                                           const cd (&b)[kRPT], double* out) {
  constexpr int CG = 4;
  constexpr int NV = 2 * CG;
  constexpr int kStep = 64 / NV;
  const int lane = threadIdx.x & 63;
  for (int j0 = 0; j0 < nc; j0 += CG) {
    double v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = 0.0;
#pragma unroll
    for (int c = 0; c < CG; ++c) {
      if (j0 + c < nc) {
        const T* __restrict__ col = P + 2 * (int64_t)(j0 + c) * ld;
        const cd z = ld2(coef + 2 * (j0 + c));
#pragma unroll
        for (int e = 0; e < kRPT; ++e) {
          const cd u = ldc<T>(col, row[e]);
          acc[e] = csub(acc[e], cmul(u, z));
          v[2 * c] += u.re * b[e].re + u.im * b[e].im;
          v[2 * c + 1] += u.re * b[e].im - u.im * b[e].re;
        }
      }
    }
    const double r = wave_reduce_scatter<NV>(v);
    if (lane % kStep == 0) {
      const int q = lane / kStep;
      if (j0 + q / 2 < nc) out[2 * j0 + q] = r;
    }
  }
}

// Two coefficient sets over one panel in one sweep.
template <typename T>
__device__ __forceinline__ void cgemv2(const T* __restrict__ P, int64_t ld,
                                       int nc, const int64_t (&row)[kRPT],
                                       const double* __restrict__ c1,
                                       const double* __restrict__ c2,
                                       cd (&a1)[kRPT], cd (&a2)[kRPT]) {
  for (int j = 0; j < nc; ++j) {
    const cd z1 = ld2(c1 + 2 * j), z2 = ld2(c2 + 2 * j);
#pragma unroll
    for (int e = 0; e < kRPT; ++e) {
      const cd u = ldc<T>(P + 2 * (int64_t)j * ld, row[e]);
      a1[e] = csub(a1[e], cmul(u, z1));
      a2[e] = csub(a2[e], cmul(u, z2));
    }
  }
}

// ------------------------------------------------------------- L1 dots --

struct DotsJob {
  const void* P1;
  const void* P2;
  int nc1, nc2;
  int64_t ld, dim;
  const void* x;       // the vector, or null: the draw of (key, step)
  PhiloxKey key;
  uint32_t step;
  int64_t glo;         // drawn rows >= glo
  void* wcol;          // non-null: rows > glo of the draw written here
  double* piv;         // non-null: the draw's row glo (FP64) written here
  double* part;        // per-wave partial rows (pstride doubles each)
  int pstride;
  int slot1, slot2;    // partial slots of the P1 and P2 dots
  int ssq_slot;        // >= 0: sum |b_i|^2 over rows >= glo
  int pk;              // >= 0: P1's column pk (rows > pk) is a second
  int pslot;           //   right-hand side for its columns < pk (slots pslot)
  int nwg;
};

template <typename T>
__device__ __forceinline__ void dots_job(const DotsJob& j, int64_t blk) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t row[kRPT];
  cd b[kRPT];
  double ssq = 0.0;
#pragma unroll
  for (int e = 0; e < kRPT; ++e) {
    row[e] = row_of(blk, e);
    const int64_t i = row[e];
    cd v{0.0, 0.0};
    if (i < j.dim) {
      if (j.x) {
        v = ldc<T>((const T*)j.x, i);
      } else if (i >= j.glo) {
        v = cdraw(j.key, j.step, i);
        if (i > j.glo && j.wcol) {
          v = roundc<T>(v);
          stc<T>((T*)j.wcol, i, v);
        }
      }
      if (i >= j.glo) ssq += v.re * v.re + v.im * v.im;
      if (i == j.glo && j.piv) {
        // the pivot row of a new column enters its dots in the small step,
        // with the pivot of u
        st2(j.piv, v);
        v = {0.0, 0.0};
      }
    }
    b[e] = v;
  }
  double* out = j.part + (blk * kWaves + wave) * (int64_t)j.pstride;
  if (j.pk >= 0) {
    // the pending T column of this panel: the dots of its earlier columns
    // with column pk (rows > pk), in the same sweep as the dots with b
    const T* pc = (const T*)j.P1 + 2 * (int64_t)j.pk * j.ld;
    cd b1[kRPT];
#pragma unroll
    for (int e = 0; e < kRPT; ++e)
      b1[e] = row[e] > j.pk ? ldc<T>(pc, row[e]) : cd{0.0, 0.0};
    cdots<T, 2>((const T*)j.P1, j.ld, j.nc1, row, b, b1, j.pk,
                out + j.slot1, out + j.pslot);
  } else if (j.nc1 > 0) {
    cdots<T, 1>((const T*)j.P1, j.ld, j.nc1, row, b, b, 0, out + j.slot1,
                nullptr);
  }
  if (j.nc2 > 0)
    cdots<T, 1>((const T*)j.P2, j.ld, j.nc2, row, b, b, 0, out + j.slot2,
                nullptr);
  if (j.ssq_slot >= 0) {
    const double s = wave_sum(ssq);
    if (lane == 0) out[j.ssq_slot] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_cx_dots(DotsJob j0, DotsJob j1) {
  const int64_t b = blockIdx.x;
  if (b < j0.nwg)
    dots_job<T>(j0, b);
  else
    dots_job<T>(j1, b - j0.nwg);
}

// ------------------------------------------------------------- reduce ----

struct RedJob {
  const double* part;
  int64_t nrows;
  int pstride;
  int start[3], count[3];  // slot ranges
  double* out;             // out[slot] = sum over rows of part[row][slot]
  double* stage;           // block partials of the first stage
};

constexpr int kRedRows = 256;  // rows per block of the first stage
constexpr int kRedSlots = 32;  // slots per block of the first stage

__device__ __forceinline__ int red_slots(const RedJob& j) {
  return j.count[0] + j.count[1] + j.count[2];
}
__device__ __forceinline__ int red_slot(const RedJob& j, int q) {
  int slot = -1;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    if (slot < 0) {
      if (q < j.count[r])
        slot = j.start[r] + q;
      else
        q -= j.count[r];
    }
  }
  return slot;
}
__device__ __forceinline__ int red_blocks(const RedJob& j) {
  return red_slots(j) ? (int)((j.nrows + kRedRows - 1) / kRedRows) : 0;
}

__device__ __forceinline__ int red_groups(const RedJob& j) {
  return (red_slots(j) + kRedSlots - 1) / kRedSlots;
}

// Two-stage fixed-order sums of the partial rows.  Stage 1: a block takes R
// rows and 32 consecutive slots of one job; its 8 x 32 threads sum rows
// r = rl, rl + 8, ... (each row read as a contiguous run of slots), then
// the 8 row lanes are added in order.  Stage 2: one thread per slot adds the
// row blocks in order.
__global__ __launch_bounds__(kWG) void k_cx_reduce1(RedJob a, RedJob b) {
  __shared__ double lds[kWG];
  const int na = red_blocks(a) * red_groups(a);
  const bool first = (int)blockIdx.x < na;
  const RedJob& j = first ? a : b;
  const int id = first ? (int)blockIdx.x : (int)blockIdx.x - na;
  const int ng = red_groups(j);
  const int blk = id / ng, sg = id % ng;
  const int ns = red_slots(j);
  const int sl = threadIdx.x % kRedSlots, rl = threadIdx.x / kRedSlots;
  const int q = sg * kRedSlots + sl;
  const int64_t r0 = (int64_t)blk * kRedRows;
  const int64_t r1 = r0 + kRedRows < j.nrows ? r0 + kRedRows : j.nrows;
  double s = 0.0;
  if (q < ns) {
    const int slot = red_slot(j, q);
#pragma unroll 8
    for (int64_t r = r0 + rl; r < r1; r += kWG / kRedSlots)
      s += j.part[r * j.pstride + slot];
  }
  lds[threadIdx.x] = s;
  __syncthreads();
  if (rl == 0 && q < ns) {
    double t = 0.0;
    for (int k = 0; k < kWG / kRedSlots; ++k) t += lds[k * kRedSlots + sl];
    j.stage[(int64_t)blk * ns + q] = t;
  }
}

// Stage 2: a block takes 32 consecutive slots of one job; its 8 x 32
// threads add row blocks k = rl, rl + 8, ..., then the 8 row lanes in order.
__global__ __launch_bounds__(kWG) void k_cx_reduce2(RedJob a, RedJob b) {
  __shared__ double lds[kWG];
  const int ga = red_groups(a);
  const bool first = (int)blockIdx.x < ga;
  const RedJob& j = first ? a : b;
  const int sg = first ? (int)blockIdx.x : (int)blockIdx.x - ga;
  const int ns = red_slots(j), nb = red_blocks(j);
  const int sl = threadIdx.x % kRedSlots, rl = threadIdx.x / kRedSlots;
  const int q = sg * kRedSlots + sl;
  double s = 0.0;
  if (q < ns)
    for (int k = rl; k < nb; k += kWG / kRedSlots)
      s += j.stage[(int64_t)k * ns + q];
  lds[threadIdx.x] = s;
  __syncthreads();
  if (rl == 0 && q < ns) {
    double t = 0.0;
    for (int k = 0; k < kWG / kRedSlots; ++k) t += lds[k * kRedSlots + sl];
    j.out[red_slot(j, q)] = t;
  }
}

// ------------------------------------------------------------ L2 / L3 ----

enum { kModeData = 0, kModeHaarOut = 1, kModeGinOut = 2 };

struct CxPassArgs {
  const void* U;     // reflector panel of the pass's side
  const void* B;     // basis panel (Ginibre output pass)
  int64_t ld, dim;
  int k;             // columns of U used (data: old reflectors)
  int kb;            // columns of B used (Ginibre)
  const double* coef;  // LayCoef base
  CoefLay cl;
  const double* del;   // phase prefix of the data side (data pass)
  // data pass
  const void* x;
  double* head;        // rows < k of p (FP64), and row k
  double* piv;
  void* newcol;        // column k of U (rows > k)
  double* part;
  int pstride, ssq_slot;
  // output passes
  void* y;
  const void* comb;    // non-null: y = (comb + y) / sqrt(2)
  void* bcol;          // Ginibre: the new basis column
  const double* scal;
  double sigma;
  PhiloxKey key;
  uint32_t step;
  int64_t glo;         // Ginibre: drawn rows >= glo
  // fused map x_next = tanh(ma |y|) e^{i arg y} + mb x (Haar output pass)
  const void* xmap;
  void* xnext;
  double ma, mb;
  // Haar output pass, lookahead (pf): the next query's draw (step pf_step,
  // rows >= k + 1) written as column k + 1 (rows > k + 1), its pivot and
  // the norm of its tail, and its dots with columns 0..k -- what the next
  // query's dots launch would compute for this side
  int pf;
  uint32_t pf_step;
  void* pf_col;
  double* pf_piv;
  int pf_slot, pf_ssq;
};

template <typename T, int MODE>
__global__ __launch_bounds__(kWG) void k_cx_pass(CxPassArgs a) {
  const int64_t blk = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t row[kRPT];
  cd acc[kRPT], acc2[kRPT];
#pragma unroll
  for (int e = 0; e < kRPT; ++e) {
    row[e] = row_of(blk, e);
    acc[e] = {0.0, 0.0};
    acc2[e] = {0.0, 0.0};
  }
  const T* __restrict__ U = (const T*)a.U;
  if (MODE == kModeData) {
    cgemv<T>(U, a.ld, a.k, row, a.coef + a.cl.z, acc);
    const int k = a.k;
    double ssq = 0.0;
#pragma unroll
    for (int e = 0; e < kRPT; ++e) {
      const int64_t i = row[e];
      if (i < a.dim) {
        cd p = cadd(ldc<T>((const T*)a.x, i), acc[e]);
        if (k > 0) p = cmul(ld2(a.del + 2 * (i < k ? i : k - 1)), p);
        if (i < k) {
          st2(a.head + 2 * i, p);
        } else if (i == k) {
          st2(a.head + 2 * i, p);
          st2(a.piv, p);
          ssq += p.re * p.re + p.im * p.im;
        } else {
          const cd un = roundc<T>(p);
          stc<T>((T*)a.newcol, i, un);
          ssq += un.re * un.re + un.im * un.im;
        }
      }
    }
    double* out = a.part + (blk * kWaves + wave) * (int64_t)a.pstride;
    const double s = wave_sum(ssq);
    if (lane == 0) out[a.ssq_slot] = s;
    return;
  }
  if (MODE == kModeHaarOut) {
    // y = s - U c over k + 1 columns (s: rows <= k)
    if (a.pf) {
      const int64_t lo = a.k + 1;
      cd b[kRPT];
      double ssq = 0.0;
#pragma unroll
      for (int e = 0; e < kRPT; ++e) {
        const int64_t i = row[e];
        cd v{0.0, 0.0};
        if (i < a.dim && i >= lo) {
          v = cdraw(a.key, a.pf_step, i);
          if (i > lo) {
            v = roundc<T>(v);
            stc<T>((T*)a.pf_col, i, v);
          }
          ssq += v.re * v.re + v.im * v.im;
          if (i == lo) {
            st2(a.pf_piv, v);
            v = {0.0, 0.0};
          }
        }
        b[e] = v;
      }
      double* out = a.part + (blk * kWaves + wave) * (int64_t)a.pstride;
      cgemv_dots<T>(U, a.ld, a.k + 1, row, a.coef + a.cl.c1, acc, b,
                    out + a.pf_slot);
      const double sq = wave_sum(ssq);
      if (lane == 0) out[a.pf_ssq] = sq;
    } else {
      cgemv<T>(U, a.ld, a.k + 1, row, a.coef + a.cl.c1, acc);
    }
#pragma unroll
    for (int e = 0; e < kRPT; ++e) {
      const int64_t i = row[e];
      if (i >= a.dim) continue;
      cd y = acc[e];
      if (i <= a.k) y = cadd(y, ld2(a.coef + a.cl.s + 2 * i));
      if (a.comb) y = cscale(kRs2, cadd(y, ldc<T>((const T*)a.comb, i)));
      const cd ys = roundc<T>(y);
      if (a.y) stc<T>((T*)a.y, i, ys);
      if (a.xnext) {
        const double mag = sqrt(ys.re * ys.re + ys.im * ys.im);
        cd xn = cscale(a.mb, ldc<T>((const T*)a.xmap, i));
        if (mag > 0.0) xn = cadd(xn, cscale(tanh(a.ma * mag) / mag, ys));
        stc<T>((T*)a.xnext, i, xn);
      }
    }
    return;
  }
  // Ginibre output pass: acc = -U c', acc2 = -U c_b, then the basis panel
  cgemv2<T>(U, a.ld, a.k, row, a.coef + a.cl.c2, a.coef + a.cl.c3, acc, acc2);
  cd bsum[kRPT];
#pragma unroll
  for (int e = 0; e < kRPT; ++e) bsum[e] = {0.0, 0.0};
  cgemv<T>((const T*)a.B, a.ld, a.kb, row, a.coef + a.cl.c1, bsum);
  const cd ph = ld2(a.scal + kScPh);
  const double nu = a.scal[kScNuD];
#pragma unroll
  for (int e = 0; e < kRPT; ++e) {
    const int64_t i = row[e];
    if (i >= a.dim) continue;
    cd un = acc[e];
    if (i >= a.glo) un = cadd(un, cmul(ph, cdraw(a.key, a.step, i)));
    un = roundc<T>(un);
    stc<T>((T*)a.bcol, i, un);
    // bsum holds -(B a): y = sigma (B a + nu u_t + s - U c_b)
    cd y = cadd(csub(acc2[e], bsum[e]), cscale(nu, un));
    if (i < a.k) y = cadd(y, ld2(a.coef + a.cl.s + 2 * i));
    y = cscale(a.sigma, y);
    if (a.comb) y = cscale(kRs2, cadd(y, ldc<T>((const T*)a.comb, i)));
    stc<T>((T*)a.y, i, y);
  }
}

// -------------------------------------------------------------- small ----

struct SideDev {
  void* U;
  int64_t ld;
  double* T;     // kmax x kmax complex, column-major
  double* ref;   // kRefStride per reflector
  double* del;   // phase prefix (complex)
};

struct SmallArgs {
  SideDev D, G;
  int kmax;
  int kD, kG;          // reflectors before this query
  const double* red;
  RedLay rl;
  double* coef;
  CoefLay cl;
  const double* head;  // data side p, rows <= kD
  double* scal;
  int* flag;
  int f64;
  SideDev P;           // side with a pending T column (pk >= 0)
  int pk;
};

__device__ __forceinline__ double* tij(double* T, int kmax, int i, int j) {
  return T + 2 * ((int64_t)i + (int64_t)j * kmax);
}

// Panel entry (row i, column j) of a side stored as T.
template <typename T>
__device__ __forceinline__ cd uent_t(const SideDev& S, int64_t i, int j) {
  return ldc<T>((const T*)S.U + 2 * (int64_t)j * S.ld, i);
}
// The same in the side's storage type.
__device__ __forceinline__ cd uent(const SideDev& S, int f64, int64_t i,
                                   int j) {
  return f64 ? uent_t<double>(S, i, j) : uent_t<float>(S, i, j);
}
__device__ __forceinline__ void uset(const SideDev& S, int f64, int64_t i,
                                     int j, cd v) {
  if (f64)
    stc<double>((double*)S.U + 2 * (int64_t)j * S.ld, i, v);
  else
    stc<float>((float*)S.U + 2 * (int64_t)j * S.ld, i, v);
}

// Reflector k of a side from the norm^2 of its tail and its pivot: scalars,
// the pivot entry of its column, and the phase prefix; returns the pivot of
// u in `upiv` (FP64).  One thread.
__device__ void build_reflector(const SideDev& S, int f64, int k, double ss,
                                cd piv, cd& upiv, int* flag) {
  double* rf = S.ref + (int64_t)k * kRefStride;
  const double nu = sqrt(ss);
  if (!isfinite(nu)) atomicOr(flag, 1);
  const double ap = sqrt(piv.re * piv.re + piv.im * piv.im);
  double cth = 1.0, sth = 0.0;
  if (ap > 0.0) {
    cth = piv.re / ap;
    sth = piv.im / ap;
  }
  cd c{1.0, 0.0};  // identity: no phase
  if (nu > 0.0) {
    const double r = ap / nu;
    rf[kRefR] = r;
    rf[kRefTau] = 1.0 / (nu * nu * (1.0 + r));
    rf[kRefIdent] = 0.0;
    upiv = {piv.re + cth * nu, piv.im + sth * nu};
    c = {-cth, sth};  // -e^{-i theta}
  } else {
    rf[kRefR] = 0.0;
    rf[kRefTau] = 0.0;
    rf[kRefIdent] = 1.0;
    upiv = {0.0, 0.0};
  }
  rf[kRefNu] = nu;
  rf[kRefCos] = cth;
  rf[kRefSin] = sth;
  rf[kRefUp] = upiv.re;
  rf[kRefUp + 1] = upiv.im;
  uset(S, f64, k, k, upiv);
  const cd prev = k > 0 ? ld2(S.del + 2 * (k - 1)) : cd{1.0, 0.0};
  st2(S.del + 2 * k, cmul(prev, c));
}

constexpr int kTriGroup = 8;  // loads in flight per lane in t_row_sums

// out(j, s_j) for j < n with s_j = sum over i in [j, n) of T[j, i] v(i):
// the row sums of the leading n x n block of a side's complex T factor
// (column-major, leading dimension kmax, upper triangle set).  The lanes
// take the rows and the waves the columns in turn, so every load reads
// consecutive entries of one column (a thread summing its own row would
// touch one cache line per entry, in a serial chain), and kTriGroup columns
// are loaded before any is added: the indexes are clamped into the upper
// triangle, so no load sits behind a branch (which would wait out each
// load on its own); per block of 64 rows the waves' partial sums are added
// in fixed order through `lds` (kWG entries).  Every thread of the
// workgroup calls it; it ends with a barrier.
template <typename V, typename Out>
__device__ void t_row_sums(const double* __restrict__ T, int kmax, int n,
                           V v, Out out, cd* lds) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int r0 = 0; r0 < n; r0 += 64) {
    const int j = r0 + lane;
    cd s{0.0, 0.0};
    for (int i0 = r0 + wave; i0 < n; i0 += kWaves * kTriGroup) {
      cd t[kTriGroup];
#pragma unroll
      for (int u = 0; u < kTriGroup; ++u) {
        const int i = min(i0 + u * kWaves, n - 1);
        t[u] = cmul(ld2(tij((double*)T, kmax, min(j, i), i)), v(i));
      }
#pragma unroll
      for (int u = 0; u < kTriGroup; ++u) {
        const int i = i0 + u * kWaves;
        if (i < n && j <= i) s = cadd(s, t[u]);
      }
    }
    lds[tid] = s;
    __syncthreads();
    if (wave == 0 && j < n) {
      cd t{0.0, 0.0};
      for (int w = 0; w < kWaves; ++w) t = cadd(t, lds[w * 64 + lane]);
      out(j, t);
    }
    __syncthreads();
  }
}

// out(j, s_j) for j < nc with s_j = sum over i in [lo(j), hi(j)) of
// f(i, j), where f reads column j of a column-major factor (a panel or T),
// lo, hi never decrease with j and lo(j) < hi(j).  Each wave takes CG
// consecutive columns at a time and the lanes the rows, 64 at a time: a
// load reads consecutive entries of one column, and the CG loads of a lane
// are all issued before any is added (one column at a time would wait out
// a memory round trip per 64 rows of every column); f is called with
// indexes clamped into the column, so that no load sits behind a branch.
// A butterfly over the wave adds the lanes' terms of each column.  Every
// thread of the workgroup calls it; no barrier.
template <int CG, typename Lo, typename Hi, typename F, typename Out>
__device__ void col_dots(int nc, Lo lo, Hi hi, F f, Out out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int jb = wave * CG; jb < nc; jb += kWaves * CG) {
    const int jl = min(jb + CG, nc) - 1;
    const int r1 = hi(jl);
    cd s[CG];
#pragma unroll
    for (int c = 0; c < CG; ++c) s[c] = {0.0, 0.0};
    for (int r = lo(jb); r < r1; r += 64) {
      const int i = r + lane;
      cd v[CG];
#pragma unroll
      for (int c = 0; c < CG; ++c) {
        const int j = min(jb + c, jl);
        v[c] = f(min(max(i, lo(j)), hi(j) - 1), j);
      }
#pragma unroll
      for (int c = 0; c < CG; ++c) {
        const int j = jb + c;
        if (j <= jl && i >= lo(j) && i < hi(j)) s[c] = cadd(s[c], v[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < CG; ++c) {
      const double re = wave_sum(s[c].re), im = wave_sum(s[c].im);
      if (lane == 0 && jb + c <= jl) out(jb + c, cd{re, im});
    }
  }
}

// T column k of a side: T[j, k] = -tau sum_{i = j}^{k-1} T[j, i] h_i,
// T[k, k] = tau, with h (LDS) the dots of the old columns with the new one.
__device__ void t_column(const SideDev& S, int kmax, int k, const cd* h,
                         cd* lds) {
  const double tau = S.ref[(int64_t)k * kRefStride + kRefTau];
  double* T = S.T;
  t_row_sums(
      T, kmax, k, [=](int i) { return h[i]; },
      [=](int j, cd s) { st2(tij(T, kmax, j, k), cscale(-tau, s)); }, lds);
  if (threadIdx.x == 0) st2(tij(S.T, kmax, k, k), {tau, 0.0});
}

constexpr int kSmallMax = kMaxT + 1;
constexpr int kColGroup = 8;  // columns per wave in col_dots

// PH 0: z = T_D^H w.  PH 1: Haar S2.  PH 2: Ginibre S2.
template <int PH>
__global__ __launch_bounds__(kWG) void k_cx_small(SmallArgs a) {
  __shared__ cd h[kSmallMax];
  __shared__ cd h2[kSmallMax];
  __shared__ cd piv[2];
  __shared__ cd lds[kWG];
  const int tid = threadIdx.x, kmax = a.kmax;
  if (PH == 0) {
    if (a.pk >= 0) {
      // the pending T column: dots of the earlier columns with the new one,
      // rows > pk from this query's dots launch, the pivot row here
      const int pk = a.pk;
      const cd up = ld2(a.P.ref + (int64_t)pk * kRefStride + kRefUp);
      for (int j = tid; j < pk; j += kWG)
        h[j] = cadd(ld2(a.red + a.rl.t + 2 * j), cjmul(uent(a.P, a.f64, pk, j), up));
      __syncthreads();
      t_column(a.P, kmax, pk, h, lds);
      __syncthreads();
    }
    // z_j = sum over i <= j of conj(T_D[i, j]) w_i
    double* T = a.D.T;
    const double* w = a.red + a.rl.w;
    double* z = a.coef + a.cl.z;
    col_dots<kColGroup>(
        a.kD, [](int) { return 0; }, [](int j) { return j + 1; },
        [=](int i, int j) { return cjmul(ld2(tij(T, kmax, i, j)), ld2(w + 2 * i)); },
        [=](int j, cd v) { st2(z + 2 * j, v); });
    return;
  }
  const int kD = a.kD;
  // the data side's new reflector
  if (tid == 0) {
    cd up;
    build_reflector(a.D, a.f64, kD, a.red[a.rl.s + 0], ld2(a.scal + kScPivD),
                    up, a.flag);
    a.scal[kScNuD] = a.D.ref[(int64_t)kD * kRefStride + kRefNu];
    if (PH == 1) {
      build_reflector(a.G, a.f64, kD, a.red[a.rl.s + 1],
                      ld2(a.scal + kScPivG), up, a.flag);
      piv[1] = up;
    }
  }
  __syncthreads();
  // the data side's T column waits for the next query's dots launch; the
  // draw side's (Haar) is complete: rows > k from this query's dots launch,
  // row k (the pivot) here
  if (PH == 1) {
    for (int j = tid; j < kD; j += kWG)
      h2[j] = cadd(ld2(a.red + a.rl.e + 2 * j), cjmul(uent(a.G, a.f64, kD, j), piv[1]));
    __syncthreads();
    t_column(a.G, kmax, kD, h2, lds);
    __syncthreads();
  }
  if (PH == 1) {
    // s = Delta_G^* (p_0..p_{k-1}, nu_D) over rows <= k, then
    // c = T_G (U_G^H s) over the k + 1 columns
    const int k = kD;
    const double nu = a.scal[kScNuD];
    for (int i = tid; i <= k; i += kWG) {
      const cd r = i < k ? ld2(a.head + 2 * i) : cd{nu, 0.0};
      const cd s = cjmul(ld2(a.G.del + 2 * i), r);
      h[i] = s;
      st2(a.coef + a.cl.s + 2 * i, s);
    }
    __syncthreads();
    // h2_j = sum over i in [j, k] of conj(U_G[i, j]) s_i (the new pivot
    // entry in FP64)
    const SideDev G = a.G;
    const cd pk = piv[1];
    auto dots = [&](auto tag) {
      using T = decltype(tag);
      col_dots<kColGroup>(
          k + 1, [](int j) { return j; }, [=](int) { return k + 1; },
          [=](int i, int j) {
            const cd u = uent_t<T>(G, i, j);
            return cjmul(i == k && j == k ? pk : u, h[i]);
          },
          [=](int j, cd v) { h2[j] = v; });
    };
    if (a.f64)
      dots(double{});
    else
      dots(float{});
    __syncthreads();
    double* coef = a.coef + a.cl.c1;
    t_row_sums(
        a.G.T, kmax, k + 1, [=](int i) { return h2[i]; },
        [=](int j, cd c) { st2(coef + 2 * j, c); }, lds);
    return;
  }
  // PH 2 (Ginibre): G has kG reflectors and gets none
  const int kG = a.kG;
  const cd ph = kG > 0 ? cconj(ld2(a.G.del + 2 * (kG - 1))) : cd{1.0, 0.0};
  if (tid == 0) st2(a.scal + kScPh, ph);
  for (int i = tid; i < kG; i += kWG) {
    // e' = ph e (the dots with Delta^* Z g), s = Delta^* b
    h[i] = cmul(ph, ld2(a.red + a.rl.e + 2 * i));
    const cd s = cjmul(ld2(a.G.del + 2 * i), ld2(a.red + a.rl.d + 2 * i));
    h2[i] = s;
    st2(a.coef + a.cl.s + 2 * i, s);
  }
  for (int j = tid; j <= kD; j += kWG) {
    const cd aj = j < kD ? ld2(a.head + 2 * j) : cd{a.scal[kScNuD], 0.0};
    st2(a.coef + a.cl.c1 + 2 * j, aj);
  }
  __syncthreads();
  // c' = T_G e'; U_G^H s over the head rows (into piv-free scratch h below)
  {
    double* coef = a.coef + a.cl.c2;
    t_row_sums(
        a.G.T, kmax, kG, [=](int i) { return h[i]; },
        [=](int j, cd c) { st2(coef + 2 * j, c); }, lds);
  }
  {
    const SideDev G = a.G;
    auto dots = [&](auto tag) {
      using T = decltype(tag);
      col_dots<kColGroup>(
          kG, [](int j) { return j; }, [=](int) { return kG; },
          [=](int i, int j) { return cjmul(uent_t<T>(G, i, j), h2[i]); },
          [=](int j, cd v) { h[j] = v; });
    };
    if (a.f64)
      dots(double{});
    else
      dots(float{});
  }
  __syncthreads();
  {
    double* coef = a.coef + a.cl.c3;
    t_row_sums(
        a.G.T, kmax, kG, [=](int i) { return h[i]; },
        [=](int j, cd c) { st2(coef + 2 * j, c); }, lds);
  }
}

}  // namespace cx
}  // namespace hd

// =================================================================== host ==

using namespace hd;
using namespace hd::cx;

struct hd_cctx {
  int ens, f64, es;
  int64_t m, n;
  int tmax, kmax;
  uint32_t seed, trial;
  double sigma;
  hipStream_t stream;
  int t, r, l;
  int pend_side, pend_k;  // the side whose last T column is pending
  int pf_side, pf_t;      // draw dots prepared for query pf_t on pf_side
  SideDev S[2];     // 0: R (C^n), 1: L (C^m)
  void* B[2];       // Ginibre basis panels
  int64_t dim[2];
  int nwg[2];
  double* part[2];
  double* stage[2];  // first-stage partials of the two jobs of a reduction
  int pstride;
  RedLay rl;
  CoefLay cl;
  double* red;
  double* coef;
  double* head;
  double* scal;
  int* flag;
  void* ybuf;       // the first answer of a GUE step
  std::vector<void*> allocs;
  // timing of the panel launches (events recorded by the dispatches)
  struct Rec {
    int kind;
    hipEvent_t a, b;
    double bytes;
  };
  int prof = 0;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  std::vector<Rec> recs;
};

namespace {

int cx_fail(hipError_t) { return HD_ERR_HIP; }

#define CXHIP(call)                             \
  do {                                          \
    hipError_t e_ = (call);                     \
    if (e_ != hipSuccess) return cx_fail(e_);   \
  } while (0)

void cx_release(hd_cctx* h) {
  (void)hipStreamSynchronize(h->stream);
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
  for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
  h->pool.clear();
}

// A pair of events for one panel launch when profiling (else null).
bool cx_events(hd_cctx* h, int kind, double bytes, hipEvent_t* a,
               hipEvent_t* b) {
  *a = *b = nullptr;
  if (!h->prof) return false;
  for (int q = 0; q < 2; ++q) {
    if (h->pool_used == h->pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return false;
      h->pool.push_back(e);
    }
    (q ? *b : *a) = h->pool[h->pool_used++];
  }
  h->recs.push_back(hd_cctx::Rec{kind, *a, *b, bytes});
  return true;
}

template <typename... KArgs, typename... Args>
void cx_launch(hd_cctx* h, int kind, double bytes, void (*k)(KArgs...),
               dim3 grid, Args... args) {
  hipEvent_t a, b;
  if (cx_events(h, kind, bytes, &a, &b))
    hipExtLaunchKernelGGL(k, grid, dim3(kWG), 0, h->stream, a, b, 0,
                          args...);
  else
    hipLaunchKernelGGL(k, grid, dim3(kWG), 0, h->stream, args...);
}

template <typename P>
int cx_alloc(hd_cctx* h, P** out, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes ? bytes : 8) != hipSuccess) {
    (void)hipGetLastError();
    return HD_ERR_NOMEM;
  }
  h->allocs.push_back(p);
  *out = (P*)p;
  return HD_OK;
}

int cx_zero_state(hd_cctx* h) {
  // panels, T, scalars: every query reads only what earlier queries wrote,
  // except the zero rows above each panel column's pivot
  for (int s = 0; s < 2; ++s) {
    const size_t pb = (size_t)h->es * h->S[s].ld * h->kmax;
    CXHIP(hipMemsetAsync(h->S[s].U, 0, pb, h->stream));
    if (h->B[s]) CXHIP(hipMemsetAsync(h->B[s], 0, pb, h->stream));
  }
  CXHIP(hipMemsetAsync(h->flag, 0, sizeof(int), h->stream));
  return HD_OK;
}

DotsJob no_job() {
  DotsJob j;
  std::memset(&j, 0, sizeof(j));
  j.ssq_slot = -1;
  j.pk = -1;
  return j;
}

RedJob red_job(const double* part, int64_t nrows, int pstride, double* out) {
  RedJob j;
  std::memset(&j, 0, sizeof(j));
  j.part = part;
  j.nrows = nrows;
  j.pstride = pstride;
  j.out = out;
  return j;
}

// Algorithmic bytes of a dots job: its panel columns and vector read, and
// the new column written.
double dots_bytes(const hd_cctx* h, const DotsJob& j) {
  if (!j.nwg) return 0.0;
  double cols = j.nc1 + j.nc2 + (j.x ? 1 : 0) + (j.wcol ? 1 : 0) +
                (j.pk >= 0 ? 1 : 0);
  return cols * (double)j.dim * h->es;
}

int launch_dots(hd_cctx* h, const DotsJob& a, const DotsJob& b) {
  const int grid = a.nwg + b.nwg;
  if (grid == 0) return HD_OK;
  const double by = dots_bytes(h, a) + dots_bytes(h, b);
  if (h->f64)
    cx_launch(h, 0, by, k_cx_dots<double>, dim3(grid), a, b);
  else
    cx_launch(h, 0, by, k_cx_dots<float>, dim3(grid), a, b);
  CXHIP(hipGetLastError());
  return HD_OK;
}

int launch_reduce(hd_cctx* h, RedJob a, RedJob b) {
  auto slots = [](const RedJob& j) {
    return j.count[0] + j.count[1] + j.count[2];
  };
  auto blocks = [&](const RedJob& j) {
    const int rows = slots(j) ? (int)((j.nrows + kRedRows - 1) / kRedRows) : 0;
    return rows * ((slots(j) + kRedSlots - 1) / kRedSlots);
  };
  const int ns = slots(a) + slots(b);
  if (ns == 0) return HD_OK;
  a.stage = h->stage[0];
  b.stage = h->stage[1];
  hipLaunchKernelGGL(k_cx_reduce1, dim3(blocks(a) + blocks(b)), dim3(kWG), 0,
                     h->stream, a, b);
  CXHIP(hipGetLastError());
  const int groups = (slots(a) + kRedSlots - 1) / kRedSlots +
                     (slots(b) + kRedSlots - 1) / kRedSlots;
  hipLaunchKernelGGL(k_cx_reduce2, dim3(groups), dim3(kWG), 0, h->stream, a,
                     b);
  CXHIP(hipGetLastError());
  return HD_OK;
}

template <int PH>
int launch_small(hd_cctx* h, const SmallArgs& a) {
  hipLaunchKernelGGL(k_cx_small<PH>, dim3(1), dim3(kWG), 0, h->stream, a);
  CXHIP(hipGetLastError());
  return HD_OK;
}

// Algorithmic bytes of a pass: every panel column once, the vectors read
// and written.
template <int MODE>
double pass_bytes(const hd_cctx* h, const CxPassArgs& a) {
  double cols;
  if (MODE == kModeData)
    cols = a.k + 2;  // panel, x, new column
  else if (MODE == kModeHaarOut)
    cols = a.k + 1 + (a.y ? 1 : 0) + (a.xnext ? 2 : 0) + (a.comb ? 1 : 0) +
           (a.pf ? 1 : 0);
  else
    cols = a.k + a.kb + 2 + (a.comb ? 1 : 0);  // panels, new column, y
  return cols * (double)a.dim * h->es;
}

template <int MODE>
int launch_pass(hd_cctx* h, int side, const CxPassArgs& a) {
  const dim3 grid(h->nwg[side]);
  const double by = pass_bytes<MODE>(h, a);
  if (h->f64)
    cx_launch(h, MODE == kModeData ? 1 : 2, by, k_cx_pass<double, MODE>,
              grid, a);
  else
    cx_launch(h, MODE == kModeData ? 1 : 2, by, k_cx_pass<float, MODE>,
              grid, a);
  CXHIP(hipGetLastError());
  return HD_OK;
}

#define CXCHK(call)              \
  do {                           \
    const int rc_ = (call);      \
    if (rc_ != HD_OK) return rc_; \
  } while (0)

// One query: y = Q x (adj = 0) or Q^H x; optional fused map into xnext
// (Haar) and combination (comb + y) / sqrt(2).
int cx_query(hd_cctx* h, int adj, const void* x, void* y, const void* comb,
             const void* xmap, void* xnext, double ma, double mb,
             int lookahead = 0) {
  const int D = adj ? 1 : 0, G = 1 - D;
  const int haar = h->ens == HD_HAAR;
  const int kD = haar ? h->t : (D == 0 ? h->r : h->l);
  const int kG = haar ? h->t : (G == 0 ? h->r : h->l);
  const uint32_t step = (uint32_t)(h->t + 1);
  const PhiloxKey key{h->seed, h->trial};
  const SideDev& SD = h->S[D];
  const SideDev& SG = h->S[G];
  const int es2 = h->es;  // bytes per complex entry

  // L1: data dots | random-side dots with the draw (unless the previous
  // output pass prepared the latter)
  const bool g_ready = haar && h->pf_side == G && h->pf_t == h->t &&
                       h->pend_side != G;
  h->pf_side = h->pf_t = -1;
  DotsJob jd = no_job(), jg = no_job();
  if (kD + (haar ? 0 : kG) > 0) {
    jd.P1 = SD.U;
    jd.nc1 = kD;
    jd.P2 = haar ? nullptr : h->B[D];
    jd.nc2 = haar ? 0 : kG;
    jd.ld = SD.ld;
    jd.dim = h->dim[D];
    jd.x = x;
    jd.glo = 0;
    jd.part = h->part[D];
    jd.pstride = h->pstride;
    jd.slot1 = h->rl.w;
    jd.slot2 = h->rl.d;
    jd.nwg = h->nwg[D];
    if (h->pend_side == D) {
      jd.pk = h->pend_k;
      jd.pslot = h->rl.t;
    }
  }
  if ((haar || kG > 0) && !g_ready) {
    jg.P1 = SG.U;
    jg.nc1 = kG;
    jg.ld = SG.ld;
    jg.dim = h->dim[G];
    jg.x = nullptr;
    jg.key = key;
    jg.step = step;
    jg.glo = kG;
    if (haar) {
      jg.wcol = (char*)SG.U + (size_t)es2 * SG.ld * kG;
      jg.piv = h->scal + kScPivG;
      jg.ssq_slot = h->rl.s + 1;
    }
    jg.part = h->part[G];
    jg.pstride = h->pstride;
    jg.slot1 = h->rl.e;
    jg.nwg = h->nwg[G];
    if (h->pend_side == G) {
      jg.pk = h->pend_k;
      jg.pslot = h->rl.t;
    }
  }
  CXCHK(launch_dots(h, jd, jg));
  RedJob rd = red_job(h->part[D], (int64_t)h->nwg[D] * kWaves, h->pstride,
                      h->red);
  RedJob rg = red_job(h->part[G], (int64_t)h->nwg[G] * kWaves, h->pstride,
                      h->red);
  if (jd.nwg) {
    rd.start[0] = h->rl.w;
    rd.count[0] = 2 * kD;
    rd.start[1] = h->rl.d;
    rd.count[1] = haar ? 0 : 2 * kG;
    rd.start[2] = h->rl.t;
    rd.count[2] = jd.pk >= 0 ? 2 * jd.pk : 0;
  }
  if (jg.nwg || g_ready) {
    rg.start[0] = h->rl.e;
    rg.count[0] = 2 * kG;
    rg.start[1] = h->rl.s + 1;
    rg.count[1] = haar ? 1 : 0;
    rg.start[2] = h->rl.t;
    rg.count[2] = jg.pk >= 0 ? 2 * jg.pk : 0;
  }
  CXCHK(launch_reduce(h, rd, rg));

  SmallArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.D = SD;
  sa.G = SG;
  sa.kmax = h->kmax;
  sa.kD = kD;
  sa.kG = kG;
  sa.red = h->red;
  sa.rl = h->rl;
  sa.coef = h->coef;
  sa.cl = h->cl;
  sa.head = h->head;
  sa.scal = h->scal;
  sa.flag = h->flag;
  sa.f64 = h->f64;
  sa.pk = -1;
  if (h->pend_side >= 0) {
    sa.P = h->S[h->pend_side];
    sa.pk = h->pend_k;
  }
  if (kD > 0 || sa.pk >= 0) CXCHK(launch_small<0>(h, sa));
  h->pend_side = h->pend_k = -1;

  // L2: data pass
  CxPassArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.U = SD.U;
  pa.ld = SD.ld;
  pa.dim = h->dim[D];
  pa.k = kD;
  pa.coef = h->coef;
  pa.cl = h->cl;
  pa.del = SD.del;
  pa.x = x;
  pa.head = h->head;
  pa.piv = h->scal + kScPivD;
  pa.newcol = (char*)SD.U + (size_t)es2 * SD.ld * kD;
  pa.part = h->part[D];
  pa.pstride = h->pstride;
  pa.ssq_slot = h->rl.s + 0;
  CXCHK(launch_pass<kModeData>(h, D, pa));
  RedJob r2 = red_job(h->part[D], (int64_t)h->nwg[D] * kWaves, h->pstride,
                      h->red);
  r2.start[0] = h->rl.s + 0;
  r2.count[0] = 1;
  CXCHK(launch_reduce(h, r2, red_job(nullptr, 0, 0, nullptr)));

  // S2 and L3
  CxPassArgs po;
  std::memset(&po, 0, sizeof(po));
  po.U = SG.U;
  po.ld = SG.ld;
  po.dim = h->dim[G];
  po.coef = h->coef;
  po.cl = h->cl;
  po.y = y;
  po.comb = comb;
  po.scal = h->scal;
  if (haar) {
    CXCHK(launch_small<1>(h, sa));
    h->pend_side = D;
    h->pend_k = kD;
    po.k = kD;
    po.xmap = xmap;
    po.xnext = xnext;
    po.ma = ma;
    po.mb = mb;
    if (lookahead) {
      // the next query (Q again, so this side is its draw side) finds its
      // draw's column, pivot, norm and dots ready
      po.pf = 1;
      po.key = key;
      po.pf_step = step + 1;
      po.pf_col = (char*)SG.U + (size_t)es2 * SG.ld * (kD + 1);
      po.pf_piv = h->scal + kScPivG;
      po.part = h->part[G];
      po.pstride = h->pstride;
      po.pf_slot = h->rl.e;
      po.pf_ssq = h->rl.s + 1;
    }
    CXCHK(launch_pass<kModeHaarOut>(h, G, po));
    h->t += 1;
    h->r += 1;
    h->l += 1;
    if (lookahead) {
      h->pf_side = G;
      h->pf_t = h->t;
    }
  } else {
    CXCHK(launch_small<2>(h, sa));
    h->pend_side = D;
    h->pend_k = kD;
    po.k = kG;
    po.B = h->B[G];
    po.kb = kD;
    po.bcol = (char*)h->B[G] + (size_t)es2 * SG.ld * kD;
    po.sigma = h->sigma;
    po.key = key;
    po.step = step;
    po.glo = kG;
    CXCHK(launch_pass<kModeGinOut>(h, G, po));
    h->t += 1;
    if (D == 0)
      h->r += 1;
    else
      h->l += 1;
  }
  return HD_OK;
}

}  // namespace

extern "C" {

int hd_cinit(int32_t ensemble, int32_t storage, int64_t m, int64_t n,
             int32_t t_max, uint32_t seed, uint32_t trial, double sigma,
             void* stream, hd_chandle* out) {
  if (!out) return HD_ERR_INVALID;
  *out = nullptr;
  if (ensemble != HD_GINIBRE && ensemble != HD_HAAR) return HD_ERR_INVALID;
  if (storage != HD_F32 && storage != HD_F64) return HD_ERR_INVALID;
  if (m < 1 || n < 1 || t_max < 1 || t_max > kMaxT) return HD_ERR_INVALID;
  if (ensemble == HD_HAAR && (m != n || t_max > n)) return HD_ERR_INVALID;
  if (ensemble == HD_GINIBRE && !(sigma > 0.0 && std::isfinite(sigma)))
    return HD_ERR_INVALID;
  if (n > ((int64_t)1 << 40) || m > ((int64_t)1 << 40)) return HD_ERR_INVALID;
  hd_cctx* h = new (std::nothrow) hd_cctx();
  if (!h) return HD_ERR_NOMEM;
  h->ens = ensemble;
  h->f64 = storage == HD_F64;
  h->es = h->f64 ? 16 : 8;
  h->m = m;
  h->n = n;
  h->tmax = t_max;
  h->kmax = t_max + 1;
  h->seed = seed;
  h->trial = trial;
  h->sigma = ensemble == HD_HAAR ? 1.0 : sigma;
  h->stream = (hipStream_t)stream;
  h->dim[0] = n;
  h->dim[1] = m;
  h->rl = red_lay(h->kmax);
  h->cl = coef_lay(h->kmax);
  h->pstride = h->rl.end;
  const int kmax = h->kmax;
  int rc = HD_OK;
  auto fail = [&](int r) {
    cx_release(h);
    delete h;
    return r;
  };
#define CXA(ptr, bytes)                    \
  do {                                     \
    rc = cx_alloc(h, &(ptr), (bytes));     \
    if (rc != HD_OK) return fail(rc);      \
  } while (0)
  for (int s = 0; s < 2; ++s) {
    SideDev& S = h->S[s];
    S.ld = (h->dim[s] + kRowsWG - 1) / kRowsWG * kRowsWG;
    h->nwg[s] = (int)(S.ld / kRowsWG);
    const size_t pb = (size_t)h->es * S.ld * kmax;
    if ((double)pb > 1.2e11) return fail(HD_ERR_NOMEM);
    CXA(S.U, pb);
    h->B[s] = nullptr;
    if (ensemble == HD_GINIBRE) CXA(h->B[s], pb);
    CXA(S.T, sizeof(double) * 2 * (size_t)kmax * kmax);
    CXA(S.ref, sizeof(double) * kRefStride * (size_t)kmax);
    CXA(S.del, sizeof(double) * 2 * (size_t)kmax);
    CXA(h->part[s], sizeof(double) * (size_t)h->pstride * h->nwg[s] * kWaves);
  }
  {
    // first-stage partials: at most (rows / kRedRows) blocks x pstride slots
    int64_t rows = 0;
    for (int s = 0; s < 2; ++s)
      rows = std::max(rows, (int64_t)h->nwg[s] * kWaves);
    const size_t sb = sizeof(double) * (size_t)h->pstride *
                      (size_t)((rows + kRedRows - 1) / kRedRows);
    CXA(h->stage[0], sb);
    CXA(h->stage[1], sb);
  }
  CXA(h->red, sizeof(double) * (size_t)h->rl.end);
  CXA(h->coef, sizeof(double) * (size_t)h->cl.end);
  CXA(h->head, sizeof(double) * 2 * (size_t)(kmax + 1));
  CXA(h->scal, sizeof(double) * kScCount);
  CXA(h->flag, sizeof(int) * 4);
  h->ybuf = nullptr;
  h->pend_side = h->pend_k = -1;
  h->pf_side = h->pf_t = -1;
#undef CXA
  rc = cx_zero_state(h);
  if (rc != HD_OK) return fail(rc);
  if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(HD_ERR_HIP);
  *out = h;
  return HD_OK;
}

int hd_cstep(hd_chandle h, int32_t adjoint, const void* x, void* y) {
  if (!h || !x || !y || x == y) return HD_ERR_INVALID;
  const int adj = adjoint != 0;
  if (h->t + 1 > h->tmax) return HD_ERR_CAPACITY;
  if (h->ens == HD_GINIBRE) {
    if (!adj && h->r + 1 > h->n) return HD_ERR_CAPACITY;
    if (adj && h->l + 1 > h->m) return HD_ERR_CAPACITY;
  }
  return cx_query(h, adj, x, y, nullptr, nullptr, nullptr, 0.0, 0.0);
}

int hd_crun(hd_chandle h, int32_t T, double a, double b, void* X, void* Y) {
  if (!h || !X || T < 0) return HD_ERR_INVALID;
  if (h->ens != HD_HAAR) return HD_ERR_UNSUPPORTED;
  if (h->t + T > h->tmax) return HD_ERR_CAPACITY;
  const size_t row = (size_t)h->es * h->n;
  for (int t = 0; t < T; ++t) {
    const char* xt = (const char*)X + row * t;
    char* xn = (char*)X + row * (t + 1);
    void* yt = Y ? (void*)((char*)Y + row * t) : nullptr;
    // every query but the last prepares the next one's draw
    CXCHK(cx_query(h, 0, xt, yt, nullptr, xt, xn, a, b, t + 1 < T));
  }
  return HD_OK;
}

int hd_cgue_step(hd_chandle h, const void* x, void* y) {
  if (!h || !x || !y || x == y) return HD_ERR_INVALID;
  if (h->ens != HD_GINIBRE || h->m != h->n) return HD_ERR_INVALID;
  if (h->t + 2 > h->tmax || h->r + 1 > h->n || h->l + 1 > h->m)
    return HD_ERR_CAPACITY;
  if (!h->ybuf) {
    if (cx_alloc(h, &h->ybuf, (size_t)h->es * h->n) != HD_OK)
      return HD_ERR_NOMEM;
  }
  CXCHK(cx_query(h, 0, x, h->ybuf, nullptr, nullptr, nullptr, 0.0, 0.0));
  return cx_query(h, 1, x, y, h->ybuf, nullptr, nullptr, 0.0, 0.0);
}

int hd_creset(hd_chandle h, uint32_t seed, uint32_t trial) {
  if (!h) return HD_ERR_INVALID;
  h->seed = seed;
  h->trial = trial;
  h->t = h->r = h->l = 0;
  h->pend_side = h->pend_k = -1;
  h->pf_side = h->pf_t = -1;
  return cx_zero_state(h);
}

int hd_ccounts(hd_chandle h, int32_t* t, int32_t* r, int32_t* l) {
  if (!h || !t || !r || !l) return HD_ERR_INVALID;
  *t = h->t;
  *r = h->r;
  *l = h->l;
  return HD_OK;
}

int hd_cstatus(hd_chandle h) {
  if (!h) return HD_ERR_INVALID;
  CXHIP(hipStreamSynchronize(h->stream));
  int flag = 0;
  CXHIP(hipMemcpy(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost));
  return flag ? HD_ERR_NONFINITE : HD_OK;
}

int hd_cset_stream(hd_chandle h, void* stream) {
  if (!h) return HD_ERR_INVALID;
  h->stream = (hipStream_t)stream;
  return HD_OK;
}

int hd_cprofile(hd_chandle h, int32_t enable) {
  if (!h) return HD_ERR_INVALID;
  CXHIP(hipStreamSynchronize(h->stream));
  h->prof = enable ? 1 : 0;
  if (enable) {
    h->recs.clear();
    h->pool_used = 0;
  }
  return HD_OK;
}

int hd_cprofile_read(hd_chandle h, int32_t kind, double* ms,
                     int64_t* launches, double* bytes) {
  if (!h) return HD_ERR_INVALID;
  CXHIP(hipStreamSynchronize(h->stream));
  double tot = 0.0, by = 0.0;
  int64_t cnt = 0;
  for (const hd_cctx::Rec& r : h->recs) {
    if (r.kind != kind) continue;
    float e = 0.f;
    CXHIP(hipEventElapsedTime(&e, r.a, r.b));
    tot += e;
    by += r.bytes;
    ++cnt;
  }
  if (ms) *ms = tot;
  if (launches) *launches = cnt;
  if (bytes) *bytes = by;
  return HD_OK;
}

int hd_cfree(hd_chandle h) {
  if (!h) return HD_OK;
  cx_release(h);
  delete h;
  return HD_OK;
}

}  // extern "C"
