// HIP kernels (gfx950) for the Householder Dice step.
//
// A panel is the column-major array V (ld x t_max) of the stored reflector
// vectors u_j = p[j:] + s_j ||p[j:]|| e_j (Sec. 3.1, eq. (Householder)), one
// column per reflector, zero above the diagonal.  The product of the
// reflectors is kept in compact-WY form with a diagonal sign prefix:
//   R_k..R_1 = Delta_k (I - V T' V'),   R_1..R_k = (I - V T V') Delta_k,
// Delta_k = diag(pi[min(i+1,k)]), pi[j] = prod_{l<j} (-s_l)
// (the -sign(v1) factor of eq. (Householder) commutes with every later
// reflector, so all of them collect into Delta).
//
// Every panel kernel is one streaming sweep over its rows, with all
// accumulation in FP64.  A lane holds four consecutive rows (one 16-byte load
// per FP32 column, two per FP64 column), a chunk is the 256 rows of one
// wave's 64 lanes, and a workgroup covers CPT chunks; its four waves split
// the columns (wave w takes columns w, w + 4, w + 8, ...), so every wave has
// a full chunk of rows in flight per column even when the panel is short
// (the TDOT of four-chunk workgroups splits the rows instead; see rs_sweep).
//   tdot     : w = V' b (column dots), optionally a second right-hand side
//   pass     : out = Delta a - V z (GEMV-N), the new panel column, the dots of
//              every column with the next query's Philox draw (prefetch) and,
//              when asked, of the earlier columns with the new one
//   gin_pass : the random side of a Ginibre query (two GEMV-N plus the
//              explicit basis panel)
// Column dots are summed per wave with a reduce-scatter on permlane swaps
// and DPP moves, across workgroups by k_reduce in fixed order, so results
// are bitwise reproducible run to run.  GEMV-N rows are summed over the four
// waves through LDS in fixed order.  Small one-workgroup FP64 kernels update
// the WY factor T and the reflector scalars.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "hd_device.hpp"
#include "hd_internal.hpp"

namespace hd {

constexpr int kLaneRows = 4;                  // consecutive rows per lane
constexpr int kChunkRows = 64 * kLaneRows;    // rows of one wave (256)
// Columns per group of a wave's sweep.  Each lane keeps one partial sum per
// column of the group in registers and the compiler issues all CG * CPT
// loads of a group together, so groups narrow as chunks are added (wider
// groups spill to scratch).
template <int CPT, int ND, int NZ>
constexpr int col_group() {
  return (ND <= 1 && NZ == 0) ? 16 : 8 / CPT;
}

// Draws g_step[i] for the four rows i0..i0+3 of one lane; rows outside
// (lo, n) get 0.  Values are rounded to the storage type when `round`.
template <typename T>
__device__ __forceinline__ void draw_rows(PhiloxKey key, uint32_t step,
                                          int64_t i0, int64_t lo, int64_t n,
                                          bool round, double (&out)[4]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) out[e] = 0.0;
  if (i0 >= n || i0 + 3 <= lo) return;
  double g[4];
  normals4(key, step, 0u, (uint64_t)(i0 >> 2), g);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t i = i0 + e;
    if (i > lo && i < n) out[e] = round ? (double)(T)g[e] : g[e];
  }
}

// The draw of `step` for the CPT * 256 rows of a workgroup into LDS
// (g[q] for row blk0 + q), computed once per workgroup: one Philox block of
// four normals per thread.  The caller synchronises before reading.
template <typename T, int CPT>
__device__ __forceinline__ void draw_block(PhiloxKey key, uint32_t step,
                                           int64_t blk0, int64_t lo, int64_t n,
                                           bool round, double* g) {
  for (int q = threadIdx.x; q < CPT * 64; q += kWG) {
    double v[4];
    draw_rows<T>(key, step, blk0 + 4 * (int64_t)q, lo, n, round, v);
#pragma unroll
    for (int e = 0; e < 4; ++e) g[4 * q + e] = v[e];
  }
}

// The lane's four rows of chunk c from a workgroup vector in LDS.
template <int CPT>
__device__ __forceinline__ void lane_rows(const double* g,
                                          double (&out)[CPT][4]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e) out[c][e] = g[c * kChunkRows + 4 * lane + e];
}

// Sum over the four waves (fixed order) of the lane-layout partial rows acc:
// afterwards thread t holds in out[c] the total for row c * 256 + t of the
// workgroup.  `lds` holds kWaves * CPT * 256 doubles.  Two barriers.
template <int CPT>
__device__ __forceinline__ void combine_rows(const double (&acc)[CPT][4],
                                             double* lds, double (&out)[CPT]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      lds[(wave * CPT + c) * kChunkRows + 4 * lane + e] = acc[c][e];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += lds[(w * CPT + c) * kChunkRows + tid];
    out[c] = s;
  }
  __syncthreads();
}

// One sweep of this wave's columns (j = wave + 4 q < nc) of a panel over the
// workgroup's rows (CPT chunks from blk0):
//   dots (ND = 1 or 2, when `dots`): sum_rows V[r, j] * rhs0[r] -> out0[j],
//        and likewise rhs1 -> out1 (per-workgroup partials);
//   GEMV-N (NZ = 0, 1 or 2): acc_q[r] -= zs_q * sum_j V[r, j] * z_q[j] over
//        this wave's columns (rows are summed over waves afterwards).
// Every panel row of the workgroup is allocated (ld is a multiple of the
// workgroup's rows); rows at or beyond n are zero.  NT: non-temporal panel
// loads (used for multi-chunk workgroups -- panels far beyond the caches --
// when no second sweep re-reads the rows).
template <typename T, int CPT, int ND, int NZ, bool NT = false, bool DB = false>
__device__ __forceinline__ void sweep(
    const T* __restrict__ V, int64_t ld, int nc, int64_t blk0,
    const double (&rhs0)[CPT][4], const double (&rhs1)[CPT][4], bool dots,
    const double* __restrict__ z0, double zs0, const double* __restrict__ z1,
    double zs1, double (&acc0)[CPT][4], double (&acc1)[CPT][4], double* out0,
    double* out1) {
  constexpr int kCG = col_group<CPT, ND, NZ>();
  constexpr int kGroup = 64 / kCG;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ncw = nc > wave ? (nc - wave + kWaves - 1) / kWaves : 0;
  const T* __restrict__ Vl = V + blk0 + 4 * lane;
  if constexpr (DB && sizeof(T) == 4) {
    // DB: the raw entries of the next column group are loaded before the
    // current group's arithmetic, so two groups of loads are in flight (for
    // workgroups alone on their CU, where nothing else hides the latency)
    hd_f4 cur[CPT][kCG], nxt[CPT][kCG];
    auto load = [&](int g0, hd_f4 (&buf)[CPT][kCG]) {
#pragma unroll
      for (int c = 0; c < CPT; ++c)
#pragma unroll
        for (int jj = 0; jj < kCG; ++jj) {
          const int j = wave + kWaves * min(g0 + jj, ncw - 1);
          const hd_f4* p = (const hd_f4*)(Vl + (int64_t)j * ld + c * kChunkRows);
          if constexpr (NT)
            buf[c][jj] = __builtin_nontemporal_load(p);
          else
            buf[c][jj] = *p;
        }
    };
    if (ncw > 0) load(0, cur);
#pragma unroll 1
    for (int g0 = 0; g0 < ncw; g0 += kCG) {
      if (g0 + kCG < ncw) load(g0 + kCG, nxt);
      double p0[kCG], p1[ND == 2 ? kCG : 1];
      double q0[NZ >= 1 ? kCG : 1], q1[NZ == 2 ? kCG : 1];
#pragma unroll
      for (int jj = 0; jj < kCG; ++jj) {
        const bool ok = g0 + jj < ncw;
        const int j = wave + kWaves * (g0 + jj);
        p0[jj] = 0.0;
        if constexpr (ND == 2) p1[jj] = 0.0;
        if constexpr (NZ >= 1) q0[jj] = ok ? zs0 * z0[j] : 0.0;
        if constexpr (NZ == 2) q1[jj] = ok ? zs1 * z1[j] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
#pragma unroll
        for (int jj = 0; jj < kCG; ++jj) {
          double v[4] = {cur[c][jj].x, cur[c][jj].y, cur[c][jj].z, cur[c][jj].w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if constexpr (NZ >= 1) acc0[c][e] -= v[e] * q0[jj];
            if constexpr (NZ == 2) acc1[c][e] -= v[e] * q1[jj];
            if constexpr (ND >= 1) p0[jj] += v[e] * rhs0[c][e];
            if constexpr (ND == 2) p1[jj] += v[e] * rhs1[c][e];
          }
        }
      }
      if constexpr (ND >= 1) {
        if (dots) {
          const int q = g0 + lane / kGroup;
          const bool owner = (lane % kGroup) == 0 && q < ncw;
          const double s0 = wave_reduce_scatter<kCG>(p0);
          if (owner) out0[wave + kWaves * q] = s0;
          if constexpr (ND == 2) {
            const double s1 = wave_reduce_scatter<kCG>(p1);
            if (owner) out1[wave + kWaves * q] = s1;
          }
        }
      }
      if (g0 + kCG < ncw) {
#pragma unroll
        for (int c = 0; c < CPT; ++c)
#pragma unroll
          for (int jj = 0; jj < kCG; ++jj) cur[c][jj] = nxt[c][jj];
      }
    }
    return;
  }
#pragma unroll 1
  for (int g0 = 0; g0 < ncw; g0 += kCG) {
    double p0[kCG], p1[ND == 2 ? kCG : 1];
    double q0[NZ >= 1 ? kCG : 1], q1[NZ == 2 ? kCG : 1];
#pragma unroll
    for (int jj = 0; jj < kCG; ++jj) {
      const bool ok = g0 + jj < ncw;
      const int j = wave + kWaves * (g0 + jj);
      p0[jj] = 0.0;
      if constexpr (ND == 2) p1[jj] = 0.0;
      if constexpr (NZ >= 1) q0[jj] = ok ? zs0 * z0[j] : 0.0;
      if constexpr (NZ == 2) q1[jj] = ok ? zs1 * z1[j] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
#pragma unroll
      for (int jj = 0; jj < kCG; ++jj) {
        const int j = wave + kWaves * min(g0 + jj, ncw - 1);
        double v[4];
        load4<NT>(Vl + (int64_t)j * ld + c * kChunkRows, v);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if constexpr (NZ >= 1) acc0[c][e] -= v[e] * q0[jj];
          if constexpr (NZ == 2) acc1[c][e] -= v[e] * q1[jj];
          if constexpr (ND >= 1) p0[jj] += v[e] * rhs0[c][e];
          if constexpr (ND == 2) p1[jj] += v[e] * rhs1[c][e];
        }
      }
    }
    if constexpr (ND >= 1) {
      if (dots) {
        const int q = g0 + lane / kGroup;
        const bool owner = (lane % kGroup) == 0 && q < ncw;
        const double s0 = wave_reduce_scatter<kCG>(p0);
        if (owner) out0[wave + kWaves * q] = s0;
        if constexpr (ND == 2) {
          const double s1 = wave_reduce_scatter<kCG>(p1);
          if (owner) out1[wave + kWaves * q] = s1;
        }
      }
    }
  }
}

// ------------------------------------------ row-split four-chunk sweeps --
//
// The TDOT of a four-chunk workgroup splits the rows over the waves instead
// of the columns: wave w owns chunk w (rows blk0 + 256 w + 4 lane + e) and
// sweeps every column of the panel over it.  The right-hand sides and draws
// of a lane are its own four rows (registers, no LDS copy: 104 VGPRs and four
// waves per SIMD for two right-hand sides, against 146 and three in the
// column split), and the column dots are added over the four waves through
// LDS, a block of kRsBlk columns at a time (fixed order).  The GEMV-N passes
// keep the column split: the row-split form of them (no LDS row sums, 124
// VGPRs) measured no faster at n = 1e7.

constexpr int kRsCG = 8;     // columns per group of a wave's sweep
constexpr int kRsBlk = 256;  // columns per block of the cross-wave dot sums

// Sweep of columns [0, nc) over the lane's four rows starting at row0 (ND
// dot streams with r0 / r1 into out0 / out1, GEMV-N acc -= V z when NZ).
// Every thread of the workgroup calls it with the same nc (it contains
// barriers when ND > 0).  dl holds ND * kWaves * kRsBlk doubles.
template <typename T, int ND, int NZ, bool NT>
__device__ __forceinline__ void rs_sweep(
    const T* __restrict__ V, int64_t ld, int nc, int64_t row0,
    const double (&r0)[4], const double (&r1)[4],
    const double* __restrict__ z, double (&acc)[4], double* dl,
    double* out0, double* out1) {
  constexpr int kGroup = 64 / kRsCG;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const T* __restrict__ Vl = V + row0;
#pragma unroll 1
  for (int jb = 0; jb < nc; jb += kRsBlk) {
    const int je = min(nc, jb + kRsBlk);
#pragma unroll 1
    for (int g0 = jb; g0 < je; g0 += kRsCG) {
      double p0[kRsCG], p1[ND == 2 ? kRsCG : 1], q[NZ ? kRsCG : 1];
      double v[kRsCG][4];
#pragma unroll
      for (int jj = 0; jj < kRsCG; ++jj) {
        const int j = min(g0 + jj, je - 1);
        load4<NT>(Vl + (int64_t)j * ld, v[jj]);
        if constexpr (NZ) q[jj] = g0 + jj < je ? z[g0 + jj] : 0.0;
      }
#pragma unroll
      for (int jj = 0; jj < kRsCG; ++jj) {
        p0[jj] = 0.0;
        if constexpr (ND == 2) p1[jj] = 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if constexpr (NZ) acc[e] -= v[jj][e] * q[jj];
          if constexpr (ND >= 1) p0[jj] += v[jj][e] * r0[e];
          if constexpr (ND == 2) p1[jj] += v[jj][e] * r1[e];
        }
      }
      if constexpr (ND >= 1) {
        const int jl = g0 - jb + lane / kGroup;
        const bool owner = (lane % kGroup) == 0 && g0 + lane / kGroup < je;
        const double s0 = wave_reduce_scatter<kRsCG>(p0);
        if (owner) dl[wave * kRsBlk + jl] = s0;
        if constexpr (ND == 2) {
          const double s1 = wave_reduce_scatter<kRsCG>(p1);
          if (owner) dl[(kWaves + wave) * kRsBlk + jl] = s1;
        }
      }
    }
    if constexpr (ND >= 1) {
      __syncthreads();
      const int t = threadIdx.x;
      if (t < je - jb) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
          s0 += dl[w * kRsBlk + t];
          if constexpr (ND == 2) s1 += dl[(kWaves + w) * kRsBlk + t];
        }
        out0[jb + t] = s0;
        if constexpr (ND == 2) out1[jb + t] = s1;
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------- small FP64 steps ------
//
// The small steps are O(k^2) sums over the T factors and the head rows of the
// panels.  One thread per output with a serial loop would issue its loads one
// small batch at a time; instead P = 256 / nout threads share each output,
// each summing a strided subset of the terms (so every thread has only a few
// independent loads, all issued at once), and the P partial sums are added
// through LDS in fixed order.

// out(j, s_j) for j < nout with s_j = sum over i in [lo(j), hi(j)) of
// term(i, j); with two terms (NT = 2) both sums share the loop.  Every thread
// of the workgroup calls it; `lds` holds 2 * kWG doubles.  Ends with a
// barrier.
template <int NT, typename Lo, typename Hi, typename Term, typename Out>
__device__ __forceinline__ void wg_sums(int nout, Lo lo, Hi hi, Term term,
                                        Out out, double* lds) {
  if (nout <= 0) return;
  const int tid = threadIdx.x;
  const int P = nout >= kWG ? 1 : kWG / nout;  // threads per output
  const int per = kWG / P;                     // outputs per round
  for (int base = 0; base < nout; base += per) {
    const int j = base + tid / P, ph = tid % P;
    double s0 = 0.0, s1 = 0.0;
    if (tid / P < per && j < nout) {
      const int h = hi(j);
#pragma unroll 8
      for (int i = lo(j) + ph; i < h; i += P) {
        double t0, t1;
        term(i, j, t0, t1);
        s0 += t0;
        if (NT == 2) s1 += t1;
      }
    }
    lds[tid] = s0;
    if (NT == 2) lds[kWG + tid] = s1;
    __syncthreads();
    if (ph == 0 && tid / P < per && j < nout) {
      double r0 = 0.0, r1 = 0.0;
      for (int q = 0; q < P; ++q) {
        r0 += lds[tid + q];
        if (NT == 2) r1 += lds[kWG + tid + q];
      }
      out(j, r0, r1);
    }
    __syncthreads();
  }
}

// out(j, s_j) for j < nout with s_j = sum over i in [lo(j), hi(j)) of
// term(i, j), where term reads column j of a column-major matrix (a panel
// head or T), lo and hi never decrease with j, and lo(j) < hi(j).  Each wave
// takes kColGroup consecutive outputs at a time and its lanes the rows, 64
// at a time, so that a load reads consecutive entries of one column (one
// thread per output would read its column alone, every lane of a load in
// another column: a cache line, and for the panels a page, per lane); the
// loads of a group are all issued before any is added, at indexes clamped
// into the column, and a butterfly over the wave adds the lanes' terms.
// Every thread of the workgroup calls it; ends with a barrier.
constexpr int kColGroup = 8;
template <typename Lo, typename Hi, typename Term, typename Out>
__device__ __forceinline__ void col_sums(int nout, Lo lo, Hi hi, Term term,
                                         Out out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int jb = wave * kColGroup; jb < nout; jb += kWaves * kColGroup) {
    const int jl = min(jb + kColGroup, nout) - 1;
    const int r1 = hi(jl);
    double s[kColGroup];
#pragma unroll
    for (int c = 0; c < kColGroup; ++c) s[c] = 0.0;
    for (int r = lo(jb); r < r1; r += 64) {
      const int i = r + lane;
      double v[kColGroup];
#pragma unroll
      for (int c = 0; c < kColGroup; ++c) {
        const int j = min(jb + c, jl);
        v[c] = term(min(max(i, lo(j)), hi(j) - 1), j);
      }
#pragma unroll
      for (int c = 0; c < kColGroup; ++c) {
        const int j = jb + c;
        if (j <= jl && i >= lo(j) && i < hi(j)) s[c] += v[c];
      }
    }
    // every lane holds every sum after the butterfly: lane c writes output
    // jb + c, so that the loads out() may make are issued together
    double mine = 0.0;
#pragma unroll
    for (int c = 0; c < kColGroup; ++c) {
      const double t = wave_sum(s[c]);
      if (lane == c) mine = t;
    }
    if (lane < kColGroup && jb + lane <= jl) out(jb + lane, mine);
  }
  __syncthreads();
}

// The column sums of a small step: by col_sums where they read the panel
// head in a single-trial kernel (one workgroup, latency-bound, COLS), by
// wg_sums in the batched ones, where thousands of workgroups run side by
// side and the butterflies' arithmetic costs more than it hides, and for
// z = T'w, whose T factor is small and stays cached.
template <bool COLS, typename Lo, typename Hi, typename Term, typename Out>
__device__ __forceinline__ void head_sums(int nout, Lo lo, Hi hi, Term term,
                                          Out out, double* lds) {
  if constexpr (COLS) {
    col_sums(nout, lo, hi, term, out);
  } else {
    wg_sums<1>(
        nout, lo, hi,
        [=](int i, int j, double& t0, double& t1) {
          t0 = term(i, j);
          t1 = 0.0;
        },
        [=](int j, double v, double) { out(j, v); }, lds);
  }
}

// out(j, s0_j, s1_j) for j < n with s_r,j = sum over l in [j, n) of
// T[j, l] coef_r(l) (coef_1 only when NT = 2): the row sums of the leading
// n x n block of an upper-triangular factor T (column-major, leading
// dimension tm) against one or two coefficient vectors.  The lanes take the
// rows and the waves the columns in turn, so every load reads consecutive
// entries of one column (reading T by rows would touch one cache line per
// entry).  With GRP (the single-trial kernels, latency-bound) kTriGroup
// columns are loaded before any is added, at indexes clamped into the
// triangle: a load behind the j <= l branch would wait out its own round
// trip before the next one is issued.  The batched kernels, thousands of
// workgroups side by side, keep the plain loop, whose skipped entries cost
// nothing there and whose latency the other workgroups hide.  Per block of 64 rows
// the waves' partial sums are added in fixed order through LDS.  Every
// thread of the workgroup calls it; `lds` holds 2 * kWG doubles.  Ends with
// a barrier.
constexpr int kTriGroup = 8;
template <int NT, bool GRP, typename C0, typename C1, typename Out>
__device__ __forceinline__ void tri_row_sums(const double* __restrict__ T,
                                             int tm, int n, C0 coef0,
                                             C1 coef1, Out out, double* lds) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int r0 = 0; r0 < n; r0 += 64) {
    const int j = r0 + lane;
    double s0 = 0.0, s1 = 0.0;
    if constexpr (!GRP) {
#pragma unroll 16
      for (int l = r0 + wave; l < n; l += kWaves) {
        if (j <= l) {
          const double t = T[j + (int64_t)l * tm];
          s0 += t * coef0(l);
          if (NT == 2) s1 += t * coef1(l);
        }
      }
    } else {
      for (int l0 = r0 + wave; l0 < n; l0 += kWaves * kTriGroup) {
        double t[kTriGroup], c0[kTriGroup], c1[kTriGroup];
#pragma unroll
        for (int u = 0; u < kTriGroup; ++u) {
          const int l = min(l0 + u * kWaves, n - 1);
          t[u] = T[min(j, l) + (int64_t)l * tm];
          c0[u] = coef0(l);
          c1[u] = NT == 2 ? coef1(l) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kTriGroup; ++u) {
          const int l = l0 + u * kWaves;
          if (l < n && j <= l) {
            s0 += t[u] * c0[u];
            if (NT == 2) s1 += t[u] * c1[u];
          }
        }
      }
    }
    lds[tid] = s0;
    if (NT == 2) lds[kWG + tid] = s1;
    __syncthreads();
    if (wave == 0 && j < n) {
      double a0 = 0.0, a1 = 0.0;
      for (int w = 0; w < kWaves; ++w) {
        a0 += lds[w * 64 + lane];
        if (NT == 2) a1 += lds[kWG + w * 64 + lane];
      }
      out(j, a0, a1);
    }
    __syncthreads();
  }
}

// Column kp of T from the dots c = V[:, :kp]' u_kp (compact-WY recurrence of
// Schreiber and Van Loan), then z = T' w for the leading k x k block.
template <bool COLS = false, bool GRP = false>
__device__ void small_data_body(const SmallDataArgs& a) {
  __shared__ double lds[2 * kWG];
  const int tm = a.tmax, kp = a.kp;
  const double* __restrict__ Tm = a.T;
  if (kp > 0) {
    const double tau = a.tau[kp];
    const double* c = a.c;
    double* Tw = a.T;
    tri_row_sums<1, GRP>(
        Tm, tm, kp, [=](int l) { return c[l]; }, [](int) { return 0.0; },
        [=](int j, double r0, double) { Tw[j + (int64_t)kp * tm] = -tau * r0; },
        lds);
  }
  if (a.w) {
    const double* w = a.w;
    double* z = a.z;
    head_sums<COLS>(
        a.k, [](int) { return 0; }, [](int j) { return j + 1; },
        [=](int i, int j) { return Tm[i + (int64_t)j * tm] * w[i]; },
        [=](int j, double r0) { z[j] = r0; }, lds);
  }
}

// Data-side reflector of a query from p (pivot p_k, ss = ||p[k+1:]||^2 of the
// stored entries): nu = ||p[k:]||, s = sign(p_k), stored pivot u_k = p_k + s nu
// rounded to storage, tau = 2/||u||^2 from the stored entries.  nu = 0 gives
// the identity (tau = 0, no sign).  Written by one thread; returns nu.
template <typename T>
__device__ double data_reflector(const PanelDev& D, int k, int tm, double ss,
                                 double pk, int* flag, double* up_out,
                                 double* tau_out) {
  T* V = (T*)D.V;
  const double nu = sqrt(ss + pk * pk);
  double s = 1.0, tau = 0.0, up = 0.0;
  if (nu > 0.0) {
    s = pk >= 0.0 ? 1.0 : -1.0;
    up = (double)(T)(pk + s * nu);
    tau = 2.0 / (ss + up * up);
  }
  if (!isfinite(nu) || !isfinite(tau)) flag[0] = 1;
  V[(int64_t)k * D.ld + k] = (T)up;
  D.tau[k] = tau;
  D.nu[k] = nu;
  D.piv[k] = pk;
  D.sgn[k] = s;
  D.pi[k + 1] = nu > 0.0 ? D.pi[k] * (-s) : D.pi[k];
  D.T[k + (int64_t)k * tm] = tau;
  *up_out = up;
  *tau_out = tau;
  return nu;
}

// Column k of the data side's T factor from the dots c_j (j < k) of its
// columns with the stored rows > k of u_k, summed by the data pass, plus the
// pivot row (V[k, j] * u_k[k]): T[:k, k] = -tau_k T[:k, :k] c.  Every thread
// of the workgroup calls it.
template <typename T, bool GRP = false>
__device__ void data_tcol(const PanelDev& D, int k, int tm, double up,
                          double tau, const double* c, double* lds) {
  const T* __restrict__ V = (const T*)D.V;
  const double* __restrict__ Tm = D.T;
  double* Tw = D.T;
  const int64_t ld = D.ld;
  tri_row_sums<1, GRP>(
      Tm, tm, k,
      [=](int l) { return c[l] + (double)V[(int64_t)l * ld + k] * up; },
      [](int) { return 0.0; },
      [=](int j, double r0, double) { Tw[j + (int64_t)k * tm] = -tau * r0; },
      lds);
}

// Haar, after the data-side pass of query t (k = t-1 reflectors per panel):
// the data reflector R_t, then L_t = H_t(g_t) from the prefetched dots V'g
// over rows > k and ||g[k+1:]||^2, its T column, s_vec = V' Delta w for
// w = [p[:k]; (nu/||g[k:]||) g[k:]] (the vector L_t R_t p_t of eq. (Qtxt)
// before L_1..L_{t-1}), and z_G = T_G s_vec.
template <typename T, bool COLS = false>
__device__ void haar_small_body(const HaarSmallArgs& a) {
  __shared__ double sh[6];
  __shared__ double lds[2 * kWG];
  const int k = a.k, tid = threadIdx.x, tm = a.tmax;
  T* VG = (T*)a.G.V;
  const int64_t ldG = a.G.ld;
  double* cG = a.zG + tm;
  double* sv = a.zG + 2 * tm;
  if (tid == 0) {
    const double nu = data_reflector<T>(a.D, k, tm,
                                        a.D.red[a.extra + kSlotSS], *a.pivot,
                                        a.flag, &sh[4], &sh[5]);
    const PhiloxKey key{a.key.k0, a.key.k1};
    const double gk = normal_at(key, a.step, 0u, (uint64_t)k);
    const double ssG = a.G.red[a.extra + kSlotPFSS];
    const double nuG = sqrt(ssG + gk * gk);
    double sG = 1.0, tauG = 0.0, upG = 0.0;
    if (nuG > 0.0) {
      sG = gk >= 0.0 ? 1.0 : -1.0;
      upG = (double)(T)(gk + sG * nuG);
      tauG = 2.0 / (ssG + upG * upG);
    }
    if (!isfinite(nuG) || !isfinite(tauG)) a.flag[0] = 1;
    VG[(int64_t)k * ldG + k] = (T)upG;
    a.G.tau[k] = tauG;
    a.G.nu[k] = nuG;
    a.G.piv[k] = gk;
    a.G.sgn[k] = sG;
    a.G.pi[k + 1] = nuG > 0.0 ? a.G.pi[k] * (-sG) : a.G.pi[k];
    a.G.T[k + (int64_t)k * tm] = tauG;
    const double cs = nuG > 0.0 ? nu / nuG : 0.0;
    *a.cscale = cs;
    sh[0] = tauG;
    sh[1] = cs;
    sh[2] = gk;
    sh[3] = upG;
  }
  __syncthreads();
  const double tauG = sh[0], cs = sh[1], gk = sh[2], upG = sh[3];
  const double piGk = a.G.pi[k];
  const T* __restrict__ VGr = VG;
  const double* __restrict__ piG = a.G.pi;
  const double* __restrict__ head = a.head;
  const double* __restrict__ gdot = a.G.red;
  // hg_j = sum_{j <= i < k} V_G[i, j] pi_{i+1} head_i; then the dots of the
  // new random reflector (cG) and s_vec (sv)
  head_sums<COLS>(
      k, [](int j) { return j; }, [k](int) { return k; },
      [=](int i, int j) {
        return (double)VGr[(int64_t)j * ldG + i] * piG[i + 1] * head[i];
      },
      [=](int j, double hg) {
        const double vk = (double)VGr[(int64_t)j * ldG + k];
        cG[j] = gdot[j] + vk * upG;
        sv[j] = hg + piGk * cs * (gdot[j] + vk * gk);
      },
      lds);
  const double* __restrict__ TG = a.G.T;
  double* TGw = a.G.T;
  double* zG = a.zG;
  tri_row_sums<2, COLS>(
      TG, tm, k, [=](int l) { return sv[l]; }, [=](int l) { return cG[l]; },
      [=](int j, double zz, double tg) {
        zG[j] = zz;
        TGw[j + (int64_t)k * tm] = -tauG * tg;
      },
      lds);
  if (a.cslot >= 0)
    data_tcol<T, COLS>(a.D, k, tm, sh[4], sh[5], a.D.red + a.cslot, lds);
}

// Ginibre: the data reflector, then the random-side coefficients
// s1 = V_G' Delta_G [0; g] = pi_l (prefetched dots over rows >= l),
// s2 = V_G' Delta_G h (head rows only) + nu s1; z1 = T_G s1, z2 = T_G s2.
template <typename T, bool COLS = false>
__device__ void gin_small_body(const GinSmallArgs& a) {
  __shared__ double sh[3];
  __shared__ double lds[2 * kWG];
  const int k = a.k, l = a.l, tid = threadIdx.x, tm = a.tmax;
  const T* __restrict__ VG = (const T*)a.G.V;
  const int64_t ldG = a.G.ld;
  double* s1 = a.z1 + tm;
  double* s2 = a.z1 + 2 * tm;
  if (tid == 0) {
    const double nu = data_reflector<T>(a.D, k, tm,
                                        a.D.red[a.D_extra + kSlotSS], *a.pivot,
                                        a.flag, &sh[1], &sh[2]);
    a.scal[0] = nu;
    sh[0] = nu;
  }
  __syncthreads();
  const double nu = sh[0];
  const double pil = a.G.pi[l];
  const double* __restrict__ piG = a.G.pi;
  const double* __restrict__ h = a.h;
  const double* __restrict__ gdot = a.G.red;
  head_sums<COLS>(
      l, [](int j) { return j; }, [l](int) { return l; },
      [=](int i, int j) {
        return (double)VG[(int64_t)j * ldG + i] * piG[i + 1] * h[i];
      },
      [=](int j, double hs) {
        const double v1 = pil * gdot[j];
        s1[j] = v1;
        s2[j] = hs + nu * v1;
      },
      lds);
  const double* __restrict__ TG = a.G.T;
  double* z1 = a.z1;
  double* z2 = a.z2;
  tri_row_sums<2, COLS>(
      TG, tm, l, [=](int q) { return s1[q]; }, [=](int q) { return s2[q]; },
      [=](int j, double r0, double r1) {
        z1[j] = r0;
        z2[j] = r1;
      },
      lds);
  if (a.cslot >= 0)
    data_tcol<T, COLS>(a.D, k, tm, sh[1], sh[2], a.D.red + a.cslot, lds);
}

__device__ __forceinline__ double soft(double v, double th) {
  const double m = fabs(v) - th;
  return m > 0.0 ? copysign(m, v) : 0.0;
}

// Element-wise epilogue on row i of a query's output y (already rounded to
// storage): the built-in f_t, or one piece of an unrolled ISTA layer.
template <typename T>
__device__ __forceinline__ double dyn_store(const DynFuse& d, int64_t i,
                                            double y) {
  double out;
  if (d.kind == kDynTanhAbs || d.kind == kDynHead) {
    // maps of y alone (d.x is not read)
    if (d.kind == kDynTanhAbs) {
      out = d.a * tanh(fabs(y));
    } else {
      out = i < d.len ? d.a * y : 0.0;
      if (i < d.len) ((T*)d.aux)[i] = (T)out;
    }
    const T st = (T)out;
    ((T*)d.xnext)[i] = st;
    return (double)st;
  }
  if (d.kind == kDynScale && d.len > 0 && i >= d.len) return 0.0;
  const double x = (double)((const T*)d.x)[i];
  if (d.kind == kDynTanh) {
    out = tanh(d.a * y) + d.b * x;
  } else if (d.kind == kDynSoftHist) {
    out = soft(y, d.a) + d.b * (double)((const T*)d.xprev)[i];
  } else if (d.kind == kDynResidual) {
    out = x - y;  // observation minus Q x_t
  } else if (d.kind == kDynLista) {
    const T v = (T)(x + d.a * y);  // v_t = x_t + a_t Q'(.)
    ((T*)d.aux)[i] = v;
    out = soft((double)v, d.b);
  } else if (d.kind == kDynScale) {
    out = x * y;  // a diagonal matrix times y
  } else {  // kDynAxpy
    out = d.b * x - d.a * y;
  }
  const T stored = (T)out;
  ((T*)d.xnext)[i] = stored;
  return (double)stored;
}

// ------------------------------------------------------------------ TDOT --

// TDOT of a four-chunk workgroup in the row-split layout.
template <typename T, bool GEN, bool TWO>
__device__ __forceinline__ void tdot_rs(const TdotArgs& a, int blk) {
  __shared__ double dl[(TWO ? 2 : 1) * kWaves * kRsBlk];
  __shared__ double scr[kWaves];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 =
      (int64_t)blk * (kChunkRows * 4) + wave * kChunkRows + 4 * lane;
  const PhiloxKey key{a.key.k0, a.key.k1};
  double r0[4], r1[4];
  if (GEN) draw_rows<T>(key, a.gen_step, row0, a.lo, a.n, true, r0);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t i = row0 + e;
    if (!GEN) r0[e] = (i < a.n && i > a.lo) ? (double)((const T*)a.b)[i] : 0.0;
    r1[e] = (TWO && i < a.n) ? (double)((const T*)a.b2)[i] : 0.0;
  }
  double* out = a.partials + (int64_t)blk * a.pstride;
  double acc[4];
  rs_sweep<T, TWO ? 2 : 1, 0, true>((const T*)a.V, a.ld, a.ncols, row0, r0,
                                    r1, nullptr, acc, dl, out,
                                    out + a.slot2);
  if (a.ncols2 > 0)
    rs_sweep<T, 1, 0, true>((const T*)a.V2, a.ld, a.ncols2, row0, r0, r1,
                            nullptr, acc, dl, out + a.ncols, nullptr);
  if (a.want_ss) {
    double ss = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) ss += r0[e] * r0[e];
    const double s = block_sum(ss, scr);
    if (tid == 0) out[a.extra + kSlotPFSS] = s;
  }
}

template <typename T, int CPT, bool GEN, bool TWO, bool DB = false>
__device__ __forceinline__ void tdot_body(const TdotArgs& a, int blk) {
  if constexpr (CPT == 4) {
    tdot_rs<T, GEN, TWO>(a, blk);
    return;
  }
  __shared__ double g[GEN ? CPT * kChunkRows : 1];
  __shared__ double scr[kWaves];
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t blk0 = (int64_t)blk * (kChunkRows * CPT);
  const PhiloxKey key{a.key.k0, a.key.k1};
  double rhs0[CPT][4], rhs1[CPT][4];
  if (GEN) {
    draw_block<T, CPT>(key, a.gen_step, blk0, a.lo, a.n, true, g);
    __syncthreads();
    lane_rows<CPT>(g, rhs0);
  }
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int64_t i0 = blk0 + c * kChunkRows + 4 * lane;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = i0 + e;
      if (!GEN)
        rhs0[c][e] = (i < a.n && i > a.lo) ? (double)((const T*)a.b)[i] : 0.0;
      rhs1[c][e] = (TWO && i < a.n) ? (double)((const T*)a.b2)[i] : 0.0;
    }
  }
  double* out = a.partials + (int64_t)blk * a.pstride;
  double acc[CPT][4];
  constexpr bool kNT = CPT > 1;
  sweep<T, CPT, TWO ? 2 : 1, 0, kNT, DB>((const T*)a.V, a.ld, a.ncols, blk0,
                                         rhs0,
                                     rhs1, true, nullptr, 0.0, nullptr, 0.0,
                                     acc, acc, out, out + a.slot2);
  if (a.ncols2 > 0)
    sweep<T, CPT, 1, 0, kNT, DB>((const T*)a.V2, a.ld, a.ncols2, blk0, rhs0,
                                 rhs1,
                             true, nullptr, 0.0, nullptr, 0.0, acc, acc,
                             out + a.ncols, nullptr);
  if (a.want_ss) {
    // sum of squares over the workgroup's rows, once per row
    double ss = 0.0;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int64_t i = blk0 + c * kChunkRows + tid;
      double v = 0.0;
      if (GEN)
        v = g[c * kChunkRows + tid];
      else if (i < a.n && i > a.lo)
        v = (double)((const T*)a.b)[i];
      ss += v * v;
    }
    const double s = block_sum(ss, scr);
    if (tid == 0) out[a.extra + kSlotPFSS] = s;
  }
}

// ---------------------------------------------------------------- GEMV-N --

template <typename T, int CPT, int MODE, bool DB = false, bool GRP = false>
__device__ __forceinline__ void pass_body(const PassArgs& a, int blk) {
  __shared__ double gpf[CPT * kChunkRows];   // next draw (prefetch)
  __shared__ double gcur[CPT * kChunkRows];  // this draw, or the new column
  __shared__ double comb[kWaves * CPT * kChunkRows];
  __shared__ double scr[kWaves];
  const int tid = threadIdx.x;
  const int k = a.k;
  const int64_t blk0 = (int64_t)blk * (kChunkRows * CPT);
  T* __restrict__ V = (T*)a.V;
  const PhiloxKey key{a.key.k0, a.key.k1};
  if (a.pf) draw_block<T, CPT>(key, a.pf_step, blk0, a.pf_cut, a.n, true, gpf);
  if (MODE == kPassRandHaar)
    draw_block<T, CPT>(key, a.step, blk0, (int64_t)k - 1, a.n, false, gcur);
  __syncthreads();
  double gn[CPT][4], acc[CPT][4];
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      gn[c][e] = 0.0;
      acc[c][e] = 0.0;
    }
  if (a.pf) lane_rows<CPT>(gpf, gn);
  double* out = a.partials + (int64_t)blk * a.pstride;
  const double* z = a.z;
  if constexpr (MODE == kPassData && CPT <= 2) {
    // z = T' w (and T column kp) computed by every workgroup (see zpro)
    __shared__ double zl[kZproMax], tc[kZproMax];
    if (a.zpro) {
      const int kp = a.kp, tm = a.tmax;
      const double* __restrict__ Tm = a.T;
      const double* __restrict__ cc = a.c;
      const double* __restrict__ w = a.w;
      double* Tw = a.T;
      const bool first = blk == 0;
      if (kp > 0) {
        const double tau = a.tau[kp];
        tri_row_sums<1, GRP>(
            Tm, tm, kp, [=](int l) { return cc[l]; }, [](int) { return 0.0; },
            [=](int j, double r0, double) {
              tc[j] = -tau * r0;
              if (first) Tw[j + (int64_t)kp * tm] = -tau * r0;
            },
            comb);
      }
      wg_sums<1>(
          k, [](int) { return 0; }, [](int j) { return j + 1; },
          [=](int i, int j, double& t0, double& t1) {
            const double tij =
                (j == kp && i < kp) ? tc[i] : Tm[i + (int64_t)j * tm];
            t0 = tij * w[i];
            t1 = 0.0;
          },
          [=](int j, double r0, double) { zl[j] = r0; }, comb);
      z = zl;
    }
  }
  // the second sweeps below re-read these rows: keep them cached then
  const bool reread = (MODE == kPassData && a.cslot >= 0) ||
                      (MODE == kPassRandHaar && a.wnext);
  if (CPT > 1 && !reread)
    sweep<T, CPT, 1, 1, true, DB>(V, a.ld, k, blk0, gn, gn, a.pf != 0, z, 1.0,
                              nullptr, 0.0, acc, acc, out, nullptr);
  else
    sweep<T, CPT, 1, 1, false, DB>(V, a.ld, k, blk0, gn, gn, a.pf != 0, z, 1.0,
                                   nullptr,
                        0.0, acc, acc, out, nullptr);
  double vz[CPT];  // -(V z) for this thread's rows
  combine_rows<CPT>(acc, comb, vz);

  // Epilogue, one row per thread and chunk: the output rows, the new column
  // k, and the extras.
  double ssq = 0.0, pfnew = 0.0, pfss = 0.0, ysq = 0.0;
  const double pik = a.pi[k];
  const double cs = (MODE == kPassRandHaar) ? *a.cscale : 0.0;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int q = c * kChunkRows + tid;
    const int64_t i = blk0 + q;
    const double gnext = a.pf ? gpf[q] : 0.0;
    pfss += gnext * gnext;
    double unew = 0.0;
    if (i < a.n) {
      const double sg = (i < k) ? a.pi[i + 1] : pik;
      if (MODE == kPassData) {
        const double p = sg * ((double)((const T*)a.x)[i] + vz[c]);
        if (i < k) {
          a.head[i] = p;
        } else if (i == k) {
          *a.pivot = p;
        } else {
          const T ps = (T)p;
          V[(int64_t)k * a.ld + i] = ps;
          unew = (double)ps;
          ssq += unew * unew;
          pfnew += unew * gnext;
        }
      } else {
        const double w = (i < k) ? a.head[i] : cs * gcur[q];
        const T ys = (T)(sg * w + vz[c]);
        if (a.y) ((T*)a.y)[i] = ys;
        ysq += (double)ys * (double)ys;
        double xn = 0.0;
        if (a.dyn.kind) xn = dyn_store<T>(a.dyn, i, (double)ys);
        if (i > k) {
          const T gs = (T)gcur[q];
          V[(int64_t)k * a.ld + i] = gs;
          pfnew += (double)gs * gnext;
        }
        gcur[q] = xn;  // this thread's own entry, already used
      }
    }
    if (MODE == kPassData) gcur[q] = unew;
    if (MODE == kPassRandHaar && i >= a.n) gcur[q] = 0.0;
  }
  if (MODE == kPassRandHaar && a.wnext) {
    // the next query's TDOT over this panel (columns 0..k) with x_{t+1}
    __syncthreads();
    double xr[CPT][4];
    lane_rows<CPT>(gcur, xr);
    sweep<T, CPT, 1, 0, false, DB>(V, a.ld, k + 1, blk0, xr, xr, true, nullptr,
                                   0.0,
                        nullptr, 0.0, acc, acc, out, nullptr);
  }
  if (MODE == kPassData && a.cslot >= 0) {
    // dots of the earlier columns with the new one, for its T column (these
    // rows of V were just read, so they mostly come from L2)
    __syncthreads();
    double ur[CPT][4];
    lane_rows<CPT>(gcur, ur);
    sweep<T, CPT, 1, 0, false, DB>(V, a.ld, k, blk0, ur, ur, true, nullptr, 0.0,
                                   nullptr,
                        0.0, acc, acc, out + a.cslot, nullptr);
  }
  if (MODE == kPassData) {
    const double s = block_sum(ssq, scr);
    if (tid == 0) out[a.extra + kSlotSS] = s;
  } else if (a.want_ysq) {
    const double s = block_sum(ysq, scr);
    if (tid == 0) out[a.extra + kSlotYSQ] = s;
  }
  if (a.pf) {
    const double s1 = block_sum(pfnew, scr);
    const double s2 = block_sum(pfss, scr);
    if (tid == 0) {
      out[k] = s1;
      out[a.extra + kSlotPFSS] = s2;
    }
  }
}

// ------------------------------------------------- Ginibre random side --

template <typename T, int CPT, bool DB = false, bool GRP = false>
__device__ __forceinline__ void gin_pass_body(const GinPassArgs& a, int blk) {
  __shared__ double gpf[CPT * kChunkRows];
  __shared__ double gcur[CPT * kChunkRows];
  __shared__ double comb[kWaves * CPT * kChunkRows];
  const int tid = threadIdx.x;
  const int k = a.k, nb = a.nb;
  const int64_t blk0 = (int64_t)blk * (kChunkRows * CPT);
  T* __restrict__ B = (T*)a.B;
  const PhiloxKey key{a.key.k0, a.key.k1};
  if (a.pf) draw_block<T, CPT>(key, a.pf_step, blk0, a.pf_cut, a.n, true, gpf);
  draw_block<T, CPT>(key, a.step, blk0, (int64_t)k - 1, a.n, false, gcur);
  __syncthreads();
  double gn[CPT][4], acc0[CPT][4], acc1[CPT][4];
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      gn[c][e] = 0.0;
      acc0[c][e] = 0.0;
      acc1[c][e] = 0.0;
    }
  if (a.pf) lane_rows<CPT>(gpf, gn);
  double* out = a.partials + (int64_t)blk * a.pstride;
  const double* z1 = a.z1;
  const double* z2 = a.z2;
  double nu = 0.0;
  bool have_nu = false;
  if constexpr (CPT <= 2) {
    // the reflector step (as in gin_small_body), computed by every workgroup
    __shared__ double s1l[kZproMax], s2l[kZproMax], z1l[kZproMax],
        z2l[kZproMax], shr[3];
    if (a.spro) {
      const GinSmallArgs& g = a.small;
      const int kD = g.k, l = g.l, tm = g.tmax;
      const double ss = g.D.red[g.D_extra + kSlotSS], pk = *g.pivot;
      if (blk == 0 && tid == 0) {
        g.scal[0] = data_reflector<T>(g.D, kD, tm, ss, pk, g.flag, &shr[1],
                                      &shr[2]);
      }
      nu = sqrt(ss + pk * pk);  // the same expression as data_reflector's
      have_nu = true;
      const double pil = g.G.pi[l];
      const T* __restrict__ VG = (const T*)g.G.V;
      const int64_t ldG = g.G.ld;
      const double* __restrict__ piG = g.G.pi;
      const double* __restrict__ hh = g.h;
      const double* __restrict__ gdot = g.G.red;
      const double nuv = nu;
      wg_sums<1>(
          l, [](int j) { return j; }, [l](int) { return l; },
          [=](int i, int j, double& t0, double& t1) {
            t0 = (double)VG[(int64_t)j * ldG + i] * piG[i + 1] * hh[i];
            t1 = 0.0;
          },
          [=](int j, double hs, double) {
            const double v1 = pil * gdot[j];
            s1l[j] = v1;
            s2l[j] = hs + nuv * v1;
          },
          comb);
      const double* __restrict__ TG = g.G.T;
      tri_row_sums<2, GRP>(
          TG, tm, l, [=](int q) { return s1l[q]; },
          [=](int q) { return s2l[q]; },
          [=](int j, double r0, double r1) {
            z1l[j] = r0;
            z2l[j] = r1;
          },
          comb);
      z1 = z1l;
      z2 = z2l;
      if (blk == 0 && g.cslot >= 0)
        data_tcol<T, GRP>(g.D, kD, tm, shr[1], shr[2], g.D.red + g.cslot, comb);
    }
  }
  // reflector panel: acc0 -= V z1 (new basis vector), acc1 -= V z2 (output),
  // and the prefetch dots
  if (CPT > 1 && !a.wnext) {
    sweep<T, CPT, 1, 2, true, DB>((const T*)a.V, a.ld, k, blk0, gn, gn,
                              a.pf != 0, z1, 1.0, z2, 1.0, acc0, acc1, out,
                              nullptr);
    // explicit basis panel: acc1 += B c
    if (nb > 0)
      sweep<T, CPT, 0, 1, true, DB>((const T*)B, a.ld, nb, blk0, gn, gn, false,
                                a.c, -1.0, nullptr, 0.0, acc1, acc1, nullptr,
                                nullptr);
  } else {
    sweep<T, CPT, 1, 2, false, DB>((const T*)a.V, a.ld, k, blk0, gn, gn,
                                   a.pf != 0, z1,
                        1.0, z2, 1.0, acc0, acc1, out, nullptr);
    // explicit basis panel: acc1 += B c
    if (nb > 0)
      sweep<T, CPT, 0, 1, false, DB>((const T*)B, a.ld, nb, blk0, gn, gn, false,
                                     a.c,
                          -1.0, nullptr, 0.0, acc1, acc1, nullptr, nullptr);
  }
  double u0[CPT], u1[CPT];
  combine_rows<CPT>(acc0, comb, u0);
  combine_rows<CPT>(acc1, comb, u1);
  if (!have_nu) nu = a.scal[0];
  const double sigma = a.scal[1];
  const double pik = a.pi[k];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int q = c * kChunkRows + tid;
    const int64_t i = blk0 + q;
    double xn = 0.0;
    if (i < a.n) {
      const double sg = (i < k) ? a.pi[i + 1] : pik;
      const double gi = gcur[q];
      B[(int64_t)nb * a.ld + i] = (T)(sg * gi + u0[c]);
      const double hv = (i < k) ? a.h[i] : 0.0;
      const T ys = (T)(sigma * (u1[c] + sg * (hv + nu * gi)));
      if (a.y) ((T*)a.y)[i] = ys;
      if (a.dyn.kind) xn = dyn_store<T>(a.dyn, i, (double)ys);
    }
    gcur[q] = xn;  // this thread's own entry, already used
  }
  if (a.wnext) {
    // the next query's TDOT over this side's panels with x_{t+1}: the
    // reflector columns 0..k-1 and the basis columns 0..nb (the new one
    // included; its rows were written above by this workgroup)
    __syncthreads();
    double xr[CPT][4];
    lane_rows<CPT>(gcur, xr);
    sweep<T, CPT, 1, 0, false, DB>((const T*)a.V, a.ld, k, blk0, xr, xr, true,
                                   nullptr,
                        0.0, nullptr, 0.0, acc0, acc0, out, nullptr);
    sweep<T, CPT, 1, 0, false, DB>((const T*)B, a.ld, nb + 1, blk0, xr, xr,
                                   true, nullptr,
                        0.0, nullptr, 0.0, acc0, acc0, out + k, nullptr);
  }
}

// ---------------------------------------------------- kernel wrappers ----

template <typename T, int CPT, bool GEN, bool TWO, bool DB = false>
__global__ __launch_bounds__(kWG) void k_tdot(TdotArgs a) {
  tdot_body<T, CPT, GEN, TWO, DB>(a, blockIdx.x);
}

template <typename T, int CPT, int MODE, bool DB = false>
__global__ __launch_bounds__(kWG) void k_pass(PassArgs a) {
  pass_body<T, CPT, MODE, DB, true>(a, blockIdx.x);
}

template <typename T, int CPT, bool DB = false>
__global__ __launch_bounds__(kWG) void k_gin_pass(GinPassArgs a) {
  gin_pass_body<T, CPT, DB, true>(a, blockIdx.x);
}

// --------------------------------------------------- ISTA layer adjoint --

// One layer of the reverse pass: gbar = g * [|v| > theta] and the per-block
// sums of gbar * u (for dL/da) and of -g * sign(v) * [|v| > theta] (for
// dL/dtheta) into part[2 b], part[2 b + 1].
template <typename T>
__global__ __launch_bounds__(kWG) void k_lista_adj(ListaAdjArgs a) {
  __shared__ double scr[kWaves];
  const T* g = (const T*)a.g;
  const T* v = (const T*)a.v;
  const T* u = (const T*)a.u;
  T* gbar = (T*)a.gbar;
  double sa = 0.0, st = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * kWG) {
    const double vi = (double)v[i], gi = (double)g[i];
    const bool on = fabs(vi) > a.theta;
    const double gb = on ? gi : 0.0;
    gbar[i] = (T)gb;
    sa += gb * (double)u[i];
    if (on) st -= vi > 0.0 ? gi : -gi;
  }
  sa = block_sum(sa, scr);
  st = block_sum(st, scr);
  if (threadIdx.x == 0) {
    a.part[2 * blockIdx.x] = sa;
    a.part[2 * blockIdx.x + 1] = st;
  }
}

// Fixed-order sum of the per-block pairs into grad_a[t], grad_theta[t].
__global__ __launch_bounds__(kWG) void k_lista_sum(const double* part,
                                                   int nblk, double* ga,
                                                   double* gt) {
  __shared__ double scr[kWaves];
  double sa = 0.0, st = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kWG) {
    sa += part[2 * b];
    st += part[2 * b + 1];
  }
  sa = block_sum(sa, scr);
  st = block_sum(st, scr);
  if (threadIdx.x == 0) {
    *ga = sa;
    *gt = st;
  }
}

// ------------------------------------------------------- batched kernels --

template <typename T>
__device__ __forceinline__ const T* batch_vec(const void* base, int mod,
                                              int64_t n, int64_t t) {
  return (const T*)base + ((t - 1) % mod) * n;
}

template <typename T, int CPT, bool TWO>
__global__ __launch_bounds__(kWG) void k_tdot_batch(const TrialDev* D,
                                                    BatchMap m, BatchStep st) {
  const int trial = m.blk_trial[blockIdx.x];
  const TrialDev& d = D[trial];
  TdotArgs a = d.td;
  a.ncols = st.k;
  a.b = batch_vec<T>(d.xbase, d.xmod, a.n, st.step);
  // the column made by the previous query still needs its T column
  a.b2 = TWO ? (const void*)((const T*)a.V + (int64_t)(st.k - 1) * a.ld)
             : nullptr;
  tdot_body<T, CPT, false, TWO>(a, blockIdx.x - m.blk_first[trial]);
}

template <typename T, int CPT, int MODE>
__global__ __launch_bounds__(kWG) void k_pass_batch(const TrialDev* D,
                                                    BatchMap m, BatchStep st) {
  const int trial = m.blk_trial[blockIdx.x];
  const TrialDev& d = D[trial];
  PassArgs a = MODE == kPassData ? d.pd : d.pr;
  const int64_t n = a.n, t = st.step;
  a.k = st.k;
  a.step = st.step;
  if (MODE == kPassData) {
    a.x = batch_vec<T>(d.xbase, d.xmod, n, t);
  } else {
    // y is stored only when the run records it (the map reads it from
    // registers)
    a.y = d.ybase ? (void*)batch_vec<T>(d.ybase, d.ymod, n, t) : nullptr;
    a.pf = (int)st.step < d.T;
    a.pf_step = st.step + 1;
    a.pf_cut = st.k + 1;
    if (a.dyn.kind) {
      a.dyn.x = batch_vec<T>(d.xbase, d.xmod, n, t);
      a.dyn.xprev = t == 1 ? d.x0 : batch_vec<T>(d.xbase, d.xmod, n, t - 1);
      a.dyn.xnext = (void*)batch_vec<T>(d.xbase, d.xmod, n, t + 1);
    }
  }
  pass_body<T, CPT, MODE>(a, blockIdx.x - m.blk_first[trial]);
}

template <typename T, int CPT>
__global__ __launch_bounds__(kWG) void k_prefetch1_batch(const TrialDev* D,
                                                         BatchMap m) {
  const int trial = m.blk_trial[blockIdx.x];
  const PassArgs& pr = D[trial].pr;
  TdotArgs a{};
  a.V = pr.V;
  a.ld = pr.ld;
  a.gen = 1;
  a.key = pr.key;
  a.gen_step = 1;
  a.lo = 0;
  a.n = pr.n;
  a.want_ss = 1;
  a.partials = pr.partials;
  a.pstride = pr.pstride;
  a.extra = pr.extra;
  tdot_body<T, CPT, true, false>(a, blockIdx.x - m.blk_first[trial]);
}

__global__ __launch_bounds__(kWG) void k_copy_jobs(const CopyJob* jobs) {
  const CopyJob j = jobs[blockIdx.x];
  const uint32_t* __restrict__ src = (const uint32_t*)j.src;
  uint32_t* __restrict__ dst = (uint32_t*)j.dst;
  for (int64_t i = threadIdx.x; i < j.words; i += kWG) dst[i] = src[i];
}

// One workgroup per running trial: the fixed-order sums of its partial rows
// (workgroup-wide, several threads per slot), then its small step.
//   after the TDOT: w (k slots), the previous query's T-column dots, and the
//     previous random pass's prefetch dots and ||g||^2; then T column k-1 and
//     z = T' w;
//   after the data pass: ||p[k+1:]||^2; then the reflector scalars of both
//     sides and the random side's coefficients.
__device__ __forceinline__ void wg_reduce(const double* P, int pstride,
                                          int nrows, int s0, int count,
                                          double* out, double* lds) {
  wg_sums<1>(
      count, [](int) { return 0; }, [nrows](int) { return nrows; },
      [=](int r, int j, double& t0, double& t1) {
        t0 = P[(int64_t)r * pstride + s0 + j];
        t1 = 0.0;
      },
      [=](int j, double v, double) { out[s0 + j] = v; }, lds);
}

template <typename T, int OP>
__global__ __launch_bounds__(kWG) void k_trial_small(const TrialDev* D,
                                                     BatchStep st) {
  __shared__ double lds[2 * kWG];
  const TrialDev& d = D[blockIdx.x];
  const int k = st.k;
  if (OP == kBatchAfterTdot) {
    const TdotArgs& td = d.td;
    wg_reduce(td.partials, td.pstride, d.nwg, 0, k, (double*)d.sd.w, lds);
    const int kp = k - 1;
    if (kp > 0)
      wg_reduce(td.partials, td.pstride, d.nwg, td.slot2, kp,
                (double*)d.sd.w, lds);
    {
      // prefetch of the previous random pass (or of the query-1 kernel):
      // k dots and the extras
      const PassArgs& pr = d.pr;
      wg_reduce(pr.partials, pr.pstride, d.nwg, 0, k, d.hs.G.red, lds);
      wg_reduce(pr.partials, pr.pstride, d.nwg, pr.extra, kNumExtra,
                d.hs.G.red, lds);
    }
    SmallDataArgs a = d.sd;
    a.kp = kp;
    a.c = d.sd.w + td.slot2;
    a.k = k;
    if (kp > 0 || k > 0) small_data_body(a);
  } else {
    const PassArgs& pd = d.pd;
    wg_reduce(pd.partials, pd.pstride, d.nwg, pd.extra, kNumExtra, d.hs.D.red,
              lds);
    HaarSmallArgs a = d.hs;
    a.k = k;
    a.step = st.step;
    a.cslot = -1;
    haar_small_body<T>(a);
  }
}

// ------------------------------------------------ Gaussian ISTA batches --
//
// One query of every trial of an ISTA batch (all trials in lockstep, one
// chunk of 256 rows per workgroup).  The data side ds is R for Q-queries
// (query 0, the observation y = sigma Q x* + w, and the first query of
// every layer) and L for Q'-queries (the second query of every layer).

// Row r of trial i's trajectory X ((L + 1) x n).
template <typename T>
__device__ __forceinline__ T* ista_row(const IstaStep& st, int64_t n,
                                       int trial, int r) {
  return (T*)st.X + ((int64_t)trial * (st.L + 1) + r) * n;
}

template <typename T>
__device__ __forceinline__ const void* ista_input(const IstaTrialDev& d,
                                                  int trial, int ds,
                                                  const IstaStep& st) {
  const int64_t n = d.s[0].td.n;
  if (ds == 1) return d.res;
  if (st.bwd) return d.gbar;
  if (st.q == 0) return (const T*)st.xstar + (int64_t)trial * n;
  // query 2t - 1 reads x_t, row t - 1 of X
  return ista_row<T>(st, n, trial, (st.q - 1) / 2);
}

template <typename T, int CPT>
__global__ __launch_bounds__(kWG) void k_ista_tdot(const IstaTrialDev* D,
                                                   int ds, IstaStep st) {
  const int nwg = D[0].s[ds].nwg;
  const int trial = blockIdx.x / nwg;
  const IstaTrialDev& d = D[trial];
  TdotArgs a = d.s[ds].td;
  a.ncols = ds == 0 ? st.kR : st.kL;
  a.ncols2 = ds == 0 ? st.kL : st.kR;
  a.b = ista_input<T>(d, trial, ds, st);
  tdot_body<T, CPT, false, false>(a, blockIdx.x % nwg);
}

template <typename T, int CPT>
__global__ __launch_bounds__(kWG) void k_ista_data(const IstaTrialDev* D,
                                                   int ds, IstaStep st) {
  const int nwg = D[0].s[ds].nwg;
  const int trial = blockIdx.x / nwg;
  const IstaTrialDev& d = D[trial];
  PassArgs a = d.s[ds].pd;
  const int kD = ds == 0 ? st.kR : st.kL;
  a.k = kD;
  a.x = ista_input<T>(d, trial, ds, st);
  // this side is the random side of the next query except after query 0
  a.pf = st.q >= 1 && !st.last;
  a.pf_step = st.step + 1;
  a.pf_cut = kD;
  a.cslot = kD > 0 ? a.cslot : -1;
  pass_body<T, CPT, kPassData>(a, blockIdx.x % nwg);
}

template <typename T, int CPT>
__global__ __launch_bounds__(kWG) void k_ista_rand(const IstaTrialDev* D,
                                                   int gs, IstaStep st) {
  const int nwg = D[0].s[gs].nwg;
  const int trial = blockIdx.x / nwg;
  const IstaTrialDev& d = D[trial];
  GinPassArgs a = d.s[gs].gp;
  a.k = gs == 0 ? st.kR : st.kL;
  a.nb = gs == 0 ? st.kL : st.kR;
  a.h = a.h + a.nb;  // the basis-panel dots follow the reflector dots
  a.step = st.step;
  a.dyn.xprev = nullptr;
  a.dyn.aux = nullptr;
  if (st.q == 0) {
    // y = sigma Q x* + w (Q x* itself is not kept)
    a.y = nullptr;
    a.dyn.kind = kDynAxpy;
    a.dyn.a = -1.0;
    a.dyn.b = 1.0;
    a.dyn.x = (const T*)st.noise + (int64_t)trial * d.s[1].td.n;
    a.dyn.xnext = d.yobs;
  } else if (st.bwd && gs == 1) {
    // reverse pass: q = Q gbar
    a.y = d.res;
    a.dyn.kind = 0;
  } else if (st.bwd) {
    // reverse pass: g <- gbar - a_t Q' q, in place in G
    const int64_t n = d.s[0].td.n;
    a.y = d.U;
    a.dyn.kind = kDynAxpy;
    a.dyn.a = st.a;
    a.dyn.b = 1.0;
    a.dyn.x = d.gbar;
    a.dyn.xnext = (T*)st.G + (int64_t)trial * n;
  } else if (gs == 1) {
    // Q x_t, then y - Q x_t (only the residual is kept)
    a.y = nullptr;
    a.dyn.kind = kDynResidual;
    a.dyn.x = d.yobs;
    a.dyn.xnext = d.res;
  } else {
    // u_t = Q'(y - Q x_t), v_t = x_t + a_t u_t, x_{t+1} = soft(v_t, theta_t)
    const int64_t n = d.s[0].td.n;
    const int t = st.q / 2;  // 1-based layer
    a.y = d.U;
    a.dyn.aux = d.V;
    if (st.Urec) {
      // kept for the reverse pass
      const int64_t row = ((int64_t)trial * st.L + (t - 1)) * n;
      a.y = (T*)st.Urec + row;
      a.dyn.aux = (T*)st.Vrec + row;
    }
    a.dyn.kind = kDynLista;
    a.dyn.a = st.a;
    a.dyn.b = st.theta;
    a.dyn.x = ista_row<T>(st, n, trial, t - 1);
    a.dyn.xnext = ista_row<T>(st, n, trial, t);
  }
  gin_pass_body<T, CPT>(a, blockIdx.x % nwg);
}

// One workgroup per trial: the fixed-order sums of its partial rows, then
//   phase 0 (after the TDOT): z = T' w of the data side;
//   phase 1 (after the data pass): the data reflector's scalars, its T
//     column and the random side's coefficients (gin_small_body).
template <typename T, int PHASE>
__global__ __launch_bounds__(kWG) void k_ista_small(const IstaTrialDev* D,
                                                    int ds, IstaStep st) {
  __shared__ double lds[2 * kWG];
  const IstaTrialDev& d = D[blockIdx.x];
  const IstaSide& S = d.s[ds];
  const int kD = ds == 0 ? st.kR : st.kL;
  const int kG = ds == 0 ? st.kL : st.kR;
  const TdotArgs& td = S.td;
  if (PHASE == 0) {
    double* w = (double*)S.sd.w;
    wg_reduce(td.partials, td.pstride, S.nwg, 0, kD + kG, w, lds);
    if (kD > 0) {
      SmallDataArgs a = S.sd;
      a.kp = -1;
      a.k = kD;
      small_data_body(a);
    }
  } else {
    double* red = S.gs.D.red;
    const bool pf = st.q >= 1 && !st.last;
    if (pf) wg_reduce(td.partials, td.pstride, S.nwg, 0, kD + 1, red, lds);
    if (kD > 0)
      wg_reduce(td.partials, td.pstride, S.nwg, S.pd.cslot, kD, red, lds);
    wg_reduce(td.partials, td.pstride, S.nwg, td.extra, kNumExtra, red, lds);
    GinSmallArgs a = S.gs;
    a.k = kD;
    a.l = kG;
    a.h = a.h + kD;
    a.cslot = kD > 0 ? S.pd.cslot : -1;
    gin_small_body<T>(a);
  }
}

// The reverse pass of layer t for every trial (one workgroup per 256 rows of
// a trial): gbar = g [|v_t| > theta_t], and the workgroup's sums of
// gbar u_t and -g sign(v_t) [|v_t| > theta_t] (dL/da_t, dL/dtheta_t).
template <typename T>
__global__ __launch_bounds__(kWG) void k_ista_adj(IstaAdjArgs a) {
  __shared__ double scr[kWaves];
  const int trial = blockIdx.x / a.nwg, wg = blockIdx.x % a.nwg;
  const int64_t i = (int64_t)wg * kWG + threadIdx.x;
  const int64_t row = ((int64_t)trial * a.L + a.t) * a.n;
  double sa = 0.0, st = 0.0;
  if (i < a.n) {
    const double vi = (double)((const T*)a.Vrec)[row + i];
    const double gi = (double)((const T*)a.G)[(int64_t)trial * a.n + i];
    const bool on = fabs(vi) > a.theta;
    const double gb = on ? gi : 0.0;
    ((T*)a.D[trial].gbar)[i] = (T)gb;
    sa = gb * (double)((const T*)a.Urec)[row + i];
    if (on) st = vi > 0.0 ? -gi : gi;
  }
  sa = block_sum(sa, scr);
  st = block_sum(st, scr);
  if (threadIdx.x == 0) {
    double* p = a.part + 2 * ((int64_t)trial * a.nwg + wg);
    p[0] = sa;
    p[1] = st;
  }
}

// Fixed-order sums of a trial's workgroup pairs into its gradients.
__global__ __launch_bounds__(kWG) void k_ista_adjsum(IstaAdjArgs a) {
  __shared__ double scr[kWaves];
  const int trial = blockIdx.x;
  const double* p = a.part + 2 * (int64_t)trial * a.nwg;
  double sa = 0.0, st = 0.0;
  for (int b = threadIdx.x; b < a.nwg; b += kWG) {
    sa += p[2 * b];
    st += p[2 * b + 1];
  }
  sa = block_sum(sa, scr);
  st = block_sum(st, scr);
  if (threadIdx.x == 0) {
    a.grad_a[(int64_t)trial * a.L + a.t] = sa;
    a.grad_theta[(int64_t)trial * a.L + a.t] = st;
  }
}

// ------------------------------------------------- standalone kernels ----

__device__ __forceinline__ int slot_of(const SlotRanges& rg, int b) {
  int slot = -1;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (slot < 0) {
      if (b < rg.count[q])
        slot = rg.start[q] + b;
      else
        b -= rg.count[q];
    }
  }
  return slot;
}

__global__ __launch_bounds__(kWG) void k_reduce(ReduceJob ja, ReduceJob jb) {
  __shared__ double scr[kWaves];
  const int na = ja.rg.count[0] + ja.rg.count[1] + ja.rg.count[2];
  const bool first = (int)blockIdx.x < na;
  const ReduceJob& j = first ? ja : jb;
  const int slot = slot_of(j.rg, first ? blockIdx.x : blockIdx.x - na);
  double s = 0.0;
  for (int w = threadIdx.x; w < j.nwg; w += kWG)
    s += j.P[(int64_t)w * j.pstride + slot];
  s = block_sum(s, scr);
  if (threadIdx.x == 0) j.out[slot] = s;
}

// Two-stage form for many partial rows.  Stage 1: block (rb, pg) sums rows
// [rb * kRed1Rows, (rb + 1) * kRed1Rows) of slot positions pg * 32 .. + 31
// (positions count the slots of rg in order): thread (rl, sl) takes rows
// rl, rl + 8, ... of position sl, so the 32 threads of a row read one
// contiguous run of its slots; the 8 row lanes are added in order.
constexpr int kRed1Pos = 32;
constexpr int kRed1Lanes = kWG / kRed1Pos;

__device__ __forceinline__ int red_positions(const ReduceJob& j) {
  return j.rg.count[0] + j.rg.count[1] + j.rg.count[2];
}
__device__ __forceinline__ int red_blocks1(const ReduceJob& j) {
  const int np = red_positions(j);
  return np > 0 ? ((j.nwg + kRed1Rows - 1) / kRed1Rows) *
                      ((np + kRed1Pos - 1) / kRed1Pos)
                : 0;
}

__device__ __forceinline__ void reduce1_job(const ReduceJob& j, int b,
                                            double* lds) {
  const int np = red_positions(j);
  const int npg = (np + kRed1Pos - 1) / kRed1Pos;
  const int rb = b / npg, pg = b % npg;
  const int tid = threadIdx.x, sl = tid % kRed1Pos, rl = tid / kRed1Pos;
  const int p = pg * kRed1Pos + sl;
  double s = 0.0;
  if (p < np) {
    const int slot = slot_of(j.rg, p);
    const int r1 = min(j.nwg, (rb + 1) * kRed1Rows);
#pragma unroll 8
    for (int r = rb * kRed1Rows + rl; r < r1; r += kRed1Lanes)
      s += j.P[(int64_t)r * j.pstride + slot];
  }
  lds[tid] = s;
  __syncthreads();
  if (rl == 0 && p < np) {
    double t = 0.0;
    for (int q = 0; q < kRed1Lanes; ++q) t += lds[q * kRed1Pos + sl];
    j.stage[(int64_t)rb * np + p] = t;
  }
}

__global__ __launch_bounds__(kWG) void k_reduce1(ReduceJob ja, ReduceJob jb) {
  __shared__ double lds[kWG];
  const int na = red_blocks1(ja);
  if ((int)blockIdx.x < na)
    reduce1_job(ja, blockIdx.x, lds);
  else
    reduce1_job(jb, blockIdx.x - na, lds);
}

// Stage 2: one thread per slot position, the block sums in row-block order.
__global__ __launch_bounds__(kWG) void k_reduce2(ReduceJob ja, ReduceJob jb) {
  const int g = blockIdx.x * kWG + threadIdx.x;
  const int na = red_positions(ja);
  const bool first = g < na;
  const ReduceJob& j = first ? ja : jb;
  const int p = first ? g : g - na;
  const int np = red_positions(j);
  if (p >= np) return;
  const int nrb = (j.nwg + kRed1Rows - 1) / kRed1Rows;
  double s = 0.0;
#pragma unroll 8
  for (int rb = 0; rb < nrb; ++rb) s += j.stage[(int64_t)rb * np + p];
  j.out[slot_of(j.rg, p)] = s;
}

__global__ __launch_bounds__(kWG) void k_small_data(SmallDataArgs a) {
  small_data_body<false, true>(a);  // z = T'w: strided sums (T is cached)
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_haar_small(HaarSmallArgs a) {
  haar_small_body<T, true>(a);
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_gin_small(GinSmallArgs a) {
  gin_small_body<T, true>(a);
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_dyn(DynArgs a) {
  const T* y = (const T*)a.y;
  const T* x = (const T*)a.x;
  const T* xp = (const T*)a.xprev;
  T* xn = (T*)a.xnext;
  double inv = 1.0;
  if (a.kind == kDynNormalize) {
    const double q = *a.ysq;
    inv = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
  }
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * kWG) {
    const double yi = (double)y[i];
    double v;
    if (a.kind == kDynTanh) {
      v = tanh(a.a * yi) + a.b * (double)x[i];
    } else if (a.kind == kDynSoftHist) {
      const double m = fabs(yi) - a.a;
      const double st = m > 0.0 ? copysign(m, yi) : 0.0;
      v = st + a.b * (double)xp[i];
    } else {
      v = yi * inv + a.b * (double)x[i];
    }
    xn[i] = (T)v;
  }
}

// Zero `words` 4-byte words (a fill kernel rather than a memset node, so
// that the clearing can sit in a captured HIP graph).
__global__ __launch_bounds__(kWG) void k_zero(uint32_t* p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * kWG)
    p[i] = 0u;
}

__global__ __launch_bounds__(kWG) void k_fill(double* p, double v,
                                              int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * kWG)
    p[i] = v;
}

// ------------------------------------------------------------- launchers --

#define HD_CHECK_LAUNCH()                 \
  do {                                    \
    hipError_t e_ = hipGetLastError();    \
    if (e_ != hipSuccess) return (int)e_; \
  } while (0)

// Launch shapes: CPT = 1, 2 or 4 chunks of 256 rows per workgroup.
#define HD_DISPATCH_SHAPE(SH, KERNEL_T, ...)                            \
  do {                                                                  \
    if ((SH).cpt == 1)                                                  \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(KERNEL_T(1)), __VA_ARGS__);    \
    else if ((SH).cpt == 2)                                             \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(KERNEL_T(2)), __VA_ARGS__);    \
    else if ((SH).cpt == 4)                                             \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(KERNEL_T(4)), __VA_ARGS__);    \
    else                                                                \
      return -1;                                                        \
  } while (0)

// Launch of a panel kernel, with the timing events inside the dispatch when
// given.
template <typename... KArgs, typename... Args>
static void panel_launch(void (*k)(KArgs...), int nwg, hipStream_t s,
                         LaunchEvents ev, Args... args) {
  if (ev.start)
    hipExtLaunchKernelGGL(k, dim3(nwg), dim3(kWG), 0, s, ev.start, ev.stop, 0,
                          args...);
  else
    hipLaunchKernelGGL(k, dim3(nwg), dim3(kWG), 0, s, args...);
}

#define HD_DISPATCH_EV(SH, KERNEL_T, S, EV, ...)                  \
  do {                                                            \
    if ((SH).cpt == 1)                                            \
      panel_launch(KERNEL_T(1), (SH).nwg, S, EV, __VA_ARGS__);    \
    else if ((SH).cpt == 2)                                       \
      panel_launch(KERNEL_T(2), (SH).nwg, S, EV, __VA_ARGS__);    \
    else if ((SH).cpt == 4)                                       \
      panel_launch(KERNEL_T(4), (SH).nwg, S, EV, __VA_ARGS__);    \
    else                                                          \
      return -1;                                                  \
  } while (0)

// One-chunk FP32 launches of up to four workgroups per CU (the panels below
// 256K rows) take the sweeps with two column groups in flight (DB): few
// waves per CU are left to hide their load latency.  Wider launches keep
// the lighter single-group form.
constexpr int kDbMaxWG = 1024;
template <typename T>
bool use_db(Shape sh) {
  return sizeof(T) == 4 && sh.cpt == 1 && sh.nwg <= kDbMaxWG;
}

template <typename T, bool GEN, bool TWO>
static int tdot_shape(Shape sh, const TdotArgs& a, hipStream_t s,
                      LaunchEvents ev) {
  if (use_db<T>(sh)) {
    panel_launch(k_tdot<T, 1, GEN, TWO, true>, sh.nwg, s, ev, a);
    HD_CHECK_LAUNCH();
    return 0;
  }
#define K_(C) k_tdot<T, C, GEN, TWO>
  HD_DISPATCH_EV(sh, K_, s, ev, a);
#undef K_
  HD_CHECK_LAUNCH();
  return 0;
}

template <typename T>
static int tdot_t(Shape sh, const TdotArgs& a, hipStream_t s,
                  LaunchEvents ev) {
  if (a.gen) return tdot_shape<T, true, false>(sh, a, s, ev);
  if (a.b2) return tdot_shape<T, false, true>(sh, a, s, ev);
  return tdot_shape<T, false, false>(sh, a, s, ev);
}

int launch_tdot(int f64, Shape sh, const TdotArgs& a, hipStream_t s,
                LaunchEvents ev) {
  return f64 ? tdot_t<double>(sh, a, s, ev) : tdot_t<float>(sh, a, s, ev);
}

template <typename T, int MODE>
static int pass_shape(Shape sh, const PassArgs& a, hipStream_t s,
                      LaunchEvents ev) {
  if (use_db<T>(sh)) {
    panel_launch(k_pass<T, 1, MODE, true>, sh.nwg, s, ev, a);
    HD_CHECK_LAUNCH();
    return 0;
  }
#define K_(C) k_pass<T, C, MODE>
  HD_DISPATCH_EV(sh, K_, s, ev, a);
#undef K_
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_pass(int f64, Shape sh, int mode, const PassArgs& a,
                hipStream_t s, LaunchEvents ev) {
  if (f64)
    return mode == kPassData ? pass_shape<double, kPassData>(sh, a, s, ev)
                             : pass_shape<double, kPassRandHaar>(sh, a, s, ev);
  return mode == kPassData ? pass_shape<float, kPassData>(sh, a, s, ev)
                           : pass_shape<float, kPassRandHaar>(sh, a, s, ev);
}

template <typename T>
static int gin_shape(Shape sh, const GinPassArgs& a, hipStream_t s,
                     LaunchEvents ev) {
  if (use_db<T>(sh)) {
    panel_launch(k_gin_pass<T, 1, true>, sh.nwg, s, ev, a);
    HD_CHECK_LAUNCH();
    return 0;
  }
#define K_(C) k_gin_pass<T, C>
  HD_DISPATCH_EV(sh, K_, s, ev, a);
#undef K_
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_gin_pass(int f64, Shape sh, const GinPassArgs& a, hipStream_t s,
                    LaunchEvents ev) {
  return f64 ? gin_shape<double>(sh, a, s, ev) : gin_shape<float>(sh, a, s, ev);
}

int launch_tdot_batch(int f64, int cpt, int nblk, int two, const TrialDev* d,
                      BatchMap m, BatchStep st, hipStream_t s) {
  if (nblk <= 0) return 0;
  Shape sh{cpt, nblk};
  if (f64) {
    if (two) {
#define K_(C) k_tdot_batch<double, C, true>
      HD_DISPATCH_SHAPE(sh, K_, dim3(nblk), dim3(kWG), 0, s, d, m, st);
#undef K_
    } else {
#define K_(C) k_tdot_batch<double, C, false>
      HD_DISPATCH_SHAPE(sh, K_, dim3(nblk), dim3(kWG), 0, s, d, m, st);
#undef K_
    }
  } else {
    if (two) {
#define K_(C) k_tdot_batch<float, C, true>
      HD_DISPATCH_SHAPE(sh, K_, dim3(nblk), dim3(kWG), 0, s, d, m, st);
#undef K_
    } else {
#define K_(C) k_tdot_batch<float, C, false>
      HD_DISPATCH_SHAPE(sh, K_, dim3(nblk), dim3(kWG), 0, s, d, m, st);
#undef K_
    }
  }
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_pass_batch(int f64, int cpt, int nblk, int mode, const TrialDev* d,
                      BatchMap m, BatchStep st, hipStream_t s) {
  if (nblk <= 0) return 0;
  Shape sh{cpt, nblk};
  if (f64) {
    if (mode == kPassData) {
#define K_(C) k_pass_batch<double, C, kPassData>
      HD_DISPATCH_SHAPE(sh, K_, dim3(nblk), dim3(kWG), 0, s, d, m, st);
#undef K_
    } else {
#define K_(C) k_pass_batch<double, C, kPassRandHaar>
      HD_DISPATCH_SHAPE(sh, K_, dim3(nblk), dim3(kWG), 0, s, d, m, st);
#undef K_
    }
  } else {
    if (mode == kPassData) {
#define K_(C) k_pass_batch<float, C, kPassData>
      HD_DISPATCH_SHAPE(sh, K_, dim3(nblk), dim3(kWG), 0, s, d, m, st);
#undef K_
    } else {
#define K_(C) k_pass_batch<float, C, kPassRandHaar>
      HD_DISPATCH_SHAPE(sh, K_, dim3(nblk), dim3(kWG), 0, s, d, m, st);
#undef K_
    }
  }
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_trial_small(int f64, int op, int ntrials, const TrialDev* d,
                       BatchStep st, hipStream_t s) {
  if (ntrials <= 0) return 0;
  if (op == kBatchAfterTdot) {
    if (f64)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trial_small<double, kBatchAfterTdot>),
                         dim3(ntrials), dim3(kWG), 0, s, d, st);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trial_small<float, kBatchAfterTdot>),
                         dim3(ntrials), dim3(kWG), 0, s, d, st);
  } else {
    if (f64)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trial_small<double, kBatchAfterData>),
                         dim3(ntrials), dim3(kWG), 0, s, d, st);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trial_small<float, kBatchAfterData>),
                         dim3(ntrials), dim3(kWG), 0, s, d, st);
  }
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_prefetch1_batch(int f64, int cpt, int nblk, const TrialDev* d,
                           BatchMap m, hipStream_t s) {
  if (nblk <= 0) return 0;
  Shape sh{cpt, nblk};
  if (f64) {
#define K_(C) k_prefetch1_batch<double, C>
    HD_DISPATCH_SHAPE(sh, K_, dim3(nblk), dim3(kWG), 0, s, d, m);
#undef K_
  } else {
#define K_(C) k_prefetch1_batch<float, C>
    HD_DISPATCH_SHAPE(sh, K_, dim3(nblk), dim3(kWG), 0, s, d, m);
#undef K_
  }
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_ista_tdot(int f64, int cpt, int side, int nblk,
                     const IstaTrialDev* d, IstaStep st, hipStream_t s) {
  if (nblk <= 0) return 0;
#define HD_ISTA_LAUNCH(T, C)                                              \
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ista_tdot<T, C>), dim3(nblk), dim3(kWG), \
                     0, s, d, side, st)
  if (f64) {
    if (cpt == 4)
      HD_ISTA_LAUNCH(double, 4);
    else if (cpt == 2)
      HD_ISTA_LAUNCH(double, 2);
    else
      HD_ISTA_LAUNCH(double, 1);
  } else {
    if (cpt == 4)
      HD_ISTA_LAUNCH(float, 4);
    else if (cpt == 2)
      HD_ISTA_LAUNCH(float, 2);
    else
      HD_ISTA_LAUNCH(float, 1);
  }
#undef HD_ISTA_LAUNCH
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_ista_small(int f64, int phase, int side, int ntrials,
                      const IstaTrialDev* d, IstaStep st, hipStream_t s) {
  if (ntrials <= 0) return 0;
  if (phase == 0) {
    if (f64)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ista_small<double, 0>),
                         dim3(ntrials), dim3(kWG), 0, s, d, side, st);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ista_small<float, 0>),
                         dim3(ntrials), dim3(kWG), 0, s, d, side, st);
  } else {
    if (f64)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ista_small<double, 1>),
                         dim3(ntrials), dim3(kWG), 0, s, d, side, st);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ista_small<float, 1>),
                         dim3(ntrials), dim3(kWG), 0, s, d, side, st);
  }
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_ista_data(int f64, int cpt, int side, int nblk,
                     const IstaTrialDev* d, IstaStep st, hipStream_t s) {
  if (nblk <= 0) return 0;
#define HD_ISTA_LAUNCH(T, C)                                              \
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ista_data<T, C>), dim3(nblk), dim3(kWG), \
                     0, s, d, side, st)
  if (f64) {
    if (cpt == 4)
      HD_ISTA_LAUNCH(double, 4);
    else if (cpt == 2)
      HD_ISTA_LAUNCH(double, 2);
    else
      HD_ISTA_LAUNCH(double, 1);
  } else {
    if (cpt == 4)
      HD_ISTA_LAUNCH(float, 4);
    else if (cpt == 2)
      HD_ISTA_LAUNCH(float, 2);
    else
      HD_ISTA_LAUNCH(float, 1);
  }
#undef HD_ISTA_LAUNCH
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_ista_adj(int f64, int ntrials, const IstaAdjArgs& a,
                    hipStream_t s) {
  const int nblk = ntrials * a.nwg;
  if (f64)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ista_adj<double>), dim3(nblk),
                       dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ista_adj<float>), dim3(nblk),
                       dim3(kWG), 0, s, a);
  HD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_ista_adjsum, dim3(ntrials), dim3(kWG), 0, s, a);
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_ista_rand(int f64, int cpt, int side, int nblk,
                     const IstaTrialDev* d, IstaStep st, hipStream_t s) {
  if (nblk <= 0) return 0;
#define HD_ISTA_LAUNCH(T, C)                                              \
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ista_rand<T, C>), dim3(nblk), dim3(kWG), \
                     0, s, d, side, st)
  if (f64) {
    if (cpt == 4)
      HD_ISTA_LAUNCH(double, 4);
    else if (cpt == 2)
      HD_ISTA_LAUNCH(double, 2);
    else
      HD_ISTA_LAUNCH(double, 1);
  } else {
    if (cpt == 4)
      HD_ISTA_LAUNCH(float, 4);
    else if (cpt == 2)
      HD_ISTA_LAUNCH(float, 2);
    else
      HD_ISTA_LAUNCH(float, 1);
  }
#undef HD_ISTA_LAUNCH
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_copy_jobs(const CopyJob* jobs, int count, hipStream_t s) {
  if (count <= 0) return 0;
  hipLaunchKernelGGL(k_copy_jobs, dim3(count), dim3(kWG), 0, s, jobs);
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_lista_adj(int f64, const ListaAdjArgs& a, double* ga, double* gt,
                     hipStream_t s) {
  const int nblk = lista_blocks(a.n);
  if (f64)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_lista_adj<double>), dim3(nblk),
                       dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_lista_adj<float>), dim3(nblk),
                       dim3(kWG), 0, s, a);
  HD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_lista_sum, dim3(1), dim3(kWG), 0, s, a.part, nblk, ga,
                     gt);
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_reduce(const ReduceJob& a, const ReduceJob& b, hipStream_t s) {
  const int na = a.rg.count[0] + a.rg.count[1] + a.rg.count[2];
  const int nb = b.rg.count[0] + b.rg.count[1] + b.rg.count[2];
  if (na + nb <= 0) return 0;
  // HD_RED_TWO_STAGE overrides the row count from which two stages are used
  static const int from = [] {
    const char* e = std::getenv("HD_RED_TWO_STAGE");
    const int v = e ? std::atoi(e) : 0;
    return v >= 1 ? v : kRedTwoStage;
  }();
  const bool two = (na > 0 && a.nwg > from) || (nb > 0 && b.nwg > from);
  if (!two) {
    hipLaunchKernelGGL(k_reduce, dim3(na + nb), dim3(kWG), 0, s, a, b);
    HD_CHECK_LAUNCH();
    return 0;
  }
  if ((na > 0 && !a.stage) || (nb > 0 && !b.stage)) return 1;
  auto blocks1 = [](const ReduceJob& j, int np) {
    return np > 0 ? ((j.nwg + kRed1Rows - 1) / kRed1Rows) *
                        ((np + kRed1Pos - 1) / kRed1Pos)
                  : 0;
  };
  hipLaunchKernelGGL(k_reduce1, dim3(blocks1(a, na) + blocks1(b, nb)),
                     dim3(kWG), 0, s, a, b);
  HD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_reduce2, dim3((na + nb + kWG - 1) / kWG), dim3(kWG), 0,
                     s, a, b);
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_small_data(const SmallDataArgs& a, hipStream_t s) {
  if (a.kp <= 0 && (!a.w || a.k <= 0)) return 0;
  hipLaunchKernelGGL(k_small_data, dim3(1), dim3(kWG), 0, s, a);
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_haar_small(int f64, const HaarSmallArgs& a, hipStream_t s) {
  if (f64)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_haar_small<double>), dim3(1),
                       dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_haar_small<float>), dim3(1),
                       dim3(kWG), 0, s, a);
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_gin_small(int f64, const GinSmallArgs& a, hipStream_t s) {
  if (f64)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gin_small<double>), dim3(1),
                       dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gin_small<float>), dim3(1),
                       dim3(kWG), 0, s, a);
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_dyn(int f64, const DynArgs& a, hipStream_t s) {
  int64_t blocks = (a.n + kWG - 1) / kWG;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  if (f64)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_dyn<double>), dim3((int)blocks),
                       dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_dyn<float>), dim3((int)blocks),
                       dim3(kWG), 0, s, a);
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t words = (int64_t)(bytes / 4);
  if (words <= 0) return 0;
  int64_t blocks = (words + kWG - 1) / kWG;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_zero, dim3((int)blocks), dim3(kWG), 0, s,
                     (uint32_t*)p, words);
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_fill(double* p, double v, int64_t count, hipStream_t s) {
  if (count <= 0) return 0;
  int64_t blocks = (count + kWG - 1) / kWG;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill, dim3((int)blocks), dim3(kWG), 0, s, p, v, count);
  HD_CHECK_LAUNCH();
  return 0;
}

}  // namespace hd
