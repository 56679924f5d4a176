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
// Panel kernels stream the panel once per pass, RPL rows per lane (4: one
// 16-byte load per column for FP32; 1 for small panels, to give them more
// workgroups), and keep every accumulation in FP64:
//   k_tdot     : w = V' b (per-workgroup partials; column sums by a wave
//                reduce-scatter, then LDS across the four waves)
//   k_pass     : out = Delta a - V z (GEMV-N); writes the new panel column
//                and the dot products with the next query's Philox draw
//   k_gin_pass : the random side of a Ginibre query (two GEMV-N plus the
//                explicit basis panel)
// Cross-workgroup sums are fixed-order, so results are bitwise reproducible
// run to run.  For small grids the last workgroup to finish does that sum and
// the query's FP64 scalar step itself (Tail); otherwise k_reduce and a small
// one-workgroup kernel follow.
#include <hip/hip_runtime.h>

#include "hd_device.hpp"
#include "hd_internal.hpp"

namespace hd {

constexpr int kCG = 16;  // columns per group in the panel loops

// Draws g_step[i] for the RPL rows i0..i0+RPL-1 of one lane; rows outside
// (lo, n) get 0.  Values are rounded to the storage type when `round`.
template <typename T, int RPL>
__device__ __forceinline__ void draw_rows(PhiloxKey key, uint32_t step,
                                          int64_t i0, int64_t lo, int64_t n,
                                          bool round, double (&out)[RPL]) {
#pragma unroll
  for (int e = 0; e < RPL; ++e) out[e] = 0.0;
  if (i0 >= n || i0 + RPL - 1 <= lo) return;
  double g[4];
  normals4(key, step, 0u, (uint64_t)(i0 >> 2), g);
#pragma unroll
  for (int e = 0; e < RPL; ++e) {
    const int64_t i = i0 + e;
    const double v = g[(RPL == 4) ? e : (int)(i & 3)];
    if (i > lo && i < n) out[e] = round ? (double)(T)v : v;
  }
}

// ------------------------------------------------- small FP64 steps ------

// Column kp of T from the dots c = V[:, :kp]' u_kp (compact-WY recurrence of
// Schreiber and Van Loan), then z = T' w for the leading k x k block.
__device__ void small_data_body(const SmallDataArgs& a) {
  const int tm = a.tmax, kp = a.kp;
  if (kp > 0) {
    const double tau = a.tau[kp];
    for (int j = threadIdx.x; j < kp; j += kWG) {
      double s = 0.0;
      for (int l = j; l < kp; ++l) s += a.T[j + (int64_t)l * tm] * a.c[l];
      a.T[j + (int64_t)kp * tm] = -tau * s;
    }
  }
  __threadfence_block();
  __syncthreads();
  if (a.w) {
    for (int j = threadIdx.x; j < a.k; j += kWG) {
      double s = 0.0;
      for (int i = 0; i <= j; ++i) s += a.T[i + (int64_t)j * tm] * a.w[i];
      a.z[j] = s;
    }
  }
}

// Data-side reflector of a query from p (pivot p_k, ss = ||p[k+1:]||^2 of the
// stored entries): nu = ||p[k:]||, s = sign(p_k), stored pivot u_k = p_k + s nu
// rounded to storage, tau = 2/||u||^2 from the stored entries.  nu = 0 gives
// the identity (tau = 0, no sign).  Written by one thread; returns nu.
template <typename T>
__device__ double data_reflector(const PanelDev& D, int k, int tm, double ss,
                                 double pk, int* flag) {
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
  return nu;
}

// Haar, after the data-side pass of query t (k = t-1 reflectors per panel):
// the data reflector R_t, then L_t = H_t(g_t) from the prefetched dots V'g
// over rows > k and ||g[k+1:]||^2, its T column, s_vec = V' Delta w for
// w = [p[:k]; (nu/||g[k:]||) g[k:]] (the vector L_t R_t p_t of eq. (Qtxt)
// before L_1..L_{t-1}), and z_G = T_G s_vec.
template <typename T>
__device__ void haar_small_body(const HaarSmallArgs& a) {
  __shared__ double sh[4];
  const int k = a.k, tid = threadIdx.x, tm = a.tmax;
  T* VG = (T*)a.G.V;
  const int64_t ldG = a.G.ld;
  double* cG = a.zG + tm;
  double* sv = a.zG + 2 * tm;
  if (tid == 0) {
    const double nu = data_reflector<T>(a.D, k, tm,
                                        a.D.red[a.extra + kSlotSS], *a.pivot,
                                        a.flag);
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
  __threadfence_block();
  __syncthreads();
  const double tauG = sh[0], cs = sh[1], gk = sh[2], upG = sh[3];
  const double piGk = a.G.pi[k];
  for (int j = tid; j < k; j += kWG) {
    const T* colG = VG + (int64_t)j * ldG;
    double hg = 0.0;
    for (int i = 0; i < k; ++i)
      hg += (double)colG[i] * a.G.pi[i + 1] * a.head[i];
    const double gdot = a.G.red[j];
    cG[j] = gdot + (double)colG[k] * upG;
    sv[j] = hg + piGk * cs * (gdot + (double)colG[k] * gk);
  }
  __threadfence_block();
  __syncthreads();
  for (int j = tid; j < k; j += kWG) {
    double tG = 0.0, zz = 0.0;
    for (int l = j; l < k; ++l) {
      const double tjl = a.G.T[j + (int64_t)l * tm];
      tG += tjl * cG[l];
      zz += tjl * sv[l];
    }
    a.zG[j] = zz;
    a.G.T[j + (int64_t)k * tm] = -tauG * tG;
  }
}

// Ginibre: the data reflector, then the random-side coefficients
// s1 = V_G' Delta_G [0; g] = pi_l (prefetched dots over rows >= l),
// s2 = V_G' Delta_G h (head rows only) + nu s1; z1 = T_G s1, z2 = T_G s2.
template <typename T>
__device__ void gin_small_body(const GinSmallArgs& a) {
  __shared__ double sh[1];
  const int k = a.k, l = a.l, tid = threadIdx.x, tm = a.tmax;
  const T* VG = (const T*)a.G.V;
  const int64_t ldG = a.G.ld;
  double* s1 = a.z1 + tm;
  double* s2 = a.z1 + 2 * tm;
  if (tid == 0) {
    const double nu = data_reflector<T>(a.D, k, tm,
                                        a.D.red[a.D_extra + kSlotSS], *a.pivot,
                                        a.flag);
    a.scal[0] = nu;
    sh[0] = nu;
  }
  __threadfence_block();
  __syncthreads();
  const double nu = sh[0];
  const double pil = a.G.pi[l];
  for (int j = tid; j < l; j += kWG) {
    const T* col = VG + (int64_t)j * ldG;
    double hs = 0.0;
    for (int i = 0; i < l; ++i) hs += (double)col[i] * a.G.pi[i + 1] * a.h[i];
    const double v1 = pil * a.G.red[j];
    s1[j] = v1;
    s2[j] = hs + nu * v1;
  }
  __threadfence_block();
  __syncthreads();
  for (int j = tid; j < l; j += kWG) {
    double z1 = 0.0, z2 = 0.0;
    for (int q = j; q < l; ++q) {
      const double tjq = a.G.T[j + (int64_t)q * tm];
      z1 += tjq * s1[q];
      z2 += tjq * s2[q];
    }
    a.z1[j] = z1;
    a.z2[j] = z2;
  }
}

// Last-workgroup epilogue of a panel kernel: sum the partial rows in a fixed
// order, then run the query's small step.  A no-op without a counter.
template <typename T>
__device__ __forceinline__ void run_tail(const Tail& tl,
                                         const double* partials, int pstride) {
  if (!tl.counter) return;
  const int nwg = gridDim.x;
  const int g = blockIdx.x / tl.gsz;
  const int ng = (nwg + tl.gsz - 1) / tl.gsz;
  const int w0 = g * tl.gsz, w1 = min(w0 + tl.gsz, nwg);
  if (!arrive_last(tl.counter + 1 + g, w1 - w0)) return;
  if (ng == 1) {
    reduce_rows(partials, pstride, w0, w1, tl.rg, tl.out);
  } else {
    reduce_rows(partials, pstride, w0, w1, tl.rg,
                tl.gpart + (int64_t)g * pstride);
    if (!arrive_last(tl.counter, ng)) return;
    reduce_rows(tl.gpart, pstride, 0, ng, tl.rg, tl.out);
  }
  __threadfence();
  if (tl.op == kTailSmallData)
    small_data_body(tl.sd);
  else if (tl.op == kTailHaarSmall)
    haar_small_body<T>(tl.hs);
  else if (tl.op == kTailGinSmall)
    gin_small_body<T>(tl.gs);
}

// Element-wise map f_t on one row (y already rounded to storage).
__device__ __forceinline__ double dyn_row(const DynFuse& d, double yi,
                                          double xi, double xpi) {
  if (d.kind == kDynTanh) return tanh(d.a * yi) + d.b * xi;
  const double m = fabs(yi) - d.a;
  return (m > 0.0 ? copysign(m, yi) : 0.0) + d.b * xpi;
}

// ------------------------------------------------------------------ TDOT --

template <typename T, int RPL, int CPT, bool GEN, bool TWO>
__global__ __launch_bounds__(kWG) void k_tdot(TdotArgs a) {
  constexpr int kRows = kWG * RPL;
  __shared__ double lds[kWaves * kCG];
  __shared__ double scr[kWaves];
  const int tid = threadIdx.x;
  const int64_t blk0 = (int64_t)blockIdx.x * (kRows * CPT);
  double b[CPT][RPL];
  double b2[CPT][RPL];
  bool cvalid[CPT];
  double ss = 0.0;
  const PhiloxKey key{a.key.k0, a.key.k1};
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int64_t row0 = blk0 + (int64_t)c * kRows;
    cvalid[c] = row0 < a.ld;
    const int64_t i0 = row0 + RPL * tid;
    if (GEN) {
      draw_rows<T, RPL>(key, a.gen_step, i0, a.lo, cvalid[c] ? a.n : 0, true,
                        b[c]);
    }
#pragma unroll
    for (int e = 0; e < RPL; ++e) {
      const int64_t i = i0 + e;
      const bool in = cvalid[c] && i < a.n;
      if (!GEN) b[c][e] = (in && i > a.lo) ? (double)((const T*)a.b)[i] : 0.0;
      b2[c][e] = (TWO && in) ? (double)((const T*)a.b2)[i] : 0.0;
      ss += b[c][e] * b[c][e];
    }
  }
  double* out = a.partials + (int64_t)blockIdx.x * a.pstride;
#pragma unroll 1
  for (int seg = 0; seg < 2; ++seg) {
    const T* V = (const T*)(seg ? a.V2 : a.V);
    const int nc = seg ? a.ncols2 : a.ncols;
    const int slot0 = seg ? a.ncols : 0;
#pragma unroll 1
    for (int j0 = 0; j0 < nc; j0 += kCG) {
      double acc[kCG], acc2[kCG];
#pragma unroll
      for (int jj = 0; jj < kCG; ++jj) {
        acc[jj] = 0.0;
        acc2[jj] = 0.0;
      }
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        if (!cvalid[c]) continue;
        const int64_t r = blk0 + (int64_t)c * kRows + RPL * tid;
#pragma unroll
        for (int jj = 0; jj < kCG; ++jj) {
          const int j = min(j0 + jj, nc - 1);
          double v[RPL];
          load_rows<RPL>(V + (int64_t)j * a.ld + r, v);
#pragma unroll
          for (int e = 0; e < RPL; ++e) {
            acc[jj] += v[e] * b[c][e];
            if (TWO) acc2[jj] += v[e] * b2[c][e];
          }
        }
      }
      const double s = block_column_sums<kCG>(acc, lds);
      if (tid < kCG && j0 + tid < nc) out[slot0 + j0 + tid] = s;
      if (TWO && seg == 0) {
        const double s2 = block_column_sums<kCG>(acc2, lds);
        if (tid < kCG && j0 + tid < nc) out[a.slot2 + j0 + tid] = s2;
      }
    }
  }
  if (a.want_ss) {
    const double s = block_sum(ss, scr);
    if (tid == 0) out[a.extra + kSlotPFSS] = s;
  }
  run_tail<T>(a.tail, a.partials, a.pstride);
}

// ---------------------------------------------------------------- GEMV-N --

template <typename T, int RPL, int CPT, int MODE>
__global__ __launch_bounds__(kWG) void k_pass(PassArgs a) {
  constexpr int kRows = kWG * RPL;
  __shared__ double lds[kWaves * kCG];
  __shared__ double scr[kWaves];
  const int tid = threadIdx.x;
  const int k = a.k;
  const int64_t blk0 = (int64_t)blockIdx.x * (kRows * CPT);
  T* __restrict__ V = (T*)a.V;
  const PhiloxKey key{a.key.k0, a.key.k1};
  double acc[CPT][RPL];
  double gn[CPT][RPL];
  bool cvalid[CPT];
  double pfss = 0.0;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int64_t row0 = blk0 + (int64_t)c * kRows;
    cvalid[c] = row0 < a.ld;
    draw_rows<T, RPL>(key, a.pf_step, row0 + RPL * tid, a.pf_cut,
                      (a.pf && cvalid[c]) ? a.n : 0, true, gn[c]);
#pragma unroll
    for (int e = 0; e < RPL; ++e) {
      acc[c][e] = 0.0;
      pfss += gn[c][e] * gn[c][e];
    }
  }
  double* out = a.partials + (int64_t)blockIdx.x * a.pstride;

#pragma unroll 1
  for (int j0 = 0; j0 < k; j0 += kCG) {
    double zz[kCG];
    double pacc[kCG];
#pragma unroll
    for (int jj = 0; jj < kCG; ++jj) {
      zz[jj] = (j0 + jj < k) ? a.z[j0 + jj] : 0.0;
      pacc[jj] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if (!cvalid[c]) continue;
      const int64_t r = blk0 + (int64_t)c * kRows + RPL * tid;
#pragma unroll
      for (int jj = 0; jj < kCG; ++jj) {
        const int j = min(j0 + jj, k - 1);
        double v[RPL];
        load_rows<RPL>(V + (int64_t)j * a.ld + r, v);
#pragma unroll
        for (int e = 0; e < RPL; ++e) {
          acc[c][e] -= v[e] * zz[jj];
          pacc[jj] += v[e] * gn[c][e];
        }
      }
    }
    if (a.pf) {
      const double s = block_column_sums<kCG>(pacc, lds);
      if (tid < kCG && j0 + tid < k) out[j0 + tid] = s;
    }
  }

  // Epilogue: form the output rows, write the new column k, and the extras.
  double ssq = 0.0, pfnew = 0.0, ysq = 0.0;
  const double pik = a.pi[k];
  const double cs = (MODE == kPassRandHaar) ? *a.cscale : 0.0;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    if (!cvalid[c]) continue;
    const int64_t i0 = blk0 + (int64_t)c * kRows + RPL * tid;
    double gt[RPL];
    if (MODE == kPassRandHaar)
      draw_rows<T, RPL>(key, a.step, i0, (int64_t)k - 1, a.n, false, gt);
#pragma unroll
    for (int e = 0; e < RPL; ++e) {
      const int64_t i = i0 + e;
      if (i >= a.n) continue;
      const double sg = (i < k) ? a.pi[i + 1] : pik;
      if (MODE == kPassData) {
        const double p = sg * ((double)((const T*)a.x)[i] + acc[c][e]);
        if (i < k) {
          a.head[i] = p;
        } else if (i == k) {
          *a.pivot = p;
        } else {
          const T ps = (T)p;
          V[(int64_t)k * a.ld + i] = ps;
          const double pd = (double)ps;
          ssq += pd * pd;
          pfnew += pd * gn[c][e];
        }
      } else {
        const double w = (i < k) ? a.head[i] : cs * gt[e];
        const T ys = (T)(sg * w + acc[c][e]);
        ((T*)a.y)[i] = ys;
        ysq += (double)ys * (double)ys;
        if (a.dyn.kind) {
          const double xi = (double)((const T*)a.dyn.x)[i];
          const double xpi = a.dyn.kind == kDynSoftHist
                                 ? (double)((const T*)a.dyn.xprev)[i]
                                 : 0.0;
          ((T*)a.dyn.xnext)[i] = (T)dyn_row(a.dyn, (double)ys, xi, xpi);
        }
        if (i > k) {
          const T gs = (T)gt[e];
          V[(int64_t)k * a.ld + i] = gs;
          pfnew += (double)gs * gn[c][e];
        }
      }
    }
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
  run_tail<T>(a.tail, a.partials, a.pstride);
}

// ------------------------------------------------- Ginibre random side --

template <typename T, int RPL, int CPT>
__global__ __launch_bounds__(kWG) void k_gin_pass(GinPassArgs a) {
  constexpr int kRows = kWG * RPL;
  __shared__ double lds[kWaves * kCG];
  const int tid = threadIdx.x;
  const int k = a.k, nb = a.nb;
  const int64_t blk0 = (int64_t)blockIdx.x * (kRows * CPT);
  const T* __restrict__ V = (const T*)a.V;
  T* __restrict__ B = (T*)a.B;
  const PhiloxKey key{a.key.k0, a.key.k1};
  double acc1[CPT][RPL], acc2[CPT][RPL], gn[CPT][RPL];
  bool cvalid[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int64_t row0 = blk0 + (int64_t)c * kRows;
    cvalid[c] = row0 < a.ld;
    draw_rows<T, RPL>(key, a.pf_step, row0 + RPL * tid, a.pf_cut,
                      (a.pf && cvalid[c]) ? a.n : 0, true, gn[c]);
#pragma unroll
    for (int e = 0; e < RPL; ++e) {
      acc1[c][e] = 0.0;
      acc2[c][e] = 0.0;
    }
  }
  double* out = a.partials + (int64_t)blockIdx.x * a.pstride;
  // reflector panel: two GEMV-N (z1 -> new basis vector, z2 -> output) and
  // the prefetch dots
#pragma unroll 1
  for (int j0 = 0; j0 < k; j0 += kCG) {
    double za[kCG], zb[kCG], pacc[kCG];
#pragma unroll
    for (int jj = 0; jj < kCG; ++jj) {
      const bool ok = j0 + jj < k;
      za[jj] = ok ? a.z1[j0 + jj] : 0.0;
      zb[jj] = ok ? a.z2[j0 + jj] : 0.0;
      pacc[jj] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if (!cvalid[c]) continue;
      const int64_t r = blk0 + (int64_t)c * kRows + RPL * tid;
#pragma unroll
      for (int jj = 0; jj < kCG; ++jj) {
        const int j = min(j0 + jj, k - 1);
        double v[RPL];
        load_rows<RPL>(V + (int64_t)j * a.ld + r, v);
#pragma unroll
        for (int e = 0; e < RPL; ++e) {
          acc1[c][e] -= v[e] * za[jj];
          acc2[c][e] -= v[e] * zb[jj];
          pacc[jj] += v[e] * gn[c][e];
        }
      }
    }
    if (a.pf) {
      const double s = block_column_sums<kCG>(pacc, lds);
      if (tid < kCG && j0 + tid < k) out[j0 + tid] = s;
    }
  }
  // explicit basis panel: + B c
#pragma unroll 1
  for (int j0 = 0; j0 < nb; j0 += kCG) {
    double cv[kCG];
#pragma unroll
    for (int jj = 0; jj < kCG; ++jj)
      cv[jj] = (j0 + jj < nb) ? a.c[j0 + jj] : 0.0;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if (!cvalid[c]) continue;
      const int64_t r = blk0 + (int64_t)c * kRows + RPL * tid;
#pragma unroll
      for (int jj = 0; jj < kCG; ++jj) {
        const int j = min(j0 + jj, nb - 1);
        double v[RPL];
        load_rows<RPL>(B + (int64_t)j * a.ld + r, v);
#pragma unroll
        for (int e = 0; e < RPL; ++e) acc2[c][e] += v[e] * cv[jj];
      }
    }
  }
  const double nu = a.scal[0], sigma = a.scal[1];
  const double pik = a.pi[k];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    if (!cvalid[c]) continue;
    const int64_t i0 = blk0 + (int64_t)c * kRows + RPL * tid;
    double gt[RPL];
    draw_rows<T, RPL>(key, a.step, i0, (int64_t)k - 1, a.n, false, gt);
#pragma unroll
    for (int e = 0; e < RPL; ++e) {
      const int64_t i = i0 + e;
      if (i >= a.n) continue;
      const double sg = (i < k) ? a.pi[i + 1] : pik;
      const double gi = gt[e];
      B[(int64_t)nb * a.ld + i] = (T)(sg * gi + acc1[c][e]);
      const double hv = (i < k) ? a.h[i] : 0.0;
      const T ys = (T)(sigma * (acc2[c][e] + sg * (hv + nu * gi)));
      ((T*)a.y)[i] = ys;
      if (a.dyn.kind) {
        const double xi = (double)((const T*)a.dyn.x)[i];
        const double xpi = a.dyn.kind == kDynSoftHist
                               ? (double)((const T*)a.dyn.xprev)[i]
                               : 0.0;
        ((T*)a.dyn.xnext)[i] = (T)dyn_row(a.dyn, (double)ys, xi, xpi);
      }
    }
  }
  run_tail<T>(a.tail, a.partials, a.pstride);
}

// ------------------------------------------------- standalone kernels ----

__global__ __launch_bounds__(kWG) void k_reduce(const double* __restrict__ P,
                                                int pstride, int nwg,
                                                SlotRanges rg,
                                                double* __restrict__ out) {
  __shared__ double scr[kWaves];
  int b = blockIdx.x, slot = -1;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (slot < 0) {
      if (b < rg.count[q])
        slot = rg.start[q] + b;
      else
        b -= rg.count[q];
    }
  }
  double s = 0.0;
  for (int w = threadIdx.x; w < nwg; w += kWG)
    s += P[(int64_t)w * pstride + slot];
  s = block_sum(s, scr);
  if (threadIdx.x == 0) out[slot] = s;
}

__global__ __launch_bounds__(kWG) void k_small_data(SmallDataArgs a) {
  small_data_body(a);
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_haar_small(HaarSmallArgs a) {
  haar_small_body<T>(a);
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_gin_small(GinSmallArgs a) {
  gin_small_body<T>(a);
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

// Launch shapes (rpl, cpt): (1,1) for small panels, (4, 1|2|4|8) otherwise.
template <typename T, bool GEN, bool TWO>
static int tdot_shape(Shape sh, const TdotArgs& a, hipStream_t s) {
  const dim3 g(sh.nwg), b(kWG);
  if (sh.rpl == 1 && sh.cpt == 1)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_tdot<T, 1, 1, GEN, TWO>), g, b, 0, s, a);
  else if (sh.rpl == 4 && sh.cpt == 1)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_tdot<T, 4, 1, GEN, TWO>), g, b, 0, s, a);
  else if (sh.rpl == 4 && sh.cpt == 2)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_tdot<T, 4, 2, GEN, TWO>), g, b, 0, s, a);
  else if (sh.rpl == 4 && sh.cpt == 4)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_tdot<T, 4, 4, GEN, TWO>), g, b, 0, s, a);
  else if (sh.rpl == 4 && sh.cpt == 8)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_tdot<T, 4, 8, GEN, TWO>), g, b, 0, s, a);
  else
    return -1;
  HD_CHECK_LAUNCH();
  return 0;
}

template <typename T>
static int tdot_t(Shape sh, const TdotArgs& a, hipStream_t s) {
  if (a.gen) return tdot_shape<T, true, false>(sh, a, s);
  if (a.b2) return tdot_shape<T, false, true>(sh, a, s);
  return tdot_shape<T, false, false>(sh, a, s);
}

int launch_tdot(int f64, Shape sh, const TdotArgs& a, hipStream_t s) {
  return f64 ? tdot_t<double>(sh, a, s) : tdot_t<float>(sh, a, s);
}

template <typename T, int MODE>
static int pass_shape(Shape sh, const PassArgs& a, hipStream_t s) {
  const dim3 g(sh.nwg), b(kWG);
  if (sh.rpl == 1 && sh.cpt == 1)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pass<T, 1, 1, MODE>), g, b, 0, s, a);
  else if (sh.rpl == 4 && sh.cpt == 1)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pass<T, 4, 1, MODE>), g, b, 0, s, a);
  else if (sh.rpl == 4 && sh.cpt == 2)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pass<T, 4, 2, MODE>), g, b, 0, s, a);
  else if (sh.rpl == 4 && sh.cpt == 4)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pass<T, 4, 4, MODE>), g, b, 0, s, a);
  else if (sh.rpl == 4 && sh.cpt == 8)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pass<T, 4, 8, MODE>), g, b, 0, s, a);
  else
    return -1;
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_pass(int f64, Shape sh, int mode, const PassArgs& a,
                hipStream_t s) {
  if (f64)
    return mode == kPassData ? pass_shape<double, kPassData>(sh, a, s)
                             : pass_shape<double, kPassRandHaar>(sh, a, s);
  return mode == kPassData ? pass_shape<float, kPassData>(sh, a, s)
                           : pass_shape<float, kPassRandHaar>(sh, a, s);
}

template <typename T>
static int gin_shape(Shape sh, const GinPassArgs& a, hipStream_t s) {
  const dim3 g(sh.nwg), b(kWG);
  if (sh.rpl == 1 && sh.cpt == 1)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gin_pass<T, 1, 1>), g, b, 0, s, a);
  else if (sh.rpl == 4 && sh.cpt == 1)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gin_pass<T, 4, 1>), g, b, 0, s, a);
  else if (sh.rpl == 4 && sh.cpt == 2)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gin_pass<T, 4, 2>), g, b, 0, s, a);
  else if (sh.rpl == 4 && sh.cpt == 4)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gin_pass<T, 4, 4>), g, b, 0, s, a);
  else if (sh.rpl == 4 && sh.cpt == 8)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gin_pass<T, 4, 8>), g, b, 0, s, a);
  else
    return -1;
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_gin_pass(int f64, Shape sh, const GinPassArgs& a, hipStream_t s) {
  return f64 ? gin_shape<double>(sh, a, s) : gin_shape<float>(sh, a, s);
}

int launch_reduce(const double* partials, int pstride, int nwg,
                  const SlotRanges& r, double* out, hipStream_t s) {
  const int total = r.count[0] + r.count[1] + r.count[2];
  if (total <= 0) return 0;
  hipLaunchKernelGGL(k_reduce, dim3(total), dim3(kWG), 0, s, partials,
                     pstride, nwg, r, out);
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

int launch_fill(double* p, double v, int64_t count, hipStream_t s) {
  if (count <= 0) return 0;
  int64_t blocks = (count + kWG - 1) / kWG;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill, dim3((int)blocks), dim3(kWG), 0, s, p, v, count);
  HD_CHECK_LAUNCH();
  return 0;
}

}  // namespace hd
