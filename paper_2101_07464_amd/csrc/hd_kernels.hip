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
// Every panel kernel is one streaming sweep over its rows (RPL rows per lane:
// 4 = one 16-byte load per column for FP32, 1 for small panels to give them
// more workgroups) with all accumulation in FP64:
//   tdot     : w = V' b (column dots), optionally a second right-hand side
//   pass     : out = Delta a - V z (GEMV-N), the new panel column, and the dots
//              of every column with the next query's Philox draw (prefetch)
//   gin_pass : the random side of a Ginibre query (two GEMV-N plus the
//              explicit basis panel)
// Column dots are summed per wave with a barrier-free reduce-scatter into an
// LDS window, per workgroup in fixed order, and across workgroups by k_reduce
// (or k_trial_small for batches) in fixed order, so results are bitwise
// reproducible run to run.  Small one-workgroup FP64 kernels update the WY
// factor T and the reflector scalars.
#include <hip/hip_runtime.h>

#include "hd_device.hpp"
#include "hd_internal.hpp"

namespace hd {

constexpr int kFlush = 256;  // columns per LDS window of the column sums

// Columns per group of the panel sweeps: each lane keeps one partial sum per
// column of the group in registers (wider groups spill to scratch).
constexpr int kCG = 16;

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

// One sweep over columns [0, nc) of a panel, over the rows of this workgroup
// (CPT chunks of kWG * RPL rows starting at blk0):
//   dots (ND = 1 or 2, when `dots`): d0[j] = sum_rows V[r, j] * rhs0[r]
//        -> out0[j], and likewise rhs1 -> out1 (per-workgroup partials);
//   GEMV-N (NZ = 0, 1 or 2): acc_q[r] -= zs_q * sum_j V[r, j] * z_q[j].
template <typename T, int RPL, int CPT, int ND, int NZ>
__device__ __forceinline__ void sweep(
    const T* __restrict__ V, int64_t ld, int nc, int64_t blk0,
    const bool (&cvalid)[CPT], const double (&rhs0)[CPT][RPL],
    const double (&rhs1)[CPT][RPL], bool dots, const double* __restrict__ z0,
    double zs0, const double* __restrict__ z1, double zs1,
    double (&acc0)[CPT][RPL], double (&acc1)[CPT][RPL], double* wacc,
    double* out0, double* out1) {
  constexpr int CG = kCG;
  constexpr int kRows = kWG * RPL;
  constexpr int kGroup = 64 / CG;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll 1
  for (int w0 = 0; w0 < nc; w0 += kFlush) {
    const int wend = min(nc, w0 + kFlush);
#pragma unroll 1
    for (int j0 = w0; j0 < wend; j0 += CG) {
      double p0[CG], p1[ND == 2 ? CG : 1];
      double q0[NZ >= 1 ? CG : 1], q1[NZ == 2 ? CG : 1];
#pragma unroll
      for (int jj = 0; jj < CG; ++jj) {
        const bool ok = j0 + jj < nc;
        p0[jj] = 0.0;
        if constexpr (ND == 2) p1[jj] = 0.0;
        if constexpr (NZ >= 1) q0[jj] = ok ? zs0 * z0[j0 + jj] : 0.0;
        if constexpr (NZ == 2) q1[jj] = ok ? zs1 * z1[j0 + jj] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        if (!cvalid[c]) continue;
        const int64_t r = blk0 + (int64_t)c * kRows + RPL * tid;
#pragma unroll
        for (int jj = 0; jj < CG; ++jj) {
          const int j = min(j0 + jj, nc - 1);
          double v[RPL];
          load_rows<RPL>(V + (int64_t)j * ld + r, v);
#pragma unroll
          for (int e = 0; e < RPL; ++e) {
            if constexpr (NZ >= 1) acc0[c][e] -= v[e] * q0[jj];
            if constexpr (NZ == 2) acc1[c][e] -= v[e] * q1[jj];
            if constexpr (ND >= 1) p0[jj] += v[e] * rhs0[c][e];
            if constexpr (ND == 2) p1[jj] += v[e] * rhs1[c][e];
          }
        }
      }
      if constexpr (ND >= 1) {
        if (dots) {
          const int col = j0 + lane / kGroup;
          const bool owner = (lane % kGroup) == 0 && col < wend;
          const double s0 = wave_reduce_scatter<CG>(p0);
          if (owner) wacc[wave * kFlush + (col - w0)] = s0;
          if constexpr (ND == 2) {
            const double s1 = wave_reduce_scatter<CG>(p1);
            if (owner) wacc[(kWaves + wave) * kFlush + (col - w0)] = s1;
          }
        }
      }
    }
    if (ND >= 1 && dots) {
      __syncthreads();
      for (int jj = tid; jj < wend - w0; jj += kWG) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
          s0 += wacc[w * kFlush + jj];
          if (ND == 2) s1 += wacc[(kWaves + w) * kFlush + jj];
        }
        out0[w0 + jj] = s0;
        if (ND == 2) out1[w0 + jj] = s1;
      }
      __syncthreads();
    }
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
// columns with the stored rows > k of u_k, summed by the data pass: adds the
// pivot row (V[k, j] * u_k[k]), then T[:k, k] = -tau_k T[:k, :k] c.  c is
// updated in place.  Two barriers; every thread of the workgroup calls it.
template <typename T>
__device__ void data_tcol(const PanelDev& D, int k, int tm, double up,
                          double tau, double* c) {
  const T* V = (const T*)D.V;
  for (int j = threadIdx.x; j < k; j += kWG)
    c[j] += (double)V[(int64_t)j * D.ld + k] * up;
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += kWG) {
    double s = 0.0;
    for (int l = j; l < k; ++l) s += D.T[j + (int64_t)l * tm] * c[l];
    D.T[j + (int64_t)k * tm] = -tau * s;
  }
  __syncthreads();
}

// Haar, after the data-side pass of query t (k = t-1 reflectors per panel):
// the data reflector R_t, then L_t = H_t(g_t) from the prefetched dots V'g
// over rows > k and ||g[k+1:]||^2, its T column, s_vec = V' Delta w for
// w = [p[:k]; (nu/||g[k:]||) g[k:]] (the vector L_t R_t p_t of eq. (Qtxt)
// before L_1..L_{t-1}), and z_G = T_G s_vec.
template <typename T>
__device__ void haar_small_body(const HaarSmallArgs& a) {
  __shared__ double sh[6];
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
  for (int j = tid; j < k; j += kWG) {
    const T* colG = VG + (int64_t)j * ldG;
    double hg = 0.0;
    for (int i = 0; i < k; ++i)
      hg += (double)colG[i] * a.G.pi[i + 1] * a.head[i];
    const double gdot = a.G.red[j];
    cG[j] = gdot + (double)colG[k] * upG;
    sv[j] = hg + piGk * cs * (gdot + (double)colG[k] * gk);
  }
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
  if (a.cslot >= 0) data_tcol<T>(a.D, k, tm, sh[4], sh[5], a.D.red + a.cslot);
}

// Ginibre: the data reflector, then the random-side coefficients
// s1 = V_G' Delta_G [0; g] = pi_l (prefetched dots over rows >= l),
// s2 = V_G' Delta_G h (head rows only) + nu s1; z1 = T_G s1, z2 = T_G s2.
template <typename T>
__device__ void gin_small_body(const GinSmallArgs& a) {
  __shared__ double sh[3];
  const int k = a.k, l = a.l, tid = threadIdx.x, tm = a.tmax;
  const T* VG = (const T*)a.G.V;
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
  for (int j = tid; j < l; j += kWG) {
    const T* col = VG + (int64_t)j * ldG;
    double hs = 0.0;
    for (int i = 0; i < l; ++i) hs += (double)col[i] * a.G.pi[i + 1] * a.h[i];
    const double v1 = pil * a.G.red[j];
    s1[j] = v1;
    s2[j] = hs + nu * v1;
  }
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
  if (a.cslot >= 0) data_tcol<T>(a.D, k, tm, sh[1], sh[2], a.D.red + a.cslot);
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
__device__ __forceinline__ void tdot_body(const TdotArgs& a, int blk) {
  constexpr int kRows = kWG * RPL;
  __shared__ double wacc[2 * kWaves * kFlush];
  __shared__ double scr[kWaves];
  const int tid = threadIdx.x;
  const int64_t blk0 = (int64_t)blk * (kRows * CPT);
  double rhs[2][CPT][RPL];
  bool cvalid[CPT];
  double ss = 0.0;
  const PhiloxKey key{a.key.k0, a.key.k1};
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int64_t row0 = blk0 + (int64_t)c * kRows;
    cvalid[c] = row0 < a.ld;
    const int64_t i0 = row0 + RPL * tid;
    if (GEN)
      draw_rows<T, RPL>(key, a.gen_step, i0, a.lo, cvalid[c] ? a.n : 0, true,
                        rhs[0][c]);
#pragma unroll
    for (int e = 0; e < RPL; ++e) {
      const int64_t i = i0 + e;
      const bool in = cvalid[c] && i < a.n;
      if (!GEN)
        rhs[0][c][e] = (in && i > a.lo) ? (double)((const T*)a.b)[i] : 0.0;
      rhs[1][c][e] = (TWO && in) ? (double)((const T*)a.b2)[i] : 0.0;
      ss += rhs[0][c][e] * rhs[0][c][e];
    }
  }
  double* out = a.partials + (int64_t)blk * a.pstride;
  double acc[CPT][RPL];
  sweep<T, RPL, CPT, TWO ? 2 : 1, 0>((const T*)a.V, a.ld, a.ncols, blk0,
                                     cvalid, rhs[0], rhs[1], true, nullptr,
                                     0.0, nullptr, 0.0, acc, acc, wacc, out,
                                     out + a.slot2);
  if (a.ncols2 > 0)
    sweep<T, RPL, CPT, 1, 0>((const T*)a.V2, a.ld, a.ncols2, blk0, cvalid,
                             rhs[0], rhs[1], true, nullptr, 0.0, nullptr, 0.0,
                             acc, acc, wacc, out + a.ncols, nullptr);
  if (a.want_ss) {
    const double s = block_sum(ss, scr);
    if (tid == 0) out[a.extra + kSlotPFSS] = s;
  }
}

// ---------------------------------------------------------------- GEMV-N --

template <typename T, int RPL, int CPT, int MODE>
__device__ __forceinline__ void pass_body(const PassArgs& a, int blk) {
  constexpr int kRows = kWG * RPL;
  __shared__ double wacc[kWaves * kFlush];
  __shared__ double scr[kWaves];
  const int tid = threadIdx.x;
  const int k = a.k;
  const int64_t blk0 = (int64_t)blk * (kRows * CPT);
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
  double* out = a.partials + (int64_t)blk * a.pstride;
  sweep<T, RPL, CPT, 1, 1>(V, a.ld, k, blk0, cvalid, gn, gn, a.pf != 0, a.z,
                           1.0, nullptr, 0.0, acc, acc, wacc, out, nullptr);

  // Epilogue: form the output rows, write the new column k, and the extras.
  double ssq = 0.0, pfnew = 0.0, ysq = 0.0;
  double ur[CPT][RPL];  // stored rows > k of the new column (data mode)
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
      ur[c][e] = 0.0;
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
          ur[c][e] = pd;
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
  if (MODE == kPassData && a.cslot >= 0) {
    // dots of the earlier columns with the new one, for its T column (these
    // rows of V were just read, so they mostly come from L2)
#pragma unroll
    for (int c = 0; c < CPT; ++c)
      if (!cvalid[c]) {
#pragma unroll
        for (int e = 0; e < RPL; ++e) ur[c][e] = 0.0;
      }
    sweep<T, RPL, CPT, 1, 0>(V, a.ld, k, blk0, cvalid, ur, ur, true, nullptr,
                             0.0, nullptr, 0.0, acc, acc, wacc, out + a.cslot,
                             nullptr);
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

template <typename T, int RPL, int CPT>
__device__ __forceinline__ void gin_pass_body(const GinPassArgs& a, int blk) {
  constexpr int kRows = kWG * RPL;
  __shared__ double wacc[kWaves * kFlush];
  const int tid = threadIdx.x;
  const int k = a.k, nb = a.nb;
  const int64_t blk0 = (int64_t)blk * (kRows * CPT);
  T* __restrict__ B = (T*)a.B;
  const PhiloxKey key{a.key.k0, a.key.k1};
  double acc0[CPT][RPL], acc1[CPT][RPL], gn[CPT][RPL];
  bool cvalid[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int64_t row0 = blk0 + (int64_t)c * kRows;
    cvalid[c] = row0 < a.ld;
    draw_rows<T, RPL>(key, a.pf_step, row0 + RPL * tid, a.pf_cut,
                      (a.pf && cvalid[c]) ? a.n : 0, true, gn[c]);
#pragma unroll
    for (int e = 0; e < RPL; ++e) {
      acc0[c][e] = 0.0;
      acc1[c][e] = 0.0;
    }
  }
  double* out = a.partials + (int64_t)blk * a.pstride;
  // reflector panel: acc0 -= V z1 (new basis vector), acc1 -= V z2 (output),
  // and the prefetch dots
  sweep<T, RPL, CPT, 1, 2>((const T*)a.V, a.ld, k, blk0, cvalid, gn, gn,
                           a.pf != 0, a.z1, 1.0, a.z2, 1.0, acc0, acc1, wacc,
                           out, nullptr);
  // explicit basis panel: acc1 += B c
  if (nb > 0)
    sweep<T, RPL, CPT, 0, 1>((const T*)B, a.ld, nb, blk0, cvalid, gn, gn,
                             false, a.c, -1.0, nullptr, 0.0, acc1, acc1, wacc,
                             nullptr, nullptr);
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
      B[(int64_t)nb * a.ld + i] = (T)(sg * gi + acc0[c][e]);
      const double hv = (i < k) ? a.h[i] : 0.0;
      const T ys = (T)(sigma * (acc1[c][e] + sg * (hv + nu * gi)));
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
}

// ---------------------------------------------------- kernel wrappers ----

template <typename T, int RPL, int CPT, bool GEN, bool TWO>
__global__ __launch_bounds__(kWG) void k_tdot(TdotArgs a) {
  tdot_body<T, RPL, CPT, GEN, TWO>(a, blockIdx.x);
}

template <typename T, int RPL, int CPT, int MODE>
__global__ __launch_bounds__(kWG) void k_pass(PassArgs a) {
  pass_body<T, RPL, CPT, MODE>(a, blockIdx.x);
}

template <typename T, int RPL, int CPT>
__global__ __launch_bounds__(kWG) void k_gin_pass(GinPassArgs a) {
  gin_pass_body<T, RPL, CPT>(a, blockIdx.x);
}

// Ring of three trajectory vectors of a batched trial, stride ld: x_t is
// slot (t-1) % 3.
template <typename T>
__device__ __forceinline__ const T* ring_slot(const void* base, int64_t ld,
                                              int slot) {
  return (const T*)base + (int64_t)slot * ld;
}

template <typename T, int RPL, int CPT, bool GEN, bool TWO>
__global__ __launch_bounds__(kWG) void k_tdot_batch(const TdotArgs* A,
                                                    BatchMap bm, StepPatch p) {
  const int trial = bm.blk_trial[blockIdx.x];
  TdotArgs a = A[trial];
  a.ncols = p.k;
  if (GEN) {
    a.gen_step = p.step;
    a.lo = p.k;
    a.want_ss = p.want_ss;
  } else {
    a.b = ring_slot<T>(a.b, a.ld, (int)((p.step - 1) % 3));
    a.b2 = TWO ? (const void*)((const T*)a.V + (int64_t)p.kp * a.ld) : nullptr;
  }
  tdot_body<T, RPL, CPT, GEN, TWO>(a, blockIdx.x - bm.blk_first[trial]);
}

template <typename T, int RPL, int CPT, int MODE>
__global__ __launch_bounds__(kWG) void k_pass_batch(const PassArgs* A,
                                                    BatchMap bm, StepPatch p) {
  const int trial = bm.blk_trial[blockIdx.x];
  PassArgs a = A[trial];
  a.k = p.k;
  a.step = p.step;
  a.pf = p.pf;
  a.pf_step = p.step + 1;
  a.pf_cut = p.k + 1;
  if (MODE == kPassData) a.x = ring_slot<T>(a.x, a.ld, (int)((p.step - 1) % 3));
  if (a.dyn.kind) {
    // dyn.x holds the ring base: x_t, x_{t-1}, x_{t+1} are its slots
    const void* ring = a.dyn.x;
    a.dyn.x = ring_slot<T>(ring, a.ld, (int)((p.step - 1) % 3));
    a.dyn.xprev = ring_slot<T>(ring, a.ld, (int)((p.step + 1) % 3));
    a.dyn.xnext = (void*)ring_slot<T>(ring, a.ld, (int)(p.step % 3));
  }
  pass_body<T, RPL, CPT, MODE>(a, blockIdx.x - bm.blk_first[trial]);
}

// One workgroup per trial: fixed-order sums of the trial's partial rows,
// then the trial's small FP64 step.
template <typename T>
__global__ __launch_bounds__(kWG) void k_trial_small(int op,
                                                     const TrialSums* sums,
                                                     SlotRanges rg,
                                                     const SmallDataArgs* sd,
                                                     const HaarSmallArgs* hs,
                                                     StepPatch p) {
  const int trial = blockIdx.x;
  const TrialSums S = sums[trial];
  reduce_rows(S.partials, S.pstride, 0, S.nwg, rg, S.out);
  if (op == kTrialSmallData) {
    SmallDataArgs a = sd[trial];
    a.kp = p.kp;
    a.k = p.k;
    small_data_body(a);
  } else if (op == kTrialHaarSmall) {
    HaarSmallArgs a = hs[trial];
    a.k = p.k;
    a.step = p.step;
    haar_small_body<T>(a);
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
#define HD_DISPATCH_SHAPE(SH, KERNEL_T, ...)                                 \
  do {                                                                       \
    if ((SH).rpl == 1 && (SH).cpt == 1)                                      \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(KERNEL_T(1, 1)), __VA_ARGS__);      \
    else if ((SH).rpl == 4 && (SH).cpt == 1)                                 \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(KERNEL_T(4, 1)), __VA_ARGS__);      \
    else if ((SH).rpl == 4 && (SH).cpt == 2)                                 \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(KERNEL_T(4, 2)), __VA_ARGS__);      \
    else if ((SH).rpl == 4 && (SH).cpt == 4)                                 \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(KERNEL_T(4, 4)), __VA_ARGS__);      \
    else if ((SH).rpl == 4 && (SH).cpt == 8)                                 \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(KERNEL_T(4, 8)), __VA_ARGS__);      \
    else                                                                     \
      return -1;                                                             \
  } while (0)

template <typename T, bool GEN, bool TWO>
static int tdot_shape(Shape sh, const TdotArgs& a, hipStream_t s) {
#define K_(R, C) k_tdot<T, R, C, GEN, TWO>
  HD_DISPATCH_SHAPE(sh, K_, dim3(sh.nwg), dim3(kWG), 0, s, a);
#undef K_
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

template <typename T, bool GEN, bool TWO>
static int tdot_batch_shape(Shape sh, const TdotArgs* A, BatchMap bm,
                            StepPatch p, hipStream_t s) {
#define K_(R, C) k_tdot_batch<T, R, C, GEN, TWO>
  HD_DISPATCH_SHAPE(sh, K_, dim3(bm.nblk), dim3(kWG), 0, s, A, bm, p);
#undef K_
  HD_CHECK_LAUNCH();
  return 0;
}

template <typename T>
static int tdot_batch_t(Shape sh, const TdotArgs* A, BatchMap bm, StepPatch p,
                        int gen, hipStream_t s) {
  if (gen) return tdot_batch_shape<T, true, false>(sh, A, bm, p, s);
  if (p.kp > 0) return tdot_batch_shape<T, false, true>(sh, A, bm, p, s);
  return tdot_batch_shape<T, false, false>(sh, A, bm, p, s);
}

int launch_tdot_batch(int f64, Shape sh, const TdotArgs* args, BatchMap bm,
                      StepPatch p, int gen, hipStream_t s) {
  if (bm.nblk <= 0) return 0;
  return f64 ? tdot_batch_t<double>(sh, args, bm, p, gen, s)
             : tdot_batch_t<float>(sh, args, bm, p, gen, s);
}

template <typename T, int MODE>
static int pass_shape(Shape sh, const PassArgs& a, hipStream_t s) {
#define K_(R, C) k_pass<T, R, C, MODE>
  HD_DISPATCH_SHAPE(sh, K_, dim3(sh.nwg), dim3(kWG), 0, s, a);
#undef K_
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

template <typename T, int MODE>
static int pass_batch_shape(Shape sh, const PassArgs* A, BatchMap bm,
                            StepPatch p, hipStream_t s) {
#define K_(R, C) k_pass_batch<T, R, C, MODE>
  HD_DISPATCH_SHAPE(sh, K_, dim3(bm.nblk), dim3(kWG), 0, s, A, bm, p);
#undef K_
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_pass_batch(int f64, Shape sh, int mode, const PassArgs* args,
                      BatchMap bm, StepPatch p, hipStream_t s) {
  if (bm.nblk <= 0) return 0;
  if (f64)
    return mode == kPassData
               ? pass_batch_shape<double, kPassData>(sh, args, bm, p, s)
               : pass_batch_shape<double, kPassRandHaar>(sh, args, bm, p, s);
  return mode == kPassData
             ? pass_batch_shape<float, kPassData>(sh, args, bm, p, s)
             : pass_batch_shape<float, kPassRandHaar>(sh, args, bm, p, s);
}

template <typename T>
static int gin_shape(Shape sh, const GinPassArgs& a, hipStream_t s) {
#define K_(R, C) k_gin_pass<T, R, C>
  HD_DISPATCH_SHAPE(sh, K_, dim3(sh.nwg), dim3(kWG), 0, s, a);
#undef K_
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_gin_pass(int f64, Shape sh, const GinPassArgs& a, hipStream_t s) {
  return f64 ? gin_shape<double>(sh, a, s) : gin_shape<float>(sh, a, s);
}

int launch_trial_small(int f64, int op, int ntrials, const TrialSums* sums,
                       SlotRanges rg, const SmallDataArgs* sd,
                       const HaarSmallArgs* hs, StepPatch p, hipStream_t s) {
  if (ntrials <= 0) return 0;
  if (f64)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trial_small<double>), dim3(ntrials),
                       dim3(kWG), 0, s, op, sums, rg, sd, hs, p);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trial_small<float>), dim3(ntrials),
                       dim3(kWG), 0, s, op, sums, rg, sd, hs, p);
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_reduce(const ReduceJob& a, const ReduceJob& b, hipStream_t s) {
  const int na = a.rg.count[0] + a.rg.count[1] + a.rg.count[2];
  const int nb = b.rg.count[0] + b.rg.count[1] + b.rg.count[2];
  if (na + nb <= 0) return 0;
  hipLaunchKernelGGL(k_reduce, dim3(na + nb), dim3(kWG), 0, s, a, b);
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
