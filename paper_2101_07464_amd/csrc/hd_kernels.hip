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
// Hot kernels stream the panel once per pass with 16-byte loads, four rows
// per lane, and keep every accumulation in FP64:
//   k_tdot  : w = V' b (per-workgroup partials; column sums by a wave
//             reduce-scatter, then LDS across the four waves)
//   k_pass  : out = Delta a - V z (GEMV-N), writes the new panel column and
//             the fused dot products with the next query's Philox draw.
// Cross-workgroup sums go through k_reduce in a fixed order, so results are
// bitwise reproducible run to run.  Small FP64 kernels (one workgroup)
// update the triangular factor T and the Gram matrix of each panel.
#include <hip/hip_runtime.h>

#include "hd_device.hpp"
#include "hd_internal.hpp"

namespace hd {

constexpr int kCG = 16;  // columns per group in the panel loops

// ------------------------------------------------------------------ TDOT --

template <typename T, int CPT, bool GEN, bool TWO>
__global__ __launch_bounds__(kWG) void k_tdot(TdotArgs a) {
  __shared__ double lds[kWaves * kCG];
  __shared__ double scr[kWaves];
  const int tid = threadIdx.x;
  const int64_t blk0 = (int64_t)blockIdx.x * (kChunk * CPT);
  double b[CPT][4];
  double b2[CPT][4];
  bool cvalid[CPT];
  double ss = 0.0;
  const PhiloxKey key{a.key.k0, a.key.k1};
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int64_t row0 = blk0 + (int64_t)c * kChunk;
    cvalid[c] = row0 < a.ld;
    const int64_t i0 = row0 + 4 * tid;
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    if (GEN) {
      if (cvalid[c] && i0 < a.n && i0 + 3 > a.lo)
        normals4(key, a.gen_step, 0u, (uint64_t)(i0 >> 2), g);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = i0 + e;
      double v = 0.0, v2 = 0.0;
      if (cvalid[c] && i > a.lo && i < a.n) {
        v = GEN ? (double)(T)g[e] : (double)((const T*)a.b)[i];
      }
      if (TWO && cvalid[c] && i < a.n) v2 = (double)((const T*)a.b2)[i];
      b[c][e] = v;
      b2[c][e] = v2;
      ss += v * v;
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
        const int64_t r = blk0 + (int64_t)c * kChunk + 4 * tid;
#pragma unroll
        for (int jj = 0; jj < kCG; ++jj) {
          const int j = min(j0 + jj, nc - 1);
          double v[4];
          load4(V + (int64_t)j * a.ld + r, v);
          acc[jj] += v[0] * b[c][0] + v[1] * b[c][1] + v[2] * b[c][2] +
                     v[3] * b[c][3];
          if (TWO && seg == 0)
            acc2[jj] += v[0] * b2[c][0] + v[1] * b2[c][1] + v[2] * b2[c][2] +
                        v[3] * b2[c][3];
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
}

// ---------------------------------------------------------------- GEMV-N --

template <typename T, int CPT, int MODE>
__global__ __launch_bounds__(kWG) void k_pass(PassArgs a) {
  __shared__ double lds[kWaves * kCG];
  __shared__ double scr[kWaves];
  const int tid = threadIdx.x;
  const int k = a.k;
  const int64_t blk0 = (int64_t)blockIdx.x * (kChunk * CPT);
  T* __restrict__ V = (T*)a.V;
  const PhiloxKey key{a.key.k0, a.key.k1};
  double acc[CPT][4];
  double gn[CPT][4];
  bool cvalid[CPT];
  double pfss = 0.0;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int64_t row0 = blk0 + (int64_t)c * kChunk;
    cvalid[c] = row0 < a.ld;
    const int64_t i0 = row0 + 4 * tid;
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    if (a.pf && cvalid[c] && i0 < a.n && i0 + 3 > a.pf_cut)
      normals4(key, a.pf_step, 0u, (uint64_t)(i0 >> 2), g);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = i0 + e;
      acc[c][e] = 0.0;
      double v = 0.0;
      if (a.pf && cvalid[c] && i > a.pf_cut && i < a.n) v = (double)(T)g[e];
      gn[c][e] = v;
      pfss += v * v;
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
      const int64_t r = blk0 + (int64_t)c * kChunk + 4 * tid;
#pragma unroll
      for (int jj = 0; jj < kCG; ++jj) {
        const int j = min(j0 + jj, k - 1);
        double v[4];
        load4(V + (int64_t)j * a.ld + r, v);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
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
    const int64_t i0 = blk0 + (int64_t)c * kChunk + 4 * tid;
    double gt[4] = {0.0, 0.0, 0.0, 0.0};
    if (MODE == kPassRandHaar && i0 < a.n && i0 + 3 >= k)
      normals4(key, a.step, 0u, (uint64_t)(i0 >> 2), gt);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
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
}

// ---------------------------------------------------------------- reduce --

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
  for (int w = threadIdx.x; w < nwg; w += kWG) s += P[(int64_t)w * pstride + slot];
  s = block_sum(s, scr);
  if (threadIdx.x == 0) out[slot] = s;
}

// Column kp of T from the dots c = V[:, :kp]' u_kp (compact-WY recurrence of
// Schreiber and Van Loan), then z = T' w for the leading k x k block.
__global__ __launch_bounds__(kWG) void k_small_data(SmallDataArgs a) {
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

// --------------------------------------------------- Haar scalar updates --
//
// After the data-side pass of query t (k = t-1 reflectors stored per panel):
//  data side  : nu = ||p[k:]||, s = sign(p_k), stored pivot u_k = p_k + s nu,
//               tau = 2/||u||^2 (from the stored entries).  Its T column is
//               completed later from direct dots V'u_k (k_small_data).
//  random side: L_t = H_t(g_t) from the prefetched dots V'g over rows > k and
//               ||g[k+1:]||^2; its T column; s_vec = V' Delta w for
//               w = [p[:k]; (nu/||g[k:]||) g[k:]], the vector L_t R_t p_t of
//               eq. (Qtxt) before L_1..L_{t-1}; and z_G = T_G s_vec.
template <typename T>
__global__ __launch_bounds__(kWG) void k_haar_small(HaarSmallArgs a) {
  __shared__ double sh[8];
  const int k = a.k, tid = threadIdx.x, tm = a.tmax;
  T* VD = (T*)a.D.V;
  T* VG = (T*)a.G.V;
  const int64_t ldD = a.D.ld, ldG = a.G.ld;
  double* cG = a.zG + tm;
  double* sv = a.zG + 2 * tm;
  if (tid == 0) {
    const double ss = a.D.red[a.extra + kSlotSS];
    const double pk = *a.pivot;
    const double nu = sqrt(ss + pk * pk);
    double s = 1.0, tau = 0.0, up = 0.0;
    if (nu > 0.0) {
      s = pk >= 0.0 ? 1.0 : -1.0;
      up = (double)(T)(pk + s * nu);
      tau = 2.0 / (ss + up * up);
    }
    if (!isfinite(nu) || !isfinite(tau)) a.flag[0] = 1;
    VD[(int64_t)k * ldD + k] = (T)up;
    a.D.tau[k] = tau;
    a.D.nu[k] = nu;
    a.D.piv[k] = pk;
    a.D.sgn[k] = s;
    // an identity reflector (nu = 0) contributes no sign
    a.D.pi[k + 1] = nu > 0.0 ? a.D.pi[k] * (-s) : a.D.pi[k];
    a.D.T[k + (int64_t)k * tm] = tau;

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
}

// ------------------------------------------------- Ginibre random side --

template <typename T, int CPT>
__global__ __launch_bounds__(kWG) void k_gin_pass(GinPassArgs a) {
  __shared__ double lds[kWaves * kCG];
  const int tid = threadIdx.x;
  const int k = a.k, nb = a.nb;
  const int64_t blk0 = (int64_t)blockIdx.x * (kChunk * CPT);
  const T* __restrict__ V = (const T*)a.V;
  T* __restrict__ B = (T*)a.B;
  const PhiloxKey key{a.key.k0, a.key.k1};
  double acc1[CPT][4], acc2[CPT][4], gn[CPT][4];
  bool cvalid[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int64_t row0 = blk0 + (int64_t)c * kChunk;
    cvalid[c] = row0 < a.ld;
    const int64_t i0 = row0 + 4 * tid;
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    if (a.pf && cvalid[c] && i0 < a.n && i0 + 3 > a.pf_cut)
      normals4(key, a.pf_step, 0u, (uint64_t)(i0 >> 2), g);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = i0 + e;
      acc1[c][e] = 0.0;
      acc2[c][e] = 0.0;
      gn[c][e] = (a.pf && cvalid[c] && i > a.pf_cut && i < a.n)
                     ? (double)(T)g[e]
                     : 0.0;
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
      const int64_t r = blk0 + (int64_t)c * kChunk + 4 * tid;
#pragma unroll
      for (int jj = 0; jj < kCG; ++jj) {
        const int j = min(j0 + jj, k - 1);
        double v[4];
        load4(V + (int64_t)j * a.ld + r, v);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
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
      const int64_t r = blk0 + (int64_t)c * kChunk + 4 * tid;
#pragma unroll
      for (int jj = 0; jj < kCG; ++jj) {
        const int j = min(j0 + jj, nb - 1);
        double v[4];
        load4(B + (int64_t)j * a.ld + r, v);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc2[c][e] += v[e] * cv[jj];
      }
    }
  }
  const double nu = a.scal[0], sigma = a.scal[1];
  const double pik = a.pi[k];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    if (!cvalid[c]) continue;
    const int64_t i0 = blk0 + (int64_t)c * kChunk + 4 * tid;
    double gt[4] = {0.0, 0.0, 0.0, 0.0};
    if (i0 < a.n && i0 + 3 >= k)
      normals4(key, a.step, 0u, (uint64_t)(i0 >> 2), gt);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = i0 + e;
      if (i >= a.n) continue;
      const double sg = (i < k) ? a.pi[i + 1] : pik;
      const double gi = (i >= k) ? gt[e] : 0.0;
      B[(int64_t)nb * a.ld + i] = (T)(sg * gi + acc1[c][e]);
      const double hv = (i < k) ? a.h[i] : 0.0;
      ((T*)a.y)[i] = (T)(sigma * (acc2[c][e] + sg * (hv + nu * gi)));
    }
  }
}

// Data-side scalars (as for Haar) and the random-side coefficients of a
// Ginibre query: s1 = V_G' Delta_G [0; g] = pi_l * (prefetched dots),
// s2 = V_G' Delta_G h (head rows only) + nu s1; z1 = T_G s1, z2 = T_G s2.
template <typename T>
__global__ __launch_bounds__(kWG) void k_gin_small(GinSmallArgs a) {
  __shared__ double sh[2];
  const int k = a.k, l = a.l, tid = threadIdx.x, tm = a.tmax;
  T* VD = (T*)a.D.V;
  const T* VG = (const T*)a.G.V;
  const int64_t ldD = a.D.ld, ldG = a.G.ld;
  double* s1 = a.z1 + tm;
  double* s2 = a.z1 + 2 * tm;
  if (tid == 0) {
    const double ss = a.D.red[a.D_extra + kSlotSS];
    const double pk = *a.pivot;
    const double nu = sqrt(ss + pk * pk);
    double s = 1.0, tau = 0.0, up = 0.0;
    if (nu > 0.0) {
      s = pk >= 0.0 ? 1.0 : -1.0;
      up = (double)(T)(pk + s * nu);
      tau = 2.0 / (ss + up * up);
    }
    if (!isfinite(nu) || !isfinite(tau)) a.flag[0] = 1;
    VD[(int64_t)k * ldD + k] = (T)up;
    a.D.tau[k] = tau;
    a.D.nu[k] = nu;
    a.D.piv[k] = pk;
    a.D.sgn[k] = s;
    a.D.pi[k + 1] = nu > 0.0 ? a.D.pi[k] * (-s) : a.D.pi[k];
    a.D.T[k + (int64_t)k * tm] = tau;
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
}

// ------------------------------------------------------------- dynamics --

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

#define HD_CHECK_LAUNCH()                                    \
  do {                                                       \
    hipError_t e_ = hipGetLastError();                       \
    if (e_ != hipSuccess) return (int)e_;                    \
  } while (0)

template <typename T, bool GEN, bool TWO>
static int tdot_cpt(int cpt, const TdotArgs& a, int nwg, hipStream_t s) {
  switch (cpt) {
    case 1: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_tdot<T, 1, GEN, TWO>), dim3(nwg), dim3(kWG), 0, s, a); break;
    case 2: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_tdot<T, 2, GEN, TWO>), dim3(nwg), dim3(kWG), 0, s, a); break;
    case 4: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_tdot<T, 4, GEN, TWO>), dim3(nwg), dim3(kWG), 0, s, a); break;
    case 8: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_tdot<T, 8, GEN, TWO>), dim3(nwg), dim3(kWG), 0, s, a); break;
    default: return -1;
  }
  HD_CHECK_LAUNCH();
  return 0;
}

template <typename T>
static int tdot_t(int cpt, const TdotArgs& a, int nwg, hipStream_t s) {
  if (a.gen) return tdot_cpt<T, true, false>(cpt, a, nwg, s);
  if (a.b2) return tdot_cpt<T, false, true>(cpt, a, nwg, s);
  return tdot_cpt<T, false, false>(cpt, a, nwg, s);
}

int launch_tdot(int f64, int cpt, const TdotArgs& a, int nwg, hipStream_t s) {
  return f64 ? tdot_t<double>(cpt, a, nwg, s) : tdot_t<float>(cpt, a, nwg, s);
}

template <typename T, int MODE>
static int pass_cpt(int cpt, const PassArgs& a, int nwg, hipStream_t s) {
  switch (cpt) {
    case 1: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pass<T, 1, MODE>), dim3(nwg), dim3(kWG), 0, s, a); break;
    case 2: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pass<T, 2, MODE>), dim3(nwg), dim3(kWG), 0, s, a); break;
    case 4: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pass<T, 4, MODE>), dim3(nwg), dim3(kWG), 0, s, a); break;
    case 8: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pass<T, 8, MODE>), dim3(nwg), dim3(kWG), 0, s, a); break;
    default: return -1;
  }
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_pass(int f64, int cpt, int mode, const PassArgs& a, int nwg,
                hipStream_t s) {
  if (f64)
    return mode == kPassData ? pass_cpt<double, kPassData>(cpt, a, nwg, s)
                             : pass_cpt<double, kPassRandHaar>(cpt, a, nwg, s);
  return mode == kPassData ? pass_cpt<float, kPassData>(cpt, a, nwg, s)
                           : pass_cpt<float, kPassRandHaar>(cpt, a, nwg, s);
}

int launch_reduce(const double* partials, int pstride, int nwg,
                  const SlotRanges& r, double* out, hipStream_t s) {
  const int total = r.count[0] + r.count[1] + r.count[2];
  if (total <= 0) return 0;
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_reduce), dim3(total), dim3(kWG), 0, s, partials, pstride, nwg, r, out);
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_small_data(const SmallDataArgs& a, hipStream_t s) {
  if (a.kp <= 0 && (!a.w || a.k <= 0)) return 0;
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_small_data), dim3(1), dim3(kWG), 0, s, a);
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_haar_small(int f64, const HaarSmallArgs& a, hipStream_t s) {
  if (f64)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_haar_small<double>), dim3(1), dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_haar_small<float>), dim3(1), dim3(kWG), 0, s, a);
  HD_CHECK_LAUNCH();
  return 0;
}

template <typename T>
static int gin_pass_cpt(int cpt, const GinPassArgs& a, int nwg,
                        hipStream_t s) {
  switch (cpt) {
    case 1: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gin_pass<T, 1>), dim3(nwg), dim3(kWG), 0, s, a); break;
    case 2: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gin_pass<T, 2>), dim3(nwg), dim3(kWG), 0, s, a); break;
    case 4: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gin_pass<T, 4>), dim3(nwg), dim3(kWG), 0, s, a); break;
    case 8: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gin_pass<T, 8>), dim3(nwg), dim3(kWG), 0, s, a); break;
    default: return -1;
  }
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_gin_pass(int f64, int cpt, const GinPassArgs& a, int nwg,
                    hipStream_t s) {
  return f64 ? gin_pass_cpt<double>(cpt, a, nwg, s)
             : gin_pass_cpt<float>(cpt, a, nwg, s);
}

int launch_gin_small(int f64, const GinSmallArgs& a, hipStream_t s) {
  if (f64)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gin_small<double>), dim3(1), dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gin_small<float>), dim3(1), dim3(kWG), 0, s, a);
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_dyn(int f64, const DynArgs& a, hipStream_t s) {
  int64_t blocks = (a.n + kWG - 1) / kWG;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  if (f64)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_dyn<double>), dim3((int)blocks), dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_dyn<float>), dim3((int)blocks), dim3(kWG), 0, s, a);
  HD_CHECK_LAUNCH();
  return 0;
}

int launch_fill(double* p, double v, int64_t count, hipStream_t s) {
  if (count <= 0) return 0;
  int64_t blocks = (count + kWG - 1) / kWG;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fill), dim3((int)blocks), dim3(kWG), 0, s, p, v, count);
  HD_CHECK_LAUNCH();
  return 0;
}

}  // namespace hd
