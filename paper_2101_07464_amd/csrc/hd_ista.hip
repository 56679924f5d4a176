// hd_ista.hip -- C-ABI runtime of batches of unrolled-ISTA trials on
// Gaussian matrices of one shape m x n (Sec. 2.1, eq. (ista), on Algorithm 1),
// run in lockstep.  All arithmetic runs in the kernels of hd_kernels.hip;
// this file lays out every trial's state in one device arena and orders the
// launches of each query index.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "hd.h"
#include "hd_internal.hpp"

using namespace hd;

struct hd_ista_ctx {
  int f64;
  int es;
  hipStream_t stream;
  int count;
  int L;
  int64_t dim[2];  // n (side R), m (side L)
  int nwg[2];      // workgroups of 256 rows per side
  IstaTrialDev* dev = nullptr;
  char* arena = nullptr;
  CopyJob* jobs = nullptr;  // pi[0] = 1 on both sides and sigma, per trial
  double* consts = nullptr;
  int* flag = nullptr;
  std::vector<void*> allocs;
};

namespace {

thread_local char i_err[256];

int ifail(hipError_t e) {
  std::snprintf(i_err, sizeof(i_err), "%s", hipGetErrorString(e));
  return HD_ERR_HIP;
}

#define IHIP(call)                            \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) return ifail(e_);   \
  } while (0)

#define ILCHK(call)                                           \
  do {                                                        \
    int e_ = (call);                                          \
    if (e_ != 0) return ifail((hipError_t)(e_ > 0 ? e_ : 1)); \
  } while (0)

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

void release(hd_ista_ctx* b) {
  (void)hipStreamSynchronize(b->stream);
  for (void* p : b->allocs) (void)hipFree(p);
  b->allocs.clear();
}

template <typename P>
int ialloc(hd_ista_ctx* b, P** out, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes ? bytes : 8) != hipSuccess) {
    (void)hipGetLastError();
    return HD_ERR_NOMEM;
  }
  b->allocs.push_back(p);
  if (hipMemsetAsync(p, 0, bytes ? bytes : 8, b->stream) != hipSuccess)
    return ifail(hipGetLastError());
  *out = (P*)p;
  return HD_OK;
}

// Offsets of one trial's buffers inside its block of the arena.
struct Lay {
  size_t V[2], B[2], T[2], tau[2], nu[2], piv[2], sgn[2], pi[2], red[2];
  size_t part, w, zD, zG, z2, head, scal, gscal, yobs, res, U, V2, Yq;
  size_t end;
};

Lay layout(const int64_t* ld, int L, int es, int pstride, int maxwg,
           int64_t n, int64_t m) {
  Lay y;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = up256(o + bytes);
    return at;
  };
  const int tm = L + 1;
  // side R gets a reflector per Q-query (L + 1 of them) and keeps the v's
  // of the L Q'-queries; side L the reverse
  const int cv[2] = {L + 1, L}, cb[2] = {L, L + 1};
  for (int s = 0; s < 2; ++s) {
    y.V[s] = take((size_t)es * ld[s] * cv[s]);
    y.B[s] = take((size_t)es * ld[s] * cb[s]);
    y.T[s] = take(sizeof(double) * (size_t)tm * tm);
    y.tau[s] = take(sizeof(double) * tm);
    y.nu[s] = take(sizeof(double) * tm);
    y.piv[s] = take(sizeof(double) * tm);
    y.sgn[s] = take(sizeof(double) * tm);
    y.pi[s] = take(sizeof(double) * (tm + 1));
    y.red[s] = take(sizeof(double) * pstride);
  }
  y.part = take(sizeof(double) * (size_t)maxwg * pstride);
  y.w = take(sizeof(double) * pstride);
  y.zD = take(sizeof(double) * tm);
  y.zG = take(sizeof(double) * 3 * (size_t)tm);
  y.z2 = take(sizeof(double) * tm);
  y.head = take(sizeof(double) * tm);
  y.scal = take(sizeof(double) * 8);
  y.gscal = take(sizeof(double) * 8);
  y.yobs = take((size_t)es * m);
  y.res = take((size_t)es * m);
  y.Yq = take((size_t)es * m);
  y.U = take((size_t)es * n);
  y.V2 = take((size_t)es * n);
  y.end = o;
  return y;
}

}  // namespace

extern "C" {

int hd_ista_init(int32_t storage, int64_t m, int64_t n, int32_t L,
                 int32_t count, uint32_t seed, uint32_t trial0, double sigma,
                 void* stream, hd_ista* out) {
  if (!out) return HD_ERR_INVALID;
  *out = nullptr;
  if (storage != HD_F32 && storage != HD_F64) return HD_ERR_INVALID;
  if (m < 1 || n < 1 || L < 1 || count < 1) return HD_ERR_INVALID;
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return HD_ERR_INVALID;
  // Algorithm 1 needs r <= n (L + 1 Q-queries) and l <= m (L Q'-queries)
  if ((int64_t)L + 1 > n || (int64_t)L > m) return HD_ERR_INVALID;
  if (n > ((int64_t)1 << 31) || m > ((int64_t)1 << 31)) return HD_ERR_INVALID;
  hd_ista_ctx* b = new (std::nothrow) hd_ista_ctx();
  if (!b) return HD_ERR_NOMEM;
  b->f64 = storage == HD_F64;
  b->es = b->f64 ? 8 : 4;
  b->stream = (hipStream_t)stream;
  b->count = count;
  b->L = L;
  b->dim[0] = n;
  b->dim[1] = m;
  int64_t ld[2];
  for (int s = 0; s < 2; ++s) {
    ld[s] = (b->dim[s] + 255) / 256 * 256;
    b->nwg[s] = (int)(ld[s] / 256);
  }
  const int tm = L + 1, Q = 2 * L + 1;
  const int slot2 = Q + 1, extra = slot2 + tm + 1;
  const int pstride = extra + kNumExtra;
  const int maxwg = b->nwg[0] > b->nwg[1] ? b->nwg[0] : b->nwg[1];
  const Lay lay = layout(ld, L, b->es, pstride, maxwg, n, m);
  const size_t per = lay.end;
  if ((double)per * count > 2.5e11) {
    delete b;
    return HD_ERR_NOMEM;
  }
  int rc = HD_OK;
#define IALLOC(ptr, bytes)           \
  do {                               \
    rc = ialloc(b, &(ptr), (bytes)); \
    if (rc != HD_OK) {               \
      release(b);                    \
      delete b;                      \
      return rc;                     \
    }                                \
  } while (0)
  IALLOC(b->arena, per * (size_t)count);
  IALLOC(b->dev, sizeof(IstaTrialDev) * (size_t)count);
  IALLOC(b->jobs, sizeof(CopyJob) * 3 * (size_t)count);
  IALLOC(b->consts, sizeof(double) * 4);
  IALLOC(b->flag, sizeof(int) * 4);
#undef IALLOC
  auto fail = [&](int r) {
    release(b);
    delete b;
    return r;
  };
  // per-trial arguments; pi[0] = 1 on both sides and sigma come from copies
  // of two constants
  const double cst[2] = {1.0, sigma};
  std::vector<IstaTrialDev> host((size_t)count);
  std::vector<CopyJob> jobs(3 * (size_t)count);
  for (int i = 0; i < count; ++i) {
    char* A = b->arena + per * (size_t)i;
    PanelDev P[2];
    for (int s = 0; s < 2; ++s) {
      P[s].V = A + lay.V[s];
      P[s].ld = ld[s];
      P[s].T = (double*)(A + lay.T[s]);
      P[s].tau = (double*)(A + lay.tau[s]);
      P[s].nu = (double*)(A + lay.nu[s]);
      P[s].piv = (double*)(A + lay.piv[s]);
      P[s].sgn = (double*)(A + lay.sgn[s]);
      P[s].pi = (double*)(A + lay.pi[s]);
      P[s].red = (double*)(A + lay.red[s]);
    }
    const Key key{seed, trial0 + (uint32_t)i};
    double* part = (double*)(A + lay.part);
    double* w = (double*)(A + lay.w);
    double* zD = (double*)(A + lay.zD);
    double* zG = (double*)(A + lay.zG);
    double* z2 = (double*)(A + lay.z2);
    double* head = (double*)(A + lay.head);
    double* scal = (double*)(A + lay.scal);
    double* gscal = (double*)(A + lay.gscal);
    IstaTrialDev d;
    std::memset(&d, 0, sizeof(d));
    for (int s = 0; s < 2; ++s) {
      IstaSide& S = d.s[s];
      void* Bs = A + lay.B[s];
      S.nwg = b->nwg[s];
      S.td.V = P[s].V;
      S.td.ld = ld[s];
      S.td.V2 = Bs;
      S.td.slot2 = slot2;
      S.td.key = key;
      S.td.lo = -1;
      S.td.n = b->dim[s];
      S.td.partials = part;
      S.td.pstride = pstride;
      S.td.extra = extra;
      S.sd.T = P[s].T;
      S.sd.tau = P[s].tau;
      S.sd.tmax = tm;
      S.sd.kp = -1;
      S.sd.w = w;
      S.sd.z = zD;
      S.pd.V = P[s].V;
      S.pd.ld = ld[s];
      S.pd.z = zD;
      S.pd.pi = P[s].pi;
      S.pd.n = b->dim[s];
      S.pd.head = head;
      S.pd.pivot = scal;
      S.pd.cslot = slot2;
      S.pd.key = key;
      S.pd.partials = part;
      S.pd.pstride = pstride;
      S.pd.extra = extra;
      S.gs.D = P[s];
      S.gs.G = P[1 - s];
      S.gs.tmax = tm;
      S.gs.h = w;
      S.gs.z1 = zG;
      S.gs.z2 = z2;
      S.gs.pivot = scal;
      S.gs.scal = gscal;
      S.gs.D_extra = extra;
      S.gs.cslot = -1;
      S.gs.flag = b->flag;
      S.gp.V = P[s].V;
      S.gp.ld = ld[s];
      S.gp.z1 = zG;
      S.gp.z2 = z2;
      S.gp.pi = P[s].pi;
      S.gp.B = Bs;
      S.gp.c = head;
      S.gp.h = w;
      S.gp.scal = gscal;
      S.gp.n = b->dim[s];
      S.gp.key = key;
      S.gp.partials = part;
      S.gp.pstride = pstride;
      S.gp.extra = extra;
    }
    d.yobs = A + lay.yobs;
    d.res = A + lay.res;
    d.Yq = A + lay.Yq;
    d.U = A + lay.U;
    d.V = A + lay.V2;
    host[i] = d;
    jobs[3 * (size_t)i] = CopyJob{b->consts, P[0].pi, 2};
    jobs[3 * (size_t)i + 1] = CopyJob{b->consts, P[1].pi, 2};
    jobs[3 * (size_t)i + 2] = CopyJob{b->consts + 1, gscal + 1, 2};
  }
  if (hipStreamSynchronize(b->stream) != hipSuccess)
    return fail(ifail(hipGetLastError()));
  hipError_t e = hipMemcpy(b->consts, cst, sizeof(cst), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->dev, host.data(), sizeof(IstaTrialDev) * host.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->jobs, jobs.data(), sizeof(CopyJob) * jobs.size(),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(ifail(e));
  if (launch_copy_jobs(b->jobs, 3 * count, b->stream) != 0 ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return fail(ifail(hipGetLastError()));
  *out = b;
  return HD_OK;
}

int hd_ista_run(hd_ista b, const float* a, const float* theta,
                const void* xstar, const void* noise, void* X) {
  if (!b || !a || !theta || !xstar || !noise || !X) return HD_ERR_INVALID;
  const int L = b->L, C = b->count, f64 = b->f64;
  // every run starts from fresh matrices: the reflector counts restart
  // and every array a query reads is rewritten before it is read
  IstaStep st;
  std::memset(&st, 0, sizeof(st));
  st.L = L;
  st.xstar = xstar;
  st.noise = noise;
  st.X = X;
  int kR = 0, kL = 0;
  for (int q = 0; q <= 2 * L; ++q) {
    const int ds = (q == 0 || q % 2 == 1) ? 0 : 1;
    const int gs = 1 - ds;
    st.q = q;
    st.kR = kR;
    st.kL = kL;
    st.step = (uint32_t)(q + 1);
    st.last = q == 2 * L;
    if (ds == 1) {
      st.a = a[q / 2 - 1];
      st.theta = theta[q / 2 - 1];
    }
    if (kR + kL > 0) {
      ILCHK(launch_ista_tdot(f64, ds, C * b->nwg[ds], b->dev, st, b->stream));
      ILCHK(launch_ista_small(f64, 0, ds, C, b->dev, st, b->stream));
    }
    ILCHK(launch_ista_data(f64, ds, C * b->nwg[ds], b->dev, st, b->stream));
    ILCHK(launch_ista_small(f64, 1, ds, C, b->dev, st, b->stream));
    ILCHK(launch_ista_rand(f64, gs, C * b->nwg[gs], b->dev, st, b->stream));
    if (ds == 0)
      ++kR;
    else
      ++kL;
  }
  return HD_OK;
}

int hd_ista_status(hd_ista b) {
  if (!b) return HD_ERR_INVALID;
  IHIP(hipStreamSynchronize(b->stream));
  int flag = 0;
  IHIP(hipMemcpy(&flag, b->flag, sizeof(int), hipMemcpyDeviceToHost));
  return flag ? HD_ERR_NONFINITE : HD_OK;
}

int hd_ista_set_stream(hd_ista b, void* stream) {
  if (!b) return HD_ERR_INVALID;
  b->stream = (hipStream_t)stream;
  return HD_OK;
}

int hd_ista_free(hd_ista b) {
  if (!b) return HD_OK;
  release(b);
  delete b;
  return HD_OK;
}

}  // extern "C"
