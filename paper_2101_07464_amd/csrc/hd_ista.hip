// hd_ista.hip -- C-ABI runtime of batches of unrolled-ISTA trials on
// Gaussian matrices of one shape m x n (Sec. 2.1, eq. (ista), on Algorithm 1),
// run in lockstep, and of their reverse pass (the gradient with respect to
// the per-layer step and threshold, on the same lazy matrices).  All
// arithmetic runs in the kernels of hd_kernels.hip; this file lays out every
// trial's state in one device arena and orders the launches of each query
// index.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
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
  int grad;        // room and buffers for the reverse pass
  int ran;         // a forward run has ended and no reverse pass followed
  int kR, kL;      // reflector counts after the last query
  void* Urec = nullptr;
  void* Vrec = nullptr;
  double* adj_part = nullptr;
  int nwg_adj;     // 256-row workgroups over n (reverse-pass reductions)
  int64_t dim[2];  // n (side R), m (side L)
  int cpt[2];      // 256-row chunks per workgroup, per side
  int nwg[2];      // workgroups per trial and side
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

// Chunks of 256 rows per workgroup for a side of `dim` rows: the largest of
// 4, 2, 1 whose padding stays within 1/16 of the one-chunk rows (a whole
// trial side then takes few workgroups, each with longer sweeps and fewer
// reductions per row).  HD_ISTA_CPT = 1, 2 or 4 overrides it.
int ista_cpt(int64_t dim) {
  const char* e = std::getenv("HD_ISTA_CPT");
  if (e) {
    const int v = std::atoi(e);
    if (v == 1 || v == 2 || v == 4) return v;
  }
  const int64_t base = (dim + 255) / 256 * 256;
  for (int c = 4; c > 1; c /= 2) {
    const int64_t q = 256 * (int64_t)c;
    if ((dim + q - 1) / q * q * 16 <= base * 17) return c;
  }
  return 1;
}

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
  size_t part, w, zD, zG, z2, head, scal, gscal, yobs, res, U, V2, gbar;
  size_t end;
};

// Panel columns per side: side R gets a reflector per Q-query and keeps the
// basis vectors v of the Q'-queries, side L the reverse.  The forward pass
// is L + 1 Q-queries and L Q'-queries; the reverse pass adds L - 1 of each.
void capacities(int L, int grad, int cv[2], int cb[2]) {
  cv[0] = grad ? 2 * L : L + 1;
  cv[1] = grad ? 2 * L - 1 : L;
  cb[0] = cv[1];
  cb[1] = cv[0];
}

Lay layout(const int64_t* ld, int L, int grad, int es, int pstride,
           int maxwg, int64_t n, int64_t m) {
  Lay y;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = up256(o + bytes);
    return at;
  };
  int cv[2], cb[2];
  capacities(L, grad, cv, cb);
  const int tm = cv[0];
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
  y.U = take((size_t)es * n);
  y.V2 = take((size_t)es * n);
  y.gbar = grad ? take((size_t)es * n) : 0;
  y.end = o;
  return y;
}

// One query index for every trial: data side R (Q-queries) or L.
int ista_query(hd_ista_ctx* b, IstaStep& st, int ds) {
  const int gs = 1 - ds, C = b->count, f64 = b->f64;
  st.kR = b->kR;
  st.kL = b->kL;
  st.step = (uint32_t)(st.q + 1);
  if (b->kR + b->kL > 0) {
    ILCHK(launch_ista_tdot(f64, b->cpt[ds], ds, C * b->nwg[ds], b->dev, st,
                           b->stream));
    ILCHK(launch_ista_small(f64, 0, ds, C, b->dev, st, b->stream));
  }
  ILCHK(launch_ista_data(f64, b->cpt[ds], ds, C * b->nwg[ds], b->dev, st,
                         b->stream));
  ILCHK(launch_ista_small(f64, 1, ds, C, b->dev, st, b->stream));
  ILCHK(launch_ista_rand(f64, b->cpt[gs], gs, C * b->nwg[gs], b->dev, st,
                         b->stream));
  if (ds == 0)
    ++b->kR;
  else
    ++b->kL;
  return HD_OK;
}

}  // namespace

extern "C" {

int hd_ista_init(int32_t storage, int64_t m, int64_t n, int32_t L,
                 int32_t count, uint32_t seed, uint32_t trial0, double sigma,
                 int32_t flags, void* stream, hd_ista* out) {
  if (!out) return HD_ERR_INVALID;
  *out = nullptr;
  if (storage != HD_F32 && storage != HD_F64) return HD_ERR_INVALID;
  if (m < 1 || n < 1 || L < 1 || count < 1) return HD_ERR_INVALID;
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return HD_ERR_INVALID;
  if (flags & ~HD_ISTA_GRAD) return HD_ERR_INVALID;
  const int grad = (flags & HD_ISTA_GRAD) != 0;
  // Algorithm 1 needs r <= n (reflectors from Q-queries) and l <= m
  int cv[2], cb[2];
  capacities(L, grad, cv, cb);
  if ((int64_t)cv[0] > n || (int64_t)cv[1] > m) return HD_ERR_INVALID;
  if (n > ((int64_t)1 << 31) || m > ((int64_t)1 << 31)) return HD_ERR_INVALID;
  hd_ista_ctx* b = new (std::nothrow) hd_ista_ctx();
  if (!b) return HD_ERR_NOMEM;
  b->f64 = storage == HD_F64;
  b->es = b->f64 ? 8 : 4;
  b->stream = (hipStream_t)stream;
  b->count = count;
  b->L = L;
  b->grad = grad;
  b->ran = 0;
  b->kR = b->kL = 0;
  b->nwg_adj = (int)((n + 255) / 256);
  b->dim[0] = n;
  b->dim[1] = m;
  int64_t ld[2];
  for (int s = 0; s < 2; ++s) {
    b->cpt[s] = ista_cpt(b->dim[s]);
    const int64_t rows = 256 * (int64_t)b->cpt[s];
    ld[s] = (b->dim[s] + rows - 1) / rows * rows;
    b->nwg[s] = (int)(ld[s] / rows);
  }
  const int tm = cv[0], Q = grad ? 4 * L - 1 : 2 * L + 1;
  const int slot2 = Q + 1, extra = slot2 + tm + 1;
  const int pstride = extra + kNumExtra;
  const int maxwg = b->nwg[0] > b->nwg[1] ? b->nwg[0] : b->nwg[1];
  const Lay lay = layout(ld, L, grad, b->es, pstride, maxwg, n, m);
  const size_t per = lay.end;
  const double rec = grad ? 2.0 * b->es * (double)L * n * count : 0.0;
  if ((double)per * count + rec > 2.5e11) {
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
  if (grad) {
    const size_t rb = (size_t)b->es * L * (size_t)n * count;
    IALLOC(b->Urec, rb);
    IALLOC(b->Vrec, rb);
    IALLOC(b->adj_part, sizeof(double) * 2 * (size_t)b->nwg_adj * count);
  }
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
    d.U = A + lay.U;
    d.V = A + lay.V2;
    d.gbar = grad ? A + lay.gbar : nullptr;
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
  const int L = b->L;
  // every run starts from fresh matrices: the reflector counts restart
  // and every array a query reads is rewritten before it is read
  IstaStep st;
  std::memset(&st, 0, sizeof(st));
  st.L = L;
  st.xstar = xstar;
  st.noise = noise;
  st.X = X;
  st.Urec = b->Urec;
  st.Vrec = b->Vrec;
  b->kR = b->kL = 0;
  b->ran = 0;
  for (int q = 0; q <= 2 * L; ++q) {
    const int ds = (q == 0 || q % 2 == 1) ? 0 : 1;
    st.q = q;
    // with a reverse pass to come, the last forward query still prepares
    // the next one (its data side is the next query's random side)
    st.last = q == 2 * L && !b->grad;
    if (ds == 1) {
      st.a = a[q / 2 - 1];
      st.theta = theta[q / 2 - 1];
    }
    const int rc = ista_query(b, st, ds);
    if (rc) return rc;
  }
  b->ran = 1;
  return HD_OK;
}

int hd_ista_grad(hd_ista b, const float* a, const float* theta, void* G,
                 double* grad_a, double* grad_theta) {
  if (!b || !a || !theta || !G || !grad_a || !grad_theta)
    return HD_ERR_INVALID;
  if (!b->grad || !b->ran) return HD_ERR_INVALID;
  const int L = b->L, C = b->count;
  IstaStep st;
  std::memset(&st, 0, sizeof(st));
  st.L = L;
  st.bwd = 1;
  st.G = G;
  IstaAdjArgs ad;
  std::memset(&ad, 0, sizeof(ad));
  ad.D = b->dev;
  ad.G = G;
  ad.Urec = b->Urec;
  ad.Vrec = b->Vrec;
  ad.L = L;
  ad.nwg = b->nwg_adj;
  ad.n = b->dim[0];
  ad.part = b->adj_part;
  ad.grad_a = grad_a;
  ad.grad_theta = grad_theta;
  int q = 2 * L + 1;
  b->ran = 0;  // the reverse pass uses up the room it was given
  for (int t = L - 1; t >= 0; --t) {
    ad.t = t;
    ad.theta = theta[t];
    ILCHK(launch_ista_adj(b->f64, C, ad, b->stream));
    if (t == 0) break;
    // g <- gbar - a_t Q'Q gbar: two more queries on every trial's Q
    st.a = a[t];
    st.q = q++;
    st.last = 0;
    int rc = ista_query(b, st, 0);
    if (rc) return rc;
    st.q = q++;
    st.last = t == 1;
    rc = ista_query(b, st, 1);
    if (rc) return rc;
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
