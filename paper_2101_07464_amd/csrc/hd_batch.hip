// hd_batch.hip -- C-ABI runtime of batches of independent Haar trials
// (Algorithm 2, all Q-queries) run in lockstep.  All arithmetic runs in the
// batched kernels of hd_kernels.hip; this file lays out the per-trial state
// in one device arena and orders the launches of each query index.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "hd.h"
#include "hd_internal.hpp"

using namespace hd;

struct hd_batch_ctx {
  int f64;
  int es;
  hipStream_t stream;
  int count;
  int cpt;
  int tmax;                        // longest trial
  std::vector<hd_batch_trial> tr;  // in run order (T descending)
  std::vector<int> order;          // run position -> caller index
  std::vector<int> blk_first;      // count + 1 (host copy)
  std::vector<int> active;         // active[t] = trials with T >= t
  std::vector<TrialDev> host;      // last arguments copied to the device
  bool uploaded = false;
  std::vector<CopyJob> jobs_h;     // copies of x_1 (first count) and of
                                   // x_{T+1} (next count) now on the device
  TrialDev* dev = nullptr;
  int* blk_trial = nullptr;
  int* blk_first_d = nullptr;
  CopyJob* jobs = nullptr;         // 2 * count entries
  char* arena = nullptr;
  std::vector<size_t> ring_off;    // per run position: x ring (3 n)
  int* flag = nullptr;
  void* zeros = nullptr;
  std::vector<void*> allocs;
  // HIP graphs of a run's launch sequence (without, with the x_{T+1} copy),
  // captured on first use when enabled; every launch argument is fixed by
  // the trial set, and what changes between runs lives in device buffers
  bool use_graph = false;
  hipGraphExec_t exec[2] = {nullptr, nullptr};
};

namespace {

thread_local char b_err[256];

int bfail(hipError_t e) {
  std::snprintf(b_err, sizeof(b_err), "%s", hipGetErrorString(e));
  return HD_ERR_HIP;
}

#define BHIP(call)                             \
  do {                                         \
    hipError_t e_ = (call);                    \
    if (e_ != hipSuccess) return bfail(e_);    \
  } while (0)

#define BLCHK(call)                                          \
  do {                                                       \
    int e_ = (call);                                         \
    if (e_ != 0) return bfail((hipError_t)(e_ > 0 ? e_ : 1)); \
  } while (0)

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

// Chunks of 256 rows per workgroup for every trial of a batch (panels are
// padded to 1024 rows, so 1, 2 and 4 all tile them).  Four: a batch has
// workgroups to spare, so longer sweeps with fewer reductions per row win
// (4096 ragged Haar trials of 1e3..1e5 rows: 1717, 1520 and 1429 ms per run
// at 1, 2 and 4).  HD_BATCH_CPT = 1, 2 or 4 overrides it.
int batch_cpt() {
  const char* e = std::getenv("HD_BATCH_CPT");
  if (e) {
    const int v = std::atoi(e);
    if (v == 1 || v == 2 || v == 4) return v;
  }
  return 4;
}
int64_t round_up(int64_t v, int64_t q) { return (v + q - 1) / q * q; }

int launch_run(hd_batch_ctx* b, bool copy_out);
int apply_shape(hd_batch_ctx* b, int cpt);

void release(hd_batch_ctx* b) {
  (void)hipStreamSynchronize(b->stream);
  for (auto& e : b->exec)
    if (e) {
      (void)hipGraphExecDestroy(e);
      e = nullptr;
    }
  for (void* p : b->allocs) (void)hipFree(p);
  b->allocs.clear();
}

template <typename P>
int balloc(hd_batch_ctx* b, P** out, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes ? bytes : 8) != hipSuccess) {
    (void)hipGetLastError();
    return HD_ERR_NOMEM;
  }
  b->allocs.push_back(p);
  if (hipMemsetAsync(p, 0, bytes ? bytes : 8, b->stream) != hipSuccess)
    return bfail(hipGetLastError());
  *out = (P*)p;
  return HD_OK;
}

// Offsets of one trial's buffers inside the arena.
struct Layout {
  size_t V[2], T[2], tau[2], nu[2], piv[2], sgn[2], pi[2], red[2];
  size_t part, part2, w, zD, zG, head, scal, ring;
  size_t end;
};

Layout layout_of(size_t base, int64_t n, int T, int es, int nwg,
                 int pstride) {
  Layout L;
  size_t o = base;
  const int64_t ld = round_up(n, kChunk);
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = up256(o + bytes);
    return at;
  };
  for (int s = 0; s < 2; ++s) {
    L.V[s] = take((size_t)es * ld * T);
    L.T[s] = take(sizeof(double) * (size_t)T * T);
    L.tau[s] = take(sizeof(double) * T);
    L.nu[s] = take(sizeof(double) * T);
    L.piv[s] = take(sizeof(double) * T);
    L.sgn[s] = take(sizeof(double) * T);
    L.pi[s] = take(sizeof(double) * (T + 1));
    L.red[s] = take(sizeof(double) * pstride);
  }
  L.part = take(sizeof(double) * (size_t)nwg * pstride);
  L.part2 = take(sizeof(double) * (size_t)nwg * pstride);
  L.w = take(sizeof(double) * pstride);
  L.zD = take(sizeof(double) * T);
  L.zG = take(sizeof(double) * 3 * (size_t)T);
  L.head = take(sizeof(double) * T);
  L.scal = take(sizeof(double) * 8);
  L.ring = take((size_t)es * 3 * n);
  L.end = o;
  return L;
}

}  // namespace

extern "C" {

int hd_batch_init(int32_t storage, const hd_batch_trial* trials,
                  int32_t count, void* stream, hd_batch* out) {
  if (!out) return HD_ERR_INVALID;
  *out = nullptr;
  if (!trials || count < 1) return HD_ERR_INVALID;
  if (storage != HD_F32 && storage != HD_F64) return HD_ERR_INVALID;
  for (int i = 0; i < count; ++i) {
    const hd_batch_trial& t = trials[i];
    if (t.n < 1 || t.T < 1 || (int64_t)t.T > t.n) return HD_ERR_INVALID;
    if (t.n > ((int64_t)1 << 31)) return HD_ERR_INVALID;
  }
  hd_batch_ctx* b = new (std::nothrow) hd_batch_ctx();
  if (!b) return HD_ERR_NOMEM;
  b->f64 = storage == HD_F64;
  b->es = b->f64 ? 8 : 4;
  b->stream = (hipStream_t)stream;
  b->count = count;
  b->cpt = batch_cpt();
  // run order: longest trial first, so the running trials are a prefix
  b->order.resize(count);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
    return trials[x].T > trials[y].T;
  });
  for (int i = 0; i < count; ++i) b->tr.push_back(trials[b->order[i]]);
  b->tmax = b->tr[0].T;
  b->active.assign(b->tmax + 2, 0);
  for (const auto& t : b->tr)
    for (int s = 1; s <= t.T; ++s) b->active[s]++;
  // arena layout; partial rows and the block map are sized for the most
  // workgroups any shape launches (one chunk per workgroup)
  std::vector<Layout> lay(count);
  std::vector<int> nwg(count), pstride(count), slot2(count), extra(count);
  size_t arena = 0;
  int64_t nmax = 0;
  int nblk = 0;
  for (int i = 0; i < count; ++i) {
    const auto& t = b->tr[i];
    const int64_t ld = round_up(t.n, kChunk);
    nwg[i] = (int)(ld / 256);
    slot2[i] = t.T + 1;
    extra[i] = slot2[i] + t.T + 1;
    pstride[i] = extra[i] + kNumExtra;
    lay[i] = layout_of(arena, t.n, t.T, b->es, nwg[i], pstride[i]);
    arena = lay[i].end;
    nblk += nwg[i];
    nmax = std::max(nmax, t.n);
  }
  int rc = HD_OK;
#define BALLOC(ptr, bytes)          \
  do {                              \
    rc = balloc(b, &(ptr), (bytes)); \
    if (rc != HD_OK) {              \
      release(b);                   \
      delete b;                     \
      return rc;                    \
    }                               \
  } while (0)
  BALLOC(b->arena, arena);
  BALLOC(b->dev, sizeof(TrialDev) * count);
  BALLOC(b->blk_trial, sizeof(int) * nblk);
  BALLOC(b->blk_first_d, sizeof(int) * (count + 1));
  BALLOC(b->jobs, sizeof(CopyJob) * 2 * count);
  BALLOC(b->flag, sizeof(int) * 4);
  BALLOC(b->zeros, (size_t)b->es * nmax + 8);
#undef BALLOC
  // the pi[0] = 1 entries
  auto fail = [&](hipError_t e) {
    int r = bfail(e);
    release(b);
    delete b;
    return r;
  };
  if (hipStreamSynchronize(b->stream) != hipSuccess)
    return fail(hipGetLastError());
  // pi[0] = 1 on both sides of every trial: copies of one double kept at the
  // end of the zero vector
  const double one = 1.0;
  double* d_one = (double*)((char*)b->zeros + (size_t)b->es * nmax);
  hipError_t e =
      hipMemcpy(d_one, &one, sizeof(double), hipMemcpyHostToDevice);
  std::vector<CopyJob> pij(2 * (size_t)count);
  for (int i = 0; i < count; ++i)
    for (int s = 0; s < 2; ++s)
      pij[2 * i + s] = CopyJob{d_one, b->arena + lay[i].pi[s], 2};
  if (e == hipSuccess)
    e = hipMemcpy(b->jobs, pij.data(), sizeof(CopyJob) * 2 * count,
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(e);
  if (launch_copy_jobs(b->jobs, 2 * count, b->stream) != 0 ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return fail(hipGetLastError());
  // per-trial arguments (vector pointers are set by each run)
  b->host.resize(count);
  b->ring_off.resize(count);
  for (int i = 0; i < count; ++i) {
    const auto& t = b->tr[i];
    const Layout& L = lay[i];
    char* A = b->arena;
    PanelDev P[2];
    for (int s = 0; s < 2; ++s) {
      P[s].V = A + L.V[s];
      P[s].ld = round_up(t.n, kChunk);
      P[s].T = (double*)(A + L.T[s]);
      P[s].tau = (double*)(A + L.tau[s]);
      P[s].nu = (double*)(A + L.nu[s]);
      P[s].piv = (double*)(A + L.piv[s]);
      P[s].sgn = (double*)(A + L.sgn[s]);
      P[s].pi = (double*)(A + L.pi[s]);
      P[s].red = (double*)(A + L.red[s]);
    }
    const Key key{t.seed, t.trial};
    TrialDev d;
    std::memset(&d, 0, sizeof(d));
    d.td.V = P[0].V;
    d.td.ld = P[0].ld;
    d.td.slot2 = slot2[i];
    d.td.key = key;
    d.td.lo = -1;
    d.td.n = t.n;
    d.td.partials = (double*)(A + L.part);
    d.td.pstride = pstride[i];
    d.td.extra = extra[i];
    for (int q = 0; q < 2; ++q) {
      PassArgs& a = q == 0 ? d.pd : d.pr;
      const int side = q;  // data side R (0), random side L (1)
      a.V = P[side].V;
      a.ld = P[side].ld;
      a.pi = P[side].pi;
      a.n = t.n;
      a.head = (double*)(A + L.head);
      a.key = key;
      a.pstride = pstride[i];
      a.extra = extra[i];
      a.cslot = -1;
    }
    d.pd.z = (double*)(A + L.zD);
    d.pd.pivot = (double*)(A + L.scal);
    d.pd.partials = (double*)(A + L.part);
    d.pr.z = (double*)(A + L.zG);
    d.pr.cscale = (double*)(A + L.scal) + 1;
    d.pr.partials = (double*)(A + L.part2);
    d.sd.T = P[0].T;
    d.sd.tau = P[0].tau;
    d.sd.tmax = t.T;
    d.sd.w = (double*)(A + L.w);
    d.sd.z = (double*)(A + L.zD);
    d.hs.D = P[0];
    d.hs.G = P[1];
    d.hs.tmax = t.T;
    d.hs.zG = (double*)(A + L.zG);
    d.hs.head = (double*)(A + L.head);
    d.hs.pivot = (double*)(A + L.scal);
    d.hs.cscale = (double*)(A + L.scal) + 1;
    d.hs.key = key;
    d.hs.extra = extra[i];
    d.hs.cslot = -1;
    d.hs.flag = b->flag;
    d.x0 = b->zeros;
    d.T = t.T;
    b->host[i] = d;
    b->ring_off[i] = L.ring;
  }
  const int rs = apply_shape(b, batch_cpt());
  if (rs != HD_OK) {
    release(b);
    delete b;
    return rs;
  }
  *out = b;
  return HD_OK;
}

int hd_batch_set_shape(hd_batch b, int32_t chunks) {
  if (!b || (chunks != 1 && chunks != 2 && chunks != 4)) return HD_ERR_INVALID;
  return chunks == b->cpt ? HD_OK : apply_shape(b, chunks);
}

int hd_batch_shape(hd_batch b) { return b ? b->cpt : HD_ERR_INVALID; }

int hd_batch_autotune(hd_batch b, const hd_dynamics* dyn,
                      const void* const* x1, int32_t reps, double* ms,
                      int32_t* chosen) {
  if (!b || !dyn || !x1 || reps < 1 || reps > 100) return HD_ERR_INVALID;
  static const int kShapes[3] = {1, 2, 4};
  const int builtin = batch_cpt();
  const bool graph = b->use_graph;
  b->use_graph = false;
  double t[3] = {0, 0, 0};
  hipEvent_t ev[2] = {nullptr, nullptr};
  int rc = HD_OK;
  for (auto& v : ev)
    if (rc == HD_OK && hipEventCreate(&v) != hipSuccess)
      rc = bfail(hipGetLastError());
  for (int i = 0; i < 3 && rc == HD_OK; ++i) {
    rc = hd_batch_set_shape(b, kShapes[i]);
    // one untimed run (it also uploads the changed per-trial arguments)
    if (rc == HD_OK) rc = hd_batch_run(b, dyn, x1, nullptr, nullptr, nullptr);
    if (rc == HD_OK && hipEventRecord(ev[0], b->stream) != hipSuccess)
      rc = bfail(hipGetLastError());
    for (int r = 0; r < reps && rc == HD_OK; ++r)
      rc = hd_batch_run(b, dyn, x1, nullptr, nullptr, nullptr);
    float el = 0.f;
    if (rc == HD_OK && (hipEventRecord(ev[1], b->stream) != hipSuccess ||
                        hipEventSynchronize(ev[1]) != hipSuccess ||
                        hipEventElapsedTime(&el, ev[0], ev[1]) != hipSuccess))
      rc = bfail(hipGetLastError());
    t[i] = (double)el / reps;
  }
  for (auto& v : ev)
    if (v) (void)hipEventDestroy(v);
  b->use_graph = graph;
  if (rc != HD_OK) return rc;
  // the built-in shape stays unless another is at least 3% faster
  const int ib = builtin == 1 ? 0 : builtin == 2 ? 1 : 2;
  int imin = 0;
  for (int i = 1; i < 3; ++i)
    if (t[i] < t[imin]) imin = i;
  const int best = t[imin] < 0.97 * t[ib] ? kShapes[imin] : builtin;
  if (ms)
    for (int i = 0; i < 3; ++i) ms[i] = t[i];
  if (chosen) *chosen = best;
  return hd_batch_set_shape(b, best);
}

int hd_batch_set_stream(hd_batch b, void* stream) {
  if (!b) return HD_ERR_INVALID;
  b->stream = (hipStream_t)stream;
  return HD_OK;
}

int hd_batch_free(hd_batch b) {
  if (!b) return HD_OK;
  release(b);
  delete b;
  return HD_OK;
}

int hd_batch_status(hd_batch b) {
  if (!b) return HD_ERR_INVALID;
  BHIP(hipStreamSynchronize(b->stream));
  int flag = 0;
  BHIP(hipMemcpy(&flag, b->flag, sizeof(int), hipMemcpyDeviceToHost));
  return flag ? HD_ERR_NONFINITE : HD_OK;
}

int hd_batch_run(hd_batch b, const hd_dynamics* dyn, const void* const* x1,
                 void* const* x_out, void* const* traj_x,
                 void* const* traj_y) {
  if (!b || !dyn || !x1) return HD_ERR_INVALID;
  if (dyn->kind != HD_DYN_TANH && dyn->kind != HD_DYN_SOFT_HIST)
    return HD_ERR_UNSUPPORTED;
  if (dyn->pattern != HD_PATTERN_Q) return HD_ERR_UNSUPPORTED;
  const int C = b->count;
  for (int i = 0; i < C; ++i) {
    const int c = b->order[i];
    if (!x1[c] || (traj_x && !traj_x[c]) || (traj_y && !traj_y[c]) ||
        (x_out && !x_out[c]))
      return HD_ERR_INVALID;
  }
  // vector pointers and the map of this run
  std::vector<TrialDev> next = b->host;
  for (int i = 0; i < C; ++i) {
    const int c = b->order[i];
    TrialDev& d = next[i];
    const auto& t = b->tr[i];
    char* ring = b->arena + b->ring_off[i];
    d.xbase = traj_x ? traj_x[c] : ring;
    d.xmod = traj_x ? t.T + 1 : 3;
    d.ybase = traj_y ? traj_y[c] : nullptr;  // unrecorded answers: not stored
    d.ymod = traj_y ? t.T : 1;
    d.pr.dyn.kind = dyn->kind;
    d.pr.dyn.a = dyn->a;
    d.pr.dyn.b = dyn->b;
  }
  if (std::memcmp(next.data(), b->host.data(), sizeof(TrialDev) * C) != 0 ||
      !b->uploaded) {
    b->uploaded = true;
    b->host = next;
    BHIP(hipMemcpyAsync(b->dev, b->host.data(), sizeof(TrialDev) * C,
                        hipMemcpyHostToDevice, b->stream));
    BHIP(hipStreamSynchronize(b->stream));
  }
  // copies of x_1 into slot 1 and, after the run, of x_{T+1} out
  std::vector<CopyJob> jobs(2 * (size_t)C);
  for (int i = 0; i < C; ++i) {
    const int c = b->order[i];
    const auto& t = b->tr[i];
    const TrialDev& d = b->host[i];
    const int64_t words = t.n * b->es / 4;
    jobs[i].src = x1[c];
    jobs[i].dst = (void*)d.xbase;
    // x1 may already be row 0 of traj_x
    jobs[i].words = x1[c] == d.xbase ? 0 : words;
    jobs[C + i].src = (const char*)d.xbase +
                      (size_t)b->es * t.n * (size_t)(t.T % d.xmod);
    jobs[C + i].dst = x_out ? x_out[c] : nullptr;
    jobs[C + i].words = x_out ? words : 0;
  }
  if (jobs.size() != b->jobs_h.size() ||
      std::memcmp(jobs.data(), b->jobs_h.data(),
                  sizeof(CopyJob) * jobs.size()) != 0) {
    b->jobs_h = jobs;
    BHIP(hipMemcpyAsync(b->jobs, b->jobs_h.data(),
                        sizeof(CopyJob) * jobs.size(), hipMemcpyHostToDevice,
                        b->stream));
    BHIP(hipStreamSynchronize(b->stream));
  }
  const int gi = x_out ? 1 : 0;
  if (b->use_graph && b->exec[gi]) {
    BHIP(hipGraphLaunch(b->exec[gi], b->stream));
    return HD_OK;
  }
  if (b->use_graph) {
    // record this run's launches once; they run from the graph below
    BHIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int rc = launch_run(b, x_out != nullptr);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) return bfail(ec);
    const hipError_t ei = hipGraphInstantiate(&b->exec[gi], g, nullptr,
                                              nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      b->exec[gi] = nullptr;
      return bfail(ei);
    }
    BHIP(hipGraphLaunch(b->exec[gi], b->stream));
    return HD_OK;
  }
  return launch_run(b, x_out != nullptr);
}

int hd_batch_set_graph(hd_batch b, int32_t enable) {
  if (!b || (enable != 0 && enable != 1)) return HD_ERR_INVALID;
  if (enable && !b->stream) return HD_ERR_UNSUPPORTED;
  b->use_graph = enable != 0;
  return HD_OK;
}

}  // extern "C"

namespace {

// Workgroups of `cpt` chunks for every trial: the block map (workgroup ->
// trial, each trial's first workgroup) and each trial's partial-row count.
// Recorded graphs hold the old launch sizes and are dropped.
int apply_shape(hd_batch_ctx* b, int cpt) {
  const int C = b->count;
  std::vector<int> first(C + 1, 0);
  for (int i = 0; i < C; ++i)
    first[i + 1] = first[i] + (int)(round_up(b->tr[i].n, kChunk) / (256 * cpt));
  std::vector<int> bt(first[C]);
  for (int i = 0; i < C; ++i)
    for (int q = first[i]; q < first[i + 1]; ++q) bt[q] = i;
  BHIP(hipStreamSynchronize(b->stream));
  for (auto& e : b->exec)
    if (e) {
      BHIP(hipGraphExecDestroy(e));
      e = nullptr;
    }
  BHIP(hipMemcpy(b->blk_trial, bt.data(), sizeof(int) * bt.size(),
                 hipMemcpyHostToDevice));
  BHIP(hipMemcpy(b->blk_first_d, first.data(), sizeof(int) * (C + 1),
                 hipMemcpyHostToDevice));
  for (int i = 0; i < C; ++i) b->host[i].nwg = first[i + 1] - first[i];
  b->blk_first = first;
  b->cpt = cpt;
  b->uploaded = false;  // the next run copies the new nwg to the device
  return HD_OK;
}

// The launches of one run: x_1 in, every step, x_{T+1} out (when asked).
int launch_run(hd_batch_ctx* b, bool copy_out) {
  const int C = b->count;
  BLCHK(launch_copy_jobs(b->jobs, C, b->stream));
  const BatchMap map{b->blk_trial, b->blk_first_d};
  const int f64 = b->f64, cpt = b->cpt;
  for (int t = 1; t <= b->tmax; ++t) {
    const int A = b->active[t];
    const int nblk = b->blk_first[A];
    const BatchStep st{t - 1, (uint32_t)t};
    if (t == 1)
      BLCHK(launch_prefetch1_batch(f64, cpt, nblk, b->dev, map, b->stream));
    else
      BLCHK(launch_tdot_batch(f64, cpt, nblk, t >= 3, b->dev, map, st,
                              b->stream));
    BLCHK(launch_trial_small(f64, kBatchAfterTdot, A, b->dev, st, b->stream));
    BLCHK(launch_pass_batch(f64, cpt, nblk, kPassData, b->dev, map, st,
                            b->stream));
    BLCHK(launch_trial_small(f64, kBatchAfterData, A, b->dev, st, b->stream));
    BLCHK(launch_pass_batch(f64, cpt, nblk, kPassRandHaar, b->dev, map, st,
                            b->stream));
  }
  if (copy_out) BLCHK(launch_copy_jobs(b->jobs + C, C, b->stream));
  return HD_OK;
}

}  // namespace
