// hd_api.hip -- C-ABI runtime of libhd.so: handle state, validation, and the
// per-query launch sequence.  All arithmetic runs in the kernels of
// hd_kernels.hip; this file only orders launches on the handle's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "hd.h"
#include "hd_internal.hpp"

using namespace hd;

namespace {

struct ProfRec {
  int kind;
  hipEvent_t a, b;
  double bytes;
};

}  // namespace

struct hd_ctx {
  hd_config cfg;
  int f64;
  int es;          // bytes per stored element
  int64_t dim[2];  // n (side 0, R), m (side 1, L)
  int64_t ld[2];   // leading dimension of the panels of each side
  Shape sh[2];     // launch shape of the panel kernels of each side
  int pstride, slot2, extra;
  hipStream_t stream;
  PanelDev P[2];   // 0 = R (acts on R^n), 1 = L (acts on R^m)
  int pf_step[2];  // query index whose random-side prefetch P[s].red holds
  int pending[2];  // data column whose T column still needs V'u, or -1
  int hint;        // transpose flag of the next query: -1 unknown, 0 or 1,
                   // kHintNone when no query is expected to follow
  double* partials;
  double* partials2;  // partial rows of the random-side pass
  double* red_stage;  // two-stage reduction: one region per job (a, b)
  size_t red_half;    // doubles per region
  ReduceJob deferred; // its sums, launched with the next reduction
  // The next query's TDOT dots, computed by the last random pass (its panel
  // is the next data side and its epilogue made the next input): valid for
  // query `step` on side `side` with input `x` and `nslots` dots.
  struct {
    int valid, step, side, nslots;
    const void* x;
  } wready;
  // The data pass forms z = T' w itself (its prologue) from h->w, with the
  // pending T column kp (dots in h->w + slot2) when kp > 0.
  struct {
    int use, kp;
  } zpro;
  double* w;       // TDOT results (pstride)
  double* wc;      // dots of a pending column's T-column pass (pstride)
  double* zD;      // T' w (t_max)
  double* zG;      // random-side coefficients + scratch (3 t_max)
  double* z2;      // Ginibre: second coefficient vector of the random side
  double* head;    // rows < k of p (t_max)
  double* scal;    // [0] pivot, [1] cscale
  double* gscal;   // Ginibre: [0] nu, [1] sigma
  void* B[2];      // Ginibre explicit basis vectors: B[0] (n rows) holds v_t
                   // of Q'-queries, B[1] (m rows) u_t of Q-queries
  int* flag;
  void* ring[3];   // internal trajectory vectors for hd_run
  void* ybuf;
  void* zeros;
  void* ista[6];   // unrolled-ISTA work vectors (max(m, n) entries each)
  double* ista_part;
  int t, r, l;
  // Buffers carved from a caller-independent static region instead of
  // hipMalloc (the allocation-free entry point): base, used and capacity in
  // bytes.  base == nullptr with active set only measures the layout.
  struct {
    int active;
    char* base;
    size_t used, cap;
  } carve;
  std::vector<void*> allocs;
  // profiling
  int prof;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  size_t pool_used;
};

namespace {

constexpr int kHintNone = 2;

thread_local char g_err[256];

int hip_fail(hipError_t e) {
  std::snprintf(g_err, sizeof(g_err), "%s", hipGetErrorString(e));
  return HD_ERR_HIP;
}

#define HIPC(call)                               \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hip_fail(e_);   \
  } while (0)

#define LCHK(call)                                              \
  do {                                                          \
    int e_ = (call);                                            \
    if (e_ != 0) return hip_fail((hipError_t)(e_ > 0 ? e_ : 1)); \
  } while (0)

int64_t round_up(int64_t v, int64_t q) { return (v + q - 1) / q * q; }

int env_int(const char* name, int dflt) {
  const char* e = std::getenv(name);
  return e ? std::atoi(e) : dflt;
}


// Workgroups cover 256 * cpt rows.  Built-in rule, from tuner sweeps of
// both ensembles and storage types (16- and 64-query trajectories): one
// chunk below 256K rows, two below 512K, four from there on.  hd_autotune installs measured shapes per
// ensemble and storage type: (panel length, cpt), sorted by length.  A
// panel takes the entry whose length is nearest its own in ratio, if that
// ratio is at most 2.  HD_CPT overrides both.  The tables are read by
// hd_init and replaced by hd_autotune / hd_autotune_clear under g_tune_mu.
std::vector<std::pair<int64_t, int>> g_tuned[2][2];
std::mutex g_tune_mu;

int tuned_cpt(int ens, int f64, int64_t dim) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  int cpt = 0;
  double best = 2.0;
  for (const auto& e : g_tuned[ens == HD_HAAR ? 1 : 0][f64 ? 1 : 0]) {
    const double r = e.first > dim ? (double)e.first / (double)dim
                                   : (double)dim / (double)e.first;
    if (r <= best) {
      best = r;
      cpt = e.second;
    }
  }
  return cpt;
}

Shape shape_of(int64_t ld, int cpt) {
  Shape sh;
  sh.cpt = cpt;
  sh.nwg = (int)(ld / ((int64_t)256 * cpt));
  return sh;
}

// Set only inside hd_autotune, for its own thread: sizes its scratch
// handle for the one-chunk shape (the most workgroups, hence the largest
// partial-sum buffers); handles other threads create meanwhile are not
// affected.
thread_local int g_force_cpt = 0;

// The built-in rule's chunks per workgroup for a panel of `dim` rows.
int dim_rule(int64_t dim) {
  return dim < ((int64_t)1 << 18) ? 1 : (dim < ((int64_t)1 << 19) ? 2 : 4);
}

// A tuned shape replaces the built-in one only when at least this much
// faster.
constexpr double kTuneMargin = 0.03;

Shape pick_shape(int ens, int f64, int64_t dim, int64_t ld) {
  if (g_force_cpt) return shape_of(ld, g_force_cpt);
  int c = dim_rule(dim);
  const int t = tuned_cpt(ens, f64, dim);
  if (t) c = t;
  const int e = env_int("HD_CPT", 0);
  if (e == 1 || e == 2 || e == 4) c = e;
  return shape_of(ld, c);
}

template <typename P>
int dalloc(hd_ctx* h, P** out, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 8;
  if (h->carve.active) {
    // 256-byte aligned slices of the static region, cleared together by the
    // caller once the layout is complete
    const size_t at = (h->carve.used + 255) / 256 * 256;
    if (at + bytes > h->carve.cap) return HD_ERR_NOMEM;
    h->carve.used = at + bytes;
    *out = (P*)(h->carve.base ? h->carve.base + at : nullptr);
    return HD_OK;
  }
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return HD_ERR_NOMEM;
  }
  h->allocs.push_back(p);
  if (hipMemsetAsync(p, 0, bytes, h->stream) != hipSuccess)
    return hip_fail(hipGetLastError());
  *out = (P*)p;
  return HD_OK;
}

void free_all(hd_ctx* h) {
  (void)hipStreamSynchronize(h->stream);
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
  for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
  h->pool.clear();
}

// ------------------------------------------------------------ profiling --

hipEvent_t prof_event(hd_ctx* h) {
  if (h->pool_used == h->pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->pool.push_back(e);
  }
  return h->pool[h->pool_used++];
}

// Timing of one panel launch: when profiling, a pair of events that the
// dispatch itself records at the kernel's start and end.
struct ProfScope {
  LaunchEvents ev;
  ProfScope(hd_ctx* h, int kind, double bytes) {
    if (!h->prof) return;
    hipEvent_t a = prof_event(h), b = prof_event(h);
    if (!a || !b) return;
    ev.start = a;
    ev.stop = b;
    h->recs.push_back(ProfRec{kind, a, b, bytes});
  }
};

// ------------------------------------------------------- launch helpers --

SlotRanges ranges(int s0, int n0, int s1 = 0, int n1 = 0, int s2 = 0,
                  int n2 = 0) {
  SlotRanges r;
  r.start[0] = s0;
  r.count[0] = n0;
  r.start[1] = s1;
  r.count[1] = n1;
  r.start[2] = s2;
  r.count[2] = n2;
  return r;
}

TdotArgs tdot_base(hd_ctx* h, int side) {
  TdotArgs a;
  std::memset(&a, 0, sizeof(a));
  a.V = h->P[side].V;
  a.ld = h->ld[side];
  a.n = h->dim[side];
  a.partials = h->partials;
  a.pstride = h->pstride;
  a.slot2 = h->slot2;
  a.extra = h->extra;
  a.key = Key{h->cfg.seed, h->cfg.trial};
  a.lo = -1;
  return a;
}

PassArgs pass_base(hd_ctx* h, int side) {
  PassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.V = h->P[side].V;
  a.ld = h->ld[side];
  a.n = h->dim[side];
  a.pi = h->P[side].pi;
  a.partials = h->partials;
  a.pstride = h->pstride;
  a.extra = h->extra;
  a.key = Key{h->cfg.seed, h->cfg.trial};
  a.cslot = -1;
  return a;
}

SmallDataArgs small_data_args(hd_ctx* h, int side, int kp, const double* c,
                              int k, const double* w, double* z) {
  SmallDataArgs sd;
  sd.T = h->P[side].T;
  sd.tau = h->P[side].tau;
  sd.tmax = h->cfg.t_max;
  sd.kp = kp;
  sd.c = c;
  sd.k = k;
  sd.w = w;
  sd.z = z;
  return sd;
}

// What follows a panel pass: the fixed-order sums of its partial rows into
// `out` (k_reduce), then optionally one small FP64 step.
struct After {
  SlotRanges rg;
  double* out;
  int op;  // 0 none, 1 small_data, 2 haar_small, 3 gin_small
  SmallDataArgs sd;
  HaarSmallArgs hs;
  GinSmallArgs gs;
};

After after_of(SlotRanges rg, double* out, int op) {
  After t;
  std::memset(&t, 0, sizeof(t));
  t.rg = rg;
  t.out = out;
  t.op = op;
  return t;
}

ReduceJob no_job() {
  ReduceJob j;
  std::memset(&j, 0, sizeof(j));
  return j;
}

int run_after(hd_ctx* h, int side, const After& af) {
  ReduceJob ja;
  ja.P = h->partials;
  ja.pstride = h->pstride;
  ja.nwg = h->sh[side].nwg;
  ja.rg = af.rg;
  ja.out = af.out;
  ja.stage = h->red_stage;
  LCHK(launch_reduce(ja, h->deferred, h->stream));
  h->deferred = no_job();
  if (af.op == 1) LCHK(launch_small_data(af.sd, h->stream));
  if (af.op == 2) LCHK(launch_haar_small(h->f64, af.hs, h->stream));
  if (af.op == 3) LCHK(launch_gin_small(h->f64, af.gs, h->stream));
  return HD_OK;
}

int do_tdot(hd_ctx* h, int side, const TdotArgs& a, const After& af,
            double bytes) {
  {
    ProfScope ps(h, 0, bytes);
    LCHK(launch_tdot(h->f64, h->sh[side], a, h->stream, ps.ev));
  }
  return run_after(h, side, af);
}

int do_pass(hd_ctx* h, int side, int mode, const PassArgs& a,
            const After& af, int kind, double bytes) {
  {
    ProfScope ps(h, kind, bytes);
    LCHK(launch_pass(h->f64, h->sh[side], mode, a, h->stream, ps.ev));
  }
  return run_after(h, side, af);
}

// The random-side pass ends a query.  Its partial rows (in partials2) are
// summed by the next reduction launch, which always precedes the next read
// of P[side].red.
void defer_after(hd_ctx* h, int side, const After& af) {
  h->deferred.P = h->partials2;
  h->deferred.pstride = h->pstride;
  h->deferred.nwg = h->sh[side].nwg;
  h->deferred.rg = af.rg;
  h->deferred.out = af.out;
  h->deferred.stage = h->red_stage + h->red_half;
}

// Which of this query's by-products the next one uses.  pf_data: the data
// pass's dots of its panel with the next draw (the data side is the next
// random side); pf_rand: likewise for the random pass; tcol: the data side's
// new T column is formed now (in the data pass) rather than by a later pass.
struct Plan {
  bool pf_data, pf_rand, tcol, wnext;
};

Plan plan_of(const hd_ctx* h, int ds, int step) {
  Plan p;
  const bool room = step + 1 <= h->cfg.t_max;
  p.wnext = false;
  if (h->hint == kHintNone) {
    p.pf_data = p.pf_rand = p.tcol = false;
  } else if (h->hint < 0) {
    p.pf_data = p.pf_rand = room;
    p.tcol = false;
  } else {
    const int next_gs = 1 - (h->hint ? 1 : 0);
    p.pf_data = room && next_gs == ds;
    p.pf_rand = room && next_gs != ds;
    p.tcol = next_gs == ds;
    // the next data side is this query's random side
    p.wnext = room && next_gs == ds;
  }
  return p;
}

const void* panel_col(hd_ctx* h, int side, int j) {
  return (const char*)h->P[side].V + (size_t)h->es * (size_t)h->ld[side] * j;
}

// Prefetch of the random side for query `step` on panel `side` holding k
// columns: dots of its columns with g_step over rows > lo, and (Haar) the
// squared norm of those rows of g_step, into P[side].red.
int prefetch(hd_ctx* h, int side, int k, int step, int64_t lo, int want_ss) {
  TdotArgs a = tdot_base(h, side);
  a.ncols = k;
  a.gen = 1;
  a.gen_step = (uint32_t)step;
  a.lo = lo;
  a.want_ss = want_ss;
  const After want = after_of(ranges(0, k, h->extra, want_ss ? kNumExtra : 0),
                            h->P[side].red, 0);
  int rc = do_tdot(h, side, a, want, (double)h->es * (double)h->ld[side] * k);
  if (rc) return rc;
  h->pf_step[side] = step;
  return HD_OK;
}

// Complete the pending T column of a panel about to serve as the random
// side: one pass of direct dots V[:, :kp]' u_kp.
int resolve_pending(hd_ctx* h, int side) {
  const int kp = h->pending[side];
  h->pending[side] = -1;
  if (kp <= 0) return HD_OK;
  TdotArgs a = tdot_base(h, side);
  a.ncols = kp;
  a.b = panel_col(h, side, kp);
  After want = after_of(ranges(0, kp), h->wc, 1);
  want.sd = small_data_args(h, side, kp, h->wc, 0, nullptr, nullptr);
  return do_tdot(h, side, a, want,
                 (double)h->es * ((double)h->ld[side] * kp + h->dim[side]));
}

// w = V_D' x (+ B_D' x for Ginibre, + V_D' u_kp for the pending column kp),
// then T column kp and z_D = T_D' w.
int data_tdot(hd_ctx* h, int ds, const void* x, int kD, int nb2) {
  const int kp = h->pending[ds];
  h->pending[ds] = -1;
  const int step = h->t + 1;
  const bool ready = h->wready.valid && h->wready.step == step &&
                     h->wready.side == ds && h->wready.x == x &&
                     h->wready.nslots == kD + nb2 && kp <= 0;
  if (h->wready.valid && !ready) h->deferred = no_job();  // unused dots
  h->wready.valid = 0;
  h->zpro.use = 0;
  if (kD + nb2 == 0) return HD_OK;
  // z-step in the data pass's prologue where its shape allows (at most
  // two chunks per workgroup; k within the LDS arrays)
  const bool zp = h->sh[ds].cpt <= 2 && kD <= kZproMax;
  if (zp) {
    h->zpro.use = 1;
    h->zpro.kp = ready ? -1 : kp;
  }
  if (ready) {
    // the dots are in the deferred partial rows: sum them (and take the
    // z-step), with no TDOT launch
    After want = after_of(ranges(0, 0), h->w, zp ? 0 : 1);
    want.sd = small_data_args(h, ds, -1, nullptr, kD,
                              kD > 0 ? h->w : nullptr, h->zD);
    return run_after(h, ds, want);
  }
  TdotArgs a = tdot_base(h, ds);
  a.ncols = kD;
  a.V2 = nb2 ? h->B[ds] : nullptr;
  a.ncols2 = nb2;
  a.b = x;
  a.b2 = kp > 0 ? panel_col(h, ds, kp) : nullptr;
  After want = after_of(ranges(0, kD + nb2, h->slot2, kp > 0 ? kp : 0), h->w,
                      zp ? 0 : 1);
  want.sd = small_data_args(h, ds, kp, h->w + h->slot2, kD,
                            kD > 0 ? h->w : nullptr, h->zD);
  const double n = (double)h->dim[ds];
  return do_tdot(h, ds, a, want,
                 (double)h->es * ((double)h->ld[ds] * (kD + nb2) + n +
                                  (kp > 0 ? n : 0.0)));
}

// The data pass's z prologue (see hd_ctx::zpro).
void set_zpro(hd_ctx* h, int ds, PassArgs& a) {
  if (!h->zpro.use) return;
  a.zpro = 1;
  a.w = h->w;
  a.c = h->w + h->slot2;
  a.kp = h->zpro.kp;
  a.T = h->P[ds].T;
  a.tau = h->P[ds].tau;
  a.tmax = h->cfg.t_max;
  h->zpro.use = 0;
}

DynFuse no_dyn() {
  DynFuse d;
  std::memset(&d, 0, sizeof(d));
  return d;
}

// ---------------------------------------------------------- Haar query --

// Algorithm 2: data side D (R for y = Q x, L for y = Q' x) and random side G.
int haar_query(hd_ctx* h, int transpose, const void* x, void* y, int want_ysq,
               const DynFuse& dyn) {
  const int k = h->t;  // reflectors per side before this query
  const int step = k + 1;
  const int64_t n = h->cfg.n;
  const int ds = transpose ? 1 : 0;
  const int gs = 1 - ds;
  const double es = (double)h->es;
  int rc = resolve_pending(h, gs);
  if (rc) return rc;
  if (h->pf_step[gs] != step) {
    rc = prefetch(h, gs, k, step, k, 1);
    if (rc) return rc;
  }
  const Plan pl = plan_of(h, ds, step);
  rc = data_tdot(h, ds, x, k, 0);
  if (rc) return rc;
  // p = Delta_D (x - V_D z_D); new column k of V_D; prefetch for step+1;
  // then the scalars of R_t and L_t and the random side's coefficients
  {
    PassArgs a = pass_base(h, ds);
    a.k = k;
    a.z = h->zD;
    a.x = x;
    a.head = h->head;
    a.pivot = h->scal;
    a.pf = pl.pf_data ? 1 : 0;
    a.pf_step = (uint32_t)(step + 1);
    a.pf_cut = k + 1;
    a.cslot = pl.tcol && k > 0 ? h->slot2 : -1;
    set_zpro(h, ds, a);
    After want = after_of(ranges(0, pl.pf_data ? k + 1 : 0, h->slot2,
                                 a.cslot >= 0 ? k : 0, h->extra, kNumExtra),
                          h->P[ds].red, 2);
    HaarSmallArgs& hs = want.hs;
    hs.D = h->P[ds];
    hs.G = h->P[gs];
    hs.k = k;
    hs.tmax = h->cfg.t_max;
    hs.zG = h->zG;
    hs.head = h->head;
    hs.pivot = h->scal;
    hs.cscale = h->scal + 1;
    hs.key = Key{h->cfg.seed, h->cfg.trial};
    hs.step = (uint32_t)step;
    hs.extra = h->extra;
    hs.cslot = a.cslot;
    hs.flag = h->flag;
    rc = do_pass(h, ds, kPassData, a, want, 1,
                 es * ((double)h->ld[ds] * k + n + (n - k)));
    if (rc) return rc;
  }
  // y = (I - V_G T_G V_G') Delta_G w, w = [p[:k]; (nu/nu_G) g[k:]]
  {
    PassArgs a = pass_base(h, gs);
    a.partials = h->partials2;
    a.k = k;
    a.z = h->zG;
    a.head = h->head;
    a.cscale = h->scal + 1;
    a.y = dyn.kind && dyn.y_unused ? nullptr : y;
    a.step = (uint32_t)step;
    a.want_ysq = want_ysq;
    a.dyn = dyn;
    a.pf = pl.pf_rand ? 1 : 0;
    a.pf_step = (uint32_t)(step + 1);
    a.pf_cut = k + 1;
    a.wnext = pl.wnext && !pl.pf_rand && dyn.kind && dyn.next_input;
    After want =
        after_of(ranges(0, pl.pf_rand ? k + 1 : 0, h->extra,
                        (pl.pf_rand || want_ysq) ? kNumExtra : 0),
                 h->P[gs].red, 0);
    if (a.wnext) {
      want = after_of(ranges(0, k + 1), h->w, 0);
      h->wready = {1, step + 1, gs, k + 1, dyn.xnext};
    }
    {
      ProfScope ps(h, 2,
                   es * ((double)h->ld[gs] * k + (a.y ? n : 0) + (n - k) +
                         (dyn.kind ? 2.0 * n : 0.0)));
      LCHK(launch_pass(h->f64, h->sh[gs], kPassRandHaar, a, h->stream,
                       ps.ev));
    }
    defer_after(h, gs, want);
    if (want_ysq) {
      // ||y||^2 is read right after the query
      After none = after_of(ranges(0, 0), h->P[gs].red, 0);
      rc = run_after(h, gs, none);
      if (rc) return rc;
    }
  }
  h->t = step;
  h->r = step;
  h->l = step;
  h->pf_step[ds] = pl.pf_data ? step + 1 : 0;
  h->pf_step[gs] = pl.pf_rand ? step + 1 : 0;
  h->pending[ds] = pl.tcol ? -1 : k;
  return HD_OK;
}

// -------------------------------------------------------- Ginibre query --

// Algorithm 1.  The data side D (R for y = Q x, L for y = Q' x) gets a new
// reflector from p = D_k..D_1 x; the random side G answers
//   y = sigma sum_i (v_i' x) u_i
// with the implicit basis vectors of G (reflector products applied to the
// coefficients h = B_D' x of the TDOT pass) and the explicit ones in B[G]
// (coefficients = the head of p, because the data-type basis vectors are
// R_1..R_j e_j), and stores the new explicit vector (L..L Z g or R..R Z g).
int gin_query(hd_ctx* h, int transpose, const void* x, void* y,
              const DynFuse& dyn) {
  const int ds = transpose ? 1 : 0;
  const int gs = 1 - ds;
  const int kD = ds == 0 ? h->r : h->l;
  const int kG = ds == 0 ? h->l : h->r;
  const int step = h->t + 1;
  const int64_t nD = h->dim[ds], nG = h->dim[gs];
  const double es = (double)h->es;
  int rc = resolve_pending(h, gs);
  if (rc) return rc;
  if (kG > 0 && h->pf_step[gs] != step) {
    rc = prefetch(h, gs, kG, step, kG - 1, 0);
    if (rc) return rc;
  }
  const Plan pl = plan_of(h, ds, step);
  rc = data_tdot(h, ds, x, kD, kG);
  if (rc) return rc;
  bool spro = false;
  GinSmallArgs small;
  std::memset(&small, 0, sizeof(small));
  {
    PassArgs a = pass_base(h, ds);
    a.k = kD;
    a.z = h->zD;
    a.x = x;
    a.head = h->head;
    a.pivot = h->scal;
    a.pf = pl.pf_data ? 1 : 0;
    a.pf_step = (uint32_t)(step + 1);
    a.pf_cut = kD;
    a.cslot = pl.tcol && kD > 0 ? h->slot2 : -1;
    set_zpro(h, ds, a);
    After want = after_of(ranges(0, pl.pf_data ? kD + 1 : 0, h->slot2,
                                 a.cslot >= 0 ? kD : 0, h->extra, kNumExtra),
                          h->P[ds].red, 3);
    GinSmallArgs& gsa = want.gs;
    gsa.D = h->P[ds];
    gsa.G = h->P[gs];
    gsa.k = kD;
    gsa.l = kG;
    gsa.tmax = h->cfg.t_max;
    gsa.h = h->w + kD;
    gsa.z1 = h->zG;
    gsa.z2 = h->z2;
    gsa.pivot = h->scal;
    gsa.scal = h->gscal;
    gsa.D_extra = h->extra;
    gsa.cslot = a.cslot;
    gsa.flag = h->flag;
    // the reflector step runs as the random pass's prologue where its
    // shape allows (at most two chunks per workgroup, l within the LDS
    // arrays)
    spro = h->sh[gs].cpt <= 2 && kG <= kZproMax;
    if (spro) {
      small = gsa;
      want.op = 0;
    }
    rc = do_pass(h, ds, kPassData, a, want, 1,
                 es * ((double)h->ld[ds] * kD + nD + (nD - kD)));
    if (rc) return rc;
  }
  {
    GinPassArgs a;
    std::memset(&a, 0, sizeof(a));
    a.spro = spro ? 1 : 0;
    a.small = small;
    a.V = h->P[gs].V;
    a.ld = h->ld[gs];
    a.k = kG;
    a.z1 = h->zG;
    a.z2 = h->z2;
    a.pi = h->P[gs].pi;
    a.B = h->B[gs];
    a.nb = kD;
    a.c = h->head;
    a.h = h->w + kD;
    a.scal = h->gscal;
    a.n = nG;
    a.y = dyn.kind && dyn.y_unused ? nullptr : y;
    a.key = Key{h->cfg.seed, h->cfg.trial};
    a.step = (uint32_t)step;
    a.dyn = dyn;
    a.pf = pl.pf_rand ? 1 : 0;
    a.pf_step = (uint32_t)(step + 1);
    a.pf_cut = kG - 1;
    a.partials = h->partials2;
    a.pstride = h->pstride;
    a.extra = h->extra;
    a.wnext = pl.wnext && !pl.pf_rand && dyn.kind && dyn.next_input;
    After want = after_of(ranges(0, pl.pf_rand ? kG : 0), h->P[gs].red, 0);
    if (a.wnext) {
      // next query: data side gs with kG reflectors and kD + 1 basis columns
      want = after_of(ranges(0, kG + kD + 1), h->w, 0);
      h->wready = {1, step + 1, gs, kG + kD + 1, dyn.xnext};
    }
    {
      ProfScope ps(h, 2,
                   es * ((double)h->ld[gs] * (kG + kD) + (a.y ? 2.0 : 1.0) * nG +
                         (dyn.kind ? 2.0 * nG : 0.0)));
      LCHK(launch_gin_pass(h->f64, h->sh[gs], a, h->stream, ps.ev));
    }
    defer_after(h, gs, want);
  }
  h->t = step;
  if (ds == 0)
    h->r = kD + 1;
  else
    h->l = kD + 1;
  h->pending[ds] = pl.tcol ? -1 : kD;
  h->pf_step[ds] = pl.pf_data ? step + 1 : 0;
  h->pf_step[gs] = pl.pf_rand ? step + 1 : 0;
  return HD_OK;
}

int check_query(hd_ctx* h, int transpose, const void* x, const void* y) {
  if (!h || !x || !y || x == y) return HD_ERR_INVALID;
  if (h->t >= h->cfg.t_max) return HD_ERR_CAPACITY;
  if (h->cfg.ensemble == HD_GINIBRE) {
    // Algorithm 1 needs r <= n and l <= m
    const int kD = transpose ? h->l : h->r;
    if ((int64_t)kD >= h->dim[transpose ? 1 : 0]) return HD_ERR_CAPACITY;
  }
  return HD_OK;
}

int query(hd_ctx* h, int transpose, const void* x, void* y, int want_ysq,
          const DynFuse& dyn) {
  if (h->cfg.ensemble == HD_HAAR)
    return haar_query(h, transpose, x, y, want_ysq, dyn);
  return gin_query(h, transpose, x, y, dyn);
}

}  // namespace

// ------------------------------------------------------ checkpoint state --
//
// Layout of an exported state (host byte order): StateHeader, then for each
// side s = 0 (R), 1 (L): vcols[s] panel columns of dim[s] entries (storage
// type), T (t_max^2 FP64, column-major), tau, nu, pivot, sign (t_max FP64
// each), pi (t_max + 1 FP64), the reduced results of the side's last pass
// (pstride FP64); then, for the Gaussian ensemble, bcols[s] explicit basis
// columns of dim[s] entries per side.

namespace {

constexpr char kStateMagic[8] = {'H', 'D', 'S', 'T', 'A', 'T', 'E', '1'};

struct StateHeader {
  char magic[8];
  int32_t ensemble, storage, t_max, pstride;
  int64_t m, n;
  uint32_t seed, trial;
  double sigma;
  int32_t t, r, l, flag;
  int32_t pf_step[2], pending[2];
  int32_t vcols[2], bcols[2];
  uint64_t total_bytes;
};

size_t state_bytes(const StateHeader& H) {
  const size_t es = H.storage == HD_F64 ? 8 : 4;
  const size_t tm = (size_t)H.t_max;
  const int64_t dims[2] = {H.n, H.m};
  size_t b = sizeof(StateHeader);
  for (int s = 0; s < 2; ++s) {
    b += es * (size_t)dims[s] * (size_t)H.vcols[s];
    b += 8 * (tm * tm + 5 * tm + 1 + (size_t)H.pstride);
    b += es * (size_t)dims[s] * (size_t)H.bcols[s];
  }
  return b;
}

StateHeader header_of(const hd_ctx* h) {
  StateHeader H;
  std::memset(&H, 0, sizeof(H));
  std::memcpy(H.magic, kStateMagic, sizeof(kStateMagic));
  H.ensemble = h->cfg.ensemble;
  H.storage = h->cfg.storage;
  H.t_max = h->cfg.t_max;
  H.pstride = h->pstride;
  H.m = h->cfg.m;
  H.n = h->cfg.n;
  H.seed = h->cfg.seed;
  H.trial = h->cfg.trial;
  H.sigma = h->cfg.ensemble == HD_GINIBRE ? h->cfg.sigma : 0.0;
  H.t = h->t;
  H.r = h->r;
  H.l = h->l;
  for (int s = 0; s < 2; ++s) {
    H.pf_step[s] = h->pf_step[s];
    H.pending[s] = h->pending[s];
  }
  if (h->cfg.ensemble == HD_HAAR) {
    H.vcols[0] = H.vcols[1] = h->t;
  } else {
    // reflectors: R gets one per Q-query, L one per Q'-query; explicit
    // basis: B[0] holds v of Q'-queries, B[1] u of Q-queries
    H.vcols[0] = h->r;
    H.vcols[1] = h->l;
    H.bcols[0] = h->l;
    H.bcols[1] = h->r;
  }
  H.total_bytes = 0;
  H.total_bytes = state_bytes(H);
  return H;
}

// Copies `cols` columns of `rows` entries between a panel (leading dimension
// ld) and a packed host block, synchronously.
int copy_cols(void* dev, int64_t ld, char* host, int64_t rows, int cols,
              size_t es, bool to_host) {
  if (cols <= 0 || rows <= 0) return HD_OK;
  const size_t w = es * (size_t)rows;
  hipError_t e;
  if (to_host)
    e = hipMemcpy2D(host, w, dev, es * (size_t)ld, w, (size_t)cols,
                    hipMemcpyDeviceToHost);
  else
    e = hipMemcpy2D(dev, es * (size_t)ld, host, w, w, (size_t)cols,
                    hipMemcpyHostToDevice);
  return e == hipSuccess ? HD_OK : hip_fail(e);
}

int copy_block(void* dev, char* host, size_t bytes, bool to_host) {
  const hipError_t e =
      to_host ? hipMemcpy(host, dev, bytes, hipMemcpyDeviceToHost)
              : hipMemcpy(dev, host, bytes, hipMemcpyHostToDevice);
  return e == hipSuccess ? HD_OK : hip_fail(e);
}

// Moves every array of the state between the handle and `buf` (after the
// header), in the documented order.
int move_state(hd_ctx* h, const StateHeader& H, char* buf, bool to_host) {
  char* p = buf + sizeof(StateHeader);
  const size_t es = (size_t)h->es;
  const size_t tm = (size_t)h->cfg.t_max;
  int rc = HD_OK;
  for (int s = 0; s < 2 && !rc; ++s) {
    PanelDev& P = h->P[s];
    rc = copy_cols(P.V, P.ld, p, h->dim[s], H.vcols[s], es, to_host);
    p += es * (size_t)h->dim[s] * (size_t)H.vcols[s];
    void* arrays[6] = {P.T, P.tau, P.nu, P.piv, P.sgn, P.pi};
    const size_t sizes[6] = {tm * tm, tm, tm, tm, tm, tm + 1};
    for (int a = 0; a < 6 && !rc; ++a) {
      rc = copy_block(arrays[a], p, 8 * sizes[a], to_host);
      p += 8 * sizes[a];
    }
    if (!rc) rc = copy_block(P.red, p, 8 * (size_t)h->pstride, to_host);
    p += 8 * (size_t)h->pstride;
  }
  for (int s = 0; s < 2 && !rc; ++s) {
    if (H.bcols[s] <= 0) continue;
    rc = copy_cols(h->B[s], h->ld[s], p, h->dim[s], H.bcols[s], es, to_host);
    p += es * (size_t)h->dim[s] * (size_t)H.bcols[s];
  }
  return rc;
}

// Validation of a configuration (hd_init's rules).
int check_config(const hd_config* cfg) {
  if (cfg->ensemble != HD_GINIBRE && cfg->ensemble != HD_HAAR)
    return HD_ERR_INVALID;
  if (cfg->storage != HD_F32 && cfg->storage != HD_F64) return HD_ERR_INVALID;
  if (cfg->m <= 0 || cfg->n <= 0 || cfg->t_max < 1) return HD_ERR_INVALID;
  if (cfg->ensemble == HD_HAAR && cfg->m != cfg->n) return HD_ERR_INVALID;
  const int64_t cap = cfg->m < cfg->n ? cfg->m : cfg->n;
  if ((int64_t)cfg->t_max > cap) return HD_ERR_INVALID;
  if (cfg->ensemble == HD_GINIBRE && !(cfg->sigma > 0.0))
    return HD_ERR_INVALID;
  if (cfg->n > ((int64_t)1 << 40)) return HD_ERR_NOMEM;
  return HD_OK;
}

// Sizes, launch shapes and device buffers of a handle (zeroed by dalloc, or
// left for the caller to clear when carved).
int init_layout(hd_ctx* h, const hd_config* cfg) {
  h->cfg = *cfg;
  h->stream = (hipStream_t)cfg->stream;
  h->f64 = cfg->storage == HD_F64;
  h->es = h->f64 ? 8 : 4;
  const int64_t dims[2] = {cfg->n, cfg->m};
  h->dim[0] = cfg->n;
  h->dim[1] = cfg->m;
  const int tm = cfg->t_max;
  h->slot2 = (cfg->ensemble == HD_GINIBRE ? 2 * tm : tm) + 1;
  h->extra = h->slot2 + tm + 1;
  h->pstride = h->extra + kNumExtra;
  int maxwg = 1;
  for (int s = 0; s < 2; ++s) {
    h->ld[s] = round_up(dims[s], kChunk);
    h->sh[s] = pick_shape(cfg->ensemble, h->f64, dims[s], h->ld[s]);
    if (h->sh[s].nwg > maxwg) maxwg = h->sh[s].nwg;
  }
  int rc = HD_OK;
#define ALLOC(ptr, bytes)              \
  do {                                 \
    rc = dalloc(h, &(ptr), (bytes));   \
    if (rc != HD_OK) return rc;        \
  } while (0)
  for (int s = 0; s < 2; ++s) {
    PanelDev& P = h->P[s];
    P.ld = h->ld[s];
    ALLOC(P.V, (size_t)h->es * (size_t)h->ld[s] * (size_t)tm);
    ALLOC(P.T, sizeof(double) * (size_t)tm * tm);
    ALLOC(P.tau, sizeof(double) * tm);
    ALLOC(P.nu, sizeof(double) * tm);
    ALLOC(P.piv, sizeof(double) * tm);
    ALLOC(P.sgn, sizeof(double) * tm);
    ALLOC(P.pi, sizeof(double) * (tm + 1));
    ALLOC(P.red, sizeof(double) * h->pstride);
    h->pf_step[s] = 0;
    h->pending[s] = -1;
  }
  ALLOC(h->partials, sizeof(double) * (size_t)maxwg * h->pstride);
  ALLOC(h->partials2, sizeof(double) * (size_t)maxwg * h->pstride);
  h->red_half = red_stage_doubles(maxwg, h->pstride);
  ALLOC(h->red_stage, sizeof(double) * 2 * h->red_half);
  h->hint = -1;
  h->deferred = no_job();
  ALLOC(h->w, sizeof(double) * h->pstride);
  ALLOC(h->wc, sizeof(double) * h->pstride);
  ALLOC(h->zD, sizeof(double) * tm);
  ALLOC(h->zG, sizeof(double) * 3 * (size_t)tm);
  ALLOC(h->head, sizeof(double) * tm);
  ALLOC(h->scal, sizeof(double) * 8);
  ALLOC(h->gscal, sizeof(double) * 8);
  ALLOC(h->z2, sizeof(double) * (size_t)tm);
  if (cfg->ensemble == HD_GINIBRE) {
    for (int s = 0; s < 2; ++s)
      ALLOC(h->B[s], (size_t)h->es * (size_t)h->ld[s] * (size_t)tm);
  }
  ALLOC(h->flag, sizeof(int) * 4);
#undef ALLOC
  return HD_OK;
}

// The non-zero initial values: pi[0] = 1 on both sides, sigma.
int init_values(hd_ctx* h) {
  for (int s = 0; s < 3; ++s) {
    double* p = s < 2 ? h->P[s].pi : h->gscal + 1;
    const double v = s < 2 ? 1.0 : h->cfg.sigma;
    if (launch_fill(p, v, 1, h->stream) != 0) return HD_ERR_HIP;
  }
  return HD_OK;
}

}  // namespace

extern "C" {

const char* hd_strerror(int code) {
  switch (code) {
    case HD_OK: return "ok";
    case HD_ERR_INVALID: return "invalid argument";
    case HD_ERR_CAPACITY: return "capacity exhausted (t_max or min(m,n))";
    case HD_ERR_NOMEM: return "device allocation failed";
    case HD_ERR_HIP: return g_err[0] ? g_err : "HIP runtime error";
    case HD_ERR_NONFINITE: return "non-finite reflector norm";
    case HD_ERR_UNSUPPORTED: return "unsupported configuration";
    case HD_ERR_TOO_LARGE:
      return "problem exceeds the static scratch of the allocation-free "
             "entry point";
    default: return "unknown error";
  }
}

int hd_init(const hd_config* cfg, hd_handle* out) {
  if (!cfg || !out) return HD_ERR_INVALID;
  *out = nullptr;
  int rc = check_config(cfg);
  if (rc) return rc;
  hd_ctx* h = new (std::nothrow) hd_ctx();
  if (!h) return HD_ERR_NOMEM;
  rc = init_layout(h, cfg);
  if (!rc) rc = init_values(h);
  if (!rc && hipStreamSynchronize(h->stream) != hipSuccess)
    rc = hip_fail(hipGetLastError());
  if (rc) {
    free_all(h);
    delete h;
    return rc;
  }
  *out = h;
  return HD_OK;
}

int hd_free(hd_handle h) {
  if (!h) return HD_OK;
  free_all(h);
  delete h;
  return HD_OK;
}

int hd_reset(hd_handle h, uint32_t seed, uint32_t trial) {
  if (!h) return HD_ERR_INVALID;
  // Panel entries above each column's diagonal are never written, so they
  // are still zero; every other entry a query reads is rewritten before it
  // is read.  The host-side counters and the key change, and the sticky
  // device flag is cleared (stream-ordered) for the fresh matrix.
  LCHK(launch_zero(h->flag, sizeof(int) * 4, h->stream));
  h->cfg.seed = seed;
  h->cfg.trial = trial;
  h->t = h->r = h->l = 0;
  for (int s = 0; s < 2; ++s) {
    h->pf_step[s] = 0;
    h->pending[s] = -1;
  }
  h->hint = -1;
  h->deferred = no_job();
  h->wready.valid = 0;
  h->zpro.use = 0;
  return HD_OK;
}

int hd_set_stream(hd_handle h, void* stream) {
  if (!h) return HD_ERR_INVALID;
  h->stream = (hipStream_t)stream;
  return HD_OK;
}

int hd_step(hd_handle h, const void* x, void* y) {
  int rc = check_query(h, 0, x, y);
  if (rc) return rc;
  return query(h, 0, x, y, 0, no_dyn());
}

int hd_apply_T(hd_handle h, const void* x, void* y) {
  int rc = check_query(h, 1, x, y);
  if (rc) return rc;
  return query(h, 1, x, y, 0, no_dyn());
}

int hd_status(hd_handle h) {
  if (!h) return HD_ERR_INVALID;
  HIPC(hipStreamSynchronize(h->stream));
  int flag = 0;
  HIPC(hipMemcpy(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost));
  return flag ? HD_ERR_NONFINITE : HD_OK;
}

int hd_counts(hd_handle h, int32_t* t, int32_t* r, int32_t* l) {
  if (!h) return HD_ERR_INVALID;
  if (t) *t = h->t;
  if (r) *r = h->r;
  if (l) *l = h->l;
  return HD_OK;
}

int hd_export(hd_handle h, void* host_buf, size_t* size) {
  if (!h || !size) return HD_ERR_INVALID;
  const StateHeader H0 = header_of(h);
  if (!host_buf) {
    *size = (size_t)H0.total_bytes;
    return HD_OK;
  }
  if (*size < H0.total_bytes) {
    *size = (size_t)H0.total_bytes;
    return HD_ERR_INVALID;
  }
  // finish the deferred reduction of the last random pass, so that every
  // reduced result is in place
  if (h->deferred.rg.count[0] + h->deferred.rg.count[1] +
          h->deferred.rg.count[2] > 0) {
    LCHK(launch_reduce(h->deferred, no_job(), h->stream));
    h->deferred = no_job();
  }
  HIPC(hipStreamSynchronize(h->stream));
  StateHeader H = H0;
  int flag = 0;
  HIPC(hipMemcpy(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost));
  H.flag = flag;
  std::memcpy(host_buf, &H, sizeof(H));
  const int rc = move_state(h, H, (char*)host_buf, true);
  if (rc == HD_OK) *size = (size_t)H.total_bytes;
  return rc;
}

int hd_import(const hd_config* cfg, const void* host_buf, size_t size,
              hd_handle* out) {
  if (!cfg || !host_buf || !out) return HD_ERR_INVALID;
  *out = nullptr;
  if (size < sizeof(StateHeader)) return HD_ERR_INVALID;
  StateHeader H;
  std::memcpy(&H, host_buf, sizeof(H));
  if (std::memcmp(H.magic, kStateMagic, sizeof(kStateMagic)) != 0)
    return HD_ERR_INVALID;
  if (H.ensemble != cfg->ensemble || H.storage != cfg->storage ||
      H.t_max != cfg->t_max || H.m != cfg->m || H.n != cfg->n)
    return HD_ERR_INVALID;
  if (H.ensemble == HD_GINIBRE && H.sigma != cfg->sigma)
    return HD_ERR_INVALID;
  if (H.t < 0 || H.t > H.t_max || H.r < 0 || H.l < 0 || H.r > H.t ||
      H.l > H.t)
    return HD_ERR_INVALID;
  hd_config c = *cfg;
  c.seed = H.seed;
  c.trial = H.trial;
  hd_handle h = nullptr;
  int rc = hd_init(&c, &h);
  if (rc) return rc;
  // the header must describe exactly this handle's state arrays
  StateHeader want = header_of(h);
  want.t = H.t;
  want.r = H.r;
  want.l = H.l;
  if (H.ensemble == HD_HAAR) {
    want.vcols[0] = want.vcols[1] = H.t;
  } else {
    want.vcols[0] = want.bcols[1] = H.r;
    want.vcols[1] = want.bcols[0] = H.l;
  }
  want.total_bytes = 0;
  want.total_bytes = state_bytes(want);
  if (H.pstride != want.pstride || H.vcols[0] != want.vcols[0] ||
      H.vcols[1] != want.vcols[1] || H.bcols[0] != want.bcols[0] ||
      H.bcols[1] != want.bcols[1] || H.total_bytes != want.total_bytes ||
      size < H.total_bytes) {
    hd_free(h);
    return HD_ERR_INVALID;
  }
  for (int s = 0; s < 2; ++s)
    if (H.pending[s] < -1 || H.pending[s] >= H.vcols[s] || H.pf_step[s] < 0) {
      hd_free(h);
      return HD_ERR_INVALID;
    }
  rc = move_state(h, H, (char*)host_buf, false);
  if (!rc && hipMemcpy(h->flag, &H.flag, sizeof(int),
                       hipMemcpyHostToDevice) != hipSuccess)
    rc = hip_fail(hipGetLastError());
  if (rc) {
    hd_free(h);
    return rc;
  }
  h->t = H.t;
  h->r = H.r;
  h->l = H.l;
  for (int s = 0; s < 2; ++s) {
    h->pf_step[s] = H.pf_step[s];
    h->pending[s] = H.pending[s];
  }
  *out = h;
  return HD_OK;
}

int hd_pivots(hd_handle h, int32_t side, int32_t count, double* nu,
              double* pivot, int32_t* sign) {
  if (!h || (side != 0 && side != 1) || count < 0) return HD_ERR_INVALID;
  const int have = side == 0 ? h->r : h->l;
  if (count > have) return HD_ERR_INVALID;
  if (count == 0) return HD_OK;
  HIPC(hipStreamSynchronize(h->stream));
  const PanelDev& P = h->P[side];
  if (nu)
    HIPC(hipMemcpy(nu, P.nu, sizeof(double) * count, hipMemcpyDeviceToHost));
  if (pivot)
    HIPC(hipMemcpy(pivot, P.piv, sizeof(double) * count,
                   hipMemcpyDeviceToHost));
  if (sign) {
    std::vector<double> s(count);
    HIPC(hipMemcpy(s.data(), P.sgn, sizeof(double) * count,
                   hipMemcpyDeviceToHost));
    for (int i = 0; i < count; ++i) sign[i] = s[i] < 0 ? -1 : 1;
  }
  return HD_OK;
}

// hd_run after its argument checks: T steps of a built-in map (every map,
// including the normalising one that hd_run refuses).
static int run_dynamics(hd_handle h, const hd_dynamics* dyn, int32_t T,
                        const void* x1, const void* x0, void* x_out,
                        void* traj_x, void* traj_y) {
  if (dyn->pattern != HD_PATTERN_Q && dyn->pattern != HD_PATTERN_ALT)
    return HD_ERR_INVALID;
  if ((int64_t)h->t + T > h->cfg.t_max) return HD_ERR_CAPACITY;
  if (h->cfg.ensemble == HD_GINIBRE) {
    int nq = 0;
    for (int t = 1; t <= T; ++t)
      nq += !(dyn->pattern == HD_PATTERN_ALT && t % 2 == 0);
    if ((int64_t)h->r + nq > h->cfg.n || (int64_t)h->l + (T - nq) > h->cfg.m)
      return HD_ERR_CAPACITY;
  }
  const int64_t n = h->cfg.n;
  const size_t vb = (size_t)h->es * (size_t)n;
  if (!traj_x && !h->ring[0]) {
    for (int i = 0; i < 3; ++i) {
      int rc = dalloc(h, &h->ring[i], vb);
      if (rc) return rc;
    }
  }
  if (!traj_y && !h->ybuf) {
    int rc = dalloc(h, &h->ybuf, vb);
    if (rc) return rc;
  }
  if (!x0 && !h->zeros) {
    int rc = dalloc(h, &h->zeros, vb);
    if (rc) return rc;
  }
  auto xrow = [&](int t) -> void* {  // x_t, t = 1..T+1
    if (traj_x) return (char*)traj_x + (size_t)(t - 1) * vb;
    return h->ring[(t - 1) % 3];
  };
  const void* xprev0 = x0 ? x0 : h->zeros;
  if (xrow(1) != x1)
    HIPC(hipMemcpyAsync(xrow(1), x1, vb, hipMemcpyDeviceToDevice, h->stream));
  for (int t = 1; t <= T; ++t) {
    const int transpose = (dyn->pattern == HD_PATTERN_ALT && t % 2 == 0);
    void* y = traj_y ? (char*)traj_y + (size_t)(t - 1) * vb : h->ybuf;
    const void* xprev = t == 1 ? xprev0 : xrow(t - 1);
    h->hint = t < T ? (dyn->pattern == HD_PATTERN_ALT && (t + 1) % 2 == 0)
                    : kHintNone;
    DynFuse fz = no_dyn();
    if (dyn->kind == HD_DYN_TANH || dyn->kind == HD_DYN_SOFT_HIST) {
      // element-wise maps run in the random-side pass epilogue
      fz.kind = dyn->kind;
      fz.a = dyn->a;
      fz.b = dyn->b;
      fz.x = xrow(t);
      fz.xprev = xprev;
      fz.xnext = xrow(t + 1);
      fz.next_input = t < T;
      // the internal buffer's answers are read by nobody
      fz.y_unused = traj_y == nullptr;
    }
    int rc = query(h, transpose, xrow(t), y, dyn->kind == HD_DYN_NORMALIZE,
                   fz);
    h->hint = -1;
    if (rc) return rc;
    if (fz.kind) continue;
    DynArgs d;
    d.kind = dyn->kind;
    d.a = dyn->a;
    d.b = dyn->b;
    d.y = y;
    d.x = xrow(t);
    d.xprev = t == 1 ? xprev0 : xrow(t - 1);
    d.xnext = xrow(t + 1);
    d.n = n;
    d.ysq = h->P[transpose ? 0 : 1].red + h->extra + kSlotYSQ;
    LCHK(launch_dyn(h->f64, d, h->stream));
  }
  if (x_out && T >= 0 && x_out != xrow(T + 1))
    HIPC(hipMemcpyAsync(x_out, xrow(T + 1), vb, hipMemcpyDeviceToDevice,
                        h->stream));
  return HD_OK;
}

int hd_run(hd_handle h, const hd_dynamics* dyn, int32_t T, const void* x1,
           const void* x0, void* x_out, void* traj_x, void* traj_y) {
  if (!h || !dyn || !x1 || T < 0) return HD_ERR_INVALID;
  if (h->cfg.m != h->cfg.n) return HD_ERR_INVALID;
  if (dyn->kind < HD_DYN_TANH || dyn->kind > HD_DYN_NORMALIZE)
    return HD_ERR_INVALID;
  // The normalising map is switched off: its one run on the GPU ended in a
  // memory-aperture fault whose cause has not been shown (the CPU emulation
  // of exactly this path in tests/emu is clean and matches the oracle).  It
  // stays off until a cause is found.
  if (dyn->kind == HD_DYN_NORMALIZE) return HD_ERR_UNSUPPORTED;
  return run_dynamics(h, dyn, T, x1, x0, x_out, traj_x, traj_y);
}

// Work buffers of the unrolled-ISTA entry points, allocated on first use.
static int ista_buffers(hd_ctx* h) {
  if (h->ista[0]) return HD_OK;
  const int64_t len = h->cfg.m > h->cfg.n ? h->cfg.m : h->cfg.n;
  for (int i = 0; i < 6; ++i) {
    int rc = dalloc(h, &h->ista[i], (size_t)h->es * (size_t)len);
    if (rc) return rc;
  }
  return dalloc(h, &h->ista_part, sizeof(double) * 2 * 1024);
}

// Room for `nq` more queries, pq of them Q-queries (Ginibre also needs
// r <= n and l <= m).
int hd_goe_step(hd_handle h, const void* x, void* y) {
  if (!h || !x || !y || x == y) return HD_ERR_INVALID;
  if (h->cfg.ensemble != HD_GINIBRE || h->cfg.m != h->cfg.n)
    return HD_ERR_INVALID;
  if (h->t + 2 > h->cfg.t_max) return HD_ERR_CAPACITY;
  if ((int64_t)h->r >= h->dim[0] || (int64_t)h->l >= h->dim[1])
    return HD_ERR_CAPACITY;
  int rc = ista_buffers(h);  // two work vectors: Q x and Q' x
  if (rc) return rc;
  void* qx = h->ista[0];
  void* qtx = h->ista[1];
  h->hint = 1;
  rc = query(h, 0, x, qx, 0, no_dyn());
  h->hint = -1;
  if (rc) return rc;
  // y = (Q x + Q' x) / sqrt(2), formed in the second query's epilogue
  DynFuse f = no_dyn();
  f.kind = kDynAxpy;
  f.a = -M_SQRT1_2;
  f.b = M_SQRT1_2;
  f.x = qx;
  f.xnext = y;
  return query(h, 1, x, qtx, 0, f);
}

int hd_usv_step(hd_handle U, hd_handle V, const void* s, int32_t transpose,
                const void* x, void* y) {
  if (!U || !V || U == V || !s || !x || !y || x == y) return HD_ERR_INVALID;
  if (transpose != 0 && transpose != 1) return HD_ERR_INVALID;
  if (U->cfg.ensemble != HD_HAAR || V->cfg.ensemble != HD_HAAR ||
      U->cfg.storage != V->cfg.storage || U->stream != V->stream)
    return HD_ERR_INVALID;
  // y = U (S (V x)), or y = V' (S' (U' x)) with S = diag(s) in R^{m x n}:
  // the first handle's query forms the first min(m, n) entries of S times
  // its answer in its epilogue (into the second handle's work vector, whose
  // other entries are zero), the second answers that
  hd_ctx* first = transpose ? U : V;
  hd_ctx* second = transpose ? V : U;
  if (first->t >= first->cfg.t_max || second->t >= second->cfg.t_max)
    return HD_ERR_CAPACITY;
  int rc = ista_buffers(first);
  if (!rc) rc = ista_buffers(second);
  if (rc) return rc;
  const int64_t d1 = first->cfg.n, d2 = second->cfg.n;
  const int64_t p = d1 < d2 ? d1 : d2;
  void* mid = second->ista[1];
  if (d2 > d1)
    LCHK(launch_zero((char*)mid + (size_t)first->es * (size_t)d1,
                     (size_t)first->es * (size_t)(d2 - d1), first->stream));
  DynFuse f = no_dyn();
  f.kind = kDynScale;
  f.x = s;
  f.len = p;
  f.xnext = mid;
  rc = query(first, transpose, x, first->ista[0], 0, f);
  if (rc) return rc;
  return query(second, transpose, mid, y, 0, no_dyn());
}

int hd_spectral_power(hd_handle h, int64_t n, const void* xi, const void* x1,
                      int32_t K, double scale, void* z, void* X) {
  if (!h || !xi || !x1 || K < 0 || n < 1) return HD_ERR_INVALID;
  if (h->cfg.ensemble != HD_HAAR || n >= h->cfg.n || !std::isfinite(scale))
    return HD_ERR_INVALID;
  if (z == xi || X == xi || (X && X == z)) return HD_ERR_INVALID;
  if ((int64_t)h->t + 1 + 2 * (int64_t)K > h->cfg.t_max)
    return HD_ERR_CAPACITY;
  int rc = ista_buffers(h);  // six work vectors of m entries
  if (rc) return rc;
  const int64_t m = h->cfg.n;
  const size_t es = (size_t)h->es;
  void* pad[2] = {h->ista[0], h->ista[5]};  // query inputs [x; 0]
  void* wts = h->ista[1];                     // y = tanh|A' xi|
  void* u = h->ista[2];
  void* w = h->ista[3];
  void* v = h->ista[4];
  // [xi; 0]; the tail stays zero in both input buffers (the head-keeping
  // map writes zeros there)
  LCHK(launch_zero((char*)pad[0] + es * (size_t)n, es * (size_t)(m - n),
                   h->stream));
  HIPC(hipMemcpyAsync(pad[0], xi, es * (size_t)n, hipMemcpyDeviceToDevice,
                      h->stream));
  // the measurements: A' xi = Q' [xi; 0], and y = tanh|A' xi| in the
  // epilogue
  DynFuse f0 = no_dyn();
  f0.kind = kDynTanhAbs;
  f0.a = 1.0;
  f0.xnext = wts;
  h->hint = K > 0 ? 1 : kHintNone;
  rc = query(h, 1, pad[0], z ? z : u, 0, f0);
  if (rc == HD_OK && K > 0) {
    rc = hipMemcpyAsync(pad[0], x1, es * (size_t)n, hipMemcpyDeviceToDevice,
                        h->stream) == hipSuccess ? HD_OK
                                                 : hip_fail(hipGetLastError());
    if (rc == HD_OK && X &&
        hipMemcpyAsync(X, x1, es * (size_t)n, hipMemcpyDeviceToDevice,
                       h->stream) != hipSuccess)
      rc = hip_fail(hipGetLastError());
  }
  for (int k = 0; k < K && rc == HD_OK; ++k) {
    // u = Q' [x_k; 0], then w = y .* u (epilogue)
    DynFuse fa = no_dyn();
    fa.kind = kDynScale;
    fa.x = wts;
    fa.xnext = w;
    fa.next_input = 1;
    h->hint = 0;
    rc = query(h, 1, pad[k & 1], u, 0, fa);
    if (rc) break;
    // v = Q w; x_{k+1} = scale * v[:n] (epilogue: the next input [x; 0]
    // and the row of X)
    DynFuse fb = no_dyn();
    fb.kind = kDynHead;
    fb.a = scale;
    fb.len = n;
    fb.xnext = pad[(k + 1) & 1];
    fb.aux = X ? (void*)((char*)X + es * (size_t)n * (size_t)(k + 1)) : v;
    fb.next_input = k + 1 < K;
    h->hint = k + 1 < K ? 1 : kHintNone;
    rc = query(h, 0, w, v, 0, fb);
  }
  h->hint = -1;
  return rc;
}

static int ista_room(const hd_ctx* h, int nq, int pq) {
  if ((int64_t)h->t + nq > h->cfg.t_max) return HD_ERR_CAPACITY;
  if (h->cfg.ensemble == HD_GINIBRE &&
      ((int64_t)h->r + pq > h->cfg.n || (int64_t)h->l + (nq - pq) > h->cfg.m))
    return HD_ERR_CAPACITY;
  return HD_OK;
}

int hd_lista_forward(hd_handle h, int32_t L, const float* a,
                     const float* theta, const void* yobs, void* X, void* U,
                     void* V) {
  if (!h || L < 1 || !a || !theta || !yobs || !X || !U || !V)
    return HD_ERR_INVALID;
  int rc = ista_room(h, 2 * L, L);
  if (rc) return rc;
  rc = ista_buffers(h);
  if (rc) return rc;
  const size_t vn = (size_t)h->es * (size_t)h->cfg.n;
  void* r = h->ista[0];
  void* res = h->ista[1];
  for (int t = 0; t < L; ++t) {
    const void* xt = (const char*)X + vn * t;
    // y - Q x_t, fused into the Q-query's epilogue
    DynFuse f1 = no_dyn();
    f1.kind = kDynResidual;
    f1.x = yobs;
    f1.xnext = res;
    f1.next_input = 1;
    h->hint = 1;
    rc = query(h, 0, xt, r, 0, f1);
    if (rc) break;
    // u_t = Q'(y - Q x_t); v_t = x_t + a_t u_t; x_{t+1} = soft(v_t, theta_t)
    DynFuse f2 = no_dyn();
    f2.kind = kDynLista;
    f2.a = a[t];
    f2.b = theta[t];
    f2.x = xt;
    f2.xnext = (char*)X + vn * (t + 1);
    f2.aux = (char*)V + vn * t;
    f2.next_input = t + 1 < L;
    h->hint = t + 1 < L ? 0 : -1;
    rc = query(h, 1, res, (char*)U + vn * t, 0, f2);
    if (rc) break;
  }
  h->hint = -1;
  return rc;
}

int hd_lista_backward(hd_handle h, int32_t L, const float* a,
                      const float* theta, const void* U, const void* V,
                      const void* g, double* grad_a, double* grad_theta,
                      void* g_x1) {
  if (!h || L < 1 || !a || !theta || !U || !V || !g || !grad_a ||
      !grad_theta)
    return HD_ERR_INVALID;
  const int pairs = L - 1 + (g_x1 ? 1 : 0);
  int rc = ista_room(h, 2 * pairs, pairs);
  if (rc) return rc;
  rc = ista_buffers(h);
  if (rc) return rc;
  const int64_t n = h->cfg.n;
  const size_t vn = (size_t)h->es * (size_t)n;
  void* gbar = h->ista[2];
  void* q = h->ista[3];
  void* w = h->ista[4];
  void* gnext = h->ista[5];
  const void* gcur = g;
  for (int t = L - 1; t >= 0; --t) {
    ListaAdjArgs k;
    k.g = gcur;
    k.v = (const char*)V + vn * t;
    k.u = (const char*)U + vn * t;
    k.gbar = gbar;
    k.theta = theta[t];
    k.n = n;
    k.part = h->ista_part;
    LCHK(launch_lista_adj(h->f64, k, grad_a + t, grad_theta + t, h->stream));
    if (t == 0 && !g_x1) break;
    // dL/dx_t = gbar - a_t Q'Q gbar: two more queries on the same Q
    h->hint = 1;
    rc = query(h, 0, gbar, q, 0, no_dyn());
    if (rc) break;
    DynFuse f = no_dyn();
    f.kind = kDynAxpy;
    f.a = a[t];
    f.b = 1.0;
    f.x = gbar;
    f.xnext = t == 0 ? g_x1 : gnext;
    h->hint = t > 0 && (t > 1 || g_x1) ? 0 : -1;
    rc = query(h, 1, q, w, 0, f);
    if (rc) break;
    gcur = gnext;
  }
  h->hint = -1;
  return rc;
}

int hd_autotune(int32_t ensemble, int32_t storage, const int64_t* lengths,
                int32_t count, int32_t k, void* stream, double* report) {
  if (ensemble != HD_GINIBRE && ensemble != HD_HAAR) return HD_ERR_INVALID;
  if (storage != HD_F32 && storage != HD_F64) return HD_ERR_INVALID;
  if (!lengths || count < 1 || k < 2) return HD_ERR_INVALID;
  for (int i = 0; i < count; ++i)
    if (lengths[i] < k || lengths[i] > ((int64_t)1 << 31)) return HD_ERR_INVALID;
  const int f64 = storage == HD_F64;
  const int cands[3] = {1, 2, 4};
  std::vector<std::pair<int64_t, int>> table;
  for (int i = 0; i < count; ++i) {
    const int64_t n = lengths[i];
    hd_config cfg;
    std::memset(&cfg, 0, sizeof(cfg));
    cfg.ensemble = ensemble;
    cfg.storage = storage;
    cfg.m = cfg.n = n;
    cfg.t_max = k;
    cfg.sigma = 1.0 / std::sqrt((double)n);
    cfg.stream = stream;
    g_force_cpt = 1;
    hd_handle h = nullptr;
    int rc = hd_init(&cfg, &h);
    g_force_cpt = 0;
    if (rc) return rc;
    void* x1 = nullptr;
    rc = dalloc(h, &x1, (size_t)h->es * (size_t)n);
    // any finite nonzero start vector: every byte 0x3F
    if (!rc && hipMemsetAsync(x1, 0x3F, (size_t)h->es * (size_t)n,
                              h->stream) != hipSuccess)
      rc = hip_fail(hipGetLastError());
    // Haar: queries with Q only; Gaussian: Q and Q' alternating, so both
    // sides grow
    hd_dynamics dyn;
    dyn.kind = HD_DYN_TANH;
    dyn.pattern = ensemble == HD_HAAR ? HD_PATTERN_Q : HD_PATTERN_ALT;
    dyn.a = 1.0;
    dyn.b = 0.5;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc && (hipEventCreate(&e0) != hipSuccess ||
                hipEventCreate(&e1) != hipSuccess))
      rc = hip_fail(hipGetLastError());
    double best = 0.0, rule_us = 0.0;
    int best_cpt = 1;
    for (int c = 0; c < 3 && !rc; ++c) {
      for (int s = 0; s < 2; ++s) h->sh[s] = shape_of(h->ld[s], cands[c]);
      // one untimed trajectory, then three timed ones (each a fresh Q)
      float ms = 0.f;
      for (int rep = 0; rep < 4 && !rc; ++rep) {
        rc = hd_reset(h, 0, (uint32_t)rep);
        if (!rc && rep == 1 && hipEventRecord(e0, h->stream) != hipSuccess)
          rc = hip_fail(hipGetLastError());
        if (!rc) rc = hd_run(h, &dyn, k, x1, nullptr, nullptr, nullptr, nullptr);
      }
      if (!rc && hipEventRecord(e1, h->stream) != hipSuccess)
        rc = hip_fail(hipGetLastError());
      if (!rc && hipEventSynchronize(e1) != hipSuccess)
        rc = hip_fail(hipGetLastError());
      if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        rc = hip_fail(hipGetLastError());
      const double us = 1e3 * ms / 3.0;
      if (report) report[3 * i + c] = us;
      if (cands[c] == dim_rule(n)) rule_us = us;
      if (!rc && (c == 0 || us < best)) {
        best = us;
        best_cpt = cands[c];
      }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    hd_free(h);
    if (rc) return rc;
    // keep the built-in shape unless another is clearly faster (ties are
    // run-to-run noise, and the built-in shape keeps the fused prologues
    // where the trajectory timed here does not exercise them all)
    const int rule = dim_rule(n);
    if (best_cpt != rule && best > (1.0 - kTuneMargin) * rule_us)
      best_cpt = rule;
    table.push_back({n, best_cpt});
  }
  std::sort(table.begin(), table.end());
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tuned[ensemble == HD_HAAR ? 1 : 0][f64] = table;
  return HD_OK;
}

int hd_shape_rule(int32_t ensemble, int32_t storage, int64_t n, int32_t* cpt) {
  if (ensemble != HD_GINIBRE && ensemble != HD_HAAR) return HD_ERR_INVALID;
  if ((storage != HD_F32 && storage != HD_F64) || n < 1 || !cpt)
    return HD_ERR_INVALID;
  const int64_t ld = round_up(n, kChunk);
  *cpt = pick_shape(ensemble, storage == HD_F64, n, ld).cpt;
  return HD_OK;
}

int hd_autotune_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  for (auto& e : g_tuned)
    for (auto& t : e) t.clear();
  return HD_OK;
}

}  // extern "C"

// ------------------------------------------------ allocation-free run --
//
// hd_run_noalloc carries a whole handle (panels, FP64 scalars, partial-sum
// rows, trajectory vectors) in one file-scope device array per GPU instead of
// hipMalloc'd buffers.  The array is reached through the address
// hipGetSymbolAddress reports for the current device (the array's name is
// only a host-side stand-in in host code).

namespace {

constexpr size_t kScratchBytes = (size_t)HD_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// The device address of `scratch` on the current device, looked up once per
// device.
int scratch_base(void** out) {
  int dev = -1;
  HIPC(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return HD_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPC(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return HD_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HD_OK;
}

// Lays out a handle for cfg plus hd_run's internal vectors (a ring of three
// x_t, y_t and the zero x_0) in the carve region of h.
int noalloc_layout(hd_ctx* h, const hd_config* cfg) {
  int rc = init_layout(h, cfg);
  if (rc) return rc;
  const size_t vb = (size_t)h->es * (size_t)cfg->n;
  for (int i = 0; i < 3 && !rc; ++i) rc = dalloc(h, &h->ring[i], vb);
  if (!rc) rc = dalloc(h, &h->ybuf, vb);
  if (!rc) rc = dalloc(h, &h->zeros, vb);
  return rc;
}

}  // namespace

extern "C" {

int hd_noalloc_scratch_bytes(const hd_config* cfg, size_t* bytes) {
  if (!cfg || !bytes) return HD_ERR_INVALID;
  int rc = check_config(cfg);
  if (rc) return rc;
  hd_ctx h{};
  h.carve.active = 1;
  h.carve.base = nullptr;
  h.carve.used = 0;
  h.carve.cap = ~(size_t)0;
  rc = noalloc_layout(&h, cfg);
  if (rc) return rc;
  *bytes = h.carve.used;
  return HD_OK;
}

int hd_run_noalloc(const hd_config* cfg, const hd_dynamics* dyn, int32_t T,
                   const void* x1, const void* x0, void* x_out, void* traj_x,
                   void* traj_y) {
  if (!cfg || !dyn || !x1 || T < 0) return HD_ERR_INVALID;
  int rc = check_config(cfg);
  if (rc) return rc;
  if (cfg->m != cfg->n) return HD_ERR_INVALID;
  size_t need = 0;
  rc = hd_noalloc_scratch_bytes(cfg, &need);
  if (rc) return rc;
  if (need > kScratchBytes) return HD_ERR_TOO_LARGE;
  void* base = nullptr;
  rc = scratch_base(&base);
  if (rc) return rc;
  hd_ctx h{};
  h.carve.active = 1;
  h.carve.base = (char*)base;
  h.carve.used = 0;
  h.carve.cap = kScratchBytes;
  rc = noalloc_layout(&h, cfg);
  if (rc) return rc == HD_ERR_NOMEM ? HD_ERR_TOO_LARGE : rc;
  // every call starts from a cleared region: the panels' rows above each
  // column's diagonal and beyond n must be zero, and the previous call's
  // contents are still there
  LCHK(launch_zero(base, (h.carve.used + 3) / 4 * 4, h.stream));
  rc = init_values(&h);
  if (rc) return rc;
  return hd_run(&h, dyn, T, x1, x0, x_out, traj_x, traj_y);
}

int hd_profile(hd_handle h, int32_t enable) {
  if (!h) return HD_ERR_INVALID;
  HIPC(hipStreamSynchronize(h->stream));
  h->prof = enable ? 1 : 0;
  if (enable) {
    h->recs.clear();
    h->pool_used = 0;
  }
  return HD_OK;
}

int hd_profile_read(hd_handle h, int32_t kind, double* ms, int64_t* launches,
                    double* bytes) {
  if (!h) return HD_ERR_INVALID;
  HIPC(hipStreamSynchronize(h->stream));
  double tot = 0.0, by = 0.0;
  int64_t cnt = 0;
  for (const ProfRec& r : h->recs) {
    if (r.kind != kind) continue;
    float e = 0.f;
    HIPC(hipEventElapsedTime(&e, r.a, r.b));
    tot += e;
    by += r.bytes;
    ++cnt;
  }
  if (ms) *ms = tot;
  if (launches) *launches = cnt;
  if (bytes) *bytes = by;
  return HD_OK;
}

}  // extern "C"
