// Internal interfaces between the C-ABI runtime (hd_api.hip) and the kernel
// launchers (hd_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hd {

constexpr int kWG = 256;  // threads per workgroup (4 waves of 64)
constexpr int kWaves = kWG / 64;
constexpr int kChunk = kWG * 4;  // panel row padding quantum (1024 rows)

// Layout of the per-workgroup partial-sum rows and of the reduced vectors.
// A row has `pstride` doubles: slots [0, slot2) hold the column dots with the
// first right-hand side, [slot2, extra) those with the second one, and
// extra + ExtraSlot the scalar extras below.
enum ExtraSlot {
  kSlotSS = 0,    // sum over rows > k of fl(new column)^2
  kSlotPFSS = 1,  // sum over rows > cut of fl(g_next)^2 (prefetch)
  kSlotYSQ = 2,   // sum of y_i^2 (for normalising dynamics)
  kNumExtra = 4
};

// Up to three ranges [start, start + count) of slots.
struct SlotRanges {
  int start[3];
  int count[3];
};

struct Key {
  uint32_t k0, k1;
};

// Per-side device state of the compact-WY representation.
struct PanelDev {
  void* V;        // ld x t_max, column-major
  int64_t ld;
  double* T;      // t_max x t_max upper triangular (column-major)
  double* tau;    // t_max
  double* nu;     // t_max: norm of the vector the reflector was built from
  double* piv;    // t_max: its first entry
  double* sgn;    // t_max: sign s
  double* pi;     // t_max + 1: pi[j] = prod_{l<j} (-s_l), pi[0] = 1
  double* red;    // pstride: reduced results of the last pass over the panel
};

// Completes column kp of a panel's T factor from c = V[:, :kp]' u_kp
// (T[:kp, kp] = -tau_kp T[:kp, :kp] c), then z = T' w for the leading k x k
// block when w is given.
struct SmallDataArgs {
  double* T;
  const double* tau;
  int tmax;
  int kp;           // pending column, or -1
  const double* c;  // kp dots
  int k;
  const double* w;  // k dots, or null
  double* z;        // out (k)
};

struct HaarSmallArgs {
  PanelDev D, G;
  int k;
  int tmax;
  double* zG;       // out: coefficients for the random-side pass (k);
                    // zG + tmax and zG + 2 tmax are scratch
  const double* head;
  const double* pivot;
  double* cscale;   // out: nu / nu_G
  Key key;
  uint32_t step;
  int extra;
  int cslot;        // >= 0: complete T_D column k from D.red[cslot..] (the
                    // data pass's dots of V_D[:, :k] with rows > k of u_k)
  int* flag;
};

// Scalars of the data-side reflector and the coefficients of the random side
// of a Ginibre query.
struct GinSmallArgs {
  PanelDev D, G;
  int k;            // data-side reflectors before this query
  int l;            // random-side reflectors
  int tmax;
  const double* h;  // l coefficients of the implicit random-side basis
  double* z1;       // out (l); z1 + tmax, z1 + 2 tmax are scratch
  double* z2;       // out (l)
  const double* pivot;
  double* scal;     // out: [0] nu; [1] sigma (set by the host)
  int D_extra;      // offset of the extra slots in D.red
  int cslot;        // >= 0: complete T_D column k (as in HaarSmallArgs)
  int* flag;
};

// Element-wise map fused into the random-side epilogue (kind 0: none):
// the built-in f_t, or a piece of an unrolled ISTA layer (eq. (ista) with a
// learned step a and threshold b per layer).
enum DynKind {
  kDynNone = 0,
  kDynTanh = 1,      // xnext = tanh(a y) + b x
  kDynSoftHist = 2,  // xnext = soft(y, a) + b xprev
  kDynNormalize = 3, // (unfused; see k_dyn)
  kDynResidual = 4,  // xnext = x - y                (x: the observation)
  kDynLista = 5,     // aux = v = x + a y; xnext = soft(v, b)
  kDynAxpy = 6,      // xnext = b x - a y
  kDynScale = 7,     // xnext = x y (x: a diagonal, entrywise); with
                     // len > 0 only rows < len (x and xnext of len rows)
  kDynTanhAbs = 8,   // xnext = a tanh(|y|)
  kDynHead = 9       // xnext = a y on rows < len, 0 below; aux = a y on
                     // rows < len (a vector of len entries)
};

struct DynFuse {
  int kind;
  double a, b;
  const void* x;      // x_t
  const void* xprev;  // x_{t-1}
  void* xnext;        // x_{t+1}
  void* aux;          // second output (kDynLista, kDynHead)
  int64_t len;        // kDynHead: rows kept; kDynScale: rows written
  int next_input;     // host only: xnext is the next query's input
  int y_unused;       // host only: nothing reads the answer y afterwards, so
                      // the pass that fuses the map does not store it
};

// Partial dots of panel columns with a right-hand side b (from memory, or the
// Philox draw of `gen_step` when gen != 0), over rows r with lo < r < n
// (lo = -1 for all rows).  Two column segments share the rows.  When b2 is
// set, the columns of the first segment are also dotted with b2 (a stored
// panel column), into slots slot2 + j.
struct TdotArgs {
  const void* V;
  int64_t ld;
  int ncols;
  const void* V2;
  int ncols2;
  const void* b;
  const void* b2;
  int slot2;
  int gen;
  Key key;
  uint32_t gen_step;
  int64_t lo;
  int64_t n;
  int want_ss;  // also sum of fl(b_i)^2 -> slot extra + kSlotPFSS
  double* partials;
  int pstride;
  int extra;
};

// One GEMV-N pass over a panel (columns 0..k-1) producing an output vector,
// writing the new column k, and the fused prefetch dots of columns 0..k with
// the next draw over rows > pf_cut.
enum PassMode { kPassData = 0, kPassRandHaar = 1 };

struct PassArgs {
  void* V;
  int64_t ld;
  int k;
  const double* z;   // k coefficients
  const double* pi;  // prefix sign products pi[0..k]
  int64_t n;
  // data mode, z from a prologue (zpro): every workgroup forms
  // z = T' w itself (with T column kp from the dots c when kp > 0; block 0
  // stores that column), instead of reading z
  int zpro;
  const double* w;
  const double* c;
  int kp;
  double* T;
  const double* tau;
  int tmax;
  // data mode: out = Delta (x - V z)
  const void* x;
  double* head;   // rows < k of the output (FP64)
  double* pivot;  // row k of the output (FP64)
  int cslot;      // >= 0: also the dots of columns 0..k-1 with rows > k of
                  // the new column (a second sweep), into slots cslot + j
  // random (Haar) mode: y = Delta w - V z, w = [head; cscale * g_step]
  const double* cscale;
  void* y;
  Key key;
  uint32_t step;
  int want_ysq;
  DynFuse dyn;
  // next query's column dots: when set (and pf is not), the dots of columns
  // 0..k (this panel, including the new column) with the stored x_{t+1}
  // rows, into slots 0..k -- the TDOT of the next query when this panel is
  // its data side
  int wnext;
  // fused prefetch
  int pf;
  uint32_t pf_step;
  int64_t pf_cut;
  double* partials;
  int pstride;
  int extra;
};

// Random-side pass of a Ginibre query (Algorithm 1).  With G the random side
// (l = k reflectors in V, Delta = diag(pi[min(i+1,l)])) and g the draw:
//   u   = Delta [0_l; g[l:]] - V z1                (new explicit basis vector)
//   out = sigma (B c + Delta (h + nu [0_l; g[l:]]) - V z2)
// where B holds nb explicit basis vectors with coefficients c (FP64), h
// (length l) the coefficients of the implicit basis vectors.  u is written to
// column nb of B.  Fused prefetch of V' g_next over rows > pf_cut.
struct GinPassArgs {
  void* V;
  int64_t ld;
  int k;
  const double* z1;
  const double* z2;
  const double* pi;
  void* B;
  int nb;
  const double* c;
  const double* h;
  const double* scal;  // [0] nu, [1] sigma
  int64_t n;
  void* y;
  Key key;
  uint32_t step;
  DynFuse dyn;
  // next query's column dots (as in PassArgs): V columns 0..k-1 into slots
  // 0..k-1 and B columns 0..nb (including the new one) into slots k..k+nb
  int wnext;
  // reflector step in a prologue (spro): every workgroup forms nu and the
  // coefficients z1, z2 from `small` itself (instead of reading z1, z2 and
  // scal[0]); workgroup 0 also stores the data reflector's scalars and, when
  // small.cslot >= 0, the data side's new T column
  int spro;
  GinSmallArgs small;
  int pf;
  uint32_t pf_step;
  int64_t pf_cut;
  double* partials;
  int pstride;
  int extra;
};

struct DynArgs {
  int kind;
  double a, b;
  const void* y;
  const void* x;
  const void* xprev;
  void* xnext;
  int64_t n;
  const double* ysq;  // normalise: ||y||^2
};

// Launch shape of a panel pass: chunks of 256 rows per workgroup (1, 2 or
// 4) and the number of workgroups.  The panel's leading dimension is a
// multiple of 256 * cpt.
struct Shape {
  int cpt;
  int nwg;
};

// ------------------------------------------------------------- batches --
//
// Many independent Haar trials advance in lockstep, one query index at a
// time, all Q-queries.  Trials are sorted by their number of steps (longest
// first), so the trials still running at a step are a prefix of the list and
// their workgroups a prefix of the block map.  Every workgroup covers 256 rows
// and the same number of columns, whatever its trial.

// Per-trial arguments in device memory; the per-step fields are patched by
// the batched kernels.
struct TrialDev {
  TdotArgs td;        // data-side TDOT (partials = the trial's partial rows)
  PassArgs pd;        // data pass
  PassArgs pr;        // random pass (partials = the trial's second buffer)
  SmallDataArgs sd;
  HaarSmallArgs hs;
  const void* xbase;  // x_t at xbase + ((t - 1) % xmod) * n elements
  int xmod;
  void* ybase;        // y_t at ybase + ((t - 1) % ymod) * n elements
  int ymod;
  const void* x0;     // x_0 (zeros)
  int T;              // queries of the trial
  int nwg;            // workgroups of its panels
};

struct BatchMap {
  const int* blk_trial;  // trial of each workgroup
  const int* blk_first;  // first workgroup of each trial
};

struct BatchStep {
  int k;          // reflectors per panel before this query (step - 1)
  uint32_t step;  // 1-based query index
};

enum BatchSmallOp { kBatchAfterTdot = 0, kBatchAfterData = 1 };

int launch_tdot_batch(int f64, int cpt, int nblk, int two, const TrialDev* d,
                      BatchMap m, BatchStep st, hipStream_t s);
int launch_pass_batch(int f64, int cpt, int nblk, int mode, const TrialDev* d,
                      BatchMap m, BatchStep st, hipStream_t s);
int launch_trial_small(int f64, int op, int ntrials, const TrialDev* d,
                       BatchStep st, hipStream_t s);
// Query 1 of every trial: ||g_1[1:]||^2 of the random side into the second
// partial buffer (the prefetch a previous query would have left there).
int launch_prefetch1_batch(int f64, int cpt, int nblk, const TrialDev* d,
                           BatchMap m, hipStream_t s);

// ------------------------------------------------ Gaussian ISTA batches --
//
// Independent trials of unrolled ISTA (eq. (ista)) on Gaussian matrices of
// one shape m x n, all advancing in lockstep, one query index at a time:
// query 0 observes y = sigma Q x* + w, then every layer is a Q-query and a
// Q'-query, so the two sides alternate as data and random side
// (Algorithm 1) and every running trial has the same reflector counts.

// The arguments of one side s (0: R, n rows; 1: L, m rows) of one trial.
struct IstaSide {
  TdotArgs td;       // TDOT with the side as data side (V2 = its basis panel)
  SmallDataArgs sd;  // z = T' w on it
  PassArgs pd;       // its data pass
  GinSmallArgs gs;   // the reflector step after its data pass (G = 1 - s)
  GinPassArgs gp;    // the random pass with the side as random side
  int nwg;           // workgroups over its rows
};

struct IstaTrialDev {
  IstaSide s[2];
  void* yobs;  // m: the observation y = sigma Q x* + w
  void* res;   // m: y - Q x_t (reverse pass: Q gbar)
  void* U;     // n: Q'(y - Q x_t) (query output)
  void* V;     // n: x_t + a_t Q'(y - Q x_t)
  void* gbar;  // n: reverse pass, g masked by the threshold (or null)
};

struct IstaStep {
  int q;             // query index, 0-based
  int kR, kL;        // reflectors on each side before the query
  uint32_t step;     // 1-based query index (the Philox step)
  int last;          // no query follows
  double a, theta;   // the layer's step and threshold (Q'-queries)
  int L;             // layers
  // the caller's arrays, trial i at offset i * (rows): x* (n), w (m) and
  // the trajectory X ((L + 1) x n, row 0 = x_1 = 0)
  const void* xstar;
  const void* noise;
  void* X;
  // kept for the reverse pass (or null): u_t and v_t of every layer,
  // trial i's layer t at offset (i * L + t) * n
  void* Urec;
  void* Vrec;
  // reverse pass: 1 for its queries (Q gbar, then Q'(.) with
  // g <- gbar - a_t Q'Q gbar written into G, trial i at offset i * n)
  int bwd;
  void* G;
};

// The reverse pass's per-layer reductions for every trial of a batch.
struct IstaAdjArgs {
  const IstaTrialDev* D;
  const void* G;      // dL/dx_{t+1}, count x n
  const void* Urec;
  const void* Vrec;
  int t, L, nwg;      // layer (0-based), layers, workgroups per trial
  int64_t n;
  double theta;
  double* part;       // count x nwg x 2
  double* grad_a;     // count x L (FP64)
  double* grad_theta;
};

// Phases of one query for all trials; each returns 0 or a HIP error.
int launch_ista_tdot(int f64, int cpt, int side, int nblk,
                     const IstaTrialDev* d, IstaStep st, hipStream_t s);
int launch_ista_small(int f64, int phase, int side, int ntrials,
                      const IstaTrialDev* d, IstaStep st, hipStream_t s);
int launch_ista_data(int f64, int cpt, int side, int nblk,
                     const IstaTrialDev* d, IstaStep st, hipStream_t s);
int launch_ista_rand(int f64, int cpt, int side, int nblk,
                     const IstaTrialDev* d, IstaStep st, hipStream_t s);
int launch_ista_adj(int f64, int ntrials, const IstaAdjArgs& a,
                    hipStream_t s);

// Device-to-device copies of 4-byte words, one workgroup per job.// Device-to-device copies of 4-byte words, one workgroup per job.
struct CopyJob {
  const void* src;
  void* dst;
  int64_t words;
};
int launch_copy_jobs(const CopyJob* jobs, int count, hipStream_t s);

// Optional events recorded by the dispatch itself at the kernel's start and
// end (hipExtLaunchKernelGGL), for timing without extra packets around it.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};

// Largest k for the data pass's z prologue (its LDS holds 2 * kZproMax
// doubles); shapes of up to two chunks per workgroup use it (and the
// Gaussian random pass's reflector-step prologue).
constexpr int kZproMax = 512;

int launch_tdot(int f64, Shape sh, const TdotArgs& a, hipStream_t s,
                LaunchEvents ev = LaunchEvents());
int launch_pass(int f64, Shape sh, int mode, const PassArgs& a,
                hipStream_t s, LaunchEvents ev = LaunchEvents());
int launch_gin_pass(int f64, Shape sh, const GinPassArgs& a, hipStream_t s,
                    LaunchEvents ev = LaunchEvents());
// Fixed-order sums of the partial rows of one pass: out[slot] = sum over
// rows w < nwg of P[w * pstride + slot], for the slots in rg.  stage: room
// for red_stage_doubles(nwg, pstride) doubles (the two-stage form's
// per-block sums).
struct ReduceJob {
  const double* P;
  int pstride;
  int nwg;
  SlotRanges rg;
  double* out;
  double* stage;
};

// Partial rows per block of the two-stage reduction's first stage, and the
// row count from which it is used (below it one block per slot reads the
// rows directly; the environment variable HD_RED_TWO_STAGE overrides it).
constexpr int kRed1Rows = 256;
constexpr int kRedTwoStage = 1024;
inline size_t red_stage_doubles(int nwg, int pstride) {
  return (size_t)((nwg + kRed1Rows - 1) / kRed1Rows) * (size_t)pstride;
}

// The sums of one or two jobs (job b may have no slots): one launch when
// both have at most kRedTwoStage rows, else two (blocks of kRed1Rows rows x
// 32 consecutive slots, each row segment read as one contiguous run, then
// the block sums per slot).
int launch_reduce(const ReduceJob& a, const ReduceJob& b, hipStream_t s);
int launch_small_data(const SmallDataArgs& a, hipStream_t s);
int launch_haar_small(int f64, const HaarSmallArgs& a, hipStream_t s);
int launch_gin_small(int f64, const GinSmallArgs& a, hipStream_t s);
int launch_dyn(int f64, const DynArgs& a, hipStream_t s);

// Reverse pass of one unrolled ISTA layer (element-wise part): gbar and the
// two parameter-gradient sums (see k_lista_adj).
struct ListaAdjArgs {
  const void* g;  // dL/dx_{t+1}
  const void* v;  // v_t
  const void* u;  // u_t
  void* gbar;     // out
  double theta;
  int64_t n;
  double* part;   // 2 * lista_blocks(n) doubles
};
inline int lista_blocks(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}
int launch_lista_adj(int f64, const ListaAdjArgs& a, double* ga, double* gt,
                     hipStream_t s);
int launch_fill(double* p, double v, int64_t count, hipStream_t s);
// Zero `bytes` (a multiple of 4) at p.
int launch_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace hd
