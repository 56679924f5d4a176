/*
 * hd.h -- C ABI of the MI355X (gfx950) Householder Dice library, libhd.so.
 *
 * Householder Dice (Y. M. Lu, arXiv 2101.07464) simulates dynamics
 *     x_{t+1} = f_t(M_t x_t, x_t, ..., x_{t-d}),  M_t in {Q, Q'},
 * (eq. (dynamics), Sec. 1) for a random matrix Q drawn from the Ginibre
 * ensemble GE(m,n) (Sec. 3.2, Algorithm 1) or the Haar ensemble on O(n)
 * (Sec. 3.3, Algorithm 2) without ever forming Q: every query reveals only the
 * randomness it needs, stored as Householder reflectors (eq. (Householder),
 * eq. (Householder_e)).  Memory is O((m+n) T) and a query costs O((m+n) t).
 *
 * Conventions for every entry point:
 *   - Vectors are device pointers (hipMalloc'd, or torch CUDA tensors) of the
 *     handle's storage type: float for HD_F32, double for HD_F64, contiguous,
 *     element-aligned.  The caller owns them; they must stay valid until the
 *     handle's stream has passed the call.  Outputs must not alias inputs.
 *   - Calls are asynchronous and stream-ordered on the handle's stream.
 *   - Return value: HD_OK (0) or a negative HD_ERR_* code.  A call that fails
 *     host-side validation leaves the handle unchanged.  Conditions found on
 *     the device (a non-finite norm) set a sticky flag reported by hd_status.
 *   - A handle is not thread-safe; different handles are independent.
 *   - The realisation is fixed by the key (seed, trial): the fresh Gaussian
 *     vector g_t of query t (1-based) is the Philox4x32-10 stream with key
 *     (seed, trial), counter (lo32(i/4), t, 0, hi32(i/4)), Box-Muller in FP64
 *     (pair (w0,w1) -> entries 4b, 4b+1 as r cos, r sin; (w2,w3) -> 4b+2, 4b+3).
 */
#ifndef HD_H_
#define HD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HD_OK = 0,
  HD_ERR_INVALID = -1,   /* bad argument, null pointer, dimension mismatch */
  HD_ERR_CAPACITY = -2,  /* t_max reached, or T <= min(m,n) would break */
  HD_ERR_NOMEM = -3,     /* device allocation failed */
  HD_ERR_HIP = -4,       /* a HIP runtime call failed */
  HD_ERR_NONFINITE = -5, /* a reflector norm was NaN/Inf (sticky) */
  HD_ERR_UNSUPPORTED = -6,
  HD_ERR_TOO_LARGE = -7  /* beyond the allocation-free entry point's scratch */
};

enum { HD_GINIBRE = 0, HD_HAAR = 1 };
enum { HD_F32 = 0, HD_F64 = 1 };

typedef struct hd_ctx* hd_handle;

typedef struct {
  int32_t ensemble; /* HD_GINIBRE (Alg. 1) or HD_HAAR (Alg. 2) */
  int32_t storage;  /* HD_F32 or HD_F64: panels and vectors; norms, signs,
                       the WY factor T and all accumulations are FP64 */
  int64_t m, n;     /* Q is m x n; Haar requires m == n */
  int32_t t_max;    /* number of queries the handle can answer;
                       must satisfy 1 <= t_max <= min(m, n) (Alg. 1 and 2
                       require T <= min(m, n)) */
  uint32_t seed;    /* Philox key word 0 */
  uint32_t trial;   /* Philox key word 1 */
  double sigma;     /* Ginibre: entries of Q are N(0, sigma^2); Haar: unused */
  void* stream;     /* hipStream_t for all work of the handle; NULL = null
                       stream */
} hd_config;

/* Create a lazy random matrix.  Allocates and owns all device buffers
 * (panels of t_max columns, FP64 scalars); no query is answered yet.
 * Errors: HD_ERR_INVALID (bad cfg, out == NULL), HD_ERR_NOMEM, HD_ERR_HIP. */
int hd_init(const hd_config* cfg, hd_handle* out);

/* Release the handle after its stream has drained.  NULL is a no-op. */
int hd_free(hd_handle h);

/* y = Q x: x has n entries, y has m entries (device).  One query of the
 * dynamics with M_t = Q (Alg. 1 "if M_t = Q" branch; Alg. 2 Q branch).
 * Errors: HD_ERR_INVALID, HD_ERR_CAPACITY (state unchanged), HD_ERR_HIP. */
int hd_step(hd_handle h, const void* x, void* y);

/* y = Q' x: x has m entries, y has n entries (device).  M_t = Q'. */
int hd_apply_T(hd_handle h, const void* x, void* y);

/* Synchronise the handle's stream and report the sticky device flag:
 * HD_OK, HD_ERR_NONFINITE or HD_ERR_HIP. */
int hd_status(hd_handle h);

/* Query counters: t (queries answered), r (|{R_i}|), l (|{L_i}|).  For Haar
 * every query adds one reflector to each side, so r = l = t. */
int hd_counts(hd_handle h, int32_t* t, int32_t* r, int32_t* l);

/* Forget every revealed reflector and restart at t = 0 with a new key
 * (seed, trial), reusing the handle's device buffers: the next query is the
 * first query of a fresh, independent Q.  Also clears the sticky device flag
 * (hd_status reports HD_OK again unless a later query sets it).
 * Stream-ordered; no allocation.  Errors: HD_ERR_INVALID, HD_ERR_HIP. */
int hd_reset(hd_handle h, uint32_t seed, uint32_t trial);

/* Change the stream used by later calls (hipStream_t, NULL = null stream). */
int hd_set_stream(hd_handle h, void* stream);

/* ------------------------------------------------------------------------
 * Gaussian orthogonal ensemble from the Gaussian one (section "Other Random
 * Matrix Ensembles"): for Q with i.i.d. N(0, s^2) entries,
 * G = (Q + Q')/sqrt(2) is GOE of scale s (diagonal N(0, 2 s^2),
 * off-diagonal N(0, s^2)).  hd_goe_step answers y = G x = (Q x + Q' x)/sqrt(2)
 * with two queries on a square Gaussian handle of sigma = s (Q x first, then
 * Q' x with the sum and the 1/sqrt(2) formed in its epilogue).  Each call
 * uses two of the handle's t_max queries (one reflector per side).  x, y:
 * device vectors of n entries (storage type), not aliased.  Errors:
 * HD_ERR_INVALID (not a square Gaussian handle, null or aliased pointers),
 * HD_ERR_CAPACITY, HD_ERR_NOMEM, HD_ERR_HIP. */
int hd_goe_step(hd_handle h, const void* x, void* y);

/* Q = U S V (section "Other Random Matrix Ensembles") with U ~ Haar(m) and
 * V ~ Haar(n) independent (two Haar handles of sizes m and n, the same
 * storage type and stream) and S in R^{m x n} with diagonal s (min(m, n)
 * entries) and zeros elsewhere: transpose = 0 answers y = Q x =
 * U (S (V x)) (x: n entries, y: m), transpose = 1 answers y = Q' x =
 * V' (S' (U' x)) (x: m entries, y: n); one query on each handle, the
 * product with S formed in the first query's epilogue.  s, x, y: device
 * vectors (storage type); x and y not aliased.  Errors: HD_ERR_INVALID
 * (not two distinct Haar handles of equal storage and stream; null or
 * aliased pointers), HD_ERR_CAPACITY, HD_ERR_NOMEM, HD_ERR_HIP. */
int hd_usv_step(hd_handle U, hd_handle V, const void* s, int32_t transpose,
                const void* x, void* y);

/* Spectral method for generalized linear models (Sec. 2.2): on a Haar
 * handle of size m (the m x m Q), with A = [I_n 0] Q (eq. (A_ortho)) for a
 * signal dimension 1 <= n < m, measurements y_i = tanh|a_i' xi| and
 * D = (1/m) A diag(y) A' (eq. (D_mtx)), runs K steps of the power iteration
 * x_{k+1} = scale * m * D x_k from x_1.  The measurements take one query
 * (A' xi = Q' [xi; 0]) and every step two (Q' [x_k; 0], then Q of y times
 * that), 1 + 2K queries in all, the element-wise maps fused into the
 * queries' epilogues.  scale keeps the iterates in range (the eigenvalues
 * of m D lie in [0, 1)); the iterates are not normalised.
 * xi, x1: device vectors of n entries.  z: NULL or device m entries
 * receiving A' xi.  X: NULL or device (K+1) x n row-major receiving
 * x_1 .. x_{K+1}.  Stream-ordered; uses six work vectors of the handle
 * (allocated on first use).  Errors: HD_ERR_INVALID (not a Haar handle,
 * n >= m, K < 0, non-finite scale, null or aliased pointers),
 * HD_ERR_CAPACITY (1 + 2K more queries than t_max allows; checked before
 * any work), HD_ERR_NOMEM, HD_ERR_HIP. */
int hd_spectral_power(hd_handle h, int64_t n, const void* xi, const void* x1,
                      int32_t K, double scale, void* z, void* X);

/* ------------------------------------------------------------------------
 * Checkpoint and resume.  The state of a handle after its last query is
 * what Algorithms 1 and 2 carry from one query to the next: the stored
 * reflectors of both sides (panels, T factors, tau, the norms, pivots and
 * signs), the Gaussian ensemble's explicit basis vectors, the query
 * counters, the Philox key, the sticky device flag and the data-independent
 * dots already computed for the next query.
 *
 * hd_export: host_buf == NULL stores the required size in *size; otherwise
 * *size is the capacity of host_buf (host memory, caller-owned), which
 * receives the state (a self-describing byte block of that size).  Finishes
 * the stream's pending work for the handle and synchronises it; the handle
 * is unchanged and can continue.  Works also after a device error.
 * Errors: HD_ERR_INVALID (h or size NULL, capacity too small: *size is set
 * to the required size), HD_ERR_HIP.
 *
 * hd_import: creates a handle (as hd_init, on cfg->stream) holding an
 * exported state; the next query continues the exported sequence exactly
 * (same realisation of Q).  cfg must repeat the exporter's ensemble,
 * storage, m, n, t_max (and sigma for the Gaussian ensemble); seed and
 * trial come from the state.  The launch shape may differ from the
 * exporter's.  Errors: HD_ERR_INVALID (mismatching cfg, malformed or short
 * buffer), HD_ERR_NOMEM, HD_ERR_HIP. */
int hd_export(hd_handle h, void* host_buf, size_t* size);
int hd_import(const hd_config* cfg, const void* host_buf, size_t size,
              hd_handle* out);

/* Copy to host, for the first `count` reflectors of one side
 * (side 0 = R, acting on R^n; side 1 = L, acting on R^m): the norm nu of the
 * vector it was built from, that vector's first entry (the pivot) and the
 * sign s in {-1,+1}.  Synchronises the stream.  Any output may be NULL. */
int hd_pivots(hd_handle h, int32_t side, int32_t count, double* nu,
              double* pivot, int32_t* sign);

/* Built-in dynamics for hd_run (the maps f_t of the workloads). */
enum {
  HD_DYN_TANH = 1,      /* x_{t+1} = tanh(a y_t) + b x_t          */
  HD_DYN_SOFT_HIST = 2, /* x_{t+1} = soft(y_t, a) + b x_{t-1}     */
  HD_DYN_NORMALIZE = 3  /* x_{t+1} = y_t / ||y_t|| + b x_t        */
};
enum {
  HD_PATTERN_Q = 0,  /* M_t = Q for every t */
  HD_PATTERN_ALT = 1 /* M_t = Q for odd t, Q' for even t */
};

typedef struct {
  int32_t kind;    /* HD_DYN_* */
  int32_t pattern; /* HD_PATTERN_* */
  double a, b;
} hd_dynamics;

/* Run T steps of eq. (dynamics) on the device with a built-in f_t.
 * x1: the initial condition x_1 (n entries).  x0: x_0 for the history term
 * (n entries) or NULL for zeros.  x_out: receives x_{T+1} (n entries) or NULL.
 * traj_x: NULL or (T+1) x n row-major buffer receiving x_1..x_{T+1};
 * traj_y: NULL or T x m buffer receiving y_1..y_T.  Requires m == n.
 * Errors as hd_step; on HD_ERR_CAPACITY nothing is launched. */
int hd_run(hd_handle h, const hd_dynamics* dyn, int32_t T, const void* x1,
           const void* x0, void* x_out, void* traj_x, void* traj_y);

/* ------------------------------------------------------------------------
 * Allocation-free trajectory, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).
 *
 * hd_run_noalloc(cfg, ...) does what hd_init(cfg) + hd_run(...) + hd_free
 * would do -- a fresh Q with the key (cfg->seed, cfg->trial), T steps of the
 * built-in dynamics, the same kernels and launch shapes, hence the same
 * results -- but every device buffer the library needs (panels, FP64
 * scalars, partial sums, hd_run's internal x ring, y and zero vectors) lives
 * in one static device array of HD_NOALLOC_SCRATCH_BYTES per GPU, which each
 * GPU the library runs on holds until the process ends.  The call performs
 * no hipMalloc, hipFree or other allocating routine and no synchronisation;
 * it clears the region with a fill kernel on cfg->stream and launches the
 * trajectory there.  The caller still owns x1, x0, x_out, traj_x and traj_y
 * (as for hd_run; requires m == n).  Every call on a GPU shares that GPU's
 * array, whose contents are the last call's: calls that overlap on one GPU
 * (different streams, or host threads) race and must be serialised by the
 * caller.  hd_noalloc_scratch_bytes reports the bytes cfg needs.
 * Errors: HD_ERR_INVALID (bad cfg or arguments, m != n),
 * HD_ERR_TOO_LARGE (the layout exceeds the array), HD_ERR_UNSUPPORTED
 * (as hd_run's maps and patterns), HD_ERR_CAPACITY, HD_ERR_HIP. */
#define HD_NOALLOC_SCRATCH_BYTES (64u << 20)
int hd_noalloc_scratch_bytes(const hd_config* cfg, size_t* bytes);
int hd_run_noalloc(const hd_config* cfg, const hd_dynamics* dyn, int32_t T,
                   const void* x1, const void* x0, void* x_out, void* traj_x,
                   void* traj_y);

/* ------------------------------------------------------------------------
 * Unrolled ISTA with learned per-layer parameters, and its gradient.
 *
 * Layer t = 1..L is the ISTA step of eq. (ista) with the step tau replaced
 * by a_t and the threshold lambda tau by theta_t:
 *     u_t = Q'(y - Q x_t),  v_t = x_t + a_t u_t,  x_{t+1} = eta_{theta_t}(v_t)
 * (eta the element-wise soft threshold).  Every product with Q or Q' is a
 * query on this handle, so all layers, and the reverse pass, see one fixed
 * matrix Q: the reverse pass is the exact gradient of the unrolled map for
 * that Q, and its own products with Q are further queries (Q'Q gbar per
 * layer), revealing randomness as needed.
 * ------------------------------------------------------------------------ */

/* Forward pass, 2L queries (Q then Q' per layer).  a, theta: host arrays of
 * L floats.  yobs: device, m entries.  X: device (L+1) x n row-major, row 0
 * holds x_1 on entry, rows 1..L receive x_2..x_{L+1}.  U, V: device L x n,
 * receive u_t and v_t (kept for the reverse pass).
 * Errors: HD_ERR_INVALID, HD_ERR_CAPACITY (checked before any query: t_max,
 * and for Ginibre r <= n, l <= m), HD_ERR_NOMEM, HD_ERR_HIP. */
int hd_lista_forward(hd_handle h, int32_t L, const float* a,
                     const float* theta, const void* yobs, void* X, void* U,
                     void* V);

/* Reverse pass for g = dL/dx_{L+1} (device, n entries), with U, V from the
 * forward pass and the same a, theta.  grad_a, grad_theta: device arrays of
 * L doubles receiving dL/da_t and dL/dtheta_t (threshold derivative taken as
 * the indicator of |v| > theta).  g_x1: NULL, or device n entries receiving
 * dL/dx_1.  Uses 2(L-1) queries (2L with g_x1).  Errors as the forward. */
int hd_lista_backward(hd_handle h, int32_t L, const float* a,
                      const float* theta, const void* U, const void* V,
                      const void* g, double* grad_a, double* grad_theta,
                      void* g_x1);

/* ------------------------------------------------------------------------
 * Launch-shape autotuner.  The panel kernels' workgroups cover 1, 2 or 4
 * chunks of 256 rows; the built-in rule uses 1 below 256K rows, 2 below
 * 512K, 4 from there on.  hd_autotune times on the device, for every panel length in
 * `lengths`, a whole trajectory of k queries on a scratch handle of that
 * size (x_{t+1} = tanh(y_t) + 0.5 x_t; Haar: M_t = Q; Gaussian: sigma^2 =
 * 1/n, Q and Q' alternating) under each candidate shape, and installs the
 * fastest (the built-in shape unless another is at least 3% faster),
 * process-wide, for the ensemble and storage type (replacing its earlier
 * entries).  A handle created afterwards uses, per panel, the entry
 * whose length is nearest its own in ratio, if within a factor of 2, and
 * the built-in rule otherwise.  report: NULL or 3 * count doubles receiving
 * the mean microseconds per trajectory under 1, 2 and 4 chunks.  The
 * tables are replaced atomically with respect to concurrent hd_init calls
 * on other threads (each handle takes the shapes installed when it is
 * created).  The environment variable HD_CPT
 * (1, 2 or 4), when set, overrides tuned and built-in shapes.
 * Errors: HD_ERR_INVALID (ensemble, storage, count < 1, k < 2, a length
 * below k or above 2^31), HD_ERR_NOMEM, HD_ERR_HIP. */
int hd_autotune(int32_t ensemble, int32_t storage, const int64_t* lengths,
                int32_t count, int32_t k, void* stream, double* report);

/* The chunks per workgroup a handle's panel of length n would use now. */
int hd_shape_rule(int32_t ensemble, int32_t storage, int64_t n, int32_t* cpt);

/* Forget every tuned shape (back to the built-in rule). */
int hd_autotune_clear(void);

/* Timing of the panel kernels with HIP events on the handle's stream.
 * hd_profile(h, 1) starts recording (clears previous records), 0 stops. */
int hd_profile(hd_handle h, int32_t enable);

/* Totals since recording started, for one kernel kind:
 * 0 = panel TDOT (V'x), 1 = data-side GEMV-N pass, 2 = random-side GEMV-N
 * pass.  ms: summed durations; launches: count; bytes: algorithmic bytes
 * (panel elements read + vector elements read/written, times the element
 * size).  Synchronises the stream. */
int hd_profile_read(hd_handle h, int32_t kind, double* ms, int64_t* launches,
                    double* bytes);

/* ------------------------------------------------------------------------
 * Batches of independent Haar trials.
 *
 * Many independent trials of eq. (dynamics) with Haar Q (Alg. 2), each with
 * its own n, number of queries T and Philox key (seed, trial), all with
 * M_t = Q and the same built-in f_t, run to completion together: the trials
 * advance in lockstep one query index at a time and every launch covers all
 * trials still running, so a step costs a handful of launches for the whole
 * batch instead of for every trial.  Each trial's answers equal those of a
 * separate handle with the same key (hd_run) up to the order of the FP64
 * partial sums.
 * ------------------------------------------------------------------------ */
typedef struct hd_batch_ctx* hd_batch;

typedef struct {
  int64_t n;      /* dimension of the trial's Q (n x n), n >= 1 */
  int32_t T;      /* queries of the trial, 1 <= T <= n */
  uint32_t seed;  /* Philox key word 0 */
  uint32_t trial; /* Philox key word 1 */
} hd_batch_trial;

/* Allocate the device state of `count` trials (storage HD_F32 or HD_F64) on
 * `stream` (hipStream_t, NULL = null stream).  The handle owns one arena
 * holding every trial's two panels (n rounded up to 1024 rows, T columns),
 * FP64 scalars and work vectors.  The trial list is copied.
 * Errors: HD_ERR_INVALID (count < 1, bad n or T, out == NULL),
 * HD_ERR_NOMEM, HD_ERR_HIP. */
int hd_batch_init(int32_t storage, const hd_batch_trial* trials,
                  int32_t count, void* stream, hd_batch* out);

/* Run every trial from a fresh Q (query 1) to its own T with the built-in map
 * dyn->kind (HD_DYN_TANH or HD_DYN_SOFT_HIST; dyn->pattern must be
 * HD_PATTERN_Q; x_0 = 0).  x1: host array of `count` device pointers, x_1 of
 * each trial (n_i entries), in the order given to hd_batch_init.  x_out: NULL
 * or host array of device pointers receiving x_{T_i+1}.  traj_x / traj_y:
 * NULL or host arrays of device pointers to (T_i+1) x n_i and T_i x n_i
 * row-major buffers receiving x_1..x_{T_i+1} and y_1..y_{T_i}.  Each call
 * starts the trials over with the same keys.  Stream-ordered; the pointer
 * arrays are read before the call returns.
 * Errors: HD_ERR_INVALID, HD_ERR_UNSUPPORTED (other maps or patterns),
 * HD_ERR_HIP. */
int hd_batch_run(hd_batch b, const hd_dynamics* dyn, const void* const* x1,
                 void* const* x_out, void* const* traj_x, void* const* traj_y);

/* Synchronise and report the sticky device flag (as hd_status). */
int hd_batch_status(hd_batch b);

/* Replay mode for hd_batch_run (enable = 1): the first run with a given
 * x_out mode (NULL or not) records its whole launch sequence into a HIP
 * graph; every later run uploads its per-run pointers and map parameters
 * (as always) and launches that graph, one submission for all trials and
 * steps.  Requires a non-null stream (set at init or by
 * hd_batch_set_stream) for the recording.  enable = 0 returns to direct
 * launches (recorded graphs are kept for a later enable).
 * Errors: HD_ERR_INVALID, HD_ERR_UNSUPPORTED (null stream). */
int hd_batch_set_graph(hd_batch b, int32_t enable);

/* Launch shape of the batched panel kernels: every workgroup covers
 * `chunks` (1, 2 or 4) chunks of 256 rows of one trial's panels (panels are
 * padded to 1024 rows, so every shape tiles every trial).  More chunks mean
 * longer sweeps and fewer partial rows to reduce; fewer mean more workgroups
 * in flight.  The initial shape is 4 (environment HD_BATCH_CPT = 1, 2 or 4
 * overrides it).  The answers do not depend on the shape beyond the order of
 * the FP64 partial sums.  Synchronises the batch's stream and drops graphs
 * recorded by hd_batch_set_graph (the next run records anew).
 * Errors: HD_ERR_INVALID (other values), HD_ERR_HIP. */
int hd_batch_set_shape(hd_batch b, int32_t chunks);

/* The current shape (1, 2 or 4), or HD_ERR_INVALID for a NULL handle. */
int hd_batch_shape(hd_batch b);

/* Autotuner for the batch's launch shape: for each shape 1, 2 and 4, one
 * untimed run and `reps` (1..100) timed runs of the whole batch with the map
 * dyn and inputs x1 (as hd_batch_run, outputs kept in the batch's own
 * buffers; HIP events on the batch's stream, direct launches), then installs
 * the fastest shape if it is at least 3% faster than the initial shape's
 * default, else that default.  ms: NULL or 3 doubles receiving the mean
 * milliseconds per run at 1, 2 and 4 chunks; chosen: NULL or the installed
 * shape.  Blocks until the timed runs end.
 * Errors: as hd_batch_run and hd_batch_set_shape; HD_ERR_INVALID for reps
 * out of range. */
int hd_batch_autotune(hd_batch b, const hd_dynamics* dyn,
                      const void* const* x1, int32_t reps, double* ms,
                      int32_t* chosen);

/* Change the stream of later calls. */
int hd_batch_set_stream(hd_batch b, void* stream);

/* Release the batch after its stream has drained.  NULL is a no-op. */
int hd_batch_free(hd_batch b);

/* ------------------------------------------------------------------------
 * Batches of unrolled-ISTA trials on Gaussian matrices (Sec. 2.1).
 *
 * count independent trials, each with its own m x n Gaussian Q (entries
 * N(0, sigma^2), Philox key (seed, trial0 + i)), run the lasso experiment's
 * dynamics together: the observation y = Q x* + w (one query), then L
 * layers of eq. (ista) with per-layer step a_t and threshold theta_t,
 *     x_{t+1} = eta_{theta_t}(x_t + a_t Q'(y - Q x_t))
 * (two queries each, Algorithm 1).  All trials advance in lockstep, one
 * query index at a time, so a query costs a handful of launches for the
 * whole batch; each trial's answers are those of a separate handle with the
 * same key up to the order of the FP64 partial sums.  With HD_ISTA_GRAD the
 * batch also runs the reverse pass of the unrolled map (the fixed-Q
 * gradient of hd_lista_backward, for every trial together).
 * ------------------------------------------------------------------------ */
typedef struct hd_ista_ctx* hd_ista;

#define HD_ISTA_GRAD 1 /* keep u_t, v_t and room for the reverse pass */

/* Allocate the device state of `count` trials (one arena: per trial four
 * panels, FP64 scalars, work vectors) on `stream`.  flags: 0 or
 * HD_ISTA_GRAD (then also count x L x n arrays for u_t and v_t, and panel
 * room for the 2(L - 1) queries of the reverse pass).  Requires L + 1 <= n
 * and L <= m (Algorithm 1's capacity), with HD_ISTA_GRAD 2L <= n and
 * 2L - 1 <= m; sigma > 0.  Errors: HD_ERR_INVALID, HD_ERR_NOMEM (also
 * beyond 250 GB), HD_ERR_HIP. */
int hd_ista_init(int32_t storage, int64_t m, int64_t n, int32_t L,
                 int32_t count, uint32_t seed, uint32_t trial0, double sigma,
                 int32_t flags, void* stream, hd_ista* out);

/* Run every trial from fresh matrices (the same keys at every call).
 * a, theta: host arrays of L floats.  xstar: device count x n (x* of trial
 * i in row i), noise: device count x m (w), X: device count x (L + 1) x n
 * whose row 0 of every trial holds x_1 on entry; rows 1..L receive
 * x_2..x_{L+1}.  Stream-ordered.  Errors: HD_ERR_INVALID, HD_ERR_HIP. */
int hd_ista_run(hd_ista b, const float* a, const float* theta,
                const void* xstar, const void* noise, void* X);

/* Reverse pass after hd_ista_run on a batch made with HD_ISTA_GRAD, with the
 * same a and theta: G (device count x n) holds dL/dx_{L+1} of every trial on
 * entry and is overwritten (it carries dL/dx_t from layer to layer); grad_a
 * and grad_theta (device count x L, FP64) receive, for trial i,
 * dL/da_t = sum(gbar_t u_t) and dL/dtheta_t = -sum(g_{t+1} sign(v_t) m_t)
 * with the mask m_t = [|v_t| > theta_t], gbar_t = g_{t+1} m_t and
 * g_t = gbar_t - a_t Q'Q gbar_t (two more queries on the trial's Q per
 * layer, as hd_lista_backward).  One reverse pass per forward run.
 * Stream-ordered.  Errors: HD_ERR_INVALID (no HD_ISTA_GRAD, no forward run
 * since the last reverse pass, null pointers), HD_ERR_HIP. */
int hd_ista_grad(hd_ista b, const float* a, const float* theta, void* G,
                 double* grad_a, double* grad_theta);

/* Synchronise and report the sticky device flag (as hd_status). */
int hd_ista_status(hd_ista b);

/* Change the stream of later calls. */
int hd_ista_set_stream(hd_ista b, void* stream);

/* Release the batch after its stream has drained.  NULL is a no-op. */
int hd_ista_free(hd_ista b);

/* ------------------------------------------------------------------------
 * Complex HD (Sec. 3.4): the complex Ginibre ensemble (entries with
 * E|Q_ij|^2 = sigma^2, real and imaginary parts N(0, sigma^2 / 2)), the
 * Haar ensemble on the unitary group U(n), and the Gaussian unitary ensemble
 * G = (Q + Q^H) / sqrt(2) as two queries on a square complex Ginibre handle.
 * Reflectors are the unitary reflectors of eq. (Householder_c); Algorithms
 * 1 and 2 run with the conjugate transpose in place of the transpose, and
 * where the real algorithms apply a (symmetric) reflector to build an output
 * or an output-space basis vector, the conjugate transpose of the unitary
 * one is applied: Haar y = Q x is L_1^H .. L_t^H R_t p_t; Ginibre
 * u_t = L_1^H .. L_l^H Z_{1:l} g_t, v_t = R_1^H .. R_r^H e_r, y = sigma
 * sum_i (v_i^H x) u_i (and the mirror images for y = Q^H x).
 *
 * Vectors are device arrays of interleaved (re, im) pairs in the storage
 * type (HD_F32: complex float, HD_F64: complex double); scalars, reflector
 * norms and phases, T factors and the phase prefix are FP64.  Complex normal
 * i of query t is (N_2i + i N_2i+1) / sqrt(2) from the real stream of the
 * header's draws (key (seed, trial), step t, tag 0).  Launches are ordered
 * on the handle's stream; calls on one handle must not overlap.
 * ------------------------------------------------------------------------ */
typedef struct hd_cctx* hd_chandle;

/* Allocate a complex handle: ensemble HD_GINIBRE (m x n) or HD_HAAR (m == n),
 * at most t_max <= 1024 queries (Haar: t_max <= n; Ginibre: at most n
 * Q-queries and m Q^H-queries), panels of t_max + 1 columns per side (plus
 * basis panels on Ginibre).  sigma: entry scale of Ginibre (ignored on Haar).
 * Errors: HD_ERR_INVALID (bad configuration, out == NULL), HD_ERR_NOMEM,
 * HD_ERR_HIP. */
int hd_cinit(int32_t ensemble, int32_t storage, int64_t m, int64_t n,
             int32_t t_max, uint32_t seed, uint32_t trial, double sigma,
             void* stream, hd_chandle* out);

/* One query: y = Q x (adjoint = 0; x of length n, y of length m) or
 * y = Q^H x (adjoint != 0).  x and y must not alias.  Errors:
 * HD_ERR_INVALID, HD_ERR_CAPACITY (state unchanged), HD_ERR_HIP. */
int hd_cstep(hd_chandle h, int32_t adjoint, const void* x, void* y);

/* T queries y_t = Q x_t on a Haar handle with the fused map
 * x_{t+1} = tanh(a |y_t|) e^{i arg y_t} + b x_t (entrywise; 0 where y = 0).
 * X: device (T + 1) x n, row 0 = x_1 on entry, rows 1..T receive
 * x_2..x_{T+1}; Y: NULL or device T x n for the answers.  Errors:
 * HD_ERR_INVALID, HD_ERR_UNSUPPORTED (not a Haar handle), HD_ERR_CAPACITY
 * (checked before any query), HD_ERR_HIP. */
int hd_crun(hd_chandle h, int32_t T, double a, double b, void* X, void* Y);

/* GUE: y = G x with G = (Q + Q^H) / sqrt(2) on a square complex Ginibre
 * handle (two queries, the second combining the first answer; entries of G
 * have E|G_ij|^2 = sigma^2, the diagonal real).  The first answer is staged
 * in a buffer allocated on first use.  Errors: HD_ERR_INVALID (not a square
 * Ginibre handle, null or aliased pointers), HD_ERR_CAPACITY, HD_ERR_NOMEM,
 * HD_ERR_HIP. */
int hd_cgue_step(hd_chandle h, const void* x, void* y);

/* Start a fresh matrix with key (seed, trial) on the same allocation (the
 * sticky flag is cleared too).  Stream-ordered.  Errors: HD_ERR_INVALID,
 * HD_ERR_HIP. */
int hd_creset(hd_chandle h, uint32_t seed, uint32_t trial);

/* Queries so far and the reflector counts |R|, |L|. */
int hd_ccounts(hd_chandle h, int32_t* t, int32_t* r, int32_t* l);

/* Synchronise the stream; HD_OK, HD_ERR_NONFINITE (a reflector norm was not
 * finite since the last reset) or HD_ERR_HIP. */
int hd_cstatus(hd_chandle h);

/* Change the stream of later calls. */
int hd_cset_stream(hd_chandle h, void* stream);

/* Timing of the complex panel launches with events recorded by the
 * dispatches on the handle's stream: hd_cprofile(h, 1) starts recording
 * (clears earlier records), 0 stops; hd_cprofile_read gives, for one kind
 * (0 = dots of L1, 1 = data pass, 2 = output pass), the summed durations,
 * the launch count and the algorithmic bytes (every panel column once, the
 * vectors read and written).  Both synchronise the stream. */
int hd_cprofile(hd_chandle h, int32_t enable);
int hd_cprofile_read(hd_chandle h, int32_t kind, double* ms,
                     int64_t* launches, double* bytes);

/* Release the handle after its stream has drained.  NULL is a no-op. */
int hd_cfree(hd_chandle h);

/* Message for an HD_* code (static storage). */
const char* hd_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* HD_H_ */
