/*
 * hd_oracle.c -- plain FP64 CPU reference for Householder Dice (HD).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it; the product library never links or calls it,
 * and it shares no code with the HIP sources.
 *
 * What it computes (Y. M. Lu, "Householder Dice", arXiv 2101.07464):
 *   - the Householder reflector H(v) of Sec. 3.1, eq. (Householder), with the
 *     sign rule read as sign(v1) = +1 for v1 >= 0 and -1 otherwise (the text
 *     prints "0 otherwise", which would make H(v) singular);
 *   - the generalised reflector H_k(p) of eq. (Householder_e), equal to the
 *     identity when p[k:n] = 0;
 *   - Algorithm 1 (Ginibre ensemble GE(m,n), Sec. 3.2) and Algorithm 2 (Haar
 *     ensemble on O(n), Sec. 3.3), each query applying the stored reflectors
 *     one at a time, exactly in the order the algorithms state.  No blocking,
 *     no compact-WY form, no fusion.
 *
 * The paper draws "g_t ~ GE(.,1)" without naming a generator.  The draws here
 * follow one fixed, published recipe so that another implementation can
 * reproduce the same realisation:
 *   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = (seed, trial),
 *   counter = (lo32(i>>2), step, tag, hi32(i>>2)); the four output words give
 *   two uniforms pairs u = (w + 0.5) * 2^-32, and Box-Muller (1958) in FP64
 *   turns pair (w0,w1) into normals i%4 = 0 (cos), 1 (sin) and (w2,w3) into
 *   i%4 = 2 (cos), 3 (sin).  The radius uses the even word, the angle the odd
 *   word.  HD draws use tag 0 and the 1-based query index as "step".
 *
 * Index convention: the paper is 1-based; this file stores arrays 0-based, and
 * a reflector created at 1-based index k acts on entries k..dim (0-based
 * k-1..dim-1).
 *
 * Parity note: the realisation (which numbers a seed produces) is fixed by the
 * generator recipe above, not by the paper; the paper fixes the law.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define HDO_GINIBRE 0
#define HDO_HAAR 1
#define HDO_SIDE_R 0 /* reflectors acting on R^n (input side of Q) */
#define HDO_SIDE_L 1 /* reflectors acting on R^m (output side of Q) */

/* ------------------------------------------------------------------ */
/* Philox4x32-10 and the normal draws                                   */
/* ------------------------------------------------------------------ */

/* One Philox4x32 round: two 32x32->64 products, words permuted and xored
 * with the round key (SC'11, Sec. 5, the Philox-4x32 S-box). */
void hdo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { /* key schedule: Weyl sequence */
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

static double word_to_open_unit(uint32_t w) {
  return ((double)w + 0.5) * (1.0 / 4294967296.0);
}

/* Normal number i of the stream (seed, trial, step, tag). */
static double draw_one(uint32_t seed, uint32_t trial, uint32_t step,
                       uint32_t tag, uint64_t i) {
  uint64_t blk = i >> 2;
  uint32_t ctr[4] = {(uint32_t)(blk & 0xffffffffu), step, tag,
                     (uint32_t)(blk >> 32)};
  uint32_t key[2] = {seed, trial};
  uint32_t w[4];
  hdo_philox4x32_10(ctr, key, w);
  int pair = (int)((i >> 1) & 1u);
  double ua = word_to_open_unit(w[2 * pair]);
  double ub = word_to_open_unit(w[2 * pair + 1]);
  double radius = sqrt(-2.0 * log(ua));
  double angle = 6.283185307179586 * ub;
  return (i & 1u) ? radius * sin(angle) : radius * cos(angle);
}

void hdo_normals(uint32_t seed, uint32_t trial, uint32_t step, uint32_t tag,
                 int64_t i0, int64_t count, double* out) {
  for (int64_t j = 0; j < count; ++j)
    out[j] = draw_one(seed, trial, step, tag, (uint64_t)(i0 + j));
}

/* ------------------------------------------------------------------ */
/* Householder reflectors, eq. (Householder) and eq. (Householder_e)    */
/* ------------------------------------------------------------------ */

typedef struct {
  int64_t k;   /* 1-based first row it acts on */
  int64_t len; /* dim - k + 1 */
  double* u;   /* u = v + s*||v||*e1, length len (NULL if identity) */
  double tau;  /* 2 / (u'u) */
  int s;       /* sign(v1) under the reading above */
  double nu;   /* ||v|| */
  double pivot; /* v1 */
  int ident;   /* 1 when v = 0: H_k(p) = I by convention */
} hdo_refl;

/* Build H(v) for v of length len; forced_sign = 0 follows the rule. */
static int refl_build(hdo_refl* R, int64_t k, const double* v, int64_t len,
                      int forced_sign) {
  double ss = 0.0;
  for (int64_t i = 0; i < len; ++i) ss += v[i] * v[i];
  R->k = k;
  R->len = len;
  R->nu = sqrt(ss);
  R->pivot = len > 0 ? v[0] : 0.0;
  R->u = NULL;
  if (R->nu == 0.0) {
    R->ident = 1;
    R->s = 1;
    R->tau = 0.0;
    return 0;
  }
  R->ident = 0;
  R->s = (v[0] >= 0.0) ? 1 : -1;
  if (forced_sign == 1 || forced_sign == -1) R->s = forced_sign;
  R->u = (double*)malloc((size_t)len * sizeof(double));
  if (!R->u) return -1;
  memcpy(R->u, v, (size_t)len * sizeof(double));
  R->u[0] += (double)R->s * R->nu;
  double uu = 0.0;
  for (int64_t i = 0; i < len; ++i) uu += R->u[i] * R->u[i];
  R->tau = 2.0 / uu;
  return 0;
}

/* z <- H_k(p) z for a full-length vector z (entries before k untouched). */
static void refl_apply(const hdo_refl* R, double* z) {
  if (R->ident) return;
  double* seg = z + (R->k - 1);
  double d = 0.0;
  for (int64_t i = 0; i < R->len; ++i) d += R->u[i] * seg[i];
  double f = R->tau * d;
  double ms = -(double)R->s;
  for (int64_t i = 0; i < R->len; ++i) seg[i] = ms * (seg[i] - f * R->u[i]);
}

/* out <- H(v) z for one vector, used by the tests of the identities in
 * eq. (Householder_property) and eq. (ortho).  Returns 1 for the identity. */
int hdo_apply_householder(const double* v, int64_t len, const double* z,
                          double* out, int forced_sign) {
  hdo_refl R;
  if (refl_build(&R, 1, v, len, forced_sign) != 0) return -1;
  memcpy(out, z, (size_t)len * sizeof(double));
  refl_apply(&R, out);
  int id = R.ident;
  free(R.u);
  return id;
}

/* ------------------------------------------------------------------ */
/* HD state                                                             */
/* ------------------------------------------------------------------ */

typedef struct {
  int ensemble;
  int64_t m, n;
  int tmax;
  uint32_t seed, trial;
  double sigma;
  int t, r, l; /* queries so far, |R| and |L| (Alg. 1 counters) */
  hdo_refl* R; /* R_1..R_r (acting on R^n) */
  hdo_refl* L; /* L_1..L_l (acting on R^m) */
  /* Ginibre basis vectors u_i in R^m, v_i in R^n (Alg. 1) */
  double** U;
  double** V;
  int* kind; /* 0 = query with Q, 1 = query with Q^T, per step */
  int* forceR;
  int* forceL;
} hdo_state;

static void state_free(hdo_state* h) {
  if (!h) return;
  for (int i = 0; i < h->r; ++i) free(h->R[i].u);
  for (int i = 0; i < h->l; ++i) free(h->L[i].u);
  if (h->U)
    for (int i = 0; i < h->t; ++i) free(h->U[i]);
  if (h->V)
    for (int i = 0; i < h->t; ++i) free(h->V[i]);
  free(h->R);
  free(h->L);
  free(h->U);
  free(h->V);
  free(h->kind);
  free(h->forceR);
  free(h->forceL);
  free(h);
}

void hdo_delete(hdo_state* h) { state_free(h); }

hdo_state* hdo_new(int ensemble, int64_t m, int64_t n, int tmax, uint32_t seed,
                   uint32_t trial, double sigma) {
  if (ensemble != HDO_GINIBRE && ensemble != HDO_HAAR) return NULL;
  if (n <= 0 || m <= 0 || tmax < 0) return NULL;
  if (ensemble == HDO_HAAR && m != n) return NULL;
  int64_t cap = m < n ? m : n;
  if (ensemble == HDO_HAAR && tmax > cap) return NULL;
  hdo_state* h = (hdo_state*)calloc(1, sizeof(hdo_state));
  if (!h) return NULL;
  h->ensemble = ensemble;
  h->m = m;
  h->n = n;
  h->tmax = tmax;
  h->seed = seed;
  h->trial = trial;
  h->sigma = (ensemble == HDO_HAAR) ? 1.0 : sigma;
  int cap_t = tmax > 0 ? tmax : 1;
  h->R = (hdo_refl*)calloc((size_t)cap_t, sizeof(hdo_refl));
  h->L = (hdo_refl*)calloc((size_t)cap_t, sizeof(hdo_refl));
  h->kind = (int*)calloc((size_t)cap_t, sizeof(int));
  h->forceR = (int*)calloc((size_t)cap_t, sizeof(int));
  h->forceL = (int*)calloc((size_t)cap_t, sizeof(int));
  if (ensemble == HDO_GINIBRE) {
    h->U = (double**)calloc((size_t)cap_t, sizeof(double*));
    h->V = (double**)calloc((size_t)cap_t, sizeof(double*));
  }
  if (!h->R || !h->L || !h->kind || !h->forceR || !h->forceL ||
      (ensemble == HDO_GINIBRE && (!h->U || !h->V))) {
    state_free(h);
    return NULL;
  }
  return h;
}

void hdo_counts(const hdo_state* h, int* t, int* r, int* l) {
  *t = h->t;
  *r = h->r;
  *l = h->l;
}

/* Mode-B sign following: force the sign of reflector `index1` (1-based) of a
 * side before it is built.  s = 0 restores the rule. */
int hdo_force_sign(hdo_state* h, int side, int index1, int s) {
  if (index1 < 1 || index1 > h->tmax) return -1;
  if (side == HDO_SIDE_R)
    h->forceR[index1 - 1] = s;
  else
    h->forceL[index1 - 1] = s;
  return 0;
}

/* ---- Algorithm 2: Haar ensemble on O(n) ---------------------------- */
/* Q-query:   p_t = R_{t-1}..R_1 x_t,  R_t = H_t(p_t),  L_t = H_t(g_t),
 *            y_t = L_1..L_t R_t p_t.
 * Q^T-query: the same with the roles of {R_i} and {L_i} exchanged.        */
static int haar_query(hdo_state* h, int transpose, const double* x,
                      double* y) {
  int64_t n = h->n;
  int t = h->t + 1; /* 1-based index of this query */
  hdo_refl* D = transpose ? h->L : h->R; /* reflectors built from the data */
  hdo_refl* G = transpose ? h->R : h->L; /* reflectors built from g_t */
  int* forceD = transpose ? h->forceL : h->forceR;
  int* forceG = transpose ? h->forceR : h->forceL;
  double* g = (double*)malloc((size_t)n * sizeof(double));
  double* p = (double*)malloc((size_t)n * sizeof(double));
  if (!g || !p) {
    free(g);
    free(p);
    return -1;
  }
  hdo_normals(h->seed, h->trial, (uint32_t)t, 0u, 0, n, g);
  memcpy(p, x, (size_t)n * sizeof(double));
  for (int j = 0; j < t - 1; ++j) refl_apply(&D[j], p); /* eq. (pt) */
  int rc = refl_build(&D[t - 1], t, p + (t - 1), n - t + 1, forceD[t - 1]);
  if (rc == 0)
    rc = refl_build(&G[t - 1], t, g + (t - 1), n - t + 1, forceG[t - 1]);
  if (rc != 0) {
    free(g);
    free(p);
    return -1;
  }
  memcpy(y, p, (size_t)n * sizeof(double));
  refl_apply(&D[t - 1], y);                            /* R_t p_t */
  for (int j = t - 1; j >= 0; --j) refl_apply(&G[j], y); /* L_1..L_t (.) */
  h->t = t;
  h->r = t;
  h->l = t;
  h->kind[t - 1] = transpose;
  free(g);
  free(p);
  return 0;
}

/* ---- Algorithm 1: Ginibre ensemble GE(m,n) ------------------------- */
/* Q-query:   r++, g_t ~ GE(m,1), R_r = H_r(R_{r-1}..R_1 x_t),
 *            u_t = L_1..L_l Z_{1:l} g_t, v_t = R_1..R_r e_r,
 *            y_t = sum_{i<=t} (v_i' x_t) u_i.
 * Q^T-query: l++, g_t ~ GE(n,1), L_l = H_l(L_{l-1}..L_1 x_t),
 *            u_t = L_1..L_l e_l, v_t = R_1..R_r Z_{1:r} g_t,
 *            y_t = sum_{i<=t} (u_i' x_t) v_i.
 * The entries of Q have variance sigma^2: the output is scaled by sigma. */
static int ginibre_query(hdo_state* h, int transpose, const double* x,
                         double* y) {
  int64_t m = h->m, n = h->n;
  int t = h->t + 1;
  int64_t din = transpose ? m : n;   /* length of x */
  int64_t dout = transpose ? n : m;  /* length of y */
  double* g = (double*)malloc((size_t)dout * sizeof(double));
  double* p = (double*)malloc((size_t)din * sizeof(double));
  double* ut = (double*)calloc((size_t)m, sizeof(double));
  double* vt = (double*)calloc((size_t)n, sizeof(double));
  if (!g || !p || !ut || !vt) goto fail;
  hdo_normals(h->seed, h->trial, (uint32_t)t, 0u, 0, dout, g);
  memcpy(p, x, (size_t)din * sizeof(double));
  if (!transpose) {
    int r = h->r + 1;
    for (int j = 0; j < r - 1; ++j) refl_apply(&h->R[j], p);
    if (refl_build(&h->R[r - 1], r, p + (r - 1), n - r + 1,
                   h->forceR[r - 1]) != 0)
      goto fail;
    /* u_t = L_1..L_l Z_{1:l} g_t */
    for (int64_t i = h->l; i < m; ++i) ut[i] = g[i];
    for (int j = h->l - 1; j >= 0; --j) refl_apply(&h->L[j], ut);
    /* v_t = R_1..R_r e_r */
    vt[r - 1] = 1.0;
    for (int j = r - 1; j >= 0; --j) refl_apply(&h->R[j], vt);
    h->r = r;
  } else {
    int l = h->l + 1;
    for (int j = 0; j < l - 1; ++j) refl_apply(&h->L[j], p);
    if (refl_build(&h->L[l - 1], l, p + (l - 1), m - l + 1,
                   h->forceL[l - 1]) != 0)
      goto fail;
    /* u_t = L_1..L_l e_l */
    ut[l - 1] = 1.0;
    for (int j = l - 1; j >= 0; --j) refl_apply(&h->L[j], ut);
    /* v_t = R_1..R_r Z_{1:r} g_t */
    for (int64_t i = h->r; i < n; ++i) vt[i] = g[i];
    for (int j = h->r - 1; j >= 0; --j) refl_apply(&h->R[j], vt);
    h->l = l;
  }
  h->U[t - 1] = ut;
  h->V[t - 1] = vt;
  h->kind[t - 1] = transpose;
  h->t = t;
  for (int64_t i = 0; i < dout; ++i) y[i] = 0.0;
  for (int i = 0; i < t; ++i) {
    const double* a = transpose ? h->U[i] : h->V[i]; /* dotted with x */
    const double* b = transpose ? h->V[i] : h->U[i]; /* accumulated */
    double c = 0.0;
    for (int64_t j = 0; j < din; ++j) c += a[j] * x[j];
    for (int64_t j = 0; j < dout; ++j) y[j] += c * b[j];
  }
  for (int64_t j = 0; j < dout; ++j) y[j] *= h->sigma;
  free(g);
  free(p);
  return 0;
fail:
  free(g);
  free(p);
  free(ut);
  free(vt);
  return -1;
}

/* One query of the dynamics: y = Q x (transpose = 0) or y = Q' x.
 * Returns 0, -1 on allocation failure, -2 when the capacity T <= min(m,n)
 * of Algorithms 1 and 2 would be exceeded (state unchanged). */
int hdo_query(hdo_state* h, int transpose, const double* x, double* y) {
  if (h->t >= h->tmax) return -2;
  if (h->ensemble == HDO_HAAR) {
    if (h->t >= h->n) return -2;
    return haar_query(h, transpose, x, y);
  }
  if (!transpose && h->r >= h->n) return -2;
  if (transpose && h->l >= h->m) return -2;
  return ginibre_query(h, transpose, x, y);
}

/* Read back reflector `index1` (1-based) of a side: u is written to
 * u_out[0..len-1] where len = dim - k + 1 (zeros when it is the identity). */
int hdo_reflector(const hdo_state* h, int side, int index1, double* u_out,
                  double* tau, int* sign, double* nu, double* pivot,
                  int* ident) {
  int cnt = (side == HDO_SIDE_R) ? h->r : h->l;
  if (index1 < 1 || index1 > cnt) return -1;
  const hdo_refl* R = (side == HDO_SIDE_R) ? &h->R[index1 - 1]
                                           : &h->L[index1 - 1];
  if (R->ident)
    memset(u_out, 0, (size_t)R->len * sizeof(double));
  else
    memcpy(u_out, R->u, (size_t)R->len * sizeof(double));
  *tau = R->tau;
  *sign = R->s;
  *nu = R->nu;
  *pivot = R->pivot;
  *ident = R->ident;
  return 0;
}

/* Ginibre basis vectors of step `step1` (1-based): u in R^m, v in R^n. */
int hdo_basis(const hdo_state* h, int step1, double* u_out, double* v_out) {
  if (h->ensemble != HDO_GINIBRE || step1 < 1 || step1 > h->t) return -1;
  memcpy(u_out, h->U[step1 - 1], (size_t)h->m * sizeof(double));
  memcpy(v_out, h->V[step1 - 1], (size_t)h->n * sizeof(double));
  return 0;
}
