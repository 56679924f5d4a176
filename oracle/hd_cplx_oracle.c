/*
 * hd_cplx_oracle.c -- plain FP64 CPU reference for the complex-valued
 * Householder Dice (HD) of Sec. 3.4 (Y. M. Lu, arXiv 2101.07464).
 *
 * TEST INFRASTRUCTURE ONLY.  Like hd_oracle.c, this file is the oracle the GPU
 * library is checked against; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it, and it shares no code with the
 * HIP sources.
 *
 * What it computes:
 *   - the unitary reflector H(v) of eq. (Householder_c): with
 *     v_1 / ||v|| = r e^{i theta} (theta = 0 when v_1 = 0),
 *       H(v) = (-e^{-i theta}) [I - w w^H / (1 + r)],
 *       w = v / ||v|| + e^{i theta} e_1,
 *     so that H(v) v = ||v|| e_1 and H(v)^H e_1 = v / ||v||; H_k(p) acts on
 *     entries k..dim as in eq. (Householder_e) and is the identity when
 *     p[k:dim] = 0;
 *   - Algorithm 2 on the unitary group U(n) and Algorithm 1 on the complex
 *     Ginibre ensemble, with the conjugate transpose in place of the
 *     transpose.  The real algorithms use that a real reflector is its own
 *     transpose; a unitary reflector is not Hermitian, so each place where
 *     the real algorithm applies a reflector to produce an output (or a
 *     basis vector of the output space) applies its conjugate transpose here
 *     (the reading behind this: Q is written as L_1^H..L_t^H D R_t..R_1, which
 *     for real reflectors is the factorisation the real algorithms use):
 *       Haar, y = Q x:   p = R_{t-1}..R_1 x,  R_t = H_t(p),  L_t = H_t(g_t),
 *                        y = L_1^H..L_t^H R_t p;
 *       Haar, y = Q^H x: the same with the roles of {R_i} and {L_i} exchanged;
 *       Ginibre, y = Q x:   r++, R_r = H_r(R_{r-1}..R_1 x),
 *                           u_t = L_1^H..L_l^H Z_{1:l} g_t,
 *                           v_t = R_1^H..R_r^H e_r,
 *                           y = sigma sum_{i<=t} (v_i^H x) u_i;
 *       Ginibre, y = Q^H x: l++, L_l = H_l(L_{l-1}..L_1 x),
 *                           u_t = L_1^H..L_l^H e_l,
 *                           v_t = R_1^H..R_r^H Z_{1:r} g_t,
 *                           y = sigma sum_{i<=t} (u_i^H x) v_i.
 *     Every reflector is applied one at a time, in the algorithms' order.
 *
 * Complex normal draws: entry i of a complex stream is
 * (N_{2i} + i N_{2i+1}) / sqrt(2), where N_j is normal j of the real stream
 * (seed, trial, step, tag) of hd_oracle.c, so E|g_i|^2 = 1.  The entries of
 * the complex Ginibre matrix have E|Q_ij|^2 = sigma^2 (real and imaginary
 * parts N(0, sigma^2 / 2)).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define HDOC_GINIBRE 0
#define HDOC_HAAR 1
#define HDOC_SIDE_R 0 /* reflectors acting on C^n (input side of Q) */
#define HDOC_SIDE_L 1 /* reflectors acting on C^m (output side of Q) */

typedef double complex cplx;

/* real normals of hd_oracle.c (the same library) */
void hdo_normals(uint32_t seed, uint32_t trial, uint32_t step, uint32_t tag,
                 int64_t i0, int64_t count, double* out);

/* Complex normals i0..i0+count-1 of the stream (seed, trial, step, tag). */
void hdoc_normals(uint32_t seed, uint32_t trial, uint32_t step, uint32_t tag,
                  int64_t i0, int64_t count, cplx* out) {
  if (count <= 0) return;
  double* re = (double*)malloc((size_t)(2 * count) * sizeof(double));
  if (!re) {
    for (int64_t i = 0; i < count; ++i) out[i] = NAN;
    return;
  }
  hdo_normals(seed, trial, step, tag, 2 * i0, 2 * count, re);
  const double s = 1.0 / sqrt(2.0);
  for (int64_t i = 0; i < count; ++i)
    out[i] = CMPLX(re[2 * i] * s, re[2 * i + 1] * s);
  free(re);
}

/* ------------------------------------------------------------------ */
/* The unitary reflector of eq. (Householder_c)                         */
/* ------------------------------------------------------------------ */

typedef struct {
  int64_t k;    /* 1-based first entry it acts on */
  int64_t len;  /* dim - k + 1 */
  cplx* w;      /* w = v/||v|| + e^{i theta} e_1 (NULL for the identity) */
  double r;     /* |v_1| / ||v|| */
  double theta; /* arg v_1, 0 when v_1 = 0 */
  double nu;    /* ||v|| */
  cplx pivot;   /* v_1 */
  int ident;    /* 1 when v = 0 */
} hdoc_refl;

static int crefl_build(hdoc_refl* R, int64_t k, const cplx* v, int64_t len) {
  double ss = 0.0;
  for (int64_t i = 0; i < len; ++i)
    ss += creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);
  R->k = k;
  R->len = len;
  R->nu = sqrt(ss);
  R->pivot = len > 0 ? v[0] : 0.0;
  R->w = NULL;
  if (R->nu == 0.0) {
    R->ident = 1;
    R->r = 0.0;
    R->theta = 0.0;
    return 0;
  }
  R->ident = 0;
  R->r = cabs(v[0]) / R->nu;
  R->theta = (v[0] == 0.0) ? 0.0 : carg(v[0]);
  R->w = (cplx*)malloc((size_t)len * sizeof(cplx));
  if (!R->w) return -1;
  for (int64_t i = 0; i < len; ++i) R->w[i] = v[i] / R->nu;
  R->w[0] += cexp(I * R->theta);
  return 0;
}

/* z <- H_k(p) z (adjoint = 0) or z <- H_k(p)^H z (adjoint = 1) for a
 * full-length z; entries before k are untouched. */
static void crefl_apply(const hdoc_refl* R, int adjoint, cplx* z) {
  if (R->ident) return;
  cplx* seg = z + (R->k - 1);
  cplx d = 0.0;
  for (int64_t i = 0; i < R->len; ++i) d += conj(R->w[i]) * seg[i];
  const cplx f = d / (1.0 + R->r);
  const cplx ph = adjoint ? -cexp(I * R->theta) : -cexp(-I * R->theta);
  for (int64_t i = 0; i < R->len; ++i) seg[i] = ph * (seg[i] - f * R->w[i]);
}

/* out <- H(v) z or H(v)^H z for one vector (the identities below eq.
 * (Householder_c) are tested through this).  Returns 1 for the identity,
 * -1 on allocation failure. */
int hdoc_apply_householder(const cplx* v, int64_t len, const cplx* z,
                           int adjoint, cplx* out) {
  hdoc_refl R;
  if (crefl_build(&R, 1, v, len) != 0) return -1;
  memcpy(out, z, (size_t)len * sizeof(cplx));
  crefl_apply(&R, adjoint, out);
  const int id = R.ident;
  free(R.w);
  return id;
}

/* ------------------------------------------------------------------ */
/* State                                                                */
/* ------------------------------------------------------------------ */

typedef struct {
  int ensemble;
  int64_t m, n;
  int tmax;
  uint32_t seed, trial;
  double sigma;
  int t, r, l;
  hdoc_refl* R; /* acting on C^n */
  hdoc_refl* L; /* acting on C^m */
  cplx** U;     /* Ginibre basis vectors u_i in C^m */
  cplx** V;     /* and v_i in C^n */
  int* kind;    /* 0 = query with Q, 1 = with Q^H */
} hdoc_state;

static void cstate_free(hdoc_state* h) {
  if (!h) return;
  for (int i = 0; i < h->r; ++i) free(h->R[i].w);
  for (int i = 0; i < h->l; ++i) free(h->L[i].w);
  if (h->U)
    for (int i = 0; i < h->t; ++i) free(h->U[i]);
  if (h->V)
    for (int i = 0; i < h->t; ++i) free(h->V[i]);
  free(h->R);
  free(h->L);
  free(h->U);
  free(h->V);
  free(h->kind);
  free(h);
}

void hdoc_delete(hdoc_state* h) { cstate_free(h); }

hdoc_state* hdoc_new(int ensemble, int64_t m, int64_t n, int tmax,
                     uint32_t seed, uint32_t trial, double sigma) {
  if (ensemble != HDOC_GINIBRE && ensemble != HDOC_HAAR) return NULL;
  if (n <= 0 || m <= 0 || tmax < 0) return NULL;
  if (ensemble == HDOC_HAAR && (m != n || tmax > n)) return NULL;
  hdoc_state* h = (hdoc_state*)calloc(1, sizeof(hdoc_state));
  if (!h) return NULL;
  h->ensemble = ensemble;
  h->m = m;
  h->n = n;
  h->tmax = tmax;
  h->seed = seed;
  h->trial = trial;
  h->sigma = ensemble == HDOC_HAAR ? 1.0 : sigma;
  const int cap = tmax > 0 ? tmax : 1;
  h->R = (hdoc_refl*)calloc((size_t)cap, sizeof(hdoc_refl));
  h->L = (hdoc_refl*)calloc((size_t)cap, sizeof(hdoc_refl));
  h->kind = (int*)calloc((size_t)cap, sizeof(int));
  if (ensemble == HDOC_GINIBRE) {
    h->U = (cplx**)calloc((size_t)cap, sizeof(cplx*));
    h->V = (cplx**)calloc((size_t)cap, sizeof(cplx*));
  }
  if (!h->R || !h->L || !h->kind ||
      (ensemble == HDOC_GINIBRE && (!h->U || !h->V))) {
    cstate_free(h);
    return NULL;
  }
  return h;
}

void hdoc_counts(const hdoc_state* h, int* t, int* r, int* l) {
  *t = h->t;
  *r = h->r;
  *l = h->l;
}

/* ---- Algorithm 2 on U(n) ------------------------------------------- */
static int chaar_query(hdoc_state* h, int adjoint, const cplx* x, cplx* y) {
  const int64_t n = h->n;
  const int t = h->t + 1;
  hdoc_refl* D = adjoint ? h->L : h->R; /* built from the data */
  hdoc_refl* G = adjoint ? h->R : h->L; /* built from g_t */
  cplx* g = (cplx*)malloc((size_t)n * sizeof(cplx));
  cplx* p = (cplx*)malloc((size_t)n * sizeof(cplx));
  int rc = -1;
  if (!g || !p) goto done;
  hdoc_normals(h->seed, h->trial, (uint32_t)t, 0u, 0, n, g);
  memcpy(p, x, (size_t)n * sizeof(cplx));
  for (int j = 0; j < t - 1; ++j) crefl_apply(&D[j], 0, p);
  if (crefl_build(&D[t - 1], t, p + (t - 1), n - t + 1) != 0) goto done;
  if (crefl_build(&G[t - 1], t, g + (t - 1), n - t + 1) != 0) goto done;
  memcpy(y, p, (size_t)n * sizeof(cplx));
  crefl_apply(&D[t - 1], 0, y);                            /* R_t p */
  for (int j = t - 1; j >= 0; --j) crefl_apply(&G[j], 1, y); /* L_1^H.. */
  h->t = t;
  h->r = t;
  h->l = t;
  h->kind[t - 1] = adjoint;
  rc = 0;
done:
  free(g);
  free(p);
  return rc;
}

/* ---- Algorithm 1 on the complex Ginibre ensemble --------------------- */
static int cginibre_query(hdoc_state* h, int adjoint, const cplx* x,
                          cplx* y) {
  const int64_t m = h->m, n = h->n;
  const int t = h->t + 1;
  const int64_t din = adjoint ? m : n, dout = adjoint ? n : m;
  cplx* g = (cplx*)malloc((size_t)dout * sizeof(cplx));
  cplx* p = (cplx*)malloc((size_t)din * sizeof(cplx));
  cplx* ut = (cplx*)calloc((size_t)m, sizeof(cplx));
  cplx* vt = (cplx*)calloc((size_t)n, sizeof(cplx));
  if (!g || !p || !ut || !vt) goto fail;
  hdoc_normals(h->seed, h->trial, (uint32_t)t, 0u, 0, dout, g);
  memcpy(p, x, (size_t)din * sizeof(cplx));
  if (!adjoint) {
    const int r = h->r + 1;
    for (int j = 0; j < r - 1; ++j) crefl_apply(&h->R[j], 0, p);
    if (crefl_build(&h->R[r - 1], r, p + (r - 1), n - r + 1) != 0) goto fail;
    for (int64_t i = h->l; i < m; ++i) ut[i] = g[i]; /* Z_{1:l} g_t */
    for (int j = h->l - 1; j >= 0; --j) crefl_apply(&h->L[j], 1, ut);
    vt[r - 1] = 1.0;
    for (int j = r - 1; j >= 0; --j) crefl_apply(&h->R[j], 1, vt);
    h->r = r;
  } else {
    const int l = h->l + 1;
    for (int j = 0; j < l - 1; ++j) crefl_apply(&h->L[j], 0, p);
    if (crefl_build(&h->L[l - 1], l, p + (l - 1), m - l + 1) != 0) goto fail;
    ut[l - 1] = 1.0;
    for (int j = l - 1; j >= 0; --j) crefl_apply(&h->L[j], 1, ut);
    for (int64_t i = h->r; i < n; ++i) vt[i] = g[i]; /* Z_{1:r} g_t */
    for (int j = h->r - 1; j >= 0; --j) crefl_apply(&h->R[j], 1, vt);
    h->l = l;
  }
  h->U[t - 1] = ut;
  h->V[t - 1] = vt;
  h->kind[t - 1] = adjoint;
  h->t = t;
  for (int64_t i = 0; i < dout; ++i) y[i] = 0.0;
  for (int i = 0; i < t; ++i) {
    const cplx* a = adjoint ? h->U[i] : h->V[i]; /* dotted with x */
    const cplx* b = adjoint ? h->V[i] : h->U[i]; /* accumulated */
    cplx c = 0.0;
    for (int64_t j = 0; j < din; ++j) c += conj(a[j]) * x[j];
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

/* One query: y = Q x (adjoint = 0) or y = Q^H x.  Returns 0, -1 on
 * allocation failure, -2 when the capacity would be exceeded. */
int hdoc_query(hdoc_state* h, int adjoint, const cplx* x, cplx* y) {
  if (h->t >= h->tmax) return -2;
  if (h->ensemble == HDOC_HAAR) return chaar_query(h, adjoint, x, y);
  if (!adjoint && h->r >= h->n) return -2;
  if (adjoint && h->l >= h->m) return -2;
  return cginibre_query(h, adjoint, x, y);
}

/* Reflector `index1` (1-based) of a side: w (len = dim - k + 1 entries,
 * zeros for the identity), r, theta, nu, pivot, ident. */
int hdoc_reflector(const hdoc_state* h, int side, int index1, cplx* w_out,
                   double* r, double* theta, double* nu, cplx* pivot,
                   int* ident) {
  const int cnt = side == HDOC_SIDE_R ? h->r : h->l;
  if (index1 < 1 || index1 > cnt) return -1;
  const hdoc_refl* R =
      side == HDOC_SIDE_R ? &h->R[index1 - 1] : &h->L[index1 - 1];
  if (R->ident)
    memset(w_out, 0, (size_t)R->len * sizeof(cplx));
  else
    memcpy(w_out, R->w, (size_t)R->len * sizeof(cplx));
  *r = R->r;
  *theta = R->theta;
  *nu = R->nu;
  *pivot = R->pivot;
  *ident = R->ident;
  return 0;
}

/* Ginibre basis vectors of step `step1` (1-based): u in C^m, v in C^n. */
int hdoc_basis(const hdoc_state* h, int step1, cplx* u_out, cplx* v_out) {
  if (h->ensemble != HDOC_GINIBRE || step1 < 1 || step1 > h->t) return -1;
  memcpy(u_out, h->U[step1 - 1], (size_t)h->m * sizeof(cplx));
  memcpy(v_out, h->V[step1 - 1], (size_t)h->n * sizeof(cplx));
  return 0;
}
