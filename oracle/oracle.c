/*
 * CPU oracle for the iterative refinement of Schur decompositions
 * (Bujanovic, Kressner, Schroder, arXiv 2203.10879).
 *
 * TEST INFRASTRUCTURE ONLY: called by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg. It shares no code with the GPU library.
 *
 * Plain, slow and direct: triple-loop products in IEEE binary128, the paper's
 * steps in the paper's order. OpenMP only splits independent output columns.
 * See oracle.h for the entry points and what pins each one.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 quad;

/* ---------------------------------------------------------------- lp variants */
#define R float
#define SUF f
#define R_SQRT sqrtf
#define R_HYPOT hypotf
#define R_EPS (FLT_EPSILON * 0.5f)
#define R_FINITE isfinite
#include "oracle_lp.inc"
#undef R
#undef SUF
#undef R_SQRT
#undef R_HYPOT
#undef R_EPS
#undef R_FINITE

#define R double
#define SUF d
#define R_SQRT sqrt
#define R_HYPOT hypot
#define R_EPS (DBL_EPSILON * 0.5)
#define R_FINITE isfinite
#include "oracle_lp.inc"
#undef R
#undef SUF
#undef R_SQRT
#undef R_HYPOT
#undef R_EPS
#undef R_FINITE

static int quad_finite(quad x) { return !isnanq(x) && !isinfq(x); }
#define R quad
#define SUF q
#define R_SQRT sqrtq
#define R_HYPOT hypotq
#define R_EPS (FLT128_EPSILON * 0.5Q)
#define R_FINITE quad_finite
#include "oracle_lp.inc"
#undef R
#undef SUF
#undef R_SQRT
#undef R_HYPOT
#undef R_EPS
#undef R_FINITE

/* ------------------------------------------------------------ hp complex math */
static inline orc_qc qc_mk(quad re, quad im)
{
  orc_qc z;
  z.re = re;
  z.im = im;
  return z;
}
static inline quad qc_abs2(orc_qc a) { return a.re * a.re + a.im * a.im; }

static void* xmalloc(size_t bytes)
{
  void* p = malloc(bytes ? bytes : 1);
  if (!p) abort();
  return p;
}
#define NEWQ(count) ((orc_qc*)xmalloc(sizeof(orc_qc) * (size_t)(count)))

static quad fro2(const orc_qc* X, long count)
{
  quad s = 0;
  for (long z = 0; z < count; z++) s += qc_abs2(X[z]);
  return s;
}

/* ---------------------------------------------------------------- conversions */
void orc_from_dd(long count, const double* hi, const double* lo, orc_qc* out)
{
  for (long z = 0; z < count; z++) {
    quad re = (quad)hi[2 * z], im = (quad)hi[2 * z + 1];
    if (lo) {
      re += (quad)lo[2 * z];
      im += (quad)lo[2 * z + 1];
    }
    out[z] = qc_mk(re, im);
  }
}

void orc_to_dd(long count, const orc_qc* in, double* hi, double* lo)
{
  for (long z = 0; z < count; z++) {
    double hr = (double)in[z].re, hi_ = (double)in[z].im;
    hi[2 * z] = hr;
    hi[2 * z + 1] = hi_;
    if (lo) {
      lo[2 * z] = (double)(in[z].re - (quad)hr);
      lo[2 * z + 1] = (double)(in[z].im - (quad)hi_);
    }
  }
}

/* --------------------------------------------------------------- hp products */
void orc_gemm(int opa, int m, int n, int k, const orc_qc* A, const orc_qc* B, orc_qc* C)
{
#pragma omp parallel for schedule(static)
  for (int j = 0; j < n; j++) {
    for (int i = 0; i < m; i++) {
      quad sr = 0, si = 0;
      for (int p = 0; p < k; p++) {
        quad ar, ai;
        if (opa) {
          ar = A[p + (long)i * k].re;
          ai = -A[p + (long)i * k].im;
        } else {
          ar = A[i + (long)p * m].re;
          ai = A[i + (long)p * m].im;
        }
        quad br = B[p + (long)j * k].re, bi = B[p + (long)j * k].im;
        sr += ar * br - ai * bi;
        si += ar * bi + ai * br;
      }
      C[i + (long)j * m] = qc_mk(sr, si);
    }
  }
}

/* ----------------------------------------------------- lp dispatch (3 kinds) */
static void* lp_alloc(int lp, long count)
{
  size_t sz = lp == ORC_LP_FLOAT ? sizeof(lc_f) : lp == ORC_LP_DOUBLE ? sizeof(lc_d) : sizeof(lc_q);
  return xmalloc(sz * (size_t)count);
}
static void lp_from_q(int lp, long count, const orc_qc* x, void* out)
{
  for (long z = 0; z < count; z++) {
    if (lp == ORC_LP_FLOAT) ((lc_f*)out)[z] = lc_from_q_f(x[z]);
    else if (lp == ORC_LP_DOUBLE) ((lc_d*)out)[z] = lc_from_q_d(x[z]);
    else ((lc_q*)out)[z] = lc_from_q_q(x[z]);
  }
}
static void lp_to_q(int lp, long count, const void* x, orc_qc* out)
{
  for (long z = 0; z < count; z++) {
    if (lp == ORC_LP_FLOAT) out[z] = lc_to_q_f(((const lc_f*)x)[z]);
    else if (lp == ORC_LP_DOUBLE) out[z] = lc_to_q_d(((const lc_d*)x)[z]);
    else out[z] = lc_to_q_q(((const lc_q*)x)[z]);
  }
}
/* C = A B in lp for hp operands: both rounded to lp, product formed in lp,
 * widened back exactly. */
static void lp_product(int lp, int n, const orc_qc* A, const orc_qc* B, orc_qc* C)
{
  long nn = (long)n * n;
  void* a = lp_alloc(lp, nn);
  void* b = lp_alloc(lp, nn);
  void* c = lp_alloc(lp, nn);
  lp_from_q(lp, nn, A, a);
  lp_from_q(lp, nn, B, b);
  if (lp == ORC_LP_FLOAT) lp_gemm_f(n, n, n, (lc_f*)a, (lc_f*)b, (lc_f*)c);
  else if (lp == ORC_LP_DOUBLE) lp_gemm_d(n, n, n, (lc_d*)a, (lc_d*)b, (lc_d*)c);
  else lp_gemm_q(n, n, n, (lc_q*)a, (lc_q*)b, (lc_q*)c);
  lp_to_q(lp, nn, c, C);
  free(a);
  free(b);
  free(c);
}

int orc_trisolve(int lp, int order, int n, const orc_qc* T, const orc_qc* E, orc_qc* L,
                 double trunc)
{
  long nn = (long)n * n;
  orc_qc* Tu = NEWQ(nn);
  orc_qc* El = NEWQ(nn);
  for (int j = 0; j < n; j++)
    for (int i = 0; i < n; i++) {
      long z = i + (long)j * n;
      Tu[z] = i <= j ? T[z] : qc_mk(0, 0);
      El[z] = i > j ? E[z] : qc_mk(0, 0);
    }
  void* t = lp_alloc(lp, nn);
  void* e = lp_alloc(lp, nn);
  void* l = lp_alloc(lp, nn);
  lp_from_q(lp, nn, Tu, t);
  lp_from_q(lp, nn, El, e);
  int rc;
  if (lp == ORC_LP_FLOAT) rc = trisolve_f(n, order, (lc_f*)t, (lc_f*)e, (lc_f*)l, trunc);
  else if (lp == ORC_LP_DOUBLE) rc = trisolve_d(n, order, (lc_d*)t, (lc_d*)e, (lc_d*)l, trunc);
  else rc = trisolve_q(n, order, (lc_q*)t, (lc_q*)e, (lc_q*)l, trunc);
  lp_to_q(lp, nn, l, L);
  free(t);
  free(e);
  free(l);
  free(Tu);
  free(El);
  return rc;
}

/* ------------------------------------------------------------ orthogonalising */
void orc_ns(int n, const orc_qc* Qh, orc_qc* Q)
{
  long nn = (long)n * n;
  orc_qc* G = NEWQ(nn);
  orc_gemm(1, n, n, n, Qh, Qh, G); /* G = Qh^H Qh */
  for (int j = 0; j < n; j++)      /* G <- 3I - G  */
    for (int i = 0; i < n; i++) {
      long z = i + (long)j * n;
      G[z].re = (i == j ? (quad)3 : (quad)0) - G[z].re;
      G[z].im = -G[z].im;
    }
  orc_gemm(0, n, n, n, Qh, G, Q); /* Q = Qh (3I - G) */
  for (long z = 0; z < nn; z++) {
    Q[z].re /= 2;
    Q[z].im /= 2;
  }
  free(G);
}

void orc_ns_merged(int lp, int n, const orc_qc* Q, const orc_qc* W, int full, orc_qc* Qn)
{
  long nn = (long)n * n;
  orc_qc* Y = NEWQ(nn);
  orc_qc* YW = NEWQ(nn);
  orc_qc* W2 = NEWQ(nn);
  orc_qc* W3 = NEWQ(nn);
  orc_qc* W2Y = NEWQ(nn);
  orc_qc* W2YW = NEWQ(nn);
  orc_qc* S = NEWQ(nn);
  orc_gemm(1, n, n, n, Q, Q, Y); /* Y = Q^H Q - I (hp) */
  for (int i = 0; i < n; i++) Y[i + (long)i * n].re -= 1;
  lp_product(lp, n, Y, W, YW); /* Y W   (lp) */
  lp_product(lp, n, W, W, W2); /* W^2   (lp) */
  lp_product(lp, n, W2, W, W3); /* W^3  (lp) */
  if (full) {
    lp_product(lp, n, W2, Y, W2Y);     /* W^2 Y   (lp) */
    lp_product(lp, n, W2Y, W, W2YW);   /* W^2 Y W (lp) */
  }
  /* Sigma = 2I + 2W - Y - YW + W^2 + W^3 [+ W^2 Y + W^2 Y W]  (hp sum) */
  for (int j = 0; j < n; j++)
    for (int i = 0; i < n; i++) {
      long z = i + (long)j * n;
      quad re = (i == j ? (quad)2 : (quad)0) + 2 * W[z].re - Y[z].re - YW[z].re + W2[z].re + W3[z].re;
      quad im = 2 * W[z].im - Y[z].im - YW[z].im + W2[z].im + W3[z].im;
      if (full) {
        re += W2Y[z].re + W2YW[z].re;
        im += W2Y[z].im + W2YW[z].im;
      }
      S[z] = qc_mk(re, im);
    }
  orc_gemm(0, n, n, n, Q, S, Qn); /* Qn = 1/2 Q Sigma (hp) */
  for (long z = 0; z < nn; z++) {
    Qn[z].re /= 2;
    Qn[z].im /= 2;
  }
  free(Y);
  free(YW);
  free(W2);
  free(W3);
  free(W2Y);
  free(W2YW);
  free(S);
}

/* ---------------------------------------------------------------- Algorithm 4 */
int orc_refine(int lp, int n, const orc_qc* A, const orc_qc* Qh, int maxit, double tol,
               int flags, orc_qc* Qout, orc_qc* Tout, double* hist, int* iters)
{
  long nn = (long)n * n;
  orc_qc* Q = NEWQ(nn);
  orc_qc* Qn = NEWQ(nn);
  orc_qc* AQ = NEWQ(nn);
  orc_qc* Th = NEWQ(nn);
  orc_qc* T = NEWQ(nn);
  orc_qc* E = NEWQ(nn);
  orc_qc* L = NEWQ(nn);
  orc_qc* W = NEWQ(nn);
  int status = ORC_NOT_CONVERGED, passes = 0;
  double trunc = (flags & ORC_TRUNC) ? 1e-5 : 0.0;

  orc_ns(n, Qh, Q); /* Q = 1/2 Qh (3I - Qh^H Qh) */
  quad normA = sqrtq(fro2(A, nn));

  for (int p = 0; p < maxit; p++) {
    orc_gemm(0, n, n, n, A, Q, AQ); /* That = Q^H A Q */
    orc_gemm(1, n, n, n, Q, AQ, Th);
    for (int j = 0; j < n; j++) /* E = stril(That), T = That - E */
      for (int i = 0; i < n; i++) {
        long z = i + (long)j * n;
        E[z] = i > j ? Th[z] : qc_mk(0, 0);
        T[z] = i > j ? qc_mk(0, 0) : Th[z];
      }
    quad eps = sqrtq(fro2(E, nn)) / normA;
    hist[p] = (double)eps;
    passes = p + 1;
    memcpy(Tout, T, sizeof(orc_qc) * (size_t)nn);
    if (!quad_finite(eps)) {
      status = ORC_BREAKDOWN;
      break;
    }
    if (eps <= (quad)tol) {
      status = ORC_OK;
      break;
    }
    if (p >= 2 && hist[p] > hist[p - 1] && hist[p - 1] > hist[p - 2]) {
      status = ORC_DIVERGED;
      break;
    }
    if (p == maxit - 1) break; /* no update after the last evaluation */
    if (orc_trisolve(lp, 0, n, T, E, L, trunc) != ORC_OK) {
      status = ORC_BREAKDOWN;
      break;
    }
    for (int j = 0; j < n; j++) /* W = L - L^H */
      for (int i = 0; i < n; i++) {
        orc_qc a = L[i + (long)j * n], b = L[j + (long)i * n];
        W[i + (long)j * n] = qc_mk(a.re - b.re, a.im + b.im);
      }
    orc_ns_merged(lp, n, Q, W, flags & ORC_FULL_NS, Qn);
    orc_qc* tmp = Q;
    Q = Qn;
    Qn = tmp;
  }
  memcpy(Qout, Q, sizeof(orc_qc) * (size_t)nn);
  *iters = passes;
  free(Q);
  free(Qn);
  free(AQ);
  free(Th);
  free(T);
  free(E);
  free(L);
  free(W);
  return status;
}

/* ------------------------------------------------------------------ evaluation */
void orc_eval(int n, const orc_qc* A, const orc_qc* Q, const orc_qc* T, double out[4])
{
  long nn = (long)n * n;
  orc_qc* AQ = NEWQ(nn);
  orc_qc* Th = NEWQ(nn);
  orc_qc* G = NEWQ(nn);
  orc_gemm(0, n, n, n, A, Q, AQ);
  orc_gemm(1, n, n, n, Q, AQ, Th);
  orc_gemm(1, n, n, n, Q, Q, G);
  quad s = 0, o = 0, t = 0;
  for (int j = 0; j < n; j++)
    for (int i = 0; i < n; i++) {
      long z = i + (long)j * n;
      if (i > j) s += qc_abs2(Th[z]);
      orc_qc g = G[z];
      if (i == j) g.re -= 1;
      o += qc_abs2(g);
      if (T) {
        orc_qc d = T[z];
        if (i <= j) {
          d.re -= Th[z].re;
          d.im -= Th[z].im;
        }
        t += qc_abs2(d);
      }
    }
  quad normA = sqrtq(fro2(A, nn));
  out[0] = (double)(sqrtq(s) / normA);
  out[1] = (double)sqrtq(o);
  out[2] = (double)sqrtq(t);
  out[3] = (double)normA;
  free(AQ);
  free(Th);
  free(G);
}

void orc_eval_rows(int n, const orc_qc* A, const orc_qc* Q, int nr, const int* rows,
                   double out[4])
{
  quad* srow = (quad*)xmalloc(sizeof(quad) * (size_t)nr);
  quad* orow = (quad*)xmalloc(sizeof(quad) * (size_t)nr);
#pragma omp parallel for schedule(dynamic)
  for (int r = 0; r < nr; r++) {
    int i = rows[r];
    orc_qc* v = NEWQ(n);
    /* v = q_i^H A */
    for (int j = 0; j < n; j++) {
      quad sr = 0, si = 0;
      for (int k = 0; k < n; k++) {
        orc_qc q = Q[k + (long)i * n], a = A[k + (long)j * n];
        sr += q.re * a.re + q.im * a.im;
        si += q.re * a.im - q.im * a.re;
      }
      v[j] = qc_mk(sr, si);
    }
    quad ss = 0, oo = 0;
    for (int j = 0; j < n; j++) {
      /* row i, column j of Q^H A Q and of Q^H Q */
      quad tr = 0, ti = 0, gr = 0, gi = 0;
      for (int k = 0; k < n; k++) {
        orc_qc q = Q[k + (long)j * n], qi = Q[k + (long)i * n];
        tr += v[k].re * q.re - v[k].im * q.im;
        ti += v[k].re * q.im + v[k].im * q.re;
        gr += qi.re * q.re + qi.im * q.im;
        gi += qi.re * q.im - qi.im * q.re;
      }
      if (j < i) ss += tr * tr + ti * ti;
      if (j == i) gr -= 1;
      oo += gr * gr + gi * gi;
    }
    srow[r] = ss;
    orow[r] = oo;
    free(v);
  }
  long nn = (long)n * n;
  quad normA = sqrtq(fro2(A, nn));
  quad ssum = 0, smax = 0, osum = 0;
  for (int r = 0; r < nr; r++) {
    ssum += srow[r];
    osum += orow[r];
    if (srow[r] > smax) smax = srow[r];
  }
  quad scale = (quad)n / (quad)nr;
  out[0] = (double)(sqrtq(scale * ssum) / normA);
  out[1] = (double)(sqrtq(smax) / normA);
  out[2] = (double)sqrtq(scale * osum);
  out[3] = (double)normA;
  free(srow);
  free(orow);
}

/* ------------------------------------------------------------ lp Schur (start) */
int orc_schur_qr(int lp, int n, const orc_qc* A, orc_qc* Z, orc_qc* S)
{
  long nn = (long)n * n;
  void* h = lp_alloc(lp, nn);
  void* z = lp_alloc(lp, nn);
  lp_from_q(lp, nn, A, h);
  int rc;
  if (lp == ORC_LP_FLOAT) rc = schur_qr_f(n, (lc_f*)h, (lc_f*)z);
  else if (lp == ORC_LP_DOUBLE) rc = schur_qr_d(n, (lc_d*)h, (lc_d*)z);
  else rc = schur_qr_q(n, (lc_q*)h, (lc_q*)z);
  lp_to_q(lp, nn, z, Z);
  lp_to_q(lp, nn, h, S);
  free(h);
  free(z);
  return rc;
}

/* ------------------------------------------------------- reordering of the start */
void orc_reorder(int n, const orc_qc* A, const orc_qc* Qh, double theta, orc_qc* Qout, int* perm)
{
  long nn = (long)n * n;
  orc_qc* P = NEWQ(nn);
  orc_qc* T = NEWQ(nn);
  orc_gemm(0, n, n, n, A, Qh, P); /* P = A Qh */
  orc_gemm(1, n, n, n, Qh, P, T); /* T = Qh^H A Qh, then its upper triangle */
  for (int j = 0; j < n; j++)
    for (int i = j + 1; i < n; i++) T[i + (long)j * n] = qc_mk(0, 0);
  memcpy(Qout, Qh, sizeof(orc_qc) * nn);
  double* key = (double*)xmalloc(sizeof(double) * n);
  const double c = cos(theta), s = sin(theta);
  for (int i = 0; i < n; i++) {
    key[i] = (double)T[i + (long)i * n].re * c + (double)T[i + (long)i * n].im * s;
    perm[i] = i;
  }
  for (int p = 0; p < n; p++) {
    for (int i = p & 1; i + 1 < n; i += 2) {
      if (!(key[i] > key[i + 1])) continue;
      const orc_qc a = T[i + (long)i * n], b = T[i + (long)(i + 1) * n], d = T[(i + 1) + (long)(i + 1) * n];
      const quad xr = d.re - a.re, xi = d.im - a.im;
      const quad r = sqrtq(b.re * b.re + b.im * b.im + xr * xr + xi * xi);
      const orc_qc g1 = qc_mk(b.re / r, b.im / r), g2 = qc_mk(xr / r, xi / r);
      /* T <- G^H T G on rows / columns i, i+1 with G = [[g1, -conj(g2)], [g2, conj(g1)]];
         Q <- Q G */
      for (int j = 0; j < n; j++) {
        const orc_qc u = T[i + (long)j * n], v = T[(i + 1) + (long)j * n];
        /* row i: conj(g1) u + conj(g2) v; row i+1: -g2 u + g1 v */
        T[i + (long)j * n] = qc_mk(g1.re * u.re + g1.im * u.im + g2.re * v.re + g2.im * v.im,
                                   g1.re * u.im - g1.im * u.re + g2.re * v.im - g2.im * v.re);
        T[(i + 1) + (long)j * n] = qc_mk(-(g2.re * u.re - g2.im * u.im) + g1.re * v.re - g1.im * v.im,
                                         -(g2.re * u.im + g2.im * u.re) + g1.re * v.im + g1.im * v.re);
      }
      for (int m = 0; m < 2; m++) {
        orc_qc* X = m ? Qout : T;
        for (int r2 = 0; r2 < n; r2++) {
          const orc_qc u = X[r2 + (long)i * n], v = X[r2 + (long)(i + 1) * n];
          /* column i: g1 u + g2 v; column i+1: -conj(g2) u + conj(g1) v */
          X[r2 + (long)i * n] = qc_mk(g1.re * u.re - g1.im * u.im + g2.re * v.re - g2.im * v.im,
                                      g1.re * u.im + g1.im * u.re + g2.re * v.im + g2.im * v.re);
          X[r2 + (long)(i + 1) * n] = qc_mk(-(g2.re * u.re + g2.im * u.im) + g1.re * v.re + g1.im * v.im,
                                            -(g2.re * u.im - g2.im * u.re) + g1.re * v.im - g1.im * v.re);
        }
      }
      T[(i + 1) + (long)i * n] = qc_mk(0, 0);
      const double tk = key[i];
      key[i] = key[i + 1];
      key[i + 1] = tk;
      const int tp = perm[i];
      perm[i] = perm[i + 1];
      perm[i + 1] = tp;
    }
  }
  free(key);
  free(T);
  free(P);
}

/* ------------------------------------------------------- real Schur variant */
/* Block starts from the 2 x 2 markers: blk[i] = 1 when rows and columns i, i + 1
 * form one diagonal block. Returns the block count, or -1 for an invalid marker
 * (a block past the end, or overlapping blocks). */
static int real_blocks(int n, const int* blk, int* bs)
{
  int nb = 0;
  for (int i = 0; i < n;) {
    bs[nb++] = i;
    if (blk && blk[i]) {
      if (i + 1 >= n || blk[i + 1]) return -1;
      i += 2;
    } else {
      i += 1;
    }
  }
  bs[nb] = n;
  return nb;
}

/* whether (i, j), i > j, lies in the block strictly lower part */
static int below_blocks(int i, int j, const int* blk) { return i > j && !(i == j + 1 && blk && blk[j]); }

int orc_trisolve_real(int lp, int n, const int* blk, const orc_qc* T, const orc_qc* E, orc_qc* L)
{
  long nn = (long)n * n;
  int* bs = (int*)xmalloc(sizeof(int) * (size_t)(n + 1));
  int nb = real_blocks(n, blk, bs);
  if (nb < 0) {
    free(bs);
    return ORC_BREAKDOWN;
  }
  int rc;
  if (lp == ORC_LP_FLOAT) {
    float *t = (float*)xmalloc(sizeof(float) * nn), *e = (float*)xmalloc(sizeof(float) * nn),
          *l = (float*)xmalloc(sizeof(float) * nn);
    for (long z = 0; z < nn; z++) {
      t[z] = (float)T[z].re;
      e[z] = (float)E[z].re;
    }
    rc = trisolve_real_f(n, nb, bs, t, e, l);
    for (long z = 0; z < nn; z++) L[z] = qc_mk((quad)l[z], 0);
    free(t);
    free(e);
    free(l);
  } else if (lp == ORC_LP_DOUBLE) {
    double *t = (double*)xmalloc(sizeof(double) * nn), *e = (double*)xmalloc(sizeof(double) * nn),
           *l = (double*)xmalloc(sizeof(double) * nn);
    for (long z = 0; z < nn; z++) {
      t[z] = (double)T[z].re;
      e[z] = (double)E[z].re;
    }
    rc = trisolve_real_d(n, nb, bs, t, e, l);
    for (long z = 0; z < nn; z++) L[z] = qc_mk((quad)l[z], 0);
    free(t);
    free(e);
    free(l);
  } else {
    quad *t = (quad*)xmalloc(sizeof(quad) * nn), *e = (quad*)xmalloc(sizeof(quad) * nn),
         *l = (quad*)xmalloc(sizeof(quad) * nn);
    memset(t, 0, sizeof(quad) * nn);
    memset(e, 0, sizeof(quad) * nn);
    for (long z = 0; z < nn; z++) {
      t[z] = T[z].re;
      e[z] = E[z].re;
    }
    rc = trisolve_real_q(n, nb, bs, t, e, l);
    for (long z = 0; z < nn; z++) L[z] = qc_mk(l[z], 0);
    free(t);
    free(e);
    free(l);
  }
  free(bs);
  return rc;
}

int orc_refine_real(int lp, int n, const orc_qc* A, const orc_qc* Qh, const int* blk, int maxit, double tol,
                    orc_qc* Qout, orc_qc* Tout, double* hist, int* iters)
{
  long nn = (long)n * n;
  orc_qc* Q = NEWQ(nn);
  orc_qc* Qn = NEWQ(nn);
  orc_qc* AQ = NEWQ(nn);
  orc_qc* Th = NEWQ(nn);
  orc_qc* T = NEWQ(nn);
  orc_qc* E = NEWQ(nn);
  orc_qc* L = NEWQ(nn);
  orc_qc* W = NEWQ(nn);
  int status = ORC_NOT_CONVERGED, passes = 0;
  /* real data stay real through the complex products: every imaginary part is 0 */
  orc_ns(n, Qh, Q);
  quad normA = sqrtq(fro2(A, nn));
  for (int p = 0; p < maxit; p++) {
    orc_gemm(0, n, n, n, A, Q, AQ); /* That = Q^T A Q */
    orc_gemm(1, n, n, n, Q, AQ, Th);
    for (int j = 0; j < n; j++) /* E = the block strictly lower part, T = That - E */
      for (int i = 0; i < n; i++) {
        long z = i + (long)j * n;
        int low = below_blocks(i, j, blk);
        E[z] = low ? Th[z] : qc_mk(0, 0);
        T[z] = low ? qc_mk(0, 0) : Th[z];
      }
    quad eps = sqrtq(fro2(E, nn)) / normA;
    hist[p] = (double)eps;
    passes = p + 1;
    memcpy(Tout, T, sizeof(orc_qc) * (size_t)nn);
    if (!quad_finite(eps)) {
      status = ORC_BREAKDOWN;
      break;
    }
    if (eps <= (quad)tol) {
      status = ORC_OK;
      break;
    }
    if (p >= 2 && hist[p] > hist[p - 1] && hist[p - 1] > hist[p - 2]) {
      status = ORC_DIVERGED;
      break;
    }
    if (p == maxit - 1) break;
    if (orc_trisolve_real(lp, n, blk, T, E, L) != ORC_OK) {
      status = ORC_BREAKDOWN;
      break;
    }
    for (int j = 0; j < n; j++) /* W = L - L^T */
      for (int i = 0; i < n; i++) W[i + (long)j * n] = qc_mk(L[i + (long)j * n].re - L[j + (long)i * n].re, 0);
    orc_ns_merged(lp, n, Q, W, 0, Qn);
    orc_qc* tmp = Q;
    Q = Qn;
    Qn = tmp;
  }
  memcpy(Qout, Q, sizeof(orc_qc) * (size_t)nn);
  *iters = passes;
  free(Q);
  free(Qn);
  free(AQ);
  free(Th);
  free(T);
  free(E);
  free(L);
  free(W);
  return status;
}

void orc_eval_real(int n, const orc_qc* A, const orc_qc* Q, const orc_qc* T, const int* blk, double out[4])
{
  long nn = (long)n * n;
  orc_qc* AQ = NEWQ(nn);
  orc_qc* Th = NEWQ(nn);
  orc_qc* G = NEWQ(nn);
  orc_gemm(0, n, n, n, A, Q, AQ);
  orc_gemm(1, n, n, n, Q, AQ, Th);
  orc_gemm(1, n, n, n, Q, Q, G);
  quad s = 0, o = 0, t = 0;
  for (int j = 0; j < n; j++)
    for (int i = 0; i < n; i++) {
      long z = i + (long)j * n;
      int low = below_blocks(i, j, blk);
      if (low) s += qc_abs2(Th[z]);
      orc_qc g = G[z];
      if (i == j) g.re -= 1;
      o += qc_abs2(g);
      if (T) {
        orc_qc d = T[z];
        if (!low) {
          d.re -= Th[z].re;
          d.im -= Th[z].im;
        }
        t += qc_abs2(d);
      }
    }
  quad normA = sqrtq(fro2(A, nn));
  out[0] = (double)(sqrtq(s) / normA);
  out[1] = (double)sqrtq(o);
  out[2] = (double)sqrtq(t);
  out[3] = (double)normA;
  free(AQ);
  free(Th);
  free(G);
}
