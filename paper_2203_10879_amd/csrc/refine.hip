// Host driver and C interface of the Schur refinement (Algorithm 4 of
// Bujanovic, Kressner, Schroder, arXiv 2203.10879, from its second step: the
// start Q-hat is an input).
//
// One call runs, on the caller's stream:
//   Newton-Schulz start      Y0 = Qh^H Qh - I, Q = Qh + Qh (-Y0/2)         (eq. (alg:eq:NS))
//   per pass                 P = A Q, That = Q^H P (split into T, E; eps)   (2 hp products)
//                            stop if eps <= tol
//                            L from stril(T L - L T) = -E in FP32           (eq. (7))
//                            Y = Q^H Q - I, W = L - L^H, lp products        (1 hp product)
//                            Q <- Q + Q Delta, Delta = Sigma/2 - I          (1 hp product)
// The update is the merged Newton-Schulz formula (eq. (alg:eq:NSmerged)) without
// the W^2 Y and W^2 Y W terms, written as a correction Q + Q Delta so that its
// rounding error is relative to the small Delta rather than to Q.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/schur_refine.h"
#include "kernels.hpp"
#include "real.hpp"

using namespace sr;

namespace {

constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

int partial_slots(int n) {
  int a = gemm_tiles(n, n), b = form_w_parts(n);
  int m = a > b ? a : b;
  return m > 1024 ? m : 1024;
}

// Ozaki mode: slice counts. P = A Q and the Gram matrix of the start take
// kOzSlices 8-bit digits per operand (about 55 bits below the row maxima) with
// pairs up to s + t = kOzSlices + 1; the products Q Delta take between kOzMinUpd
// and kOzMaxUpd, chosen from ||Delta||.
constexpr int kOzSlices = 7, kOzMinUpd = 2, kOzMaxUpd = 7;
// CRT mode (Ozaki scheme II): bits of the scaled integers of every operand of the
// main products (2^-55 of the row maxima, as 7 digits), and the range for Q Delta.
constexpr int kCrtBits = 55, kCrtMinUpd = 12;
constexpr int kLpMaxDigits = 7;  // the all-pairs kernel's digit limit

struct Work {
  zc *Qa, *QH, *P, *Y;
  cc *Tlp, *Elp, *Llp, *W, *W2, *W3, *YW, *Ylp;
  double* partials;
  double* scal;
  unsigned* status;
  void* tri;
  // Ozaki mode only (NULL otherwise): row slices of A, column slices of Q, row
  // slices of Q and column slices of Delta, with their exponents.
  int8_t *sA, *sQc, *sQr, *sD;
  int *eA, *eQc, *eQr, *eD;
  void* oz_scratch;  // FP64 partial sums of the large-tile product, or the CRT
                     // product's residues between moduli (may be NULL)
  // lp products on INT8 digits (sr_opts.lp_digits > 0 and the all-pairs kernel at
  // this size; lp_s = 0 otherwise): row and column slices of W, row slices of the
  // left operand of the second product
  int8_t *sWr, *sWc, *sXr;
  int *eWr, *eWc, *eXr;
  int lp_s;
  bool oz_all;  // Ozaki mode: That and Y from slices too
  bool crt;     // CRT mode: the slices are residues, oz_s and the update counts bits
  int oz_s;
  size_t bytes;
};

// The split and product steps of the two split forms: digit slices (prec = digits
// per operand, pairs up to prec + 1) or residues (prec = bits of the scaled
// integers).
hipError_t w_split_cols(const Work& w, const zc* X, int n, int prec, int8_t* out, int* e, hipStream_t st) {
  return w.crt ? crt_split_cols(X, n, n, n, prec, out, e, st) : oz_split_cols(X, nullptr, n, n, n, prec, out, e, st);
}
hipError_t w_split_rows(const Work& w, const zc* X, int n, int prec, int8_t* out, int* e, hipStream_t st) {
  return w.crt ? crt_split_rows(X, n, n, n, prec, out, e, st) : oz_split_rows(X, nullptr, n, n, n, prec, out, e, st);
}
hipError_t w_prod(const Work& w, int epi, const int8_t* A, const int* ea, const int8_t* B, const int* eb, int prec,
                  int conjA, const GemmArgs& g, hipStream_t st) {
  return w.crt ? crt_gemm(epi, A, ea, B, eb, conjA, prec, g, w.oz_scratch, st)
               : oz_gemm(epi, A, ea, prec, B, eb, prec, conjA, prec + 1, g, w.oz_scratch, st);
}
int w_tiles(const Work& w, int n, bool herm, int prec) {
  return w.crt ? crt_gemm_tiles(n, n, herm) : oz_gemm_tiles(n, n, n, false, herm, prec, prec, prec + 1);
}

int oz_main_slices(const sr_opts* o) {
  return (o && o->slices > 0) ? o->slices : kOzSlices;
}

int crt_main_bits(const sr_opts* o) { return (o && o->slices > 0) ? o->slices : kCrtBits; }

// Leaf size of the recursive solve in 16-row tiles (default 64 rows).
int rec_leaf_tiles(const sr_opts& o) {
  const int rows = o.rec_leaf > 0 ? o.rec_leaf : 64;
  return (rows + 15) / 16;
}

Work carve(void* base, int n, const sr_opts* o = nullptr) {
  Work w;
  uintptr_t p = (uintptr_t)base;
  const size_t z = align256((size_t)n * n * sizeof(zc));
  const size_t c = align256((size_t)n * n * sizeof(cc));
  auto take = [&](size_t b) {
    void* r = (void*)p;
    p += b;
    return r;
  };
  w.Qa = (zc*)take(z);
  w.QH = (zc*)take(z);
  w.P = (zc*)take(z);
  w.Y = (zc*)take(z);
  w.Tlp = (cc*)take(c);
  w.Elp = (cc*)take(c);
  w.Llp = (cc*)take(c);
  w.W = (cc*)take(c);
  w.W2 = (cc*)take(c);
  w.W3 = (cc*)take(c);
  w.YW = (cc*)take(c);
  w.Ylp = (cc*)take(c);
  w.partials = (double*)take(align256((size_t)partial_slots(n) * sizeof(double)));
  w.scal = (double*)take(256);
  w.status = (unsigned*)take(256);
  {
    size_t tb = trisolve_ws_bytes(n);
    if (o && o->solver == SR_SOLVER_RECURSIVE) tb = std::max(tb, trisolve_rec_ws_bytes(n, rec_leaf_tiles(*o)));
    w.tri = take(align256(tb));
  }
  w.sA = w.sQc = w.sQr = w.sD = nullptr;
  w.eA = w.eQc = w.eQr = w.eD = nullptr;
  w.oz_scratch = nullptr;
  w.oz_s = 0;
  w.oz_all = false;
  w.crt = false;
  w.sWr = w.sWc = w.sXr = nullptr;
  w.eWr = w.eWc = w.eXr = nullptr;
  w.lp_s = 0;
  if (o && o->lp_digits > 0 && o->lp_digits <= kLpMaxDigits && o->gemm != SR_GEMM_FP64 &&
      oz_allpairs_ok(n, n, n, o->lp_digits)) {
    w.lp_s = o->lp_digits;
    const size_t sb = align256(oz_slice_bytes(n, n, w.lp_s));
    const size_t eb = align256((size_t)n * sizeof(int));
    w.sWr = (int8_t*)take(sb);
    w.sWc = (int8_t*)take(sb);
    w.sXr = (int8_t*)take(sb);
    w.eWr = (int*)take(eb);
    w.eWc = (int*)take(eb);
    w.eXr = (int*)take(eb);
  }
  if (o && o->gemm == SR_GEMM_OZAKI_CRT) {
    // residues of A's rows, Q's columns, Q's rows and Delta's (and P's) columns
    // for the main bit count (the update never takes more)
    w.crt = w.oz_all = true;
    w.oz_s = crt_main_bits(o);
    const int N = crt_moduli(n, w.oz_s);
    const size_t rb = align256(crt_residue_bytes(n, n, N));
    w.sA = (int8_t*)take(rb);
    w.sQc = (int8_t*)take(rb);
    w.sQr = (int8_t*)take(rb);
    w.sD = (int8_t*)take(rb);
    w.eA = (int*)take(align256((size_t)n * sizeof(int)));
    w.eQc = (int*)take(align256((size_t)n * sizeof(int)));
    w.eQr = (int*)take(align256((size_t)n * sizeof(int)));
    w.eD = (int*)take(align256((size_t)n * sizeof(int)));
    // (also the all-pairs scratch of the lp products on digits)
    w.oz_scratch = take(align256(std::max(crt_scratch_bytes(n, n, N), w.lp_s ? oz_gemm_scratch_bytes(n, n) : 0)));
  } else if (o && (o->gemm == SR_GEMM_OZAKI_I8 || o->gemm == SR_GEMM_OZAKI_I8_ALL)) {
    w.oz_all = o->gemm == SR_GEMM_OZAKI_I8_ALL;
    const int S = oz_main_slices(o);
    const int Su = o->update_slices > 0 ? o->update_slices : kOzMaxUpd;
    w.oz_s = S;
    w.sA = (int8_t*)take(align256(oz_slice_bytes(n, n, S)));
    w.sQc = (int8_t*)take(align256(oz_slice_bytes(n, n, S)));
    w.sQr = (int8_t*)take(align256(oz_slice_bytes(n, n, Su)));
    // the column slices of Delta, and before them those of P (for That)
    w.sD = (int8_t*)take(align256(oz_slice_bytes(n, n, Su > S ? Su : S)));
    w.eA = (int*)take(align256((size_t)n * sizeof(int)));
    w.eQc = (int*)take(align256((size_t)n * sizeof(int)));
    w.eQr = (int*)take(align256((size_t)n * sizeof(int)));
    w.eD = (int*)take(align256((size_t)n * sizeof(int)));
    const size_t scr = oz_gemm_scratch_bytes(n, n);
    if (scr) w.oz_scratch = take(align256(scr));
  }
  w.bytes = (size_t)(p - (uintptr_t)base);
  return w;
}

// Library-owned workspace, used when the caller passes none. One buffer per
// device, grown on demand; calls without a workspace on one device serialise.
struct Cache {
  std::mutex mu;
  std::vector<void*> ptr;
  std::vector<size_t> size;
};
Cache& cache() {
  static Cache c;
  return c;
}

// Pinned host buffer for reading back residuals and norms.
double* host_scratch() {
  static thread_local double* h = nullptr;
  if (!h) {
    if (hipHostMalloc((void**)&h, 256, hipHostMallocDefault) != hipSuccess) h = nullptr;
  }
  return h;
}

int read_back(hipStream_t st, const Work& w, int count, double* out, unsigned* status) {
  double* h = host_scratch();
  if (!h) return SR_ENOMEM;
  if (hipMemcpyAsync(h, w.scal, sizeof(double) * count, hipMemcpyDeviceToHost, st) != hipSuccess)
    return SR_EHIP;
  if (hipMemcpyAsync(h + 16, w.status, sizeof(unsigned), hipMemcpyDeviceToHost, st) != hipSuccess)
    return SR_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SR_EHIP;
  memcpy(out, h, sizeof(double) * count);
  unsigned s;
  memcpy(&s, h + 16, sizeof(unsigned));
  *status = s;
  return SR_OK;
}

// Side stream for the Hermitian product Y beside the solve: one per (device,
// caller stream), created on first use (non-blocking, default priority) and kept
// for the process, so that calls on different streams never share one. After
// kMaxSideStreams distinct pairs no more are made and Y runs on the caller's
// stream (NULL return).
constexpr int kSideYMaxN = 2048, kSideYMaxNdd = 2048;
constexpr size_t kMaxSideStreams = 64;
hipStream_t side_stream(hipStream_t caller) {
  struct Entry {
    int dev;
    hipStream_t caller, side;
  };
  static std::mutex mu;
  static std::vector<Entry> tab;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  for (const Entry& e : tab)
    if (e.dev == dev && e.caller == caller) return e.side;
  if (tab.size() >= kMaxSideStreams) return nullptr;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
  tab.push_back({dev, caller, s});
  return s;
}

// Events of one refinement call, released on every return path.
struct CallEvents {
  hipEvent_t t0 = nullptr, t1 = nullptr, fork = nullptr, join = nullptr;
  ~CallEvents() {
    for (hipEvent_t e : {t0, t1, fork, join})
      if (e) hipEventDestroy(e);
  }
};

GemmArgs gargs(int m, int n, int k, const void* A, long lda, const void* B, long ldb, void* C,
               long ldc) {
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.m = m;
  g.n = n;
  g.k = k;
  g.A = A;
  g.lda = lda;
  g.B = B;
  g.ldb = ldb;
  g.C = C;
  g.ldc = ldc;
  return g;
}

#define CK(expr)                                  \
  do {                                            \
    hipError_t _e = (expr);                       \
    if (_e != hipSuccess) return SR_EHIP;         \
  } while (0)

// Optional HIP-event timing of launch groups on the call's stream:
// category 0 = hp products, 1 = triangular solves, 2 = the full split products
// with the main digit count (product kernel alone, inside a category-0 group).
struct Timer {
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> ev[3];
  int count[3] = {0, 0, 0};
  int herm = 0;                  // timed hp products that were Hermitian (Y)
  std::vector<char> herm_pair;   // per event pair of channel 0
  void mark(int c) {
    hipEvent_t e;
    if (hipEventCreate(&e) == hipSuccess) {
      hipEventRecord(e, st);
      ev[c].push_back(e);
    }
  }
  // after the stream has been synchronised; only_herm: 0 all pairs, 1 the
  // Hermitian ones
  float total(int c, int only_herm = 0) const {
    float s = 0;
    for (size_t i = 0; i + 1 < ev[c].size(); i += 2) {
      if (only_herm && !(c == 0 && i / 2 < herm_pair.size() && herm_pair[i / 2])) continue;
      float ms = 0;
      hipEventElapsedTime(&ms, ev[c][i], ev[c][i + 1]);
      s += ms;
    }
    return s;
  }
  ~Timer() {
    for (auto& v : ev)
      for (hipEvent_t e : v) hipEventDestroy(e);
  }
};
#define TIC(tm, c) \
  if (tm) (tm)->mark(c)
#define TOC(tm, c)                                                   \
  if (tm) {                                                          \
    (tm)->mark(c);                                                   \
    (tm)->count[c]++;                                                \
    if ((c) == 0) (tm)->herm_pair.resize((tm)->ev[0].size() / 2, 0); \
  }
#define TOC_HERM(tm)                                             \
  if (tm) {                                                      \
    (tm)->mark(0);                                               \
    (tm)->count[0]++;                                            \
    (tm)->herm++;                                                \
    (tm)->herm_pair.resize((tm)->ev[0].size() / 2, 0);           \
    if (!(tm)->herm_pair.empty()) (tm)->herm_pair.back() = 1;    \
  }

// Newton-Schulz start into Qout: Y0 = Qh^H Qh - I, Qout = Qh + Qh (-Y0/2);
// QHout (may be NULL) receives Qout^H.
// Ozaki mode: Qout = Q + Q D (QHout = Qout^H if given) from Su slices per operand.
int oz_update(const zc* Q, const zc* D, zc* Qout, zc* QHout, int n, int Su, const Work& w,
              hipStream_t st) {
  CK(w_split_rows(w, Q, n, Su, w.sQr, w.eQr, st));
  CK(w_split_cols(w, D, n, Su, w.sD, w.eD, st));
  GemmArgs u = gargs(n, n, n, nullptr, 0, nullptr, 0, Qout, n);
  u.Cin = Q;
  u.ldcin = n;
  u.CH = QHout;
  u.ldch = n;
  CK(w_prod(w, EPI_ADD, w.sQr, w.eQr, w.sD, w.eD, Su, 0, u, st));
  return SR_OK;
}

// Digits per operand of Q Delta. With pairs kept up to s + t = Su + 1, the
// product is exact to about 2^(-8 Su) relative to sum_k |q_ik| |delta_kj|
// <= ||q_i|| ||delta_j||; Q's rows have norm ~1 and its entries ~1/sqrt(n), a
// column of Delta ~||Delta||_F / sqrt(n), so the error relative to Q's entries is
// ~2^(-8 Su) ||Delta||_F, and Su is the least count with that under 0.05 u.
int update_slices(const sr_opts& o, double norm_delta) {
  if (o.gemm == SR_GEMM_OZAKI_CRT) {
    // the same rule in bits: 2^-b ||Delta||_F under 0.05 u
    if (o.update_slices > 0) return o.update_slices;
    const int top = crt_main_bits(&o);
    if (!(norm_delta > 0)) return kCrtMinUpd;
    int b = (int)ceil(log2(norm_delta / (0.05 * kU64)));
    if (b < kCrtMinUpd) b = kCrtMinUpd;
    if (b > top) b = top;
    return b;
  }
  if (o.update_slices > 0) return o.update_slices;
  if (!(norm_delta > 0)) return kOzMinUpd;
  const double bits = log2(norm_delta / (0.05 * kU64));
  int s = (int)ceil(bits / 8.0);
  if (s < kOzMinUpd) s = kOzMinUpd;
  if (s > kOzMaxUpd) s = kOzMaxUpd;
  return s;
}

int ns_init(const zc* Qh, zc* Qout, zc* QHout, int n, int comp, const Work& w, hipStream_t st,
            Timer* tm = nullptr, const sr_opts* o = nullptr, int* su_used = nullptr) {
  if (w.oz_s) {
    // The Gram matrix Qh^H Qh from the column slices of Qh, used for both operands.
    const int S = w.oz_s;
    TIC(tm, 0);
    CK(w_split_cols(w, Qh, n, S, w.sQc, w.eQc, st));
    GemmArgs g = gargs(n, n, n, nullptr, 0, nullptr, 0, w.Y, n);
    g.partials = w.partials;
    g.herm = 1;
    CK(w_prod(w, EPI_YDEF, w.sQc, w.eQc, w.sQc, w.eQc, S, 1, g, st));
    TOC_HERM(tm);
    CK(reduce_partials(w.partials, w_tiles(w, n, true, S), w.scal + 2, st));
    double nrm[3];
    unsigned dst = 0;
    int rc = read_back(st, w, 3, nrm, &dst);
    if (rc != SR_OK) return rc;
    CK(form_delta(nullptr, w.Y, nullptr, nullptr, nullptr, w.P, n, st));
    const int Su = update_slices(*o, 0.5 * sqrt(nrm[2]));
    if (su_used) *su_used = Su;
    TIC(tm, 0);
    if ((rc = oz_update(Qh, w.P, Qout, QHout, n, Su, w, st)) != SR_OK) return rc;
    TOC(tm, 0);
    return SR_OK;
  }
  GemmArgs g = gargs(n, n, n, Qh, n, Qh, n, w.Y, n);
  g.partials = w.partials;
  g.herm = 1;
  TIC(tm, 0);
  CK(zgemm(1, EPI_YDEF, comp, g, st));
  TOC_HERM(tm);
  CK(form_delta(nullptr, w.Y, nullptr, nullptr, nullptr, w.P, n, st));
  GemmArgs u = gargs(n, n, n, Qh, n, w.P, n, Qout, n);
  u.Cin = Qh;
  u.ldcin = n;
  u.CH = QHout;
  u.ldch = n;
  TIC(tm, 0);
  CK(zgemm(0, EPI_ADD, 0, u, st));
  TOC(tm, 0);
  return SR_OK;
}

// P = A Q, That = Q^H P with the split epilogue, scal[1] = ||stril(That)||_F^2.
// With QH (= Q^H) given, That is formed as the plain product QH P.
// Ozaki mode: P from the row slices of A (split once per call) and the column
// slices of Q (kept in sQc for Y of the same pass); with oz_all also That, from
// the conjugated column slices of Q and the column slices of P.
int residual(const zc* A, const zc* Q, const zc* QH, zc* T, int n, int comp, const Work& w,
             hipStream_t st, Timer* tm = nullptr) {
  GemmArgs g = gargs(n, n, n, A, n, Q, n, w.P, n);
  GemmArgs s = gargs(n, n, n, QH ? QH : Q, n, w.P, n, T, n);
  s.Tlp = w.Tlp;
  s.Elp = w.Elp;
  s.ldlp = n;
  s.partials = w.partials;
  TIC(tm, 0);
  if (w.oz_s) {
    const int S = w.oz_s;
    CK(w_split_cols(w, Q, n, S, w.sQc, w.eQc, st));
    TIC(tm, 2);
    CK(w_prod(w, EPI_STORE, w.sA, w.eA, w.sQc, w.eQc, S, 0, g, st));
    TOC(tm, 2);
  } else {
    CK(zgemm(0, EPI_STORE, comp, g, st));
  }
  TOC(tm, 0);
  if (w.oz_all) {
    const int S = w.oz_s;
    TIC(tm, 0);
    CK(w_split_cols(w, w.P, n, S, w.sD, w.eD, st));
    TIC(tm, 2);
    CK(w_prod(w, EPI_SPLIT, w.sQc, w.eQc, w.sD, w.eD, S, 1, s, st));
    TOC(tm, 2);
    TOC(tm, 0);
    CK(reduce_partials(w.partials, w_tiles(w, n, false, S), w.scal + 1, st));
    return SR_OK;
  }
  TIC(tm, 0);
  CK(zgemm(QH ? 0 : 1, EPI_SPLIT, comp, s, st));
  TOC(tm, 0);
  CK(reduce_partials(w.partials, gemm_tiles(n, n), w.scal + 1, st));
  return SR_OK;
}

// Y = Q^H Q - I (scal[2] = ||Y||^2).
// oz_all: from the column slices of Q that residual() left in sQc (the same Q).
int ydef(const zc* Q, const zc* QH, int n, int comp, const Work& w, hipStream_t st, Timer* tm) {
  GemmArgs g = gargs(n, n, n, QH ? QH : Q, n, Q, n, w.Y, n);
  g.partials = w.partials;
  g.herm = 1;
  if (w.oz_all) {
    const int S = w.oz_s;
    TIC(tm, 0);
    CK(w_prod(w, EPI_YDEF, w.sQc, w.eQc, w.sQc, w.eQc, S, 1, g, st));
    TOC_HERM(tm);
    CK(reduce_partials(w.partials, w_tiles(w, n, true, S), w.scal + 2, st));
    return SR_OK;
  }
  TIC(tm, 0);
  CK(zgemm(QH ? 0 : 1, EPI_YDEF, comp, g, st));
  TOC_HERM(tm);
  CK(reduce_partials(w.partials, gemm_tiles_herm(n), w.scal + 2, st));
  return SR_OK;
}

// Y = Q^H Q - I (scal[2] = ||Y||^2), W = L - L^H (scal[3] = ||W||^2).
int defects(const zc* Q, const zc* QH, int n, int comp, const Work& w, hipStream_t st,
            Timer* tm = nullptr) {
  GemmArgs g = gargs(n, n, n, QH ? QH : Q, n, Q, n, w.Y, n);
  g.partials = w.partials;
  g.herm = 1;
  TIC(tm, 0);
  CK(zgemm(QH ? 0 : 1, EPI_YDEF, comp, g, st));
  TOC_HERM(tm);
  CK(reduce_partials(w.partials, gemm_tiles_herm(n), w.scal + 2, st));
  CK(form_w(w.Llp, w.W, n, w.partials, st));
  CK(reduce_partials(w.partials, form_w_parts(n), w.scal + 3, st));
  return SR_OK;
}

struct Gate {
  bool w2, w3, yw;
};

// lp products, Delta, and Qout = Q + Q Delta (QHout, if given, receives Qout^H).
// The lp products from INT8 digits (w.lp_s per operand, pairs s + t <= lp_s + 1):
// C = X W with X given by its row slices (complex64 out; herm as GemmArgs::herm).
int lp_digit_product(const int8_t* sX, const int* eX, cc* C, int herm, int n, const Work& w, hipStream_t st) {
  GemmArgs g = gargs(n, n, n, nullptr, 0, nullptr, 0, C, n);
  g.c64 = 1;
  g.herm = herm;
  CK(oz_gemm(EPI_STORE, sX, eX, w.lp_s, w.sWc, w.eWc, w.lp_s, 0, w.lp_s + 1, g, w.oz_scratch, st));
  return SR_OK;
}

int lp_products_digits(Gate gt, bool both, int n, const Work& w, hipStream_t st, int* np) {
  const int S = w.lp_s;
  CK(oz_split_cols_c64(w.W, n, n, n, S, w.sWc, w.eWc, st));
  if (gt.w2 || gt.w3) {
    CK(oz_split_rows_c64(w.W, n, n, n, S, w.sWr, w.eWr, st));
    const int rc = lp_digit_product(w.sWr, w.eWr, w.W2, 1, n, w, st);  // W^2: Hermitian
    if (rc != SR_OK) return rc;
    (*np)++;
  }
  const cc* X = nullptr;
  cc* out = nullptr;
  int herm = 0;
  if (both) {
    CK(w2_minus_y(w.W2, w.Y, w.Ylp, (long)n * n, st));
    X = w.Ylp;
    out = w.W3;
  } else if (gt.w3) {
    X = w.W2;
    out = w.W3;
    herm = -1;  // W^3: skew-Hermitian
  } else if (gt.yw) {
    CK(to_c64(w.Y, w.Ylp, (long)n * n, st));
    X = w.Ylp;
    out = w.YW;
  }
  if (X) {
    CK(oz_split_rows_c64(X, n, n, n, S, w.sXr, w.eXr, st));
    const int rc = lp_digit_product(w.sXr, w.eXr, out, herm, n, w, st);
    if (rc != SR_OK) return rc;
    (*np)++;
  }
  return SR_OK;
}

// The lp products in FP32 on MFMA.
int lp_products_fp32(Gate gt, bool both, int n, const Work& w, hipStream_t st, int* np) {
  if (gt.w2 || gt.w3) {
    GemmArgs a2 = gargs(n, n, n, w.W, n, w.W, n, w.W2, n);
    a2.herm = 1;  // W is skew-Hermitian: W^2 is Hermitian
    CK(cgemm(a2, st));
    (*np)++;
  }
  if (both) {
    CK(w2_minus_y(w.W2, w.Y, w.Ylp, (long)n * n, st));
    CK(cgemm(gargs(n, n, n, w.Ylp, n, w.W, n, w.W3, n), st));
    (*np)++;
  } else if (gt.w3) {
    GemmArgs a3 = gargs(n, n, n, w.W2, n, w.W, n, w.W3, n);
    a3.herm = -1;  // and W^3 skew-Hermitian
    CK(cgemm(a3, st));
    (*np)++;
  } else if (gt.yw) {
    CK(to_c64(w.Y, w.Ylp, (long)n * n, st));
    CK(cgemm(gargs(n, n, n, w.Ylp, n, w.W, n, w.YW, n), st));
    (*np)++;
  }
  return SR_OK;
}

int apply_update(const zc* Q, zc* Qout, zc* QHout, int n, Gate gt, const Work& w, hipStream_t st,
                 int* nprod, Timer* tm = nullptr, int Su = 0, bool no_y = false) {
  int np = 0;
  // With both W^3 and YW, one product gives their difference: (W^2 - Y) W (into W3).
  const bool both = gt.w3 && gt.yw;
  const int lrc = w.lp_s ? lp_products_digits(gt, both, n, w, st, &np) : lp_products_fp32(gt, both, n, w, st, &np);
  if (lrc != SR_OK) return lrc;
  CK(form_delta(w.Llp, no_y ? nullptr : w.Y, gt.w2 ? w.W2 : nullptr, gt.w3 ? w.W3 : nullptr,
                gt.yw && !both ? w.YW : nullptr, w.P, n, st));
  TIC(tm, 0);
  if (w.oz_s) {
    const int rc = oz_update(Q, w.P, Qout, QHout, n, Su, w, st);
    if (rc != SR_OK) return rc;
  } else {
    GemmArgs u = gargs(n, n, n, Q, n, w.P, n, Qout, n);
    u.Cin = Q;
    u.ldcin = n;
    u.CH = QHout;
    u.ldch = n;
    CK(zgemm(0, EPI_ADD, 0, u, st));
  }
  TOC(tm, 0);
  if (nprod) *nprod += np;
  return SR_OK;
}

Gate gate_terms(bool gate, double nw, double ny) {
  const double thr = 0.1 * kU64;
  Gate g;
  if (!gate) {
    g.w2 = g.w3 = g.yw = true;
    return g;
  }
  g.w2 = nw * nw > thr;
  g.w3 = nw * nw * nw > thr;
  g.yw = ny * nw > thr;
  return g;
}

int get_ws(const sr_opts& o, size_t need, void** out) {
  if (o.workspace) {
    if (o.workspace_bytes < need) return SR_ENOMEM;
    *out = o.workspace;
    return SR_OK;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SR_EHIP;
  Cache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  if ((int)c.ptr.size() <= dev) {
    c.ptr.resize(dev + 1, nullptr);
    c.size.resize(dev + 1, 0);
  }
  if (c.size[dev] < need) {
    if (c.ptr[dev]) {
      if (hipDeviceSynchronize() != hipSuccess) return SR_EHIP;
      hipFree(c.ptr[dev]);
      c.ptr[dev] = nullptr;
      c.size[dev] = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) return SR_ENOMEM;
    c.ptr[dev] = p;
    c.size[dev] = need;
  }
  *out = c.ptr[dev];
  return SR_OK;
}

// Outcome of a pass from its residual eps (-1: go on). eps1, eps2: the residuals
// of the two passes before (-1 if none); nw_last: ||W||_F of the last update.
// With opts.strict_stop, eps <= tol also needs an update to have been made and its
// correction to have been negligible to second order (||W||^2 <= u, so that the
// next one would fall below roundoff): on matrices whose entries span many orders
// of magnitude the normwise residual reaches tol (even at the start) while the
// small parts of Q still move. While eps <= tol waits for that, the divergence
// and stagnation tests are not applied.
int stop_test(const sr_opts& o, double eps, double tol, double eps1, double eps2, int updates,
              double nw_last, double u, int n) {
  if (eps <= tol) {
    if (!o.strict_stop || (updates > 0 && nw_last * nw_last <= u)) return SR_OK;
    return -1;
  }
  if (eps2 >= 0 && eps > eps1 && eps1 > eps2) return SR_DIVERGED;
  if (eps1 >= 0 && eps > 0.5 * eps1 && eps < 100.0 * u * sqrt((double)n)) return SR_STAGNATED;
  return -1;
}

void info_init(sr_info* info) {
  if (info) memset(info, 0, sizeof(*info));
}

}  // namespace

extern "C" {

void sr_default_opts(sr_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->gemm = SR_GEMM_FP64;
  o->compensated = 1;
  o->gate_lp_terms = 1;
}

size_t sr_workspace_bytes(int n, const sr_opts* opts) {
  if (n < 1) return 0;
  return carve(nullptr, n, opts).bytes + 256;
}

const char* sr_status_string(int s) {
  switch (s) {
    case SR_OK: return "converged";
    case SR_NOT_CONVERGED: return "not converged within the pass limit";
    case SR_STAGNATED: return "residual stagnated at the accumulation floor";
    case SR_BREAKDOWN: return "breakdown (non-finite value or equal diagonal entries)";
    case SR_DIVERGED: return "diverged (residual rose on two consecutive passes)";
    case SR_EINVAL: return "invalid argument";
    case SR_EHIP: return "HIP runtime error";
    case SR_ENOMEM: return "insufficient workspace or memory";
    case SR_ENOSYS: return "option not supported";
    default: return "unknown status";
  }
}

static int refine_fp64(const void* A_, void* Q_, void* T_, int n, int iters, double tol,
                       const sr_opts* opts_in, sr_info* info) {
  info_init(info);
  if (!A_ || !Q_ || !T_ || n < 1 || iters < 1 || !(tol > 0)) {
    if (info) info->status = SR_EINVAL;
    return SR_EINVAL;
  }
  sr_opts o;
  if (opts_in) o = *opts_in;
  else sr_default_opts(&o);
  const bool crt = o.gemm == SR_GEMM_OZAKI_CRT;
  const bool ozaki = o.gemm == SR_GEMM_OZAKI_I8 || o.gemm == SR_GEMM_OZAKI_I8_ALL;
  if (crt && (o.slices < 0 || o.slices > kCrtBits || o.update_slices < 0 || o.update_slices > crt_main_bits(&o) ||
              !crt_plan_ok(n, crt_main_bits(&o)))) {
    if (info) info->status = SR_EINVAL;
    return SR_EINVAL;
  }
  if (o.gemm != SR_GEMM_FP64 && !ozaki && !crt) {
    if (info) info->status = o.gemm == SR_GEMM_OZAKI_BF16 ? SR_ENOSYS : SR_EINVAL;
    return o.gemm == SR_GEMM_OZAKI_BF16 ? SR_ENOSYS : SR_EINVAL;
  }
  if ((o.solver != SR_SOLVER_WAVEFRONT && o.solver != SR_SOLVER_RECURSIVE) || o.rec_leaf < 0) {
    if (info) info->status = SR_EINVAL;
    return SR_EINVAL;
  }
  if (o.lp_digits < 0 || o.lp_digits > kLpMaxDigits || (o.lp_digits && !ozaki && !crt)) {
    if (info) info->status = SR_EINVAL;
    return SR_EINVAL;
  }
  if (ozaki &&
      (o.slices < 0 || o.slices > 16 || o.update_slices < 0 || o.update_slices > kOzMaxUpd ||
       !oz_gemm_exact(n, n, n, oz_main_slices(&o), oz_main_slices(&o)))) {
    if (info) info->status = SR_EINVAL;
    return SR_EINVAL;
  }
  hipStream_t st = (hipStream_t)o.stream;
  const zc* A = (const zc*)A_;
  zc* Q = (zc*)Q_;
  zc* T = (zc*)T_;

  if (n == 1) {
    zc a, q;
    CK(hipMemcpyAsync(&a, A, sizeof(zc), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(&q, Q, sizeof(zc), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    const double m = hypot(q.re, q.im);
    if (!(m > 0) || !isfinite(a.re) || !isfinite(a.im)) {
      if (info) info->status = SR_BREAKDOWN;
      return SR_BREAKDOWN;
    }
    zc qn = mk<double>(q.re / m, q.im / m);
    CK(hipMemcpyAsync(T, &a, sizeof(zc), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(Q, &qn, sizeof(zc), hipMemcpyHostToDevice, st));
    CK(hipStreamSynchronize(st));
    if (info) {
      info->status = SR_OK;
      info->iters = 1;
    }
    return SR_OK;
  }

  void* base = nullptr;
  int rc = get_ws(o, sr_workspace_bytes(n, &o), &base);
  if (rc != SR_OK) {
    if (info) info->status = rc;
    return rc;
  }
  const Work w = carve(base, n, &o);
  const int comp = o.compensated ? 1 : 0;

  Timer timer;
  timer.st = st;
  Timer* tm = o.timing ? &timer : nullptr;
  CallEvents ev;
  CK(hipEventCreate(&ev.t0));
  CK(hipEventCreate(&ev.t1));
  CK(hipEventRecord(ev.t0, st));
  CK(fill_zero(w.status, 256, st));
  CK(fro2_partials(A, (long)n * n, w.partials, 1024, st));
  CK(reduce_partials(w.partials, 1024, w.scal, st));

  int status = SR_NOT_CONVERGED;
  int passes = 0, updates = 0, nprod = 0, skips = 0;
  double eps = 0, eps1 = -1, eps2 = -1, orth = 0, nw_last = 0;
  double y_pred = INFINITY;  // skip_orth: predicted ||Q^H Q - I|| before the next update
  bool skipped_last = false;
  zc* cur = w.Qa;
  zc* other = Q;
  hipStream_t sst = n <= kSideYMaxN ? side_stream(st) : nullptr;
  if (sst) {
    CK(hipEventCreateWithFlags(&ev.fork, hipEventDisableTiming));
    CK(hipEventCreateWithFlags(&ev.join, hipEventDisableTiming));
  }
  if (w.oz_s) CK(w_split_rows(w, A, n, w.oz_s, w.sA, w.eA, st));
  int su = 0;
  // the explicit Q^H serves the native That and Y; with oz_all they use the column
  // slices of Q instead
  zc* const QH = w.oz_all ? nullptr : w.QH;
  if ((rc = ns_init(Q, w.Qa, QH, n, comp, w, st, tm, &o, &su)) != SR_OK) return rc;
  if (info) info->update_slices_hist[0] = su;

  for (int p = 0; p < iters; p++) {
    if ((rc = residual(A, cur, QH, T, n, comp, w, st, tm)) != SR_OK) return rc;
    double s[2];
    unsigned dst = 0;
    if ((rc = read_back(st, w, 2, s, &dst)) != SR_OK) return rc;
    eps = sqrt(s[1]) / sqrt(s[0]);
    passes = p + 1;
    if (info && p < 16) info->resid_hist[p] = eps;
    if (!isfinite(eps)) {
      status = SR_BREAKDOWN;
      break;
    }
    const int stop = stop_test(o, eps, tol, eps1, eps2, updates, nw_last, kU64, n);
    if (stop >= 0) {
      status = stop;
      break;
    }
    eps2 = eps1;
    eps1 = eps;
    if (p == iters - 1) break;

    // Y does not depend on L. Up to kSideYMaxN it runs beside the solve on a side
    // stream: the solve's early tile levels leave most CUs idle (measured: +7.5% per
    // refinement at n = 1024, +2.7% at 2048). At n = 4096 Y's blocks take the CUs the
    // solve's later levels need (the solve doubled, the pass gained 1.5%), so there
    // the two run one after the other.
    // skip_orth: Y is left out when the prediction says it would be below u_hp
    const bool try_skip = o.skip_orth && !skipped_last && y_pred <= kU64;
    const bool side = sst && n <= kSideYMaxN && !try_skip;
    if (side) {
      CK(hipEventRecord(ev.fork, st));
      CK(hipStreamWaitEvent(sst, ev.fork, 0));
      hipStream_t keep = tm ? tm->st : nullptr;
      if (tm) tm->st = sst;
      rc = ydef(cur, QH, n, comp, w, sst, tm);
      if (tm) tm->st = keep;
      if (rc != SR_OK) return rc;
      CK(hipEventRecord(ev.join, sst));
    }
    TIC(tm, 1);
    if (o.solver == SR_SOLVER_RECURSIVE)
      CK(trisolve_rec(w.Tlp, w.Elp, w.Llp, n, rec_leaf_tiles(o), o.trunc ? 1e-5f : 0.f, w.tri, w.status, st));
    else
      CK(trisolve(w.Tlp, w.Elp, w.Llp, n, o.trunc ? 1e-5f : 0.f, w.tri, w.status, st));
    TOC(tm, 1);
    if (side) CK(hipStreamWaitEvent(st, ev.join, 0));
    else if (!try_skip && (rc = ydef(cur, QH, n, comp, w, st, tm)) != SR_OK) return rc;
    CK(form_w(w.Llp, w.W, n, w.partials, st));
    CK(reduce_partials(w.partials, form_w_parts(n), w.scal + 3, st));
    double nrm[4];
    if ((rc = read_back(st, w, 4, nrm, &dst)) != SR_OK) return rc;
    if (dst & DEV_BREAKDOWN) {
      status = SR_BREAKDOWN;
      break;
    }
    double nw = sqrt(nrm[3]);
    bool skip = try_skip && nw * nw <= kU64;
    if (try_skip && !skip) {
      // the prediction held but W is not small enough: form Y after all
      if ((rc = ydef(cur, QH, n, comp, w, st, tm)) != SR_OK) return rc;
      if ((rc = read_back(st, w, 4, nrm, &dst)) != SR_OK) return rc;
    }
    const double ny = skip ? 0.0 : sqrt(nrm[2]);
    if (!skip) orth = ny;
    nw_last = nw;
    if (info && updates < 16) info->norm_w_hist[updates] = nw;
    if (!isfinite(ny) || !isfinite(nw)) {
      status = SR_BREAKDOWN;
      break;
    }
    const Gate gt = gate_terms(o.gate_lp_terms != 0, nw, ny);
    su = w.oz_s ? update_slices(o, nw + 0.5 * ny) : 0;
    if (info && updates + 1 < 16) info->update_slices_hist[updates + 1] = su;
    if ((rc = apply_update(cur, other, QH, n, gt, w, st, &nprod, tm, su, skip)) != SR_OK) return rc;
    // Predicted ||Y|| after this update (its exact-arithmetic part; the rounding of
    // the hp products adds about sqrt(n) u_hp, which no update removes). With
    // X = (I + W)^H (I + Y) (I + W) - I, ||X|| <= ||Y|| (1 + ||W||)^2 + ||W||^2, one
    // Newton-Schulz step leaves -3/4 X^2 + 1/4 X^3 (Lemma 2), and the dropped terms
    // W^2 Y, W^2 Y W add about ||W||^2 ||Y||. After a skip: ||X|| itself.
    {
      const double yk = skip ? y_pred : ny;
      const double x = yk * (1 + nw) * (1 + nw) + nw * nw;
      y_pred = skip ? x : 0.75 * x * x + 0.25 * x * x * x + nw * nw * yk * (1 + nw);
    }
    skipped_last = skip;
    skips += skip ? 1 : 0;
    zc* t = cur;
    cur = other;
    other = t;
    updates++;
  }
  if (cur != Q) CK(hipMemcpyAsync(Q, cur, (size_t)n * n * sizeof(zc), hipMemcpyDeviceToDevice, st));
  CK(hipEventRecord(ev.t1, st));
  CK(hipEventSynchronize(ev.t1));
  float ms = 0;
  hipEventElapsedTime(&ms, ev.t0, ev.t1);
  if (info) {
    info->status = status;
    info->iters = passes;
    info->updates = updates;
    info->hp_gemms = 2 + 4 * updates + 2 * (passes - updates) - skips;
    info->lp_products = nprod;
    info->resid = eps;
    info->orth = orth;
    info->ms_total = ms;
    if (tm) {
      info->ms_hp_gemm = timer.total(0);
      info->hp_gemm_launches = timer.count[0];
      info->hp_gemm_herm_launches = timer.herm;
      info->ms_hp_gemm_herm = timer.total(0, 1);
      info->ms_solve = timer.total(1);
      info->ms_oz_full = timer.total(2);
      info->oz_full_launches = timer.count[2];
      info->oz_full_pairs = w.crt ? crt_moduli(n, w.oz_s) : w.oz_s ? w.oz_s * (w.oz_s + 1) / 2 : 0;
    }
  }
  return status;
}

int schur_refine(const void* A, void* Q, void* T, int n, int iters, double tol, const sr_opts* opts,
                 sr_info* info) {
  const int rc = refine_fp64(A, Q, T, n, iters, tol, opts, info);
  if (rc < 0 && info) info->status = rc;
  return rc;
}

}  // extern "C"

namespace {
// ------------------------------------------------------------------------
// Double-double tier: hp = double-double (every hp product is an Ozaki split
// product of double-double operands with double-double accumulation), lp = FP64
// (the solve and the lp products).

constexpr double kUDD = 4.930380657631324e-32;  // 2^-104
constexpr int kDDSlices = 14, kDDMaxUpd = 14;

struct DDWork {
  zc *Qh, *Ql, *Ph, *Pl, *Yh, *Yl, *Dh, *Dl;
  zc *Tlp, *Elp, *L, *W, *W2, *W3, *YW;
  int8_t *sA, *sQc, *sP, *sQr, *sD;
  int *eA, *eQc, *eP, *eQr, *eD;
  void* scratch;
  double* partials;
  double* scal;
  unsigned* status;
  void* tri;
  int S;
  size_t bytes;
};

int dd_main_slices(const sr_opts* o) { return (o && o->slices > 0) ? o->slices : kDDSlices; }

// Host double-double helpers for the n = 1 case (Dekker's product via fma).
struct HDD {
  double h, l;
};
HDD hdd_add(HDD a, HDD b) {
  const double s = a.h + b.h, bb = s - a.h;
  double e = (a.h - (s - bb)) + (b.h - bb) + a.l + b.l;
  const double r = s + e;
  return {r, e - (r - s)};
}
HDD hdd_mul(HDD a, HDD b) {
  const double p = a.h * b.h;
  const double e = fma(a.h, b.h, -p) + a.h * b.l + a.l * b.h;
  const double r = p + e;
  return {r, e - (r - p)};
}
HDD hdd_div(HDD a, HDD b) {
  const double q1 = a.h / b.h;
  const HDD r = hdd_add(a, hdd_mul({-q1, 0.0}, b));
  const double q2 = r.h / b.h;
  const double s = q1 + q2;
  return {s, q2 - (s - q1)};
}
HDD hdd_sqrt(HDD a) {
  if (!(a.h > 0)) return {0.0, 0.0};
  const double r0 = sqrt(a.h);
  const HDD d = hdd_add(a, hdd_mul({-r0, 0.0}, {r0, 0.0}));
  const double c = d.h / (2.0 * r0);
  const double s = r0 + c;
  return {s, c - (s - r0)};
}

DDWork carve_dd(void* base, int n, const sr_opts* o) {
  DDWork w;
  uintptr_t p = (uintptr_t)base;
  auto take = [&](size_t b) {
    void* r = (void*)p;
    p += align256(b);
    return r;
  };
  const size_t z = (size_t)n * n * sizeof(zc);
  w.Qh = (zc*)take(z);
  w.Ql = (zc*)take(z);
  w.Ph = (zc*)take(z);
  w.Pl = (zc*)take(z);
  w.Yh = (zc*)take(z);
  w.Yl = (zc*)take(z);
  w.Dh = (zc*)take(z);
  w.Dl = (zc*)take(z);
  w.Tlp = (zc*)take(z);
  w.Elp = (zc*)take(z);
  w.L = (zc*)take(z);
  w.W = (zc*)take(z);
  w.W2 = (zc*)take(z);
  w.W3 = (zc*)take(z);
  w.YW = (zc*)take(z);
  w.S = dd_main_slices(o);
  int Su = w.S > kDDMaxUpd ? w.S : kDDMaxUpd;
  if (o && o->update_slices > 0) Su = o->update_slices;
  w.sA = (int8_t*)take(oz_slice_bytes(n, n, w.S));
  w.sQc = (int8_t*)take(oz_slice_bytes(n, n, w.S));
  w.sP = (int8_t*)take(oz_slice_bytes(n, n, w.S));
  w.sQr = (int8_t*)take(oz_slice_bytes(n, n, Su));
  w.sD = (int8_t*)take(oz_slice_bytes(n, n, Su));
  w.eA = (int*)take(n * sizeof(int));
  w.eQc = (int*)take(n * sizeof(int));
  w.eP = (int*)take(n * sizeof(int));
  w.eQr = (int*)take(n * sizeof(int));
  w.eD = (int*)take(n * sizeof(int));
  w.scratch = take(oz_gemm_scratch_bytes(n, n, true));
  int np = oz_gemm_tiles(n, n, n, true, false, w.S, w.S, w.S + 1);
  if (form_w_parts(n) > np) np = form_w_parts(n);
  if (np < 1024) np = 1024;
  w.partials = (double*)take((size_t)np * sizeof(double));
  w.scal = (double*)take(256);
  w.status = (unsigned*)take(256);
  w.tri = take(trisolve_ws_bytes(n));
  w.bytes = (size_t)(p - (uintptr_t)base);
  return w;
}

int read_back_dd(hipStream_t st, const DDWork& w, int count, double* out, unsigned* status) {
  Work v;
  memset(&v, 0, sizeof(v));
  v.scal = w.scal;
  v.status = w.status;
  return read_back(st, v, count, out, status);
}

// Digits per operand of Q Delta in the double-double tier. By default the same as
// the other hp products: the digits of Q are relative to its row maxima, and the
// Schur vectors of a badly scaled matrix have entries far below them, which need
// the full count. update_slices = -1 takes the count from ||Delta|| as in the FP64
// tier (for the unit roundoff 2^-104), which suffices for well-scaled matrices.
int dd_update_slices(const sr_opts& o, int S, double norm_delta) {
  if (o.update_slices > 0) return o.update_slices;
  if (o.update_slices == 0) return S;
  if (!(norm_delta > 0)) return 2;
  int s = (int)ceil(log2(norm_delta / (0.05 * kUDD)) / 8.0);
  if (s < 2) s = 2;
  if (s > kDDMaxUpd) s = kDDMaxUpd;
  return s;
}

GemmArgs dd_args(int n, zc* Ch, zc* Cl) {
  GemmArgs g = gargs(n, n, n, nullptr, 0, nullptr, 0, Ch, n);
  g.Clo = Cl;
  return g;
}

// Qout = Q + Q D in double-double from Su digits per operand.
int dd_update(const zc* Qh, const zc* Ql, zc* Oh, zc* Ol, int n, int Su, const DDWork& w,
              hipStream_t st) {
  CK(oz_split_rows(Qh, Ql, n, n, n, Su, w.sQr, w.eQr, st));
  CK(oz_split_cols(w.Dh, w.Dl, n, n, n, Su, w.sD, w.eD, st));
  GemmArgs u = dd_args(n, Oh, Ol);
  u.Cin = Qh;
  u.Cinlo = Ql;
  u.ldcin = n;
  CK(oz_gemm(EPI_ADD, w.sQr, w.eQr, Su, w.sD, w.eD, Su, 0, Su + 1, u, w.scratch, st, true));
  return SR_OK;
}

// Y = Q^H Q - I (DD) from the column slices of Q in w.sQc; scal[2] = ||Y||^2.
int dd_ydef(int n, const DDWork& w, hipStream_t st) {
  GemmArgs g = dd_args(n, w.Yh, w.Yl);
  g.partials = w.partials;
  g.herm = 1;
  CK(oz_gemm(EPI_YDEF, w.sQc, w.eQc, w.S, w.sQc, w.eQc, w.S, 1, w.S + 1, g, w.scratch, st, true));
  CK(reduce_partials(w.partials, oz_gemm_tiles(n, n, n, true, true, w.S, w.S, w.S + 1), w.scal + 2, st));
  return SR_OK;
}

}  // namespace

extern "C" {

static int refine_dd(const void* A_hi, const void* A_lo, void* Q_hi, void* Q_lo, void* T_hi,
                     void* T_lo, int n, int iters, double tol, const sr_opts* opts_in,
                     sr_info* info) {
  info_init(info);
  if (!A_hi || !A_lo || !Q_hi || !Q_lo || !T_hi || !T_lo || n < 1 || iters < 1 || !(tol > 0)) {
    if (info) info->status = SR_EINVAL;
    return SR_EINVAL;
  }
  sr_opts o;
  if (opts_in) o = *opts_in;
  else sr_default_opts(&o);
  if (o.slices < 0 || o.slices > 32 || o.update_slices < -1 || o.update_slices > 32) {
    if (info) info->status = SR_EINVAL;
    return SR_EINVAL;
  }
  if (o.solver != SR_SOLVER_WAVEFRONT || o.skip_orth || o.lp_digits) {
    if (info) info->status = SR_ENOSYS;
    return SR_ENOSYS;
  }
  hipStream_t st = (hipStream_t)o.stream;
  const zc* Ah = (const zc*)A_hi;
  const zc* Al = (const zc*)A_lo;
  zc* Th = (zc*)T_hi;
  zc* Tl = (zc*)T_lo;
  if (n == 1) {
    // T = A, Q = q / |q| in double-double arithmetic on the host
    zc v[4];
    CK(hipMemcpyAsync(&v[0], Ah, sizeof(zc), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(&v[1], Al, sizeof(zc), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(&v[2], Q_hi, sizeof(zc), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(&v[3], Q_lo, sizeof(zc), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    const HDD qr = hdd_add({v[2].re, 0.0}, {v[3].re, 0.0});
    const HDD qi = hdd_add({v[2].im, 0.0}, {v[3].im, 0.0});
    const HDD m = hdd_sqrt(hdd_add(hdd_mul(qr, qr), hdd_mul(qi, qi)));
    if (!(m.h > 0) || !isfinite(m.h) || !isfinite(v[0].re) || !isfinite(v[0].im)) {
      if (info) info->status = SR_BREAKDOWN;
      return SR_BREAKDOWN;
    }
    const HDD ur = hdd_div(qr, m), ui = hdd_div(qi, m);
    zc out[2] = {mk<double>(ur.h, ui.h), mk<double>(ur.l, ui.l)};
    CK(hipMemcpyAsync(T_hi, &v[0], sizeof(zc), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(T_lo, &v[1], sizeof(zc), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(Q_hi, &out[0], sizeof(zc), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(Q_lo, &out[1], sizeof(zc), hipMemcpyHostToDevice, st));
    CK(hipStreamSynchronize(st));
    if (info) {
      info->status = SR_OK;
      info->iters = 1;
    }
    return SR_OK;
  }
  void* base = nullptr;
  int rc = get_ws(o, sr_workspace_bytes_dd(n, &o), &base);
  if (rc != SR_OK) {
    if (info) info->status = rc;
    return rc;
  }
  const DDWork w = carve_dd(base, n, &o);
  const int S = w.S;

  Timer timer;
  timer.st = st;
  Timer* tm = o.timing ? &timer : nullptr;
  CallEvents ev;
  CK(hipEventCreate(&ev.t0));
  CK(hipEventCreate(&ev.t1));
  CK(hipEventRecord(ev.t0, st));
  CK(fill_zero(w.status, 256, st));
  CK(fro2_partials(Ah, (long)n * n, w.partials, 1024, st));
  CK(reduce_partials(w.partials, 1024, w.scal, st));
  CK(oz_split_rows(Ah, Al, n, n, n, S, w.sA, w.eA, st));
  hipStream_t sst = n <= kSideYMaxNdd ? side_stream(st) : nullptr;
  if (sst) {
    CK(hipEventCreateWithFlags(&ev.fork, hipEventDisableTiming));
    CK(hipEventCreateWithFlags(&ev.join, hipEventDisableTiming));
  }

  // Newton-Schulz start from Q-hat = (Q_hi, Q_lo)
  zc* curh = w.Qh;
  zc* curl = w.Ql;
  zc* othh = (zc*)Q_hi;
  zc* othl = (zc*)Q_lo;
  TIC(tm, 0);
  CK(oz_split_cols(othh, othl, n, n, n, S, w.sQc, w.eQc, st));
  if ((rc = dd_ydef(n, w, st)) != SR_OK) return rc;
  TOC_HERM(tm);
  double nrm[4] = {0, 0, 0, 0};
  unsigned dst = 0;
  if ((rc = read_back_dd(st, w, 3, nrm, &dst)) != SR_OK) return rc;
  CK(form_delta_dd(nullptr, w.Yh, w.Yl, nullptr, nullptr, nullptr, w.Dh, w.Dl, n, st));
  int su = dd_update_slices(o, S, 0.5 * sqrt(nrm[2]));
  if (info) info->update_slices_hist[0] = su;
  TIC(tm, 0);
  if ((rc = dd_update(othh, othl, curh, curl, n, su, w, st)) != SR_OK) return rc;
  TOC(tm, 0);

  int status = SR_NOT_CONVERGED, passes = 0, updates = 0, nprod = 0;
  double eps = 0, eps1 = -1, eps2 = -1, orth = 0, nw_last = 0;
  for (int p = 0; p < iters; p++) {
    TIC(tm, 0);
    CK(oz_split_cols(curh, curl, n, n, n, S, w.sQc, w.eQc, st));
    {
      GemmArgs g = dd_args(n, w.Ph, w.Pl);
      TIC(tm, 2);
      CK(oz_gemm(EPI_STORE, w.sA, w.eA, S, w.sQc, w.eQc, S, 0, S + 1, g, w.scratch, st, true));
      TOC(tm, 2);
    }
    TOC(tm, 0);
    TIC(tm, 0);
    CK(oz_split_cols(w.Ph, w.Pl, n, n, n, S, w.sP, w.eP, st));
    {
      GemmArgs g = dd_args(n, Th, Tl);
      g.Tlp64 = w.Tlp;
      g.Elp64 = w.Elp;
      g.ldlp = n;
      g.partials = w.partials;
      TIC(tm, 2);
      CK(oz_gemm(EPI_SPLIT, w.sQc, w.eQc, S, w.sP, w.eP, S, 1, S + 1, g, w.scratch, st, true));
      TOC(tm, 2);
    }
    TOC(tm, 0);
    CK(reduce_partials(w.partials, oz_gemm_tiles(n, n, n, true, false, w.S, w.S, w.S + 1), w.scal + 1, st));
    double s2[2];
    if ((rc = read_back_dd(st, w, 2, s2, &dst)) != SR_OK) return rc;
    eps = sqrt(s2[1]) / sqrt(s2[0]);
    passes = p + 1;
    if (info && p < 16) info->resid_hist[p] = eps;
    if (!isfinite(eps)) {
      status = SR_BREAKDOWN;
      break;
    }
    const int stop = stop_test(o, eps, tol, eps1, eps2, updates, nw_last, kUDD, n);
    if (stop >= 0) {
      status = stop;
      break;
    }
    eps2 = eps1;
    eps1 = eps;
    if (p == iters - 1) break;

    // Y beside the solve on the side stream up to kSideYMaxNdd (see the FP64 tier)
    const bool side = sst && n <= kSideYMaxNdd;
    if (side) {
      CK(hipEventRecord(ev.fork, st));
      CK(hipStreamWaitEvent(sst, ev.fork, 0));
      hipStream_t keep = tm ? tm->st : nullptr;
      if (tm) tm->st = sst;
      TIC(tm, 0);
      rc = dd_ydef(n, w, sst);
      if (rc == SR_OK) TOC_HERM(tm);
      if (tm) tm->st = keep;
      if (rc != SR_OK) return rc;
      CK(hipEventRecord(ev.join, sst));
    }
    TIC(tm, 1);
    CK(trisolve64(w.Tlp, w.Elp, w.L, n, w.tri, w.status, st));
    TOC(tm, 1);
    if (side) {
      CK(hipStreamWaitEvent(st, ev.join, 0));
    } else {
      TIC(tm, 0);
      if ((rc = dd_ydef(n, w, st)) != SR_OK) return rc;
      TOC_HERM(tm);
    }
    CK(form_w64(w.L, w.W, n, w.partials, st));
    CK(reduce_partials(w.partials, form_w_parts(n), w.scal + 3, st));
    if ((rc = read_back_dd(st, w, 4, nrm, &dst)) != SR_OK) return rc;
    if (dst & DEV_BREAKDOWN) {
      status = SR_BREAKDOWN;
      break;
    }
    const double ny = sqrt(nrm[2]), nw = sqrt(nrm[3]);
    orth = ny;
    nw_last = nw;
    if (info && updates < 16) info->norm_w_hist[updates] = nw;
    if (!isfinite(ny) || !isfinite(nw)) {
      status = SR_BREAKDOWN;
      break;
    }
    // lp products in FP64, gated against the double-double roundoff
    const double thr = 0.1 * kUDD;
    const bool gw2 = !o.gate_lp_terms || nw * nw > thr;
    const bool gw3 = !o.gate_lp_terms || nw * nw * nw > thr;
    const bool gyw = !o.gate_lp_terms || ny * nw > thr;
    if (gw2 || gw3) {
      GemmArgs a2 = gargs(n, n, n, w.W, n, w.W, n, w.W2, n);
      a2.herm = 1;  // W is skew-Hermitian: W^2 is Hermitian
      CK(zgemm(0, EPI_STORE, 0, a2, st));
      nprod++;
    }
    // With both W^3 and YW, one product gives their difference: (W^2 - Y) W (into W3).
    const bool both = gw3 && gyw;
    if (both) {
      CK(w2_minus_y(w.W2, w.Yh, w.YW, (long)n * n, st));
      CK(zgemm(0, EPI_STORE, 0, gargs(n, n, n, w.YW, n, w.W, n, w.W3, n), st));
      nprod++;
    } else if (gw3) {
      GemmArgs a3 = gargs(n, n, n, w.W2, n, w.W, n, w.W3, n);
      a3.herm = -1;  // and W^3 skew-Hermitian
      CK(zgemm(0, EPI_STORE, 0, a3, st));
      nprod++;
    } else if (gyw) {
      CK(zgemm(0, EPI_STORE, 0, gargs(n, n, n, w.Yh, n, w.W, n, w.YW, n), st));
      nprod++;
    }
    CK(form_delta_dd(w.L, w.Yh, w.Yl, gw2 ? w.W2 : nullptr, gw3 ? w.W3 : nullptr,
                     gyw && !both ? w.YW : nullptr, w.Dh, w.Dl, n, st));
    su = dd_update_slices(o, S, nw + 0.5 * ny);
    if (info && updates + 1 < 16) info->update_slices_hist[updates + 1] = su;
    TIC(tm, 0);
    if ((rc = dd_update(curh, curl, othh, othl, n, su, w, st)) != SR_OK) return rc;
    TOC(tm, 0);
    zc* t = curh;
    curh = othh;
    othh = t;
    t = curl;
    curl = othl;
    othl = t;
    updates++;
  }
  if (curh != (zc*)Q_hi) {
    CK(hipMemcpyAsync(Q_hi, curh, (size_t)n * n * sizeof(zc), hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(Q_lo, curl, (size_t)n * n * sizeof(zc), hipMemcpyDeviceToDevice, st));
  }
  CK(hipEventRecord(ev.t1, st));
  CK(hipEventSynchronize(ev.t1));
  float ms = 0;
  hipEventElapsedTime(&ms, ev.t0, ev.t1);
  if (info) {
    info->status = status;
    info->iters = passes;
    info->updates = updates;
    info->hp_gemms = 2 + 4 * updates + 2 * (passes - updates);
    info->lp_products = nprod;
    info->resid = eps;
    info->orth = orth;
    info->ms_total = ms;
    if (tm) {
      info->ms_hp_gemm = timer.total(0);
      info->hp_gemm_launches = timer.count[0];
      info->hp_gemm_herm_launches = timer.herm;
      info->ms_hp_gemm_herm = timer.total(0, 1);
      info->ms_solve = timer.total(1);
      // the product launches P and That alone (no splits)
      info->ms_oz_full = timer.total(2);
      info->oz_full_launches = timer.count[2];
      info->oz_full_pairs = S * (S + 1) / 2;
    }
  }
  return status;
}

int schur_refine_dd(const void* A_hi, const void* A_lo, void* Q_hi, void* Q_lo, void* T_hi, void* T_lo,
                    int n, int iters, double tol, const sr_opts* opts, sr_info* info) {
  const int rc = refine_dd(A_hi, A_lo, Q_hi, Q_lo, T_hi, T_lo, n, iters, tol, opts, info);
  if (rc < 0 && info) info->status = rc;
  return rc;
}

}  // extern "C"

namespace {
// ------------------------------------------------------------------------
// Triple-double tier: hp = triple-double (three-term expansions; every hp product an
// Ozaki split product of the triple-double operands into 22 digits, the windowed
// kernel's three-term accumulation kept to the end), lp = FP64 as in the
// double-double tier.

constexpr double kUTD = 7.006492321624085e-46;  // 2^-150: the products keep about 150 bits
constexpr int kTDSlices = 20;  // 160 bits: floors near 1e-47, 15 digit windows

struct TDWork {
  zc* Q[3];
  zc* P[3];
  zc* Y[3];
  zc* D[3];
  zc *Tlp, *Elp, *L, *W, *W2, *W3, *YW;
  int8_t *sA, *sQc, *sP, *sQr, *sD;
  int *eA, *eQc, *eP, *eQr, *eD;
  void* scratch;
  double* partials;
  double* scal;
  unsigned* status;
  void* tri;
  int S;
  size_t bytes;
};

int td_main_slices(const sr_opts* o) { return (o && o->slices > 0) ? o->slices : kTDSlices; }

TDWork carve_td(void* base, int n, const sr_opts* o) {
  TDWork w;
  uintptr_t p = (uintptr_t)base;
  auto take = [&](size_t b) {
    void* r = (void*)p;
    p += align256(b);
    return r;
  };
  const size_t z = (size_t)n * n * sizeof(zc);
  for (int t = 0; t < 3; t++) w.Q[t] = (zc*)take(z);
  for (int t = 0; t < 3; t++) w.P[t] = (zc*)take(z);
  for (int t = 0; t < 3; t++) w.Y[t] = (zc*)take(z);
  for (int t = 0; t < 3; t++) w.D[t] = (zc*)take(z);
  w.Tlp = (zc*)take(z);
  w.Elp = (zc*)take(z);
  w.L = (zc*)take(z);
  w.W = (zc*)take(z);
  w.W2 = (zc*)take(z);
  w.W3 = (zc*)take(z);
  w.YW = (zc*)take(z);
  w.S = td_main_slices(o);
  w.sA = (int8_t*)take(oz_slice_bytes(n, n, w.S));
  w.sQc = (int8_t*)take(oz_slice_bytes(n, n, w.S));
  w.sP = (int8_t*)take(oz_slice_bytes(n, n, w.S));
  w.sQr = (int8_t*)take(oz_slice_bytes(n, n, w.S));
  w.sD = (int8_t*)take(oz_slice_bytes(n, n, w.S));
  w.eA = (int*)take(n * sizeof(int));
  w.eQc = (int*)take(n * sizeof(int));
  w.eP = (int*)take(n * sizeof(int));
  w.eQr = (int*)take(n * sizeof(int));
  w.eD = (int*)take(n * sizeof(int));
  w.scratch = take(oz_gemm_scratch_bytes(n, n, true));
  int np = oz_gemm_tiles(n, n, n, true, false, w.S, w.S, w.S + 1, true);
  if (form_w_parts(n) > np) np = form_w_parts(n);
  if (np < 1024) np = 1024;
  w.partials = (double*)take((size_t)np * sizeof(double));
  w.scal = (double*)take(256);
  w.status = (unsigned*)take(256);
  w.tri = take(trisolve_ws_bytes(n));
  w.bytes = (size_t)(p - (uintptr_t)base);
  return w;
}

int read_back_td(hipStream_t st, const TDWork& w, int count, double* out, unsigned* status) {
  Work v;
  memset(&v, 0, sizeof(v));
  v.scal = w.scal;
  v.status = w.status;
  return read_back(st, v, count, out, status);
}

GemmArgs td_args(int n, zc* const* C) {
  GemmArgs g = gargs(n, n, n, nullptr, 0, nullptr, 0, C[0], n);
  g.Cmid = C[1];
  g.Clo = C[2];
  return g;
}

// Qout = Q + Q D (triple-double) from S digits per operand.
int td_update(zc* const* Q, zc* const* O, int n, const TDWork& w, hipStream_t st) {
  const int S = w.S;
  CK(oz_split_rows3(Q[0], Q[1], Q[2], n, n, n, S, w.sQr, w.eQr, st));
  CK(oz_split_cols3(w.D[0], w.D[1], w.D[2], n, n, n, S, w.sD, w.eD, st));
  GemmArgs u = td_args(n, O);
  u.Cin = Q[0];
  u.Cinmid = Q[1];
  u.Cinlo = Q[2];
  u.ldcin = n;
  CK(oz_gemm(EPI_ADD, w.sQr, w.eQr, S, w.sD, w.eD, S, 0, S + 1, u, w.scratch, st, true));
  return SR_OK;
}

// Y = Q^H Q - I (triple-double) from the column slices of Q in w.sQc; scal[2] = ||Y||^2.
int td_ydef(int n, const TDWork& w, hipStream_t st) {
  GemmArgs g = td_args(n, w.Y);
  g.partials = w.partials;
  g.herm = 1;
  CK(oz_gemm(EPI_YDEF, w.sQc, w.eQc, w.S, w.sQc, w.eQc, w.S, 1, w.S + 1, g, w.scratch, st, true));
  CK(reduce_partials(w.partials, oz_gemm_tiles(n, n, n, true, true, w.S, w.S, w.S + 1, true), w.scal + 2, st));
  return SR_OK;
}

int refine_td(const void* const* A_, void* const* Q_, void* const* T_, int n, int iters, double tol,
              const sr_opts* opts_in, sr_info* info) {
  info_init(info);
  if (!A_ || !Q_ || !T_ || n < 2 || iters < 1 || !(tol > 0)) return SR_EINVAL;
  for (int t = 0; t < 3; t++)
    if (!A_[t] || !Q_[t] || !T_[t]) return SR_EINVAL;
  sr_opts o;
  if (opts_in) o = *opts_in;
  else sr_default_opts(&o);
  if (o.slices < 0 || o.slices > 32 || (o.slices > 0 && o.slices < 20)) return SR_EINVAL;
  if (o.solver != SR_SOLVER_WAVEFRONT || o.skip_orth || o.lp_digits || o.gemm != SR_GEMM_FP64) return SR_ENOSYS;
  if (!oz_td_ok(n, n, n, td_main_slices(&o))) return SR_EINVAL;
  hipStream_t st = (hipStream_t)o.stream;
  const zc* A[3] = {(const zc*)A_[0], (const zc*)A_[1], (const zc*)A_[2]};
  zc* Tt[3] = {(zc*)T_[0], (zc*)T_[1], (zc*)T_[2]};
  void* base = nullptr;
  int rc = get_ws(o, sr_workspace_bytes_td(n, &o), &base);
  if (rc != SR_OK) return rc;
  const TDWork w = carve_td(base, n, &o);
  const int S = w.S;

  Timer timer;
  timer.st = st;
  Timer* tm = o.timing ? &timer : nullptr;
  CallEvents ev;
  CK(hipEventCreate(&ev.t0));
  CK(hipEventCreate(&ev.t1));
  CK(hipEventRecord(ev.t0, st));
  CK(fill_zero(w.status, 256, st));
  CK(fro2_partials(A[0], (long)n * n, w.partials, 1024, st));
  CK(reduce_partials(w.partials, 1024, w.scal, st));
  CK(oz_split_rows3(A[0], A[1], A[2], n, n, n, S, w.sA, w.eA, st));

  // Newton-Schulz start from the given Q-hat
  zc* cur[3] = {w.Q[0], w.Q[1], w.Q[2]};
  zc* oth[3] = {(zc*)Q_[0], (zc*)Q_[1], (zc*)Q_[2]};
  TIC(tm, 0);
  CK(oz_split_cols3(oth[0], oth[1], oth[2], n, n, n, S, w.sQc, w.eQc, st));
  if ((rc = td_ydef(n, w, st)) != SR_OK) return rc;
  TOC_HERM(tm);
  double nrm[4] = {0, 0, 0, 0};
  unsigned dst = 0;
  if ((rc = read_back_td(st, w, 3, nrm, &dst)) != SR_OK) return rc;
  CK(form_delta_td(nullptr, w.Y[0], w.Y[1], w.Y[2], nullptr, nullptr, nullptr, w.D[0], w.D[1], w.D[2], n, st));
  TIC(tm, 0);
  if ((rc = td_update(oth, cur, n, w, st)) != SR_OK) return rc;
  TOC(tm, 0);

  int status = SR_NOT_CONVERGED, passes = 0, updates = 0, nprod = 0;
  double eps = 0, eps1 = -1, eps2 = -1, orth = 0, nw_last = 0;
  for (int p = 0; p < iters; p++) {
    TIC(tm, 0);
    CK(oz_split_cols3(cur[0], cur[1], cur[2], n, n, n, S, w.sQc, w.eQc, st));
    {
      GemmArgs g = td_args(n, w.P);
      TIC(tm, 2);
      CK(oz_gemm(EPI_STORE, w.sA, w.eA, S, w.sQc, w.eQc, S, 0, S + 1, g, w.scratch, st, true));
      TOC(tm, 2);
    }
    TOC(tm, 0);
    TIC(tm, 0);
    CK(oz_split_cols3(w.P[0], w.P[1], w.P[2], n, n, n, S, w.sP, w.eP, st));
    {
      GemmArgs g = td_args(n, Tt);
      g.Tlp64 = w.Tlp;
      g.Elp64 = w.Elp;
      g.ldlp = n;
      g.partials = w.partials;
      TIC(tm, 2);
      CK(oz_gemm(EPI_SPLIT, w.sQc, w.eQc, S, w.sP, w.eP, S, 1, S + 1, g, w.scratch, st, true));
      TOC(tm, 2);
    }
    TOC(tm, 0);
    CK(reduce_partials(w.partials, oz_gemm_tiles(n, n, n, true, false, S, S, S + 1, true), w.scal + 1, st));
    double s2[2];
    if ((rc = read_back_td(st, w, 2, s2, &dst)) != SR_OK) return rc;
    eps = sqrt(s2[1]) / sqrt(s2[0]);
    passes = p + 1;
    if (info && p < 16) info->resid_hist[p] = eps;
    if (!isfinite(eps)) {
      status = SR_BREAKDOWN;
      break;
    }
    const int stop = stop_test(o, eps, tol, eps1, eps2, updates, nw_last, kUTD, n);
    if (stop >= 0) {
      status = stop;
      break;
    }
    eps2 = eps1;
    eps1 = eps;
    if (p == iters - 1) break;

    TIC(tm, 1);
    CK(trisolve64(w.Tlp, w.Elp, w.L, n, w.tri, w.status, st));
    TOC(tm, 1);
    TIC(tm, 0);
    if ((rc = td_ydef(n, w, st)) != SR_OK) return rc;
    TOC_HERM(tm);
    CK(form_w64(w.L, w.W, n, w.partials, st));
    CK(reduce_partials(w.partials, form_w_parts(n), w.scal + 3, st));
    if ((rc = read_back_td(st, w, 4, nrm, &dst)) != SR_OK) return rc;
    if (dst & DEV_BREAKDOWN) {
      status = SR_BREAKDOWN;
      break;
    }
    const double ny = sqrt(nrm[2]), nw = sqrt(nrm[3]);
    orth = ny;
    nw_last = nw;
    if (info && updates < 16) info->norm_w_hist[updates] = nw;
    if (!isfinite(ny) || !isfinite(nw)) {
      status = SR_BREAKDOWN;
      break;
    }
    // lp products in FP64, gated against the triple-double roundoff
    const double thr = 0.1 * kUTD;
    const bool gw2 = !o.gate_lp_terms || nw * nw > thr;
    const bool gw3 = !o.gate_lp_terms || nw * nw * nw > thr;
    const bool gyw = !o.gate_lp_terms || ny * nw > thr;
    if (gw2 || gw3) {
      GemmArgs a2 = gargs(n, n, n, w.W, n, w.W, n, w.W2, n);
      a2.herm = 1;
      CK(zgemm(0, EPI_STORE, 0, a2, st));
      nprod++;
    }
    const bool both = gw3 && gyw;
    if (both) {
      CK(w2_minus_y(w.W2, w.Y[0], w.YW, (long)n * n, st));
      CK(zgemm(0, EPI_STORE, 0, gargs(n, n, n, w.YW, n, w.W, n, w.W3, n), st));
      nprod++;
    } else if (gw3) {
      GemmArgs a3 = gargs(n, n, n, w.W2, n, w.W, n, w.W3, n);
      a3.herm = -1;
      CK(zgemm(0, EPI_STORE, 0, a3, st));
      nprod++;
    } else if (gyw) {
      CK(zgemm(0, EPI_STORE, 0, gargs(n, n, n, w.Y[0], n, w.W, n, w.YW, n), st));
      nprod++;
    }
    CK(form_delta_td(w.L, w.Y[0], w.Y[1], w.Y[2], gw2 ? w.W2 : nullptr, gw3 ? w.W3 : nullptr,
                     gyw && !both ? w.YW : nullptr, w.D[0], w.D[1], w.D[2], n, st));
    TIC(tm, 0);
    if ((rc = td_update(cur, oth, n, w, st)) != SR_OK) return rc;
    TOC(tm, 0);
    for (int t = 0; t < 3; t++) {
      zc* x = cur[t];
      cur[t] = oth[t];
      oth[t] = x;
    }
    updates++;
  }
  if (cur[0] != (zc*)Q_[0])
    for (int t = 0; t < 3; t++)
      CK(hipMemcpyAsync(Q_[t], cur[t], (size_t)n * n * sizeof(zc), hipMemcpyDeviceToDevice, st));
  CK(hipEventRecord(ev.t1, st));
  CK(hipEventSynchronize(ev.t1));
  float ms = 0;
  hipEventElapsedTime(&ms, ev.t0, ev.t1);
  if (info) {
    info->status = status;
    info->iters = passes;
    info->updates = updates;
    info->hp_gemms = 2 + 4 * updates + 2 * (passes - updates);
    info->lp_products = nprod;
    info->resid = eps;
    info->orth = orth;
    info->ms_total = ms;
    if (tm) {
      info->ms_hp_gemm = timer.total(0);
      info->hp_gemm_launches = timer.count[0];
      info->hp_gemm_herm_launches = timer.herm;
      info->ms_hp_gemm_herm = timer.total(0, 1);
      info->ms_solve = timer.total(1);
      // the product launches P and That alone (no splits)
      info->ms_oz_full = timer.total(2);
      info->oz_full_launches = timer.count[2];
      info->oz_full_pairs = S * (S + 1) / 2;
    }
  }
  return status;
}
}  // namespace

extern "C" {

size_t sr_workspace_bytes_td(int n, const sr_opts* opts) {
  if (n < 1) return 0;
  return carve_td(nullptr, n, opts).bytes + 256;
}

int schur_refine_td(const void* const* A, void* const* Q, void* const* T, int n, int iters, double tol,
                    const sr_opts* opts, sr_info* info) {
  const int rc = refine_td(A, Q, T, n, iters, tol, opts, info);
  if (rc < 0 && info) info->status = rc;
  return rc;
}

size_t sr_workspace_bytes_dd(int n, const sr_opts* opts) {
  if (n < 1) return 0;
  return carve_dd(nullptr, n, opts).bytes + 256;
}

}  // extern "C"

namespace {
// ------------------------------------------------------------------------
// Real Schur variant: real products (FP64 MFMA, compensated by default), the block
// strictly lower residual, the FP32 block solve, the merged update on real data.

struct RealWork {
  double *Qa, *QT, *P, *Y;
  float *Tlp, *Elp, *Llp, *W, *W2, *W3, *YW, *Ylp;
  int* blk;
  double* partials;
  double* scal;
  unsigned* status;
  void* tri;
  size_t bytes;
};

int real_partial_slots(int n) {
  int a = rgemm_tiles(n, n, false), b = rform_w_parts(n);
  int m = a > b ? a : b;
  return m > 1024 ? m : 1024;
}

RealWork carve_real(void* base, int n) {
  RealWork w;
  uintptr_t p = (uintptr_t)base;
  const size_t d = align256((size_t)n * n * sizeof(double)), f = align256((size_t)n * n * sizeof(float));
  auto take = [&](size_t b) {
    void* r = (void*)p;
    p += b;
    return r;
  };
  w.Qa = (double*)take(d);
  w.QT = (double*)take(d);
  w.P = (double*)take(d);
  w.Y = (double*)take(d);
  w.Tlp = (float*)take(f);
  w.Elp = (float*)take(f);
  w.Llp = (float*)take(f);
  w.W = (float*)take(f);
  w.W2 = (float*)take(f);
  w.W3 = (float*)take(f);
  w.YW = (float*)take(f);
  w.Ylp = (float*)take(f);
  w.blk = (int*)take(align256((size_t)n * sizeof(int)));
  w.partials = (double*)take(align256((size_t)real_partial_slots(n) * sizeof(double)));
  w.scal = (double*)take(256);
  w.status = (unsigned*)take(256);
  w.tri = take(align256(trisolve_real_ws_bytes(n)));
  w.bytes = (size_t)(p - (uintptr_t)base);
  return w;
}

// the 2 x 2 markers as the oracle reads them: a block never starts at the last row
// and never overlaps the next one
bool real_blocks_valid(const int* blk, int n) {
  if (!blk) return true;
  for (int i = 0; i < n; i++) {
    if (blk[i] != 0 && blk[i] != 1) return false;
    if (blk[i] && (i + 1 >= n || blk[i + 1])) return false;
  }
  return true;
}

RGemmArgs rargs(int m, int n, int k, const void* A, long lda, const void* B, long ldb, void* C, long ldc) {
  RGemmArgs g;
  memset(&g, 0, sizeof(g));
  g.m = m;
  g.n = n;
  g.k = k;
  g.A = A;
  g.lda = lda;
  g.B = B;
  g.ldb = ldb;
  g.C = C;
  g.ldc = ldc;
  return g;
}

int read_back_real(hipStream_t st, const RealWork& w, int count, double* out, unsigned* status) {
  Work v;
  memset(&v, 0, sizeof(v));
  v.scal = w.scal;
  v.status = w.status;
  return read_back(st, v, count, out, status);
}

int refine_real_fp64(const void* A_, void* Q_, void* T_, const int* blocks, int n, int iters, double tol,
                     const sr_opts* opts_in, sr_info* info) {
  info_init(info);
  if (!A_ || !Q_ || !T_ || n < 1 || iters < 1 || !(tol > 0) || !real_blocks_valid(blocks, n)) return SR_EINVAL;
  sr_opts o;
  if (opts_in) o = *opts_in;
  else sr_default_opts(&o);
  if (o.gemm != SR_GEMM_FP64 || o.solver != SR_SOLVER_WAVEFRONT || o.skip_orth || o.lp_digits) return SR_ENOSYS;
  hipStream_t st = (hipStream_t)o.stream;
  const double* A = (const double*)A_;
  double* Q = (double*)Q_;
  double* T = (double*)T_;
  if (n == 1) {
    double a, q;
    CK(hipMemcpyAsync(&a, A, sizeof(double), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(&q, Q, sizeof(double), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (!(q != 0) || !isfinite(a)) return SR_BREAKDOWN;
    const double qs = q > 0 ? 1.0 : -1.0;
    CK(hipMemcpyAsync(T, &a, sizeof(double), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(Q, &qs, sizeof(double), hipMemcpyHostToDevice, st));
    CK(hipStreamSynchronize(st));
    if (info) {
      info->status = SR_OK;
      info->iters = 1;
    }
    return SR_OK;
  }
  void* base = nullptr;
  int rc = get_ws(o, sr_workspace_bytes_real(n, &o), &base);
  if (rc != SR_OK) return rc;
  const RealWork w = carve_real(base, n);
  const int comp = o.compensated ? 1 : 0;
  Timer timer;
  timer.st = st;
  Timer* tm = o.timing ? &timer : nullptr;
  CallEvents ev;
  CK(hipEventCreate(&ev.t0));
  CK(hipEventCreate(&ev.t1));
  CK(hipEventRecord(ev.t0, st));
  if (blocks) CK(hipMemcpyAsync(w.blk, blocks, (size_t)n * sizeof(int), hipMemcpyHostToDevice, st));
  else CK(fill_zero(w.blk, (size_t)n * sizeof(int), st));
  CK(fill_zero(w.status, 256, st));
  CK(rfro2_partials(A, (long)n * n, w.partials, 1024, st));
  CK(reduce_partials(w.partials, 1024, w.scal, st));

  // Newton-Schulz start: Y0 = Qh^T Qh - I, Qa = Qh + Qh (-Y0 / 2), QT = Qa^T
  {
    RGemmArgs g = rargs(n, n, n, Q, n, Q, n, w.Y, n);
    g.partials = w.partials;
    g.herm = 1;
    TIC(tm, 0);
    CK(dgemm(1, EPI_YDEF, comp, g, st));
    TOC_HERM(tm);
    CK(rform_delta(nullptr, w.Y, nullptr, nullptr, nullptr, w.P, n, st));
    RGemmArgs u = rargs(n, n, n, Q, n, w.P, n, w.Qa, n);
    u.Cin = Q;
    u.ldcin = n;
    u.CT = w.QT;
    u.ldct = n;
    TIC(tm, 0);
    CK(dgemm(0, EPI_ADD, 0, u, st));
    TOC(tm, 0);
  }
  int status = SR_NOT_CONVERGED, passes = 0, updates = 0, nprod = 0;
  double eps = 0, eps1 = -1, eps2 = -1, orth = 0, nw_last = 0;
  double* cur = w.Qa;
  double* other = Q;
  for (int p = 0; p < iters; p++) {
    // P = A Q; That = Q^T P split at the block structure
    RGemmArgs g = rargs(n, n, n, A, n, cur, n, w.P, n);
    TIC(tm, 0);
    CK(dgemm(0, EPI_STORE, comp, g, st));
    TOC(tm, 0);
    RGemmArgs sg = rargs(n, n, n, w.QT, n, w.P, n, T, n);
    sg.Tlp = w.Tlp;
    sg.Elp = w.Elp;
    sg.ldlp = n;
    sg.partials = w.partials;
    sg.blk = w.blk;
    TIC(tm, 0);
    CK(dgemm(0, EPI_SPLIT, comp, sg, st));
    TOC(tm, 0);
    CK(reduce_partials(w.partials, rgemm_tiles(n, n, false), w.scal + 1, st));
    double s2[2];
    unsigned dst = 0;
    if ((rc = read_back_real(st, w, 2, s2, &dst)) != SR_OK) return rc;
    eps = sqrt(s2[1]) / sqrt(s2[0]);
    passes = p + 1;
    if (info && p < 16) info->resid_hist[p] = eps;
    if (!isfinite(eps)) {
      status = SR_BREAKDOWN;
      break;
    }
    const int stop = stop_test(o, eps, tol, eps1, eps2, updates, nw_last, kU64, n);
    if (stop >= 0) {
      status = stop;
      break;
    }
    eps2 = eps1;
    eps1 = eps;
    if (p == iters - 1) break;

    TIC(tm, 1);
    CK(trisolve_real(w.Tlp, T, w.Elp, w.Llp, w.blk, n, w.tri, w.status, st));
    TOC(tm, 1);
    RGemmArgs yg = rargs(n, n, n, w.QT, n, cur, n, w.Y, n);
    yg.partials = w.partials;
    yg.herm = 1;
    TIC(tm, 0);
    CK(dgemm(0, EPI_YDEF, comp, yg, st));
    TOC_HERM(tm);
    CK(reduce_partials(w.partials, rgemm_tiles(n, n, true), w.scal + 2, st));
    CK(rform_w(w.Llp, w.W, n, w.partials, st));
    CK(reduce_partials(w.partials, rform_w_parts(n), w.scal + 3, st));
    double nrm[4];
    if ((rc = read_back_real(st, w, 4, nrm, &dst)) != SR_OK) return rc;
    if (dst & DEV_BREAKDOWN) {
      status = SR_BREAKDOWN;
      break;
    }
    const double ny = sqrt(nrm[2]), nw = sqrt(nrm[3]);
    orth = ny;
    nw_last = nw;
    if (info && updates < 16) info->norm_w_hist[updates] = nw;
    if (!isfinite(ny) || !isfinite(nw)) {
      status = SR_BREAKDOWN;
      break;
    }
    const Gate gt = gate_terms(o.gate_lp_terms != 0, nw, ny);
    if (gt.w2 || gt.w3) {
      RGemmArgs a2 = rargs(n, n, n, w.W, n, w.W, n, w.W2, n);
      a2.herm = 1;  // W is skew-symmetric: W^2 is symmetric
      CK(sgemm(a2, st));
      nprod++;
    }
    const bool both = gt.w3 && gt.yw;
    if (both) {
      CK(rw2_minus_y(w.W2, w.Y, w.Ylp, (long)n * n, st));
      CK(sgemm(rargs(n, n, n, w.Ylp, n, w.W, n, w.W3, n), st));
      nprod++;
    } else if (gt.w3) {
      RGemmArgs a3 = rargs(n, n, n, w.W2, n, w.W, n, w.W3, n);
      a3.herm = -1;  // and W^3 skew-symmetric
      CK(sgemm(a3, st));
      nprod++;
    } else if (gt.yw) {
      CK(rw2_minus_y(nullptr, w.Y, w.Ylp, (long)n * n, st));
      CK(sgemm(rargs(n, n, n, w.Ylp, n, w.W, n, w.YW, n), st));
      nprod++;
    }
    CK(rform_delta(w.Llp, w.Y, gt.w2 ? w.W2 : nullptr, gt.w3 ? w.W3 : nullptr, gt.yw && !both ? w.YW : nullptr,
                   w.P, n, st));
    RGemmArgs u = rargs(n, n, n, cur, n, w.P, n, other, n);
    u.Cin = cur;
    u.ldcin = n;
    u.CT = w.QT;
    u.ldct = n;
    TIC(tm, 0);
    CK(dgemm(0, EPI_ADD, 0, u, st));
    TOC(tm, 0);
    double* t = cur;
    cur = other;
    other = t;
    updates++;
  }
  if (cur != Q) CK(hipMemcpyAsync(Q, cur, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, st));
  CK(hipEventRecord(ev.t1, st));
  CK(hipEventSynchronize(ev.t1));
  float ms = 0;
  hipEventElapsedTime(&ms, ev.t0, ev.t1);
  if (info) {
    info->status = status;
    info->iters = passes;
    info->updates = updates;
    info->hp_gemms = 2 + 4 * updates + 2 * (passes - updates);
    info->lp_products = nprod;
    info->resid = eps;
    info->orth = orth;
    info->ms_total = ms;
    if (tm) {
      info->ms_hp_gemm = timer.total(0);
      info->hp_gemm_launches = timer.count[0];
      info->hp_gemm_herm_launches = timer.herm;
      info->ms_hp_gemm_herm = timer.total(0, 1);
      info->ms_solve = timer.total(1);
    }
  }
  return status;
}
}  // namespace

extern "C" {

size_t sr_workspace_bytes_real(int n, const sr_opts* opts) {
  (void)opts;
  if (n < 1) return 0;
  return carve_real(nullptr, n).bytes + 256;
}

int schur_refine_real(const void* A, void* Q, void* T, const int* blocks, int n, int iters, double tol,
                      const sr_opts* opts, sr_info* info) {
  const int rc = refine_real_fp64(A, Q, T, blocks, n, iters, tol, opts, info);
  if (rc < 0 && info) info->status = rc;
  return rc;
}

int sr_dgemm(int opa, int m, int n, int k, const void* A, int lda, const void* B, int ldb, const void* Cin,
             int ldcin, void* C, int ldc, int compensated, void* stream) {
  if (m < 0 || n < 0 || k < 0 || (opa != 0 && opa != 1) || !C) return SR_EINVAL;
  if (m == 0 || n == 0) return SR_OK;
  if (k > 0 && (!A || !B)) return SR_EINVAL;
  if (lda < (opa ? (k > 1 ? k : 1) : (m > 1 ? m : 1)) || ldb < (k > 1 ? k : 1) || ldc < m) return SR_EINVAL;
  if (Cin && ldcin < m) return SR_EINVAL;
  RGemmArgs g = rargs(m, n, k, A, lda, B, ldb, C, ldc);
  g.Cin = Cin;
  g.ldcin = ldcin;
  CK(dgemm(opa, Cin ? EPI_ADD : EPI_STORE, compensated ? 1 : 0, g, (hipStream_t)stream));
  return SR_OK;
}

size_t sr_trisolve_real_ws_bytes(int n) {
  if (n < 1) return 0;
  return align256(trisolve_real_ws_bytes(n)) + align256((size_t)n * sizeof(int)) + 256;
}

int sr_trisolve_real(const void* T_lp, const void* E_lp, void* L_lp, const int* blocks, int n, void* ws,
                     size_t ws_bytes, void* stream) {
  if (!T_lp || !E_lp || !L_lp || !ws || n < 1 || !real_blocks_valid(blocks, n)) return SR_EINVAL;
  if (ws_bytes < sr_trisolve_real_ws_bytes(n)) return SR_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  char* p = (char*)ws;
  void* tri = p;
  int* blk = (int*)(p + align256(trisolve_real_ws_bytes(n)));
  unsigned* status = (unsigned*)((char*)blk + align256((size_t)n * sizeof(int)));
  if (blocks) CK(hipMemcpyAsync(blk, blocks, (size_t)n * sizeof(int), hipMemcpyHostToDevice, st));
  else CK(fill_zero(blk, (size_t)n * sizeof(int), st));
  CK(fill_zero(status, sizeof(unsigned), st));
  CK(trisolve_real((const float*)T_lp, nullptr, (const float*)E_lp, (float*)L_lp, blk, n, tri, status, st));
  unsigned d = 0;
  CK(hipMemcpyAsync(&d, status, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  return (d & DEV_BREAKDOWN) ? SR_BREAKDOWN : SR_OK;
}

int sr_zgemm(int opa, int m, int n, int k, const void* A, int lda, const void* B, int ldb,
             const void* Cin, int ldcin, void* C, int ldc, int compensated, void* stream) {
  if (m < 0 || n < 0 || k < 0 || (opa != 0 && opa != 1) || !C) return SR_EINVAL;
  if (m == 0 || n == 0) return SR_OK;
  if (k > 0 && (!A || !B)) return SR_EINVAL;
  if (lda < (opa ? (k > 1 ? k : 1) : (m > 1 ? m : 1)) || ldb < (k > 1 ? k : 1) || ldc < m) return SR_EINVAL;
  if (Cin && ldcin < m) return SR_EINVAL;
  GemmArgs g = gargs(m, n, k, A, lda, B, ldb, C, ldc);
  g.Cin = Cin;
  g.ldcin = ldcin;
  CK(zgemm(opa, Cin ? EPI_ADD : EPI_STORE, compensated ? 1 : 0, g, (hipStream_t)stream));
  return SR_OK;
}

size_t sr_ozaki_ws_bytes(int m, int n, int k, int slices_a, int slices_b) {
  if (m < 0 || n < 0 || k < 0 || slices_a < 1 || slices_b < 1) return 0;
  return align256(oz_slice_bytes(m, k, slices_a)) + align256(oz_slice_bytes(n, k, slices_b)) +
         align256((size_t)(m + n) * sizeof(int)) + align256(oz_gemm_scratch_bytes(m, n, true));
}

int sr_ozaki_zgemm(int opa, int m, int n, int k, const void* A, int lda, const void* B, int ldb,
                   const void* Cin, int ldcin, void* C, int ldc, int slices_a, int slices_b, int dmax,
                   void* ws, size_t ws_bytes, void* stream) {
  if (m < 0 || n < 0 || k < 0 || (opa != 0 && opa != 1) || !C) return SR_EINVAL;
  if (slices_a < 1 || slices_b < 1 || slices_a > 32 || slices_b > 32 || dmax < 2) return SR_EINVAL;
  if (m == 0 || n == 0) return SR_OK;
  if (k > 0 && (!A || !B)) return SR_EINVAL;
  if (lda < (opa ? (k > 1 ? k : 1) : (m > 1 ? m : 1)) || ldb < (k > 1 ? k : 1) || ldc < m) return SR_EINVAL;
  if (Cin && ldcin < m) return SR_EINVAL;
  if (!oz_gemm_exact(m, n, k, slices_a, slices_b)) return SR_EINVAL;
  if (!ws || ws_bytes < sr_ozaki_ws_bytes(m, n, k, slices_a, slices_b)) return SR_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  int8_t* qa = (int8_t*)ws;
  int8_t* qb = qa + align256(oz_slice_bytes(m, k, slices_a));
  int* ea = (int*)(qb + align256(oz_slice_bytes(n, k, slices_b)));
  int* eb = ea + m;
  void* scr = (int8_t*)ea + align256((size_t)(m + n) * sizeof(int));
  if (opa == 0) CK(oz_split_rows((const zc*)A, nullptr, lda, m, k, slices_a, qa, ea, st));
  else CK(oz_split_cols((const zc*)A, nullptr, lda, k, m, slices_a, qa, ea, st));
  CK(oz_split_cols((const zc*)B, nullptr, ldb, k, n, slices_b, qb, eb, st));
  GemmArgs g = gargs(m, n, k, nullptr, 0, nullptr, 0, C, ldc);
  g.Cin = Cin;
  g.ldcin = ldcin;
  CK(oz_gemm(Cin ? EPI_ADD : EPI_STORE, qa, ea, slices_a, qb, eb, slices_b, opa, dmax, g, scr, st));
  return SR_OK;
}

int sr_crt_moduli(int k, int bits) { return (k < 1 || bits < 1 || k >= 65536) ? 0 : crt_moduli(k, bits); }

size_t sr_crt_ws_bytes(int m, int n, int k, int bits) {
  const int N = sr_crt_moduli(k, bits);
  if (m < 0 || n < 0 || !N) return 0;
  return align256(crt_residue_bytes(m, k, N)) + align256(crt_residue_bytes(n, k, N)) +
         align256((size_t)(m + n) * sizeof(int)) + align256(crt_scratch_bytes(m, n, N));
}

int sr_crt_zgemm(int opa, int m, int n, int k, const void* A, int lda, const void* B, int ldb, const void* Cin,
                 int ldcin, void* C, int ldc, int bits, void* ws, size_t ws_bytes, void* stream) {
  if (m < 0 || n < 0 || k < 0 || (opa != 0 && opa != 1) || !C) return SR_EINVAL;
  if (m == 0 || n == 0) return SR_OK;
  if (k > 0 && (!A || !B)) return SR_EINVAL;
  if (k < 1 || !sr_crt_moduli(k, bits)) return SR_EINVAL;
  if (lda < (opa ? k : (m > 1 ? m : 1)) || ldb < k || ldc < m) return SR_EINVAL;
  if (Cin && ldcin < m) return SR_EINVAL;
  if (!ws || ws_bytes < sr_crt_ws_bytes(m, n, k, bits)) return SR_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  const int N = crt_moduli(k, bits);
  int8_t* ra = (int8_t*)ws;
  int8_t* rb = ra + align256(crt_residue_bytes(m, k, N));
  int* ta = (int*)(rb + align256(crt_residue_bytes(n, k, N)));
  int* tb = ta + m;
  void* scr = (int8_t*)ta + align256((size_t)(m + n) * sizeof(int));
  if (opa == 0) CK(crt_split_rows((const zc*)A, lda, m, k, bits, ra, ta, st));
  else CK(crt_split_cols((const zc*)A, lda, k, m, bits, ra, ta, st));
  CK(crt_split_cols((const zc*)B, ldb, k, n, bits, rb, tb, st));
  GemmArgs g = gargs(m, n, k, nullptr, 0, nullptr, 0, C, ldc);
  g.Cin = Cin;
  g.ldcin = ldcin;
  CK(crt_gemm(Cin ? EPI_ADD : EPI_STORE, ra, ta, rb, tb, opa, bits, g, scr, st));
  return SR_OK;
}

int sr_ozaki_zgemm_dd(int opa, int m, int n, int k, const void* A_hi, const void* A_lo, int lda,
                      const void* B_hi, const void* B_lo, int ldb, const void* Cin_hi,
                      const void* Cin_lo, int ldcin, void* C_hi, void* C_lo, int ldc,
                      int slices_a, int slices_b, int dmax, void* ws, size_t ws_bytes,
                      void* stream) {
  if (m < 0 || n < 0 || k < 0 || (opa != 0 && opa != 1) || !C_hi || !C_lo) return SR_EINVAL;
  if (slices_a < 1 || slices_b < 1 || slices_a > 32 || slices_b > 32 || dmax < 2) return SR_EINVAL;
  if (m == 0 || n == 0) return SR_OK;
  if (k > 0 && (!A_hi || !B_hi)) return SR_EINVAL;
  if (lda < (opa ? (k > 1 ? k : 1) : (m > 1 ? m : 1)) || ldb < (k > 1 ? k : 1) || ldc < m) return SR_EINVAL;
  if (Cin_hi && ldcin < m) return SR_EINVAL;
  if (Cin_hi && !Cin_lo && ldcin != ldc) return SR_EINVAL;
  if (!ws || ws_bytes < sr_ozaki_ws_bytes(m, n, k, slices_a, slices_b)) return SR_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  int8_t* qa = (int8_t*)ws;
  int8_t* qb = qa + align256(oz_slice_bytes(m, k, slices_a));
  int* ea = (int*)(qb + align256(oz_slice_bytes(n, k, slices_b)));
  int* eb = ea + m;
  void* scr = (int8_t*)ea + align256((size_t)(m + n) * sizeof(int));
  if (opa == 0) CK(oz_split_rows((const zc*)A_hi, (const zc*)A_lo, lda, m, k, slices_a, qa, ea, st));
  else CK(oz_split_cols((const zc*)A_hi, (const zc*)A_lo, lda, k, m, slices_a, qa, ea, st));
  CK(oz_split_cols((const zc*)B_hi, (const zc*)B_lo, ldb, k, n, slices_b, qb, eb, st));
  GemmArgs g = gargs(m, n, k, nullptr, 0, nullptr, 0, C_hi, ldc);
  g.Clo = C_lo;
  const zc* zero_lo = nullptr;
  if (Cin_hi) {
    g.Cin = Cin_hi;
    g.ldcin = ldcin;
    if (!Cin_lo) {
      // a zero low part: C_lo itself, cleared (each element is read before the
      // same thread overwrites it)
      CK(fill_zero(C_lo, (size_t)ldc * n * sizeof(zc), st));
      zero_lo = (const zc*)C_lo;
    }
    g.Cinlo = Cin_lo ? Cin_lo : zero_lo;
  }
  CK(oz_gemm(Cin_hi ? EPI_ADD : EPI_STORE, qa, ea, slices_a, qb, eb, slices_b, opa, dmax, g, scr, st,
             true));
  return SR_OK;
}

int sr_ozaki_cgemm(int m, int n, int k, const void* A, int lda, const void* B, int ldb, void* C, int ldc,
                   int slices, int herm, void* ws, size_t ws_bytes, void* stream) {
  if (m < 1 || n < 1 || k < 1 || !A || !B || !C || slices < 1 || slices > kLpMaxDigits) return SR_EINVAL;
  if (herm < -1 || herm > 1 || (herm && m != n)) return SR_EINVAL;
  if (lda < m || ldb < k || ldc < m || !oz_allpairs_ok(m, n, k, slices)) return SR_EINVAL;
  if (!ws || ws_bytes < sr_ozaki_ws_bytes(m, n, k, slices, slices)) return SR_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  int8_t* qa = (int8_t*)ws;
  int8_t* qb = qa + align256(oz_slice_bytes(m, k, slices));
  int* ea = (int*)(qb + align256(oz_slice_bytes(n, k, slices)));
  int* eb = ea + m;
  void* scr = (int8_t*)ea + align256((size_t)(m + n) * sizeof(int));
  CK(oz_split_rows_c64((const cc*)A, lda, m, k, slices, qa, ea, st));
  CK(oz_split_cols_c64((const cc*)B, ldb, k, n, slices, qb, eb, st));
  GemmArgs g = gargs(m, n, k, nullptr, 0, nullptr, 0, C, ldc);
  g.c64 = 1;
  g.herm = herm;
  CK(oz_gemm(EPI_STORE, qa, ea, slices, qb, eb, slices, 0, slices + 1, g, scr, st));
  return SR_OK;
}

int sr_ozaki_zgemm_td(int opa, int m, int n, int k, const void* const* A, int lda, const void* const* B,
                      int ldb, const void* const* Cin, int ldcin, void* const* C, int ldc, int slices,
                      void* ws, size_t ws_bytes, void* stream) {
  if (m < 0 || n < 0 || k < 1 || (opa != 0 && opa != 1) || !C || !C[0] || !C[1] || !C[2]) return SR_EINVAL;
  if (slices < 1 || slices > 32) return SR_EINVAL;
  if (m == 0 || n == 0) return SR_OK;
  if (!A || !B || !A[0] || !A[1] || !A[2] || !B[0] || !B[1] || !B[2]) return SR_EINVAL;
  if (lda < (opa ? (k > 1 ? k : 1) : (m > 1 ? m : 1)) || ldb < (k > 1 ? k : 1) || ldc < m) return SR_EINVAL;
  if (Cin && (!Cin[0] || !Cin[1] || !Cin[2] || ldcin < m)) return SR_EINVAL;
  if (!oz_td_ok(m, n, k, slices)) return SR_EINVAL;
  if (!ws || ws_bytes < sr_ozaki_ws_bytes(m, n, k, slices, slices)) return SR_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  int8_t* qa = (int8_t*)ws;
  int8_t* qb = qa + align256(oz_slice_bytes(m, k, slices));
  int* ea = (int*)(qb + align256(oz_slice_bytes(n, k, slices)));
  int* eb = ea + m;
  void* scr = (int8_t*)ea + align256((size_t)(m + n) * sizeof(int));
  const zc* a[3] = {(const zc*)A[0], (const zc*)A[1], (const zc*)A[2]};
  const zc* b[3] = {(const zc*)B[0], (const zc*)B[1], (const zc*)B[2]};
  if (opa == 0) CK(oz_split_rows3(a[0], a[1], a[2], lda, m, k, slices, qa, ea, st));
  else CK(oz_split_cols3(a[0], a[1], a[2], lda, k, m, slices, qa, ea, st));
  CK(oz_split_cols3(b[0], b[1], b[2], ldb, k, n, slices, qb, eb, st));
  GemmArgs g = gargs(m, n, k, nullptr, 0, nullptr, 0, C[0], ldc);
  g.Cmid = C[1];
  g.Clo = C[2];
  if (Cin) {
    g.Cin = Cin[0];
    g.Cinmid = Cin[1];
    g.Cinlo = Cin[2];
    g.ldcin = ldcin;
  }
  CK(oz_gemm(Cin ? EPI_ADD : EPI_STORE, qa, ea, slices, qb, eb, slices, opa, slices + 1, g, scr, st, true));
  return SR_OK;
}

int sr_cgemm(int m, int n, int k, const void* A, int lda, const void* B, int ldb, void* C, int ldc,
             void* stream) {
  if (m < 0 || n < 0 || k < 0 || !C) return SR_EINVAL;
  if (m == 0 || n == 0) return SR_OK;
  if (k > 0 && (!A || !B)) return SR_EINVAL;
  if (lda < (m > 1 ? m : 1) || ldb < (k > 1 ? k : 1) || ldc < m) return SR_EINVAL;
  CK(cgemm(gargs(m, n, k, A, lda, B, ldb, C, ldc), (hipStream_t)stream));
  return SR_OK;
}

int sr_residual(const void* A, const void* Q, int n, void* T, void* T_lp, void* E_lp, double* eps,
                int compensated, void* ws, void* stream) {
  if (!A || !Q || !T || !T_lp || !E_lp || !ws || n < 1) return SR_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  Work w = carve(ws, n);
  w.Tlp = (cc*)T_lp;
  w.Elp = (cc*)E_lp;
  int rc = residual((const zc*)A, (const zc*)Q, nullptr, (zc*)T, n, compensated ? 1 : 0, w, st);
  if (rc != SR_OK) return rc;
  if (eps) {
    CK(fro2_partials((const zc*)A, (long)n * n, w.partials, 1024, st));
    CK(reduce_partials(w.partials, 1024, w.scal, st));
    double s[2];
    unsigned d;
    if ((rc = read_back(st, w, 2, s, &d)) != SR_OK) return rc;
    *eps = sqrt(s[1]) / sqrt(s[0]);
  }
  return SR_OK;
}

int sr_trisolve(const void* T_lp, const void* E_lp, void* L_lp, int n, float trunc, void* ws,
                void* stream) {
  if (!T_lp || !E_lp || !L_lp || !ws || n < 1) return SR_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  Work w = carve(ws, n);
  CK(fill_zero(w.status, 256, st));
  CK(trisolve((const cc*)T_lp, (const cc*)E_lp, (cc*)L_lp, n, trunc, w.tri, w.status, st));
  double s[1];
  unsigned d = 0;
  int rc = read_back(st, w, 1, s, &d);
  if (rc != SR_OK) return rc;
  return (d & DEV_BREAKDOWN) ? SR_BREAKDOWN : SR_OK;
}

size_t sr_reorder_ws_bytes(int n) {
  if (n < 1) return 0;
  return 2 * align256((size_t)n * n * sizeof(zc)) + align256(reorder_scratch_bytes(n));
}

size_t sr_trisolve_rec_ws_bytes(int n, int leaf_rows) {
  if (n < 1) return 0;
  const int lt = ((leaf_rows > 0 ? leaf_rows : 64) + 15) / 16;
  return align256(trisolve_rec_ws_bytes(n, lt)) + 256;
}

int sr_trisolve_rec(const void* T_lp, const void* E_lp, void* L_lp, int n, int leaf_rows, float trunc, void* ws,
                    size_t ws_bytes, void* stream) {
  if (!T_lp || !E_lp || !L_lp || !ws || n < 1 || leaf_rows < 0 || !(trunc >= 0)) return SR_EINVAL;
  if (ws_bytes < sr_trisolve_rec_ws_bytes(n, leaf_rows)) return SR_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  const int lt = ((leaf_rows > 0 ? leaf_rows : 64) + 15) / 16;
  unsigned* status = (unsigned*)((char*)ws + align256(trisolve_rec_ws_bytes(n, lt)));
  CK(fill_zero(status, sizeof(unsigned), st));
  CK(trisolve_rec((const cc*)T_lp, (const cc*)E_lp, (cc*)L_lp, n, lt, trunc, ws, status, st));
  unsigned d = 0;
  CK(hipMemcpyAsync(&d, status, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  return (d & DEV_BREAKDOWN) ? SR_BREAKDOWN : SR_OK;
}

int sr_reorder_start(const void* A, void* Q, int n, double theta, int* perm, void* ws, size_t ws_bytes,
                     void* stream) {
  if (!A || !Q || !ws || n < 1 || !isfinite(theta) || ws_bytes < sr_reorder_ws_bytes(n)) return SR_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const size_t z = align256((size_t)n * n * sizeof(zc));
  zc* P = (zc*)ws;
  zc* T = (zc*)((char*)ws + z);
  void* scratch = (char*)ws + 2 * z;
  // T = Q^H (A Q) in FP64
  CK(zgemm(0, EPI_STORE, 0, gargs(n, n, n, A, n, Q, n, P, n), st));
  CK(zgemm(1, EPI_STORE, 0, gargs(n, n, n, Q, n, P, n, T, n), st));
  CK(reorder_swaps(T, (zc*)Q, n, theta, scratch, perm, st));
  return SR_OK;
}

int sr_trisolve64(const void* T, const void* E, void* L, int n, void* ws, void* stream) {
  if (!T || !E || !L || !ws || n < 1) return SR_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  Work w = carve(ws, n);
  CK(fill_zero(w.status, 256, st));
  CK(trisolve64((const zc*)T, (const zc*)E, (zc*)L, n, w.tri, w.status, st));
  double s[1];
  unsigned d = 0;
  int rc = read_back(st, w, 1, s, &d);
  if (rc != SR_OK) return rc;
  return (d & DEV_BREAKDOWN) ? SR_BREAKDOWN : SR_OK;
}

int sr_update(const void* Q, const void* L_lp, void* Q_out, int n, int gate, int compensated,
              double* norms, void* ws, void* stream) {
  if (!Q || !L_lp || !Q_out || !ws || n < 1 || Q == Q_out) return SR_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  Work w = carve(ws, n);
  CK(hipMemcpyAsync(w.Llp, L_lp, (size_t)n * n * sizeof(cc), hipMemcpyDeviceToDevice, st));
  int rc = defects((const zc*)Q, nullptr, n, compensated ? 1 : 0, w, st);
  if (rc != SR_OK) return rc;
  double nrm[4] = {0, 0, 0, 0};
  Gate gt = gate_terms(false, 0, 0);
  if (gate || norms) {
    unsigned d;
    if ((rc = read_back(st, w, 4, nrm, &d)) != SR_OK) return rc;
    if (gate) gt = gate_terms(true, sqrt(nrm[3]), sqrt(nrm[2]));
    if (norms) {
      norms[0] = sqrt(nrm[3]);
      norms[1] = sqrt(nrm[2]);
    }
  }
  return apply_update((const zc*)Q, (zc*)Q_out, nullptr, n, gt, w, st, nullptr);
}

int sr_ns_init(const void* Qh, void* Q, int n, int compensated, void* ws, void* stream) {
  if (!Qh || !Q || !ws || n < 1 || Qh == Q) return SR_EINVAL;
  Work w = carve(ws, n);
  return ns_init((const zc*)Qh, (zc*)Q, nullptr, n, compensated ? 1 : 0, w, (hipStream_t)stream);
}

}  // extern "C"

namespace {
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
// One MFMA with the operand layout the GEMM kernels use; D is written in the
// row-major order the lane/element layout implies for the given instruction.
__global__ void diag_mfma_kernel(int kind, const double* A, const double* B, double* D) {
  const int l = threadIdx.x;
  const double a = A[(l % 16) * 4 + l / 16];
  const double b = B[(l / 16) * 16 + l % 16];
  if (kind == 0) {
    d4v c = {0, 0, 0, 0};
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    for (int v = 0; v < 4; v++) D[((l / 16) + 4 * v) * 16 + l % 16] = c[v];
  } else {
    f4v c = {0, 0, 0, 0};
    c = __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, c, 0, 0, 0);
    for (int v = 0; v < 4; v++) D[(4 * (l / 16) + v) * 16 + l % 16] = (double)c[v];
  }
}
}  // namespace

extern "C" int sr_diag_mfma(int kind, const double* A, const double* B, double* D) {
  if (!A || !B || !D || (kind != 0 && kind != 1)) return SR_EINVAL;
  double* d = nullptr;
  CK(hipMalloc(&d, sizeof(double) * (64 + 64 + 256)));
  CK(hipMemcpy(d, A, sizeof(double) * 64, hipMemcpyHostToDevice));
  CK(hipMemcpy(d + 64, B, sizeof(double) * 64, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(diag_mfma_kernel, dim3(1), dim3(64), 0, 0, kind, d, d + 64, d + 128);
  CK(hipGetLastError());
  CK(hipMemcpy(D, d + 128, sizeof(double) * 256, hipMemcpyDeviceToHost));
  CK(hipFree(d));
  return SR_OK;
}
