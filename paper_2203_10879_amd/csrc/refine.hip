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

#include <mutex>
#include <vector>

#include "../../include/schur_refine.h"
#include "kernels.hpp"

using namespace sr;

namespace {

constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

int partial_slots(int n) {
  int a = gemm_tiles(n, n), b = form_w_parts(n);
  int m = a > b ? a : b;
  return m > 1024 ? m : 1024;
}

struct Work {
  zc *Qa, *QH, *P, *Y;
  cc *Tlp, *Elp, *Llp, *W, *W2, *W3, *YW, *Ylp;
  double* partials;
  double* scal;
  unsigned* status;
  void* tri;
  size_t bytes;
};

Work carve(void* base, int n) {
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
  w.tri = take(align256(trisolve_ws_bytes(n)));
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
// category 0 = hp products, 1 = triangular solves.
struct Timer {
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> ev[2];
  int count[2] = {0, 0};
  void mark(int c) {
    hipEvent_t e;
    if (hipEventCreate(&e) == hipSuccess) {
      hipEventRecord(e, st);
      ev[c].push_back(e);
    }
  }
  float total(int c) const {  // after the stream has been synchronised
    float s = 0;
    for (size_t i = 0; i + 1 < ev[c].size(); i += 2) {
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
#define TOC(tm, c)        \
  if (tm) {               \
    (tm)->mark(c);        \
    (tm)->count[c]++;     \
  }

// Newton-Schulz start into Qout: Y0 = Qh^H Qh - I, Qout = Qh + Qh (-Y0/2);
// QHout (may be NULL) receives Qout^H.
int ns_init(const zc* Qh, zc* Qout, zc* QHout, int n, int comp, const Work& w, hipStream_t st,
            Timer* tm = nullptr) {
  GemmArgs g = gargs(n, n, n, Qh, n, Qh, n, w.Y, n);
  g.partials = w.partials;
  TIC(tm, 0);
  CK(zgemm(1, EPI_YDEF, comp, g, st));
  TOC(tm, 0);
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
int residual(const zc* A, const zc* Q, const zc* QH, zc* T, int n, int comp, const Work& w,
             hipStream_t st, Timer* tm = nullptr) {
  GemmArgs g = gargs(n, n, n, A, n, Q, n, w.P, n);
  TIC(tm, 0);
  CK(zgemm(0, EPI_STORE, comp, g, st));
  TOC(tm, 0);
  GemmArgs s = gargs(n, n, n, QH ? QH : Q, n, w.P, n, T, n);
  s.Tlp = w.Tlp;
  s.Elp = w.Elp;
  s.ldlp = n;
  s.partials = w.partials;
  TIC(tm, 0);
  CK(zgemm(QH ? 0 : 1, EPI_SPLIT, comp, s, st));
  TOC(tm, 0);
  CK(reduce_partials(w.partials, gemm_tiles(n, n), w.scal + 1, st));
  return SR_OK;
}

// Y = Q^H Q - I (scal[2] = ||Y||^2), W = L - L^H (scal[3] = ||W||^2).
int defects(const zc* Q, const zc* QH, int n, int comp, const Work& w, hipStream_t st,
            Timer* tm = nullptr) {
  GemmArgs g = gargs(n, n, n, QH ? QH : Q, n, Q, n, w.Y, n);
  g.partials = w.partials;
  TIC(tm, 0);
  CK(zgemm(QH ? 0 : 1, EPI_YDEF, comp, g, st));
  TOC(tm, 0);
  CK(reduce_partials(w.partials, gemm_tiles(n, n), w.scal + 2, st));
  CK(form_w(w.Llp, w.W, n, w.partials, st));
  CK(reduce_partials(w.partials, form_w_parts(n), w.scal + 3, st));
  return SR_OK;
}

struct Gate {
  bool w2, w3, yw;
};

// lp products, Delta, and Qout = Q + Q Delta (QHout, if given, receives Qout^H).
int apply_update(const zc* Q, zc* Qout, zc* QHout, int n, Gate gt, const Work& w, hipStream_t st,
                 int* nprod, Timer* tm = nullptr) {
  int np = 0;
  if (gt.w2 || gt.w3) {
    CK(cgemm(gargs(n, n, n, w.W, n, w.W, n, w.W2, n), st));
    np++;
  }
  if (gt.w3) {
    CK(cgemm(gargs(n, n, n, w.W2, n, w.W, n, w.W3, n), st));
    np++;
  }
  if (gt.yw) {
    CK(to_c64(w.Y, w.Ylp, (long)n * n, st));
    CK(cgemm(gargs(n, n, n, w.Ylp, n, w.W, n, w.YW, n), st));
    np++;
  }
  CK(form_delta(w.Llp, w.Y, gt.w2 ? w.W2 : nullptr, gt.w3 ? w.W3 : nullptr,
                gt.yw ? w.YW : nullptr, w.P, n, st));
  GemmArgs u = gargs(n, n, n, Q, n, w.P, n, Qout, n);
  u.Cin = Q;
  u.ldcin = n;
  u.CH = QHout;
  u.ldch = n;
  TIC(tm, 0);
  CK(zgemm(0, EPI_ADD, 0, u, st));
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
  (void)opts;
  if (n < 1) return 0;
  return carve(nullptr, n).bytes + 256;
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

int schur_refine(const void* A_, void* Q_, void* T_, int n, int iters, double tol,
                 const sr_opts* opts_in, sr_info* info) {
  info_init(info);
  if (!A_ || !Q_ || !T_ || n < 1 || iters < 1 || !(tol > 0)) {
    if (info) info->status = SR_EINVAL;
    return SR_EINVAL;
  }
  sr_opts o;
  if (opts_in) o = *opts_in;
  else sr_default_opts(&o);
  if (o.gemm != SR_GEMM_FP64) {
    if (info) info->status = SR_ENOSYS;
    return SR_ENOSYS;
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
  const Work w = carve(base, n);
  const int comp = o.compensated ? 1 : 0;

  Timer timer;
  timer.st = st;
  Timer* tm = o.timing ? &timer : nullptr;
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  CK(hipEventRecord(e0, st));
  CK(fill_zero(w.status, 256, st));
  CK(fro2_partials(A, (long)n * n, w.partials, 1024, st));
  CK(reduce_partials(w.partials, 1024, w.scal, st));

  int status = SR_NOT_CONVERGED;
  int passes = 0, updates = 0, nprod = 0;
  double eps = 0, eps1 = -1, eps2 = -1, orth = 0;
  zc* cur = w.Qa;
  zc* other = Q;
  if ((rc = ns_init(Q, w.Qa, w.QH, n, comp, w, st, tm)) != SR_OK) return rc;

  for (int p = 0; p < iters; p++) {
    if ((rc = residual(A, cur, w.QH, T, n, comp, w, st, tm)) != SR_OK) return rc;
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
    if (eps <= tol) {
      status = SR_OK;
      break;
    }
    if (eps2 >= 0 && eps > eps1 && eps1 > eps2) {
      status = SR_DIVERGED;
      break;
    }
    if (eps1 >= 0 && eps > 0.5 * eps1 && eps < 100.0 * kU64 * sqrt((double)n)) {
      status = SR_STAGNATED;
      break;
    }
    eps2 = eps1;
    eps1 = eps;
    if (p == iters - 1) break;

    TIC(tm, 1);
    CK(trisolve(w.Tlp, w.Elp, w.Llp, n, o.trunc ? 1e-5f : 0.f, w.tri, w.status, st));
    TOC(tm, 1);
    if ((rc = defects(cur, w.QH, n, comp, w, st, tm)) != SR_OK) return rc;
    double nrm[4];
    if ((rc = read_back(st, w, 4, nrm, &dst)) != SR_OK) return rc;
    if (dst & DEV_BREAKDOWN) {
      status = SR_BREAKDOWN;
      break;
    }
    const double ny = sqrt(nrm[2]), nw = sqrt(nrm[3]);
    orth = ny;
    if (info && updates < 16) info->norm_w_hist[updates] = nw;
    if (!isfinite(ny) || !isfinite(nw)) {
      status = SR_BREAKDOWN;
      break;
    }
    const Gate gt = gate_terms(o.gate_lp_terms != 0, nw, ny);
    if ((rc = apply_update(cur, other, w.QH, n, gt, w, st, &nprod, tm)) != SR_OK) return rc;
    zc* t = cur;
    cur = other;
    other = t;
    updates++;
  }
  if (cur != Q) CK(hipMemcpyAsync(Q, cur, (size_t)n * n * sizeof(zc), hipMemcpyDeviceToDevice, st));
  CK(hipEventRecord(e1, st));
  CK(hipEventSynchronize(e1));
  float ms = 0;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
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
      info->ms_solve = timer.total(1);
    }
  }
  return status;
}

int schur_refine_batched(int batch, const int* n, const void* const* A, void* const* Q,
                         void* const* T, int iters, double tol, const sr_opts* opts,
                         sr_info* info) {
  if (batch < 0 || (batch > 0 && (!n || !A || !Q || !T))) return SR_EINVAL;
  int worst = SR_OK;
  for (int b = 0; b < batch; b++) {
    const int r = schur_refine(A[b], Q[b], T[b], n[b], iters, tol, opts, info ? info + b : nullptr);
    if (r < 0) return r;
    if (r > worst) worst = r;
  }
  return worst;
}

int schur_refine_dd(const void*, const void*, void*, void*, void*, void*, int, int, double,
                    const sr_opts*, sr_info* info) {
  info_init(info);
  if (info) info->status = SR_ENOSYS;
  return SR_ENOSYS;
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
         align256((size_t)(m + n) * sizeof(int));
}

// Largest slice-pair count on one diagonal times k must keep int32 sums exact.
static bool oz_exact_ok(int k, int sa, int sb) {
  const long pairs = sa < sb ? sa : sb;
  const long kp = (k + 63) / 64 * 64;
  return pairs * kp * 127L * 127L < 2147483647L;
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
  if (!oz_exact_ok(k, slices_a, slices_b)) return SR_EINVAL;
  if (!ws || ws_bytes < sr_ozaki_ws_bytes(m, n, k, slices_a, slices_b)) return SR_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  int8_t* qa = (int8_t*)ws;
  int8_t* qb = qa + align256(oz_slice_bytes(m, k, slices_a));
  int* ea = (int*)(qb + align256(oz_slice_bytes(n, k, slices_b)));
  int* eb = ea + m;
  if (opa == 0) CK(oz_split_rows((const zc*)A, nullptr, lda, m, k, slices_a, qa, ea, st));
  else CK(oz_split_cols((const zc*)A, nullptr, lda, k, m, slices_a, qa, ea, st));
  CK(oz_split_cols((const zc*)B, nullptr, ldb, k, n, slices_b, qb, eb, st));
  GemmArgs g = gargs(m, n, k, nullptr, 0, nullptr, 0, C, ldc);
  g.Cin = Cin;
  g.ldcin = ldcin;
  CK(oz_gemm(Cin ? EPI_ADD : EPI_STORE, qa, ea, slices_a, qb, eb, slices_b, opa, dmax, g, st));
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
