// Batched refinement: many independent matrices of uneven size (Algorithm 4 run
// on each), driven as one fixed sequence of grouped launches per pass.
//
// Every step of a pass is one launch over the whole batch:
//   grouped products  P = A Q, That = Q^H P (split), Y = Q^H Q - I, the lp
//                     products and Q + Q Delta: a persistent grid walks a table of
//                     output tiles of all matrices (tile edge 64 or 32, chosen per
//                     size bucket by the autotuner below);
//   per-matrix blocks the residual test, W = L - L^H with its norm, the gates of the
//                     lp terms and Delta: one block per matrix;
//   solve             the FP32 triangular solve by tile diagonal across the batch (one
//                     launch per step, one block per tile), or one block per matrix
//                     when no matrix has more than two 16-wide tile rows.
// Loop control stays on the device: each matrix has a state record (its residual
// history and outcome) and an `active` flag that the grouped launches and blocks
// test, so matrices that have finished cost one early exit per launch. The
// sequence of two passes (the iterate alternates between two buffers) is captured
// once in a HIP graph and replayed until no matrix is active or the pass limit is
// reached; the host reads one counter per replay.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/schur_refine.h"
#include "kernels.hpp"

namespace sr {
namespace {

constexpr double kU64b = 1.1102230246251565e-16;
constexpr int BNT = 256;  // threads of the per-matrix blocks

// Per-matrix device record.
struct BMat {
  int n;
  const zc* A;
  zc* Q;  // caller's Q (start; final iterate)
  zc* T;  // caller's T
  zc *Qa, *QH, *P, *Y;
  cc *Tlp, *Elp, *L, *W, *W2, *W3, *YW, *Ylp;
  int slot0, nslots;  // partial-sum slots of its product tiles
};

// Per-matrix loop state (device).
struct BState {
  int status;  // -1 while iterating, else the sr_status
  int passes, updates, lp_products;
  int cur;     // 1: the iterate is in Qa, 0: in Q
  int gate_w2, gate_w3, gate_yw;
  unsigned flag;  // solve status bits
  double norm_a2, eps, eps1, eps2, orth;
  double resid_hist[16], norm_w_hist[16];
};

__device__ inline double block_sum_b(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int w = 0; w < BNT / 64; w++) s += red[w];
  __syncthreads();
  return s;
}

// ||A||_F^2, initial state; n = 1 is finished here (T = A, Q = q / |q|).
__global__ __launch_bounds__(BNT) void b_init_kernel(const BMat* __restrict__ mats, BState* __restrict__ st,
                                                     int* __restrict__ active) {
  __shared__ double red[BNT / 64];
  const BMat m = mats[blockIdx.x];
  const long nn = (long)m.n * m.n;
  double s = 0;
  for (long i = threadIdx.x; i < nn; i += BNT) s += m.A[i].re * m.A[i].re + m.A[i].im * m.A[i].im;
  s = block_sum_b(s, red);
  if (threadIdx.x == 0) {
    BState z;
    memset(&z, 0, sizeof(z));
    z.status = -1;
    z.cur = 1;
    z.norm_a2 = s;
    z.eps1 = z.eps2 = -1;
    if (m.n == 1) {
      const zc q = m.Q[0];
      const double a = hypot(q.re, q.im);
      if (!(a > 0) || !isfinite(m.A[0].re) || !isfinite(m.A[0].im)) {
        z.status = SR_BREAKDOWN;
      } else {
        m.Q[0] = mk<double>(q.re / a, q.im / a);
        m.T[0] = m.A[0];
        z.status = SR_OK;
        z.passes = 1;
      }
      z.cur = 0;
    }
    st[blockIdx.x] = z;
    active[blockIdx.x] = z.status == -1 ? 1 : 0;
  }
}

// Delta0 = -Y0/2 into P (the Newton-Schulz start's correction).
__global__ __launch_bounds__(BNT) void b_ns_delta_kernel(const BMat* __restrict__ mats,
                                                         const int* __restrict__ active) {
  if (!active[blockIdx.x]) return;
  const BMat m = mats[blockIdx.x];
  const long nn = (long)m.n * m.n;
  for (long i = threadIdx.x; i < nn; i += BNT) {
    const zc y = m.Y[i];
    m.P[i] = mk<double>(-0.5 * y.re, -0.5 * y.im);
  }
}

// Residual test of a pass (mirrors the single-matrix driver).
__global__ __launch_bounds__(BNT) void b_decide_kernel(const BMat* __restrict__ mats, BState* __restrict__ st,
                                                       int* __restrict__ active, const double* __restrict__ partials,
                                                       int iters, double tol, int* __restrict__ n_active) {
  __shared__ double red[BNT / 64];
  if (!active[blockIdx.x]) return;
  const BMat m = mats[blockIdx.x];
  double s = 0;
  for (int i = threadIdx.x; i < m.nslots; i += BNT) s += partials[m.slot0 + i];
  s = block_sum_b(s, red);
  if (threadIdx.x != 0) return;
  BState& z = st[blockIdx.x];
  const double eps = sqrt(s) / sqrt(z.norm_a2);
  const int p = z.passes;
  z.passes = p + 1;
  z.eps = eps;
  if (p < 16) z.resid_hist[p] = eps;
  int status = -1;
  if (!isfinite(eps)) status = SR_BREAKDOWN;
  else if (eps <= tol) status = SR_OK;
  else if (z.eps2 >= 0 && eps > z.eps1 && z.eps1 > z.eps2) status = SR_DIVERGED;
  else if (z.eps1 >= 0 && eps > 0.5 * z.eps1 && eps < 100.0 * kU64b * sqrt((double)m.n)) status = SR_STAGNATED;
  else {
    z.eps2 = z.eps1;
    z.eps1 = eps;
    if (p + 1 >= iters) status = SR_NOT_CONVERGED;
  }
  if (status >= 0) {
    z.status = status;
    active[blockIdx.x] = 0;
  } else {
    atomicAdd(n_active, 1);
  }
}

// After the solve and Y: ||Y||, W = L - L^H and ||W||, the gates of the lp terms
// (0.1 u_hp, as the single-matrix driver), Y in FP32 when YW is needed.
__global__ __launch_bounds__(BNT) void b_post_kernel(const BMat* __restrict__ mats, BState* __restrict__ st,
                                                     int* __restrict__ active, const double* __restrict__ partials,
                                                     int gate, int* __restrict__ act_w2, int* __restrict__ act_w3,
                                                     int* __restrict__ act_yw) {
  __shared__ double red[BNT / 64];
  __shared__ int go;
  const int b = blockIdx.x;
  if (!active[b]) {
    if (threadIdx.x == 0) act_w2[b] = act_w3[b] = act_yw[b] = 0;
    return;
  }
  const BMat m = mats[b];
  const int n = m.n;
  double sy = 0;
  for (int i = threadIdx.x; i < m.nslots; i += BNT) sy += partials[m.slot0 + i];
  sy = block_sum_b(sy, red);
  double sw = 0;
  const long nn = (long)n * n;
  for (long o = threadIdx.x; o < nn; o += BNT) {
    const int i = (int)(o % n), j = (int)(o / n);
    cc w = mk<float>(0.f, 0.f);
    if (i > j) {
      w = m.L[o];
    } else if (i < j) {
      const cc u = m.L[j + (long)i * n];
      w = mk<float>(-u.re, u.im);
    }
    m.W[o] = w;
    sw += (double)w.re * w.re + (double)w.im * w.im;
  }
  sw = block_sum_b(sw, red);
  if (threadIdx.x == 0) {
    BState& z = st[b];
    const double ny = sqrt(sy), nw = sqrt(sw);
    z.orth = ny;
    if (z.updates < 16) z.norm_w_hist[z.updates] = nw;
    int ok = 1;
    if ((z.flag & DEV_BREAKDOWN) || !isfinite(ny) || !isfinite(nw)) {
      z.status = SR_BREAKDOWN;
      active[b] = 0;
      ok = 0;
    }
    const double thr = 0.1 * kU64b;
    const int g2 = ok && (!gate || nw * nw > thr);
    const int g3 = ok && (!gate || nw * nw * nw > thr);
    const int gy = ok && (!gate || ny * nw > thr);
    z.gate_w2 = g2;
    z.gate_w3 = g3;
    z.gate_yw = gy;
    z.lp_products += (g2 || g3) + g3 + gy;
    act_w2[b] = g2 || g3;
    act_w3[b] = g3;
    act_yw[b] = gy;
    go = gy;
  }
  __syncthreads();
  if (go)
    for (long o = threadIdx.x; o < nn; o += BNT) m.Ylp[o] = mk<float>((float)m.Y[o].re, (float)m.Y[o].im);
}

// Delta = W - Y/2 + (W2 + W3 - YW)/2 (gated terms only) into P.
__global__ __launch_bounds__(BNT) void b_delta_kernel(const BMat* __restrict__ mats, const BState* __restrict__ st,
                                                      const int* __restrict__ active) {
  const int b = blockIdx.x;
  if (!active[b]) return;
  const BMat m = mats[b];
  const int g2 = st[b].gate_w2, g3 = st[b].gate_w3, gy = st[b].gate_yw;
  const long nn = (long)m.n * m.n;
  for (long o = threadIdx.x; o < nn; o += BNT) {
    const cc w = m.W[o];
    const zc y = m.Y[o];
    double pr = 0, pi = 0;
    if (g2) {
      pr += m.W2[o].re;
      pi += m.W2[o].im;
    }
    if (g3) {
      pr += m.W3[o].re;
      pi += m.W3[o].im;
    }
    if (gy) {
      pr -= m.YW[o].re;
      pi -= m.YW[o].im;
    }
    m.P[o] = mk<double>((double)w.re - 0.5 * y.re + 0.5 * pr, (double)w.im - 0.5 * y.im + 0.5 * pi);
  }
}

// The update of an active matrix moves its iterate to the other buffer.
__global__ void b_flip_kernel(BState* __restrict__ st, const int* __restrict__ active, int count) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < count && active[b]) {
    st[b].cur ^= 1;
    st[b].updates++;
  }
}

// Clear the per-pass counter and the solve flags (fill kernels, so that the
// sequence can be captured).
__global__ void b_pass_start_kernel(BState* __restrict__ st, int count, int* __restrict__ n_active) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b == 0) *n_active = 0;
  if (b < count) st[b].flag = 0;
}

// Final iterate into the caller's Q.
__global__ __launch_bounds__(BNT) void b_finish_kernel(const BMat* __restrict__ mats,
                                                       const BState* __restrict__ st) {
  const BMat m = mats[blockIdx.x];
  if (st[blockIdx.x].cur != 1 || m.n < 2) return;
  const long nn = (long)m.n * m.n;
  for (long i = threadIdx.x; i < nn; i += BNT) m.Q[i] = m.Qa[i];
}

// ----------------------------------------------------------------- host side

size_t a256(size_t b) { return (b + 255) / 256 * 256; }

// Size buckets of the autotuner.
int bucket_of(int n) {
  if (n <= 32) return 0;
  if (n <= 64) return 1;
  if (n <= 128) return 2;
  if (n <= 192) return 3;
  if (n <= 256) return 4;
  return 5;
}

// A tuned configuration of a bucket's products: tile edge and persistent blocks per CU.
struct TuneChoice {
  int edge = 64, bpc = 4;
  float ms = 0;  // the timed grouped product (0: loaded from a file)
};
struct Tuner {
  std::mutex mu;
  std::map<int, TuneChoice> bm;  // bucket -> choice
  int runs = 0;                  // buckets timed in this process
  bool env_loaded = false;       // SR_TUNING_FILE read
};
Tuner& tuner() {
  static Tuner t;
  return t;
}

// The device a tuning file entry belongs to: architecture name and CU count.
std::string device_key() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return std::string();
  std::string a = p.gcnArchName;
  for (char& c : a)
    if (c == ' ') c = '_';
  return a + "/" + std::to_string(p.multiProcessorCount);
}

// Tuning file: a header line, then one line per (device, bucket):
//   <device> <bucket> <edge> <blocks per CU> <ms>
constexpr const char* kTuneHeader = "schur_refine batched tuning v1";

int tuning_save_locked(const char* path) {
  const std::string dk = device_key();
  if (dk.empty()) return SR_EHIP;
  // keep the entries of other devices already in the file
  std::vector<std::string> keep;
  if (FILE* f = fopen(path, "r")) {
    char line[512];
    bool first = true;
    while (fgets(line, sizeof(line), f)) {
      if (first) {
        first = false;
        continue;
      }
      char d[256];
      if (sscanf(line, "%255s", d) == 1 && dk != d) keep.push_back(line);
    }
    fclose(f);
  }
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return SR_EINVAL;
  fprintf(f, "%s\n", kTuneHeader);
  for (const auto& l : keep) fputs(l.c_str(), f);
  for (const auto& kv : tuner().bm)
    fprintf(f, "%s %d %d %d %.4f\n", dk.c_str(), kv.first, kv.second.edge, kv.second.bpc, kv.second.ms);
  if (fclose(f) != 0 || rename(tmp.c_str(), path) != 0) return SR_EINVAL;
  return (int)tuner().bm.size();
}

int tuning_load_locked(const char* path) {
  const std::string dk = device_key();
  if (dk.empty()) return SR_EHIP;
  FILE* f = fopen(path, "r");
  if (!f) return SR_EINVAL;
  char line[512];
  int count = 0;
  if (!fgets(line, sizeof(line), f) || strncmp(line, kTuneHeader, strlen(kTuneHeader)) != 0) {
    fclose(f);
    return SR_EINVAL;
  }
  while (fgets(line, sizeof(line), f)) {
    char d[256];
    int b, e, g;
    float ms;
    if (sscanf(line, "%255s %d %d %d %f", d, &b, &e, &g, &ms) != 5) continue;
    if (dk != d || b < 0 || b > 5 || (e != 32 && e != 64) || !(g == 1 || g == 2 || g == 4 || g == 8)) continue;
    TuneChoice c;
    c.edge = e;
    c.bpc = g;
    c.ms = ms;
    tuner().bm[b] = c;
    count++;
  }
  fclose(f);
  return count;
}

// SR_TUNING_FILE: read once, before the first tuning
void tuning_env_load_locked() {
  if (tuner().env_loaded) return;
  tuner().env_loaded = true;
  if (const char* p = getenv("SR_TUNING_FILE"))
    if (*p) tuning_load_locked(p);
}

int tiles_of(int n, int bm) { return ceil_div(n, bm) * ceil_div(n, bm); }

// Workspace layout of a batch.
struct BLayout {
  std::vector<size_t> off;  // per matrix: offset of its arrays
  size_t mats, states, active, act_w2, act_w3, act_yw, counter, partials, args, tiles, tri, steps;
  size_t total;
  int nslots, ntiles64, ntiles32;
};

size_t per_matrix_bytes(int n) {
  const size_t z = a256((size_t)n * n * sizeof(zc)), c = a256((size_t)n * n * sizeof(cc));
  return 4 * z + 8 * c;
}

constexpr int kArgTables = 13;

BLayout layout(int batch, const int* n, const std::vector<int>& bm) {
  BLayout L;
  size_t p = 0;
  L.off.resize(batch);
  L.nslots = 0;
  L.ntiles64 = L.ntiles32 = 0;
  for (int b = 0; b < batch; b++) {
    L.off[b] = p;
    if (n[b] >= 2) {
      p += per_matrix_bytes(n[b]);
      const int t = tiles_of(n[b], bm[b]);
      L.nslots += t;
      if (bm[b] == 64) L.ntiles64 += t;
      else L.ntiles32 += t;
    }
  }
  auto take = [&](size_t b) {
    const size_t r = p;
    p += a256(b);
    return r;
  };
  L.mats = take(sizeof(BMat) * batch);
  L.states = take(sizeof(BState) * batch);
  L.active = take(sizeof(int) * batch);
  L.act_w2 = take(sizeof(int) * batch);
  L.act_w3 = take(sizeof(int) * batch);
  L.act_yw = take(sizeof(int) * batch);
  L.counter = take(256);
  L.partials = take(sizeof(double) * (L.nslots + 1));
  L.args = take(sizeof(GemmArgs) * batch * kArgTables);
  L.tiles = take(sizeof(GTile) * (L.ntiles64 + L.ntiles32 + 1));
  L.tri = take(trimatrix_bytes() * batch);
  L.steps = take(sizeof(TriStepTile) * (trisolve_steps_tiles(n, batch) + 1));
  L.total = p;
  return L;
}

#define BCK(expr)                          \
  do {                                     \
    hipError_t _e = (expr);                \
    if (_e != hipSuccess) return SR_EHIP;  \
  } while (0)

GemmArgs gargs_b(int n, const void* A, const void* B, void* C) {
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.m = g.n = g.k = n;
  g.A = A;
  g.lda = n;
  g.B = B;
  g.ldb = n;
  g.C = C;
  g.ldc = n;
  return g;
}

struct Launcher {
  const GemmArgs* args_dev;  // [kArgTables][batch]
  const GTile* t64;
  const GTile* t32;
  int n64, n32, batch, grid64, grid32;  // persistent grids of the two tile edges
  hipStream_t st;
  hipError_t z(int table, int opa, int epi, int comp, const int* active) const {
    const GemmArgs* a = args_dev + (size_t)table * batch;
    hipError_t e = zgemm_grouped(opa, epi, comp, 64, a, t64, n64, active, grid64, st);
    if (e != hipSuccess) return e;
    return zgemm_grouped(opa, epi, comp, 32, a, t32, n32, active, grid32, st);
  }
  hipError_t c(int table, const int* active) const {
    const GemmArgs* a = args_dev + (size_t)table * batch;
    hipError_t e = cgemm_grouped(64, a, t64, n64, active, grid64, st);
    if (e != hipSuccess) return e;
    return cgemm_grouped(32, a, t32, n32, active, grid32, st);
  }
};

// Tables: 0 NS Y0, 1 NS update, then per parity e (2 + 4e ..): P, That, Y, update;
// 10 W2, 11 W3, 12 YW.
enum { T_NSY = 0, T_NSU = 1, T_P = 2, T_T = 3, T_Y = 4, T_U = 5, T_W2 = 10, T_W3 = 11, T_YW = 12 };

// Autotuner: for a bucket seen for the first time (and not in a loaded tuning
// file), time the grouped P = A Q of (up to kTuneMax of) its matrices for both tile
// edges and persistent grids of 1, 2, 4 and 8 blocks per CU, and keep the fastest;
// among configurations within kTuneTie of it, the one with the most blocks per CU
// (the whole batch holds more tiles than the timed sample, and near-ties in the
// sample are noise). With SR_TUNING_FILE set the table is written back after each
// new tuning.
constexpr int kTuneMax = 256;
constexpr float kTuneTie = 1.03f;
int tune_bucket(int bucket, const std::vector<int>& members, const int* n, const void* const* A,
                void* const* Q, void* scratch, hipStream_t st, TuneChoice* out) {
  {
    std::lock_guard<std::mutex> lk(tuner().mu);
    tuning_env_load_locked();
    auto it = tuner().bm.find(bucket);
    if (it != tuner().bm.end()) {
      *out = it->second;
      return SR_OK;
    }
  }
  const int cnt = (int)std::min<size_t>(members.size(), kTuneMax);
  TuneChoice best;
  if (cnt > 0) {
    // scratch: outputs then tables
    std::vector<GemmArgs> args(cnt);
    uintptr_t p = (uintptr_t)scratch;
    for (int i = 0; i < cnt; i++) {
      const int b = members[i];
      args[i] = gargs_b(n[b], A[b], Q[b], (void*)p);
      p += a256((size_t)n[b] * n[b] * sizeof(zc));
    }
    GemmArgs* args_dev = (GemmArgs*)p;
    p += a256(sizeof(GemmArgs) * cnt);
    GTile* tiles_dev = (GTile*)p;
    const int edges[2] = {64, 32};
    const int bpcs[4] = {1, 2, 4, 8};
    hipEvent_t e0, e1;
    BCK(hipEventCreate(&e0));
    BCK(hipEventCreate(&e1));
    BCK(hipMemcpyAsync(args_dev, args.data(), sizeof(GemmArgs) * cnt, hipMemcpyHostToDevice, st));
    TuneChoice cand[8];
    int nc = 0;
    for (int v = 0; v < 2; v++) {
      std::vector<GTile> tl;
      for (int i = 0; i < cnt; i++) {
        const int nn = n[members[i]];
        for (int tn = 0; tn < ceil_div(nn, edges[v]); tn++)
          for (int tm = 0; tm < ceil_div(nn, edges[v]); tm++) tl.push_back({i, tm * edges[v], tn * edges[v], 0});
      }
      BCK(hipMemcpyAsync(tiles_dev, tl.data(), sizeof(GTile) * tl.size(), hipMemcpyHostToDevice, st));
      for (int gi = 0; gi < 4; gi++) {
        const int grid = (int)std::min<size_t>(tl.size(), (size_t)bpcs[gi] * kCUs);
        for (int rep = 0; rep < 3; rep++) {
          if (rep == 1) BCK(hipEventRecord(e0, st));
          BCK(zgemm_grouped(0, EPI_STORE, 1, edges[v], args_dev, tiles_dev, (int)tl.size(), nullptr, grid, st));
        }
        BCK(hipEventRecord(e1, st));
        BCK(hipEventSynchronize(e1));
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        cand[nc].edge = edges[v];
        cand[nc].bpc = bpcs[gi];
        cand[nc].ms = 0.5f * ms;
        nc++;
      }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    float fastest = cand[0].ms;
    for (int c = 1; c < nc; c++) fastest = std::min(fastest, cand[c].ms);
    bool have = false;
    for (int c = 0; c < nc; c++) {
      if (cand[c].ms > kTuneTie * fastest) continue;
      if (!have || cand[c].bpc > best.bpc || (cand[c].bpc == best.bpc && cand[c].ms < best.ms)) best = cand[c];
      have = true;
    }
  }
  std::lock_guard<std::mutex> lk(tuner().mu);
  tuner().bm[bucket] = best;
  tuner().runs++;
  if (const char* p = getenv("SR_TUNING_FILE"))
    if (*p) tuning_save_locked(p);
  *out = best;
  return SR_OK;
}

size_t tune_scratch_bytes(int batch, const int* n) {
  // kTuneMax outputs of the largest size, and the tables
  size_t mx = 0;
  for (int b = 0; b < batch; b++) mx = std::max<size_t>(mx, (size_t)n[b]);
  return kTuneMax * a256(mx * mx * sizeof(zc)) + a256(sizeof(GemmArgs) * kTuneMax) +
         a256(sizeof(GTile) * kTuneMax * (size_t)ceil_div((int)mx, 32) * ceil_div((int)mx, 32));
}

hipStream_t capture_stream() {
  static thread_local hipStream_t s = nullptr;
  if (!s) {
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
  }
  return s;
}

// Pinned host slot for the device's count of matrices still refining, made once
// per thread (the call reads it after every replay of the two-pass graph).
int* host_counter() {
  static thread_local int* h = nullptr;
  if (!h && hipHostMalloc((void**)&h, sizeof(int), hipHostMallocDefault) != hipSuccess) h = nullptr;
  return h;
}

// The instantiated two-pass graph of the last call on this thread, reused while
// everything it bakes in is unchanged: the workspace address (every kernel
// argument points into it; the per-matrix tables there are uploaded again on each
// call, so the matrices' own addresses may change), the sizes and tile edges (the
// table offsets), the persistent grids, the pass limit, tol and the options. Only calls with
// a caller-owned workspace keep their graph.
struct GraphKey {
  int dev = -1;
  const void* base = nullptr;
  std::vector<int> n, bm;
  int iters = 0, comp = 0, gate = 0, grid64 = 0, grid32 = 0;
  double tol = 0;
  float trunc = 0;
  bool operator==(const GraphKey& o) const {
    return dev == o.dev && base == o.base && n == o.n && bm == o.bm && iters == o.iters && comp == o.comp &&
           gate == o.gate && tol == o.tol && trunc == o.trunc && grid64 == o.grid64 && grid32 == o.grid32;
  }
};
struct GraphCache {
  GraphKey key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void clear() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    key = GraphKey();
  }
  ~GraphCache() { clear(); }
};
GraphCache& graph_cache() {
  static thread_local GraphCache c;
  return c;
}
std::atomic<int> g_graph_builds{0};

}  // namespace
}  // namespace sr

using namespace sr;

extern "C" {

size_t sr_workspace_bytes_batched(int batch, const int* n, const sr_opts* opts) {
  (void)opts;
  if (batch < 0 || (batch > 0 && !n)) return 0;
  std::vector<int> bm(batch, 32);  // the larger table of the two edges
  const BLayout L = layout(batch, n, bm);
  return std::max(L.total, tune_scratch_bytes(batch, n)) + 256;
}

int schur_refine_batched(int batch, const int* n, const void* const* A, void* const* Q, void* const* T,
                         int iters, double tol, const sr_opts* opts_in, sr_info* info) {
  if (batch < 0 || (batch > 0 && (!n || !A || !Q || !T)) || iters < 1 || !(tol > 0)) return SR_EINVAL;
  for (int b = 0; b < batch; b++)
    if (n[b] < 1 || !A[b] || !Q[b] || !T[b]) return SR_EINVAL;
  if (info) memset(info, 0, sizeof(sr_info) * batch);
  if (batch == 0) return SR_OK;
  sr_opts o;
  if (opts_in) o = *opts_in;
  else sr_default_opts(&o);
  if (o.gemm != SR_GEMM_FP64 || o.solver != SR_SOLVER_WAVEFRONT || o.skip_orth || o.lp_digits) return SR_ENOSYS;
  const int comp = o.compensated ? 1 : 0;
  hipStream_t user = (hipStream_t)o.stream;
  hipStream_t st = capture_stream();
  if (!st) return SR_EHIP;

  // workspace
  const size_t need = sr_workspace_bytes_batched(batch, n, &o);
  void* base = o.workspace;
  void* owned = nullptr;
  if (base) {
    if (o.workspace_bytes < need) return SR_ENOMEM;
  } else {
    if (hipMalloc(&owned, need) != hipSuccess) return SR_ENOMEM;
    base = owned;
  }
  int rc = SR_OK;
  hipEvent_t ev;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    if (owned) hipFree(owned);
    return SR_EHIP;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto fail = [&](int code) {
    rc = code;
    return code;
  };
  do {
    // order after the caller's stream
    if (hipEventRecord(ev, user) != hipSuccess || hipStreamWaitEvent(st, ev, 0) != hipSuccess) {
      fail(SR_EHIP);
      break;
    }
    // autotune the tile edge of each size bucket present
    std::map<int, std::vector<int>> buckets;
    for (int b = 0; b < batch; b++)
      if (n[b] >= 2) buckets[bucket_of(n[b])].push_back(b);
    std::vector<int> bm(batch, 64);
    int bpc64 = 0, bpc32 = 0;  // the largest blocks per CU chosen for an edge
    bool bad = false;
    for (auto& kv : buckets) {
      TuneChoice ch;
      if (tune_bucket(kv.first, kv.second, n, A, Q, base, st, &ch) != SR_OK) {
        bad = true;
        break;
      }
      for (int b : kv.second) bm[b] = ch.edge;
      int& g = ch.edge == 64 ? bpc64 : bpc32;
      g = std::max(g, ch.bpc);
    }
    if (bad) {
      fail(SR_EHIP);
      break;
    }
    const BLayout L = layout(batch, n, bm);
    char* w = (char*)base;
    // per-matrix records and tables (host)
    std::vector<BMat> mats(batch);
    std::vector<GemmArgs> args((size_t)kArgTables * batch);
    std::vector<GTile> t64, t32;
    std::vector<char> tri(trimatrix_bytes() * batch);
    // The solve goes by tile diagonal across the batch once a matrix has three or more
    // 16-wide tile rows; below that one block per matrix walks its few tiles.
    std::vector<TriStepTile> step_tiles(trisolve_steps_tiles(n, batch) + 1);
    std::vector<int> step_off(trisolve_steps_max(n, batch) + 1);
    int nsteps = 0;
    trisolve_steps_plan(n, batch, step_tiles.data(), step_off.data(), &nsteps);
    const bool by_steps = nsteps >= 3;
    int* active = (int*)(w + L.active);
    int* act_w2 = (int*)(w + L.act_w2);
    int* act_w3 = (int*)(w + L.act_w3);
    int* act_yw = (int*)(w + L.act_yw);
    BState* states = (BState*)(w + L.states);
    double* partials = (double*)(w + L.partials);
    int slot = 0;
    for (int b = 0; b < batch; b++) {
      BMat& m = mats[b];
      memset(&m, 0, sizeof(m));
      const int nb = n[b];
      m.n = nb;
      m.A = (const zc*)A[b];
      m.Q = (zc*)Q[b];
      m.T = (zc*)T[b];
      if (nb >= 2) {
        const size_t z = a256((size_t)nb * nb * sizeof(zc)), c = a256((size_t)nb * nb * sizeof(cc));
        char* p = w + L.off[b];
        m.Qa = (zc*)p;
        m.QH = (zc*)(p + z);
        m.P = (zc*)(p + 2 * z);
        m.Y = (zc*)(p + 3 * z);
        cc* cs[8];
        for (int i = 0; i < 8; i++) cs[i] = (cc*)(p + 4 * z + i * c);
        m.Tlp = cs[0];
        m.Elp = cs[1];
        m.L = cs[2];
        m.W = cs[3];
        m.W2 = cs[4];
        m.W3 = cs[5];
        m.YW = cs[6];
        m.Ylp = cs[7];
        m.slot0 = slot;
        m.nslots = tiles_of(nb, bm[b]);
        std::vector<GTile>& tl = bm[b] == 64 ? t64 : t32;
        int s = slot;
        for (int tn = 0; tn < ceil_div(nb, bm[b]); tn++)
          for (int tm = 0; tm < ceil_div(nb, bm[b]); tm++) tl.push_back({b, tm * bm[b], tn * bm[b], s++});
        slot = s;
      }
      trimatrix_fill(tri.data() + trimatrix_bytes() * b, m.Tlp, m.Elp, m.L, nb >= 2 ? nb : 0, active + b,
                     &states[b].flag);
      // product tables
      auto A_ = [&](int t) -> GemmArgs& { return args[(size_t)t * batch + b]; };
      if (nb < 2) continue;
      A_(T_NSY) = gargs_b(nb, m.Q, m.Q, m.Y);
      A_(T_NSY).partials = partials;
      A_(T_NSU) = gargs_b(nb, m.Q, m.P, m.Qa);
      A_(T_NSU).Cin = m.Q;
      A_(T_NSU).ldcin = nb;
      A_(T_NSU).CH = m.QH;
      A_(T_NSU).ldch = nb;
      for (int e = 0; e < 2; e++) {
        zc* cur = e == 0 ? m.Qa : m.Q;  // even passes start from Qa (after the start)
        zc* oth = e == 0 ? m.Q : m.Qa;
        A_(T_P + 4 * e) = gargs_b(nb, m.A, cur, m.P);
        GemmArgs& s_ = A_(T_T + 4 * e);
        s_ = gargs_b(nb, m.QH, m.P, m.T);
        s_.Tlp = m.Tlp;
        s_.Elp = m.Elp;
        s_.ldlp = nb;
        s_.partials = partials;
        A_(T_Y + 4 * e) = gargs_b(nb, m.QH, cur, m.Y);
        A_(T_Y + 4 * e).partials = partials;
        GemmArgs& u = A_(T_U + 4 * e);
        u = gargs_b(nb, cur, m.P, oth);
        u.Cin = cur;
        u.ldcin = nb;
        u.CH = m.QH;
        u.ldch = nb;
      }
      A_(T_W2) = gargs_b(nb, m.W, m.W, m.W2);
      A_(T_W3) = gargs_b(nb, m.W2, m.W, m.W3);
      A_(T_YW) = gargs_b(nb, m.Ylp, m.W, m.YW);
    }
    GTile* tiles_dev = (GTile*)(w + L.tiles);
    if (hipMemcpyAsync(w + L.mats, mats.data(), sizeof(BMat) * batch, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(w + L.args, args.data(), sizeof(GemmArgs) * args.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        (t64.size() && hipMemcpyAsync(tiles_dev, t64.data(), sizeof(GTile) * t64.size(), hipMemcpyHostToDevice, st) != hipSuccess) ||
        (t32.size() && hipMemcpyAsync(tiles_dev + t64.size(), t32.data(), sizeof(GTile) * t32.size(), hipMemcpyHostToDevice, st) != hipSuccess) ||
        hipMemcpyAsync(w + L.tri, tri.data(), tri.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        (by_steps && hipMemcpyAsync(w + L.steps, step_tiles.data(), sizeof(TriStepTile) * step_off[nsteps],
                                    hipMemcpyHostToDevice, st) != hipSuccess)) {
      fail(SR_EHIP);
      break;
    }
    const BMat* mats_dev = (const BMat*)(w + L.mats);
    int* counter = (int*)(w + L.counter);
    const int grid64 = std::max(1, (int)std::min<size_t>(t64.size(), (size_t)std::max(1, bpc64) * kCUs));
    const int grid32 = std::max(1, (int)std::min<size_t>(t32.size(), (size_t)std::max(1, bpc32) * kCUs));
    Launcher G{(const GemmArgs*)(w + L.args), tiles_dev, tiles_dev + t64.size(), (int)t64.size(),
               (int)t32.size(), batch, grid64, grid32, st};
    const int small = ceil_div(batch, 256);

    // start: norms, state, Newton-Schulz orthogonalisation of the starts
    hipLaunchKernelGGL(b_init_kernel, dim3(batch), dim3(BNT), 0, st, mats_dev, states, active);
    if (G.z(T_NSY, 1, EPI_YDEF, comp, active) != hipSuccess) { fail(SR_EHIP); break; }
    hipLaunchKernelGGL(b_ns_delta_kernel, dim3(batch), dim3(BNT), 0, st, mats_dev, active);
    if (G.z(T_NSU, 0, EPI_ADD, 0, active) != hipSuccess) { fail(SR_EHIP); break; }
    if (hipGetLastError() != hipSuccess) { fail(SR_EHIP); break; }

    // the two-pass graph: reused from the last call on this thread when nothing it
    // depends on changed, otherwise captured anew
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) { fail(SR_EHIP); break; }
    GraphKey key;
    key.dev = dev;
    key.grid64 = grid64;
    key.grid32 = grid32;
    key.base = base;
    key.n.assign(n, n + batch);
    key.bm = bm;
    key.iters = iters;
    key.comp = comp;
    key.gate = o.gate_lp_terms ? 1 : 0;
    key.tol = tol;
    key.trunc = o.trunc ? 1e-5f : 0.f;
    GraphCache& gc = graph_cache();
    const bool reuse = !owned && gc.exec && gc.key == key;
    if (reuse) {
      exec = gc.exec;
    } else {
      if (!owned) gc.clear();
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) { fail(SR_EHIP); break; }
      bool cap_ok = true;
      for (int e = 0; e < 2 && cap_ok; e++) {
        hipLaunchKernelGGL(b_pass_start_kernel, dim3(small), dim3(256), 0, st, states, batch, counter);
        cap_ok = G.z(T_P + 4 * e, 0, EPI_STORE, comp, active) == hipSuccess &&
                 G.z(T_T + 4 * e, 0, EPI_SPLIT, comp, active) == hipSuccess;
        if (!cap_ok) break;
        hipLaunchKernelGGL(b_decide_kernel, dim3(batch), dim3(BNT), 0, st, mats_dev, states, active, partials,
                           iters, tol, counter);
        const float tr = o.trunc ? 1e-5f : 0.f;
        cap_ok = (by_steps ? trisolve_batched_steps(w + L.tri, (const TriStepTile*)(w + L.steps), step_off.data(),
                                                    nsteps, tr, st)
                           : trisolve_batched(w + L.tri, batch, tr, st)) == hipSuccess &&
                 G.z(T_Y + 4 * e, 0, EPI_YDEF, comp, active) == hipSuccess;
        if (!cap_ok) break;
        hipLaunchKernelGGL(b_post_kernel, dim3(batch), dim3(BNT), 0, st, mats_dev, states, active, partials,
                           o.gate_lp_terms ? 1 : 0, act_w2, act_w3, act_yw);
        cap_ok = G.c(T_W2, act_w2) == hipSuccess && G.c(T_W3, act_w3) == hipSuccess &&
                 G.c(T_YW, act_yw) == hipSuccess;
        if (!cap_ok) break;
        hipLaunchKernelGGL(b_delta_kernel, dim3(batch), dim3(BNT), 0, st, mats_dev, states, active);
        cap_ok = G.z(T_U + 4 * e, 0, EPI_ADD, 0, active) == hipSuccess;
        hipLaunchKernelGGL(b_flip_kernel, dim3(small), dim3(256), 0, st, states, active, batch);
      }
      const hipError_t ce = hipStreamEndCapture(st, &graph);
      if (!cap_ok || ce != hipSuccess || hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        fail(SR_EHIP);
        break;
      }
      g_graph_builds++;
      if (!owned) {
        // kept for the next call on this thread
        gc.key = key;
        gc.graph = graph;
        gc.exec = exec;
        graph = nullptr;
      }
    }
    int* hcount = host_counter();
    if (!hcount) {
      fail(SR_ENOMEM);
      break;
    }
    for (int p = 0; p < iters; p += 2) {
      if (hipGraphLaunch(exec, st) != hipSuccess ||
          hipMemcpyAsync(hcount, counter, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        fail(SR_EHIP);
        break;
      }
      if (*hcount == 0) break;
    }
    if (rc != SR_OK) break;
    hipLaunchKernelGGL(b_finish_kernel, dim3(batch), dim3(BNT), 0, st, mats_dev, states);
    std::vector<BState> hs(batch);
    if (hipMemcpyAsync(hs.data(), states, sizeof(BState) * batch, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      fail(SR_EHIP);
      break;
    }
    int worst = SR_OK;
    for (int b = 0; b < batch; b++) {
      const BState& z = hs[b];
      const int s = z.status < 0 ? SR_NOT_CONVERGED : z.status;
      if (s > worst) worst = s;
      if (info) {
        sr_info& f = info[b];
        f.status = s;
        f.iters = z.passes;
        f.updates = z.updates;
        f.hp_gemms = n[b] >= 2 ? 2 + 4 * z.updates + 2 * (z.passes - z.updates) : 0;
        f.lp_products = z.lp_products;
        f.resid = z.eps;
        f.orth = z.orth;
        for (int i = 0; i < 16; i++) {
          f.resid_hist[i] = i < z.passes ? z.resid_hist[i] : 0;
          f.norm_w_hist[i] = i < z.updates ? z.norm_w_hist[i] : 0;
        }
      }
    }
    rc = worst;
    // the caller's stream continues after this call's work
    if (hipEventRecord(ev, st) != hipSuccess || hipStreamWaitEvent(user, ev, 0) != hipSuccess) fail(SR_EHIP);
  } while (false);
  // a graph kept in the thread's cache is destroyed when it is replaced
  if (exec && exec != graph_cache().exec) hipGraphExecDestroy(exec);
  if (graph) hipGraphDestroy(graph);
  hipEventDestroy(ev);
  if (owned) {
    hipStreamSynchronize(st);
    hipFree(owned);
  }
  return rc;
}

// Two-pass graphs captured and instantiated so far in this process.
int sr_batched_graph_builds(void) { return g_graph_builds.load(); }

// Bucket -> tile edge chosen so far (-1: not tuned yet); for reports and tests.
int sr_batched_tile_edge(int n) {
  std::lock_guard<std::mutex> lk(tuner().mu);
  auto it = tuner().bm.find(bucket_of(n));
  return it == tuner().bm.end() ? -1 : it->second.edge;
}

int sr_batched_tile_grid(int n) {
  std::lock_guard<std::mutex> lk(tuner().mu);
  auto it = tuner().bm.find(bucket_of(n));
  return it == tuner().bm.end() ? -1 : it->second.bpc;
}

int sr_tuning_save(const char* path) {
  if (!path) return SR_EINVAL;
  std::lock_guard<std::mutex> lk(tuner().mu);
  return tuning_save_locked(path);
}

int sr_tuning_load(const char* path) {
  if (!path) return SR_EINVAL;
  std::lock_guard<std::mutex> lk(tuner().mu);
  tuner().env_loaded = true;
  return tuning_load_locked(path);
}

void sr_tuning_reset(void) {
  std::lock_guard<std::mutex> lk(tuner().mu);
  tuner().bm.clear();
  tuner().env_loaded = true;  // a reset table is not refilled from SR_TUNING_FILE
}

int sr_tuning_runs(void) {
  std::lock_guard<std::mutex> lk(tuner().mu);
  return tuner().runs;
}

}  // extern "C"
