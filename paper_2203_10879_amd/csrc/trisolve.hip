// Triangular matrix equation stril(T L - L T) = -E (Section 2.1, eqs. (7)-(10)):
// the low-precision solve of every refinement pass, in FP32 (complex64) for the
// FP64 tier and in FP64 (complex128) for the double-double tier. The code below is
// written once for both element types.
//
// Entry (i, j), i > j, reads
//   l_ij = -( e_ij + sum_{k>i} t_ik l_kj - sum_{k<j} l_ik t_kj ) / (t_ii - t_jj),
// so an entry needs the entries below it in its column and left of it in its row:
// entries on one subdiagonal i - j = d are independent (the wavefront order the
// paper mentions after Theorem 1).
//
// GPU schedule. L is cut into TB x TB tiles (TB = 16 up to n = 2048, 32 above).
// For a tile (I, J), I >= J, the same algebra at tile level gives
//   T_II X - X T_JJ = -R_IJ,  R_IJ = E_IJ + sum_{K>I} T_IK L_KJ - sum_{K<J} L_IK T_KJ
// (for I = J only the strictly lower part, with X strictly lower): a tile depends
// on the tiles below it in its tile column and left of it in its tile row, so the
// tiles of one tile diagonal D = I - J are independent, and L_KJ, L_IK of the sum
// lie on tile diagonals > D. Only two of the block products of a tile touch
// diagonal D + 1 (K = I + 1 and K = J - 1, the "near" products); the others touch
// diagonals >= D + 2 ("far").
//
// One launch per tile diagonal D = nb-1 .. 0, with two kinds of blocks:
//   - solve blocks (one per tile of diagonal D): R = E + the far partial sums
//     computed by the previous launch + the two near products, then substitution
//     inside the tile along its anti-diagonals (2 TB - 1 dependent steps; TB - 1 on
//     the diagonal) with T_II and T_JJ in LDS and one thread per entry;
//   - partial blocks for diagonal D - 1: its far products, split over S blocks per
//     tile so that the launch fills the chip, written to a buffer selected by the
//     parity of D.
// No block waits on another and no device-scope fence is needed: all data a
// launch reads were written by earlier launches. Small matrices use one block that
// walks all tiles; batches go by tile diagonal across their matrices (one launch
// per step, one block per tile), or one block per matrix when every matrix has at
// most two tile rows.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "kernels.hpp"
namespace sr {

constexpr int kTargetBlocks = 2 * kCUs;

// ok ? v : 0, component-wise (a struct-valued select would go through scratch).
template <typename R>
__device__ inline cplx<R> keep(bool ok, cplx<R> v) {
  return mk<R>(ok ? v.re : R(0), ok ? v.im : R(0));
}

template <typename Rl>
struct TriMatrix {
  const cplx<Rl>* T;
  const cplx<Rl>* E;
  cplx<Rl>* L;
  int n;
  const int* active;  // batched use: skip the matrix when *active == 0 (may be NULL)
  unsigned* flag;     // batched use: per-matrix status bits (NULL: the shared word)
};

namespace tri16 {
constexpr int TB = 16;
#include "trisolve_tiles.inc"
}  // namespace tri16

namespace tri32 {
constexpr int TB = 32;
#include "trisolve_tiles.inc"
}  // namespace tri32

// Tile edge by size. Smaller tiles shorten a tile's substitution (2 TB - 1
// dependent steps) and its barriers (TB^2 threads) at the price of more levels and
// launches: measured per FP32 solve, 16 against 32: n = 1024 687 against 813 us,
// n = 2048 1.84 against 1.90 ms (FP64: 2.18 against 2.31), n = 4096 9.18 against
// 8.47 ms.
constexpr int kSmallTileMaxN = 2048;
static bool small_tiles(int n) { return n <= kSmallTileMaxN; }

size_t trisolve_ws_bytes(int n) { return small_tiles(n) ? tri16::ws_bytes(n) : tri32::ws_bytes(n); }

hipError_t trisolve(const cc* T, const cc* E, cc* L, int n, float trunc, void* ws,
                    unsigned* status, hipStream_t st) {
  return small_tiles(n) ? tri16::solve<float>(T, E, L, n, trunc, ws, status, st)
                        : tri32::solve<float>(T, E, L, n, trunc, ws, status, st);
}

hipError_t trisolve64(const zc* T, const zc* E, zc* L, int n, void* ws, unsigned* status,
                      hipStream_t st) {
  return small_tiles(n) ? tri16::solve<double>(T, E, L, n, 0.f, ws, status, st)
                        : tri32::solve<double>(T, E, L, n, 0.f, ws, status, st);
}

// Batched solves (n <= 256, one block per matrix): 16-wide tiles (measured on the
// 2000-matrix batch: 50.8 against 53.6 ms per batch).
hipError_t trisolve_batched(const void* mats, int count, float trunc, hipStream_t st) {
  return tri16::batched(mats, count, trunc, st);
}

static int step_rows(int n) { return n >= 2 ? (n + tri16::TB - 1) / tri16::TB : 0; }

size_t trisolve_steps_tiles(const int* n, int count) {
  size_t t = 0;
  for (int b = 0; b < count; b++) t += (size_t)step_rows(n[b]) * (step_rows(n[b]) + 1) / 2;
  return t;
}

int trisolve_steps_max(const int* n, int count) {
  int m = 0;
  for (int b = 0; b < count; b++) m = std::max(m, step_rows(n[b]));
  return m;
}

void trisolve_steps_plan(const int* n, int count, TriStepTile* tiles, int* step_off, int* steps) {
  const int S = trisolve_steps_max(n, count);
  int k = 0;
  for (int s = 0; s < S; s++) {
    step_off[s] = k;
    for (int b = 0; b < count; b++) {
      const int nb = step_rows(n[b]);
      if (nb <= s) continue;
      const int D = nb - 1 - s;
      for (int t = 0; t <= s; t++) tiles[k++] = TriStepTile{b, D + t, t};
    }
  }
  step_off[S] = k;
  *steps = S;
}

hipError_t trisolve_batched_steps(const void* mats, const TriStepTile* tiles, const int* step_off, int steps,
                                  float trunc, hipStream_t st) {
  for (int s = 0; s < steps; s++) {
    const int cnt = step_off[s + 1] - step_off[s];
    if (cnt == 0) continue;
    hipLaunchKernelGGL(tri16::trisolve_step_kernel<float>, dim3(cnt), dim3(tri16::TNT), 0, st,
                       (const TriMatrix<float>*)mats, tiles + step_off[s], trunc);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------- recursive block solve (Algorithm 3)

namespace {

constexpr int kRecTB = tri16::TB;

size_t rec_align(size_t b) { return (b + 255) / 256 * 256; }

// The whole schedule of one solve: per phase (a depth of the recursion) the steps of
// tile tasks (the Sylvester blocks of that depth's nodes and its leaves, merged by
// step index) and the grouped updates of E.
struct RecPlan {
  int n = 0, leaf = 0;
  std::vector<TileTask> tasks;
  std::vector<int> step_off;   // first task of every step, then the total
  std::vector<int> step_mf;    // most far products of a task of the step
  std::vector<int> phase_step; // first step of every phase, then the total
  std::vector<GemmArgs> gargs;
  std::vector<GTile> gtiles;
  std::vector<int> phase_tile;  // first grouped tile of every phase, then the total
  std::vector<int> phase_bm;    // tile edge of the phase's updates
  int max_tasks = 0;
};

int task_far(const TileTask& k) { return std::max(0, k.hi - k.I - 2) + std::max(0, k.J - 1 - k.lo); }

// The plan for size n with leaves of at most `leaf` tiles. Pointers of the updates
// are filled by rec_bind.
RecPlan rec_plan(int n, int leaf) {
  RecPlan pl;
  pl.n = n;
  pl.leaf = leaf = std::max(1, leaf);
  const int nb = ceil_div(n, kRecTB);
  std::vector<std::pair<int, int>> nodes{{0, nb}};
  pl.phase_step.push_back(0);
  pl.phase_tile.push_back(0);
  while (!nodes.empty()) {
    std::vector<std::vector<TileTask>> steps;
    std::vector<std::pair<int, int>> next;
    std::vector<std::pair<int, int>> split;  // (lo, hi) of nodes with updates, mid at half
    auto put = [&](int step, TileTask t) {
      if ((int)steps.size() <= step) steps.resize(step + 1);
      steps[step].push_back(t);
    };
    for (auto [lo, hi] : nodes) {
      const int nt = hi - lo;
      if (nt <= leaf) {
        for (int I = lo; I < hi; I++)
          for (int J = lo; J <= I; J++) put((hi - 1 - I) + (J - lo), TileTask{I, J, lo, hi});
      } else {
        const int mid = lo + nt / 2;
        for (int I = mid; I < hi; I++)
          for (int J = lo; J < mid; J++) put((hi - 1 - I) + (J - lo), TileTask{I, J, lo, hi});
        split.push_back({lo, hi});
        next.push_back({lo, mid});
        next.push_back({mid, hi});
      }
    }
    for (auto& st : steps) {
      pl.step_off.push_back((int)pl.tasks.size());
      int mf = 0;
      for (const TileTask& t : st) mf = std::max(mf, task_far(t));
      pl.step_mf.push_back(mf);
      pl.max_tasks = std::max(pl.max_tasks, (int)st.size());
      pl.tasks.insert(pl.tasks.end(), st.begin(), st.end());
    }
    pl.phase_step.push_back((int)pl.step_off.size());
    // updates: for node (lo, mid, hi) in elements r1, m1, h,
    //   E(r1:m1, r1:m1) += T(r1:m1, m1:h) L(m1:h, r1:m1)
    //   E(m1:h, m1:h)   += L(m1:h, r1:m1) (-T)(r1:m1, m1:h)
    // only the tiles that hold entries below the diagonal
    long tiles64 = 0;
    for (auto [lo, hi] : split) {
      const int mid = lo + (hi - lo) / 2;
      const int r1 = lo * kRecTB, m1 = mid * kRecTB, h = std::min(hi * kRecTB, n);
      tiles64 += (long)ceil_div(m1 - r1, 64) * ceil_div(m1 - r1, 64) + (long)ceil_div(h - m1, 64) * ceil_div(h - m1, 64);
    }
    const int bm = tiles64 >= 2 * kCUs ? 64 : 32;
    for (auto [lo, hi] : split) {
      const int mid = lo + (hi - lo) / 2;
      const int r1 = lo * kRecTB, m1 = mid * kRecTB, h = std::min(hi * kRecTB, n);
      const int dims[2] = {m1 - r1, h - m1};
      for (int g = 0; g < 2; g++) {
        GemmArgs a;
        memset(&a, 0, sizeof(a));
        a.m = a.n = dims[g];
        a.k = dims[1 - g];
        // operand offsets (elements) kept in the pointer fields until rec_bind
        a.A = (const void*)(uintptr_t)(g == 0 ? r1 + (long)m1 * n : m1 + (long)r1 * n);
        a.B = (const void*)(uintptr_t)(g == 0 ? m1 + (long)r1 * n : r1 + (long)m1 * n);
        a.C = (void*)(uintptr_t)(g == 0 ? r1 + (long)r1 * n : m1 + (long)m1 * n);
        a.lda = a.ldb = a.ldc = a.ldcin = n;
        a.tiles_m = ceil_div(a.m, bm);
        a.tiles_n = ceil_div(a.n, bm);
        const int mat = (int)pl.gargs.size();
        pl.gargs.push_back(a);
        for (int tn = 0; tn < a.tiles_n; tn++)
          for (int tm = 0; tm < a.tiles_m; tm++)
            if (tm * bm + bm - 1 > tn * bm) pl.gtiles.push_back(GTile{mat, tm * bm, tn * bm, 0});
      }
    }
    pl.phase_tile.push_back((int)pl.gtiles.size());
    pl.phase_bm.push_back(bm);
    nodes.swap(next);
  }
  pl.step_off.push_back((int)pl.tasks.size());
  return pl;
}

struct RecLayout {
  size_t part, ew, negt, total;        // the caller's workspace
  size_t tasks, gargs, gtiles, tables;  // the library's table buffer
};

RecLayout rec_layout(const RecPlan& pl) {
  RecLayout l;
  const size_t nn = (size_t)pl.n * pl.n;
  l.part = rec_align((size_t)(kTargetBlocks + pl.max_tasks) * tri16::kTileElems * sizeof(cc));
  l.ew = rec_align(nn * sizeof(cc));
  l.negt = rec_align(nn * sizeof(cc));
  l.total = 2 * l.part + l.ew + l.negt;
  l.tasks = rec_align(pl.tasks.size() * sizeof(TileTask));
  l.gargs = rec_align(pl.gargs.size() * sizeof(GemmArgs));
  l.gtiles = rec_align(pl.gtiles.size() * sizeof(GTile));
  l.tables = l.tasks + l.gargs + l.gtiles;
  return l;
}

// Device tables of a solve (tasks, update operands and tiles), owned by the library
// and keyed on everything they hold: the device, n, the leaf size and the pointers
// the update operands are bound to (T, L and the caller's workspace). A refinement's
// passes find their tables here; nothing else writes to them. At most kRecKeep
// entries are kept (the oldest is freed after a device synchronisation).
struct RecCache {
  std::mutex mu;
  struct Entry {
    int dev, n, leaf;
    const void *T, *L, *ws;
    RecPlan plan;
    void* dtab;
  };
  std::vector<Entry> entries;
};
constexpr size_t kRecKeep = 16;
RecCache& rec_cache() {
  static RecCache c;
  return c;
}

__global__ void rec_prep_kernel(const cc* __restrict__ T, const cc* __restrict__ E, cc* __restrict__ Ew,
                                cc* __restrict__ negT, long nn) {
  for (long z = blockIdx.x * (long)blockDim.x + threadIdx.x; z < nn; z += (long)gridDim.x * blockDim.x) {
    Ew[z] = E[z];
    const cc t = T[z];
    negT[z] = mk<float>(-t.re, -t.im);
  }
}

}  // namespace

size_t trisolve_rec_ws_bytes(int n, int leaf_tiles) {
  if (n < 1) return 0;
  return rec_layout(rec_plan(n, leaf_tiles)).total;
}

hipError_t trisolve_rec(const cc* T, const cc* E, cc* L, int n, int leaf_tiles, float trunc, void* ws,
                        unsigned* status, hipStream_t st) {
  hipError_t e = fill_zero(L, (size_t)n * n * sizeof(cc), st);
  if (e != hipSuccess || n <= 1) return e;
  leaf_tiles = std::max(1, leaf_tiles);
  int dev = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  RecCache& c = rec_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  RecCache::Entry* ent = nullptr;
  for (auto& x : c.entries)
    if (x.dev == dev && x.n == n && x.leaf == leaf_tiles && x.T == T && x.L == L && x.ws == ws) ent = &x;
  if (!ent) {
    if (c.entries.size() >= kRecKeep) {
      if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
      RecCache::Entry& old = c.entries.front();
      int cur = 0;
      hipGetDevice(&cur);
      hipSetDevice(old.dev);
      hipFree(old.dtab);
      hipSetDevice(cur);
      c.entries.erase(c.entries.begin());
    }
    RecCache::Entry x{dev, n, leaf_tiles, T, L, ws, rec_plan(n, leaf_tiles), nullptr};
    const RecLayout lay = rec_layout(x.plan);
    cc* Ew = (cc*)((char*)ws + 2 * lay.part);
    cc* negT = (cc*)((char*)Ew + lay.ew);
    // bind the update operands (offsets -> pointers)
    std::vector<GemmArgs> ga = x.plan.gargs;
    for (size_t i = 0; i < ga.size(); i++) {
      const int g = (int)(i & 1);
      const uintptr_t oa = (uintptr_t)ga[i].A, ob = (uintptr_t)ga[i].B, oc = (uintptr_t)ga[i].C;
      ga[i].A = g == 0 ? (const void*)(T + oa) : (const void*)(L + oa);
      ga[i].B = g == 0 ? (const void*)(L + ob) : (const void*)(negT + ob);
      ga[i].C = Ew + oc;
      ga[i].Cin = Ew + oc;
    }
    std::vector<char> blob(lay.tables, 0);
    memcpy(blob.data(), x.plan.tasks.data(), x.plan.tasks.size() * sizeof(TileTask));
    memcpy(blob.data() + lay.tasks, ga.data(), ga.size() * sizeof(GemmArgs));
    memcpy(blob.data() + lay.tasks + lay.gargs, x.plan.gtiles.data(), x.plan.gtiles.size() * sizeof(GTile));
    if ((e = hipMalloc(&x.dtab, std::max<size_t>(lay.tables, 256))) != hipSuccess) return e;
    if ((e = hipMemcpy(x.dtab, blob.data(), blob.size(), hipMemcpyHostToDevice)) != hipSuccess) {
      hipFree(x.dtab);
      return e;
    }
    c.entries.push_back(std::move(x));
    ent = &c.entries.back();
  }
  const RecPlan& pl = ent->plan;
  const RecLayout lay = rec_layout(pl);
  char* base = (char*)ws;
  cc* part[2] = {(cc*)base, (cc*)(base + lay.part)};
  cc* Ew = (cc*)(base + 2 * lay.part);
  cc* negT = (cc*)((char*)Ew + lay.ew);
  const TileTask* dtasks = (const TileTask*)ent->dtab;
  const GemmArgs* dgargs = (const GemmArgs*)((char*)ent->dtab + lay.tasks);
  const GTile* dgtiles = (const GTile*)((char*)ent->dtab + lay.tasks + lay.gargs);
  const long nn = (long)n * n;
  hipLaunchKernelGGL(rec_prep_kernel, dim3(std::min(2048L, (nn + 255) / 256)), dim3(256), 0, st, T, E, Ew, negT,
                     nn);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int phases = (int)pl.phase_bm.size();
  for (int ph = 0; ph < phases; ph++) {
    int S_cur = 0;
    const int g0 = pl.phase_step[ph], g1 = pl.phase_step[ph + 1];
    for (int g = g0; g < g1; g++) {
      const int ncur = pl.step_off[g + 1] - pl.step_off[g];
      const bool more = g + 1 < g1;
      const int nnext = more ? pl.step_off[g + 2] - pl.step_off[g + 1] : 0;
      const int S_next = more ? tri16::task_splits(pl.step_mf[g + 1], nnext) : 0;
      tri16::TaskLevelArgs<float> a{T,     Ew,      L,       n,      dtasks + pl.step_off[g],
                                    ncur,  S_cur,   part[g & 1],     dtasks + (more ? pl.step_off[g + 1] : 0),
                                    nnext, S_next,  part[(g + 1) & 1], status, trunc};
      hipLaunchKernelGGL(tri16::trisolve_task_kernel<float>, dim3(ncur + nnext * S_next), dim3(tri16::TNT), 0,
                         st, a);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      S_cur = S_next;
    }
    const int t0 = pl.phase_tile[ph], t1 = pl.phase_tile[ph + 1];
    if (t1 > t0) {
      e = cgemm_grouped_add(pl.phase_bm[ph], dgargs, dgtiles + t0, t1 - t0, std::min(t1 - t0, 4 * kCUs), st);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

size_t trimatrix_bytes() { return sizeof(TriMatrix<float>); }
void trimatrix_fill(void* dst, const cc* T, const cc* E, cc* L, int n, const int* active,
                    unsigned* flag) {
  TriMatrix<float> m{T, E, L, n, active, flag};
  memcpy(dst, &m, sizeof(m));
}

}  // namespace sr
