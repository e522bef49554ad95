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

size_t trimatrix_bytes() { return sizeof(TriMatrix<float>); }
void trimatrix_fill(void* dst, const cc* T, const cc* E, cc* L, int n, const int* active,
                    unsigned* flag) {
  TriMatrix<float> m{T, E, L, n, active, flag};
  memcpy(dst, &m, sizeof(m));
}

}  // namespace sr
