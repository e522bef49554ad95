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
// GPU schedule. L is cut into TB x TB tiles (TB = 32). For a tile (I, J), I >= J, the
// same algebra at tile level gives
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
// launch reads were written by earlier launches. Small matrices (and the batched
// path) use one block that walks all tiles.
#include <string.h>

#include "kernels.hpp"

namespace sr {

#ifndef SR_TRI_TB
#define SR_TRI_TB 32
#endif
constexpr int TB = SR_TRI_TB;
constexpr int TNT = TB * TB;  // one thread per tile entry
constexpr int TLD = TB + 1;   // LDS column stride (elements)
constexpr int kTargetBlocks = 2 * kCUs;
constexpr int kTileElems = TB * TB;

// ok ? v : 0, component-wise (a struct-valued select would go through scratch).
template <typename R>
__device__ inline cplx<R> keep(bool ok, cplx<R> v) {
  return mk<R>(ok ? v.re : R(0), ok ? v.im : R(0));
}

// Column ownership (products, partial sums): thread t owns entry (t mod 32, t / 32).
struct Own {
  int p, q;
};
__device__ inline Own owner() {
  Own o;
  o.p = threadIdx.x & (TB - 1);
  o.q = threadIdx.x / TB;
  return o;
}

// LDS tile, column-major with padded stride: S[q * TLD + p] = G(I*TB + p, J*TB + q),
// zero outside the n x n matrix.
template <typename C>
__device__ inline void load_tile(C* S, const C* __restrict__ G, int n, int I, int J) {
  const int p = threadIdx.x & (TB - 1), q = threadIdx.x / TB;
  const int gi = I * TB + p, gj = J * TB + q;
  const bool ok = gi < n && gj < n;
  const C v = G[ok ? gi + (long)gj * n : 0];
  S[q * TLD + p] = keep(ok, v);
}

// This thread's element of tile (I, J) of G in the load_tile ownership (zero
// outside the matrix, also for a negative tile index).
template <typename C>
__device__ inline C tile_val(const C* __restrict__ G, int n, int I, int J) {
  const int p = threadIdx.x & (TB - 1), q = threadIdx.x / TB;
  const int gi = I * TB + p, gj = J * TB + q;
  const bool ok = I >= 0 && J >= 0 && gi < n && gj < n;
  const C v = G[ok ? gi + (long)gj * n : 0];
  return keep(ok, v);
}

// The same as a raw load and a flag, so that the zero padding (keep) can be
// applied where the value is used and the load stays in flight until then.
template <typename C>
struct Pending {
  C v;
  bool ok;
  __device__ C get() const { return keep(ok, v); }
};
template <typename C>
__device__ inline Pending<C> tile_load(const C* __restrict__ G, int n, int I, int J) {
  const int p = threadIdx.x & (TB - 1), q = threadIdx.x / TB;
  const int gi = I * TB + p, gj = J * TB + q;
  Pending<C> r;
  r.ok = I >= 0 && J >= 0 && gi < n && gj < n;
  r.v = G[r.ok ? gi + (long)gj * n : 0];
  return r;
}

template <int SIGN, typename C>
__device__ inline void tile_mac(C& acc, const C* F, const C* G, Own o) {
#pragma unroll 8
  for (int k = 0; k < TB; k++) {
    const C a = F[k * TLD + o.p], b = G[o.q * TLD + k];
    if (SIGN > 0) cfma(acc, a, b);
    else cfms(acc, a, b);
  }
}

// acc += the block products u0 .. u1-1 of tile (I, J) from the list
//   u < nA:  + T_{I,K} L_{K,J}, K = kA + u;   u >= nA:  - L_{I,K} T_{K,J}, K = u - nA,
// in that order. The operands of the next product are loaded into registers while
// the current one is multiplied, so a block waits for one memory round trip in
// all rather than one per product.
template <typename C>
__device__ void product_range(C& acc, const C* T, const C* L, int n, int I, int J, int kA, int nA, int u0,
                              int u1, C* S1, C* S2, Own o) {
  auto operands = [&](int u, Pending<C>& f, Pending<C>& g) {
    const bool a = u < nA;
    const int K = a ? kA + u : u - nA;
    f = tile_load(a ? T : L, n, I, K);
    g = tile_load(a ? L : T, n, K, J);
  };
  Pending<C> f, g;
  if (u0 < u1) operands(u0, f, g);
  for (int u = u0; u < u1; u++) {
    lds_barrier();  // the previous product no longer reads S1, S2
    S1[o.q * TLD + o.p] = f.get();
    S2[o.q * TLD + o.p] = g.get();
    if (u + 1 < u1) operands(u + 1, f, g);
    lds_barrier();  // the loads just issued stay in flight
    if (u < nA) tile_mac<+1>(acc, S1, S2, o);
    else tile_mac<-1>(acc, S1, S2, o);
  }
}

// All block products of tile (I, J) (K = I+1..nb-1 of the first kind, K = 0..J-1 of
// the second).
template <typename C>
__device__ void all_products(C& acc, const C* T, const C* L, int n, int nb, int I, int J, C* S1,
                             C* S2, Own o) {
  const int nA = nb - 1 - I;
  product_range(acc, T, L, n, I, J, I + 1, nA, 0, nA + J, S1, S2, o);
}

template <typename C>
__device__ inline void add_e(C& acc, const C* __restrict__ E, int n, int I, int J, Own o) {
  const int gi = I * TB + o.p, gj = J * TB + o.q;
  const bool ok = gi < n && gj < n && gi > gj;
  const C v = E[ok ? gi + (long)gj * n : 0];
  if (ok) {
    acc.re += v.re;
    acc.im += v.im;
  }
}

// Entry of rank r in anti-diagonal order (d = p - q from 31 down to -31, q
// increasing within a diagonal). Diagonals d >= 0 hold ranks 0..527.
__device__ inline void diag_rank(int r, int& p, int& q) {
  const bool upper = r < (TB * (TB + 1)) / 2;
  const int rr = upper ? r : TB * TB - 1 - r;
  int k = (int)((sqrtf(8.f * rr + 1.f) - 1.f) * 0.5f);
  while (k * (k + 1) / 2 > rr) k--;
  while ((k + 1) * (k + 2) / 2 <= rr) k++;
  const int i = rr - k * (k + 1) / 2;  // position within the diagonal
  if (upper) {
    const int d = TB - 1 - k;
    q = i;
    p = q + d;
  } else {
    const int d = -(TB - 1 - k);
    q = TB - 1 - i;
    p = q + d;
  }
}

// LDS layouts of the solve (elements):
//   TaP: T_II column-major, 63 columns of stride TLD, columns 32..62 zero, so that
//        Ta(p, q+s) is addressable for every q + s <= 62;
//   TbP: T_JJ (T_II on a diagonal tile) column-major with stride 64 and a row
//        offset of 31, rows -31..-1 zero, so that Tb(p-s, q) is addressable for
//        every p - s >= -31;
//   dv:  per step the finalized anti-diagonal by column, dv[32 + c] = X(c+s, c)
//        (0 where that entry does not exist), dv[0..31] = 0, so that X(p, p-s)
//        reads dv[32 + p - s] for every p - s >= -32.
constexpr int kTaCols = 2 * TB - 1;
constexpr int kTbLd = 2 * TB;
constexpr int kSolveS1 = kTaCols * TLD;  // elements of the first LDS buffer
constexpr int kSolveS2 = TB * kTbLd;     // elements of the second LDS buffer

// Solve T_II X - X T_JJ = -R (I > J) or stril(T_II X - X T_II) = -stril(R) (I = J)
// for the tile whose R (column ownership) is in acc; writes the tile of L.
//
// Threads take the entries in anti-diagonal order, so the entries of a wave lie
// on a few neighbouring anti-diagonals. Step s finalizes anti-diagonal p - q = s:
// its entries write x = -r / (ta_pp - tb_qq) to L and to dv (double-buffered by
// step parity); after one barrier every pending entry (p - q < s) adds the two
// contributions of that diagonal,
//   + Ta(p, q+s) X(q+s, q)   (entry below it in its column)
//   - X(p, p-s) Tb(p-s, q)   (entry left of it in its row)
// with operands that read as zero where the entry does not exist, and addresses
// that move by a constant per step. Waves whose entries are all final skip the
// update. Without truncation (TRUNC false) the finiteness of the entries is
// checked once after the loop, off the dependent chain of the steps.
// tii, tjj: this thread's elements (tile_val ownership) of T_II and T_JJ.
template <typename Rl, bool TRUNC>
__device__ void tile_solve(cplx<Rl> acc, cplx<Rl> tii, cplx<Rl> tjj, cplx<Rl>* L, int n, int I, int J,
                           float trunc, unsigned* status, cplx<Rl>* TaP, cplx<Rl>* TbP,
                           cplx<Rl>* R, Own o) {
  using C = cplx<Rl>;
  __shared__ C dv[2][2 * TB];
  __shared__ int wave_min_d[TNT / 64];
  const bool diag = (I == J);
  const C z = mk<Rl>(0, 0);
  __syncthreads();
  {
    // TaP columns 0..31 from T_II, 32..62 zero
    const int p = threadIdx.x & (TB - 1), c = threadIdx.x / TB;
    TaP[c * TLD + p] = tii;
    if (c < TB - 1) TaP[(TB + c) * TLD + p] = z;
    // TbP rows -31..31 of column c (offset 31), rows < 0 zero
    TbP[c * kTbLd + (TB - 1) + p] = tjj;
    if (p < TB - 1) TbP[c * kTbLd + p] = z;
    if (threadIdx.x < 2 * TB) {
      dv[0][threadIdx.x] = z;
      dv[1][threadIdx.x] = z;
    }
  }
  R[o.q * TLD + o.p] = acc;
  int p, q;
  diag_rank(threadIdx.x, p, q);
  const int d = p - q;
  const bool live = (I * TB + p < n) && (J * TB + q < n) && (!diag || d > 0);
  {
    int md = d;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) md = min(md, __shfl_xor(md, off, 64));
    if ((threadIdx.x & 63) == 0) wave_min_d[threadIdx.x >> 6] = md;
  }
  __syncthreads();
  C a = R[q * TLD + p];
  const int wmin = wave_min_d[threadIdx.x >> 6];
  bool bad = false;
  C rd = z;
  {
    const C ta = TaP[p * TLD + p], tb = TbP[q * kTbLd + (TB - 1) + q];
    const Rl dr = ta.re - tb.re, di = ta.im - tb.im;
    const Rl den = dr * dr + di * di;
    if (live && den == Rl(0)) bad = true;
    if (live) rd = mk<Rl>(dr / den, -di / den);
  }
  const Rl trunc2 = (Rl)trunc * (Rl)trunc;
  const int smin = diag ? 1 : -(TB - 1);
  const long gaddr = (I * TB + p) + (long)(J * TB + q) * n;
  // operand indices at s = TB - 1; per step: ta -= TLD, xb += 1, tb += 1
  int ta_i = (q + TB - 1) * TLD + p;
  int xb_i = TB + p - (TB - 1);
  int tb_i = q * kTbLd + p;
  const int r = threadIdx.x;  // column whose dv slot this thread clears when absent
  C xf = z;                   // this thread's entry of L once finalized
  // The loop touches LDS only: a global store inside it would make every barrier
  // (a workgroup release) wait for that store to complete.
  for (int s = TB - 1; s >= smin; s--) {
    C* cur = dv[s & 1];
    if (d == s) {
      C x = z;
      if (live) {
        x = cmul(a, rd);
        x.re = -x.re;
        x.im = -x.im;
        if constexpr (TRUNC) {
          bad |= !isfinite(x.re) || !isfinite(x.im);
          if (x.re * x.re + x.im * x.im > trunc2) x = z;
        }
      }
      xf = x;
      cur[TB + q] = x;
    }
    if (r < TB && (r + s > TB - 1 || r + s < 0)) cur[TB + r] = z;
    __syncthreads();
    if (wmin < s && d < s) {
      const C xa = cur[TB + q], xb = cur[xb_i];
      const C ta = TaP[ta_i], tb = TbP[tb_i];
      cfma(a, ta, xa);
      cfms(a, xb, tb);
    }
    ta_i -= TLD;
    xb_i += 1;
    tb_i += 1;
  }
  if constexpr (!TRUNC) bad |= !isfinite(xf.re) || !isfinite(xf.im);  // xf = 0 unless live
  if (live) L[gaddr] = xf;
  if (bad) atomicOr(status, (unsigned)DEV_BREAKDOWN);
}

// The truncating form only when the (FP32 or FP64) squared threshold is positive.
template <typename Rl>
__device__ inline void tile_solve_any(cplx<Rl> acc, cplx<Rl> tii, cplx<Rl> tjj, cplx<Rl>* L, int n, int I,
                                      int J, float trunc, unsigned* status, cplx<Rl>* TaP, cplx<Rl>* TbP,
                                      cplx<Rl>* R, Own o) {
  if ((Rl)trunc * (Rl)trunc > Rl(0))
    tile_solve<Rl, true>(acc, tii, tjj, L, n, I, J, trunc, status, TaP, TbP, R, o);
  else
    tile_solve<Rl, false>(acc, tii, tjj, L, n, I, J, trunc, status, TaP, TbP, R, o);
}

template <typename Rl>
struct TriLevelArgs {
  const cplx<Rl>* T;
  const cplx<Rl>* E;
  cplx<Rl>* L;
  int n, nb, D;
  int S_cur;         // partial blocks per tile that wrote diagonal D's far sums
  int S_next;        // partial blocks per tile for diagonal D - 1 (0: none)
  const cplx<Rl>* part_cur;  // [tiles(D)][S_cur][TB*TB]
  cplx<Rl>* part_next;       // [tiles(D-1)][S_next][TB*TB]
  unsigned* status;
  float trunc;
};

template <typename Rl>
__global__ __launch_bounds__(TNT) void trisolve_level_kernel(TriLevelArgs<Rl> a) {
  using C = cplx<Rl>;
  __shared__ C S1[kSolveS1], S2[kSolveS2], S3[TB * TLD];
  const Own o = owner();
  const int tiles = a.nb - a.D;
  C acc = mk<Rl>(0, 0);
  if ((int)blockIdx.x < tiles) {
    // solve block for tile (D + t, t). Every global operand is requested before
    // the first one is used (the partial sums in batches), so the block waits for
    // a few rounds of memory latency rather than one per operand; the sums are
    // still formed in the same order.
    const int t = blockIdx.x, I = a.D + t, J = t;
    const C ta = tile_val(a.T, a.n, I, I + 1), la = tile_val(a.L, a.n, I + 1, J);
    const C lb = tile_val(a.L, a.n, I, J - 1), tb = tile_val(a.T, a.n, J - 1, J);
    const C tii = tile_val(a.T, a.n, I, I), tjj = tile_val(a.T, a.n, J, J);
    // R = E_IJ (strictly lower part) + the far partial sums in order. The first
    // batch is loaded unconditionally (indices kept inside the partial buffer,
    // unused values not added) so that its loads overlap the ones above.
    const int gi = I * TB + o.p, gj = J * TB + o.q;
    const bool eok = gi < a.n && gj < a.n && gi > gj;
    const C ev = a.E[eok ? gi + (long)gj * a.n : 0];
    const C* part = a.part_cur + (long)t * a.S_cur * kTileElems + o.p + o.q * TB;
    constexpr int kBatch = 16;
    auto batch = [&](int s0) {
      C v[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; u++) v[u] = part[(long)max(0, min(s0 + u, a.S_cur - 1)) * kTileElems];
      if (s0 == 0) acc = keep(eok, ev);
#pragma unroll
      for (int u = 0; u < kBatch; u++) {
        if (s0 + u < a.S_cur) {
          acc.re += v[u].re;
          acc.im += v[u].im;
        }
      }
    };
    batch(0);
    for (int s0 = kBatch; s0 < a.S_cur; s0 += kBatch) batch(s0);
    if (I + 1 < a.nb) {
      S1[o.q * TLD + o.p] = ta;
      S2[o.q * TLD + o.p] = la;
      __syncthreads();
      tile_mac<+1>(acc, S1, S2, o);
    }
    if (J >= 1) {
      __syncthreads();
      S1[o.q * TLD + o.p] = lb;
      S2[o.q * TLD + o.p] = tb;
      __syncthreads();
      tile_mac<-1>(acc, S1, S2, o);
    }
    tile_solve_any(acc, tii, tjj, a.L, a.n, I, J, a.trunc, a.status, S1, S2, S3, o);
    return;
  }
  // partial block for diagonal D - 1: tile t2 = (D - 1 + t2, t2), split s
  const int b = blockIdx.x - tiles;
  const int t2 = b / a.S_next, s = b - (b / a.S_next) * a.S_next;
  const int I = a.D - 1 + t2, J = t2;
  const int fa = max(0, a.nb - 2 - I), fb = max(0, J - 1);
  const int m = fa + fb;
  const int u0 = (int)((long)m * s / a.S_next), u1 = (int)((long)m * (s + 1) / a.S_next);
  // far products: K = I+2..nb-1 (first kind), K = 0..J-2 (second kind)
  product_range(acc, a.T, a.L, a.n, I, J, I + 2, fa, u0, u1, S1, S2, o);
  a.part_next[((long)t2 * a.S_next + s) * kTileElems + o.p + o.q * TB] = acc;
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

// One block per matrix walks every tile diagonal; used for small n and batches.
template <typename Rl>
__global__ __launch_bounds__(TNT) void trisolve_single_kernel(const TriMatrix<Rl>* __restrict__ mats,
                                                              TriMatrix<Rl> one, unsigned* status,
                                                              float trunc) {
  using C = cplx<Rl>;
  __shared__ C S1[kSolveS1], S2[kSolveS2], S3[TB * TLD];
  const TriMatrix<Rl> mt = mats ? mats[blockIdx.x] : one;
  if (mt.active && *mt.active == 0) return;
  if (mt.flag) status = mt.flag;
  const int n = mt.n, nb = (n + TB - 1) / TB;
  const Own o = owner();
  for (int D = nb - 1; D >= 0; D--) {
    for (int t = 0; t < nb - D; t++) {
      const int I = D + t, J = t;
      C acc = mk<Rl>(0, 0);
      add_e(acc, mt.E, n, I, J, o);
      all_products(acc, mt.T, mt.L, n, nb, I, J, S1, S2, o);
      tile_solve_any(acc, tile_val(mt.T, n, I, I), tile_val(mt.T, n, J, J), mt.L, n, I, J, trunc, status,
                     S1, S2, S3, o);
    }
  }
}

// Far products per tile on diagonal D (the most of any tile there).
static int max_far(int nb, int D) {
  if (D < 0) return 0;
  const int m = nb - 1 - D;  // all products
  if (nb - D == 1) return 0;
  return m - 1;  // the first and last tile lack one near product
}

// Partial blocks per tile of diagonal D: about kProdsPerBlock far products each
// (a partial block then still ends before the solve blocks of the same launch,
// and few blocks share a CU with a solve block), but no more than kTargetBlocks
// in all, so that at large n every block carries more of the far products.
constexpr int kProdsPerBlock = 4;
static int splits(int nb, int D) {
  const int mf = max_far(nb, D);
  if (mf <= 0) return 0;
  int S = ceil_div(mf, kProdsPerBlock);
  const int cap = ceil_div(kTargetBlocks, nb - D);
  if (S > cap) S = cap;
  return S < 1 ? 1 : S;
}

// Partial-sum buffer of one parity, sized for complex128 (complex64 uses half).
static size_t part_bytes(int nb) {
  return (size_t)(kTargetBlocks + nb) * kTileElems * sizeof(zc);
}

size_t trisolve_ws_bytes(int n) {
  const int nb = ceil_div(n, TB);
  return 2 * part_bytes(nb);
}

template <typename Rl>
static hipError_t trisolve_t(const cplx<Rl>* T, const cplx<Rl>* E, cplx<Rl>* L, int n, float trunc,
                             void* ws, unsigned* status, hipStream_t st) {
  using C = cplx<Rl>;
  if (n <= 1) return fill_zero(L, (size_t)n * n * sizeof(C), st);
  const int nb = ceil_div(n, TB);
  hipError_t e = fill_zero(L, (size_t)n * n * sizeof(C), st);
  if (e != hipSuccess) return e;
  if (nb <= 2) {
    TriMatrix<Rl> one{T, E, L, n, nullptr, nullptr};
    hipLaunchKernelGGL(trisolve_single_kernel<Rl>, dim3(1), dim3(TNT), 0, st,
                       (const TriMatrix<Rl>*)nullptr, one, status, trunc);
    return hipGetLastError();
  }
  C* part[2] = {(C*)ws, (C*)((char*)ws + part_bytes(nb))};
  int S_cur = 0;  // the top diagonal has no far products
  for (int D = nb - 1; D >= 0; D--) {
    const int tiles = nb - D;
    const int S_next = D >= 1 ? splits(nb, D - 1) : 0;
    const int tiles_next = D >= 1 ? nb - D + 1 : 0;
    TriLevelArgs<Rl> a{T, E, L, n, nb, D, S_cur, S_next, part[D & 1], part[(D - 1) & 1], status, trunc};
    hipLaunchKernelGGL(trisolve_level_kernel<Rl>, dim3(tiles + tiles_next * S_next), dim3(TNT), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    S_cur = S_next;
  }
  return hipSuccess;
}

hipError_t trisolve(const cc* T, const cc* E, cc* L, int n, float trunc, void* ws,
                    unsigned* status, hipStream_t st) {
  return trisolve_t<float>(T, E, L, n, trunc, ws, status, st);
}

hipError_t trisolve64(const zc* T, const zc* E, zc* L, int n, void* ws, unsigned* status,
                      hipStream_t st) {
  return trisolve_t<double>(T, E, L, n, 0.f, ws, status, st);
}

// Batched FP32 solves: one block per matrix (entries of the device table `mats`);
// the strictly lower part of each L is written, the rest is left as it is.
hipError_t trisolve_batched(const void* mats, int count, float trunc, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(trisolve_single_kernel<float>, dim3(count), dim3(TNT), 0, st,
                     (const TriMatrix<float>*)mats, TriMatrix<float>{}, (unsigned*)nullptr, trunc);
  return hipGetLastError();
}

size_t trimatrix_bytes() { return sizeof(TriMatrix<float>); }
void trimatrix_fill(void* dst, const cc* T, const cc* E, cc* L, int n, const int* active,
                    unsigned* flag) {
  TriMatrix<float> m{T, E, L, n, active, flag};
  memcpy(dst, &m, sizeof(m));
}

}  // namespace sr
