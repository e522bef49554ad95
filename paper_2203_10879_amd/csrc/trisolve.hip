// Triangular matrix equation stril(T L - L T) = -E in FP32 (Section 2.1,
// eqs. (7)-(10)): the low-precision solve of every refinement pass.
//
// Entry (i, j), i > j, reads
//   l_ij = -( e_ij + sum_{k>i} t_ik l_kj - sum_{k<j} l_ik t_kj ) / (t_ii - t_jj),
// so an entry needs the entries below it in its column and left of it in its row:
// entries on one subdiagonal i - j = d are independent (the wavefront order the
// paper mentions after Theorem 1).
//
// GPU schedule. L is cut into 32 x 32 tiles. For a tile (I, J), I >= J, the
// same algebra at tile level gives
//   T_II X - X T_JJ = -R_IJ,  R_IJ = E_IJ + sum_{K>I} T_IK L_KJ - sum_{K<J} L_IK T_KJ
// (for I = J only the strictly lower part, with X strictly lower): a tile depends
// on the tiles below it in its tile column and left of it in its tile row, so the
// tiles of one tile diagonal D = I - J are independent. One launch per tile
// diagonal, D = nb-1 down to 0:
//   1. the nb-1-D block products of every tile of the diagonal are split over
//      S blocks (S chosen to fill the chip), each writing its partial sum;
//   2. the last block of a tile to finish (arrival counter after a device fence;
//      no block ever waits) adds E_IJ and the partials in a fixed order and
//      solves the tile by substitution along its anti-diagonals (63 dependent
//      steps; 31 for a diagonal tile), keeping T_II, T_JJ and X in LDS.
// Small matrices (and the batched path) use one block that walks all tiles.
#include "kernels.hpp"

namespace sr {

constexpr int TB = 32;
constexpr int TNT = 256;
constexpr int TLD = TB + 1;
constexpr int kTargetBlocks = 2 * kCUs;

struct Own {
  int q, p0;  // this thread owns entries (p0 + c, q), c = 0..3, of a tile
};
__device__ inline Own owner() {
  Own o;
  o.q = threadIdx.x >> 3;
  o.p0 = (threadIdx.x & 7) * 4;
  return o;
}

// LDS tile, column-major with padded stride: S[q * TLD + p] = G(I*TB + p, J*TB + q).
__device__ inline void load_tile(cc* S, const cc* __restrict__ G, int n, int I, int J) {
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int idx = r * TNT + threadIdx.x;
    const int p = idx & (TB - 1), q = idx >> 5;
    const int gi = I * TB + p, gj = J * TB + q;
    S[q * TLD + p] = (gi < n && gj < n) ? G[gi + (long)gj * n] : mk<float>(0.f, 0.f);
  }
}

template <int SIGN>
__device__ inline void tile_mac(cc acc[4], const cc* F, const cc* G, Own o) {
#pragma unroll 8
  for (int k = 0; k < TB; k++) {
    const cc b = G[o.q * TLD + k];
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const cc a = F[k * TLD + o.p0 + c];
      if (SIGN > 0) cfma(acc[c], a, b);
      else cfms(acc[c], a, b);
    }
  }
}

// acc += sum of block products number u0..u1-1 of tile (I, J): the first
// nb-1-I are + T_IK L_KJ (K = I+1..nb-1), the rest - L_IK T_KJ (K = 0..J-1).
__device__ void tile_products(cc acc[4], const cc* T, const cc* L, int n, int nb, int I, int J,
                              int u0, int u1, cc* S1, cc* S2, Own o) {
  const int mA = nb - 1 - I;
  for (int u = u0; u < u1; u++) {
    __syncthreads();
    if (u < mA) {
      const int K = I + 1 + u;
      load_tile(S1, T, n, I, K);
      load_tile(S2, L, n, K, J);
    } else {
      const int K = u - mA;
      load_tile(S1, L, n, I, K);
      load_tile(S2, T, n, K, J);
    }
    __syncthreads();
    if (u < mA) tile_mac<+1>(acc, S1, S2, o);
    else tile_mac<-1>(acc, S1, S2, o);
  }
}

__device__ inline void add_e(cc acc[4], const cc* __restrict__ E, int n, int I, int J, Own o) {
  const int gj = J * TB + o.q;
#pragma unroll
  for (int c = 0; c < 4; c++) {
    const int gi = I * TB + o.p0 + c;
    if (gi < n && gj < n && gi > gj) {
      const cc e = E[gi + (long)gj * n];
      acc[c].re += e.re;
      acc[c].im += e.im;
    }
  }
}

// Solve T_II X - X T_JJ = -R (I > J) or stril(T_II X - X T_II) = -stril(R) (I = J)
// for the tile whose R is in acc; writes the tile of L.
__device__ void tile_solve(cc acc[4], const cc* T, cc* L, int n, int I, int J, float trunc,
                           unsigned* status, cc* Ta, cc* Tb, cc* X, Own o) {
  const bool diag = (I == J);
  __syncthreads();
  load_tile(Ta, T, n, I, I);
  if (!diag) load_tile(Tb, T, n, J, J);
  for (int r = threadIdx.x; r < TB * TLD; r += TNT) X[r] = mk<float>(0.f, 0.f);
  __syncthreads();
  const cc* B = diag ? Ta : Tb;
  const int q = o.q;
  cc rd[4];
  bool live[4];
  bool bad = false;
#pragma unroll
  for (int c = 0; c < 4; c++) {
    const int p = o.p0 + c;
    live[c] = (I * TB + p < n) && (J * TB + q < n) && (!diag || p > q);
    rd[c] = mk<float>(0.f, 0.f);
    if (live[c]) {
      const cc ta = Ta[p * TLD + p], tb = B[q * TLD + q];
      const float dr = ta.re - tb.re, di = ta.im - tb.im;
      const float den = dr * dr + di * di;
      if (den == 0.f) bad = true;
      rd[c] = mk<float>(dr / den, -di / den);
    }
  }
  const int smin = diag ? 1 : -(TB - 1);
  for (int s = TB - 1; s >= smin; s--) {
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const int p = o.p0 + c;
      if (live[c] && p - q == s) {
        cc x = cmul(acc[c], rd[c]);
        x.re = -x.re;
        x.im = -x.im;
        if (!isfinite(x.re) || !isfinite(x.im)) bad = true;
        if (trunc > 0.f && x.re * x.re + x.im * x.im > trunc * trunc) x = mk<float>(0.f, 0.f);
        X[q * TLD + p] = x;
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const int p = o.p0 + c;
      if (live[c] && p - q < s) {
        const int p2 = q + s;  // finalized entry (p2, q) below in this column
        if (p2 < TB && p2 > p) cfma(acc[c], Ta[p2 * TLD + p], X[q * TLD + p2]);
        const int r = p - s;   // finalized entry (p, r) left in this row
        if (r >= 0 && r < q) cfms(acc[c], X[r * TLD + p], B[q * TLD + r]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int idx = r * TNT + threadIdx.x;
    const int p = idx & (TB - 1), qq = idx >> 5;
    const int gi = I * TB + p, gj = J * TB + qq;
    if (gi < n && gj < n) L[gi + (long)gj * n] = X[qq * TLD + p];
  }
  if (bad) atomicOr(status, (unsigned)DEV_BREAKDOWN);
}

struct TriLevelArgs {
  const cc* T;
  const cc* E;
  cc* L;
  int n, nb, D, S;
  cc* partial;
  unsigned* counters;
  unsigned* status;
  float trunc;
};

__global__ __launch_bounds__(TNT) void trisolve_level_kernel(TriLevelArgs a) {
  __shared__ cc S1[TB * TLD], S2[TB * TLD], S3[TB * TLD];
  __shared__ unsigned is_last;
  const int t = blockIdx.x / a.S, s = blockIdx.x - (blockIdx.x / a.S) * a.S;
  const int I = a.D + t, J = t;
  const Own o = owner();
  const int m = a.nb - 1 - a.D;
  cc acc[4];
#pragma unroll
  for (int c = 0; c < 4; c++) acc[c] = mk<float>(0.f, 0.f);
  const int u0 = (int)((long)m * s / a.S), u1 = (int)((long)m * (s + 1) / a.S);
  tile_products(acc, a.T, a.L, a.n, a.nb, I, J, u0, u1, S1, S2, o);
  if (a.S > 1) {
    cc* slot = a.partial + ((long)t * a.S + s) * (TB * TB);
#pragma unroll
    for (int c = 0; c < 4; c++) slot[(o.p0 + c) + o.q * TB] = acc[c];
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned prev = atomicAdd(&a.counters[t], 1u);
      is_last = (prev == (unsigned)(a.S - 1)) ? 1u : 0u;
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    if (threadIdx.x == 0) a.counters[t] = 0u;
#pragma unroll
    for (int c = 0; c < 4; c++) acc[c] = mk<float>(0.f, 0.f);
    add_e(acc, a.E, a.n, I, J, o);
    for (int s2 = 0; s2 < a.S; s2++) {
      const cc* sl = a.partial + ((long)t * a.S + s2) * (TB * TB);
#pragma unroll
      for (int c = 0; c < 4; c++) {
        const cc v = sl[(o.p0 + c) + o.q * TB];
        acc[c].re += v.re;
        acc[c].im += v.im;
      }
    }
  } else {
    add_e(acc, a.E, a.n, I, J, o);
  }
  tile_solve(acc, a.T, a.L, a.n, I, J, a.trunc, a.status, S1, S2, S3, o);
}

struct TriMatrix {
  const cc* T;
  const cc* E;
  cc* L;
  int n;
};

// One block per matrix walks every tile diagonal; used for small n and batches.
__global__ __launch_bounds__(TNT) void trisolve_single_kernel(const TriMatrix* __restrict__ mats,
                                                              TriMatrix one, unsigned* status,
                                                              float trunc) {
  __shared__ cc S1[TB * TLD], S2[TB * TLD], S3[TB * TLD];
  const TriMatrix mt = mats ? mats[blockIdx.x] : one;
  const int n = mt.n, nb = (n + TB - 1) / TB;
  const Own o = owner();
  for (int D = nb - 1; D >= 0; D--) {
    for (int t = 0; t < nb - D; t++) {
      const int I = D + t, J = t;
      cc acc[4];
#pragma unroll
      for (int c = 0; c < 4; c++) acc[c] = mk<float>(0.f, 0.f);
      add_e(acc, mt.E, n, I, J, o);
      tile_products(acc, mt.T, mt.L, n, nb, I, J, 0, nb - 1 - D, S1, S2, o);
      tile_solve(acc, mt.T, mt.L, n, I, J, trunc, status, S1, S2, S3, o);
    }
  }
}

size_t trisolve_ws_bytes(int n) {
  const int nb = ceil_div(n, TB);
  const size_t counters = ((size_t)nb * 4 + 255) / 256 * 256;
  const size_t parts = (size_t)(kTargetBlocks + nb) * TB * TB * sizeof(cc);
  return counters + parts;
}

hipError_t trisolve(const cc* T, const cc* E, cc* L, int n, float trunc, void* ws,
                    unsigned* status, hipStream_t st) {
  if (n <= 1) return fill_zero(L, (size_t)n * n * sizeof(cc), st);
  const int nb = ceil_div(n, TB);
  hipError_t e = fill_zero(L, (size_t)n * n * sizeof(cc), st);
  if (e != hipSuccess) return e;
  if (nb <= 2) {
    TriMatrix one{T, E, L, n};
    hipLaunchKernelGGL(trisolve_single_kernel, dim3(1), dim3(TNT), 0, st,
                       (const TriMatrix*)nullptr, one, status, trunc);
    return hipGetLastError();
  }
  const size_t counters_bytes = ((size_t)nb * 4 + 255) / 256 * 256;
  unsigned* counters = (unsigned*)ws;
  cc* partial = (cc*)((char*)ws + counters_bytes);
  e = fill_zero(counters, counters_bytes, st);
  if (e != hipSuccess) return e;
  for (int D = nb - 1; D >= 0; D--) {
    const int tiles = nb - D, m = nb - 1 - D;
    int S = ceil_div(kTargetBlocks, tiles);
    if (S > m) S = m;
    if (S < 1) S = 1;
    TriLevelArgs a{T, E, L, n, nb, D, S, partial, counters, status, trunc};
    hipLaunchKernelGGL(trisolve_level_kernel, dim3(tiles * S), dim3(TNT), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace sr
