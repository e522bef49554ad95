// Complex GEMM on CDNA4 matrix cores: FP64 MFMA (hp products of the refinement)
// and FP32 MFMA (its lp products), with the pass's elementwise steps fused into
// the epilogue.
//
// Tiling: a 512-thread block computes a 64 x 64 complex tile of C; its eight
// waves (2 along M x 4 along N) each own a 32 x 16 complex piece, i.e. 2 x 1
// blocks of 16 x 16, with separate real and imaginary accumulators. Every 16 x 16 x 4 step is four real
// MFMAs: re += a_re b_re - a_im b_im, im += a_re b_im + a_im b_re. op(A) and B
// tiles (K depth 16) are staged through LDS, double-buffered, with an XOR swizzle
// so that both the transposing stores and the fragment loads avoid bank
// conflicts. Complex values stay interleaved (re, im) so one 16-byte LDS read
// yields both parts of an operand.
//
// Compensated mode (FP64 only): two-level summation. The MFMA accumulators hold
// the sum of one chunk of kChunk K-tiles and are then added into a running total
// and cleared. For random-sign terms the rounding error of a length-K dot product
// drops from about u K / sqrt(2) to about u (K / sqrt(2 c) + sqrt(K c / 2)) with
// c = 16 kChunk terms per chunk: 4-6x smaller for K = 1024..4096, which brings the
// FP64 floor of ||stril(Q^H A Q)|| / ||A|| below 1e-15.
#include "epilogue.hpp"

namespace sr {

constexpr int GBM = 64, GBN = 64, GBK = 16, GNT = 512;
constexpr int kChunk = 2;  // K-tiles (32 complex terms) per chunk of the two-level sum

// Tile shapes: 64 x 64 with 512 threads (8 waves of 32 x 16) for the single
// products; the grouped products of a batch also have 32 x 32 with 256 threads
// (4 waves of 16 x 16) for small matrices.
template <int BM>
struct Shape {
  static constexpr int NT = BM == 64 ? 512 : 256;
  static constexpr int WM = BM == 64 ? 2 : 1;  // 16 x 16 blocks per wave along M
  static constexpr int WN = 1;                 // and along N
  static constexpr int LOADS = BM * GBK / NT;  // elements of each operand tile per thread
};

// LDS column swizzle: row k of a [GBK][BM] tile is permuted by XOR with 4 (k mod 16)
// (k mod 8 for 32 columns), which keeps the XOR inside the row.
template <int BM>
__device__ inline int swz(int k, int m) {
  return BM == 64 ? (m ^ ((k & 15) << 2)) : (m ^ ((k & 7) << 2));
}

// One output tile (m0, n0) of g; `slot` is the partial-sum slot of SPLIT / YDEF.
// Operand layout of v_mfma_*_16x16x4 (one block): lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; accumulator element v of lane l is D[MF<R>::row(l, v)][l % 16].
//
// KS > 1 splits K inside the block: the block has KS groups of NT threads, group
// g takes the K-tiles g, g + KS, g + 2 KS, ... with its own double-buffered
// operand tiles (As, Bs hold 2 KS buffers), and at the end the groups' sums are
// added in group order through LDS before group 0 stores the tile. A tile then
// keeps KS times the waves busy, which is what fills the CUs when there are
// fewer than two tiles per CU.
// K step after which the next K-tile is stored (of 0, 4, 8, 12). Measured against
// storing after the last step: 1-4% faster at n = 1024..4096 in FP64 and FP32.
constexpr int kStoreAt = 4;

template <typename R, int OPA, int EPI, int COMP, int BM, int KS = 1>
__device__ inline void gemm_tile(const GemmArgs& g, int m0, int n0, int slot,
                                 cplx<R> (*As)[GBK][BM], cplx<R> (*Bs)[GBK][BM], double* red) {
  using V = typename MF<R>::v4;
  using C = cplx<R>;
  using S = Shape<BM>;
  constexpr int WM = S::WM, WN = S::WN, NT = S::NT, kLoads = S::LOADS;
  const int grp = KS > 1 ? (int)threadIdx.x / NT : 0;
  const int tid = (int)threadIdx.x - grp * NT, lane = tid & 63, wave = tid >> 6;
  R* const xch = (R*)&As[0][0][0];  // the group exchange after the K loop
  As += 2 * grp;
  Bs += 2 * grp;
  const int wm = (wave & 1) * (16 * WM), wn = (wave >> 1) * (16 * WN);

  const C* __restrict__ Ap = (const C*)g.A;
  const C* __restrict__ Bp = (const C*)g.B;

  V acc_re[WM][WN], acc_im[WM][WN];
  V tot_re[WM][WN], tot_im[WM][WN];
#pragma unroll
  for (int a = 0; a < WM; a++)
#pragma unroll
    for (int b = 0; b < WN; b++)
#pragma unroll
      for (int v = 0; v < 4; v++) {
        acc_re[a][b][v] = 0;
        acc_im[a][b][v] = 0;
        tot_re[a][b][v] = 0;
        tot_im[a][b][v] = 0;
      }

  C ra[kLoads], rb[kLoads];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < kLoads; r++) {
      const int idx = r * NT + tid;
      int mm, kk;
      if (OPA == 0) {
        mm = idx & (BM - 1);
        kk = idx / BM;
      } else {
        kk = idx & 15;
        mm = idx >> 4;
      }
      const int gm = m0 + mm, gk = k0 + kk;
      C v = mk<R>(0, 0);
      if (gm < g.m && gk < g.k) {
        v = OPA == 0 ? Ap[gm + (long)gk * g.lda] : Ap[gk + (long)gm * g.lda];
        if (OPA) v.im = -v.im;
      }
      ra[r] = v;
      const int bk = idx & 15, bn = idx >> 4;
      const int gn = n0 + bn, gkb = k0 + bk;
      C w = mk<R>(0, 0);
      if (gn < g.n && gkb < g.k) w = Bp[gkb + (long)gn * g.ldb];
      rb[r] = w;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < kLoads; r++) {
      const int idx = r * NT + tid;
      int mm, kk;
      if (OPA == 0) {
        mm = idx & (BM - 1);
        kk = idx / BM;
      } else {
        kk = idx & 15;
        mm = idx >> 4;
      }
      As[buf][kk][swz<BM>(kk, mm)] = ra[r];
      const int bk = idx & 15, bn = idx >> 4;
      Bs[buf][bk][swz<BM>(bk, bn)] = rb[r];
    }
  };
  auto fold = [&]() {
    if constexpr (COMP) {
#pragma unroll
      for (int a = 0; a < WM; a++)
#pragma unroll
        for (int b = 0; b < WN; b++) {
          tot_re[a][b] += acc_re[a][b];
          tot_im[a][b] += acc_im[a][b];
#pragma unroll
          for (int v = 0; v < 4; v++) {
            acc_re[a][b][v] = 0;
            acc_im[a][b][v] = 0;
          }
        }
    }
  };

  // This group's K-tiles are kt = i KS + grp, i < iters; a K-tile past the end loads
  // zeros, which add nothing.
  const int KT = (g.k + GBK - 1) / GBK;
  const int iters = (KT + KS - 1) / KS;
  gload(grp * GBK);
  sstore(0);
  __syncthreads();
  for (int it = 0; it < iters; it++) {
    const int cur = it & 1;
    if (it + 1 < iters) gload(((it + 1) * KS + grp) * GBK);
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 4) {
      const int krow = kk + (lane >> 4);
      R a_re[WM], a_im[WM], na_im[WM], b_re[WN], b_im[WN];
#pragma unroll
      for (int mi = 0; mi < WM; mi++) {
        const C v = As[cur][krow][swz<BM>(krow, wm + mi * 16 + (lane & 15))];
        a_re[mi] = v.re;
        a_im[mi] = v.im;
        na_im[mi] = -v.im;
      }
#pragma unroll
      for (int ni = 0; ni < WN; ni++) {
        const C v = Bs[cur][krow][swz<BM>(krow, wn + ni * 16 + (lane & 15))];
        b_re[ni] = v.re;
        b_im[ni] = v.im;
      }
      // The two products that accumulate into one register are issued 2 WM WN
      // MFMAs apart, so a dependent MFMA does not wait for its predecessor.
#pragma unroll
      for (int mi = 0; mi < WM; mi++)
#pragma unroll
        for (int ni = 0; ni < WN; ni++) {
          acc_re[mi][ni] = MF<R>::op(a_re[mi], b_re[ni], acc_re[mi][ni]);
          acc_im[mi][ni] = MF<R>::op(a_re[mi], b_im[ni], acc_im[mi][ni]);
        }
#pragma unroll
      for (int mi = 0; mi < WM; mi++)
#pragma unroll
        for (int ni = 0; ni < WN; ni++) {
          acc_re[mi][ni] = MF<R>::op(na_im[mi], b_im[ni], acc_re[mi][ni]);
          acc_im[mi][ni] = MF<R>::op(a_im[mi], b_re[ni], acc_im[mi][ni]);
        }
      // The next K-tile goes to the other buffer (free since the last barrier)
      // while this one's products are still in the matrix pipe, so that the LDS
      // stores of the waves overlap other waves' MFMAs instead of the barrier.
      if (kk == kStoreAt && it + 1 < iters) sstore(cur ^ 1);
    }
    if (COMP && ((it + 1) % kChunk == 0 || it + 1 == iters)) fold();
    __syncthreads();
  }

  V(&fin_re)[WM][WN] = COMP ? tot_re : acc_re;
  V(&fin_im)[WM][WN] = COMP ? tot_im : acc_im;
  if constexpr (KS > 1) {
    // groups 1.. add their sums into group 0's, one group at a time (the operand
    // buffers are free after the loop's last barrier)
    constexpr int kVals = WM * WN * 4;
    static_assert(kVals * 2 * NT * sizeof(R) <= 2 * KS * GBK * BM * sizeof(C), "exchange fits in As");
    for (int src = 1; src < KS; src++) {
      if (grp == src) {
#pragma unroll
        for (int a = 0; a < WM; a++)
#pragma unroll
          for (int b = 0; b < WN; b++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
              const int e = (a * WN + b) * 4 + v;
              xch[(2 * e) * NT + tid] = fin_re[a][b][v];
              xch[(2 * e + 1) * NT + tid] = fin_im[a][b][v];
            }
      }
      __syncthreads();
      if (grp == 0) {
#pragma unroll
        for (int a = 0; a < WM; a++)
#pragma unroll
          for (int b = 0; b < WN; b++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
              const int e = (a * WN + b) * 4 + v;
              fin_re[a][b][v] += xch[(2 * e) * NT + tid];
              fin_im[a][b][v] += xch[(2 * e + 1) * NT + tid];
            }
      }
      __syncthreads();
    }
  }

  // Epilogue (group 0).
  double part = 0;
  if (grp == 0) {
#pragma unroll
    for (int mi = 0; mi < WM; mi++)
#pragma unroll
      for (int ni = 0; ni < WN; ni++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
          const int i = m0 + wm + mi * 16 + MF<R>::row(lane, v);
          const int j = n0 + wn + ni * 16 + (lane & 15);
          C val;
          val.re = fin_re[mi][ni][v];
          val.im = fin_im[mi][ni][v];
          if (i < g.m && j < g.n) epi_element<EPI, R>(g, i, j, val, part);
        }
  }
  if constexpr (EPI == EPI_SPLIT || EPI == EPI_YDEF) epi_reduce<NT * KS>(g, part, red, slot);
}

template <typename R, int OPA, int EPI, int COMP, int KS>
__global__ __launch_bounds__(GNT * KS) void gemm_kernel(GemmArgs g) {
  __shared__ cplx<R> As[2 * KS][GBK][GBM];
  __shared__ cplx<R> Bs[2 * KS][GBK][GBN];
  __shared__ double red[GNT * KS / 64];
  // Blocks are dispatched round-robin over the XCDs (block b on XCD b mod 8):
  // give each XCD a contiguous run of logical tiles, then walk tiles in groups of
  // kGroup tile-rows so that concurrently running blocks share A rows and B columns
  // in their XCD's L2.
  const int ntiles = gridDim.x;
  const int bid = blockIdx.x;
  int logical = bid;
  {
    const int per = ntiles / kXCDs;
    if (bid < per * kXCDs) logical = (bid % kXCDs) * per + bid / kXCDs;
  }
  int tm, tn;
  if ((EPI == EPI_YDEF || EPI == EPI_STORE) && g.herm) {
    herm_tile(logical, g.tiles_n, tm, tn);  // the upper triangle of tiles
  } else {
    constexpr int kGroup = 4;
    const int group = logical / (kGroup * g.tiles_n);
    const int first_m = group * kGroup;
    const int gsize = min(g.tiles_m - first_m, kGroup);
    const int within = logical - group * kGroup * g.tiles_n;
    tm = first_m + within % gsize;
    tn = within / gsize;
  }
  gemm_tile<R, OPA, EPI, COMP, GBM, KS>(g, tm * GBM, tn * GBN, bid, As, Bs, red);
}

// Grouped product over many matrices: a persistent grid walks a table of output
// tiles (matrix, m0, n0, partial slot); tiles of matrices whose `active` flag is 0
// are skipped, so a captured sequence can keep running while matrices finish.
template <typename R, int OPA, int EPI, int COMP, int BM>
__global__ __launch_bounds__(Shape<BM>::NT) void gemm_grouped_kernel(const GemmArgs* __restrict__ args,
                                                                     const GTile* __restrict__ tiles,
                                                                     int ntiles,
                                                                     const int* __restrict__ active) {
  __shared__ cplx<R> As[2][GBK][BM];
  __shared__ cplx<R> Bs[2][GBK][BM];
  __shared__ double red[Shape<BM>::NT / 64];
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const GTile d = tiles[t];
    if (active && !active[d.mat]) continue;
    const GemmArgs g = args[d.mat];
    gemm_tile<R, OPA, EPI, COMP, BM>(g, d.m0, d.n0, d.slot, As, Bs, red);
  }
}

int gemm_tiles(int m, int n) { return ceil_div(m, GBM) * ceil_div(n, GBN); }
int gemm_tiles_herm(int n) {
  const int t = ceil_div(n, GBM);
  return t * (t + 1) / 2;
}

template <typename R, int OPA, int EPI, int COMP>
static hipError_t launch(GemmArgs g, hipStream_t st) {
  g.tiles_m = ceil_div(g.m, GBM);
  g.tiles_n = ceil_div(g.n, GBN);
  if (g.herm && (g.m != g.n || !(EPI == EPI_STORE || (EPI == EPI_YDEF && g.herm == 1))))
    return hipErrorInvalidValue;
  const int nt = g.herm ? gemm_tiles_herm(g.n) : g.tiles_m * g.tiles_n;
  if (nt == 0) return hipSuccess;
  // Split K inside the block (KS = 2) when there are fewer than two tiles per CU, so
  // that a CU still runs four waves per SIMD, and for the compensated form, whose
  // registers (about 137 per thread) otherwise leave room for one 8-wave block per CU.
  // Measured at n = 1024 / 2048 / 4096: compensated 59 -> 62%, 64 -> 65%, 67 -> 71% of
  // peak; plain products at n = 4096 are faster unsplit (77% against 73%).
  const bool split = COMP || nt < 2 * kCUs;
  if (split)
    hipLaunchKernelGGL((gemm_kernel<R, OPA, EPI, COMP, 2>), dim3(nt), dim3(2 * GNT), 0, st, g);
  else
    hipLaunchKernelGGL((gemm_kernel<R, OPA, EPI, COMP, 1>), dim3(nt), dim3(GNT), 0, st, g);
  return hipGetLastError();
}

hipError_t zgemm(int opa, int epi, int comp, const GemmArgs& g, hipStream_t st) {
#define SR_Z(OPA, EPI)                                                     \
  if (opa == OPA && epi == EPI) {                                          \
    return comp ? launch<double, OPA, EPI, 1>(g, st) : launch<double, OPA, EPI, 0>(g, st); \
  }
  SR_Z(0, EPI_STORE)
  SR_Z(0, EPI_ADD)
  SR_Z(0, EPI_SPLIT)
  SR_Z(0, EPI_YDEF)
  SR_Z(1, EPI_STORE)
  SR_Z(1, EPI_ADD)
  SR_Z(1, EPI_SPLIT)
  SR_Z(1, EPI_YDEF)
#undef SR_Z
  return hipErrorInvalidValue;
}

hipError_t cgemm(const GemmArgs& g, hipStream_t st) { return launch<float, 0, EPI_STORE, 0>(g, st); }

template <typename R, int OPA, int EPI, int COMP, int BM>
static hipError_t launch_grouped(const GemmArgs* args, const GTile* tiles, int ntiles,
                                 const int* active, int grid, hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL((gemm_grouped_kernel<R, OPA, EPI, COMP, BM>), dim3(grid), dim3(Shape<BM>::NT), 0, st,
                     args, tiles, ntiles, active);
  return hipGetLastError();
}

hipError_t zgemm_grouped(int opa, int epi, int comp, int bm, const GemmArgs* args, const GTile* tiles,
                         int ntiles, const int* active, int grid, hipStream_t st) {
#define SR_G(OPA, EPI, BM)                                                                  \
  if (opa == OPA && epi == EPI && bm == BM) {                                               \
    return comp ? launch_grouped<double, OPA, EPI, 1, BM>(args, tiles, ntiles, active, grid, st) \
                : launch_grouped<double, OPA, EPI, 0, BM>(args, tiles, ntiles, active, grid, st); \
  }
  SR_G(0, EPI_STORE, 64)
  SR_G(0, EPI_ADD, 64)
  SR_G(0, EPI_SPLIT, 64)
  SR_G(0, EPI_YDEF, 64)
  SR_G(1, EPI_YDEF, 64)
  SR_G(0, EPI_STORE, 32)
  SR_G(0, EPI_ADD, 32)
  SR_G(0, EPI_SPLIT, 32)
  SR_G(0, EPI_YDEF, 32)
  SR_G(1, EPI_YDEF, 32)
#undef SR_G
  return hipErrorInvalidValue;
}

hipError_t cgemm_grouped_add(int bm, const GemmArgs* args, const GTile* tiles, int ntiles, int grid,
                             hipStream_t st) {
  if (bm == 64) return launch_grouped<float, 0, EPI_ADD, 0, 64>(args, tiles, ntiles, nullptr, grid, st);
  if (bm == 32) return launch_grouped<float, 0, EPI_ADD, 0, 32>(args, tiles, ntiles, nullptr, grid, st);
  return hipErrorInvalidValue;
}

hipError_t cgemm_grouped(int bm, const GemmArgs* args, const GTile* tiles, int ntiles, const int* active,
                         int grid, hipStream_t st) {
  if (bm == 64) return launch_grouped<float, 0, EPI_STORE, 0, 64>(args, tiles, ntiles, active, grid, st);
  if (bm == 32) return launch_grouped<float, 0, EPI_STORE, 0, 32>(args, tiles, ntiles, active, grid, st);
  return hipErrorInvalidValue;
}

}  // namespace sr
