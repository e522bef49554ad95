// Kernels of the real Schur variant (Section 3 extends the method to the real Schur
// form, whose factor T is quasi-triangular with 2 x 2 diagonal blocks for complex
// conjugate pairs): real products on FP64 / FP32 MFMA with the pass's elementwise
// steps fused into their epilogues, the elementwise steps, and the block solve.
//
// Blocks. blk[i] = 1 marks a 2 x 2 diagonal block at rows and columns i, i + 1. The
// block strictly lower part of a matrix is every (i, j), i > j, except the
// subdiagonal entry of a 2 x 2 block; T keeps the rest.
//
// The block solve. For a 2 x 2 block B = T_II (complex pair lambda, conj(lambda)) a
// unitary U_I with U_I^H B U_I upper triangular has the eigenvector of lambda as its
// first column; U = diag(U_I) (1 on 1 x 1 blocks) turns T into the upper triangular
// T_c = U^H T U and the block strictly lower E into E_c = U^H E U. For blocks I > J
// the equations of (T_c, E_c, U^H L U) are those of (T, E, L) in the new basis, and
// they involve no entry inside a diagonal block, so the scalar solve of
// stril(T_c L_c - L_c T_c) = -E_c (the complex sweep) gives L_c on every off-diagonal
// block, and L = U L_c U^H there (real up to rounding; its real part is taken), 0 on
// the diagonal blocks.
#include <type_traits>

#include "epilogue.hpp"
#include "real.hpp"

namespace sr {

// ----------------------------------------------------------------- products

constexpr int RBM = 64, RBK = 16, RNT = 256, RPAD = 16;
constexpr int kRChunk = 2;  // K-tiles per chunk of the two-level (compensated) sum

// whether (i, j) lies in the block strictly lower part
__device__ inline bool rlow(int i, int j, const int* __restrict__ blk) {
  return i > j && !(i == j + 1 && blk && blk[j]);
}

template <int EPI, typename R>
__device__ inline void repi(const RGemmArgs& g, int i, int j, R val, double& part) {
  R* __restrict__ C = (R*)g.C;
  const long o = i + (long)j * g.ldc;
  if constexpr (EPI == EPI_STORE) {
    if (g.herm) {
      if (i > j) return;  // the mirror of (j, i) is stored there
      if (i < j) C[j + (long)i * g.ldc] = g.herm > 0 ? val : -val;
    }
    C[o] = val;
  } else if constexpr (EPI == EPI_ADD) {
    const R r = ((const R*)g.Cin)[i + (long)j * g.ldcin] + val;
    C[o] = r;
    if (g.CT) ((R*)g.CT)[j + (long)i * g.ldct] = r;
  } else if constexpr (EPI == EPI_SPLIT) {
    const long ol = i + (long)j * g.ldlp;
    if (!rlow(i, j, g.blk)) {
      C[o] = val;
      g.Tlp[ol] = (float)val;
      g.Elp[ol] = 0.f;
    } else {
      C[o] = R(0);
      g.Tlp[ol] = 0.f;
      g.Elp[ol] = (float)val;
      part += (double)val * val;
    }
  } else {  // EPI_YDEF: Y = acc - I (symmetric with herm: the upper tiles mirrored)
    if (g.herm && i > j) return;
    if (i == j) val -= R(1);
    C[o] = val;
    part += (double)val * val;
    if (g.herm && i < j) {
      C[j + (long)i * g.ldc] = val;
      part += (double)val * val;
    }
  }
}

// A 256-thread block computes a 64 x 64 tile; each wave a 32 x 32 quarter as 2 x 2
// blocks of 16 x 16 on v_mfma_*_16x16x4 (lane l supplies op(A)[l % 16][l / 16] and
// B[l / 16][l % 16]). K-tiles of 16 pass through LDS, double-buffered; rows are
// padded by 16 elements so that the four K-rows a fragment read touches fall on
// different banks. COMP: the accumulators hold one chunk of kRChunk K-tiles and are
// then added to running totals (two-level summation, as in the complex product).
template <typename R, int OPA, int EPI, int COMP>
__global__ __launch_bounds__(RNT) void rgemm_kernel(RGemmArgs g) {
  using V = typename MF<R>::v4;
  __shared__ R As[2][RBK][RBM + RPAD];
  __shared__ R Bs[2][RBK][RBM + RPAD];
  __shared__ double red[RNT / 64];
  const int ntiles = gridDim.x, bid = blockIdx.x;
  int logical = bid;
  {
    const int per = ntiles / kXCDs;
    if (bid < per * kXCDs) logical = (bid % kXCDs) * per + bid / kXCDs;
  }
  int tm, tn;
  if ((EPI == EPI_YDEF || EPI == EPI_STORE) && g.herm) {
    herm_tile(logical, g.tiles_n, tm, tn);
  } else {
    constexpr int kGroup = 4;
    const int group = logical / (kGroup * g.tiles_n);
    const int first_m = group * kGroup;
    const int gsize = min(g.tiles_m - first_m, kGroup);
    const int within = logical - group * kGroup * g.tiles_n;
    tm = first_m + within % gsize;
    tn = within / gsize;
  }
  const int m0 = tm * RBM, n0 = tn * RBM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const R* __restrict__ Ap = (const R*)g.A;
  const R* __restrict__ Bp = (const R*)g.B;

  V acc[2][2], tot[2][2];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int v = 0; v < 4; v++) acc[a][b][v] = tot[a][b][v] = 0;

  constexpr int kLoads = RBM * RBK / RNT;  // 4 elements of each operand per thread
  R ra[kLoads], rb[kLoads];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < kLoads; r++) {
      const int idx = r * RNT + tid;
      int mm, kk;
      if (OPA == 0) {
        mm = idx & (RBM - 1);
        kk = idx / RBM;
      } else {
        kk = idx & (RBK - 1);
        mm = idx / RBK;
      }
      const int gm = m0 + mm, gk = k0 + kk;
      R v = 0;
      if (gm < g.m && gk < g.k) v = OPA == 0 ? Ap[gm + (long)gk * g.lda] : Ap[gk + (long)gm * g.lda];
      ra[r] = v;
      const int bk = idx & (RBK - 1), bn = idx / RBK;
      const int gn = n0 + bn, gkb = k0 + bk;
      R w = 0;
      if (gn < g.n && gkb < g.k) w = Bp[gkb + (long)gn * g.ldb];
      rb[r] = w;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < kLoads; r++) {
      const int idx = r * RNT + tid;
      int mm, kk;
      if (OPA == 0) {
        mm = idx & (RBM - 1);
        kk = idx / RBM;
      } else {
        kk = idx & (RBK - 1);
        mm = idx / RBK;
      }
      As[buf][kk][mm] = ra[r];
      Bs[buf][idx & (RBK - 1)][idx / RBK] = rb[r];
    }
  };

  const int KT = (g.k + RBK - 1) / RBK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < KT; kt++) {
    const int cur = kt & 1;
    if (kt + 1 < KT) gload((kt + 1) * RBK);
#pragma unroll
    for (int kk = 0; kk < RBK; kk += 4) {
      const int krow = kk + (lane >> 4);
      R a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; x++) a[x] = As[cur][krow][wm + 16 * x + (lane & 15)];
#pragma unroll
      for (int y = 0; y < 2; y++) b[y] = Bs[cur][krow][wn + 16 * y + (lane & 15)];
#pragma unroll
      for (int x = 0; x < 2; x++)
#pragma unroll
        for (int y = 0; y < 2; y++) acc[x][y] = MF<R>::op(a[x], b[y], acc[x][y]);
    }
    if (kt + 1 < KT) sstore(cur ^ 1);
    if (COMP && ((kt + 1) % kRChunk == 0 || kt + 1 == KT)) {
#pragma unroll
      for (int x = 0; x < 2; x++)
#pragma unroll
        for (int y = 0; y < 2; y++) {
          tot[x][y] += acc[x][y];
#pragma unroll
          for (int v = 0; v < 4; v++) acc[x][y][v] = 0;
        }
    }
    __syncthreads();
  }
  double part = 0;
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++)
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int i = m0 + wm + 16 * x + MF<R>::row(lane, v);
        const int j = n0 + wn + 16 * y + (lane & 15);
        if (i < g.m && j < g.n) repi<EPI, R>(g, i, j, COMP ? tot[x][y][v] : acc[x][y][v], part);
      }
  if constexpr (EPI == EPI_SPLIT || EPI == EPI_YDEF) {
    const RGemmArgs& gg = g;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    if (tid == 0) gg.partials[bid] = red[0] + red[1] + red[2] + red[3];
  }
}

// Large products (at least one 128 x 128 tile per CU, FP64): a 512-thread block per
// 128 x 128 tile, eight waves of 64 x 32 (4 x 2 blocks of 16 x 16), K-tile 16 through
// a double-buffered LDS whose rows are permuted by XOR with 2k (the transposing
// stores and the fragment reads then fall on distinct banks). The tile carries the
// flop per operand byte of the complex kernel's 64 x 64 complex tile, which the 64 x 64
// real tile has half of.
constexpr int RBB = 128, RBNT = 512;
__device__ inline int rbswz(int k, int c) { return c ^ (2 * k); }

template <int OPA, int EPI, int COMP>
__global__ __launch_bounds__(RBNT) void rgemm_big_kernel(RGemmArgs g) {
  using V = typename MF<double>::v4;
  __shared__ double As[2][RBK][RBB];
  __shared__ double Bs[2][RBK][RBB];
  __shared__ double red[RBNT / 64];
  const int ntiles = gridDim.x, bid = blockIdx.x;
  int logical = bid;
  {
    const int per = ntiles / kXCDs;
    if (bid < per * kXCDs) logical = (bid % kXCDs) * per + bid / kXCDs;
  }
  int tm, tn;
  if ((EPI == EPI_YDEF || EPI == EPI_STORE) && g.herm) {
    herm_tile(logical, g.tiles_n, tm, tn);
  } else {
    constexpr int kGroup = 4;
    const int group = logical / (kGroup * g.tiles_n);
    const int first_m = group * kGroup;
    const int gsize = min(g.tiles_m - first_m, kGroup);
    const int within = logical - group * kGroup * g.tiles_n;
    tm = first_m + within % gsize;
    tn = within / gsize;
  }
  const int m0 = tm * RBB, n0 = tn * RBB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int WM = 4, WN = 2;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 32;
  const double* __restrict__ Ap = (const double*)g.A;
  const double* __restrict__ Bp = (const double*)g.B;

  V acc[WM][WN], tot[WM][WN];
#pragma unroll
  for (int a = 0; a < WM; a++)
#pragma unroll
    for (int b = 0; b < WN; b++)
#pragma unroll
      for (int v = 0; v < 4; v++) acc[a][b][v] = tot[a][b][v] = 0;

  constexpr int kLoads = RBB * RBK / RBNT;  // 4 elements of each operand per thread
  double ra[kLoads], rb[kLoads];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < kLoads; r++) {
      const int idx = r * RBNT + tid;
      int mm, kk;
      if (OPA == 0) {
        mm = idx & (RBB - 1);
        kk = idx / RBB;
      } else {
        kk = idx & (RBK - 1);
        mm = idx / RBK;
      }
      const int gm = m0 + mm, gk = k0 + kk;
      double v = 0;
      if (gm < g.m && gk < g.k) v = OPA == 0 ? Ap[gm + (long)gk * g.lda] : Ap[gk + (long)gm * g.lda];
      ra[r] = v;
      const int bk = idx & (RBK - 1), bn = idx / RBK;
      const int gn = n0 + bn, gkb = k0 + bk;
      double w = 0;
      if (gn < g.n && gkb < g.k) w = Bp[gkb + (long)gn * g.ldb];
      rb[r] = w;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < kLoads; r++) {
      const int idx = r * RBNT + tid;
      int mm, kk;
      if (OPA == 0) {
        mm = idx & (RBB - 1);
        kk = idx / RBB;
      } else {
        kk = idx & (RBK - 1);
        mm = idx / RBK;
      }
      As[buf][kk][rbswz(kk, mm)] = ra[r];
      const int bk = idx & (RBK - 1);
      Bs[buf][bk][rbswz(bk, idx / RBK)] = rb[r];
    }
  };
  const int KT = (g.k + RBK - 1) / RBK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < KT; kt++) {
    const int cur = kt & 1;
    if (kt + 1 < KT) gload((kt + 1) * RBK);
#pragma unroll
    for (int kk = 0; kk < RBK; kk += 4) {
      const int krow = kk + (lane >> 4);
      double a[WM], b[WN];
#pragma unroll
      for (int x = 0; x < WM; x++) a[x] = As[cur][krow][rbswz(krow, wm + 16 * x + (lane & 15))];
#pragma unroll
      for (int y = 0; y < WN; y++) b[y] = Bs[cur][krow][rbswz(krow, wn + 16 * y + (lane & 15))];
#pragma unroll
      for (int x = 0; x < WM; x++)
#pragma unroll
        for (int y = 0; y < WN; y++) acc[x][y] = MF<double>::op(a[x], b[y], acc[x][y]);
      // the next K-tile goes to the other buffer while this one's products run
      if (kk == 4 && kt + 1 < KT) sstore(cur ^ 1);
    }
    if (COMP && ((kt + 1) % kRChunk == 0 || kt + 1 == KT)) {
#pragma unroll
      for (int x = 0; x < WM; x++)
#pragma unroll
        for (int y = 0; y < WN; y++) {
          tot[x][y] += acc[x][y];
#pragma unroll
          for (int v = 0; v < 4; v++) acc[x][y][v] = 0;
        }
    }
    __syncthreads();
  }
  double part = 0;
#pragma unroll
  for (int x = 0; x < WM; x++)
#pragma unroll
    for (int y = 0; y < WN; y++)
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int i = m0 + wm + 16 * x + MF<double>::row(lane, v);
        const int j = n0 + wn + 16 * y + (lane & 15);
        if (i < g.m && j < g.n) repi<EPI, double>(g, i, j, COMP ? tot[x][y][v] : acc[x][y][v], part);
      }
  if constexpr (EPI == EPI_SPLIT || EPI == EPI_YDEF) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    if (tid == 0) {
      double s2 = 0;
#pragma unroll
      for (int w = 0; w < RBNT / 64; w++) s2 += red[w];
      g.partials[bid] = s2;
    }
  }
}

// whether an FP64 product takes the 128 x 128 tile
static bool rbig(int m, int n) { return (long)ceil_div(m, RBB) * ceil_div(n, RBB) >= kCUs; }

int rgemm_tiles(int m, int n, bool herm) {
  const int e = rbig(m, n) ? RBB : RBM;
  const int t = ceil_div(n, e);
  return herm ? t * (t + 1) / 2 : ceil_div(m, e) * t;
}

template <typename R, int OPA, int EPI, int COMP>
static hipError_t rlaunch(RGemmArgs g, hipStream_t st) {
  if (g.herm && (g.m != g.n || !(EPI == EPI_STORE || (EPI == EPI_YDEF && g.herm == 1)))) return hipErrorInvalidValue;
  const bool big = std::is_same<R, double>::value && rbig(g.m, g.n);
  const int e = big ? RBB : RBM;
  g.tiles_m = ceil_div(g.m, e);
  g.tiles_n = ceil_div(g.n, e);
  const int nt = g.herm ? g.tiles_n * (g.tiles_n + 1) / 2 : g.tiles_m * g.tiles_n;
  if (nt == 0) return hipSuccess;
  if constexpr (std::is_same<R, double>::value) {
    if (big) {
      hipLaunchKernelGGL((rgemm_big_kernel<OPA, EPI, COMP>), dim3(nt), dim3(RBNT), 0, st, g);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((rgemm_kernel<R, OPA, EPI, COMP>), dim3(nt), dim3(RNT), 0, st, g);
  return hipGetLastError();
}

hipError_t dgemm(int opa, int epi, int comp, const RGemmArgs& g, hipStream_t st) {
#define SR_D(OPA, EPI)                                                                      \
  if (opa == OPA && epi == EPI)                                                             \
    return comp ? rlaunch<double, OPA, EPI, 1>(g, st) : rlaunch<double, OPA, EPI, 0>(g, st);
  SR_D(0, EPI_STORE)
  SR_D(0, EPI_ADD)
  SR_D(0, EPI_SPLIT)
  SR_D(0, EPI_YDEF)
  SR_D(1, EPI_STORE)
  SR_D(1, EPI_ADD)
  SR_D(1, EPI_SPLIT)
  SR_D(1, EPI_YDEF)
#undef SR_D
  return hipErrorInvalidValue;
}

hipError_t sgemm(const RGemmArgs& g, hipStream_t st) { return rlaunch<float, 0, EPI_STORE, 0>(g, st); }

// ------------------------------------------------------------ elementwise

constexpr int RENT = 256;

__global__ void rfro2_kernel(const double* __restrict__ x, long count, double* __restrict__ partials) {
  __shared__ double red[RENT / 64];
  double s = 0;
  for (long z = blockIdx.x * (long)RENT + threadIdx.x; z < count; z += (long)gridDim.x * RENT) s += x[z] * x[z];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

hipError_t rfro2_partials(const double* x, long count, double* partials, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(rfro2_kernel, dim3(nparts), dim3(RENT), 0, st, x, count, partials);
  return hipGetLastError();
}

// W = L - L^T (float), partials of ||W||_F^2 (one per block of 256 columns' worth)
__global__ void rform_w_kernel(const float* __restrict__ L, float* __restrict__ W, int n,
                               double* __restrict__ partials) {
  __shared__ double red[RENT / 64];
  double s = 0;
  const long nn = (long)n * n;
  for (long z = blockIdx.x * (long)RENT + threadIdx.x; z < nn; z += (long)gridDim.x * RENT) {
    const int i = (int)(z % n), j = (int)(z / n);
    const float w = L[z] - L[j + (long)i * n];
    W[z] = w;
    s += (double)w * w;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

int rform_w_parts(int n) { return min(1024, max(1, ceil_div((long)n * n, RENT))); }

hipError_t rform_w(const float* L, float* W, int n, double* partials, hipStream_t st) {
  hipLaunchKernelGGL(rform_w_kernel, dim3(rform_w_parts(n)), dim3(RENT), 0, st, L, W, n, partials);
  return hipGetLastError();
}

// D = W - Y/2 + (W2 + W3 - YW)/2 (W = L - L^T; L and the products may be NULL)
__global__ void rform_delta_kernel(const float* __restrict__ L, const double* __restrict__ Y,
                                   const float* __restrict__ W2, const float* __restrict__ W3,
                                   const float* __restrict__ YW, double* __restrict__ D, int n) {
  const long nn = (long)n * n;
  for (long z = blockIdx.x * (long)RENT + threadIdx.x; z < nn; z += (long)gridDim.x * RENT) {
    const int i = (int)(z % n), j = (int)(z / n);
    double d = -0.5 * Y[z];
    if (L) d += (double)L[z] - (double)L[j + (long)i * n];
    double h = 0;
    if (W2) h += (double)W2[z];
    if (W3) h += (double)W3[z];
    if (YW) h -= (double)YW[z];
    D[z] = d + 0.5 * h;
  }
}

hipError_t rform_delta(const float* L, const double* Y, const float* W2, const float* W3, const float* YW,
                       double* D, int n, hipStream_t st) {
  const int blocks = min(2048, max(1, ceil_div((long)n * n, RENT)));
  hipLaunchKernelGGL(rform_delta_kernel, dim3(blocks), dim3(RENT), 0, st, L, Y, W2, W3, YW, D, n);
  return hipGetLastError();
}

// X = W2 - Y (one FP32 rounding) or Y alone (W2 = NULL), as FP32
__global__ void rw2_minus_y_kernel(const float* __restrict__ W2, const double* __restrict__ Y,
                                   float* __restrict__ X, long count) {
  for (long z = blockIdx.x * (long)RENT + threadIdx.x; z < count; z += (long)gridDim.x * RENT)
    X[z] = W2 ? (float)((double)W2[z] - Y[z]) : (float)Y[z];
}

hipError_t rw2_minus_y(const float* W2, const double* Y, float* X, long count, hipStream_t st) {
  const int blocks = min(2048L, max(1L, (count + RENT - 1) / RENT));
  hipLaunchKernelGGL(rw2_minus_y_kernel, dim3(blocks), dim3(RENT), 0, st, W2, Y, X, count);
  return hipGetLastError();
}

// ------------------------------------------------------------- block solve

// block start and order of row i
__device__ inline void rblock_of(int i, const int* __restrict__ blk, int& start, int& size) {
  if (i > 0 && blk[i - 1]) {
    start = i - 1;
    size = 2;
  } else if (blk[i]) {
    start = i;
    size = 2;
  } else {
    start = i;
    size = 1;
  }
}

// U_I for every 2 x 2 block (stored at its first row, column-major 2 x 2): first
// column the unit eigenvector of lambda = (a + d)/2 + sqrt(((a - d)/2)^2 + bc) of
// B = [[a, b], [c, d]], second column its orthogonal complement. The transforms run in
// FP64 and T_c, E_c are rounded to FP32 once: an FP32 transform would move the
// diagonal of T_c by u |B| instead of u |lambda - mu| relative to the other diagonal
// entries mu, which the sweep divides by (a loss of up to |lambda| / gap in the solve).
template <typename TT>
__global__ void rblock_unitaries_kernel(const TT* __restrict__ T, const int* __restrict__ blk, int n,
                                        zc* __restrict__ U) {
  const int i = blockIdx.x * RENT + threadIdx.x;
  if (i >= n - 1 || !blk[i]) return;
  const double a = T[i + (long)i * n], b = T[i + (long)(i + 1) * n];
  const double c = T[(i + 1) + (long)i * n], d = T[(i + 1) + (long)(i + 1) * n];
  const double h = 0.5 * (a - d), disc = h * h + b * c;
  zc lam;
  if (disc < 0) lam = mk<double>(0.5 * (a + d), sqrt(-disc));
  else lam = mk<double>(0.5 * (a + d) + sqrt(disc), 0.0);
  zc v1, v2;
  if (fabs(b) >= fabs(c)) {
    v1 = mk<double>(b, 0.0);
    v2 = mk<double>(lam.re - a, lam.im);
  } else {
    v1 = mk<double>(lam.re - d, lam.im);
    v2 = mk<double>(c, 0.0);
  }
  const double r = sqrt(v1.re * v1.re + v1.im * v1.im + v2.re * v2.re + v2.im * v2.im);
  v1 = mk<double>(v1.re / r, v1.im / r);
  v2 = mk<double>(v2.re / r, v2.im / r);
  zc* u = U + 4 * (long)i;
  u[0] = v1;                           // U(0, 0)
  u[1] = v2;                           // U(1, 0)
  u[2] = mk<double>(-v2.re, v2.im);    // U(0, 1) = -conj(v2)
  u[3] = mk<double>(v1.re, -v1.im);    // U(1, 1) = conj(v1)
}

__device__ inline zc ucell(const zc* __restrict__ U, int start, int size, int r, int c) {
  if (size == 1) return mk<double>(1.0, 0.0);
  return U[4 * (long)start + r + 2 * c];
}

// Tc = U^H T U (upper triangular: its entries below the diagonal are zero, also
// inside a 2 x 2 block) and Ec = U^H E U on the block strictly lower part (zero
// elsewhere), accumulated in FP64 and rounded to complex64.
template <typename TT>
__global__ void rto_complex_kernel(const TT* __restrict__ T, const float* __restrict__ E,
                                   const int* __restrict__ blk, const zc* __restrict__ U, int n,
                                   cc* __restrict__ Tc, cc* __restrict__ Ec) {
  const long nn = (long)n * n;
  for (long z = blockIdx.x * (long)RENT + threadIdx.x; z < nn; z += (long)gridDim.x * RENT) {
    const int i = (int)(z % n), j = (int)(z / n);
    int bi, p, bj, q;
    rblock_of(i, blk, bi, p);
    rblock_of(j, blk, bj, q);
    const int a = i - bi, b = j - bj;
    const bool upper = bi <= bj;  // T's part; E's: bi > bj
    double sre = 0, sim = 0;
    for (int x = 0; x < p; x++)
      for (int y = 0; y < q; y++) {
        const long o = (bi + x) + (long)(bj + y) * n;
        const double t = upper ? (double)T[o] : (double)E[o];
        const zc ux = ucell(U, bi, p, x, a), uy = ucell(U, bj, q, y, b);
        // conj(ux) t uy
        const double cre = ux.re * t, cim = -ux.im * t;
        sre += cre * uy.re - cim * uy.im;
        sim += cre * uy.im + cim * uy.re;
      }
    const cc zero = mk<float>(0.f, 0.f);
    const cc s = mk<float>((float)sre, (float)sim);
    if (upper) {
      Tc[z] = i > j ? zero : s;
      Ec[z] = zero;
    } else {
      Tc[z] = zero;
      Ec[z] = s;
    }
  }
}

// L = Re(U Lc U^H) on the block strictly lower part (FP64 sums, one rounding), 0 elsewhere
__global__ void rfrom_complex_kernel(const cc* __restrict__ Lc, const int* __restrict__ blk,
                                     const zc* __restrict__ U, int n, float* __restrict__ L) {
  const long nn = (long)n * n;
  for (long z = blockIdx.x * (long)RENT + threadIdx.x; z < nn; z += (long)gridDim.x * RENT) {
    const int i = (int)(z % n), j = (int)(z / n);
    int bi, p, bj, q;
    rblock_of(i, blk, bi, p);
    rblock_of(j, blk, bj, q);
    double re = 0;
    if (bi > bj) {
      const int a = i - bi, b = j - bj;
      for (int x = 0; x < p; x++)
        for (int y = 0; y < q; y++) {
          const cc l = Lc[(bi + x) + (long)(bj + y) * n];
          const zc ua = ucell(U, bi, p, a, x), ub = ucell(U, bj, q, b, y);
          // Re(ua l conj(ub))
          const double tre = ua.re * l.re - ua.im * l.im, tim = ua.re * l.im + ua.im * l.re;
          re += tre * ub.re + tim * ub.im;
        }
    }
    L[z] = (float)re;
  }
}

size_t trisolve_real_ws_bytes(int n) {
  const size_t c = (size_t)n * n * sizeof(cc);
  return 3 * ((c + 255) / 256 * 256) + ((4 * (size_t)n * sizeof(zc) + 255) / 256 * 256) +
         ((trisolve_ws_bytes(n) + 255) / 256 * 256);
}

hipError_t trisolve_real(const float* T, const double* T64, const float* E, float* L, const int* blk, int n,
                         void* ws, unsigned* status, hipStream_t st) {
  if (n < 1) return hipSuccess;
  const size_t c = ((size_t)n * n * sizeof(cc) + 255) / 256 * 256;
  char* p = (char*)ws;
  cc* Tc = (cc*)p;
  cc* Ec = (cc*)(p + c);
  cc* Lc = (cc*)(p + 2 * c);
  zc* U = (zc*)(p + 3 * c);
  void* tri = p + 3 * c + ((4 * (size_t)n * sizeof(zc) + 255) / 256 * 256);
  const int blocks = min(2048, max(1, ceil_div((long)n * n, RENT)));
  if (T64) {
    hipLaunchKernelGGL(rblock_unitaries_kernel<double>, dim3(ceil_div(n, RENT)), dim3(RENT), 0, st, T64, blk, n, U);
    hipLaunchKernelGGL(rto_complex_kernel<double>, dim3(blocks), dim3(RENT), 0, st, T64, E, blk, U, n, Tc, Ec);
  } else {
    hipLaunchKernelGGL(rblock_unitaries_kernel<float>, dim3(ceil_div(n, RENT)), dim3(RENT), 0, st, T, blk, n, U);
    hipLaunchKernelGGL(rto_complex_kernel<float>, dim3(blocks), dim3(RENT), 0, st, T, E, blk, U, n, Tc, Ec);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = trisolve(Tc, Ec, Lc, n, 0.f, tri, status, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rfrom_complex_kernel, dim3(blocks), dim3(RENT), 0, st, Lc, blk, U, n, L);
  return hipGetLastError();
}

}  // namespace sr
