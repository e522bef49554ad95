// Ozaki-style split product on CDNA4 INT8 matrix cores: the high-precision
// products of the refinement (the paper's Section 3 obtains them from an
// Ozaki-scheme toolbox) computed from 8-bit slices with exact 32-bit integer
// accumulation.
//
// Splitting. For an operand role, every row of op(A) (every column of B) gets a
// power-of-two scale 2^e, the least with 256 m / 2^e < 126 for the largest
// |re|, |im| m over the row (column). A value x is written as
// 2^e sum_{s=1..S} d_s 2^{-8 s} with balanced radix-256 digits d_s in
// [-128, 127] (eight bits each, the full int8 range): r = x 2^-e; raw digit
// d = rint(256 r) in [-128, 128], r = 256 r - d in [-1/2, 1/2]; a raw 128 becomes
// -128 with a carry of one into the digit above, and carries ripple through raw
// 127s (resolved from two bit masks, see digit_carries). The top digit is at most
// 126 before its carry, so no carry leaves the expansion. Each step is exact in
// FP64 (double-double inputs are split the same way with an exact double-double
// remainder), so the retained digits reproduce x up to 2^(e - 8 S - 1), about
// 2^(-8 S + 1) of the row maximum.
//
// Product. C_ij = 2^(e_i + f_j) sum_{s,t} 2^{-8(s+t)} (A_s B_t)_ij. The slice
// pairs are grouped by d = s + t; within one d every pair has the same scale, so
// their products are summed exactly in int32 (each digit product is at most 2^14
// in magnitude; the host admits sizes that keep the sums below 2^31) with v_mfma_i32_32x32x32_i8 (the INT8 form that runs at the full
// matrix rate; the 16 x 16 x 64 form runs at half), and the int32 sums are folded
// into FP64 accumulators with scale 2^{-8 d} once d is done. Pairs with
// s + t > dmax are dropped (their weight is below 2^{-8 dmax}). A complex product
// keeps four real accumulators (re*re, im*im, re*im, im*re) so that
// op(A) = conj(A slices) only changes signs at the fold.
//
// Tiling: a 512-thread block computes a 128 x 64 complex tile; its eight waves
// (4 along M x 2 along N) each own one 32 x 32 block. Per step the block
// stages one K-tile (64) of one slice of op(A) (both parts) and one slice of B in
// LDS, double-buffered; LDS rows are padded to 80 bytes, which makes the 16-byte
// fragment reads of 16 consecutive rows conflict-free.
#include <type_traits>

#include "epilogue.hpp"
#include "ozaki_layout.hpp"

namespace sr {


constexpr int OBM = 128, OBN = 64, ONT = 512, OLD = 80;
constexpr int kSplitNT = 256;

size_t oz_slice_bytes(int rows, int K, int S) { return (size_t)S * kParts * oz_plane_bytes(rows, oz_kp(K)); }

// ------------------------------------------------------------------- splitting


// Scale exponent of a row (column) with largest magnitude m: the least e with
// 256 m / 2^e < 126 (m 256 / 126 is rounded at most twice, which keeps
// 256 |x| / 2^e below 126.5 for every |x| <= m(1 + 2^-52), so the top raw digit
// is at most 126).
__host__ __device__ inline int digit_exponent(double m) { return scale_exponent(m * (256.0 / 126.0)); }

// Raw balanced digit of r in [-1/2, 1/2] (the first call: |r| < 126.5 / 256):
// d = rint(256 r) in [-128, 128], r = 256 r - d in [-1/2, 1/2], both exact.
__host__ __device__ inline int raw_digit(double& r) {
  const double y = r * 256.0;
  const double d = rint(y);
  r = y - d;
  return (int)d;
}

// The same for a double-double remainder (rh, rl): d rounds the exact value, the
// remainder stays exact and within [-1/2, 1/2].
__host__ __device__ inline int raw_digit_dd(double& rh, double& rl) {
  const double yh = rh * 256.0, yl = rl * 256.0;
  double d = rint(yh);
  double h, l;
  two_sum(yh - d, yl, h, l);  // yh - d is exact, |yh - d| <= 1/2
  if (h > 0.5 || (h == 0.5 && l > 0.0)) {
    d += 1.0;
    h -= 1.0;  // exact: h is within an ulp of 1/2
  } else if (h < -0.5 || (h == -0.5 && l < 0.0)) {
    d -= 1.0;
    h += 1.0;
  }
  rh = h;
  rl = l;
  return (int)d;
}

// The same for a triple-double remainder (r0, r1, r2): y = 256 r exactly, d the
// rounding of y0, and the remainder (y0 - d) + y1 + y2 renormalized by error-free
// sums (exact), moved into [-1/2, 1/2] by one unit when the lower terms push it out.
__host__ __device__ inline int raw_digit_td(double& r0, double& r1, double& r2) {
  const double y0 = r0 * 256.0, y1 = r1 * 256.0, y2 = r2 * 256.0;
  double d = rint(y0);
  double h, e1, m, e2, h2, e3, m2, l2;
  two_sum(y0 - d, y1, h, e1);  // y0 - d is exact, |y0 - d| <= 1/2
  two_sum(e1, y2, m, e2);
  two_sum(h, m, h2, e3);
  two_sum(e3, e2, m2, l2);
  const bool tail_pos = m2 > 0.0 || (m2 == 0.0 && l2 > 0.0);
  const bool tail_neg = m2 < 0.0 || (m2 == 0.0 && l2 < 0.0);
  if (h2 > 0.5 || (h2 == 0.5 && tail_pos)) {
    d += 1.0;
    h2 -= 1.0;  // exact: h2 is within an ulp of 1/2
  } else if (h2 < -0.5 || (h2 == -0.5 && tail_neg)) {
    d -= 1.0;
    h2 += 1.0;
  }
  r0 = h2;
  r1 = m2;
  r2 = l2;
  return (int)d;
}

// Carries of a raw digit string. Digit s (1..S) sits at bit S - s; raw 128
// generates a carry into the digit above, raw 127 passes an incoming one on. The
// carry into every position is that of the binary sum G + (G | P), i.e.
// (G + (G | P)) ^ G ^ (G | P).
__host__ __device__ inline uint64_t digit_carries(uint64_t gen, uint64_t prop) {
  const uint64_t gp = gen | prop;
  return (gen + gp) ^ gen ^ gp;
}

// Final digit s (1..S) from its raw value and the carry mask.
__host__ __device__ inline int8_t final_digit(int raw, uint64_t carries, int s, int S) {
  int v = raw + (int)((carries >> (S - s)) & 1u);
  if (v > 127) v -= 256;
  return (int8_t)v;
}

// Carry masks of x and of -x (whose raw digits are the negated raw digits of x,
// rint being symmetric) from a first pass over the raw digits of x. The
// imaginary parts are stored negated too; -x has its own carries (a raw -128 of x
// is a raw 128 of -x).
struct Carries {
  uint64_t pos, neg;
};

__host__ __device__ inline void note_digit(int d, uint64_t bit, uint64_t (&m)[4]) {
  if (d == 128) m[0] |= bit;
  if (d == 127) m[1] |= bit;
  if (d == -128) m[2] |= bit;
  if (d == -127) m[3] |= bit;
}

__host__ __device__ inline Carries value_carries(double r, int S) {
  uint64_t m[4] = {0, 0, 0, 0};
  for (int s = 1; s <= S; s++) note_digit(raw_digit(r), 1ull << (S - s), m);
  return {digit_carries(m[0], m[1]), digit_carries(m[2], m[3])};
}

__host__ __device__ inline Carries value_carries_dd(double rh, double rl, int S) {
  uint64_t m[4] = {0, 0, 0, 0};
  for (int s = 1; s <= S; s++) note_digit(raw_digit_dd(rh, rl), 1ull << (S - s), m);
  return {digit_carries(m[0], m[1]), digit_carries(m[2], m[3])};
}

__host__ __device__ inline Carries value_carries_td(double r0, double r1, double r2, int S) {
  uint64_t m[4] = {0, 0, 0, 0};
  for (int s = 1; s <= S; s++) note_digit(raw_digit_td(r0, r1, r2), 1ull << (S - s), m);
  return {digit_carries(m[0], m[1]), digit_carries(m[2], m[3])};
}

// The raw digits of one value from a single pass, kept for the stores: digit s
// (1..S) modulo 256 in byte (s - 1) mod 8 of word (s - 1) / 8, with the carry masks
// of x and -x. (raw + carry) modulo 256 read as a signed byte is final_digit's
// value (raw in [-128, 128], the sum in [-128, 129]), and -raw modulo 256 is the
// negated byte, so the stores need no second pass over the digits. The loops run
// to the fixed maximum so that every word is addressed by a constant.
constexpr int kMaxDigits = 32;
struct Digits {
  uint64_t w[kMaxDigits / 8];
  Carries c;
};

// NT: terms of the value (1: double, 2: double-double, 3: triple-double rh, rm, rl)
template <int NT>
__host__ __device__ inline Digits split_value(double rh, double rm, double rl, int S) {
  Digits d;
  uint64_t m[4] = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < kMaxDigits / 8; q++) {
    uint64_t word = 0;
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const int s = 8 * q + j + 1;
      if (s <= S) {
        const int r = NT == 3 ? raw_digit_td(rh, rm, rl) : NT == 2 ? raw_digit_dd(rh, rl) : raw_digit(rh);
        note_digit(r, 1ull << (S - s), m);
        word |= (uint64_t)(uint8_t)r << (8 * j);
      }
    }
    d.w[q] = word;
  }
  d.c = {digit_carries(m[0], m[1]), digit_carries(m[2], m[3])};
  return d;
}

// Final digit s (1..S) from its byte (raw modulo 256, or its negation) and a carry mask.
__host__ __device__ inline int8_t byte_digit(unsigned byte, uint64_t carries, int s, int S) {
  return (int8_t)(uint8_t)(byte + (unsigned)((carries >> (S - s)) & 1u));
}

// Column exponents of X: the scale of each column's largest leading-term entry, one
// block per column.
template <typename C>
__global__ __launch_bounds__(kSplitNT) void oz_colexp_kernel(const C* __restrict__ X, long ld, int K,
                                                             int* __restrict__ exps) {
  __shared__ double red[kSplitNT / 64];
  const C* x = X + (long)blockIdx.x * ld;
  double m = 0;
  for (int k = threadIdx.x; k < K; k += kSplitNT) m = fmax(m, fmax(fabs((double)x[k].re), fabs((double)x[k].im)));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < kSplitNT / 64; w++) t = fmax(t, red[w]);
    exps[blockIdx.x] = digit_exponent(t);
  }
}

// Slices of the columns of X (K x ncols, leading dim ld) with the exponents of
// oz_colexp_kernel: block (c, b) takes K positions 256 b .. 256 b + 255 of column c of
// the padded count (padding columns and positions get zero digits), one per thread (a
// block per whole column, each thread walking a quarter of K at n = 1024, left too few
// blocks in flight). These serve as B, and as op(A) = X^H when the product applies the
// conjugation. X is complex128 (with the lower terms of an expansion) or complex64 (one
// term; its values are exact in FP64).
template <typename C>
__global__ __launch_bounds__(kSplitNT) void oz_split_cols_kernel(const C* __restrict__ X,
                                                                 const C* __restrict__ Xmid,
                                                                 const C* __restrict__ Xlo, long ld,
                                                                 int K, int ncols, int S, int Kp,
                                                                 int8_t* __restrict__ out,
                                                                 const int* __restrict__ exps) {
  const int col = blockIdx.x;
  const int k = blockIdx.y * kSplitNT + threadIdx.x;
  if (k >= Kp) return;
  const long plane = oz_plane_bytes(ncols, Kp);
  const long stride = (long)kParts * plane;  // slice s -> s+1
  const int KB = Kp / 64;
  const long o = oz_off(col, k, KB);
  int8_t* o_re = out + o;
  int8_t* o_im = out + plane + o;
  int8_t* o_ni = out + 2 * plane + o;
  if (col >= ncols) {
    for (int s = 0; s < S; s++) o_re[s * stride] = o_im[s * stride] = o_ni[s * stride] = 0;
    return;
  }
  const C* x = X + (long)col * ld;
  const C* xl = Xlo ? Xlo + (long)col * ld : nullptr;
  const C* xm = Xmid ? Xmid + (long)col * ld : nullptr;
  const int e = exps[col];
  if (k < K) {
    const C v = x[k];
    const C w = xl ? xl[k] : C{0, 0};
    const C u = xm ? xm[k] : C{0, 0};
    const double rh = ldexp((double)v.re, -e), rl = ldexp((double)w.re, -e), rm = ldexp((double)u.re, -e);
    const double ih = ldexp((double)v.im, -e), il = ldexp((double)w.im, -e), im = ldexp((double)u.im, -e);
    const Digits dr = xm ? split_value<3>(rh, rm, rl, S)
                         : xl ? split_value<2>(rh, 0.0, rl, S) : split_value<1>(rh, 0.0, 0.0, S);
    const Digits di = xm ? split_value<3>(ih, im, il, S)
                         : xl ? split_value<2>(ih, 0.0, il, S) : split_value<1>(ih, 0.0, 0.0, S);
#pragma unroll
    for (int q = 0; q < kMaxDigits / 8; q++)
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const int s = 8 * q + j + 1;
        if (s <= S) {
          const unsigned br = (unsigned)(dr.w[q] >> (8 * j)) & 255u, bi = (unsigned)(di.w[q] >> (8 * j)) & 255u;
          o_re[(s - 1) * stride] = byte_digit(br, dr.c.pos, s, S);
          o_im[(s - 1) * stride] = byte_digit(bi, di.c.pos, s, S);
          o_ni[(s - 1) * stride] = byte_digit((256u - bi) & 255u, di.c.neg, s, S);
        }
      }
  } else {
    for (int s = 0; s < S; s++) {
      o_re[s * stride] = 0;
      o_im[s * stride] = 0;
      o_ni[s * stride] = 0;
    }
  }
}

// Scale exponents of the rows of X (M x K, leading dim ld), computed over K-chunks
// of 256 in parallel and combined with an integer atomic max on the exponent
// (which is monotone in the maximum; an all-zero chunk contributes INT_MIN).
constexpr int kNoExp = -2147483647 - 1;

__global__ void oz_exp_init_kernel(int* __restrict__ exps, int M) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < M) exps[r] = kNoExp;
}

template <typename C>
__global__ __launch_bounds__(kSplitNT) void oz_rowmax_kernel(const C* __restrict__ X, long ld, int M,
                                                             int K, int* __restrict__ exps) {
  __shared__ double red[4][64];
  const int r = blockIdx.x * 64 + (threadIdx.x & 63), c = threadIdx.x >> 6;
  const int k0 = blockIdx.y * 256, k1 = min(K, k0 + 256);
  double m = 0;
  if (r < M)
    for (int k = k0 + c; k < k1; k += 4) {
      const C v = X[r + (long)k * ld];
      m = fmax(m, fmax(fabs((double)v.re), fabs((double)v.im)));
    }
  red[c][threadIdx.x & 63] = m;
  __syncthreads();
  if (c == 0 && r < M) {
    const double t = fmax(fmax(red[0][threadIdx.x], red[1][threadIdx.x]), fmax(red[2][threadIdx.x], red[3][threadIdx.x]));
    if (t > 0) atomicMax(&exps[r], digit_exponent(t));
  }
}

__global__ void oz_exp_fix_kernel(int* __restrict__ exps, int M) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < M && exps[r] == kNoExp) exps[r] = 0;
}

// Slices of the rows of X; one block per 32 x 32 tile, staged through LDS so that
// reads follow the columns and writes the rows (padding rows get zero digits). NTERM:
// the terms per value (1: X; 2: X + Xlo; 3: X + Xmid + Xlo); the LDS holds only those
// (one term: 17 KiB, eight blocks per CU instead of three).
template <typename C, int NTERM>
__global__ __launch_bounds__(kSplitNT) void oz_split_rows_kernel(const C* __restrict__ X,
                                                                 const C* __restrict__ Xmid,
                                                                 const C* __restrict__ Xlo, long ld,
                                                                 int M, int K, int S, int Kp,
                                                                 const int* __restrict__ exps,
                                                                 int8_t* __restrict__ out) {
  __shared__ zc t[32][33];
  __shared__ zc tl[NTERM >= 2 ? 32 : 1][33];
  __shared__ zc tmid[NTERM >= 3 ? 32 : 1][33];
  const int i0 = blockIdx.x * 32, k0 = blockIdx.y * 32;
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int idx = r * kSplitNT + threadIdx.x;
    const int row = idx & 31, kk = idx >> 5;
    const int gi = i0 + row, gk = k0 + kk;
    const bool ok = gi < M && gk < K;
    const long o = ok ? gi + (long)gk * ld : 0;
    const C v = X[o];
    t[kk][row] = mk<double>(ok ? (double)v.re : 0.0, ok ? (double)v.im : 0.0);
    if constexpr (NTERM >= 2) {
      const C w = Xlo[o];
      tl[kk][row] = mk<double>(ok ? (double)w.re : 0.0, ok ? (double)w.im : 0.0);
    }
    if constexpr (NTERM >= 3) {
      const C w = Xmid[o];
      tmid[kk][row] = mk<double>(ok ? (double)w.re : 0.0, ok ? (double)w.im : 0.0);
    }
  }
  __syncthreads();
  const int row = threadIdx.x >> 3, kg = (threadIdx.x & 7) * 4;
  const int gi = i0 + row;
  if (gi >= oz_rows_pad(M)) return;
  const long plane = oz_plane_bytes(M, Kp);
  const long stride = (long)kParts * plane;
  const long o = oz_off(gi, k0 + kg, Kp / 64);  // 4 consecutive k stay in one chunk
  int* o_re = (int*)(out + o);
  int* o_im = (int*)(out + plane + o);
  int* o_ni = (int*)(out + 2 * plane + o);
  if (gi >= M) {
    for (int s = 0; s < S; s++) o_re[s * stride / 4] = o_im[s * stride / 4] = o_ni[s * stride / 4] = 0;
    return;
  }
  const int e = exps[gi];
  double rh[4], rl[4], ih[4], il[4], rm[4], imd[4];
#pragma unroll
  for (int c = 0; c < 4; c++) {
    const zc v = t[kg + c][row];
    rh[c] = ldexp(v.re, -e);
    ih[c] = ldexp(v.im, -e);
    if constexpr (NTERM >= 2) {
      const zc w = tl[kg + c][row];
      rl[c] = ldexp(w.re, -e);
      il[c] = ldexp(w.im, -e);
    } else {
      rl[c] = il[c] = 0;
    }
    if constexpr (NTERM >= 3) {
      const zc w = tmid[kg + c][row];
      rm[c] = ldexp(w.re, -e);
      imd[c] = ldexp(w.im, -e);
    } else {
      rm[c] = imd[c] = 0;
    }
  }
  Carries cr[4], ci[4];
#pragma unroll
  for (int c = 0; c < 4; c++) {
    cr[c] = NTERM == 3   ? value_carries_td(rh[c], rm[c], rl[c], S)
            : NTERM == 2 ? value_carries_dd(rh[c], rl[c], S)
                         : value_carries(rh[c], S);
    ci[c] = NTERM == 3   ? value_carries_td(ih[c], imd[c], il[c], S)
            : NTERM == 2 ? value_carries_dd(ih[c], il[c], S)
                         : value_carries(ih[c], S);
  }
  for (int s = 0; s < S; s++) {
    unsigned pr = 0, pi = 0, pn = 0;
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const int dr = NTERM == 3 ? raw_digit_td(rh[c], rm[c], rl[c])
                     : NTERM == 2 ? raw_digit_dd(rh[c], rl[c]) : raw_digit(rh[c]);
      const int di = NTERM == 3 ? raw_digit_td(ih[c], imd[c], il[c])
                     : NTERM == 2 ? raw_digit_dd(ih[c], il[c]) : raw_digit(ih[c]);
      pr |= (unsigned)(uint8_t)final_digit(dr, cr[c].pos, s + 1, S) << (8 * c);
      pi |= (unsigned)(uint8_t)final_digit(di, ci[c].pos, s + 1, S) << (8 * c);
      pn |= (unsigned)(uint8_t)final_digit(-di, ci[c].neg, s + 1, S) << (8 * c);
    }
    o_re[s * stride / 4] = (int)pr;
    o_im[s * stride / 4] = (int)pi;
    o_ni[s * stride / 4] = (int)pn;
  }
}

hipError_t oz_split_cols3(const zc* X, const zc* Xmid, const zc* Xlo, long ld, int K, int ncols, int S,
                          int8_t* out, int* exps, hipStream_t st) {
  if (S < 1 || S > kMaxDigits || (Xmid && !Xlo)) return hipErrorInvalidValue;
  if (ncols == 0) return hipSuccess;
  const int Kp = oz_kp(K);
  hipLaunchKernelGGL(oz_colexp_kernel<zc>, dim3(ncols), dim3(kSplitNT), 0, st, X, ld, K, exps);
  hipLaunchKernelGGL(oz_split_cols_kernel<zc>, dim3(oz_rows_pad(ncols), ceil_div(Kp, kSplitNT)), dim3(kSplitNT), 0,
                     st, X, Xmid, Xlo, ld, K, ncols, S, Kp, out, exps);
  return hipGetLastError();
}

hipError_t oz_split_cols_c64(const cc* X, long ld, int K, int ncols, int S, int8_t* out, int* exps, hipStream_t st) {
  if (S < 1 || S > kMaxDigits) return hipErrorInvalidValue;
  if (ncols == 0) return hipSuccess;
  const int Kp = oz_kp(K);
  hipLaunchKernelGGL(oz_colexp_kernel<cc>, dim3(ncols), dim3(kSplitNT), 0, st, X, ld, K, exps);
  hipLaunchKernelGGL(oz_split_cols_kernel<cc>, dim3(oz_rows_pad(ncols), ceil_div(Kp, kSplitNT)), dim3(kSplitNT), 0,
                     st, X, (const cc*)nullptr, (const cc*)nullptr, ld, K, ncols, S, Kp, out, exps);
  return hipGetLastError();
}

hipError_t oz_split_cols(const zc* X, const zc* Xlo, long ld, int K, int ncols, int S, int8_t* out,
                         int* exps, hipStream_t st) {
  return oz_split_cols3(X, nullptr, Xlo, ld, K, ncols, S, out, exps, st);
}

hipError_t oz_split_rows(const zc* X, const zc* Xlo, long ld, int M, int K, int S, int8_t* out,
                         int* exps, hipStream_t st) {
  return oz_split_rows3(X, nullptr, Xlo, ld, M, K, S, out, exps, st);
}

template <typename C>
static hipError_t split_rows_any(const C* X, const C* Xmid, const C* Xlo, long ld, int M, int K, int S,
                                 int8_t* out, int* exps, hipStream_t st) {
  if (S < 1 || S > kMaxDigits || (Xmid && !Xlo)) return hipErrorInvalidValue;
  if (M == 0) return hipSuccess;
  hipLaunchKernelGGL(oz_exp_init_kernel, dim3(ceil_div(M, 256)), dim3(256), 0, st, exps, M);
  hipLaunchKernelGGL(oz_rowmax_kernel<C>, dim3(ceil_div(M, 64), max(1, ceil_div(K, 256))), dim3(kSplitNT), 0,
                     st, X, ld, M, K, exps);
  hipLaunchKernelGGL(oz_exp_fix_kernel, dim3(ceil_div(M, 256)), dim3(256), 0, st, exps, M);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int Kp = oz_kp(K);
  const dim3 grid(ceil_div(M, 32), Kp / 32);
  if (Xmid)
    hipLaunchKernelGGL((oz_split_rows_kernel<C, 3>), grid, dim3(kSplitNT), 0, st, X, Xmid, Xlo, ld, M, K, S, Kp,
                       exps, out);
  else if (Xlo)
    hipLaunchKernelGGL((oz_split_rows_kernel<C, 2>), grid, dim3(kSplitNT), 0, st, X, Xmid, Xlo, ld, M, K, S, Kp,
                       exps, out);
  else
    hipLaunchKernelGGL((oz_split_rows_kernel<C, 1>), grid, dim3(kSplitNT), 0, st, X, Xmid, Xlo, ld, M, K, S, Kp,
                       exps, out);
  return hipGetLastError();
}

hipError_t oz_split_rows3(const zc* X, const zc* Xmid, const zc* Xlo, long ld, int M, int K, int S,
                          int8_t* out, int* exps, hipStream_t st) {
  return split_rows_any<zc>(X, Xmid, Xlo, ld, M, K, S, out, exps, st);
}

hipError_t oz_split_rows_c64(const cc* X, long ld, int M, int K, int S, int8_t* out, int* exps, hipStream_t st) {
  return split_rows_any<cc>(X, nullptr, nullptr, ld, M, K, S, out, exps, st);
}

// -------------------------------------------------------------------- product

struct OzArgs {
  const int8_t* A;  // op(A) slices: [SA][2][m][Kp]
  const int* ea;
  const int8_t* B;  // B slices: [SB][2][n][Kp]
  const int* eb;
  int SA, SB, dmax, conjA, Kp;
  GemmArgs g;          // sizes, output and epilogue
  double2* scratch;    // large-tile kernel: FP64 partial sums between folds
};

template <int EPI>
__global__ __launch_bounds__(ONT) void oz_gemm_kernel(OzArgs a) {
  __shared__ __align__(16) int8_t As[2][2][OBM][OLD];
  __shared__ __align__(16) int8_t Bs[2][2][OBN][OLD];
  __shared__ double red[ONT / 64];
  const GemmArgs& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 3) * 32, wn = (wave >> 2) * 32;

  // XCD-aware grouped tile order (as in the FP64 kernel).
  const int ntiles = g.tiles_m * g.tiles_n;
  const int bid = blockIdx.x;
  int logical = bid;
  {
    const int per = ntiles / kXCDs;
    if (bid < per * kXCDs) logical = (bid % kXCDs) * per + bid / kXCDs;
  }
  constexpr int kGroup = 4;
  const int group = logical / (kGroup * g.tiles_n);
  const int first_m = group * kGroup;
  const int gsize = min(g.tiles_m - first_m, kGroup);
  const int within = logical - group * kGroup * g.tiles_n;
  const int m0 = (first_m + within % gsize) * OBM, n0 = (within / gsize) * OBN;

  const int KT = a.Kp / OBK;
  const long pA = oz_plane_bytes(g.m, a.Kp), pB = oz_plane_bytes(g.n, a.Kp);  // bytes per part
  const long sA = kParts * pA, sB = kParts * pB;                              // bytes per slice

  double out_re[16], out_im[16];
#pragma unroll
  for (int v = 0; v < 16; v++) out_re[v] = out_im[v] = 0;

  // staging: 2 chunks of A (16 B) and 1 of B per thread and step
  v4i ra[2], rb;
  auto gload = [&](int s, int t, int kt) {
#pragma unroll
    for (int r = 0; r < 2; r++) {
      const int idx = r * ONT + tid;  // 0..1023: part(1) row(128) chunk(4)
      const int part = idx >> 9, row = (idx >> 2) & 127, ch = idx & 3;
      const int gi = m0 + row;
      v4i v = {0, 0, 0, 0};
      if (gi < g.m) v = *(const v4i*)(a.A + (long)(s - 1) * sA + part * pA + oz_off(gi, kt * OBK + ch * 16, KT));
      ra[r] = v;
    }
    {
      const int part = tid >> 8, col = (tid >> 2) & 63, ch = tid & 3;
      const int gj = n0 + col;
      v4i v = {0, 0, 0, 0};
      if (gj < g.n) v = *(const v4i*)(a.B + (long)(t - 1) * sB + part * pB + oz_off(gj, kt * OBK + ch * 16, KT));
      rb = v;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 2; r++) {
      const int idx = r * ONT + tid;
      const int part = idx >> 9, row = (idx >> 2) & 127, ch = idx & 3;
      *(v4i*)&As[buf][part][row][ch * 16] = ra[r];
    }
    const int part = tid >> 8, col = (tid >> 2) & 63, ch = tid & 3;
    *(v4i*)&Bs[buf][part][col][ch * 16] = rb;
  };

  for (int d = 2; d <= a.dmax; d++) {
    const int s_lo = max(1, d - a.SB), s_hi = min(a.SA, d - 1);
    if (s_lo > s_hi) continue;
    const int steps = (s_hi - s_lo + 1) * KT;
    v16i rr = {}, ii = {}, ri = {}, ir = {};
    __syncthreads();  // LDS of the previous diagonal no longer read
    gload(s_lo, d - s_lo, 0);
    sstore(0);
    __syncthreads();
    for (int st = 0; st < steps; st++) {
      const int cur = st & 1;
      if (st + 1 < steps) {
        const int s = s_lo + (st + 1) / KT, kt = (st + 1) % KT;
        gload(s, d - s, kt);
      }
      const int row = wm + (lane & 31), col = wn + (lane & 31);
#pragma unroll
      for (int kh = 0; kh < 2; kh++) {
        const int kq = 32 * kh + 16 * (lane >> 5);
        const v4i far = *(const v4i*)&As[cur][0][row][kq];
        const v4i fai = *(const v4i*)&As[cur][1][row][kq];
        const v4i fbr = *(const v4i*)&Bs[cur][0][col][kq];
        const v4i fbi = *(const v4i*)&Bs[cur][1][col][kq];
        rr = __builtin_amdgcn_mfma_i32_32x32x32_i8(far, fbr, rr, 0, 0, 0);
        ii = __builtin_amdgcn_mfma_i32_32x32x32_i8(fai, fbi, ii, 0, 0, 0);
        ri = __builtin_amdgcn_mfma_i32_32x32x32_i8(far, fbi, ri, 0, 0, 0);
        ir = __builtin_amdgcn_mfma_i32_32x32x32_i8(fai, fbr, ir, 0, 0, 0);
      }
      if (st + 1 < steps) sstore(cur ^ 1);
      __syncthreads();
    }
    // fold diagonal d: scale 2^{-8 d}
    const double sc = ldexp(1.0, -8 * d);
    const double sg = a.conjA ? 1.0 : -1.0;  // re = rr + sg ii, im = ri - sg ir
#pragma unroll
    for (int v = 0; v < 16; v++) {
      out_re[v] += ((double)rr[v] + sg * (double)ii[v]) * sc;
      out_im[v] += ((double)ri[v] - sg * (double)ir[v]) * sc;
    }
  }

  double part = 0;
#pragma unroll
  for (int v = 0; v < 16; v++) {
    const int i = m0 + wm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);  // i32 32x32 accumulator rows
    const int j = n0 + wn + (lane & 31);
    if (i < g.m && j < g.n) {
      const int e = a.ea[i] + a.eb[j];
      zc val = mk<double>(ldexp(out_re[v], e), ldexp(out_im[v], e));
      epi_element<EPI, double>(g, i, j, val, part);
    }
  }
  if constexpr (EPI == EPI_SPLIT || EPI == EPI_YDEF) epi_reduce<ONT>(g, part, red, bid);
}


// ------------------------------------------------------- large-tile product
//
// For products with at least one 128 x 128 tile per CU, and for every
// double-double product. A 256-thread block computes a 128 x 128 complex tile;
// each of its four waves owns 64 x 64 as 2 x 2 blocks of 32 x 32, and two blocks
// share a CU (two waves per SIMD). Only two int32 accumulators per output are
// kept: with the negated imaginary digits of op(A) stored beside the real and
// imaginary ones, re = Ar Br + (-Ai) Bi and im = Ar Bi + Ai Br (conjugated op(A):
// re = Ar Br + Ai Bi, im = Ar Bi + (-Ai) Br), all summed exactly in int32
// (|sum| <= 2 * 64 * steps * 2^14 <= 2^30 with a diagonal folded at least every
// kSeg = 512 steps). The FP64 partial sums live between folds in a per-tile
// scratch laid out in the waves' register order (coalesced), not in registers,
// so the register file holds the large wave tile.
//
// Staging: the K-tiles go from global memory straight into LDS
// (global_load_lds_dwordx4: lane l of an instruction writes 16 bytes at
// base + 16 l), through two stages, the next step's loads issued while the
// current one is multiplied. A stage holds 3 parts of op(A) and 2 of B, each 128
// rows of 64 bytes; within a row the four 16-byte chunks are stored in the order
// chunk ^ f(row), f(row) = ((row >> 1) ^ (row >> 3)) & 3, so that fragment reads
// of 32 consecutive rows at one chunk spread over all banks.
constexpr int PBM = 128, PBN = 128, PNT = 256, kSeg = 512, kStages = 2;
constexpr int kRowBytes = 64, kPartBytes = PBM * kRowBytes;            // 8 KiB
constexpr int kStageBytes = 5 * kPartBytes;                             // 3 A parts + 2 B parts
constexpr int kLoadsPerWave = 5 * (PBM / 16) / (PNT / 64);              // 10 wave instructions

constexpr int kWaitVmStep = 0x0F70 | kLoadsPerWave;  // vmcnt(10): one step in flight
static_assert(kLoadsPerWave < 16, "vmcnt immediate");

template <int EPI, bool DD>
__global__ __launch_bounds__(PNT) __attribute__((amdgpu_waves_per_eu(2))) void oz_gemm2_kernel(OzArgs a) {
  extern __shared__ __align__(16) int8_t lds[];  // kStages * kStageBytes
  const GemmArgs& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;

  const int ntiles = gridDim.x;
  const int bid = blockIdx.x;
  int logical = bid;
  {
    const int per = ntiles / kXCDs;
    if (bid < per * kXCDs) logical = (bid % kXCDs) * per + bid / kXCDs;
  }
  int tm, tn;
  if (EPI == EPI_YDEF && g.herm) {
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
  const int m0 = tm * PBM, n0 = tn * PBN;

  const int KT = a.Kp / OBK;
  const long pA = oz_plane_bytes(g.m, a.Kp), pB = oz_plane_bytes(g.n, a.Kp);
  const long sA = kParts * pA, sB = kParts * pB;
  const int pa2 = a.conjA ? 1 : 2, pa3 = a.conjA ? 2 : 1;
  // per wave 4096 (x, y, v, lane) partial sums; the double-double product keeps
  // each as a three-term expansion (see the fold)
  constexpr int kWave = 16 * 4 * 64;
  double2* sp = a.scratch ? a.scratch + ((long)bid * 4 + wave) * (DD ? 3 * kWave : kWave) + lane : nullptr;

  // This lane's part of the wave's load instructions: instruction j of wave w is
  // q = w * 10 + j; q < 24 covers A part q / 8, row block q % 8 of the tile; the
  // rest B part (q - 24) / 8. Each instruction copies one KiB block of the digit
  // planes as it is (lane l: bytes 16 l .. 16 l + 15). Row blocks past the matrix
  // read its last block (their outputs are not stored). Offsets are relative to
  // slice 1, K-tile 0.
  const int uwave = __builtin_amdgcn_readfirstlane(wave);
  const int RBA = oz_rows_pad(g.m) / 16, RBB = oz_rows_pad(g.n) / 16;
  int goff[kLoadsPerWave];
#pragma unroll
  for (int j = 0; j < kLoadsPerWave; j++) {
    const int q = uwave * kLoadsPerWave + j;
    const bool isA = q < 24;
    const int qq = isA ? q : q - 24;
    const int part = qq >> 3;
    const int rb = min((isA ? m0 : n0) / 16 + (qq & 7), (isA ? RBA : RBB) - 1);
    goff[j] = (int)(part * (isA ? pA : pB)) + rb * KT * 1024 + lane * 16;
  }
  auto issue = [&](int s, int t, int kt, int stage) {
    const int8_t* baseA = a.A + (long)(s - 1) * sA + kt * 1024;
    const int8_t* baseB = a.B + (long)(t - 1) * sB + kt * 1024;
#pragma unroll
    for (int j = 0; j < kLoadsPerWave; j++) {
      const int q = uwave * kLoadsPerWave + j;
      const bool isA = q < 24;
      const int qq = isA ? q : q - 24;
      const int loff = (isA ? (qq >> 3) : 3 + (qq >> 3)) * kPartBytes + 16 * (qq & 7) * kRowBytes;
      const int8_t* src = (isA ? baseA : baseB) + goff[j];
      __builtin_amdgcn_global_load_lds((gbl_ptr_t*)src, (lds_ptr_t*)(lds + stage * kStageBytes + loff), 16, 0, 0);
    }
  };
  // Fragments of one K-half (32 deep) of a stage: B parts 3, 4 and A parts 0,
  // pa2, pa3 for this wave's two column and two row blocks.
  struct Frags {
    v4i b0[2], b1[2], a0[2], a2[2], a3[2];
  };
  auto load_frags = [&](Frags& f, int stage, int kh) {
    const int c = 2 * kh + (lane >> 5);
    const int8_t* base = lds + stage * kStageBytes;
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int r = wn + y * 32 + (lane & 31);
      const int o = r * kRowBytes + ((c ^ chunk_swz(r)) << 4);
      f.b0[y] = *(const v4i*)(base + 3 * kPartBytes + o);
      f.b1[y] = *(const v4i*)(base + 4 * kPartBytes + o);
    }
#pragma unroll
    for (int x = 0; x < 2; x++) {
      const int r = wm + x * 32 + (lane & 31);
      const int o = r * kRowBytes + ((c ^ chunk_swz(r)) << 4);
      f.a0[x] = *(const v4i*)(base + o);
      f.a2[x] = *(const v4i*)(base + pa2 * kPartBytes + o);
      f.a3[x] = *(const v4i*)(base + pa3 * kPartBytes + o);
    }
  };

  v16i acc_re[2][2], acc_im[2][2];
  auto mfmas = [&](const Frags& f) {
#pragma unroll
    for (int x = 0; x < 2; x++)
#pragma unroll
      for (int y = 0; y < 2; y++)
        acc_re[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a0[x], f.b0[y], acc_re[x][y], 0, 0, 0);
#pragma unroll
    for (int x = 0; x < 2; x++)
#pragma unroll
      for (int y = 0; y < 2; y++)
        acc_im[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a0[x], f.b1[y], acc_im[x][y], 0, 0, 0);
#pragma unroll
    for (int x = 0; x < 2; x++)
#pragma unroll
      for (int y = 0; y < 2; y++)
        acc_re[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a2[x], f.b1[y], acc_re[x][y], 0, 0, 0);
#pragma unroll
    for (int x = 0; x < 2; x++)
#pragma unroll
      for (int y = 0; y < 2; y++)
        acc_im[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a3[x], f.b0[y], acc_im[x][y], 0, 0, 0);
  };
  // Workgroup barrier without a memory fence: the waits before it are explicit
  // (a fenced barrier would also wait for the loads still in flight for later
  // stages). The empty asm statements keep the compiler from moving LDS accesses
  // across it.
  auto barrier = [&]() {
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };

  double part = 0;
  bool first = true;
  const int d_last = min(a.dmax, a.SA + a.SB);
  for (int d = 2; d <= d_last; d++) {
    const int s_lo = max(1, d - a.SB), s_hi = min(a.SA, d - 1);
    if (s_lo > s_hi) continue;
    const int total = (s_hi - s_lo + 1) * KT;
    for (int seg0 = 0; seg0 < total; seg0 += kSeg) {
      const int steps = min(kSeg, total - seg0);
      const bool last = d == d_last && seg0 + steps == total;
#pragma unroll
      for (int x = 0; x < 2; x++)
#pragma unroll
        for (int y = 0; y < 2; y++) acc_re[x][y] = acc_im[x][y] = v16i{};
      auto issue_step = [&](int st) {
        const int q = seg0 + st, s = s_lo + q / KT;
        issue(s, d - s, q % KT, st % kStages);
      };
      // Schedule of step st (stage st % 2): wait for its loads, barrier (its data
      // are visible; the other stage is no longer read), issue step st+1's loads
      // into the other stage, read the fragments of both K-halves, MFMAs. Two
      // blocks share a CU (80 KiB of LDS each), so one block's waits overlap the
      // other's MFMAs.
      __builtin_amdgcn_s_waitcnt(kWaitVm0);
      barrier();  // the previous segment no longer reads the ring
      issue_step(0);
      for (int st = 0; st < steps; st++) {
        const int cur = st & 1;
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        barrier();
        if (st + 1 < steps) issue_step(st + 1);
        Frags f0, f1;
        load_frags(f0, cur, 0);
        load_frags(f1, cur, 1);
        mfmas(f0);
        mfmas(f1);
      }
      // fold: partial = previous partial + acc 2^{-8 d} (acc 2^{-8 d} is exact in FP64)
      const double sc = ldexp(1.0, -8 * d);
      // one 32 x 32 block at a time (the empty asm keeps the blocks' scratch
      // accesses apart, which bounds the registers the fold needs)
      auto fold_block = [&](const v16i& ar, const v16i& ai, int x, int y) {
#pragma unroll
          for (int v = 0; v < 16; v++) {
            const int o = ((x * 2 + y) * 16 + v) * 64;
            double re = (double)ar[v] * sc, im = (double)ai[v] * sc;
            // double-double: the partial sum is a0 + a1 + a2, extended with two exact
            // TwoSum steps per fold; the partial sums can exceed the final value by
            // the ratio of the row/column scales to it, which a two-term sum would
            // turn into error of the final value
            double rm = 0, im_m = 0, rl = 0, il = 0;
            if (!first) {
              const double2 pv = sp[o];
              if constexpr (DD) {
                const double2 pm = sp[o + kWave], pl = sp[o + 2 * kWave];
                double s0, e0, s1, e1;
                two_sum(pv.x, re, s0, e0);
                two_sum(pm.x, e0, s1, e1);
                re = s0;
                rm = s1;
                rl = pl.x + e1;
                two_sum(pv.y, im, s0, e0);
                two_sum(pm.y, e0, s1, e1);
                im = s0;
                im_m = s1;
                il = pl.y + e1;
              } else {
                re = pv.x + re;
                im = pv.y + im;
              }
            }
            if (!last) {
              sp[o] = make_double2(re, im);
              if constexpr (DD) {
                sp[o + kWave] = make_double2(rm, im_m);
                sp[o + 2 * kWave] = make_double2(rl, il);
              }
            } else {
              if constexpr (DD) {
                // to double-double: (re + rm) exactly, then the third term
                double h, e;
                two_sum(re, rm, h, e);
                e += rl;
                fast_two_sum(h, e, re, rl);
                two_sum(im, im_m, h, e);
                e += il;
                fast_two_sum(h, e, im, il);
              }
              const int i = m0 + wm + x * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
              const int j = n0 + wn + y * 32 + (lane & 31);
              if (i < g.m && j < g.n) {
                const int e = a.ea[i] + a.eb[j];
                if constexpr (DD)
                  epi_element_dd<EPI>(g, i, j, mk<double>(ldexp(re, e), ldexp(im, e)),
                                      mk<double>(ldexp(rl, e), ldexp(il, e)), part);
                else
                  epi_element<EPI, double>(g, i, j, mk<double>(ldexp(re, e), ldexp(im, e)), part);
              }
            }
          }
      };
      fold_block(acc_re[0][0], acc_im[0][0], 0, 0);
      asm volatile("" ::: "memory");
      fold_block(acc_re[0][1], acc_im[0][1], 0, 1);
      asm volatile("" ::: "memory");
      fold_block(acc_re[1][0], acc_im[1][0], 1, 0);
      asm volatile("" ::: "memory");
      fold_block(acc_re[1][1], acc_im[1][1], 1, 1);
      first = false;
    }
  }
  // the ring is free once every wave is past its last fragment read: its first
  // bytes then hold the block reduction
  if constexpr (EPI == EPI_SPLIT || EPI == EPI_YDEF) {
    __syncthreads();
    epi_reduce<PNT>(g, part, (double*)lds, bid);
  }
}

// ------------------------------------------------------ all-pairs product
//
// The FP64 tier's products (at most kApS digits per operand, pairs up to
// s + t = kApS + 1) on outputs with at least one 64 x 64 tile per CU. The kernel
// above reads both slices of a pair once per pair, so every slice is fetched
// once per pair it takes part in (28 pairs from 7 + 7 slices), and those reads
// miss L2. Here a K-step (32 deep) stages the digits of every slice of both
// operands in LDS at once, and each wave forms all pairs of the step from
// registers, with one int32 accumulator pair (re, im) per diagonal s + t: the
// operand bytes per tile drop by the ratio of pairs to slices.
//
// A 512-thread block computes a 64 x 64 complex tile. Wave w owns quadrant
// w % 4 (32 x 32) and one part of the result: the real part for w < 4, the
// imaginary part for w >= 4, so that a wave keeps one int32 accumulator per
// diagonal and lane (16 x up to 7) and two waves share every SIMD: while one
// waits (a barrier, an LDS read, an MFMA result), the other issues. One block per
// CU (LDS: two stages of 70 KiB). The int32 sums of a diagonal stay exact for
// kApSeg K-steps (at most 7 pairs x 2 products x 32 terms x 2^14 per step,
// 7 * 2^28 < 2^31 over a segment); each segment is folded into FP64, the
// diagonals from the smallest weight up. After the last segment the imaginary
// parts pass through LDS to the waves of the real parts, which apply the
// epilogue.
//
// LDS layout of a stage: one 2 KiB region per part (A: 3 parts per slice, B: 2),
// 64 rows x 32 bytes (the step's half of each 64-byte K-block row). Within a row
// the two 16-byte chunks sit at position c ^ lsw(row), lsw(row) = bit 2 ^ bit 3
// of the row, so that fragment reads of 8 or 16 consecutive rows at one chunk hit
// distinct banks. The loads gather those halves from the global planes
// (global_load_lds_dwordx4: lane l writes 16 bytes at base + 16 l, i.e. row
// l / 2, position l % 2 of a 32-row half region).
constexpr int kApS = 7;
constexpr int ABM = 64, ANT = 512, kApSeg = 256;
constexpr int kApRegion = ABM * 32;                       // 2 KiB
constexpr int kApStageBytes = kApS * 5 * kApRegion;       // 70 KiB
constexpr int kApLds = 2 * kApStageBytes;
static_assert(kApS * 2 * 32 * 16384L * kApSeg < 2147483648L, "segment bound");
static_assert(4 * 16 * 64 * sizeof(double) <= (size_t)kApLds, "imaginary parts fit in the stages");
__host__ __device__ inline int ap_lsw(int row) { return ((row >> 2) ^ (row >> 3)) & 1; }

template <int EPI, int S>
__global__ __launch_bounds__(ANT) __attribute__((amdgpu_waves_per_eu(2, 2))) void oz_gemm_allpairs_kernel(
    OzArgs a) {
  extern __shared__ __align__(16) int8_t lds[];  // kApLds
  __shared__ double red[ANT / 64];
  const GemmArgs& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int quad = wave & 3;
  const bool re_part = wave < 4;
  const int wm = (quad & 1) * 32, wn = (quad >> 1) * 32;

  const int ntiles = gridDim.x, bid = blockIdx.x;
  int logical = bid;
  {
    const int per = ntiles / kXCDs;
    if (bid < per * kXCDs) logical = (bid % kXCDs) * per + bid / kXCDs;
  }
  int tm, tn;
  if ((EPI == EPI_YDEF || EPI == EPI_STORE) && g.herm) {
    herm_tile(logical, g.tiles_n, tm, tn);  // the upper triangle of tiles
  } else {
    // groups of kGroup tile rows, column by column within a group: the 32 blocks
    // an XCD runs at once share 4 row panels and 8 column panels
    constexpr int kGroup = 4;
    const int group = logical / (kGroup * g.tiles_n);
    const int first_m = group * kGroup;
    const int gsize = min(g.tiles_m - first_m, kGroup);
    const int within = logical - group * kGroup * g.tiles_n;
    tm = first_m + within % gsize;
    tn = within / gsize;
  }
  const int m0 = tm * ABM, n0 = tn * ABM;

  // S digits per operand, pairs s + t <= S + 1 (diagonals d = 2 .. S + 1)
  const int KB = a.Kp / OBK, KS = a.Kp / 32;
  const long pA = oz_plane_bytes(g.m, a.Kp), pB = oz_plane_bytes(g.n, a.Kp);
  const long sA = kParts * pA, sB = kParts * pB;
  // real part: Ar Br + (A part pa2) Bi; imaginary part: Ar Bi + (A part pa3) Br
  // (pa2 = -Ai, pa3 = Ai; conjugated op(A): pa2 = Ai, pa3 = -Ai)
  const int pax = re_part ? (a.conjA ? 1 : 2) : (a.conjA ? 2 : 1);
  const int pbf = re_part ? 0 : 1, pbs = re_part ? 1 : 0;

  // this lane's source offset within a plane for each half region (rows 0-31,
  // 32-63 of the tile) at K-block 0, K-half 0; rows past the padded matrix read
  // its last row block (their outputs are not stored)
  const int uwave = __builtin_amdgcn_readfirstlane(wave);
  const int RBA = oz_rows_pad(g.m) / 16, RBB = oz_rows_pad(g.n) / 16;
  int offA[2], offB[2];
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const int r = 32 * h + (lane >> 1);
    const int c = (lane & 1) ^ ap_lsw(r);
    const int rba = min((m0 + r) >> 4, RBA - 1), rbb = min((n0 + r) >> 4, RBB - 1);
    const int rowa = rba * 16 + (r & 15), rowb = rbb * 16 + (r & 15);
    offA[h] = rba * KB * 1024 + (r & 15) * 64 + ((c ^ chunk_swz(rowa)) << 4);
    offB[h] = rbb * KB * 1024 + (r & 15) * 64 + ((c ^ chunk_swz(rowb)) << 4);
  }
  // The step's 1 KiB load instructions: 6 S for A (slice q / 6, part (q % 6) / 2,
  // half q % 2), 4 S for B (slice q / 4, part (q / 2) % 2, half q % 2). Wave w
  // issues A instructions w, w + 8, ... and B instructions w, w + 8, ...; past
  // the last one a wave repeats it (the same bytes to the same place). Source
  // offsets (plane and lane part, K-block 0, K-half 0) and LDS offsets are fixed
  // for the whole tile.
  constexpr int NW = ANT / 64;
  constexpr int kQA = (6 * S + NW - 1) / NW, kQ = kQA + (4 * S + NW - 1) / NW;
  int goff[kQ], loff[kQ];
#pragma unroll
  for (int k = 0; k < kQ; k++) {
    if (k < kQA) {
      const int q = min(uwave + NW * k, 6 * S - 1);
      const int sl = q / 6, rem = q - 6 * sl, part = rem >> 1, h = rem & 1;
      goff[k] = (int)(sl * sA + part * pA) + offA[h];
      loff[k] = (3 * sl + part) * kApRegion + h * 1024;
    } else {
      const int q = min(uwave + NW * (k - kQA), 4 * S - 1), t = q >> 2, part = (q >> 1) & 1, h = q & 1;
      goff[k] = (int)(t * sB + part * pB) + offB[h];
      loff[k] = (3 * kApS + 2 * t + part) * kApRegion + h * 1024;
    }
  }
  // load instructions k0 .. k1-1 of step ks into a stage
  auto issue = [&](int ks, int stage, int k0, int k1) {
    const int kbo = (ks >> 1) * 1024, kx = (ks & 1) << 5;
    int8_t* lb = lds + stage * kApStageBytes;
#pragma unroll
    for (int k = 0; k < kQ; k++) {
      if (k >= k0 && k < k1) {
        // the plane offsets are multiples of 1 KiB, so the K-half flips bit 5 of
        // the lane part only
        const int8_t* src = (k < kQA ? a.A : a.B) + kbo + (goff[k] ^ kx);
        __builtin_amdgcn_global_load_lds((gbl_ptr_t*)src, (lds_ptr_t*)(lb + loff[k]), 16, 0, 0);
      }
    }
  };
  // fragment offsets of this lane within a region: row (lane & 31) of the wave's
  // block, K-chunk lane >> 5
  const int ra = wm + (lane & 31), rb = wn + (lane & 31);
  const int fa = ra * 32 + ((((lane >> 5) ^ ap_lsw(ra))) << 4);
  const int fb = rb * 32 + ((((lane >> 5) ^ ap_lsw(rb))) << 4);

  v16i acc[S];
  auto barrier = [&]() {
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  auto load_a = [&](const int8_t* lb, int s, v4i& x0, v4i& xx) {
    x0 = *(const v4i*)(lb + (3 * s) * kApRegion + fa);
    xx = *(const v4i*)(lb + (3 * s + pax) * kApRegion + fa);
  };
  // FP64 partial sums between segments (K beyond kApSeg steps) live in the
  // per-tile scratch (64 x 64 double2 per tile: one double per wave, v and lane)
  double* sp = a.scratch ? (double*)a.scratch + ((long)bid * NW + wave) * 1024 + lane : nullptr;
  double val[16];

  issue(0, 0, 0, kQ);
  for (int seg0 = 0; seg0 < KS; seg0 += kApSeg) {
    const int seg1 = min(KS, seg0 + kApSeg);
#pragma unroll
    for (int di = 0; di < S; di++) acc[di] = v16i{};
    for (int ks = seg0; ks < seg1; ks++) {
      // wait for this step's loads (issued one step earlier), barrier (every
      // wave's loads have landed; the other stage is no longer read), then all
      // pairs of this step, with the next step's loads issued between them
      __builtin_amdgcn_s_waitcnt(kWaitVm0);
      barrier();
      const int8_t* lb = lds + (ks & 1) * kApStageBytes;
      v4i bf[S], bs[S];
#pragma unroll
      for (int t = 0; t < S; t++) {
        bf[t] = *(const v4i*)(lb + (3 * kApS + 2 * t + pbf) * kApRegion + fb);
        bs[t] = *(const v4i*)(lb + (3 * kApS + 2 * t + pbs) * kApRegion + fb);
      }
      v4i a0, ax;
      load_a(lb, 0, a0, ax);
      const bool more = ks + 1 < KS;
#pragma unroll
      for (int s = 0; s < S; s++) {
        // the next slice's fragments are requested before this slice's MFMAs,
        // and with them a share of the next step's loads
        v4i n0, nx;
        if (s + 1 < S) load_a(lb, s + 1, n0, nx);
        if (more) issue(ks + 1, (ks + 1) & 1, s * kQ / S, (s + 1) * kQ / S);
#pragma unroll
        for (int t = 0; s + t < S; t++) {
          // slices s + 1, t + 1: diagonal d = s + t + 2
          acc[s + t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, bf[t], acc[s + t], 0, 0, 0);
          acc[s + t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ax, bs[t], acc[s + t], 0, 0, 0);
        }
        a0 = n0;
        ax = nx;
      }
    }
    // fold: every term acc 2^{-8 d} is exact in FP64; smallest weights first,
    // then the partial sum of the earlier segments
    const bool first = seg0 == 0, last = seg1 == KS;
#pragma unroll
    for (int v = 0; v < 16; v++) {
      double x = 0;
#pragma unroll
      for (int di = S - 1; di >= 0; di--) x += (double)acc[di][v] * __builtin_ldexp(1.0, -8 * (di + 2));
      if (!first) x = sp[v * 64] + x;
      if (!last) sp[v * 64] = x;
      val[v] = x;
    }
  }
  // imaginary parts to the waves of the real parts (the stages are free once
  // every wave is past its last fragment read)
  double* xch = (double*)lds + (quad * 16) * 64 + lane;
  __syncthreads();
  if (!re_part) {
#pragma unroll
    for (int v = 0; v < 16; v++) xch[v * 64] = val[v];
  }
  __syncthreads();
  double part = 0;
  if (re_part) {
#pragma unroll
    for (int v = 0; v < 16; v++) {
      const int i = m0 + wm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      const int j = n0 + wn + (lane & 31);
      if (i < g.m && j < g.n) {
        const int e = a.ea[i] + a.eb[j];
        const double re = ldexp(val[v], e), im = ldexp(xch[v * 64], e);
        if (EPI == EPI_STORE && g.c64) epi_element<EPI, float>(g, i, j, mk<float>((float)re, (float)im), part);
        else epi_element<EPI, double>(g, i, j, mk<double>(re, im), part);
      }
    }
  }
  if constexpr (EPI == EPI_SPLIT || EPI == EPI_YDEF) epi_reduce<ANT>(g, part, red, bid);
}

// --------------------------------------------- windowed product (double-double)
//
// The double-double tier's products: S digits per operand (14 by default) and pairs
// up to s + t = S + 1 (105 pairs), too many diagonals for one set of accumulators.
// The slices are taken in windows of kWin = 4 per operand: window (wa, wb) holds
// A slices 4 wa + 1 .. 4 wa + 4 and B slices 4 wb + 1 .. 4 wb + 4, whose pairs lie on
// the diagonals d0 .. d0 + 6, d0 = 4 (wa + wb) + 2; those up to dmax are formed
// (local s + t <= DL = min(6, dmax - d0)). With dmax = S + 1 a window at the end of
// the slice range reaches only the slices that exist (DL + 1 <= slices left). Each
// window is one K-sweep in the manner of the all-pairs kernel (64 x 64 tile, 8 waves,
// one part per wave, the staged slices limited to min(4, DL + 1) per operand: two
// LDS stages of up to 40 KiB, four for windows of one or two slices). After each segment the window's diagonal sums are
// added, smallest weight first, to a three-term FP64 expansion per output with two
// exact TwoSum steps each (the partial sums can exceed the final value by the ratio
// of the row and column scales to it, which two terms would turn into error); the
// expansion lives in the per-tile scratch between windows and becomes double-double
// after the last one.
constexpr int kWin = 4;
constexpr int kWinLds = 2 * kWin * 5 * kApRegion;  // two stages of 40 KiB
static_assert(4 * 16 * 64 * 2 * sizeof(double) <= (size_t)kWinLds, "hi and lo of the imaginary parts fit");

template <int EPI>
__global__ __launch_bounds__(ANT) __attribute__((amdgpu_waves_per_eu(2, 2))) void oz_gemm_windows_kernel(
    OzArgs a) {
  extern __shared__ __align__(16) int8_t lds[];  // kWinLds
  __shared__ double red[ANT / 64];
  const GemmArgs& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int quad = wave & 3;
  const bool re_part = wave < 4;
  const int wm = (quad & 1) * 32, wn = (quad >> 1) * 32;

  const int ntiles = gridDim.x, bid = blockIdx.x;
  int logical = bid;
  {
    const int per = ntiles / kXCDs;
    if (bid < per * kXCDs) logical = (bid % kXCDs) * per + bid / kXCDs;
  }
  int tm, tn;
  if (EPI == EPI_YDEF && g.herm) {
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
  const int m0 = tm * ABM, n0 = tn * ABM;

  const int KB = a.Kp / OBK, KS = a.Kp / 32;
  const long pA = oz_plane_bytes(g.m, a.Kp), pB = oz_plane_bytes(g.n, a.Kp);
  const long sA = kParts * pA, sB = kParts * pB;
  const int pax = re_part ? (a.conjA ? 1 : 2) : (a.conjA ? 2 : 1);
  const int pbf = re_part ? 0 : 1, pbs = re_part ? 1 : 0;

  const int uwave = __builtin_amdgcn_readfirstlane(wave);
  const int RBA = oz_rows_pad(g.m) / 16, RBB = oz_rows_pad(g.n) / 16;
  int offA[2], offB[2];
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const int r = 32 * h + (lane >> 1);
    const int c = (lane & 1) ^ ap_lsw(r);
    const int rba = min((m0 + r) >> 4, RBA - 1), rbb = min((n0 + r) >> 4, RBB - 1);
    const int rowa = rba * 16 + (r & 15), rowb = rbb * 16 + (r & 15);
    offA[h] = rba * KB * 1024 + (r & 15) * 64 + ((c ^ chunk_swz(rowa)) << 4);
    offB[h] = rbb * KB * 1024 + (r & 15) * 64 + ((c ^ chunk_swz(rowb)) << 4);
  }
  const int ra = wm + (lane & 31), rb = wn + (lane & 31);
  const int fa = ra * 32 + ((((lane >> 5) ^ ap_lsw(ra))) << 4);
  const int fb = rb * 32 + ((((lane >> 5) ^ ap_lsw(rb))) << 4);
  auto barrier = [&]() {
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };

  // the three-term expansions of this wave's 16 outputs per lane, between windows
  constexpr int NW = ANT / 64;
  double* sp = (double*)a.scratch + ((long)bid * NW + wave) * 3072 + lane;
  int nwin = 0;  // windows with at least one pair
  for (int wa = 0; wa * kWin < a.SA; wa++)
    for (int wb = 0; wb * kWin < a.SB; wb++)
      if (kWin * (wa + wb) + 2 <= a.dmax) nwin++;
  int widx = 0;
  int nfold = 0;  // folds so far
  const int nwa = (a.SA + kWin - 1) / kWin, nwb = (a.SB + kWin - 1) / kWin;

  // one band of windows (the same wa + wb, hence the same diagonals d0 .. d0 + DL):
  // their K-sweeps, accumulated into the same sums
  auto band = [&](auto dlc, int bnd) {
    constexpr int DL = decltype(dlc)::value;
    constexpr int NS = DL < kWin - 1 ? DL + 1 : kWin;  // slices staged per operand
    constexpr int nIA = 6 * NS, nI = nIA + 4 * NS, kQ = (nI + NW - 1) / NW;
    // a stage holds 3 NS A regions then 2 NS B regions; windows of one or two
    // slices have room for four stages (loads three steps ahead), the others two
    constexpr int kStB = 5 * NS * kApRegion;
    constexpr int NST = kWinLds / kStB >= 4 ? 4 : 2;
    constexpr int kVmAhead = 0x0F70 | ((NST - 2) * kQ);  // vmcnt: later steps' loads may be in flight
    static_assert((NST - 2) * kQ < 16 && NST * kStB <= kWinLds, "pipeline of a window");
    const int d0 = kWin * bnd + 2;
    int goff[kQ], loff[kQ];
#pragma unroll
    for (int k = 0; k < kQ; k++) {
      const int q = min(uwave + NW * k, nI - 1);  // past the last: repeat it
      if (q < nIA) {
        const int sl = q / 6, rem = q - 6 * sl, part = rem >> 1, h = rem & 1;
        goff[k] = (int)(sl * sA + part * pA) + offA[h];
        loff[k] = (3 * sl + part) * kApRegion + h * 1024;
      } else {
        const int qb = q - nIA, t = qb >> 2, part = (qb >> 1) & 1, h = qb & 1;
        goff[k] = (int)(t * sB + part * pB) + offB[h];
        loff[k] = (3 * NS + 2 * t + part) * kApRegion + h * 1024;
      }
    }
    v16i acc[DL + 1];
    int acc_steps = 0;  // K-steps in the sums since the last fold
    const int wa_lo = max(0, bnd - (nwb - 1)), wa_hi = min(nwa - 1, bnd);
    for (int wa = wa_lo; wa <= wa_hi; wa++) {
      const int wb = bnd - wa;
      const bool last_in_band = wa == wa_hi;
      const int8_t* Aw = a.A + (long)(kWin * wa) * sA;
      const int8_t* Bw = a.B + (long)(kWin * wb) * sB;
      auto issue = [&](int ks, int stage, int k0, int k1) {
        const int kbo = (ks >> 1) * 1024, kx = (ks & 1) << 5;
        int8_t* lb = lds + stage * kStB;
#pragma unroll
        for (int k = 0; k < kQ; k++) {
          if (k >= k0 && k < k1) {
            const int q = min(uwave + NW * k, nI - 1);
            const int8_t* src = (q < nIA ? Aw : Bw) + kbo + (goff[k] ^ kx);
            __builtin_amdgcn_global_load_lds((gbl_ptr_t*)src, (lds_ptr_t*)(lb + loff[k]), 16, 0, 0);
          }
        }
      };
      barrier();  // the previous window no longer reads the stages
#pragma unroll
      for (int j = 0; j < NST - 1; j++)
        if (j < KS) issue(j, j, 0, kQ);
      // The windows of a band (the same wa + wb) put their pairs on the same diagonals
      // with the same weights, so they accumulate into the same int32 sums; a fold
      // empties them after kApSeg K-steps (at most 4 pairs per diagonal, 2^22 per step:
      // the sums stay below 2^30) and at the end of the band. Per band one fold instead
      // of one per window: 5 instead of 15 with 20 digits, 4 instead of 10 with 14.
      for (int seg0 = 0; seg0 < KS;) {
        const int seg1 = min(KS, seg0 + (kApSeg - acc_steps));
        if (acc_steps == 0) {
#pragma unroll
          for (int di = 0; di <= DL; di++) acc[di] = v16i{};
        }
        for (int ks = seg0; ks < seg1; ks++) {
          // this step's loads have landed once at most the NST - 2 later steps' are
          // in flight (all of them near the end, where fewer were issued)
          if (ks + NST - 2 < KS) __builtin_amdgcn_s_waitcnt(kVmAhead);
          else __builtin_amdgcn_s_waitcnt(kWaitVm0);
          barrier();
          const int8_t* lb = lds + (ks % NST) * kStB;
          v4i bf[NS], bs[NS];
#pragma unroll
          for (int t = 0; t < NS; t++) {
            bf[t] = *(const v4i*)(lb + (3 * NS + 2 * t + pbf) * kApRegion + fb);
            bs[t] = *(const v4i*)(lb + (3 * NS + 2 * t + pbs) * kApRegion + fb);
          }
          v4i a0 = *(const v4i*)(lb + fa), ax = *(const v4i*)(lb + pax * kApRegion + fa);
          const int nxt = ks + NST - 1;  // the step whose loads go out now
          const bool more = nxt < KS;
#pragma unroll
          for (int s = 0; s < NS; s++) {
            v4i n0, nx;
            if (s + 1 < NS) {
              n0 = *(const v4i*)(lb + (3 * (s + 1)) * kApRegion + fa);
              nx = *(const v4i*)(lb + (3 * (s + 1) + pax) * kApRegion + fa);
            }
            if (more) issue(nxt, nxt % NST, s * kQ / NS, (s + 1) * kQ / NS);
#pragma unroll
            for (int t = 0; t < NS && s + t <= DL; t++) {
              acc[s + t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, bf[t], acc[s + t], 0, 0, 0);
              acc[s + t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ax, bs[t], acc[s + t], 0, 0, 0);
            }
            a0 = n0;
            ax = nx;
          }
        }
        acc_steps += seg1 - seg0;
        seg0 = seg1;
        if (acc_steps < kApSeg && !(last_in_band && seg1 == KS)) continue;
        // fold: x = acc 2^{-8 d} (exact) into (h, m, l) with two TwoSum steps each
        const bool first = nfold == 0;
        const bool final = widx == nwin - 1 && seg1 == KS;
        nfold++;
        acc_steps = 0;
#pragma unroll
        for (int v = 0; v < 16; v++) {
          double h = 0, m = 0, l = 0;
          if (!first) {
            h = sp[v * 64];
            m = sp[1024 + v * 64];
            l = sp[2048 + v * 64];
          }
#pragma unroll
          for (int di = DL; di >= 0; di--) {
            const double x = (double)acc[di][v] * __builtin_ldexp(1.0, -8 * (d0 + di));
            double s0, e0, s1, e1;
            two_sum(h, x, s0, e0);
            two_sum(m, e0, s1, e1);
            h = s0;
            m = s1;
            l += e1;
          }
          if (!final) {
            sp[v * 64] = h;
            sp[1024 + v * 64] = m;
            sp[2048 + v * 64] = l;
          } else if (g.Cmid) {
            // triple-double: the expansion renormalized
            double t0, t1, t2;
            td_renorm(h, m, l, t0, t1, t2);
            sp[v * 64] = t0;
            sp[1024 + v * 64] = t1;
            sp[2048 + v * 64] = t2;
          } else {
            // to double-double, kept in the first two slots for the epilogue
            double hh, e, dh, dl;
            two_sum(h, m, hh, e);
            e += l;
            fast_two_sum(hh, e, dh, dl);
            sp[v * 64] = dh;
            sp[1024 + v * 64] = dl;
          }
        }
      }
      widx++;
    }
  };
  for (int bnd = 0; bnd < nwa + nwb - 1; bnd++) {
    const int d0 = kWin * bnd + 2;
    if (d0 > a.dmax) break;
    switch (min(6, a.dmax - d0)) {
      case 6: band(std::integral_constant<int, 6>{}, bnd); break;
      case 5: band(std::integral_constant<int, 5>{}, bnd); break;
      case 4: band(std::integral_constant<int, 4>{}, bnd); break;
      case 3: band(std::integral_constant<int, 3>{}, bnd); break;
      case 2: band(std::integral_constant<int, 2>{}, bnd); break;
      case 1: band(std::integral_constant<int, 1>{}, bnd); break;
      default: band(std::integral_constant<int, 0>{}, bnd); break;
    }
  }
  double* xch = (double*)lds + (quad * 16) * 64 + lane;
  if (g.Cmid) {
    // triple-double: the imaginary parts' three terms to the waves of the real parts,
    // in two rounds through the stages (two terms, then the third)
    double x0[16], x1[16], x2[16], y2[16];
#pragma unroll
    for (int v = 0; v < 16; v++) {
      x0[v] = sp[v * 64];
      x1[v] = sp[1024 + v * 64];
      x2[v] = sp[2048 + v * 64];
    }
    __syncthreads();
    if (!re_part) {
#pragma unroll
      for (int v = 0; v < 16; v++) {
        xch[v * 64] = x0[v];
        xch[4096 + v * 64] = x1[v];
      }
    }
    __syncthreads();
    double y0[16], y1[16];
#pragma unroll
    for (int v = 0; v < 16; v++) {
      y0[v] = xch[v * 64];
      y1[v] = xch[4096 + v * 64];
    }
    __syncthreads();
    if (!re_part) {
#pragma unroll
      for (int v = 0; v < 16; v++) xch[v * 64] = x2[v];
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 16; v++) y2[v] = xch[v * 64];
    double part = 0;
    if (re_part) {
#pragma unroll
      for (int v = 0; v < 16; v++) {
        const int i = m0 + wm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int j = n0 + wn + (lane & 31);
        if (i < g.m && j < g.n) {
          const int e = a.ea[i] + a.eb[j];
          epi_element_td<EPI>(g, i, j, mk<double>(ldexp(x0[v], e), ldexp(y0[v], e)),
                              mk<double>(ldexp(x1[v], e), ldexp(y1[v], e)),
                              mk<double>(ldexp(x2[v], e), ldexp(y2[v], e)), part);
        }
      }
    }
    if constexpr (EPI == EPI_SPLIT || EPI == EPI_YDEF) epi_reduce<ANT>(g, part, red, bid);
    return;
  }
  // imaginary parts (hi, lo) to the waves of the real parts
  double hi[16], lo[16];
#pragma unroll
  for (int v = 0; v < 16; v++) {
    hi[v] = sp[v * 64];
    lo[v] = sp[1024 + v * 64];
  }
  __syncthreads();
  if (!re_part) {
#pragma unroll
    for (int v = 0; v < 16; v++) {
      xch[v * 64] = hi[v];
      xch[4096 + v * 64] = lo[v];
    }
  }
  __syncthreads();
  double part = 0;
  if (re_part) {
#pragma unroll
    for (int v = 0; v < 16; v++) {
      const int i = m0 + wm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      const int j = n0 + wn + (lane & 31);
      if (i < g.m && j < g.n) {
        const int e = a.ea[i] + a.eb[j];
        epi_element_dd<EPI>(g, i, j, mk<double>(ldexp(hi[v], e), ldexp(xch[v * 64], e)),
                            mk<double>(ldexp(lo[v], e), ldexp(xch[4096 + v * 64], e)), part);
      }
    }
  }
  if constexpr (EPI == EPI_SPLIT || EPI == EPI_YDEF) epi_reduce<ANT>(g, part, red, bid);
}

// The large-tile kernel is used when it still gives every CU a tile, and for
// every double-double product.
static bool use_large_tiles(int m, int n, bool dd) {
  return dd || ceil_div(m, PBM) * ceil_div(n, PBN) >= kCUs;
}

// The windowed kernel takes the double-double tier's products (S digits per
// operand, pairs s + t <= S + 1) with a 64 x 64 tile per CU.
static bool use_windows(int m, int n, bool dd, int SA, int SB, int dmax, int k, bool td = false) {
  const long span = (long)(SA + kWin) * kParts * oz_plane_bytes(m > n ? m : n, oz_kp(k));
  // triple-double outputs: this kernel at every size (the only one that writes them)
  return dd && SA == SB && SA >= 1 && dmax == SA + 1 && span < 2147483647L &&
         (td || ceil_div(m, ABM) * ceil_div(n, ABM) >= kCUs);
}

// The all-pairs kernel takes the FP64 tier's products (S digits per operand,
// pairs s + t <= S + 1, S <= kApS) with a 64 x 64 tile per CU.
static bool use_allpairs(int m, int n, bool dd, int SA, int SB, int dmax, int k) {
  // the kernel addresses the slices of an operand with 32-bit offsets
  const long span = (long)SA * kParts * oz_plane_bytes(m > n ? m : n, oz_kp(k));
  return !dd && SA == SB && SA >= 1 && SA <= kApS && dmax == SA + 1 && span < 2147483647L &&
         ceil_div(m, ABM) * ceil_div(n, ABM) >= kCUs;
}

bool oz_allpairs_ok(int m, int n, int k, int S) { return use_allpairs(m, n, false, S, S, S + 1, k); }

bool oz_td_ok(int m, int n, int k, int S) { return use_windows(m, n, true, S, S, S + 1, k, true); }

// Scratch for either large-tile kernel (the all-pairs one needs at most the same:
// a 64 x 64 double2 tile per 64-tile, and only for K past one segment).
size_t oz_gemm_scratch_bytes(int m, int n, bool dd) {
  // a 64 x 64 tile: one double2 per output (all-pairs), or three doubles per output
  // and part (windowed)
  const size_t t64 = (size_t)ceil_div(m, ABM) * ceil_div(n, ABM);
  const size_t ap = t64 * ABM * ABM * (dd ? 6 * sizeof(double) : sizeof(double2));
  if (!use_large_tiles(m, n, dd)) return t64 < (size_t)kCUs ? 0 : ap;
  const size_t lt = (size_t)ceil_div(m, PBM) * ceil_div(n, PBN) * PBM * PBN * sizeof(double2) * (dd ? 3 : 1);
  return lt > ap ? lt : ap;
}

// The small-tile kernel sums one product per accumulator over a whole diagonal
// (at most min(SA, SB) pairs of Kp terms, each at most 2^14 in magnitude); the
// large-tile kernel folds in segments and is exact for every size.
bool oz_gemm_exact(int m, int n, int k, int SA, int SB, bool dd) {
  if (use_large_tiles(m, n, dd)) return true;
  const long pairs = SA < SB ? SA : SB;
  return pairs * (long)oz_kp(k) * 16384L < 2147483648L;
}

int oz_gemm_tiles(int m, int n, int k, bool dd, bool herm, int SA, int SB, int dmax, bool td) {
  if (use_allpairs(m, n, dd, SA, SB, dmax, k) || use_windows(m, n, dd, SA, SB, dmax, k, td)) {
    const int t = ceil_div(n, ABM);
    return herm ? t * (t + 1) / 2 : ceil_div(m, ABM) * t;
  }
  if (use_large_tiles(m, n, dd)) {
    const int t = ceil_div(n, PBN);
    return herm ? t * (t + 1) / 2 : ceil_div(m, PBM) * t;
  }
  return ceil_div(m, OBM) * ceil_div(n, OBN);
}

template <int EPI>
static hipError_t launch_large(bool dd, int nt, const OzArgs& a, hipStream_t st) {
  const size_t lds = (size_t)kStages * kStageBytes;
  hipError_t e;
  if (dd) {
    e = hipFuncSetAttribute((const void*)oz_gemm2_kernel<EPI, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e != hipSuccess) return e;
    oz_gemm2_kernel<EPI, true><<<dim3(nt), dim3(PNT), lds, st>>>(a);
  } else {
    e = hipFuncSetAttribute((const void*)oz_gemm2_kernel<EPI, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e != hipSuccess) return e;
    oz_gemm2_kernel<EPI, false><<<dim3(nt), dim3(PNT), lds, st>>>(a);
  }
  return hipGetLastError();
}

template <int EPI, int S>
static hipError_t launch_allpairs_s(int nt, const OzArgs& a, hipStream_t st) {
  hipError_t e = hipFuncSetAttribute((const void*)oz_gemm_allpairs_kernel<EPI, S>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kApLds);
  if (e != hipSuccess) return e;
  oz_gemm_allpairs_kernel<EPI, S><<<dim3(nt), dim3(ANT), kApLds, st>>>(a);
  return hipGetLastError();
}

template <int EPI>
static hipError_t launch_windows(int nt, const OzArgs& a, hipStream_t st) {
  hipError_t e = hipFuncSetAttribute((const void*)oz_gemm_windows_kernel<EPI>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kWinLds);
  if (e != hipSuccess) return e;
  oz_gemm_windows_kernel<EPI><<<dim3(nt), dim3(ANT), kWinLds, st>>>(a);
  return hipGetLastError();
}

template <int EPI>
static hipError_t launch_allpairs(int nt, const OzArgs& a, hipStream_t st) {
  switch (a.SA) {
    case 1: return launch_allpairs_s<EPI, 1>(nt, a, st);
    case 2: return launch_allpairs_s<EPI, 2>(nt, a, st);
    case 3: return launch_allpairs_s<EPI, 3>(nt, a, st);
    case 4: return launch_allpairs_s<EPI, 4>(nt, a, st);
    case 5: return launch_allpairs_s<EPI, 5>(nt, a, st);
    case 6: return launch_allpairs_s<EPI, 6>(nt, a, st);
    case 7: return launch_allpairs_s<EPI, 7>(nt, a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t oz_gemm(int epi, const int8_t* A, const int* ea, int SA, const int8_t* B, const int* eb,
                   int SB, int conjA, int dmax, GemmArgs g, void* scratch, hipStream_t st,
                   bool dd) {
  if (g.m == 0 || g.n == 0) return hipSuccess;
  const bool ap = use_allpairs(g.m, g.n, dd, SA, SB, dmax, g.k);
  // Hermitian / skew-Hermitian STORE and complex64 outputs: the all-pairs kernel only
  const bool herm_store = epi == EPI_STORE && (g.herm == 1 || g.herm == -1) && g.m == g.n && ap;
  if (g.herm && !herm_store && (epi != EPI_YDEF || g.herm != 1 || g.m != g.n)) return hipErrorInvalidValue;
  if (g.c64 && (epi != EPI_STORE || !ap)) return hipErrorInvalidValue;
  if (ap) {
    g.tiles_m = ceil_div(g.m, ABM);
    g.tiles_n = ceil_div(g.n, ABM);
    const int nt = oz_gemm_tiles(g.m, g.n, g.k, dd, g.herm != 0, SA, SB, dmax);
    // the FP64 partial sums need the scratch only past one segment
    if (!scratch && oz_kp(g.k) / 32 > kApSeg) return hipErrorInvalidValue;
    OzArgs a{A, ea, B, eb, SA, SB, dmax, conjA, oz_kp(g.k), g, (double2*)scratch};
    switch (epi) {
      case EPI_STORE: return launch_allpairs<EPI_STORE>(nt, a, st);
      case EPI_ADD: return launch_allpairs<EPI_ADD>(nt, a, st);
      case EPI_SPLIT: return launch_allpairs<EPI_SPLIT>(nt, a, st);
      case EPI_YDEF: return launch_allpairs<EPI_YDEF>(nt, a, st);
      default: return hipErrorInvalidValue;
    }
  }
  const bool td = g.Cmid != nullptr;
  if (td && !use_windows(g.m, g.n, dd, SA, SB, dmax, g.k, true)) return hipErrorInvalidValue;
  if (use_windows(g.m, g.n, dd, SA, SB, dmax, g.k, td)) {
    if (!scratch) return hipErrorInvalidValue;
    g.tiles_m = ceil_div(g.m, ABM);
    g.tiles_n = ceil_div(g.n, ABM);
    const int nt = oz_gemm_tiles(g.m, g.n, g.k, dd, g.herm != 0, SA, SB, dmax, td);
    OzArgs a{A, ea, B, eb, SA, SB, dmax, conjA, oz_kp(g.k), g, (double2*)scratch};
    switch (epi) {
      case EPI_STORE: return launch_windows<EPI_STORE>(nt, a, st);
      case EPI_ADD: return launch_windows<EPI_ADD>(nt, a, st);
      case EPI_SPLIT: return launch_windows<EPI_SPLIT>(nt, a, st);
      case EPI_YDEF: return launch_windows<EPI_YDEF>(nt, a, st);
      default: return hipErrorInvalidValue;
    }
  }
  if (use_large_tiles(g.m, g.n, dd)) {
    if (!scratch) return hipErrorInvalidValue;
    g.tiles_m = ceil_div(g.m, PBM);
    g.tiles_n = ceil_div(g.n, PBN);
    const int nt = oz_gemm_tiles(g.m, g.n, g.k, dd, g.herm != 0, SA, SB, dmax);
    OzArgs a{A, ea, B, eb, SA, SB, dmax, conjA, oz_kp(g.k), g, (double2*)scratch};
    switch (epi) {
      case EPI_STORE: return launch_large<EPI_STORE>(dd, nt, a, st);
      case EPI_ADD: return launch_large<EPI_ADD>(dd, nt, a, st);
      case EPI_SPLIT: return launch_large<EPI_SPLIT>(dd, nt, a, st);
      case EPI_YDEF: return launch_large<EPI_YDEF>(dd, nt, a, st);
      default: return hipErrorInvalidValue;
    }
  }
  g.tiles_m = ceil_div(g.m, OBM);
  g.tiles_n = ceil_div(g.n, OBN);
  const int nt = g.tiles_m * g.tiles_n;
  OzArgs a{A, ea, B, eb, SA, SB, dmax, conjA, oz_kp(g.k), g, nullptr};
  switch (epi) {
    case EPI_STORE: hipLaunchKernelGGL(oz_gemm_kernel<EPI_STORE>, dim3(nt), dim3(ONT), 0, st, a); break;
    case EPI_ADD: hipLaunchKernelGGL(oz_gemm_kernel<EPI_ADD>, dim3(nt), dim3(ONT), 0, st, a); break;
    case EPI_SPLIT: hipLaunchKernelGGL(oz_gemm_kernel<EPI_SPLIT>, dim3(nt), dim3(ONT), 0, st, a); break;
    case EPI_YDEF: hipLaunchKernelGGL(oz_gemm_kernel<EPI_YDEF>, dim3(nt), dim3(ONT), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sr
