// Ozaki scheme II on CDNA4 INT8 matrix cores: the complex FP64 products of the
// refinement (the hp products of Algorithm 4; Section 3 computes them with an
// Ozaki-scheme toolbox) from residues modulo pairwise coprime moduli, multiplied
// exactly and combined by the Chinese remainder theorem.
//
// Scaling. Every row i of op(A) gets an exponent t_i = E_i - b, E_i the least
// exponent with |re a_ik|, |im a_ik| < 2^E_i over the row, and is replaced by the
// integers a'_ik = rint(a_ik 2^-t_i), |a'| <= 2^b; every column j of B likewise
// (u_j, b'_kj). Each entry then carries an error of at most 2^(t_i - 1), i.e.
// 2^-b of the row maximum: b = 55 matches the seven 8-bit digits of the digit
// slices (2^-55 of the row maximum).
//
// Product. The integer product C' = A' B' has |re|, |im| <= 2 K 2^2b. With
// moduli m_1 .. m_N (pairwise coprime, at most 256) and M = m_1 ... m_N >
// 8 K 2^2b, C' is the residue of its value modulo M in (-M/8, M/8). For every
// modulus the balanced residues of A' and B' (int8) are multiplied on
// v_mfma_i32_32x32x32_i8, the real part as [Ar, -Ai] [Br; Bi] and the imaginary
// part as [Ar, Ai] [Bi; Br] (the negated imaginary residues are stored beside the
// others, as the digit slices store negated digits): every sum stays exact in
// int32 for K < 2^16 (terms at most 2^14). The sums are reduced modulo m_k to
// r_k in [0, m_k).
//
// Reconstruction. X = sum_k r_k w_k - q M with w_k = (M / m_k) ((M / m_k)^-1 mod
// m_k) and q = rint(sum_k r_k w_k / M). The sum is formed exactly in 40-bit
// limbs: every r_k w_k,l is below 2^48 and a sum of at most 20 of them below
// 2^53, so each limb sum S_l is an exact double; X_l = S_l - q M_l is exact too.
// Carries between the limbs (exact integer operations) leave X = X_3 2^120 +
// X_2 2^80 + X_1 2^40 + X_0 with 0 <= X_0, X_1, X_2 < 2^40 and |X_3| < 8, which
// is summed in double-double (error below 2^-100 of |X|). Then C_ij = X 2^(t_i + u_j)
// rounded once to FP64.
//
// N products of 8 K m n int8 operations each replace the 28 slice pairs of the
// digit-slice product at the same accuracy (N = 16 for b = 55 and K <= 4096).
#include <string.h>

#include <vector>

#include "epilogue.hpp"
#include "ozaki_layout.hpp"

namespace sr {

constexpr int kCrtMaxMod = 20, kCrtLimbs = 4, kCrtLimbBits = 40;
// pairwise coprime (256 = 2^8, 255 = 3 5 17, 253 = 11 23, 247 = 13 19, 217 = 7 31,
// the rest prime), largest first
static const int kCrtModuli[kCrtMaxMod] = {256, 255, 253, 251, 247, 241, 239, 233, 229, 227,
                                           223, 217, 211, 199, 197, 193, 191, 181, 179, 173};

struct CrtConst {
  int N;
  int mod[kCrtMaxMod];
  double inv[kCrtMaxMod];                // 1 / m_k (rounded)
  double w[kCrtMaxMod][kCrtLimbs];       // limb l of w_k: bits 40 l .. 40 l + 39
  double M[kCrtLimbs];                   // limbs of M
  double Mf;                             // M rounded to FP64
};

// ------------------------------------------------------------------ host plan

// Little-endian base-2^32 integers, only as large as the products of at most 20
// moduli (160 bits).
namespace {
using Big = std::vector<uint32_t>;
Big big_mul(const Big& x, uint32_t s) {
  Big r(x.size() + 1, 0);
  uint64_t c = 0;
  for (size_t i = 0; i < x.size(); i++) {
    const uint64_t t = (uint64_t)x[i] * s + c;
    r[i] = (uint32_t)t;
    c = t >> 32;
  }
  r[x.size()] = (uint32_t)c;
  while (r.size() > 1 && r.back() == 0) r.pop_back();
  return r;
}
Big big_div(const Big& x, uint32_t s, uint32_t* rem) {
  Big q(x.size(), 0);
  uint64_t r = 0;
  for (size_t i = x.size(); i-- > 0;) {
    const uint64_t t = (r << 32) | x[i];
    q[i] = (uint32_t)(t / s);
    r = t % s;
  }
  while (q.size() > 1 && q.back() == 0) q.pop_back();
  if (rem) *rem = (uint32_t)r;
  return q;
}
// bits lo .. lo + 39 as an integer
uint64_t big_bits(const Big& x, int lo) {
  uint64_t v = 0;
  for (int b = 0; b < kCrtLimbBits; b++) {
    const int p = lo + b, wd = p / 32;
    if (wd < (int)x.size() && ((x[wd] >> (p % 32)) & 1u)) v |= 1ull << b;
  }
  return v;
}
int inverse_mod(int a, int m) {  // a^-1 mod m for gcd(a, m) = 1 (extended Euclid)
  int t = 0, nt = 1, r = m, nr = ((a % m) + m) % m;
  while (nr) {
    const int q = r / nr, tt = t - q * nt, rr = r - q * nr;
    t = nt;
    nt = tt;
    r = nr;
    nr = rr;
  }
  return ((t % m) + m) % m;
}
}  // namespace

// Number of moduli for b-bit inputs and K-term products: the least N with
// log2 M >= 2 b + ceil(log2 K) + 3 (0 if more than kCrtMaxMod would be needed).
int crt_moduli(int K, int bits) {
  int lk = 0;
  while ((1L << lk) < (long)(K > 1 ? K : 1)) lk++;
  const double need = 2.0 * bits + lk + 3;
  double have = 0;
  for (int k = 0; k < kCrtMaxMod; k++) {
    have += log2((double)kCrtModuli[k]);
    if (have >= need) return k + 1;
  }
  return 0;
}

static void crt_const(int N, CrtConst& c) {
  memset(&c, 0, sizeof(c));
  c.N = N;
  Big M{1};
  for (int k = 0; k < N; k++) M = big_mul(M, (uint32_t)kCrtModuli[k]);
  for (int k = 0; k < N; k++) {
    const int m = kCrtModuli[k];
    c.mod[k] = m;
    c.inv[k] = 1.0 / m;
    uint32_t rem = 0;
    const Big Mk = big_div(M, (uint32_t)m, nullptr);
    big_div(Mk, (uint32_t)m, &rem);
    const Big w = big_mul(Mk, (uint32_t)inverse_mod((int)rem, m));
    for (int l = 0; l < kCrtLimbs; l++) c.w[k][l] = (double)big_bits(w, kCrtLimbBits * l);
  }
  c.Mf = 0;
  for (int l = 0; l < kCrtLimbs; l++) {
    c.M[l] = (double)big_bits(M, kCrtLimbBits * l);
    c.Mf += ldexp(c.M[l], kCrtLimbBits * l);
  }
}

// ------------------------------------------------------------------ splitting

constexpr int kCrtSplitNT = 256;

// Balanced residue of the integer-valued double x modulo m, in [-(m/2), m - 1 - m/2]
// (int division), and its negation in the same range.
__device__ inline int crt_residue(double x, int m, double inv) {
  const double q = rint(x * inv);
  int r = (int)fma(-q, (double)m, x);  // exact: the true value is a small integer
  const int lo = -(m >> 1), hi = m - 1 - (m >> 1);
  if (r > hi) r -= m;
  if (r < lo) r += m;
  return r;
}
__device__ inline int crt_neg(int r, int m) {
  const int hi = m - 1 - (m >> 1);
  int s = -r;
  if (s > hi) s -= m;  // m = 256: -(-128) is 128, stored as -128 (the same class)
  return s;
}

// Exponents t = E - b of the columns of X (K x ncols): one block per column.
__global__ __launch_bounds__(kCrtSplitNT) void crt_colexp_kernel(const zc* __restrict__ X, long ld, int K,
                                                                 int bits, int* __restrict__ exps) {
  __shared__ double red[kCrtSplitNT / 64];
  const zc* x = X + (long)blockIdx.x * ld;
  double m = 0;
  for (int k = threadIdx.x; k < K; k += kCrtSplitNT) m = fmax(m, fmax(fabs(x[k].re), fabs(x[k].im)));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < kCrtSplitNT / 64; w++) t = fmax(t, red[w]);
    exps[blockIdx.x] = t > 0 ? scale_exponent(t) - bits : 0;
  }
}

// Residues of the columns of X: one block per plane block (16 columns of the padded
// count x 64 K positions; padding columns and positions get zero residues), so that
// every store of a wave fills 256 contiguous bytes of the block. Thread t takes
// column 16 blockIdx.x + t / 16 at the 4 consecutive K positions 4 (t % 16) of the
// block (one dword per part and modulus).
__global__ __launch_bounds__(kCrtSplitNT) void crt_split_cols_kernel(const zc* __restrict__ X, long ld, int K,
                                                                     int ncols, int Kp, CrtConst c,
                                                                     const int* __restrict__ exps,
                                                                     int8_t* __restrict__ out) {
  const int col = blockIdx.x * 16 + (threadIdx.x >> 4);
  const int k0 = blockIdx.y * 64 + (threadIdx.x & 15) * 4;
  const long plane = oz_plane_bytes(ncols, Kp);
  const long stride = (long)kParts * plane;  // modulus k -> k + 1
  const bool live = col < ncols;
  const int t = live ? exps[col] : 0;
  const zc* x = X + (long)(live ? col : 0) * ld;
  double vr[4], vi[4];
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const bool ok = live && k0 + q < K;
    const zc v = x[ok ? k0 + q : 0];
    vr[q] = ok ? rint(ldexp(v.re, -t)) : 0.0;
    vi[q] = ok ? rint(ldexp(v.im, -t)) : 0.0;
  }
  const long o = oz_off(col, k0, Kp / 64);  // 4 consecutive K positions stay in one chunk
  for (int k = 0; k < c.N; k++) {
    const int mo = c.mod[k];
    const double inv = c.inv[k];
    unsigned pr = 0, pi = 0, pn = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int rr = crt_residue(vr[q], mo, inv), ri = crt_residue(vi[q], mo, inv);
      pr |= (unsigned)(uint8_t)rr << (8 * q);
      pi |= (unsigned)(uint8_t)ri << (8 * q);
      pn |= (unsigned)(uint8_t)crt_neg(ri, mo) << (8 * q);
    }
    int8_t* base = out + k * stride + o;
    *(unsigned*)base = pr;
    *(unsigned*)(base + plane) = pi;
    *(unsigned*)(base + 2 * plane) = pn;
  }
}

// Row exponents: the largest scale exponent over K-chunks of 256, combined with
// an integer atomic max (monotone in the magnitude; all-zero rows keep kNoRow).
constexpr int kCrtNoRow = -2147483647 - 1;
__global__ void crt_exp_init_kernel(int* __restrict__ e, int M) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < M) e[r] = kCrtNoRow;
}
__global__ __launch_bounds__(kCrtSplitNT) void crt_rowmax_kernel(const zc* __restrict__ X, long ld, int M, int K,
                                                                 int* __restrict__ e) {
  __shared__ double red[4][64];
  const int r = blockIdx.x * 64 + (threadIdx.x & 63), c = threadIdx.x >> 6;
  const int k0 = blockIdx.y * 256, k1 = min(K, k0 + 256);
  double m = 0;
  if (r < M)
    for (int k = k0 + c; k < k1; k += 4) {
      const zc v = X[r + (long)k * ld];
      m = fmax(m, fmax(fabs(v.re), fabs(v.im)));
    }
  red[c][threadIdx.x & 63] = m;
  __syncthreads();
  if (c == 0 && r < M) {
    const double t = fmax(fmax(red[0][threadIdx.x], red[1][threadIdx.x]), fmax(red[2][threadIdx.x], red[3][threadIdx.x]));
    if (t > 0) atomicMax(&e[r], scale_exponent(t));
  }
}
__global__ void crt_exp_fix_kernel(int* __restrict__ e, int M, int bits) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < M) e[r] = e[r] == kCrtNoRow ? 0 : e[r] - bits;
}

// Residues of the rows of X (M x K); one block per 32 x 32 tile, staged through LDS
// so that reads follow the columns and writes the rows (padding rows get zeros).
__global__ __launch_bounds__(kCrtSplitNT) void crt_split_rows_kernel(const zc* __restrict__ X, long ld, int M,
                                                                     int K, int Kp, CrtConst c,
                                                                     const int* __restrict__ exps,
                                                                     int8_t* __restrict__ out) {
  __shared__ zc tile[32][33];
  const int i0 = blockIdx.x * 32, k0 = blockIdx.y * 32;
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int idx = r * kCrtSplitNT + threadIdx.x;
    const int row = idx & 31, kk = idx >> 5;
    const int gi = i0 + row, gk = k0 + kk;
    const bool ok = gi < M && gk < K;
    const zc v = X[ok ? gi + (long)gk * ld : 0];
    tile[kk][row] = mk<double>(ok ? v.re : 0.0, ok ? v.im : 0.0);
  }
  __syncthreads();
  const int row = threadIdx.x >> 3, kg = (threadIdx.x & 7) * 4;
  const int gi = i0 + row;
  if (gi >= oz_rows_pad(M)) return;
  const long plane = oz_plane_bytes(M, Kp);
  const long stride = (long)kParts * plane;
  const long o = oz_off(gi, k0 + kg, Kp / 64);
  const int t = gi < M ? exps[gi] : 0;
  double vr[4], vi[4];
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const zc v = tile[kg + q][row];  // zero for padding rows and K positions
    vr[q] = rint(ldexp(v.re, -t));
    vi[q] = rint(ldexp(v.im, -t));
  }
  for (int k = 0; k < c.N; k++) {
    const int mo = c.mod[k];
    const double inv = c.inv[k];
    unsigned pr = 0, pi = 0, pn = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int rr = crt_residue(vr[q], mo, inv), ri = crt_residue(vi[q], mo, inv);
      pr |= (unsigned)(uint8_t)rr << (8 * q);
      pi |= (unsigned)(uint8_t)ri << (8 * q);
      pn |= (unsigned)(uint8_t)crt_neg(ri, mo) << (8 * q);
    }
    int8_t* base = out + k * stride + o;
    *(unsigned*)base = pr;
    *(unsigned*)(base + plane) = pi;
    *(unsigned*)(base + 2 * plane) = pn;
  }
}

// -------------------------------------------------------------------- product
//
// A 256-thread block computes a 128 x 128 complex tile; each of its four waves
// owns 64 x 64 as 2 x 2 blocks of 32 x 32 with two int32 accumulators (re, im) per
// output. The residues of one modulus go through a two-stage LDS ring (one K-tile
// of 64 per stage: 3 parts of op(A) and 2 of B, 128 rows of 64 bytes each, copied
// from the planes with global_load_lds_dwordx4), the next step's loads issued while
// the current one is multiplied, across the moduli as one sequence of N * K/64
// steps. After a modulus the sums are reduced modulo m and the residues stored in
// the block's scratch (8 bytes: four re, four im per lane and group of four
// outputs); after the last one each lane reads its outputs' residues back,
// reconstructs, scales and applies the epilogue.
constexpr int CBM = 128, CBN = 128, CNT = 256;
constexpr int kCRow = 64, kCPart = CBM * kCRow;                     // 8 KiB
constexpr int kCStage = 5 * kCPart;                                 // 40 KiB
constexpr int kCLoadsPerWave = 5 * (CBM / 16) / (CNT / 64);         // 10
constexpr int kCScratchPerMod = (CNT / 64) * 4 * 4 * 64 * 8;       // 32 KiB per block and modulus

struct CrtArgs {
  const int8_t* A;  // op(A) residues: [N][3][rows][Kp]
  const int* ta;
  const int8_t* B;  // B residues: [N][3][cols][Kp]
  const int* tb;
  int conjA, Kp;
  GemmArgs g;
  uint8_t* scratch;
  CrtConst c;
  // Tiles past the last full round of block slots: the first nfull blocks take one
  // tile each; the tiles after them are split into ksplit blocks of consecutive
  // moduli (0: no split), whose residues meet in the tile's scratch; the last of a
  // tile's blocks to finish (counted in counters[], zero between launches)
  // reconstructs it.
  int nfull, ksplit;
  unsigned* counters;
};

// sum modulo m of a (exact) int32 sum, in [0, m)
__device__ inline int crt_reduce(int acc, int m, double inv) {
  const int q = (int)floor((double)acc * inv);
  int r = acc - q * m;
  if (r < 0) r += m;
  if (r >= m) r -= m;
  return r;
}

// X from its limb sums S_l = sum_k r_k w_kl: q, carries, double-double.
__device__ inline double crt_finish(const CrtConst& c, const double* S) {
  // q = rint(S / M): S / M = q + X / M with |X / M| < 1/8
  const double approx = ldexp(S[3], 120) + ldexp(S[2], 80) + ldexp(S[1], 40) + S[0];
  const double q = rint(approx / c.Mf);
  double X[kCrtLimbs];
#pragma unroll
  for (int l = 0; l < kCrtLimbs; l++) X[l] = fma(-q, c.M[l], S[l]);  // exact: both below 2^53
  // carries: X_0, X_1, X_2 into [0, 2^40)
#pragma unroll
  for (int l = 0; l < kCrtLimbs - 1; l++) {
    const double cy = floor(ldexp(X[l], -kCrtLimbBits));
    X[l] = fma(-cy, 0x1p40, X[l]);
    X[l + 1] += cy;
  }
  // X_3 2^120 + X_2 2^80 is exact (|X_3| < 8); the other two limbs in double-double
  double h, e;
  two_sum(ldexp(X[3], 120) + ldexp(X[2], 80), ldexp(X[1], 40), h, e);
  dd_add(h, e, X[0]);
  return h + e;
}

template <int EPI>
__global__ __launch_bounds__(CNT) __attribute__((amdgpu_waves_per_eu(2))) void crt_gemm_kernel(CrtArgs a) {
  extern __shared__ __align__(16) int8_t lds[];  // 2 stages
  const GemmArgs& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;

  const int bid = blockIdx.x, N = a.c.N;
  int logical = bid, k0 = 0, k1 = N, rem = -1;
  if (bid < a.nfull) {
    const int per = a.nfull / kXCDs;
    if (bid < per * kXCDs) logical = (bid % kXCDs) * per + bid / kXCDs;
  } else {
    // a share of the moduli of one of the tiles after the full rounds
    const int it = bid - a.nfull, part = it % a.ksplit;
    rem = it / a.ksplit;
    logical = a.nfull + rem;
    k0 = part * N / a.ksplit;
    k1 = (part + 1) * N / a.ksplit;
  }
  int tm, tn;
  if (EPI == EPI_YDEF && g.herm) {
    herm_tile(logical, g.tiles_n, tm, tn);
  } else {
    // groups of 8 tile rows: the 64 blocks an XCD runs at once cover 8 x 8 tiles, the
    // fewest distinct residue rows and columns per K-step in its L2 (groups of 4: 1.4%
    // slower at n = 4096, of 2 or 16: 2%)
    constexpr int kGroup = 8;
    const int group = logical / (kGroup * g.tiles_n);
    const int first_m = group * kGroup;
    const int gsize = min(g.tiles_m - first_m, kGroup);
    const int within = logical - group * kGroup * g.tiles_n;
    tm = first_m + within % gsize;
    tn = within / gsize;
  }
  const int m0 = tm * CBM, n0 = tn * CBN;

  const int KT = a.Kp / OBK;
  const long pA = oz_plane_bytes(g.m, a.Kp), pB = oz_plane_bytes(g.n, a.Kp);
  const long sA = kParts * pA, sB = kParts * pB;
  const int pa2 = a.conjA ? 1 : 2, pa3 = a.conjA ? 2 : 1;

  // load instruction j of wave w: q = 10 w + j; q < 24: A part q / 8, row block q % 8;
  // else B part (q - 24) / 8. Row blocks past the matrix read its last one (their
  // outputs are not stored).
  const int uwave = __builtin_amdgcn_readfirstlane(wave);
  const int RBA = oz_rows_pad(g.m) / 16, RBB = oz_rows_pad(g.n) / 16;
  int goff[kCLoadsPerWave];
#pragma unroll
  for (int j = 0; j < kCLoadsPerWave; j++) {
    const int q = uwave * kCLoadsPerWave + j;
    const bool isA = q < 24;
    const int qq = isA ? q : q - 24;
    const int part = qq >> 3;
    const int rb = min((isA ? m0 : n0) / 16 + (qq & 7), (isA ? RBA : RBB) - 1);
    goff[j] = (int)(part * (isA ? pA : pB)) + rb * KT * 1024 + lane * 16;
  }
  const int total = k1 * KT;
  // sources and stage of the loads of step st
  struct Src {
    const int8_t* A;
    const int8_t* B;
    int8_t* stage;
  };
  auto src = [&](int st) {
    const int k = st / KT, kt = st - k * KT;
    return Src{a.A + (long)k * sA + kt * 1024, a.B + (long)k * sB + kt * 1024, lds + (st & 1) * kCStage};
  };
  // load j of a step
  auto issue_one = [&](const Src& sc, int j) {
    const int8_t* baseA = sc.A;
    const int8_t* baseB = sc.B;
    int8_t* stage = sc.stage;
    const int q = uwave * kCLoadsPerWave + j;
    const bool isA = q < 24;
    const int qq = isA ? q : q - 24;
    const int loff = (isA ? (qq >> 3) : 3 + (qq >> 3)) * kCPart + 16 * (qq & 7) * kCRow;
    __builtin_amdgcn_global_load_lds((gbl_ptr_t*)((isA ? baseA : baseB) + goff[j]), (lds_ptr_t*)(stage + loff),
                                     16, 0, 0);
  };
  struct Frags {
    v4i b0[2], b1[2], a0[2], a2[2], a3[2];
  };
  auto load_frags = [&](Frags& f, const int8_t* base, int kh) {
    const int c = 2 * kh + (lane >> 5);
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int r = wn + y * 32 + (lane & 31);
      const int o = r * kCRow + ((c ^ chunk_swz(r)) << 4);
      f.b0[y] = *(const v4i*)(base + 3 * kCPart + o);
      f.b1[y] = *(const v4i*)(base + 4 * kCPart + o);
    }
#pragma unroll
    for (int x = 0; x < 2; x++) {
      const int r = wm + x * 32 + (lane & 31);
      const int o = r * kCRow + ((c ^ chunk_swz(r)) << 4);
      f.a0[x] = *(const v4i*)(base + o);
      f.a2[x] = *(const v4i*)(base + pa2 * kCPart + o);
      f.a3[x] = *(const v4i*)(base + pa3 * kCPart + o);
    }
  };
  v16i acc_re[2][2], acc_im[2][2];
  // the 32 MFMAs of a step (16 per K half), with the next step's loads (when nx <
  // total) issued one after every third MFMA: spread over the step they took 6% less
  // time at n = 4096 than issued together after the barrier
  auto mfmas = [&](const Frags& f0, const Frags& f1, int nx) {
    int jl = 0;
    const bool more = nx < total;
    const Src sc = src(more ? nx : 0);
    auto one = [&]() {
      if (more && jl < kCLoadsPerWave) issue_one(sc, jl);
      jl++;
    };
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const Frags& f = h ? f1 : f0;
#pragma unroll
      for (int x = 0; x < 2; x++)
#pragma unroll
        for (int y = 0; y < 2; y++) {
          const int i0 = ((h * 2 + x) * 2 + y) * 4;
          acc_re[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a0[x], f.b0[y], acc_re[x][y], 0, 0, 0);
          if (i0 % 3 == 1) one();
          acc_im[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a0[x], f.b1[y], acc_im[x][y], 0, 0, 0);
          if ((i0 + 1) % 3 == 1) one();
          acc_re[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a2[x], f.b1[y], acc_re[x][y], 0, 0, 0);
          if ((i0 + 2) % 3 == 1) one();
          acc_im[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a3[x], f.b0[y], acc_im[x][y], 0, 0, 0);
          if ((i0 + 3) % 3 == 1) one();
        }
    }
  };
  auto barrier = [&]() {
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  // this lane's residue slots: tile, wave, modulus, 32 x 32 block, group of four
  // outputs, lane (8 bytes)
  uint8_t* sres = a.scratch + (long)logical * N * kCScratchPerMod + (long)wave * N * (kCScratchPerMod / 4) + lane * 8;

  int st = k0 * KT;
  {
    const Src s0 = src(st);
#pragma unroll
    for (int j = 0; j < kCLoadsPerWave; j++) issue_one(s0, j);
  }
  for (int k = k0; k < k1; k++) {
#pragma unroll
    for (int x = 0; x < 2; x++)
#pragma unroll
      for (int y = 0; y < 2; y++) acc_re[x][y] = acc_im[x][y] = v16i{};
    for (int kt = 0; kt < KT; kt++, st++) {
      // wait for this step's loads, barrier (every wave's loads have landed; the
      // other stage is no longer read), then the MFMAs with the next step's loads
      __builtin_amdgcn_s_waitcnt(kWaitVm0);
      barrier();
      const int8_t* base = lds + (st & 1) * kCStage;
      Frags f0, f1;
      load_frags(f0, base, 0);
      load_frags(f1, base, 1);
      mfmas(f0, f1, st + 1);
    }
    // residues modulo m_k of this modulus' sums
    const int mo = a.c.mod[k];
    const double inv = a.c.inv[k];
#pragma unroll
    for (int x = 0; x < 2; x++)
#pragma unroll
      for (int y = 0; y < 2; y++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
          unsigned pr = 0, pi = 0;
#pragma unroll
          for (int c = 0; c < 4; c++) {
            pr |= (unsigned)crt_reduce(acc_re[x][y][4 * q + c], mo, inv) << (8 * c);
            pi |= (unsigned)crt_reduce(acc_im[x][y][4 * q + c], mo, inv) << (8 * c);
          }
          *(uint2*)(sres + ((long)k * 16 + (x * 2 + y) * 4 + q) * 512) = make_uint2(pr, pi);
        }
  }
  if (rem >= 0) {
    // a share of a split tile: the residues out (release), count the shares; the
    // last one reconstructs (acquire). The stages are free once every wave is past
    // this barrier; their first word carries the decision.
    __threadfence();
    __syncthreads();
    int* flag = (int*)lds;
    if (tid == 0) flag[0] = atomicAdd(&a.counters[rem], 1u) == (unsigned)(a.ksplit - 1);
    __syncthreads();
    if (!flag[0]) return;
    __threadfence();
    if (tid == 0) a.counters[rem] = 0u;  // ready for the next launch
  }
  // reconstruction and epilogue (each lane reads back what the lanes in its place
  // stored, in this block or in the other shares of its tile)
  double part = 0;
#pragma unroll 1
  for (int xy = 0; xy < 4; xy++) {
    const int x = xy >> 1, y = xy & 1;
#pragma unroll 1
    for (int q = 0; q < 4; q++) {
      unsigned rre[kCrtMaxMod], rim[kCrtMaxMod];
#pragma unroll
      for (int k = 0; k < kCrtMaxMod; k++) {
        uint2 v = make_uint2(0, 0);
        if (k < N) v = *(const uint2*)(sres + ((long)k * 16 + xy * 4 + q) * 512);
        rre[k] = v.x;
        rim[k] = v.y;
      }
      // limb sums of the group's 8 values (4 outputs, re and im) in one pass over the
      // moduli: each w_kl is read once for all 8, and the 32 sums are independent
      // (one value at a time re-read the weights per value and waited on 4 chains:
      // 5% slower at n = 4096)
      double S[8][kCrtLimbs];
#pragma unroll
      for (int t = 0; t < 8; t++)
#pragma unroll
        for (int l = 0; l < kCrtLimbs; l++) S[t][l] = 0.0;
#pragma unroll
      for (int k = 0; k < kCrtMaxMod; k++) {
        if (k < N) {
#pragma unroll
          for (int c = 0; c < 4; c++) {
            const double r0 = (double)((rre[k] >> (8 * c)) & 255u), r1 = (double)((rim[k] >> (8 * c)) & 255u);
#pragma unroll
            for (int l = 0; l < kCrtLimbs; l++) {
              S[c][l] = fma(r0, a.c.w[k][l], S[c][l]);
              S[4 + c][l] = fma(r1, a.c.w[k][l], S[4 + c][l]);
            }
          }
        }
      }
#pragma unroll
      for (int c = 0; c < 4; c++) {
        const int v = 4 * q + c;
        const int i = m0 + wm + x * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int j = n0 + wn + y * 32 + (lane & 31);
        if (i < g.m && j < g.n) {
          const int e = a.ta[i] + a.tb[j];
          const double re = crt_finish(a.c, S[c]), im = crt_finish(a.c, S[4 + c]);
          epi_element<EPI, double>(g, i, j, mk<double>(ldexp(re, e), ldexp(im, e)), part);
        }
      }
    }
  }
  if constexpr (EPI == EPI_SPLIT || EPI == EPI_YDEF) {
    __syncthreads();  // every wave is past its last read of the ring
    epi_reduce<CNT>(g, part, (double*)lds, logical);  // one slot per tile
  }
}

// ------------------------------------------------------------------ host side

size_t crt_residue_bytes(int rows, int K, int N) { return (size_t)N * kParts * oz_plane_bytes(rows, oz_kp(K)); }

int crt_gemm_tiles(int m, int n, bool herm) {
  const int t = ceil_div(n, CBN);
  return herm ? t * (t + 1) / 2 : ceil_div(m, CBM) * t;
}

// block slots of one round (two blocks per CU); remainders up to a quarter of a round
// are split after full rounds
constexpr int kCrtSlots = 2 * kCUs, kCrtMaxRem = kCrtSlots / 4;

// the residues of every tile between moduli
static size_t crt_residue_scratch(int m, int n, int N) {
  return (size_t)crt_gemm_tiles(m, n, false) * N * kCScratchPerMod;
}
// the residues, then one share counter per split tile (fewer than kCrtSlots)
size_t crt_scratch_bytes(int m, int n, int N) { return crt_residue_scratch(m, n, N) + kCrtSlots * sizeof(unsigned); }

bool crt_plan_ok(int K, int bits) { return K < 65536 && bits >= 1 && crt_moduli(K, bits) > 0; }

hipError_t crt_split_cols(const zc* X, long ld, int K, int ncols, int bits, int8_t* out, int* exps,
                          hipStream_t st) {
  const int N = crt_moduli(K, bits);
  if (!N) return hipErrorInvalidValue;
  if (ncols == 0) return hipSuccess;
  CrtConst c;
  crt_const(N, c);
  hipLaunchKernelGGL(crt_colexp_kernel, dim3(ncols), dim3(kCrtSplitNT), 0, st, X, ld, K, bits, exps);
  const int Kp = oz_kp(K);
  hipLaunchKernelGGL(crt_split_cols_kernel, dim3(oz_rows_pad(ncols) / 16, Kp / 64), dim3(kCrtSplitNT), 0, st, X,
                     ld, K, ncols, Kp, c, (const int*)exps, out);
  return hipGetLastError();
}

hipError_t crt_split_rows(const zc* X, long ld, int M, int K, int bits, int8_t* out, int* exps,
                          hipStream_t st) {
  const int N = crt_moduli(K, bits);
  if (!N) return hipErrorInvalidValue;
  if (M == 0) return hipSuccess;
  CrtConst c;
  crt_const(N, c);
  hipLaunchKernelGGL(crt_exp_init_kernel, dim3(ceil_div(M, 256)), dim3(256), 0, st, exps, M);
  hipLaunchKernelGGL(crt_rowmax_kernel, dim3(ceil_div(M, 64), max(1, ceil_div(K, 256))), dim3(kCrtSplitNT), 0, st,
                     X, ld, M, K, exps);
  hipLaunchKernelGGL(crt_exp_fix_kernel, dim3(ceil_div(M, 256)), dim3(256), 0, st, exps, M, bits);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int Kp = oz_kp(K);
  hipLaunchKernelGGL(crt_split_rows_kernel, dim3(ceil_div(M, 32), Kp / 32), dim3(kCrtSplitNT), 0, st, X, ld, M, K,
                     Kp, c, exps, out);
  return hipGetLastError();
}

template <int EPI>
static hipError_t launch_crt(int nt, const CrtArgs& a, hipStream_t st) {
  const size_t lds = 2 * (size_t)kCStage;
  hipError_t e = hipFuncSetAttribute((const void*)crt_gemm_kernel<EPI>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  crt_gemm_kernel<EPI><<<dim3(nt), dim3(CNT), lds, st>>>(a);
  return hipGetLastError();
}

__global__ void crt_zero_kernel(unsigned* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Blocks per launch and the split of the tiles after the last full round of
// kCrtSlots block slots (two blocks per CU) into shares of the moduli that fill a
// round: when those tiles fill at most a quarter of it, or when there is no full
// round at all (n = 2048: 256 tiles in 2 shares; n = 1024: 64 tiles in 8), as long
// as a tile gets at least two shares.
static void crt_plan_split(int tiles, int N, int* nfull, int* ksplit) {
  const int full = tiles / kCrtSlots * kCrtSlots, r = tiles - full;
  const int k = r > 0 ? std::min(N, kCrtSlots / r) : 0;
  if (k >= 2 && (full == 0 || r <= kCrtMaxRem)) {
    *nfull = full;
    *ksplit = k;
  } else {
    *nfull = tiles;
    *ksplit = 0;
  }
}

hipError_t crt_gemm(int epi, const int8_t* A, const int* ta, const int8_t* B, const int* tb, int conjA, int bits,
                    GemmArgs g, void* scratch, hipStream_t st) {
  if (g.m == 0 || g.n == 0) return hipSuccess;
  if (g.herm && (epi != EPI_YDEF || g.herm != 1 || g.m != g.n)) return hipErrorInvalidValue;
  const int N = crt_moduli(g.k, bits);
  if (!N || g.k >= 65536 || !scratch) return hipErrorInvalidValue;
  // within one modulus the kernel addresses an operand's residues with 32-bit offsets
  if ((long)kParts * oz_plane_bytes(g.m > g.n ? g.m : g.n, oz_kp(g.k)) >= 2147483647L) return hipErrorInvalidValue;
  g.tiles_m = ceil_div(g.m, CBM);
  g.tiles_n = ceil_div(g.n, CBN);
  CrtArgs a;
  a.A = A;
  a.ta = ta;
  a.B = B;
  a.tb = tb;
  a.conjA = conjA;
  a.Kp = oz_kp(g.k);
  a.g = g;
  a.scratch = (uint8_t*)scratch;
  crt_const(N, a.c);
  const int tiles = crt_gemm_tiles(g.m, g.n, g.herm != 0);
  crt_plan_split(tiles, N, &a.nfull, &a.ksplit);
  a.counters = (unsigned*)((uint8_t*)scratch + crt_residue_scratch(g.m, g.n, N));
  int nt = tiles;
  if (a.ksplit) {
    const int r = tiles - a.nfull;  // < kCrtSlots counters
    nt = a.nfull + r * a.ksplit;
    hipLaunchKernelGGL(crt_zero_kernel, dim3(ceil_div(r, 256)), dim3(256), 0, st, a.counters, r);
  }
  switch (epi) {
    case EPI_STORE: return launch_crt<EPI_STORE>(nt, a, st);
    case EPI_ADD: return launch_crt<EPI_ADD>(nt, a, st);
    case EPI_SPLIT: return launch_crt<EPI_SPLIT>(nt, a, st);
    case EPI_YDEF: return launch_crt<EPI_YDEF>(nt, a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sr
