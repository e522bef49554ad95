// Internal launch interface between the host driver and the device kernels.
#pragma once

#include "common.hpp"

namespace sr {

// Epilogues of the complex GEMM.
enum GemmEpi : int {
  EPI_STORE = 0,  // C = acc
  EPI_ADD = 1,    // C = Cin + acc (and CH = C^H when CH is set)
  EPI_SPLIT = 2,  // That: C = triu(acc) (zeros below), Tlp = fp32 triu, Elp = fp32 stril,
                  //       partials[block] = sum |stril(acc)|^2
  EPI_YDEF = 3    // Y: C = acc - I, partials[block] = sum |acc - I|^2
};

struct GemmArgs {
  int m, n, k;
  const void* A;
  long lda;
  const void* B;
  long ldb;
  void* C;
  long ldc;
  const void* Cin;
  long ldcin;
  void* CH;  // EPI_ADD: optional conjugate transpose of C
  long ldch;
  cc* Tlp;
  cc* Elp;
  long ldlp;
  double* partials;
  int tiles_m, tiles_n;
  // double-double outputs (Ozaki product with DD accumulation): low parts of C and
  // Cin (same leading dimensions), and the FP64 lp split of That
  void* Clo;
  const void* Cinlo;
  zc* Tlp64;
  zc* Elp64;
  // triple-double outputs (windowed Ozaki product): middle terms of C and Cin (the
  // low terms in Clo / Cinlo); C, Cmid, Clo form a renormalized expansion
  void* Cmid;
  const void* Cinmid;
  // EPI_STORE of the all-pairs INT8 product: C is complex64 (each value rounded
  // once from FP64)
  int c64;
  // EPI_YDEF (1) and EPI_STORE (1 or -1): the product is Hermitian (1) or
  // skew-Hermitian (-1), e.g. Q^H Q, W^2 and W^3 for a skew-Hermitian W. Only the
  // elements with i <= j are stored from the product, each with its conjugate
  // (negated for -1) at (j, i), so the result has the structure exactly; the squared
  // norm of YDEF counts both. The square FP64/FP32 kernels and the large-tile INT8
  // kernel (YDEF) then launch only the tiles on and above the diagonal.
  int herm;
};

// Number of output tiles (= blocks, = partial sums written) of a GEMM launch, and
// of a Hermitian (herm) n x n product.
int gemm_tiles(int m, int n);
int gemm_tiles_herm(int n);

// One output tile of a grouped (batched) product: matrix index, tile origin and
// the partial-sum slot its SPLIT / YDEF epilogue writes.
struct GTile {
  int mat, m0, n0, slot;
};
// Grouped products over a table of tiles (bm = 64 or 32: the tile edge); matrices
// with active[mat] == 0 are skipped (active may be NULL). grid = persistent blocks.
hipError_t zgemm_grouped(int opa, int epi, int comp, int bm, const GemmArgs* args, const GTile* tiles,
                         int ntiles, const int* active, int grid, hipStream_t st);
hipError_t cgemm_grouped(int bm, const GemmArgs* args, const GTile* tiles, int ntiles, const int* active,
                         int grid, hipStream_t st);

// complex128 product on FP64 MFMA; opa: 0 = A, 1 = A^H; comp: compensated accumulation.
hipError_t zgemm(int opa, int epi, int comp, const GemmArgs& g, hipStream_t st);
// complex64 product on FP32 MFMA (C = A B).
hipError_t cgemm(const GemmArgs& g, hipStream_t st);

// Squared Frobenius norm partials of a complex128 array: writes `nparts` values.
hipError_t fro2_partials(const zc* x, long count, double* partials, int nparts, hipStream_t st);
// out[0] = sum of partials[0..np) in a fixed order (one block).
hipError_t reduce_partials(const double* partials, int np, double* out, hipStream_t st);
// W = L - L^H (complex64, strictly lower L), partials of ||W||_F^2; returns #partials.
int form_w_parts(int n);
hipError_t form_w(const cc* L, cc* W, int n, double* partials, hipStream_t st);
// D = W - Y/2 + (W2 + W3 - YW)/2 with W = L - L^H (L may be NULL: W = 0; Y and the
// products may be NULL: absent).
hipError_t form_delta(const cc* L, const zc* Y, const cc* W2, const cc* W3, const cc* YW, zc* D,
                      int n, hipStream_t st);
hipError_t to_c64(const zc* x, cc* y, long count, hipStream_t st);
// X = W2 - Y, the left factor of (W^2 - Y) W = W^3 - YW: FP32 (Y narrowed from FP64,
// one rounding) or FP64.
hipError_t w2_minus_y(const cc* W2, const zc* Y, cc* X, long count, hipStream_t st);
hipError_t w2_minus_y(const zc* W2, const zc* Y, zc* X, long count, hipStream_t st);
// Double-double tier: W = L - L^H in FP64 (partials of ||W||^2), and
// D = W - Y/2 + (W2 + W3 - YW)/2 with Y = Yhi + Ylo and D = Dhi + Dlo in
// double-double (L and the lp products may be NULL: absent).
hipError_t form_w64(const zc* L, zc* W, int n, double* partials, hipStream_t st);
hipError_t form_delta_dd(const zc* L, const zc* Yhi, const zc* Ylo, const zc* W2, const zc* W3,
                         const zc* YW, zc* Dhi, zc* Dlo, int n, hipStream_t st);
// Triple-double tier: D = W - Y/2 + (W2 + W3 - YW)/2 with Y and D as three-term
// expansions (Y0 + Y1 + Y2, D0 + D1 + D2); L and the lp products FP64 (may be NULL).
hipError_t form_delta_td(const zc* L, const zc* Y0, const zc* Y1, const zc* Y2, const zc* W2, const zc* W3,
                         const zc* YW, zc* D0, zc* D1, zc* D2, int n, hipStream_t st);
hipError_t fill_zero(void* p, size_t bytes, hipStream_t st);

// Ozaki split products on INT8 MFMA (complex128 operands, FP64 output).
size_t oz_slice_bytes(int rows, int K, int S);
hipError_t oz_split_cols(const zc* X, const zc* Xlo, long ld, int K, int ncols, int S, int8_t* out,
                         int* exps, hipStream_t st);
hipError_t oz_split_rows(const zc* X, const zc* Xlo, long ld, int M, int K, int S, int8_t* out,
                         int* exps, hipStream_t st);
// Triple-double operands (X + Xmid + Xlo, renormalized expansions; Xmid requires Xlo).
hipError_t oz_split_cols3(const zc* X, const zc* Xmid, const zc* Xlo, long ld, int K, int ncols, int S,
                          int8_t* out, int* exps, hipStream_t st);
hipError_t oz_split_rows3(const zc* X, const zc* Xmid, const zc* Xlo, long ld, int M, int K, int S,
                          int8_t* out, int* exps, hipStream_t st);
// Complex64 operands (one term each): the lp products taken on INT8 digits.
hipError_t oz_split_cols_c64(const cc* X, long ld, int K, int ncols, int S, int8_t* out, int* exps, hipStream_t st);
hipError_t oz_split_rows_c64(const cc* X, long ld, int M, int K, int S, int8_t* out, int* exps, hipStream_t st);
// Whether an m x n x k product with S digits per operand (pairs s + t <= S + 1) runs
// on the all-pairs kernel, the one that also takes Hermitian STORE and complex64
// outputs.
bool oz_allpairs_ok(int m, int n, int k, int S);
// Whether the windowed kernel, the only one with triple-double outputs, takes an
// m x n x k product with S digits per operand (its 32-bit plane offsets bound the
// sizes: (S + 4) 3 max(m, n) k < 2^31).
bool oz_td_ok(int m, int n, int k, int S);
// Output tiles (= partial sums written) of a product; the sizes, the digit counts
// and dd (double-double accumulation) select the kernel; herm: a Hermitian
// product (GemmArgs::herm).
int oz_gemm_tiles(int m, int n, int k, bool dd, bool herm, int SA, int SB, int dmax, bool td = false);
// Bytes of scratch the product of an m x n output needs (0 for small FP64 outputs;
// double-double and triple-double outputs use the dd size).
size_t oz_gemm_scratch_bytes(int m, int n, bool dd = false);
// Whether the int32 sums of a product stay exact for these sizes.
bool oz_gemm_exact(int m, int n, int k, int SA, int SB, bool dd = false);
hipError_t oz_gemm(int epi, const int8_t* A, const int* ea, int SA, const int8_t* B, const int* eb,
                   int SB, int conjA, int dmax, GemmArgs g, void* scratch, hipStream_t st,
                   bool dd = false);

// Ozaki scheme II (CRT) products on INT8 MFMA (complex128 operands, FP64 output):
// rows of op(A) and columns of B scaled to integers of at most `bits` bits, their
// residues modulo crt_moduli(K, bits) pairwise coprime moduli (the digit-plane
// layout, one "slice" per modulus), and the product reconstructed from the
// residues of its sums. K < 65536.
int crt_moduli(int K, int bits);  // 0: not possible (more than 20 moduli)
bool crt_plan_ok(int K, int bits);
size_t crt_residue_bytes(int rows, int K, int N);
size_t crt_scratch_bytes(int m, int n, int N);
int crt_gemm_tiles(int m, int n, bool herm);
hipError_t crt_split_cols(const zc* X, long ld, int K, int ncols, int bits, int8_t* out, int* exps,
                          hipStream_t st);
hipError_t crt_split_rows(const zc* X, long ld, int M, int K, int bits, int8_t* out, int* exps, hipStream_t st);
hipError_t crt_gemm(int epi, const int8_t* A, const int* ta, const int8_t* B, const int* tb, int conjA, int bits,
                    GemmArgs g, void* scratch, hipStream_t st);

// A tile task of the recursive block solve: tile (I, J) solved inside the node of
// tile range [lo, hi) (16-wide tiles).
struct TileTask {
  int I, J, lo, hi;
};

// Triangular matrix equation in FP32 (complex64) and in FP64 (complex128); the
// workspace size serves both.
size_t trisolve_ws_bytes(int n);
hipError_t trisolve(const cc* T, const cc* E, cc* L, int n, float trunc, void* ws,
                    unsigned* status, hipStream_t st);
hipError_t trisolve64(const zc* T, const zc* E, zc* L, int n, void* ws, unsigned* status,
                      hipStream_t st);
// The same equation in FP32 by the recursive block algorithm (Algorithm 3): nodes
// split at half their tile count down to leaves of at most leaf_tiles tiles, the
// Sylvester block of every node and the leaves solved as tile tasks (one launch per
// step for all nodes of a depth), the two updates of E per node as grouped FP32
// MFMA products. E is not modified (the updates go to a copy in ws).
size_t trisolve_rec_ws_bytes(int n, int leaf_tiles);
hipError_t trisolve_rec(const cc* T, const cc* E, cc* L, int n, int leaf_tiles, float trunc, void* ws,
                        unsigned* status, hipStream_t st);
hipError_t cgemm_grouped_add(int bm, const GemmArgs* args, const GTile* tiles, int ntiles, int grid,
                             hipStream_t st);
// Reordering of the start: T (complex128 n x n, Q^H A Q on entry) is made upper
// triangular and reordered by adjacent swaps in the order of Re(lambda e^{-i theta});
// Q is updated in place; perm_out (device, may be NULL) receives the original
// position of each new diagonal entry. scratch: reorder_scratch_bytes(n) bytes.
size_t reorder_scratch_bytes(int n);
hipError_t reorder_swaps(zc* T, zc* Q, int n, double theta, void* scratch, int* perm_out, hipStream_t st);
// Batched FP32 solves over a device table of `count` matrix records, filled on the
// host with trimatrix_fill (each record trimatrix_bytes() bytes).
hipError_t trisolve_batched(const void* mats, int count, float trunc, hipStream_t st);
size_t trimatrix_bytes();
void trimatrix_fill(void* dst, const cc* T, const cc* E, cc* L, int n, const int* active,
                    unsigned* flag);
// The same solves by tile diagonal: step s takes tile diagonal nb - 1 - s of every
// matrix with nb > s tile rows (16-wide tiles), one block per tile, so that a large
// matrix's tiles run in parallel. trisolve_steps_plan lists the (matrix, tile) pairs
// of all steps (n[b] < 2: none) and the start of each step's run, ending with the
// total; trisolve_batched_steps launches the steps from a device copy of the list.
struct TriStepTile {
  int mat, I, J;
};
void trisolve_steps_plan(const int* n, int count, TriStepTile* tiles, int* step_off, int* steps);
size_t trisolve_steps_tiles(const int* n, int count);  // list length
int trisolve_steps_max(const int* n, int count);       // number of steps
hipError_t trisolve_batched_steps(const void* mats, const TriStepTile* tiles, const int* step_off, int steps,
                                  float trunc, hipStream_t st);

}  // namespace sr
