// Launch interface of the real Schur variant's kernels (real.hip).
#pragma once

#include "kernels.hpp"

namespace sr {

// Real products (the real Schur variant) on FP64 / FP32 MFMA with fused epilogues:
// STORE (herm 1 / -1: symmetric / skew-symmetric, upper tiles mirrored), ADD (C = Cin
// + acc, CT = C^T when set), SPLIT (block-aware: T gets all but the block strictly
// lower part, FP64 and FP32 copies; E_lp the block strictly lower part; partials of
// ||E||^2), YDEF (acc - I, symmetric with herm). blk: the 2 x 2 block markers (device).
struct RGemmArgs {
  int m, n, k;
  const void* A;
  long lda;
  const void* B;
  long ldb;
  void* C;
  long ldc;
  const void* Cin;
  long ldcin;
  void* CT;
  long ldct;
  float* Tlp;
  float* Elp;
  long ldlp;
  double* partials;
  const int* blk;
  int tiles_m, tiles_n;
  int herm;
};
int rgemm_tiles(int m, int n, bool herm);
hipError_t dgemm(int opa, int epi, int comp, const RGemmArgs& g, hipStream_t st);  // FP64; opa 1: A^T
hipError_t sgemm(const RGemmArgs& g, hipStream_t st);                              // FP32, C = A B
hipError_t rfro2_partials(const double* x, long count, double* partials, int nparts, hipStream_t st);
int rform_w_parts(int n);
hipError_t rform_w(const float* L, float* W, int n, double* partials, hipStream_t st);
hipError_t rform_delta(const float* L, const double* Y, const float* W2, const float* W3, const float* YW,
                       double* D, int n, hipStream_t st);
hipError_t rw2_minus_y(const float* W2, const double* Y, float* X, long count, hipStream_t st);
// The FP32 block solve of the real quasi-triangular equation through the complex
// sweep (ws: trisolve_real_ws_bytes(n)); blk on the device. T64 (may be NULL): the
// FP64 T the FP32 T was rounded from, used instead of it for the 2 x 2 transforms.
size_t trisolve_real_ws_bytes(int n);
hipError_t trisolve_real(const float* T, const double* T64, const float* E, float* L, const int* blk, int n,
                         void* ws, unsigned* status, hipStream_t st);

}  // namespace sr
