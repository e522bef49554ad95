// Digit-plane layout shared by the INT8 split products (Ozaki scheme I digit
// slices and Ozaki scheme II residues): helpers for the planes and the
// global-to-LDS loads of the product kernels.
#pragma once

#include <math.h>

#include "common.hpp"

namespace sr {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int OBK = 64;  // K positions per plane block
__host__ __device__ inline int oz_kp(int K) { return (K + OBK - 1) / OBK * OBK; }

// Slice buffers hold three parts per slice: real digits, imaginary digits and the
// negated imaginary digits (so that a product never negates on the fly). Within a
// part ("plane"), the digits of 16 rows x 64 K-positions form one contiguous KiB
// (row-block major, then K-block), so a 64-lane load of 16 bytes per lane moves
// one whole block; inside a block a row is 64 bytes whose four 16-byte chunks are
// stored in the order chunk ^ f(row) (f below), which spreads the fragment reads of
// consecutive rows over the LDS banks after the block is copied as it is.
constexpr int kParts = 3;
__host__ __device__ inline int oz_rows_pad(int rows) { return (rows + 15) / 16 * 16; }
__host__ __device__ inline int chunk_swz(int row) { return ((row >> 1) ^ (row >> 3)) & 3; }
__host__ __device__ inline long oz_plane_bytes(int rows, int Kp) { return (long)oz_rows_pad(rows) * Kp; }
// byte of (row, k) inside a plane with KB = Kp / 64 K-blocks
__device__ inline long oz_off(int row, int k, int KB) {
  return ((long)(row >> 4) * KB + (k >> 6)) * 1024 + (row & 15) * 64 + ((((k >> 4) & 3) ^ chunk_swz(row)) << 4) +
         (k & 15);
}

__host__ __device__ inline int scale_exponent(double m) {
  if (!(m > 0)) return 0;
  int e;
  frexp(m, &e);  // m = f 2^e, f in [0.5, 1): m < 2^e
  return e;
}

typedef __attribute__((address_space(3))) void lds_ptr_t;
typedef __attribute__((address_space(1))) const void gbl_ptr_t;

// s_waitcnt immediates (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4,
// lgkmcnt 11:8; a field at its maximum does not wait).
constexpr int kWaitLgkm0 = 0xC07F;                   // lgkmcnt(0)
constexpr int kWaitVm0 = 0x0F70;                     // vmcnt(0)

}  // namespace sr
