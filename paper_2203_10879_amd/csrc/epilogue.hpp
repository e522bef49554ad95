// Per-element epilogues shared by the complex GEMM kernels (FP64 MFMA and the
// Ozaki INT8 split product): they fuse the elementwise steps of a refinement
// pass into the store of a product.
#pragma once

#include "kernels.hpp"

namespace sr {

// Store one element (i, j) of a product; `part` accumulates the squared norm the
// SPLIT and YDEF epilogues report.
template <int EPI, typename R>
__device__ inline void epi_element(const GemmArgs& g, int i, int j, cplx<R> val, double& part) {
  using C = cplx<R>;
  C* __restrict__ Cp = (C*)g.C;
  const long o = i + (long)j * g.ldc;
  if constexpr (EPI == EPI_STORE) {
    if (g.herm) {
      if (i > j) return;  // the mirror of (j, i) is stored there
      if (i < j) Cp[j + (long)i * g.ldc] = g.herm > 0 ? mk<R>(val.re, -val.im) : mk<R>(-val.re, val.im);
    }
    Cp[o] = val;
  } else if constexpr (EPI == EPI_ADD) {
    const C c0 = ((const C*)g.Cin)[i + (long)j * g.ldcin];
    const C r = mk<R>(c0.re + val.re, c0.im + val.im);
    Cp[o] = r;
    // optional conjugate transpose of the result; in the MFMA accumulator layouts
    // lanes 16 apart hold consecutive columns j, so the transposed store still
    // writes runs of 16 consecutive elements
    if (g.CH) ((C*)g.CH)[j + (long)i * g.ldch] = mk<R>(r.re, -r.im);
  } else if constexpr (EPI == EPI_SPLIT) {
    const long ol = i + (long)j * g.ldlp;
    if (i <= j) {
      Cp[o] = val;
      g.Tlp[ol] = mk<float>((float)val.re, (float)val.im);
      g.Elp[ol] = mk<float>(0.f, 0.f);
    } else {
      Cp[o] = mk<R>(0, 0);
      g.Tlp[ol] = mk<float>(0.f, 0.f);
      g.Elp[ol] = mk<float>((float)val.re, (float)val.im);
      part += (double)val.re * val.re + (double)val.im * val.im;
    }
  } else {  // EPI_YDEF
    if (g.herm && i > j) return;  // the conjugate of (j, i) is stored there
    if (i == j) val.re -= 1;
    Cp[o] = val;
    const double p = (double)val.re * val.re + (double)val.im * val.im;
    part += p;
    if (g.herm && i < j) {
      // lanes 16 apart hold consecutive j, so the mirrored store writes runs of
      // consecutive elements
      Cp[j + (long)i * g.ldc] = mk<R>(val.re, -val.im);
      part += p;
    }
  }
}

// Double-double variant: the product value is hi + lo (complex128 each).
template <int EPI>
__device__ inline void epi_element_dd(const GemmArgs& g, int i, int j, zc hi, zc lo, double& part) {
  zc* __restrict__ Ch = (zc*)g.C;
  zc* __restrict__ Cl = (zc*)g.Clo;
  const long o = i + (long)j * g.ldc;
  if constexpr (EPI == EPI_STORE) {
    Ch[o] = hi;
    Cl[o] = lo;
  } else if constexpr (EPI == EPI_ADD) {
    const long oi = i + (long)j * g.ldcin;
    const zc ah = ((const zc*)g.Cin)[oi], al = ((const zc*)g.Cinlo)[oi];
    double rh = ah.re, rl = al.re, ih = ah.im, il = al.im;
    dd_add(rh, rl, hi.re, lo.re);
    dd_add(ih, il, hi.im, lo.im);
    Ch[o] = mk<double>(rh, ih);
    Cl[o] = mk<double>(rl, il);
  } else if constexpr (EPI == EPI_SPLIT) {
    const long ol = i + (long)j * g.ldlp;
    const zc z = mk<double>(0, 0);
    if (i <= j) {
      Ch[o] = hi;
      Cl[o] = lo;
      g.Tlp64[ol] = hi;
      g.Elp64[ol] = z;
    } else {
      Ch[o] = z;
      Cl[o] = z;
      g.Tlp64[ol] = z;
      g.Elp64[ol] = hi;
      part += hi.re * hi.re + hi.im * hi.im;
    }
  } else {  // EPI_YDEF
    if (g.herm && i > j) return;  // the conjugate of (j, i) is stored there
    double rh = hi.re, rl = lo.re;
    if (i == j) dd_add(rh, rl, -1.0);
    Ch[o] = mk<double>(rh, hi.im);
    Cl[o] = mk<double>(rl, lo.im);
    const double p = rh * rh + hi.im * hi.im;
    part += p;
    if (g.herm && i < j) {
      const long t = j + (long)i * g.ldc;
      Ch[t] = mk<double>(rh, -hi.im);
      Cl[t] = mk<double>(rl, -lo.im);
      part += p;
    }
  }
}

// Triple-double variant: the product value is x0 + x1 + x2 (complex128 each).
template <int EPI>
__device__ inline void epi_element_td(const GemmArgs& g, int i, int j, zc x0, zc x1, zc x2, double& part) {
  zc* __restrict__ C0 = (zc*)g.C;
  zc* __restrict__ C1 = (zc*)g.Cmid;
  zc* __restrict__ C2 = (zc*)g.Clo;
  const long o = i + (long)j * g.ldc;
  const zc z = mk<double>(0, 0);
  if constexpr (EPI == EPI_STORE) {
    C0[o] = x0;
    C1[o] = x1;
    C2[o] = x2;
  } else if constexpr (EPI == EPI_ADD) {
    const long oi = i + (long)j * g.ldcin;
    const zc a0 = ((const zc*)g.Cin)[oi], a1 = ((const zc*)g.Cinmid)[oi], a2 = ((const zc*)g.Cinlo)[oi];
    double r0, r1, r2, i0, i1, i2;
    td_add(a0.re, a1.re, a2.re, x0.re, x1.re, x2.re, r0, r1, r2);
    td_add(a0.im, a1.im, a2.im, x0.im, x1.im, x2.im, i0, i1, i2);
    C0[o] = mk<double>(r0, i0);
    C1[o] = mk<double>(r1, i1);
    C2[o] = mk<double>(r2, i2);
  } else if constexpr (EPI == EPI_SPLIT) {
    const long ol = i + (long)j * g.ldlp;
    if (i <= j) {
      C0[o] = x0;
      C1[o] = x1;
      C2[o] = x2;
      g.Tlp64[ol] = x0;
      g.Elp64[ol] = z;
    } else {
      C0[o] = z;
      C1[o] = z;
      C2[o] = z;
      g.Tlp64[ol] = z;
      g.Elp64[ol] = x0;
      part += x0.re * x0.re + x0.im * x0.im;
    }
  } else {  // EPI_YDEF
    if (g.herm && i > j) return;  // the conjugate of (j, i) is stored there
    double r0 = x0.re, r1 = x1.re, r2 = x2.re;
    if (i == j) td_add(r0, r1, r2, -1.0, 0.0, 0.0, r0, r1, r2);
    C0[o] = mk<double>(r0, x0.im);
    C1[o] = mk<double>(r1, x1.im);
    C2[o] = mk<double>(r2, x2.im);
    const double p = r0 * r0 + x0.im * x0.im;
    part += p;
    if (g.herm && i < j) {
      const long t = j + (long)i * g.ldc;
      C0[t] = mk<double>(r0, -x0.im);
      C1[t] = mk<double>(r1, -x1.im);
      C2[t] = mk<double>(r2, -x2.im);
      part += p;
    }
  }
}

// Block reduction of `part` into g.partials[slot] (fixed order).
template <int NT>
__device__ inline void epi_reduce(const GemmArgs& g, double part, double* red, int slot) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
  if (lane == 0) red[wave] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; w++) t += red[w];
    g.partials[slot] = t;
  }
}

}  // namespace sr
