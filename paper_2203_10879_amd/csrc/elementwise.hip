// HBM-bound steps of a refinement pass: Frobenius norms, W = L - L^H, the
// Newton-Schulz correction Delta, precision conversions.
//
// Reductions are deterministic: blocks write partial sums to fixed slots and one
// block adds them in a fixed order.
#include "kernels.hpp"

namespace sr {

constexpr int ENT = 256;

__device__ inline double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) s += red[w];
  }
  return s;
}

__global__ __launch_bounds__(ENT) void fro2_kernel(const zc* __restrict__ x, long count,
                                                   double* __restrict__ partials) {
  __shared__ double red[ENT / 64];
  double s = 0;
  for (long i = blockIdx.x * (long)ENT + threadIdx.x; i < count; i += (long)gridDim.x * ENT) {
    const zc v = x[i];
    s += v.re * v.re + v.im * v.im;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

hipError_t fro2_partials(const zc* x, long count, double* partials, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(fro2_kernel, dim3(nparts), dim3(ENT), 0, st, x, count, partials);
  return hipGetLastError();
}

__global__ __launch_bounds__(ENT) void reduce_kernel(const double* __restrict__ partials, int np,
                                                     double* __restrict__ out) {
  __shared__ double red[ENT / 64];
  double s = 0;
  for (int i = threadIdx.x; i < np; i += ENT) s += partials[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = s;
}

hipError_t reduce_partials(const double* partials, int np, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(ENT), 0, st, partials, np, out);
  return hipGetLastError();
}

// 32 x 32 tiles; block (bi, bj) also stages the transposed tile (bj, bi) of L so
// that both L(i, j) and L(j, i) are read with coalesced accesses.
constexpr int ET = 32;

int form_w_parts(int n) {
  const int nb = ceil_div(n, ET);
  return nb * nb;
}

template <typename R>
__global__ __launch_bounds__(ENT) void form_w_kernel(const cplx<R>* __restrict__ L,
                                                     cplx<R>* __restrict__ W, int n,
                                                     double* __restrict__ partials) {
  using cc = cplx<R>;
  __shared__ cc lt[ET][ET + 1];
  __shared__ double red[ENT / 64];
  const int nb = ceil_div(n, ET);
  const int bi = blockIdx.x % nb, bj = blockIdx.x / nb;
  // lt[a][b] = L(bj*ET + a, bi*ET + b)
  for (int r = threadIdx.x; r < ET * ET; r += ENT) {
    const int a = r & (ET - 1), b = r >> 5;
    const int gi = bj * ET + a, gj = bi * ET + b;
    cc v = mk<R>(0, 0);
    if (gi < n && gj < n && gi > gj) v = L[gi + (long)gj * n];
    lt[a][b] = v;
  }
  __syncthreads();
  double s = 0;
  for (int r = threadIdx.x; r < ET * ET; r += ENT) {
    const int a = r & (ET - 1), b = r >> 5;
    const int i = bi * ET + a, j = bj * ET + b;
    if (i < n && j < n) {
      cc w = mk<R>(0, 0);
      if (i > j) {
        w = L[i + (long)j * n];
      } else if (i < j) {
        const cc u = lt[b][a];  // L(j, i)
        w = mk<R>(-u.re, u.im);
      }
      W[i + (long)j * n] = w;
      s += (double)w.re * w.re + (double)w.im * w.im;
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

hipError_t form_w(const cc* L, cc* W, int n, double* partials, hipStream_t st) {
  hipLaunchKernelGGL(form_w_kernel<float>, dim3(form_w_parts(n)), dim3(ENT), 0, st, L, W, n, partials);
  return hipGetLastError();
}

hipError_t form_w64(const zc* L, zc* W, int n, double* partials, hipStream_t st) {
  hipLaunchKernelGGL(form_w_kernel<double>, dim3(form_w_parts(n)), dim3(ENT), 0, st, L, W, n, partials);
  return hipGetLastError();
}

// Double-double tier: D = W - Y/2 + (W2 + W3 - YW)/2 with W = L - L^H (FP64, exact
// in double-double), Y = Yhi + Ylo and the lp products in FP64.
__global__ __launch_bounds__(ENT) void form_delta_dd_kernel(
    const zc* __restrict__ L, const zc* __restrict__ Yhi, const zc* __restrict__ Ylo,
    const zc* __restrict__ W2, const zc* __restrict__ W3, const zc* __restrict__ YW,
    zc* __restrict__ Dhi, zc* __restrict__ Dlo, int n) {
  __shared__ zc lt[ET][ET + 1];
  const int nb = ceil_div(n, ET);
  const int bi = blockIdx.x % nb, bj = blockIdx.x / nb;
  if (L) {
    for (int r = threadIdx.x; r < ET * ET; r += ENT) {
      const int a = r & (ET - 1), b = r >> 5;
      const int gi = bj * ET + a, gj = bi * ET + b;
      zc v = mk<double>(0, 0);
      if (gi < n && gj < n && gi > gj) v = L[gi + (long)gj * n];
      lt[a][b] = v;
    }
    __syncthreads();
  }
  for (int r = threadIdx.x; r < ET * ET; r += ENT) {
    const int a = r & (ET - 1), b = r >> 5;
    const int i = bi * ET + a, j = bj * ET + b;
    if (i < n && j < n) {
      const long o = i + (long)j * n;
      double wr = 0, wi = 0;
      if (L) {
        if (i > j) {
          const zc u = L[o];
          wr = u.re;
          wi = u.im;
        } else if (i < j) {
          const zc u = lt[b][a];
          wr = -u.re;
          wi = u.im;
        }
      }
      double pr = 0, pi = 0;
      if (W2) {
        pr += W2[o].re;
        pi += W2[o].im;
      }
      if (W3) {
        pr += W3[o].re;
        pi += W3[o].im;
      }
      if (YW) {
        pr -= YW[o].re;
        pi -= YW[o].im;
      }
      const zc yh = Yhi[o], yl = Ylo[o];
      // (-Y/2) in double-double, then + W and + (lp terms)/2
      double rh = -0.5 * yh.re, rl = -0.5 * yl.re, ih = -0.5 * yh.im, il = -0.5 * yl.im;
      dd_add(rh, rl, wr);
      dd_add(ih, il, wi);
      dd_add(rh, rl, 0.5 * pr);
      dd_add(ih, il, 0.5 * pi);
      Dhi[o] = mk<double>(rh, ih);
      Dlo[o] = mk<double>(rl, il);
    }
  }
}

// The triple-double Delta: W - Y/2 + (W2 + W3 - YW)/2 with Y = Y0 + Y1 + Y2 and the lp
// terms (FP64) added as exact double-double sums.
__global__ __launch_bounds__(ENT) void form_delta_td_kernel(
    const zc* __restrict__ L, const zc* __restrict__ Y0, const zc* __restrict__ Y1, const zc* __restrict__ Y2,
    const zc* __restrict__ W2, const zc* __restrict__ W3, const zc* __restrict__ YW, zc* __restrict__ D0,
    zc* __restrict__ D1, zc* __restrict__ D2, int n) {
  __shared__ zc lt[ET][ET + 1];
  const int nb = ceil_div(n, ET);
  const int bi = blockIdx.x % nb, bj = blockIdx.x / nb;
  if (L) {
    for (int r = threadIdx.x; r < ET * ET; r += ENT) {
      const int a = r & (ET - 1), b = r >> 5;
      const int gi = bj * ET + a, gj = bi * ET + b;
      zc v = mk<double>(0, 0);
      if (gi < n && gj < n && gi > gj) v = L[gi + (long)gj * n];
      lt[a][b] = v;
    }
    __syncthreads();
  }
  for (int r = threadIdx.x; r < ET * ET; r += ENT) {
    const int a = r & (ET - 1), b = r >> 5;
    const int i = bi * ET + a, j = bj * ET + b;
    if (i < n && j < n) {
      const long o = i + (long)j * n;
      double wr = 0, wi = 0;
      if (L) {
        if (i > j) {
          const zc u = L[o];
          wr = u.re;
          wi = u.im;
        } else if (i < j) {
          const zc u = lt[b][a];
          wr = -u.re;
          wi = u.im;
        }
      }
      double pr = 0, pi = 0;
      if (W2) {
        pr += W2[o].re;
        pi += W2[o].im;
      }
      if (W3) {
        pr += W3[o].re;
        pi += W3[o].im;
      }
      if (YW) {
        pr -= YW[o].re;
        pi -= YW[o].im;
      }
      // W + (lp terms)/2 as an exact double-double, then + (-Y/2) in triple-double
      double sr, er, si, ei;
      two_sum(wr, 0.5 * pr, sr, er);
      two_sum(wi, 0.5 * pi, si, ei);
      const zc y0 = Y0[o], y1 = Y1[o], y2 = Y2[o];
      double r0, r1, r2, q0, q1, q2;
      td_add(-0.5 * y0.re, -0.5 * y1.re, -0.5 * y2.re, sr, er, 0.0, r0, r1, r2);
      td_add(-0.5 * y0.im, -0.5 * y1.im, -0.5 * y2.im, si, ei, 0.0, q0, q1, q2);
      D0[o] = mk<double>(r0, q0);
      D1[o] = mk<double>(r1, q1);
      D2[o] = mk<double>(r2, q2);
    }
  }
}

hipError_t form_delta_td(const zc* L, const zc* Y0, const zc* Y1, const zc* Y2, const zc* W2, const zc* W3,
                         const zc* YW, zc* D0, zc* D1, zc* D2, int n, hipStream_t st) {
  const int nb = ceil_div(n, ET);
  hipLaunchKernelGGL(form_delta_td_kernel, dim3(nb * nb), dim3(ENT), 0, st, L, Y0, Y1, Y2, W2, W3, YW, D0, D1,
                     D2, n);
  return hipGetLastError();
}

hipError_t form_delta_dd(const zc* L, const zc* Yhi, const zc* Ylo, const zc* W2, const zc* W3,
                         const zc* YW, zc* Dhi, zc* Dlo, int n, hipStream_t st) {
  const int nb = ceil_div(n, ET);
  hipLaunchKernelGGL(form_delta_dd_kernel, dim3(nb * nb), dim3(ENT), 0, st, L, Yhi, Ylo, W2, W3, YW,
                     Dhi, Dlo, n);
  return hipGetLastError();
}

// Delta = W - Y/2 + (W2 + W3 - YW)/2 in FP64, W = L - L^H widened from FP32.
__global__ __launch_bounds__(ENT) void form_delta_kernel(const cc* __restrict__ L,
                                                         const zc* __restrict__ Y,
                                                         const cc* __restrict__ W2,
                                                         const cc* __restrict__ W3,
                                                         const cc* __restrict__ YW,
                                                         zc* __restrict__ D, int n) {
  __shared__ cc lt[ET][ET + 1];
  const int nb = ceil_div(n, ET);
  const int bi = blockIdx.x % nb, bj = blockIdx.x / nb;
  if (L) {
    for (int r = threadIdx.x; r < ET * ET; r += ENT) {
      const int a = r & (ET - 1), b = r >> 5;
      const int gi = bj * ET + a, gj = bi * ET + b;
      cc v = mk<float>(0.f, 0.f);
      if (gi < n && gj < n && gi > gj) v = L[gi + (long)gj * n];
      lt[a][b] = v;
    }
    __syncthreads();
  }
  for (int r = threadIdx.x; r < ET * ET; r += ENT) {
    const int a = r & (ET - 1), b = r >> 5;
    const int i = bi * ET + a, j = bj * ET + b;
    if (i < n && j < n) {
      const long o = i + (long)j * n;
      double wr = 0, wi = 0;
      if (L) {
        if (i > j) {
          const cc u = L[o];
          wr = u.re;
          wi = u.im;
        } else if (i < j) {
          const cc u = lt[b][a];
          wr = -(double)u.re;
          wi = u.im;
        }
      }
      const zc y = Y ? Y[o] : mk<double>(0, 0);
      double pr = 0, pi = 0;
      if (W2) {
        pr += W2[o].re;
        pi += W2[o].im;
      }
      if (W3) {
        pr += W3[o].re;
        pi += W3[o].im;
      }
      if (YW) {
        pr -= YW[o].re;
        pi -= YW[o].im;
      }
      D[o] = mk<double>(wr - 0.5 * y.re + 0.5 * pr, wi - 0.5 * y.im + 0.5 * pi);
    }
  }
}

hipError_t form_delta(const cc* L, const zc* Y, const cc* W2, const cc* W3, const cc* YW, zc* D,
                      int n, hipStream_t st) {
  const int nb = ceil_div(n, ET);
  hipLaunchKernelGGL(form_delta_kernel, dim3(nb * nb), dim3(ENT), 0, st, L, Y, W2, W3, YW, D, n);
  return hipGetLastError();
}

__global__ __launch_bounds__(ENT) void to_c64_kernel(const zc* __restrict__ x, cc* __restrict__ y,
                                                     long count) {
  for (long i = blockIdx.x * (long)ENT + threadIdx.x; i < count; i += (long)gridDim.x * ENT)
    y[i] = mk<float>((float)x[i].re, (float)x[i].im);
}

hipError_t to_c64(const zc* x, cc* y, long count, hipStream_t st) {
  const int blocks = (int)std::min<long>(4096, (count + ENT - 1) / ENT);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(to_c64_kernel, dim3(blocks), dim3(ENT), 0, st, x, y, count);
  return hipGetLastError();
}

template <typename C>
__global__ __launch_bounds__(ENT) void w2_minus_y_kernel(const C* __restrict__ W2, const zc* __restrict__ Y,
                                                         C* __restrict__ X, long count) {
  using R = decltype(C::re);
  for (long i = blockIdx.x * (long)ENT + threadIdx.x; i < count; i += (long)gridDim.x * ENT) {
    const C w = W2[i];
    const zc y = Y[i];
    X[i] = mk<R>((R)((double)w.re - y.re), (R)((double)w.im - y.im));
  }
}

template <typename C>
static hipError_t launch_w2_minus_y(const C* W2, const zc* Y, C* X, long count, hipStream_t st) {
  const int blocks = (int)std::min<long>(4096, (count + ENT - 1) / ENT);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(w2_minus_y_kernel<C>, dim3(blocks), dim3(ENT), 0, st, W2, Y, X, count);
  return hipGetLastError();
}
hipError_t w2_minus_y(const cc* W2, const zc* Y, cc* X, long count, hipStream_t st) {
  return launch_w2_minus_y(W2, Y, X, count, st);
}
hipError_t w2_minus_y(const zc* W2, const zc* Y, zc* X, long count, hipStream_t st) {
  return launch_w2_minus_y(W2, Y, X, count, st);
}

__global__ __launch_bounds__(ENT) void zero_kernel(uint32_t* __restrict__ p, long words) {
  for (long i = blockIdx.x * (long)ENT + threadIdx.x; i < words; i += (long)gridDim.x * ENT) p[i] = 0u;
}

// A fill kernel rather than hipMemsetAsync, so that the call can sit inside a
// captured HIP graph.
hipError_t fill_zero(void* p, size_t bytes, hipStream_t st) {
  const long words = (long)(bytes / 4);
  const int blocks = (int)std::min<long>(2048, (words + ENT - 1) / ENT);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(ENT), 0, st, (uint32_t*)p, words);
  return hipGetLastError();
}

}  // namespace sr
