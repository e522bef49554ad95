// Shared device/host definitions of the MI355X (gfx950) Schur-refinement library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sr {

template <typename R>
struct cplx {
  R re, im;
};
using zc = cplx<double>;  // complex128, layout of C99 double _Complex
using cc = cplx<float>;   // complex64

template <typename R>
__device__ __host__ inline cplx<R> mk(R re, R im) {
  cplx<R> z;
  z.re = re;
  z.im = im;
  return z;
}
template <typename R>
__device__ inline cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return mk<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// a += b * c
template <typename R>
__device__ inline void cfma(cplx<R>& a, cplx<R> b, cplx<R> c) {
  a.re = fma(b.re, c.re, fma(-b.im, c.im, a.re));
  a.im = fma(b.re, c.im, fma(b.im, c.re, a.im));
}
// a -= b * c
template <typename R>
__device__ inline void cfms(cplx<R>& a, cplx<R> b, cplx<R> c) {
  a.re = fma(-b.re, c.re, fma(b.im, c.im, a.re));
  a.im = fma(-b.re, c.im, fma(-b.im, c.re, a.im));
}

// Workgroup barrier that orders LDS accesses only: it waits for this wave's LDS
// operations (lgkmcnt(0)) but not for global loads still in flight, which a
// __syncthreads (a workgroup release) would also wait for. The empty asm
// statements keep the compiler from moving memory accesses across it.
__device__ inline void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt fields at their maximum
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Error-free sum s + e = a + b (Knuth).
__host__ __device__ inline void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Double-double arithmetic (Dekker, Knuth): a value is hi + lo with |lo| <= ulp(hi)/2.
__host__ __device__ inline void fast_two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  e = b - (s - a);
}
// (h, l) += x
__device__ inline void dd_add(double& h, double& l, double x) {
  double s, e;
  two_sum(h, x, s, e);
  e += l;
  fast_two_sum(s, e, h, l);
}
// (h, l) += (bh, bl)
__device__ inline void dd_add(double& h, double& l, double bh, double bl) {
  double s, e;
  two_sum(h, bh, s, e);
  e += l + bl;
  fast_two_sum(s, e, h, l);
}

// Device status bits written by kernels (OR-ed into a status word).
enum : unsigned {
  DEV_BREAKDOWN = 1u,  // t_ii == t_jj or a non-finite value in the solve
};

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename R>
struct MF;
// Accumulator layout: element v of lane l holds D[row(l, v)][l % 16]. The FP64
// instruction interleaves its rows (row = l/16 + 4v); the FP32 one stacks them
// (row = 4 (l/16) + v). Both were confirmed with a one-instruction probe.
template <>
struct MF<double> {
  using v4 = d4;
  __device__ static inline v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct MF<float> {
  using v4 = f4;
  __device__ static inline v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Tile (tm, tn), tm <= tn, of the upper triangle of a T x T tile grid for logical
// index L, in groups of kHermGroup tile rows: group g holds the rows from
// kHermGroup g on and walks its columns (from its own diagonal) one by one, so the
// blocks that run at once share row panels as well as column panels.
constexpr int kHermGroup = 4;
__host__ __device__ inline void herm_tile(int L, int T, int& tm, int& tn) {
  for (int r0 = 0;; r0 += kHermGroup) {
    const int h = T - r0 < kHermGroup ? T - r0 : kHermGroup;
    const int tri = h * (h + 1) / 2, cnt = tri + h * (T - r0 - h);
    if (L < cnt) {
      if (L < tri) {
        int k = (int)((sqrtf(8.f * L + 1.f) - 1.f) * 0.5f);
        while (k * (k + 1) / 2 > L) k--;
        while ((k + 1) * (k + 2) / 2 <= L) k++;
        tm = r0 + L - k * (k + 1) / 2;
        tn = r0 + k;
      } else {
        const int q = L - tri;
        tm = r0 + q % h;
        tn = r0 + h + q / h;
      }
      return;
    }
    L -= cnt;
  }
}

constexpr int kCUs = 256;  // MI355X compute units
constexpr int kXCDs = 8;   // accelerator complex dies (one L2 each)

__host__ __device__ inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// Triple-double arithmetic on renormalized expansions (x0, x1, x2), |x1| <= ulp(x0),
// |x2| <= ulp(x1) up to small factors: renormalization by error-free sums and a sum
// that keeps about 150 bits.
//
// Renormalization of three doubles of any magnitudes (a, b, c) with h + m + l = a + b
// + c exactly: two bottom-up passes of error-free sums leave h the sum rounded to
// double (one pass is not enough: where a and b + c cancel, the first pass's error
// terms can exceed the sum it returns), and m the rest rounded likewise.
__device__ inline void td_renorm(double a, double b, double c, double& h, double& m, double& l) {
  double s, e, f, t;
  two_sum(b, c, s, e);
  two_sum(a, s, t, f);
  two_sum(f, e, s, e);
  two_sum(t, s, h, f);
  two_sum(f, e, m, l);
}
__device__ inline void td_add(double a0, double a1, double a2, double b0, double b1, double b2, double& h,
                              double& m, double& l) {
  double s0, t0, s1, t1, s2, t2, u1, v1;
  two_sum(a0, b0, s0, t0);
  two_sum(a1, b1, s1, t1);
  two_sum(a2, b2, s2, t2);
  two_sum(t0, s1, u1, v1);
  td_renorm(s0, u1, (t1 + s2) + (t2 + v1), h, m, l);
}

}  // namespace sr

#define SR_HIP_CHECK(expr)                   \
  do {                                       \
    hipError_t _e = (expr);                  \
    if (_e != hipSuccess) return SR_EHIP;    \
  } while (0)
