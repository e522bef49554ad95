// Reordering of the start (Section 2.4, the paragraph on the reordering of
// Algorithm 4): the Schur form T = triu(Qh^H A Qh) of the lp start is reordered by
// unitary swaps of adjacent diagonal entries so that the eigenvalues follow the
// order of their projections Re(lambda e^{-i theta}) onto a line with direction
// e^{i theta}; eigenvalues that lie close together become neighbours, which keeps
// the ill-conditioned part of the triangular equation local.
//
// Swap of positions (i, i+1) with block [[a, b], [0, d]]: G = [[g1, -conj(g2)],
// [g2, conj(g1)]] with (g1, g2) = (b, d - a) / r (the unit eigenvector of d) gives
// G^H [[a, b], [0, d]] G = [[d, *], [0, a]]; T <- G^H T G on rows and columns
// i, i+1, Q <- Q G. The keys are computed once and travel with their entries, so
// the swap decisions do not depend on rounding.
//
// Order: odd-even transposition, n phases; phase p swaps every pair (i, i+1) with
// i = p mod 2 whose keys are out of order. The pairs of a phase touch disjoint rows
// and disjoint columns, and left and right multiplications commute, so a phase is
// two launches: all row rotations (one block per pair), then all column rotations
// of T and Q. T stays exactly upper triangular (the rotated subdiagonal entry is
// set to zero), so rows are touched from column i on and columns up to row i+1.
#include "kernels.hpp"

namespace sr {

constexpr int kRoNT = 256;

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Strictly lower part of T to zero; keys of the diagonal; identity permutation.
// One block per column.
__global__ __launch_bounds__(kRoNT) void reorder_init_kernel(zc* __restrict__ T, int n, double c, double s,
                                                             double* __restrict__ key, int* __restrict__ perm) {
  const int j = blockIdx.x;
  for (int i = j + 1 + threadIdx.x; i < n; i += kRoNT) T[i + (long)j * n] = mk<double>(0, 0);
  if (threadIdx.x == 0) {
    const zc t = T[j + (long)j * n];
    key[j] = t.re * c + t.im * s;
    perm[j] = j;
  }
}

// Phase with pairs (i, i+1), i = 2 k + par, block k: if out of order, the
// rotation of the pair (stored for the column launch) and T <- G^H T on rows i,
// i+1, columns i .. n-1.
__global__ __launch_bounds__(kRoNT) void reorder_rows_kernel(zc* __restrict__ T, int n, int par,
                                                             const double* __restrict__ key,
                                                             double4* __restrict__ rot, int* __restrict__ on) {
  const int k = blockIdx.x, i = 2 * k + par;
  if (!(key[i] > key[i + 1])) {
    if (threadIdx.x == 0) on[k] = 0;
    return;
  }
  const zc a = T[i + (long)i * n], b = T[i + (long)(i + 1) * n], d = T[(i + 1) + (long)(i + 1) * n];
  const double xr = d.re - a.re, xi = d.im - a.im;
  const double r = sqrt(b.re * b.re + b.im * b.im + xr * xr + xi * xi);
  const double g1r = b.re / r, g1i = b.im / r, g2r = xr / r, g2i = xi / r;
  __syncthreads();  // every thread has read the pair's block before rows change
  for (int j = i + threadIdx.x; j < n; j += kRoNT) {
    const zc u = T[i + (long)j * n], v = T[(i + 1) + (long)j * n];
    // row i: conj(g1) u + conj(g2) v; row i+1: -g2 u + g1 v
    T[i + (long)j * n] = mk<double>(g1r * u.re + g1i * u.im + g2r * v.re + g2i * v.im,
                                    g1r * u.im - g1i * u.re + g2r * v.im - g2i * v.re);
    T[(i + 1) + (long)j * n] = mk<double>(-(g2r * u.re - g2i * u.im) + g1r * v.re - g1i * v.im,
                                          -(g2r * u.im + g2i * u.re) + g1r * v.im + g1i * v.re);
  }
  if (threadIdx.x == 0) {
    rot[k] = make_double4(g1r, g1i, g2r, g2i);
    on[k] = 1;
  }
}

// The same phase: T <- T G on columns i, i+1 (rows 0 .. i+1, the new subdiagonal
// entry set to zero), Q <- Q G, and the pair's keys and positions exchanged.
__global__ __launch_bounds__(kRoNT) void reorder_cols_kernel(zc* __restrict__ T, zc* __restrict__ Q, int n,
                                                             int par, double* __restrict__ key,
                                                             int* __restrict__ perm,
                                                             const double4* __restrict__ rot,
                                                             const int* __restrict__ on) {
  const int k = blockIdx.x, i = 2 * k + par;
  if (!on[k]) return;
  const double4 g = rot[k];
  const double g1r = g.x, g1i = g.y, g2r = g.z, g2i = g.w;
  for (int m = 0; m < 2; m++) {
    zc* X = m ? Q : T;
    const int rows = m ? n : i + 2;
    for (int r = threadIdx.x; r < rows; r += kRoNT) {
      const zc u = X[r + (long)i * n], v = X[r + (long)(i + 1) * n];
      // column i: g1 u + g2 v; column i+1: -conj(g2) u + conj(g1) v
      zc ci = mk<double>(g1r * u.re - g1i * u.im + g2r * v.re - g2i * v.im,
                         g1r * u.im + g1i * u.re + g2r * v.im + g2i * v.re);
      const zc cj = mk<double>(-(g2r * u.re + g2i * u.im) + g1r * v.re + g1i * v.im,
                               -(g2r * u.im - g2i * u.re) + g1r * v.im - g1i * v.re);
      if (!m && r == i + 1) ci = mk<double>(0, 0);
      X[r + (long)i * n] = ci;
      X[r + (long)(i + 1) * n] = cj;
    }
  }
  if (threadIdx.x == 0) {
    const double tk = key[i];
    key[i] = key[i + 1];
    key[i + 1] = tk;
    const int tp = perm[i];
    perm[i] = perm[i + 1];
    perm[i + 1] = tp;
  }
}

size_t reorder_scratch_bytes(int n) {
  const int pairs = (n + 1) / 2;
  return round256((size_t)n * sizeof(double)) + round256((size_t)n * sizeof(int)) +
         round256((size_t)pairs * sizeof(double4)) + round256((size_t)pairs * sizeof(int));
}

hipError_t reorder_swaps(zc* T, zc* Q, int n, double theta, void* scratch, int* perm_out, hipStream_t st) {
  char* p = (char*)scratch;
  const int pairs = (n + 1) / 2;
  double* key = (double*)p;
  p += round256((size_t)n * sizeof(double));
  int* perm = (int*)p;
  p += round256((size_t)n * sizeof(int));
  double4* rot = (double4*)p;
  p += round256((size_t)pairs * sizeof(double4));
  int* on = (int*)p;
  hipLaunchKernelGGL(reorder_init_kernel, dim3(n), dim3(kRoNT), 0, st, T, n, cos(theta), sin(theta), key, perm);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int ph = 0; ph < n; ph++) {
    const int par = ph & 1, np = (n - par) / 2;
    if (np == 0) continue;
    hipLaunchKernelGGL(reorder_rows_kernel, dim3(np), dim3(kRoNT), 0, st, T, n, par, (const double*)key, rot, on);
    hipLaunchKernelGGL(reorder_cols_kernel, dim3(np), dim3(kRoNT), 0, st, T, Q, n, par, key, perm,
                       (const double4*)rot, (const int*)on);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (perm_out) return hipMemcpyAsync(perm_out, perm, (size_t)n * sizeof(int), hipMemcpyDeviceToDevice, st);
  return hipSuccess;
}

}  // namespace sr
