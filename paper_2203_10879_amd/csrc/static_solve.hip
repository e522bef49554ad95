// Triangular matrix equation stril(T L - L T) = -E in FP32 without any allocation,
// for callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc). It runs the same kernels as
// sr_trisolve; the only difference is where their scratch lives.
//
// The solve's scratch is the far partial sums passed from one tile-diagonal launch
// to the next (two parity buffers). Here it is the file-scope device array
// `scratch`, sized for every n <= kStaticMaxN. Each GPU holds its own copy of the
// array at its own address, kept until the process ends; host code never passes
// the array's name to a kernel (in host code it is only a stand-in for the
// symbol) but the device address hipGetSymbolAddress returns, looked up once per
// device with that device current.
//
// Nothing in the array has to start at zero: every partial-sum slot a launch
// reads was written by the previous launch of the same call. All calls on one
// GPU share the array, so calls that overlap on one GPU (different streams, or
// different host threads on one stream without ordering) race.
#include <mutex>

#include "../../include/schur_refine.h"
#include "kernels.hpp"

using namespace sr;

namespace {

constexpr int kStaticMaxN = 4096;
// trisolve_ws_bytes(n) for n <= 4096: two buffers of (2 * 256 + nb) tiles of
// TB x TB complex128 slots, at most 2 * 640 * 32 * 32 * 16 B = 20 MiB (n in
// (2048, 4096], 32-wide tiles, nb <= 128; 16-wide tiles up to 2048 need 5 MiB).
constexpr size_t kStaticScratchBytes = size_t(20) << 20;

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first call
// on that device).
int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SR_EHIP;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SR_EHIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return SR_OK;
}

}  // namespace

extern "C" int sr_trisolve_static(const void* T_lp, const void* E_lp, void* L_lp, int n, float trunc,
                                  unsigned* status, void* stream) {
  if (!T_lp || !E_lp || !L_lp || !status || n < 1) return SR_EINVAL;
  if (n > kStaticMaxN || trisolve_ws_bytes(n) > kStaticScratchBytes) return SR_ENOMEM;
  void* ptr = nullptr;
  const int rc = scratch_address(&ptr);
  if (rc != SR_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  // the status word is the caller's output: cleared here by a kernel (no memset
  // node in a captured graph), then set by the solve's kernels on breakdown
  if (fill_zero(status, sizeof(unsigned), st) != hipSuccess) return SR_EHIP;
  if (trisolve((const cc*)T_lp, (const cc*)E_lp, (cc*)L_lp, n, trunc, ptr, status, st) != hipSuccess)
    return SR_EHIP;
  return SR_OK;
}
