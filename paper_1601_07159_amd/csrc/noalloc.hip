// Allocation-free apply (for callers that cannot allocate device memory: code
// under HIP graph capture on a context without a reserved workspace, tight
// serving loops, harnesses that forbid hipMalloc).  It runs the kernels of
// ace_apply, Y = -xi (dV xi^H X), with their scratch (the n_band x n_x matrix
// dV xi^H X and the split-K partial sums of the reduction product) in one
// file-scope device array instead of the context workspace.
//
// The array is part of the library's code object: every GPU that loads the
// library holds its own copy, at its own address, until the process ends.
// Its device address is looked up once per device (ace_create calls
// noalloc_setup with the device current); host code uses that address only,
// never the array's name.  Every call on a GPU shares that GPU's array, so two
// calls that overlap on one GPU (two contexts, or one context on two streams
// with no ordering between them) race on it.  Nothing in it needs clearing:
// every entry a call reads was written earlier in the same call.
#include <cstdio>
#include <mutex>

#include "ace_internal.h"

#define ACE_EXPORT extern "C" __attribute__((visibility("default")))

namespace ace {
ace_status apply_entry(ace_ctx c, const ace_grid* grid, ace_prec prec, const void* xi, int n_band,
                       long ld_xi, const void* X, int n_x, long ld_x, void* Y, long ld_y,
                       char* sub, size_t sub_bytes);

namespace {

// 48 MiB: n_band x n_x up to 256 x 256 at any grid of the library in every
// precision (partials of at most 64 K chunks in FP32 or 32 in FP64, plus the
// 1 MiB matrix).
constexpr size_t kScratchBytes = (size_t)48 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

}  // namespace

void noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_done[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) (void)hipGetLastError();
  g_ptr[device] = e == hipSuccess ? p : nullptr;
  g_err[device] = e;
  g_done[device] = true;
}

}  // namespace ace

using namespace ace;

ACE_EXPORT ace_status ace_apply_noalloc(ace_ctx c, const ace_grid* grid, ace_prec prec,
                                        const void* xi, int n_band, long ld_xi, const void* X,
                                        int n_x, long ld_x, void* Y, long ld_y) {
  if (!c) return ACE_E_ARG;
  void* p = nullptr;
  hipError_t e = hipSuccess;
  if (c->device >= 0 && c->device < kMaxDevices) {
    std::lock_guard<std::mutex> lock(g_mu);
    p = g_ptr[c->device];
    e = g_err[c->device];
  }
  if (!p) {
    char buf[128];
    snprintf(buf, sizeof buf, "allocation-free apply: no scratch address on device %d (%s)",
             c->device, e != hipSuccess ? hipGetErrorString(e) : "not set up");
    return fail(c, ACE_E_HIP, buf);
  }
  return apply_entry(c, grid, prec, xi, n_band, ld_xi, X, n_x, ld_x, Y, ld_y, (char*)p,
                     kScratchBytes);
}
