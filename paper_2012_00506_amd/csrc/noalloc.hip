// band_inertia_noalloc: Sylvester inertia with a fixed, library-owned device
// scratch, for callers that cannot allocate device memory.
//
// The scratch is a file-scope __device__ array; each device holds its own
// copy at its own address.  Host code never uses the array's name as an
// address: the device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept in a table.
#include <math.h>

#include <mutex>

#include "solve_job.h"

namespace {

static __device__ __align__(256) char scratch[FB_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch (looked up on first use).
int scratch_ptr(void** out) {
  int dev = 0;
  FB_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return FB_ERR_INTERNAL;
  std::lock_guard<std::mutex> g(g_mu);
  if (g_ptr[dev] == nullptr) {
    void* p = nullptr;
    FB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) return FB_ERR_INTERNAL;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return 0;
}

}  // namespace

extern "C" int band_inertia_noalloc(const fb_band* B, int32_t nshift, const double* shifts,
                                    int32_t* n_neg, int32_t* n_zero, int32_t* n_pos,
                                    void* stream) {
  if (fb::check_band(B)) return -1;
  if (nshift < 0) return -2;
  if (nshift > 0 && !shifts) return -3;
  if (nshift > 0 && !n_neg) return -4;
  for (int i = 0; i < nshift; ++i)
    if (!isfinite(shifts[i])) return -3;
  // size of the work as band_inertia lays it out (a host-only query)
  size_t need = 0;
  FB_TRY(band_inertia(B, nshift, shifts, n_neg, n_zero, n_pos, nullptr, &need, stream));
  if (need > (size_t)FB_NOALLOC_SCRATCH_BYTES) return FB_ERR_TOO_LARGE;
  if (nshift == 0) return 0;
  void* p = nullptr;
  FB_TRY(scratch_ptr(&p));
  size_t cap = FB_NOALLOC_SCRATCH_BYTES;
  return band_inertia(B, nshift, shifts, n_neg, n_zero, n_pos, p, &cap, stream);
}
