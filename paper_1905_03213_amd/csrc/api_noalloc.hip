// wproj_grid_noalloc: binned gridding for callers that cannot allocate device memory.
//
// It is wproj_grid with its workspace taken from a fixed array in the library's own
// device memory (`scratch`, kNoallocScratchBytes per GPU, held from module load until
// the process ends) instead of from the caller.  The address of a device's copy of the
// array is looked up once per device, with that device current, and kept; every kernel
// argument and fill that touches the scratch memory uses that address, never the
// array's host-side name.  Nothing here allocates: no hipMalloc/hipFree, no library
// routine that allocates.  All calls on one GPU share that GPU's array, so calls that
// overlap in time on one GPU (different streams or threads) race on it; the binning
// clears every counter and offset it relies on before use, so the contents left by an
// earlier call do not matter.
#include <stdio.h>

#include <mutex>

#include "wproj_tiled.h"

namespace {

constexpr int64_t kNoallocScratchBytes = 256ll << 20;  // 256 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (looked up on the first call on that device).
int scratch_for_current_device(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return WPROJ_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return WPROJ_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return WPROJ_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return WPROJ_OK;
}

}  // namespace

extern "C" {

int64_t wproj_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

int wproj_grid_noalloc(const wproj_kernels *k, int64_t nvis, const double *uvw, const void *vis,
                       const void *weight, const int64_t *image_offsets, void *grid,
                       double *weight_sum, int64_t *counters, void *stream) {
  if (!k) return wproj::set_error(WPROJ_EINVAL, "handle is NULL");
  const int64_t need = wproj_workspace_size(k, nvis);
  if (need < 0) return (int)need;
  if (need > kNoallocScratchBytes) {
    char buf[256];
    snprintf(buf, sizeof buf,
             "wproj_grid_noalloc: %lld visibilities need %lld bytes of scratch, the fixed "
             "per-GPU scratch holds %lld; use wproj_grid with a caller workspace",
             (long long)nvis, (long long)need, (long long)kNoallocScratchBytes);
    return wproj::set_error(WPROJ_EWORKSPACE, buf);
  }
  void *ws = nullptr;
  const int rc = scratch_for_current_device(&ws);
  if (rc == WPROJ_EHIP)
    return wproj::set_error(rc, "wproj_grid_noalloc: hipGetSymbolAddress of the scratch array failed");
  if (rc != WPROJ_OK) return wproj::set_error(rc, "wproj_grid_noalloc: device index beyond the supported 64");
  return wproj_grid(k, nvis, uvw, vis, weight, image_offsets, grid, weight_sum, counters, ws,
                    kNoallocScratchBytes, stream);
}

}  // extern "C"
