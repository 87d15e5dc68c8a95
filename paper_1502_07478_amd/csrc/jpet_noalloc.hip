// jpet_mlem_iterate_noalloc: the MLEM iterations of jpet_mlem_iterate with the workspace in a
// file-scope device array instead of a caller allocation, for callers that cannot allocate device
// memory (code under graph capture, serving loops, harnesses that forbid allocation).
//
// The array is part of the library's device code object: each GPU the library runs on holds its
// own copy, at its own address, until the process ends.  Host code never passes the array's name
// to a kernel (in host code it is a host-side stand-in, not a device address); the device address
// is looked up once per device with hipGetSymbolAddress and kept.
#include <mutex>

#include "jpet_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)JPET_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "the workspace is 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of scratch per device (null: not looked up yet)

// The current device's copy of scratch: looked up on the first call on that device, with that
// device current, and kept.
int scratch_of_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return jpet::record_hip_failure(e);
  if (dev < 0 || dev >= kMaxDevices) return JPET_ENOTSUP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return jpet::record_hip_failure(e);
    if (!p) return JPET_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return JPET_OK;
}

}  // namespace

extern "C" int jpet_mlem_iterate_noalloc(const jpet_geometry* g, const float* events, int64_t n, const float* s,
                                         float* rho, int32_t n_iter, uint32_t flags, jpet_stats* stats,
                                         void* stream) {
  // every call prepares its events (the array holds whatever the last call on this device left),
  // with the planned pass: flags must be 0
  if (flags != 0u || n_iter < 0 || !rho || (n > 0 && !events)) return JPET_EINVAL;
  size_t need = 0;
  int rc = jpet_mlem_workspace_size(g, n, &need);  // validates the geometry, n and the plan
  if (rc) return rc;
  if (need > kScratchBytes) return JPET_EWORKSPACE;
  void* ws = nullptr;
  if ((rc = scratch_of_current_device(&ws))) return rc;
  // the workspace's counters and accumulators are cleared by kernels inside this call
  return jpet_mlem_iterate(g, events, n, s, rho, n_iter, ws, kScratchBytes, flags, stats, stream);
}
