// labs_noalloc.hip -- labs_walks for callers that cannot allocate device
// memory (code under stream capture, tight serving loops, harnesses that
// forbid allocation): the visited tables live in a fixed device array that
// the library holds on every GPU it runs on until the process ends.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <mutex>

#include "labs.h"
#include "labs_internal.h"

namespace {

constexpr uint64_t kScratchBytes = LABS_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");

// The visited tables of labs_walks_noalloc.  In host code this name is only a
// handle for the symbol lookup below: device addresses come from
// hipGetSymbolAddress, one per device.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {nullptr};

// Device address of `scratch` on the current device (looked up once per device).
hipError_t scratch_on_current_device(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" int32_t labs_walks_noalloc(const uint64_t *starts, int32_t L, int64_t n_walks,
                                      int64_t walk_len, uint64_t seed, const labs_walk_out *out,
                                      const labs_plan *plan, void *stream) {
  // One walk's table must fit the scratch; more walks run in chunks of as
  // many tables as it holds (labs_walks' chunking).
  uint64_t one = 0;
  int32_t rc = labs_walks_min_workspace_bytes(L, walk_len, plan, &one);
  if (rc != LABS_OK) return rc;
  if (one > kScratchBytes)
    return lsaw::set_error(LABS_EINVAL,
                           "one walk's visited table needs %llu bytes; the fixed scratch of "
                           "labs_walks_noalloc holds %llu (use labs_walks with a workspace)",
                           (unsigned long long)one, (unsigned long long)kScratchBytes);
  // argument errors (and n_walks == 0) before any device call
  if (n_walks <= 0 || !out) return labs_walks(starts, L, n_walks, walk_len, seed, out, nullptr, 0, plan, stream);
  void *ws = nullptr;
  const hipError_t e = scratch_on_current_device(&ws);
  if (e != hipSuccess)
    return lsaw::set_error(LABS_EDEVICE, "scratch lookup: %s", hipGetErrorString(e));
  return labs_walks(starts, L, n_walks, walk_len, seed, out, ws, kScratchBytes, plan, stream);
}
