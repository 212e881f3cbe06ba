// wect_forward_noalloc: the forward with its workspace in a static device
// array, for callers that cannot allocate device memory.
//
// The forward is planned without the per-voxel records of the cubical
// forward, so its workspace (partial histograms of blocks that share a group,
// their sums, the per-block maxima of |w| for float weights) stays small; it
// lives here in a
// file-scope device array of kScratchBytes.  Its device address is looked up
// once per device, with that device current, and kept per device: in host
// code the array's name is only a host-side stand-in.  Every call on one GPU
// shares that GPU's array; the forward writes every part of it that it later
// reads, so nothing needs clearing between calls.

#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>
#include <vector>

#include "wect.h"
#include "wect_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB per device

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device: the address of that device's scratch

// Address of the scratch array on the current device (looked up on the first
// call on that device).  Returns nullptr and the HIP error on failure.
void* scratch_address(hipError_t* err) {
  int dev = 0;
  if (hipError_t e = hipGetDevice(&dev); e != hipSuccess) {
    *err = e;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)); e != hipSuccess) {
      *err = e;
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *err = hipSuccess;
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

wect_status wect_forward_noalloc(const wect_complex* c, const wect_grid* g, void* out, void* hip_stream) {
  if (!c || !g) return WECT_ERR_ARG;
  const size_t need = wect::workspace_bytes_lean(c, g);
  hipError_t err = hipSuccess;
  void* ws = scratch_address(&err);
  if (!ws) {
    char msg[160];
    snprintf(msg, sizeof(msg), "scratch address: %s (%d)", hipGetErrorString(err), (int)err);
    wect::set_last_error(msg);
    return WECT_ERR_DEVICE;
  }
  if (need > kScratchBytes) {
    char msg[160];
    snprintf(msg, sizeof(msg), "request needs %zu bytes of workspace, above the static scratch of %zu bytes", need,
             kScratchBytes);
    wect::set_last_error(msg);
    return WECT_ERR_WORKSPACE;
  }
  return wect::forward_lean(c, g, out, ws, kScratchBytes, hip_stream);
}

}  // extern "C"
