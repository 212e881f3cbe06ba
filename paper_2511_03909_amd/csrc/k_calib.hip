// Measurement helpers: a plain device copy (achievable HBM bandwidth, and the
// reference for scaling the FETCH_SIZE / WRITE_SIZE counters) and the rate of
// conflict-free LDS atomic adds of the three widths the kernels could use.
// Neither is part of the transform.

#include <hip/hip_runtime.h>

#include <cstdio>

#include "wect.h"
#include "wect_internal.h"

namespace {

// 16-byte loads and stores, four per thread in flight (each thread copies
// elements i, i + s, i + 2s, i + 3s of a grid-stride step of 4s), then the
// remainder one at a time; a tail of fewer than 16 bytes is copied byte by
// byte by the first thread.
__global__ __launch_bounds__(256) void k_copy(uint4* __restrict__ dst, const uint4* __restrict__ src, size_t n16,
                                              unsigned char* dtail, const unsigned char* stail, int ntail) {
  const size_t s = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * s < n16; i += 4 * s) {
    const uint4 a = src[i], b = src[i + s], c = src[i + 2 * s], d = src[i + 3 * s];
    dst[i] = a;
    dst[i + s] = b;
    dst[i + 2 * s] = c;
    dst[i + 3 * s] = d;
  }
  for (; i < n16; i += s) dst[i] = src[i];
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int k = 0; k < ntail; ++k) dtail[k] = stail[k];
}

// Every thread adds `reps` times into its lane's column of a [64][64] LDS
// table (row = (wave + r) mod 64, column = lane): the 64 lanes of one atomic
// hit 64 consecutive words, as the histogram kernels do.  Wavefront 0 then
// writes row 0 to out[block][64] so that the adds are kept.
template <typename V>
__global__ __launch_bounds__(1024) void k_lds_atomics(V* out, int reps) {
  __shared__ V tab[64 * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) tab[i] = V(0);
  __syncthreads();
  const V one = V(1);
  for (int r = 0; r < reps; ++r) {
    V* a = &tab[((wave + r) & 63) * 64 + lane];
    __hip_atomic_fetch_add(a, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __syncthreads();
  if (wave == 0) out[(size_t)blockIdx.x * 64 + lane] = tab[lane];
}

void set_error(const char* what, hipError_t e) {
  char msg[160];
  snprintf(msg, sizeof(msg), "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
  wect::set_last_error(msg);
}

}  // namespace

extern "C" {

wect_status wect_calib_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (bytes == 0) return WECT_OK;
  if (!dst || !src || (reinterpret_cast<uintptr_t>(dst) & 15) || (reinterpret_cast<uintptr_t>(src) & 15))
    return WECT_ERR_ARG;
  const size_t n16 = bytes / 16;
  const int ntail = (int)(bytes - n16 * 16);
  size_t blocks = (n16 + 1023) / 1024;  // about four elements per thread
  if (blocks > 16384) blocks = 16384;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream, (uint4*)dst,
                     (const uint4*)src, n16, (unsigned char*)dst + n16 * 16, (const unsigned char*)src + n16 * 16,
                     ntail);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) {
    set_error("copy kernel", e);
    return WECT_ERR_DEVICE;
  }
  return WECT_OK;
}

wect_status wect_calib_lds_atomics(int32_t kind, int32_t blocks, int32_t reps, void* out, void* hip_stream) {
  if (kind < 0 || kind > 2 || blocks < 1 || reps < 1 || !out) return WECT_ERR_ARG;
  hipStream_t s = (hipStream_t)hip_stream;
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_lds_atomics<uint32_t>, dim3(blocks), dim3(1024), 0, s, (uint32_t*)out, reps); break;
    case 1: hipLaunchKernelGGL(k_lds_atomics<uint64_t>, dim3(blocks), dim3(1024), 0, s, (uint64_t*)out, reps); break;
    default: hipLaunchKernelGGL(k_lds_atomics<float>, dim3(blocks), dim3(1024), 0, s, (float*)out, reps); break;
  }
  if (hipError_t e = hipGetLastError(); e != hipSuccess) {
    set_error("LDS atomics kernel", e);
    return WECT_ERR_DEVICE;
  }
  return WECT_OK;
}

}  // extern "C"
