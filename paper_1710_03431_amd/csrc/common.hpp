// Shared device/host helpers of libaqt: HIP error handling, device buffers,
// 64-lane wavefront reductions and scans.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "aqt.h"

namespace aqt {

constexpr int kWave = 64;

// ---------------------------------------------------------------- host -----
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // Grows to at least `n` bytes; contents are not preserved on growth.
  hipError_t reserve(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, n ? n : 1);
    if (e == hipSuccess) bytes = n;
    else p = nullptr;
    return e;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------- device ---
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Inclusive prefix sum over the 64 lanes (Hillis-Steele with shuffles).
__device__ __forceinline__ double wave_inclusive_scan(double v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    double u = __shfl_up(v, o, kWave);
    if (lane >= o) v += u;
  }
  return v;
}

__device__ __forceinline__ int first_set_lane(uint64_t mask) {
  return mask ? __ffsll(static_cast<unsigned long long>(mask)) - 1 : -1;
}

__device__ __forceinline__ int last_set_lane(uint64_t mask) {
  return mask ? 63 - __clzll(static_cast<unsigned long long>(mask)) : -1;
}

}  // namespace aqt
