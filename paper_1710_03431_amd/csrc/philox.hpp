// Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11),
// written from its published definition: ten rounds of two 64x64->128-bit
// multiplications with the Philox multipliers, the key advanced by the two
// Weyl constants between rounds.
//
// Draw map of the trajectory engine: key = (seed, instance_id), counter =
// (trajectory id, draw >> 2, 0, 0), word draw & 3, mapped to a double in (0, 1)
// as ((x >> 12) + 0.5) * 2^-52 (exact in binary64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace aqt {

struct Philox4 {
  uint64_t w[4];
};

__host__ __device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
#if defined(__HIP_DEVICE_COMPILE__)
  lo = a * b;
  hi = __umul64hi(a, b);
#else
  unsigned __int128 p = static_cast<unsigned __int128>(a) * b;
  lo = static_cast<uint64_t>(p);
  hi = static_cast<uint64_t>(p >> 64);
#endif
}

__host__ __device__ __forceinline__ Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                           uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
  constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll 1
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kW0;
      k1 += kW1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(kM0, c0, hi0, lo0);
    mulhilo64(kM1, c2, hi1, lo1);
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return Philox4{{c0, c1, c2, c3}};
}

__host__ __device__ __forceinline__ double uniform_open01(uint64_t x) {
  return (static_cast<double>(x >> 12) + 0.5) * 0x1.0p-52;
}

// Uniform draw number `idx` of trajectory `traj`.
__host__ __device__ __forceinline__ double draw_uniform(uint64_t seed, uint64_t iid, uint64_t traj, uint64_t idx) {
  const Philox4 r = philox4x64_10(traj, idx >> 2, 0, 0, seed, iid);
  const unsigned k = static_cast<unsigned>(idx & 3);
  // select instead of indexing so the words stay in registers
  const uint64_t x = k == 0 ? r.w[0] : (k == 1 ? r.w[1] : (k == 2 ? r.w[2] : r.w[3]));
  return uniform_open01(x);
}

}  // namespace aqt
