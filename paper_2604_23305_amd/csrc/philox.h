// Device-side Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the
// uniform / Box-Muller maps the noise kernels use.
//
// One round maps (x0, x1, x2, x3) under key (k0, k1) to
//   (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, lo(M0*x0))
// and the key advances by the Weyl constants between rounds.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gtod {

struct u32x4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox10(u32x4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
  constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
  // each 64-bit product gives both halves in one v_mad_u64_u32 (separate
  // high and low 32-bit multiplies would take two instructions)
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kM0 * c.x;
    const uint64_t p1 = (uint64_t)kM1 * c.z;
    c = u32x4{(uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
              (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0};
    k0 += kW0;
    k1 += kW1;
  }
  return c;
}

// ((o >> 9) + 1/2) * 2^-23: exact in FP32, strictly inside (0, 1).
__device__ __forceinline__ float u01(uint32_t o) {
  return (float)(o >> 9) * 1.1920928955078125e-07f + 5.9604644775390625e-08f;
}

// Box-Muller from the hardware transcendentals (about one ulp each): log2
// of u0 (normal, inside (0, 1)), the square root of -2 ln u0 (inside
// (0, 34]) and the cosine and sine of u1 revolutions, i.e. of the angle
// 2 pi u1.  The noise tolerances (the photon-noise term is about 4e-4 of
// the power; the 1/f series is held to 1e-5 of its rms) are orders of
// magnitude above these errors.
__device__ __forceinline__ float bm_radius(uint32_t o0) {
  // -2 ln u = -2 ln(2) log2(u)
  return __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u01(o0)));
}

// (r cos 2 pi u1, r sin 2 pi u1)
__device__ __forceinline__ void box_muller(uint32_t o0, uint32_t o1,
                                           float* zc, float* zs) {
  const float r = bm_radius(o0);
  const float u1 = u01(o1);
  *zc = r * __builtin_amdgcn_cosf(u1);
  *zs = r * __builtin_amdgcn_sinf(u1);
}

// r cos 2 pi u1 only (the white noise)
__device__ __forceinline__ float box_muller_cos(uint32_t o0, uint32_t o1) {
  return bm_radius(o0) * __builtin_amdgcn_cosf(u01(o1));
}

}  // namespace gtod
