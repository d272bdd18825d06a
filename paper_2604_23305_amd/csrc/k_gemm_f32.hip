// Filterbank contraction on the FP32 matrix cores, with the photon-noise
// epilogue (sections 2.5-2.7).
//
// For a tile of 128 rows (consecutive samples of one pixel) x 64 channels
// the kernel accumulates, over the frequency axis,
//   C0 = dP B0,   C1 = dP B1',   C2 = dP^2 B2
// with v_mfma_f32_32x32x2_f32.  The MFMA "A" operand is the channel-major
// response (rows = channels) and "B" the deviation panel transposed, so the
// 32x32 accumulator of a lane holds one time sample and 16 channels: the
// epilogue stores runs of 32 consecutive samples per channel, matching the
// [pixel][channel][time] output layout.
// Epilogue: P_KID = c0 + C0, NEP^2 = c1 + C1 + C2, sigma = sqrt(NEP^2 f/2),
// P_wn = sigma z with z from Philox counter (t, k, p, 0).
//
// Workgroup: 4 waves along time, each 32 samples x both (or the one live)
// 32-channel tiles of the group: 96 accumulator registers and 232 VGPRs in
// all, so two workgroups share a CU and one's barriers and epilogue overlap
// the other's MFMAs.  Operands are staged through LDS in depth chunks of 32
// frequency bins (row pitch 36 floats: the 16-byte reads of 8 or 16
// consecutive lanes fall in distinct banks), loaded into registers two
// chunks ahead; inside a chunk lane l takes bins 16*(l/32) + 4*hs .. +3 for
// the four quarter-steps hs.  Tile index -> workgroup mapping keeps the
// channel groups of one time tile on the same XCD so the panel tile is
// fetched once into that XCD's L2.
#include <hip/hip_runtime.h>

#include "gtod_internal.h"
#include "gemm_epilogue.h"
#include "philox.h"

namespace gtod {

namespace {

constexpr int MT = 128;   // rows per tile
constexpr int NT = 64;    // channels per tile
constexpr int KC = 32;    // frequency bins per LDS chunk
constexpr int LP = KC + 4;  // padded LDS row (floats)

}  // namespace

__global__ __launch_bounds__(256, 2) void k_gemm_f32(GemmArgs a) {
  const int b = blockIdx.x;
  const int xcd = b & 7;
  const int l = b >> 3;
  const int tt = (l / a.n_cg) * 8 + xcd;
  const int cg = l % a.n_cg;
  if (tt >= a.n_tt) return;
  const int64_t row0 = (int64_t)tt * MT;
  const int ch0 = cg * NT;

  constexpr int kStage = MT * LP + 3 * NT * LP;
  constexpr int kSmem = kStage > 4 * kEpiWaveFloats ? kStage : 4 * kEpiWaveFloats;
  __shared__ float smem[kSmem];
  float* sD = smem;
  float* sB = smem + MT * LP;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int h = lane >> 5, c = lane & 31;

  // wave w multiplies time tile w (32 rows) by every live channel tile of
  // the group, so all waves of a group do the same work
  f32x16 acc[3][2][1];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[m][i][0][e] = 0.f;

  // global -> register staging: panel chunk 128 rows x 16 bins = 512 float4
  // (2 per thread); response chunk 3 x 64 x 16 = 768 float4 (3 per thread)
  const int64_t Fp = a.Fp;
  const int64_t KF = (int64_t)a.Kp * Fp;
  // two staging register sets: chunk c lives in set (c & 1) from its load,
  // issued two chunks ahead, until it is stored into LDS
  float4 rdA0, rdA1, rdA2, rdA3, rbA0, rbA1, rbA2, rbA3, rbA4, rbA5;
  float4 rdB0, rdB1, rdB2, rdB3, rbB0, rbB1, rbB2, rbB3, rbB4, rbB5;
#define GTOD_LD_D(q, dst, k0n)                                               \
  {                                                                          \
    const int idx = tid + (q) * 256;                                         \
    dst = *reinterpret_cast<const float4*>(a.panel + (row0 + (idx >> 3)) * Fp + \
                                           (k0n) + 4 * (idx & 7));           \
  }
#define GTOD_LD_B(q, dst, k0n)                                               \
  {                                                                          \
    const int idx = tid + (q) * 256;                                         \
    const int m = idx >> 9, rem = idx & 511;                                 \
    const int gch = ch0 + (rem >> 3);                                        \
    dst = gch < a.Kp ? *reinterpret_cast<const float4*>(                     \
                           a.B + m * KF + (int64_t)gch * Fp + (k0n) + 4 * (rem & 7)) \
                     : make_float4(0.f, 0.f, 0.f, 0.f);                      \
  }
#define GTOD_ST_D(q, src)                                                    \
  {                                                                          \
    const int idx = tid + (q) * 256;                                         \
    *reinterpret_cast<float4*>(&sD[(idx >> 3) * LP + 4 * (idx & 7)]) = src;  \
  }
#define GTOD_ST_B(q, src)                                                    \
  {                                                                          \
    const int idx = tid + (q) * 256;                                         \
    const int m = idx >> 9, rem = idx & 511;                                 \
    *reinterpret_cast<float4*>(&sB[(m * NT + (rem >> 3)) * LP + 4 * (rem & 7)]) = src; \
  }
#define GTOD_LOAD_CHUNK(S, k0n)                                              \
  GTOD_LD_D(0, rd##S##0, k0n) GTOD_LD_D(1, rd##S##1, k0n)                    \
  GTOD_LD_D(2, rd##S##2, k0n) GTOD_LD_D(3, rd##S##3, k0n)                    \
  GTOD_LD_B(0, rb##S##0, k0n) GTOD_LD_B(1, rb##S##1, k0n)                    \
  GTOD_LD_B(2, rb##S##2, k0n) GTOD_LD_B(3, rb##S##3, k0n)                    \
  GTOD_LD_B(4, rb##S##4, k0n) GTOD_LD_B(5, rb##S##5, k0n)
#define GTOD_STORE_CHUNK(S)                                                  \
  GTOD_ST_D(0, rd##S##0) GTOD_ST_D(1, rd##S##1) GTOD_ST_D(2, rd##S##2)       \
  GTOD_ST_D(3, rd##S##3) GTOD_ST_B(0, rb##S##0) GTOD_ST_B(1, rb##S##1)       \
  GTOD_ST_B(2, rb##S##2) GTOD_ST_B(3, rb##S##3) GTOD_ST_B(4, rb##S##4)       \
  GTOD_ST_B(5, rb##S##5)

  // channel tiles of the group that hold at least one real channel
  bool live[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) live[i] = (ch0 + i * 32) < a.K;

// one chunk: four quarter-steps of 4 bins; lane takes bins 16*h + 4*hs + (0..3)
#define GTOD_COMPUTE_CHUNK \
_Pragma("unroll") \
    for (int hs = 0; hs < 4; ++hs) { \
      const float4 dv = *reinterpret_cast<const float4*>(&sD[(wave * 32 + c) * LP + 16 * h + 4 * hs]); \
      float dsq[4]; \
_Pragma("unroll") \
      for (int s4 = 0; s4 < 4; ++s4) dsq[s4] = dv[s4] * dv[s4]; \
_Pragma("unroll") \
      for (int i = 0; i < 2; ++i) { \
        if (live[i]) { \
          float4 bv[3]; \
_Pragma("unroll") \
          for (int m = 0; m < 3; ++m) \
            bv[m] = *reinterpret_cast<const float4*>( \
                &sB[(m * NT + i * 32 + c) * LP + 16 * h + 4 * hs]); \
_Pragma("unroll") \
          for (int s4 = 0; s4 < 4; ++s4) { \
            acc[0][i][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(bv[0][s4], dv[s4], acc[0][i][0], 0, 0, 0); \
            acc[1][i][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(bv[1][s4], dv[s4], acc[1][i][0], 0, 0, 0); \
            acc[2][i][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(bv[2][s4], dsq[s4], acc[2][i][0], 0, 0, 0); \
          } \
        } \
      } \
    }

  const int n_chunks = a.Fp / KC;
  GTOD_LOAD_CHUNK(A, 0)
  if (n_chunks > 1) { GTOD_LOAD_CHUNK(B, KC) }
  for (int kc = 0; kc < n_chunks; kc += 2) {
    __syncthreads();
    GTOD_STORE_CHUNK(A)
    __syncthreads();
    if (kc + 2 < n_chunks) { GTOD_LOAD_CHUNK(A, (kc + 2) * KC) }
    GTOD_COMPUTE_CHUNK
    if (kc + 1 < n_chunks) {
      __syncthreads();
      GTOD_STORE_CHUNK(B)
      __syncthreads();
      if (kc + 3 < n_chunks) { GTOD_LOAD_CHUNK(B, (kc + 3) * KC) }
      GTOD_COMPUTE_CHUNK
    }
  }

  contraction_epilogue<2, 1>(a, acc, smem, row0 + wave * 32, ch0, live);
}
#undef GTOD_LD_D
#undef GTOD_LD_B
#undef GTOD_ST_D
#undef GTOD_ST_B
#undef GTOD_LD_D
#undef GTOD_LD_B
#undef GTOD_ST_D
#undef GTOD_ST_B
#undef GTOD_LOAD_CHUNK
#undef GTOD_STORE_CHUNK
#undef GTOD_COMPUTE_CHUNK

void launch_gemm_f32(const GemmArgs& a0, hipStream_t s) {
  GemmArgs a = a0;
  a.n_cg = (a.Kp + NT - 1) / NT;
  const int64_t n_tt8 = round_up(a.n_tt, 8);
  const int64_t blocks = n_tt8 * a.n_cg;
  hipLaunchKernelGGL(k_gemm_f32, dim3((unsigned)blocks), dim3(256), 0, s, a);
}

}  // namespace gtod
