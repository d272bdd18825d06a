// Filterbank contraction with split BF16 operands on the matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation), same epilogue as the FP32
// kernel.
//
// Every FP32 operand x is carried as x_hi + x_lo with x_hi = bf16(x) and
// x_lo = bf16(x - x_hi) (round to nearest even), which keeps about 16
// significant bits.  Per tile pair the kernel accumulates
//   C0 = B0lo dPhi + B0hi dPlo + B0hi dPhi
//   C1 = B1lo dPhi + B1hi dPlo + B1hi dPhi
//   C2 = B2hi (dP^2)hi
// (the lo x lo products and the low half of the small dP^2 term are below
// the FP32 rounding of the result).  The deviations dP are a few percent
// of P, so the 16-bit operands give about 1e-7 relative error on P_KID.
// dP is split once per workgroup, when a chunk is staged into LDS; the
// response halves come pre-split from the spectral setup.
// Workgroup: 128 samples x 64 channels, 4 waves along time, each 32
// samples x both 32-channel tiles (96 accumulator registers, 234 VGPRs in
// all), so two workgroups share a CU and hide each other's barriers and
// epilogues.  Each wave stages its own 32 panel rows, so that part of LDS
// needs no barrier; the response tile, shared by the four waves, is double
// buffered, which leaves one barrier per chunk.  The 13 LDS reads of an
// MFMA step are issued before its 14 MFMAs; the loop is instantiated for
// one and for two live channel tiles so that no branch separates them.
// LDS rows are unpadded 64-byte rows with an XOR swizzle of their 16-byte
// chunks (64 KB per workgroup).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gtod_internal.h"
#include "gemm_epilogue.h"
#include "philox.h"

namespace gtod {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int MT = 128;
constexpr int NT = 64;
constexpr int KC = 32;        // bins per chunk = 2 MFMA steps of 16
// LDS rows are KC bf16 (64 bytes), unpadded; the 16-byte chunk q of row r
// sits at slot q ^ swz(r), so that the 16-byte reads of 16 consecutive
// rows at one chunk hit 16 distinct bank groups.
__device__ __forceinline__ int swz(int row) { return ((row >> 1) ^ (row >> 2)) & 3; }

}  // namespace

__global__ __launch_bounds__(256, 2) void k_gemm_bf16(GemmArgs a) {
  const int b = blockIdx.x;
  const int xcd = b & 7;
  const int l = b >> 3;
  const int tt = (l / a.n_cg) * 8 + xcd;
  const int cg = l % a.n_cg;
  if (tt >= a.n_tt) return;
  const int64_t row0 = (int64_t)tt * MT;
  const int ch0 = cg * NT;

  // sD: [3][MT][KC] dP hi, dP lo, (dP^2) hi, each wave's 32 rows written
  // and read by that wave only; sB: two buffers of [5][NT][KC] B0h B0l B1h
  // B1l B2h, shared by the four waves
  constexpr int kBBuf = 5 * NT * KC;   // bf16 per response buffer
  constexpr int kStage = (3 * MT * KC + 2 * kBBuf) / 2;
  constexpr int kSmem = kStage > 4 * kEpiWaveFloats ? kStage : 4 * kEpiWaveFloats;
  __shared__ float smem[kSmem];
  __bf16* sD = reinterpret_cast<__bf16*>(smem);
  __bf16* sB0 = sD + 3 * MT * KC;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  // wave w: rows 32 w .. 32 w + 31 x both 32-channel tiles of the group
  const int h = lane >> 5, c = lane & 31;

  f32x16 acc[3][2][1];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[m][i][0][e] = 0.f;

  const int64_t Fp = a.Fp;
  const int64_t KF = (int64_t)a.Kp * Fp;
  // panel chunk: each wave loads its own 32 rows x 32 floats = 256 float4,
  // 4 per lane; response chunk: 5 x 64 x 32 bf16 = 1280 x 16 bytes, 5 per
  // thread
  float4 rd0, rd1, rd2, rd3;
  uint4 rb0, rb1, rb2, rb3, rb4;
#define GTOD_LD_D(q, dst, k0n)                                               \
  {                                                                          \
    const int idx = lane + (q) * 64;                                         \
    dst = *reinterpret_cast<const float4*>(                                  \
        a.panel + (row0 + wave * 32 + (idx >> 3)) * Fp + (k0n) + 4 * (idx & 7)); \
  }
#define GTOD_LD_B(q, dst, k0n)                                               \
  {                                                                          \
    const int idx = tid + (q) * 256;                                         \
    const int mm = idx >> 8, rem = idx & 255;                                \
    const int gch = ch0 + (rem >> 2);                                        \
    /* mm: 0 B0h, 1 B0l, 2 B1h, 3 B1l, 4 B2h */                              \
    const uint16_t* base = (mm & 1) ? a.Bl : a.Bh;                           \
    dst = gch < a.Kp ? *reinterpret_cast<const uint4*>(                      \
                           base + (mm >> 1) * KF + (int64_t)gch * Fp + (k0n) + 8 * (rem & 3)) \
                     : make_uint4(0u, 0u, 0u, 0u);                           \
  }
// split dP into hi, lo and (dP^2) hi while staging it into LDS
#define GTOD_ST_D(q, src)                                                    \
  {                                                                          \
    const int idx = wave * 256 + lane + (q) * 64;                            \
    const float x_[4] = {src.x, src.y, src.z, src.w};                        \
    bf16x4 hi_, lo_, sq_;                                                    \
    _Pragma("unroll") for (int e = 0; e < 4; ++e) {                         \
      hi_[e] = (__bf16)x_[e];                                                \
      lo_[e] = (__bf16)(x_[e] - (float)hi_[e]);                              \
      sq_[e] = (__bf16)(x_[e] * x_[e]);                                      \
    }                                                                        \
    const int r_ = idx >> 3, q_ = (idx & 7) >> 1;                            \
    const int o_ = r_ * KC + 8 * (q_ ^ swz(r_)) + 4 * (idx & 1);             \
    *reinterpret_cast<bf16x4*>(&sD[o_]) = hi_;                               \
    *reinterpret_cast<bf16x4*>(&sD[MT * KC + o_]) = lo_;                     \
    *reinterpret_cast<bf16x4*>(&sD[2 * MT * KC + o_]) = sq_;                 \
  }
#define GTOD_ST_B(q, src)                                                    \
  {                                                                          \
    const int idx = tid + (q) * 256;                                         \
    const int mm = idx >> 8, rem = idx & 255;                                \
    const int rb_ = rem >> 2;                                                \
    *reinterpret_cast<uint4*>(&sBw[(mm * NT + rb_) * KC + 8 * ((rem & 3) ^ swz(rb_))]) = src; \
  }
#define GTOD_LOAD_CHUNK(k0n)                                                 \
  GTOD_LD_D(0, rd0, k0n) GTOD_LD_D(1, rd1, k0n) GTOD_LD_D(2, rd2, k0n)       \
  GTOD_LD_D(3, rd3, k0n)                                                     \
  GTOD_LD_B(0, rb0, k0n) GTOD_LD_B(1, rb1, k0n) GTOD_LD_B(2, rb2, k0n)       \
  GTOD_LD_B(3, rb3, k0n) GTOD_LD_B(4, rb4, k0n)
#define GTOD_STORE_CHUNK                                                     \
  GTOD_ST_D(0, rd0) GTOD_ST_D(1, rd1) GTOD_ST_D(2, rd2) GTOD_ST_D(3, rd3)   \
  GTOD_ST_B(0, rb0) GTOD_ST_B(1, rb1)                                       \
  GTOD_ST_B(2, rb2) GTOD_ST_B(3, rb3) GTOD_ST_B(4, rb4)

  bool live[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) live[i] = (ch0 + i * 32) < a.K;

  GTOD_LOAD_CHUNK(0)
  // NI live 32-channel tiles (uniform over the workgroup): the LDS reads
  // of an MFMA step are all issued before its MFMAs.  One barrier per
  // chunk: a wave's dP rows are its own (its earlier reads of them have
  // completed before its MFMAs used them), and the response buffer a chunk
  // fills was last read two chunks before, ahead of the previous barrier.
  auto run = [&](auto ni_c) {
    constexpr int NI = decltype(ni_c)::value;
    int buf = 0;
    for (int k0 = 0; k0 < a.Fp; k0 += KC, buf ^= 1) {
      __bf16* sBw = sB0 + buf * kBBuf;
      GTOD_STORE_CHUNK
      __syncthreads();
      if (k0 + KC < a.Fp) { GTOD_LOAD_CHUNK(k0 + KC) }
      const __bf16* sB = sBw;
#pragma unroll
      for (int s = 0; s < KC / 16; ++s) {
        const int rd = wave * 32 + c;
        const int o = rd * KC + 8 * ((2 * s + h) ^ swz(rd));
        const bf16x8 dh = *reinterpret_cast<const bf16x8*>(&sD[o]);
        const bf16x8 dl = *reinterpret_cast<const bf16x8*>(&sD[MT * KC + o]);
        const bf16x8 ds = *reinterpret_cast<const bf16x8*>(&sD[2 * MT * KC + o]);
        // planes: 0 B0hi, 1 B0lo, 2 B1hi, 3 B1lo, 4 B2hi
        bf16x8 bp[NI][5];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          const int rb = i * 32 + c;
          const int ob = rb * KC + 8 * ((2 * s + h) ^ swz(rb));
#pragma unroll
          for (int pl = 0; pl < 5; ++pl)
            bp[i][pl] = *reinterpret_cast<const bf16x8*>(&sB[pl * NT * KC + ob]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          acc[0][i][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bp[i][1], dh, acc[0][i][0], 0, 0, 0);
          acc[0][i][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bp[i][0], dl, acc[0][i][0], 0, 0, 0);
          acc[0][i][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bp[i][0], dh, acc[0][i][0], 0, 0, 0);
          acc[1][i][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bp[i][3], dh, acc[1][i][0], 0, 0, 0);
          acc[1][i][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bp[i][2], dl, acc[1][i][0], 0, 0, 0);
          acc[1][i][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bp[i][2], dh, acc[1][i][0], 0, 0, 0);
          acc[2][i][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bp[i][4], ds, acc[2][i][0], 0, 0, 0);
        }
      }
    }
  };
  if (live[1]) run(std::integral_constant<int, 2>{});
  else run(std::integral_constant<int, 1>{});

  contraction_epilogue<2, 1>(a, acc, smem + wave * kEpiWaveFloats, row0 + wave * 32, ch0, live);
}
#undef GTOD_LD_D
#undef GTOD_LD_B
#undef GTOD_ST_D
#undef GTOD_ST_B
#undef GTOD_LOAD_CHUNK
#undef GTOD_STORE_CHUNK

void launch_gemm_bf16(const GemmArgs& a0, hipStream_t s) {
  GemmArgs a = a0;
  a.n_cg = (a.Kp + NT - 1) / NT;
  const int64_t n_tt8 = round_up(a.n_tt, 8);
  const int64_t blocks = n_tt8 * a.n_cg;
  hipLaunchKernelGGL(k_gemm_bf16, dim3((unsigned)blocks), dim3(256), 0, s, a);
}

}  // namespace gtod
