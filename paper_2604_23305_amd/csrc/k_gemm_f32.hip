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
// 32-channel tiles of the group: 96 accumulator registers (AGPRs) beside
// 120 VGPRs, and 60 KB of LDS, so two workgroups share a CU and one's
// barriers and epilogue overlap the other's MFMAs.
//
// Operand staging: depth chunks of 16 frequency bins go straight from
// global memory into a three-stage LDS ring with global_load_lds_dwordx4
// (no register staging), issued three chunks ahead of the MFMAs.  A stage
// holds the panel [128][16] and the three responses [3][64][16] in
// unpadded 64-byte rows; the 16-byte slot of bin quad q in row r is
// q ^ swz(r), which puts the 16-byte reads of 32 consecutive rows into
// distinct bank groups.  The DMA is issued from inline assembly: the
// compiler does not know that it writes LDS, so it does not wait for it
// before every LDS read of the other stages.
// Each wave reads a chunk in two halves (bin quads 2h + hs for lane half
// h) into two register sets, and every MFMA block runs with the LDS reads
// of the next half chunk placed between its MFMAs, so no LDS latency is
// exposed.  Between the two halves of chunk c each wave waits for its own
// LDS reads and for its DMAs of chunk c + 1, then passes the one barrier
// of the chunk: chunk c + 1 is visible and no wave reads stage c mod 3
// any more, which then takes chunk c + 3.
// The chunk loop is unrolled by the ring depth, so stage addresses are
// constants (LDS reads take immediate offsets), and DMA sources are scalar
// base addresses plus 32-bit lane offsets: the loop's only vector
// arithmetic besides the MFMAs is the dP^2 products, because vector
// instructions in the MFMA stream cost matrix-core cycles.
// Tile index -> workgroup mapping: block b runs on XCD b mod 8, so the
// channel groups of one time tile are given blocks of the same XCD and
// can share the panel tile in its L2.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gtod_internal.h"
#include "gemm_epilogue.h"
#include "philox.h"

namespace gtod {

namespace {

constexpr int MT = 128;   // rows per tile
constexpr int NT = 64;    // channels per tile
constexpr int KC = 16;    // frequency bins per chunk
// One stage: panel [MT][KC] then responses [3][NT][KC], rows unpadded.
constexpr int kStageFloats = MT * KC + 3 * NT * KC;

__device__ __forceinline__ int swz(int row) { return ((row >> 1) ^ (row >> 2)) & 3; }

__device__ __forceinline__ uint32_t lds_addr(float* p) {
  return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) float*)p;
}

// One wave-wide direct-to-LDS load: lane i moves the 16 bytes at base +
// voff (base wave-uniform, in scalar registers; voff the lane's byte
// offset) to LDS byte address m0 + 16 i (m0 uniform).  Advancing base is
// scalar arithmetic, so the loop spends no vector instructions on DMA
// addresses.  M0 is a reserved register the compiler does not save around
// inline assembly; no other code in this kernel uses it.  The s_nop covers
// the M0 write -> LDS DMA hazard.
__device__ __forceinline__ void dma16(const float* base, uint32_t voff, uint32_t m0) {
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, %2"
               :: "s"(m0), "v"(voff), "s"(base) : "memory", "m0");
#pragma clang diagnostic pop
}

// s_waitcnt with vmcnt = n (< 16) and the other counters left free.
#define GTOD_WAIT_VM(n) __builtin_amdgcn_s_waitcnt(0x3f70 | (n))

}  // namespace

__global__ __launch_bounds__(256, 2) void k_gemm_f32(GemmArgs a) {
  // An (empty) use of an accumulation register makes the compiler select
  // the MFMA form with its accumulators in AGPRs rather than VGPRs: 26.6
  // against 26.9 ms per c3 launch, same results.
  asm volatile("; accumulators in AGPRs %0" :: "a"(0.0f));
  const int b = blockIdx.x;
  const int xcd = b & 7;
  const int l = b >> 3;
  const int tt = (l / a.n_cg) * 8 + xcd;
  const int cg = l % a.n_cg;
  if (tt >= a.n_tt) return;
  const int64_t row0 = (int64_t)tt * MT;
  const int ch0 = cg * NT;

  // the ring; after the loop, stage 0 holds the epilogue slices of waves
  // 0 and 1, stage 1 those of waves 2 and 3
  static_assert(kStageFloats >= 2 * kEpiWaveFloats, "epilogue LDS");
  __shared__ float ring[3 * kStageFloats];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
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
  // Direct-to-LDS loads: one wave instruction moves 16 rows x 16 bins (64
  // lanes x 16 bytes) into 1 KB of LDS, lane i to offset 16 i.  Lane i
  // takes row i / 4 of its block and the bin quad (i % 4) ^ swz(row).
  // Sources are a wave-uniform base plus a 32-bit lane offset (a response
  // plane is below 4 GiB, which the spectral setup checks).
  const int lr = lane >> 2, lq = lane & 3;
  const int wave_s = __builtin_amdgcn_readfirstlane(wave);
  // panel: wave w moves rows 32 w + 16 q + lr, q = 0, 1, from the tile's rows
  const float* const gp = a.panel + row0 * Fp;
  uint32_t vp[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int r = wave * 32 + q * 16 + lr;
    vp[q] = (uint32_t)(4 * ((int64_t)r * Fp + 4 * (lq ^ swz(r))));
  }
  // responses: wave w moves blocks u = 3 w + q: matrix u / 4, channels
  // 16 (u % 4) + lr (clamped into the padded matrix; dead rows are unused)
  const float* gb[3];
  uint32_t vb[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int u = wave_s * 3 + q;
    const int m = u >> 2, r = ((u & 3) << 4) + lr;
    const int gch = min(ch0 + r, a.Kp - 1);
    gb[q] = a.B + m * KF;
    vb[q] = (uint32_t)(4 * ((int64_t)gch * Fp + 4 * (lq ^ swz(m * NT + r))));
  }
  // issue chunk `chunk` into the stage at LDS byte address ST
#define GTOD_ISSUE(ST, chunk)                                                 \
  {                                                                           \
    const int k0_ = (chunk) * KC;                                             \
    _Pragma("unroll") for (int q = 0; q < 2; ++q)                             \
      dma16(gp + k0_, vp[q], (ST) + 4u * ((wave_s * 32 + q * 16) * KC));     \
    _Pragma("unroll") for (int q = 0; q < 3; ++q) {                           \
      const int u = wave_s * 3 + q;                                           \
      dma16(gb[q] + k0_, vb[q],                                               \
            (ST) + 4u * (MT * KC + ((u >> 2) * NT + ((u & 3) << 4)) * KC));  \
    }                                                                         \
  }

  bool live[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) live[i] = (ch0 + i * 32) < a.K;

  const int n_chunks = a.Fp / KC;
  const int rd = wave * 32 + c;
  // ring address as a wave-uniform (scalar) value for M0
  const uint32_t lds0 = __builtin_amdgcn_readfirstlane(lds_addr(ring));
  // stage of chunk c is c mod 3; chunks 0-2 are issued before the loop
#pragma unroll
  for (int c0 = 0; c0 < 3; ++c0)
    if (c0 < n_chunks) GTOD_ISSUE(lds0 + 4u * kStageFloats * c0, c0)
  // NI live 32-channel tiles (uniform over the workgroup)
  auto run = [&](auto ni_c) {
    constexpr int NI = decltype(ni_c)::value;
    constexpr int NR = 1 + 3 * NI;   // LDS reads per half chunk
    typedef float4 Ops[NR];          // dP, then the responses (i, m)
    // the operands of half hs of a chunk: lane half h takes bin quad 2h + hs
    auto read_half = [&](int st, int hs, Ops& o) {
      const float* sD = ring + kStageFloats * st;
      const float* sB = sD + MT * KC;
      const int q = 2 * h + hs;
      o[0] = *reinterpret_cast<const float4*>(&sD[rd * KC + 4 * (q ^ swz(rd))]);
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const int rb = m * NT + i * 32 + c;
          o[1 + 3 * i + m] = *reinterpret_cast<const float4*>(&sB[rb * KC + 4 * (q ^ swz(rb))]);
        }
    };
    auto mfma_half = [&](const Ops& o) {
      float dsq[4];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) dsq[s4] = o[0][s4] * o[0][s4];
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          acc[0][i][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(o[1 + 3 * i][s4], o[0][s4], acc[0][i][0], 0, 0, 0);
          acc[1][i][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(o[2 + 3 * i][s4], o[0][s4], acc[1][i][0], 0, 0, 0);
          acc[2][i][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(o[3 + 3 * i][s4], dsq[s4], acc[2][i][0], 0, 0, 0);
        }
    };
    // the next half chunk's LDS reads go early in the MFMA block, one after
    // each MFMA, so that they have landed when the next block starts
    auto interleave = [&] {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 12 * NI - NR, 0);
    };
    // Between the halves of chunk kc each wave waits for its own LDS reads
    // and for its DMA of chunk kc + 1, then passes a barrier: chunk kc + 1
    // is visible and no wave still reads stage kc mod 3, which takes chunk
    // kc + 3.
    auto sync = [&](int kc, int st) {
      __builtin_amdgcn_sched_barrier(0);    // keep the wait after the MFMAs
      __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
      if (kc + 2 < n_chunks) { GTOD_WAIT_VM(5); } else { GTOD_WAIT_VM(0); }
      __builtin_amdgcn_s_barrier();
      if (kc + 3 < n_chunks) GTOD_ISSUE(lds0 + 4u * kStageFloats * st, kc + 3)
    };
    // Every MFMA block runs with the next half chunk's LDS reads between
    // its MFMAs, into the other register set.  st = kc mod 3 is a constant
    // in the main loop (unrolled by the ring depth), so LDS addresses are
    // a base register plus immediate offsets.
    Ops oa, ob;
    auto chunk = [&](int kc, int st) {
      __builtin_amdgcn_sched_barrier(0);    // one MFMA block per scheduling region
      read_half(st, 1, ob);
      mfma_half(oa);
      interleave();
      sync(kc, st);
      read_half(st == 2 ? 0 : st + 1, 0, oa);
      mfma_half(ob);
      interleave();
    };
    if (n_chunks > 2) { GTOD_WAIT_VM(10); }
    else if (n_chunks > 1) { GTOD_WAIT_VM(5); }
    else { GTOD_WAIT_VM(0); }
    __builtin_amdgcn_s_barrier();
    read_half(0, 0, oa);
    int kc = 0;
    for (; kc + 3 < n_chunks; kc += 3) {
      chunk(kc, 0);
      chunk(kc + 1, 1);
      chunk(kc + 2, 2);
    }
    for (; kc + 1 < n_chunks; ++kc) chunk(kc, kc % 3);
    read_half(kc % 3, 1, ob);
    mfma_half(oa);
    interleave();
    sync(kc, kc % 3);
    mfma_half(ob);
  };
  if (live[1]) run(std::integral_constant<int, 2>{});
  else run(std::integral_constant<int, 1>{});
  __syncthreads();   // every wave is done with the ring before the epilogue reuses it
  float* const spk = ring + (wave >> 1) * kStageFloats + (wave & 1) * kEpiWaveFloats;
  contraction_epilogue<2, 1, 3>(a, acc, spk, row0 + wave * 32, ch0, live);
}
#undef GTOD_WAIT_VM
#undef GTOD_ISSUE

void launch_gemm_f32(const GemmArgs& a0, hipStream_t s) {
  GemmArgs a = a0;
  a.n_cg = (a.Kp + NT - 1) / NT;
  const int64_t n_tt8 = round_up(a.n_tt, 8);
  const int64_t blocks = n_tt8 * a.n_cg;
  hipLaunchKernelGGL(k_gemm_f32, dim3((unsigned)blocks), dim3(256), 0, s, a);
}

}  // namespace gtod
