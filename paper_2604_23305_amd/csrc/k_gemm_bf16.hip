// Filterbank contraction with split BF16 operands on the matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation), same epilogue as the FP32
// kernel.
//
// Every FP32 operand x is carried as x_hi + x_lo with x_hi = bf16(x) and
// x_lo = bf16(x - x_hi) (round to nearest even), which keeps about 16
// significant bits.  Per tile pair the kernel accumulates
//   C0  = B0lo dPhi + B0hi dPlo + B0hi dPhi
//   C1' = B1lo dPhi + B1hi dPlo + B1hi dPhi + (B2hi 2^-p) (dP^2)hi
// (the lo x lo products and the low half of the small dP^2 term are below
// the FP32 rounding of the result).  The dP^2 B2 term of NEP^2 carries
// 2^2p in panel units; scaling its response by 2^-p (exact, done by the
// setup) lets it share the C1 accumulator, so NEP^2 = c1 + C1' 2^-p.  The deviations dP are a
// few percent of P, so the 16-bit operands give about 1e-7 relative error
// on P_KID.  The response halves come pre-split and pre-tiled from the
// spectral setup; dP is split in registers after it is read from LDS.
//
// Workgroup: 8 waves, 256 rows x 128 channels, one per CU; wave w owns
// rows 64 (w % 4) .. + 63 (two 32-row tiles) and channels 64 (w / 4) ..
// + 63 (two 32-channel tiles): 8 accumulator tiles (128 registers), so one
// LDS read of an operand feeds two MFMA tiles and an MFMA step carries 28
// MFMAs per wave.  Each panel row is read from memory once per 128
// channels and each response bin once per 256 rows: 36 KB per step for
// 224 MFMAs.
//
// Operand staging: steps of 16 frequency bins go straight from global
// memory into a four-stage LDS ring with global_load_lds_dwordx4 (no
// register staging), three steps ahead of the MFMAs.  A stage is the panel
// [256][16] FP32 in 64-byte rows (16-byte slot of bin quad q in row r at
// q ^ swz(r)) and the five response planes B0hi B0lo B1hi B1lo B2hi, each
// [128][16] BF16 in 32-byte rows (16-byte half h of row r at h ^ swb(r)):
// 36 KB, 144 KB for the ring.  Both layouts put the 16-byte reads of each
// group of 16 lanes on distinct banks of the 256-byte-wide LDS.  The
// responses of a stage are stored in that exact layout, contiguously, by
// the setup (launch_tile_split_responses), so their 20 DMAs each move 1 KB
// of consecutive bytes; the panel's 16 DMAs move 16 rows each.  Waves
// 0-3 issue 5 DMAs per stage, waves 4-7 issue 4.  The DMA is issued from
// inline assembly; before step s is read each wave waits until at most 8
// of its DMAs (at most those of steps s + 1 and s + 2) are in flight, and
// a barrier makes every wave's part of step s visible; the stage that step
// s + 3 overwrites was last read before that barrier.
//
// The step loop is unrolled by the ring depth, so each step's stage is a
// constant and its LDS reads take immediate offsets; DMA sources are
// scalar base addresses plus 32-bit lane offsets.  The split of dP is the
// only vector arithmetic besides the MFMAs.
//
// Tile index -> workgroup mapping: block b runs on XCD b mod 8, so the
// channel groups of one time tile are given blocks of the same XCD and can
// share the panel tile in its L2.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gtod_internal.h"
#include "gemm_epilogue.h"
#include "philox.h"

namespace gtod {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr int MT = 256;   // rows per workgroup tile
constexpr int NT = 128;   // channels per workgroup tile
constexpr int KC = 16;    // bins per stage = one MFMA step
constexpr int kWaves = 8;
constexpr int kPanelBytes = MT * KC * 4;              // panel part of a stage
constexpr int kPlaneBytes = NT * KC * 2;              // one response plane
constexpr int kRespBytes = 5 * kPlaneBytes;           // responses of a stage
constexpr int kStageBytes = kPanelBytes + kRespBytes;
constexpr int kStages = 4;
constexpr int kRespBlocks = kRespBytes / 1024;        // 20 DMAs of 1 KB
static_assert(kStages * kStageBytes >= kWaves * kEpiWaveFloats * 4, "epilogue LDS");
static_assert((kStages & (kStages - 1)) == 0, "stage index by mask");

// panel rows (64 bytes, four 16-byte slots)
__device__ __forceinline__ int swz(int row) { return ((row >> 1) ^ (row >> 2)) & 3; }
// response rows (32 bytes, two 16-byte halves): rows r and r + 8 lie 256
// bytes apart, on the same banks, so their halves are swapped
__device__ __forceinline__ int swb(int row) { return (row >> 3) & 1; }

__device__ __forceinline__ uint32_t lds_addr(void* p) {
  return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) char*)p;
}

// One wave-wide direct-to-LDS load: lane i moves the 16 bytes at base +
// voff (base wave-uniform, in scalar registers; voff the lane's byte
// offset) to LDS byte address m0 + 16 i (m0 uniform).  Advancing base is
// scalar arithmetic.  M0 is a reserved register the compiler does not
// save around inline assembly; no other code in this kernel uses it.  The
// s_nop covers the M0 write -> LDS DMA hazard.
__device__ __forceinline__ void dma16(const void* base, uint32_t voff, uint32_t m0) {
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, %2"
               :: "s"(m0), "v"(voff), "s"(base) : "memory", "m0");
#pragma clang diagnostic pop
}

// s_waitcnt with vmcnt = n (< 16) and the other counters left free.
#define GTOD_WAIT_VM(n) __builtin_amdgcn_s_waitcnt(0x3f70 | (n))

}  // namespace

// Tiled split responses: for channel group g (NT channels) and step s (KC
// bins), plane m (B0hi B0lo B1hi B1lo B2hi) as [NT][KC] BF16 rows with the
// in-row swizzle applied, i.e. the LDS image of the stage, contiguous:
// Bt[g][s][m][r][slot] = B_m[g NT + r][s KC + 8 (slot ^ swb(r)) .. + 7],
// zero for channels past the padded matrix; plane B2hi is stored times
// 2^-p (b2_scale), so that it multiplies (dP^2)hi directly.
size_t split_tiled_bytes(int Kp, int Fp) {
  const size_t n_cg = (size_t)(Kp + NT - 1) / NT;
  return n_cg * (size_t)(Fp / KC) * kRespBytes;
}

__global__ void k_tile_split_responses(const uint16_t* __restrict__ Bh,
                                       const uint16_t* __restrict__ Bl,
                                       uint16_t* __restrict__ Bt, int Kp, int Fp,
                                       float b2_scale, int64_t n_slots) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slots) return;
  // i = (((g * n_steps + s) * 5 + m) * NT + r) * 2 + slot
  const int slot = (int)(i & 1);
  const int r = (int)((i >> 1) % NT);
  const int64_t q = (i >> 1) / NT;
  const int m = (int)(q % 5);
  const int64_t gs = q / 5;
  const int n_steps = Fp / KC;
  const int s = (int)(gs % n_steps);
  const int g = (int)(gs / n_steps);
  const int ch = g * NT + r;
  uint4 v = make_uint4(0u, 0u, 0u, 0u);
  if (ch < Kp) {
    const uint16_t* src = ((m & 1) ? Bl : Bh) + (int64_t)(m >> 1) * Kp * Fp +
                          (int64_t)ch * Fp + s * KC + 8 * (slot ^ swb(r));
    v = *reinterpret_cast<const uint4*>(src);
    if (m == 4) {
      // B2 hi times 2^-p: a power of two, exact on BF16 values in range
      uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float lo = __builtin_bit_cast(float, w[k] << 16) * b2_scale;
        const float hi = __builtin_bit_cast(float, w[k] & 0xffff0000u) * b2_scale;
        w[k] = (__builtin_bit_cast(uint32_t, lo) >> 16) |
               (__builtin_bit_cast(uint32_t, hi) & 0xffff0000u);
      }
      v = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
  reinterpret_cast<uint4*>(Bt)[i] = v;
}

void launch_tile_split_responses(const uint16_t* Bh, const uint16_t* Bl, uint16_t* Bt,
                                 int Kp, int Fp, float b2_scale, hipStream_t s) {
  const int64_t n_slots = (int64_t)(split_tiled_bytes(Kp, Fp) / 16);
  hipLaunchKernelGGL(k_tile_split_responses, dim3((unsigned)((n_slots + 255) / 256)),
                     dim3(256), 0, s, Bh, Bl, Bt, Kp, Fp, b2_scale, n_slots);
}

__global__ __launch_bounds__(512, 1) void k_gemm_bf16(GemmArgs a) {
  const int b = blockIdx.x;
  const int xcd = b & 7;
  const int l = b >> 3;
  const int tt = (l / a.n_cg) * 8 + xcd;
  const int cg = l % a.n_cg;
  const int n_tt = (a.n_tt + 1) >> 1;   // 256-row tiles of the chunk
  if (tt >= n_tt) return;
  const int64_t row0 = (int64_t)tt * MT;
  const int ch0 = cg * NT;
  // rows of the chunk's panel; a last tile of 128 rows reads its other
  // half from clamped addresses and stores none of it
  const int64_t n_rows = (int64_t)a.n_pix * a.Tpad;

  __shared__ __attribute__((aligned(16))) char ring[kStages * kStageBytes];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int h = lane >> 5, c = lane & 31;
  const int rw = wave & 3, cw = wave >> 2;   // row and channel quarter / half

  // acc[0]: C0, acc[1]: C1'; [channel tile][row tile]
  f32x16 acc[2][2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[m][i][j][e] = 0.f;

  const int64_t Fp = a.Fp;
  const int n_steps = a.Fp / KC;
  const int wave_s = __builtin_amdgcn_readfirstlane(wave);
  // DMA sources are a wave-uniform base plus a 32-bit lane offset (the
  // spectral setup keeps 256 panel rows below 4 GiB).
  // panel DMA: wave w moves blocks w and w + 8, rows 16 block + lane / 4,
  // lane taking bin quad (lane % 4) ^ swz(row)
  const float* const gp = a.panel + row0 * Fp;
  uint32_t vp[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int r = (wave + 8 * q) * 16 + (lane >> 2);
    const int64_t gr = min(row0 + r, n_rows - 1);
    vp[q] = (uint32_t)(4 * ((gr - row0) * Fp + 4 * ((lane & 3) ^ swz(r))));
  }
  // response DMA: wave w moves the 1 KB blocks w, w + 8 and (waves 0-3)
  // w + 16 of the stage's contiguous image
  const int n_rb = wave_s < kRespBlocks - 2 * kWaves ? 3 : 2;
  const char* const gt = reinterpret_cast<const char*>(a.Bt) +
                         (size_t)cg * n_steps * kRespBytes + wave_s * 1024;
  const uint32_t vt = (uint32_t)lane * 16u;
  const uint32_t lds0 = __builtin_amdgcn_readfirstlane(lds_addr(ring));
  // issue step `st` into the stage at LDS byte address S
#define GTOD_ISSUE(S, st)                                                     \
  {                                                                           \
    const int k0_ = (st) * KC;                                                \
    _Pragma("unroll") for (int q = 0; q < 2; ++q)                             \
      dma16(gp + k0_, vp[q], (S) + (uint32_t)((wave_s + 8 * q) * 1024));      \
    const char* t_ = gt + (size_t)(st) * kRespBytes;                          \
    _Pragma("unroll") for (int q = 0; q < 3; ++q)                             \
      if (q < n_rb)                                                           \
        dma16(t_ + q * 8 * 1024, vt,                                          \
              (S) + (uint32_t)(kPanelBytes + (wave_s + 8 * q) * 1024));       \
  }

  bool live[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) live[i] = (ch0 + cw * 64 + i * 32) < a.K;

  GTOD_ISSUE(lds0, 0)
  if (n_steps > 1) GTOD_ISSUE(lds0 + kStageBytes, 1)
  if (n_steps > 2) GTOD_ISSUE(lds0 + 2 * kStageBytes, 2)
  // NI live 32-channel tiles (uniform over the wave; every wave runs the
  // same steps and barriers)
  auto run = [&](auto ni_c) {
    constexpr int NI = decltype(ni_c)::value;
    // step s from stage sr = s mod 4; a constant in the main loop below
    // (unrolled by the ring depth), so LDS addresses are immediates
    auto step = [&](int s, int sr) {
      if (s + 2 < n_steps) { GTOD_WAIT_VM(8); }
      else if (s + 1 < n_steps) { GTOD_WAIT_VM(4); }
      else { GTOD_WAIT_VM(0); }
      __builtin_amdgcn_s_barrier();
      if (s + 3 < n_steps)
        GTOD_ISSUE(lds0 + (uint32_t)(kStageBytes * ((sr + 3) & (kStages - 1))), s + 3)
      const char* sP = ring + kStageBytes * sr;
      const char* sB = sP + kPanelBytes;
      // dP of this lane's sample in row tile j: bins 8 h .. 8 h + 7
      float4 dv[2][2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int rd = rw * 64 + j * 32 + c;
#pragma unroll
        for (int hs = 0; hs < 2; ++hs)
          dv[j][hs] = *reinterpret_cast<const float4*>(
              sP + rd * (KC * 4) + 16 * ((2 * h + hs) ^ swz(rd)));
      }
      // planes 0 B0hi, 1 B0lo, 2 B1hi, 3 B1lo, 4 B2hi 2^-p; bins 8 h ..
      // 8 h + 7 of this lane's channel
      bf16x8 bp[NI][5];
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const int rb = cw * 64 + i * 32 + c;
        const int ob = rb * (KC * 2) + 16 * (h ^ swb(rb));
#pragma unroll
        for (int pl = 0; pl < 5; ++pl)
          bp[i][pl] = *reinterpret_cast<const bf16x8*>(sB + pl * kPlaneBytes + ob);
      }
      // split dP into hi, lo and (dP^2) hi, two bins per conversion
      bf16x8 dh[2], dl[2], dq[2];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          const f32x2 x = {dv[j][e >> 2][e & 3], dv[j][e >> 2][(e & 3) + 1]};
          const bf16x2 hi = __builtin_convertvector(x, bf16x2);
          const uint32_t hb = __builtin_bit_cast(uint32_t, hi);
          const f32x2 hf = {__builtin_bit_cast(float, hb << 16),
                            __builtin_bit_cast(float, hb & 0xffff0000u)};
          const bf16x2 lo = __builtin_convertvector(x - hf, bf16x2);
          const bf16x2 sq = __builtin_convertvector(x * x, bf16x2);
          dh[j][e] = hi[0];
          dh[j][e + 1] = hi[1];
          dl[j][e] = lo[0];
          dl[j][e + 1] = lo[1];
          dq[j][e] = sq[0];
          dq[j][e + 1] = sq[1];
        }
      // 7 products per tile pair, ordered so that consecutive MFMAs write
      // different accumulators
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[0][i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bp[i][1], dh[j], acc[0][i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[1][i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bp[i][3], dh[j], acc[1][i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[0][i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bp[i][0], dl[j], acc[0][i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[1][i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bp[i][2], dl[j], acc[1][i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[0][i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bp[i][0], dh[j], acc[0][i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[1][i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bp[i][2], dh[j], acc[1][i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[1][i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bp[i][4], dq[j], acc[1][i][j], 0, 0, 0);
    };
    int s = 0;
    for (; s + kStages <= n_steps; s += kStages) {
      step(s, 0);
      step(s + 1, 1);
      step(s + 2, 2);
      step(s + 3, 3);
    }
    for (; s < n_steps; ++s) step(s, s & (kStages - 1));
  };
  if (live[1]) run(std::integral_constant<int, 2>{});
  else run(std::integral_constant<int, 1>{});
  __syncthreads();   // every wave is done with the ring before the epilogue reuses it
  float* const spk = reinterpret_cast<float*>(ring) + wave * kEpiWaveFloats;
  contraction_epilogue<2, 2, 2>(a, acc, spk, row0 + rw * 64, ch0 + cw * 64, live);
}
#undef GTOD_WAIT_VM
#undef GTOD_ISSUE

void launch_gemm_bf16(const GemmArgs& a0, hipStream_t s) {
  GemmArgs a = a0;
  a.n_cg = (a.Kp + NT - 1) / NT;
  const int64_t n_tt8 = round_up((a.n_tt + 1) / 2, 8);
  const int64_t blocks = n_tt8 * a.n_cg;
  hipLaunchKernelGGL(k_gemm_bf16, dim3((unsigned)blocks), dim3(kWaves * 64), 0, s, a);
}

}  // namespace gtod
