// Epilogue shared by the contraction kernels: reference terms, photon-noise
// sigma, Philox white noise and the store into [pixel][channel][time].
// Accumulators are in panel units (powers times 2^p); C2 holds dP^2 and
// carries 2^2p.
//
// Each wave owns NI x NJ accumulator tiles of 32 channels x 32 samples;
// tile (i, j) starts at channel ch_base + 32 i and row row_base + 32 j.
// With NP = 3 the products are C0, C1 and C2 as above; with NP = 2 the
// kernel has already added C2 2^-p into C1.  A tile is first written to the wave's own LDS slice
// (kEpiWaveFloats floats at spk, distinct for each wave) with
// static register indices, then read back by a compact loop in which lane
// l handles sample (l mod 32) of channel rows 2s + l/32: stores are runs of
// 32 consecutive samples.  The slice belongs to one wave, whose LDS
// accesses complete in order, so the waves of a workgroup go through the
// epilogue without barriers (the kernel has one before it, after the last
// read of its operand ring).
#pragma once

#include <hip/hip_runtime.h>

#include "gtod_internal.h"
#include "philox.h"

namespace gtod {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kEpiPitch = 33;
constexpr int kEpiWaveFloats = 2 * 32 * kEpiPitch;

template <int NI, int NJ, int NP>
__device__ __forceinline__ void contraction_epilogue(
    const GemmArgs& a, f32x16 (&acc)[NP][NI][NJ], float* spk,
    int64_t row_base, int ch_base, const bool (&live)[NI]) {
  static_assert(NP == 2 || NP == 3, "two or three products");
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5, c = lane & 31;
  float* sn2 = spk + 32 * kEpiPitch;
#pragma unroll
  for (int i = 0; i < NI; ++i) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int64_t row = row_base + j * 32 + c;
      const int pl = (int)(row / a.Tpad);
      const int tl = (int)(row % a.Tpad);
      const bool valid = live[i] && pl < a.n_pix && tl < a.Tc;
      const int p = a.p0 + pl;
      const int64_t t = a.t0 + tl;
      const int chb = ch_base + i * 32;
      const int64_t off0 = ((int64_t)p * a.K + chb + h) * a.out_ld + (t - a.out_t0);
      // when adding into the TOD, its 16 values are loaded first, so that
      // they are in flight together and during the LDS staging below
      float prev[16];
#pragma unroll
      for (int s = 0; s < 16; ++s)
        prev[s] = (a.accumulate && valid && chb + 2 * s + h < a.K)
                      ? a.tod[off0 + 2 * s * a.out_ld] : 0.f;
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int chl = 8 * (e >> 2) + 4 * h + (e & 3);
        spk[chl * kEpiPitch + c] = acc[0][i][j][e];
        if constexpr (NP == 3)
          sn2[chl * kEpiPitch + c] = acc[1][i][j][e] + acc[NP - 1][i][j][e] * a.pinv_f;
        else
          sn2[chl * kEpiPitch + c] = acc[1][i][j][e];
      }
      __builtin_amdgcn_wave_barrier();
      if (!valid) continue;
      for (int s = 0; s < 16; ++s) {
        const int chl = 2 * s + h;
        const int ch = chb + chl;
        if (ch >= a.K) break;
        // P_KID = c0 + C0 2^-p; NEP^2 = c1 + (C1 + C2 2^-p) 2^-p, in FP64
        // because 2^-2p lies below the FP32 normal range
        const double pkd = a.c0[ch] + (double)spk[chl * kEpiPitch + c] * a.pinv;
        const float pk = (float)pkd;
        const double n2 = a.c1[ch] + (double)sn2[chl * kEpiPitch + c] * a.pinv;
        // sigma to FP32 rounding (its tolerance is 1e-5)
        const float sg = sqrtf((float)(fmax(n2, 0.0) * (double)a.fs_half));
        float wn = 0.f;
        if (a.photon) {
          const u32x4 o = philox10(u32x4{(uint32_t)t, (uint32_t)ch, (uint32_t)(a.pix0 + p), 0u},
                                   a.key0, a.key1);
          wn = sg * box_muller_cos(o.x, o.y);
        }
        // Kelvin: (P - a_k) / b_k with the offset taken in FP64
        const float v = a.kelvin
            ? (float)(((pkd - a.kel_a[ch]) + (double)wn) * a.kel_ib[ch])
            : pk + wn;
        const int64_t off = off0 + 2 * s * a.out_ld;
        a.tod[off] = a.accumulate ? prev[s] + v : v;
        if (a.p_kid) a.p_kid[off] = pk;
        if (a.sigma) a.sigma[off] = sg;
      }
    }
  }
}

}  // namespace gtod
