// 1/f noise by the method of Timmer and Koenig (section 2.6), added into
// the TOD.
//
// Series (p, k) of N = 2^q samples (first t_total kept): bins j = 1..N/2-1
// get X_j = c_j (z_re + i z_im), c_j = sqrt(A_k f_j^-alpha_k N f_s / 4) / N,
// f_j = j f_s / N, with (z_re, z_im) the Box-Muller pair of Philox counter
// (j, k, p, 1); DC and Nyquist are zero.  x = inverse real DFT of X.
//
// The real inverse transform of length N is done as one complex inverse
// DFT of length M = N/2 on
//   Z_k = (X_k + conj X_{M-k}) + i e^{2 pi i k/N} (X_k - conj X_{M-k}),
// whose output z_m = x_{2m} + i x_{2m+1}.  The complex DFT uses the
// four-step split M = M1 * M2 (M2 <= 4096), k = k1 + M1 k2, m = m1 M2 + m2:
//   pass 1, per (series, k1): length-M2 DFT over k2 of Z (generated on the
//     fly, so the stride costs nothing), times e^{2 pi i k1 m2 / M}, stored
//     contiguous in m2;
//   pass 2, per (series, block of B2 consecutive m2): length-M1 DFTs over
//     k1, read and written as runs of B2 consecutive m2.
// With M1 = 1 pass 1 writes the output directly.  Each DFT runs in LDS as
// radix-2 decimation in time on bit-reversed input, twiddles from a table
// of e^{2 pi i m / L} evaluated with sincospi on exact arguments.
#include <hip/hip_runtime.h>

#include "gtod_internal.h"
#include "philox.h"

namespace gtod {

namespace {

constexpr int kLdsC = 4096;   // complex values per workgroup

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ float2 twiddle(uint32_t num, int lg_den) {
  // e^{2 pi i num / 2^lg_den}, num < 2^lg_den <= 2^24
  const float x = ldexpf((float)num, 1 - lg_den);  // 2 num / den, exact
  float s, c;
  sincospif(x, &s, &c);
  return make_float2(c, s);
}

__device__ __forceinline__ uint32_t bitrev(uint32_t v, int bits) {
  return bits == 0 ? 0u : (__brev(v) >> (32 - bits));
}

// In-place inverse DFTs of `batch` contiguous transforms of length 2^lg
// held in bit-reversed order in buf; tw holds e^{2 pi i m / L}, m < L/2.
__device__ void lds_dit(float2* buf, const float2* tw, int lg, int batch) {
  const int L = 1 << lg;
  const int half_total = (L >> 1) * batch;
  for (int s = 1; s <= lg; ++s) {
    const int half = 1 << (s - 1);
    const int tstride = L >> s;     // table step for this stage
    for (int bf = threadIdx.x; bf < half_total; bf += blockDim.x) {
      const int tr = bf / (L >> 1);
      const int b = bf % (L >> 1);
      const int pos = b % half;
      const int i = tr * L + (b / half) * 2 * half + pos;
      const int jx = i + half;
      const float2 u = buf[i];
      const float2 v = cmul(buf[jx], tw[pos * tstride]);
      buf[i] = make_float2(u.x + v.x, u.y + v.y);
      buf[jx] = make_float2(u.x - v.x, u.y - v.y);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ float2 spectrum_bin(const PinkArgs& a, int64_t j,
                                               int k, int p, float sc,
                                               float alpha) {
  if (j <= 0 || j >= a.M) return make_float2(0.f, 0.f);
  const u32x4 o = philox10(u32x4{(uint32_t)j, (uint32_t)k, (uint32_t)p, 1u},
                           a.key0, a.key1);
  float zc, zs;
  box_muller(o.x, o.y, &zc, &zs);
  const float f = (float)j * (float)(a.fs / (double)a.N);
  const float cj = sc * powf(f, -0.5f * alpha);
  return make_float2(cj * zc, cj * zs);
}

__device__ __forceinline__ void store_out(const PinkArgs& a, int64_t series,
                                          int64_t m, float2 z) {
  const int64_t t = 2 * m;
  float* dst = a.tod + series * a.out_ld;
  if (t < a.t_total) {
    if (a.accumulate) dst[t] += z.x; else dst[t] = z.x;
  }
  if (t + 1 < a.t_total) {
    if (a.accumulate) dst[t + 1] += z.y; else dst[t + 1] = z.y;
  }
}

}  // namespace

__global__ __launch_bounds__(256) void k_pink_pass1(PinkArgs a) {
  __shared__ float2 buf[kLdsC];
  __shared__ float2 tw[kLdsC / 2];
  const int k1 = blockIdx.x;
  const int sl = blockIdx.y;
  const int64_t series = a.s0 + sl;
  const int p = (int)(series / a.K);
  const int k = (int)(series % a.K);
  const float sc = a.scale[k];
  const float alpha = a.alpha[k];
  const int M2 = a.M2;
  const int lgN = a.lgM1 + a.lgM2 + 1;

  for (int m = threadIdx.x; m < M2 / 2; m += blockDim.x) tw[m] = twiddle(m, a.lgM2);
  for (int k2 = threadIdx.x; k2 < M2; k2 += blockDim.x) {
    const int64_t kk = k1 + (int64_t)a.M1 * k2;
    const float2 xa = spectrum_bin(a, kk, k, p, sc, alpha);
    const float2 xb = spectrum_bin(a, a.M - kk, k, p, sc, alpha);
    // E = X_k + conj(X_{M-k}), O = X_k - conj(X_{M-k})
    const float2 ev = make_float2(xa.x + xb.x, xa.y - xb.y);
    const float2 od = make_float2(xa.x - xb.x, xa.y + xb.y);
    const float2 w = twiddle((uint32_t)kk, lgN);
    const float2 wo = cmul(w, od);
    buf[bitrev(k2, a.lgM2)] = make_float2(ev.x - wo.y, ev.y + wo.x);
  }
  __syncthreads();
  lds_dit(buf, tw, a.lgM2, 1);
  if (a.M1 == 1) {
    for (int m2 = threadIdx.x; m2 < M2; m2 += blockDim.x) store_out(a, series, m2, buf[m2]);
  } else {
    float2* dst = a.scratch + ((int64_t)sl * a.M1 + k1) * M2;
    const int lgM = a.lgM1 + a.lgM2;
    for (int m2 = threadIdx.x; m2 < M2; m2 += blockDim.x) {
      const uint32_t e = (uint32_t)(((uint64_t)k1 * m2) & ((1ull << lgM) - 1));
      dst[m2] = cmul(buf[m2], twiddle(e, lgM));
    }
  }
}

__global__ __launch_bounds__(256) void k_pink_pass2(PinkArgs a) {
  __shared__ float2 buf[kLdsC];
  __shared__ float2 tw[kLdsC / 2];
  const int nb = blockIdx.x;
  const int sl = blockIdx.y;
  const int64_t series = a.s0 + sl;
  const int M1 = a.M1, M2 = a.M2, B2 = a.B2;
  const int m20 = nb * B2;
  for (int m = threadIdx.x; m < M1 / 2; m += blockDim.x) tw[m] = twiddle(m, a.lgM1);
  const float2* src = a.scratch + (int64_t)sl * M1 * M2;
  for (int idx = threadIdx.x; idx < M1 * B2; idx += blockDim.x) {
    const int k1 = idx / B2, bb = idx % B2;
    buf[bb * M1 + bitrev(k1, a.lgM1)] = src[(int64_t)k1 * M2 + m20 + bb];
  }
  __syncthreads();
  lds_dit(buf, tw, a.lgM1, B2);
  for (int idx = threadIdx.x; idx < M1 * B2; idx += blockDim.x) {
    const int m1 = idx / B2, bb = idx % B2;
    store_out(a, series, (int64_t)m1 * M2 + m20 + bb, buf[bb * M1 + m1]);
  }
}

void launch_pink_pass1(const PinkArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_pink_pass1, dim3(a.M1, a.n_series), dim3(256), 0, s, a);
}

void launch_pink_pass2(const PinkArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_pink_pass2, dim3(a.M2 / a.B2, a.n_series), dim3(256), 0,
                     s, a);
}

__global__ void k_philox(const uint32_t* ctr, uint32_t* out, int64_t n,
                         uint32_t k0, uint32_t k1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const u32x4 o = philox10(u32x4{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2],
                                 ctr[4 * i + 3]}, k0, k1);
  out[4 * i] = o.x;
  out[4 * i + 1] = o.y;
  out[4 * i + 2] = o.z;
  out[4 * i + 3] = o.w;
}

void launch_philox(const uint32_t* ctr, uint32_t* out, int64_t n, uint32_t k0,
                   uint32_t k1, hipStream_t s) {
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_philox, dim3((unsigned)blocks), dim3(256), 0, s, ctr, out,
                     n, k0, k1);
}

}  // namespace gtod
