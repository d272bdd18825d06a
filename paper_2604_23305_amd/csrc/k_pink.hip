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
//   pass 1, per (series, column set closed under k -> M-k): the spectrum
//     bins of those columns drawn once, Z built in place, length-M2 DFTs
//     over k2 (the stride costs nothing as nothing is read), times
//     e^{2 pi i k1 m2 / M}, stored contiguous in m2;
//   pass 2, per (series, block of B2 consecutive m2): length-M1 DFTs over
//     k1, read and written as runs of B2 consecutive m2.
// With M1 = 1 pass 1 writes the output directly.  Each DFT runs in LDS as
// radix-2 decimation in frequency (pass 1, natural input) or in time (pass
// 2, bit-reversed input).  Twiddles come from per-stage tables in global
// memory (stage with half-length h reads entries h - 1 .. 2h - 2, holding
// e^{2 pi i pos / 2h}), so that the lanes of a stage read consecutive
// entries; the tables are evaluated with sincospi on exact arguments once
// per batch.  All index arithmetic is shifts and masks (lengths are powers
// of two).
#include <hip/hip_runtime.h>

#include <algorithm>

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

// In-place inverse DFTs of 2^lgb contiguous transforms of length 2^lg
// held in bit-reversed order in buf; tws is the per-stage twiddle table.
__device__ void lds_dit(float2* buf, const float2* __restrict__ tws, int lg,
                        int lgb) {
  if (lg == 0) return;
  const int hl = lg - 1;                  // log2 of the butterflies per transform
  const int half_total = 1 << (hl + lgb);
  for (int s = 1; s <= lg; ++s) {
    const int half = 1 << (s - 1);
    const float2* tw = tws + (half - 1);
    for (int bf = threadIdx.x; bf < half_total; bf += blockDim.x) {
      const int tr = bf >> hl;
      const int b = bf & ((1 << hl) - 1);
      const int pos = b & (half - 1);
      const int i = (tr << lg) + ((b >> (s - 1)) << s) + pos;
      const int jx = i + half;
      const float2 u = buf[i];
      const float2 v = cmul(buf[jx], tw[pos]);
      buf[i] = make_float2(u.x + v.x, u.y + v.y);
      buf[jx] = make_float2(u.x - v.x, u.y - v.y);
    }
    __syncthreads();
  }
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

// In-place inverse DFT of one transform of length 2^lg, natural-order
// input, bit-reversed output (decimation in frequency).
__device__ void lds_dif(float2* buf, const float2* __restrict__ tws, int lg) {
  if (lg == 0) return;
  const int half_total = 1 << (lg - 1);
  for (int s = lg; s >= 1; --s) {
    const int half = 1 << (s - 1);
    const float2* tw = tws + (half - 1);
    for (int bf = threadIdx.x; bf < half_total; bf += blockDim.x) {
      const int pos = bf & (half - 1);
      const int i = ((bf >> (s - 1)) << s) + pos;
      const int jx = i + half;
      const float2 u = buf[i];
      const float2 v = buf[jx];
      buf[i] = make_float2(u.x + v.x, u.y + v.y);
      buf[jx] = cmul(make_float2(u.x - v.x, u.y - v.y), tw[pos]);
    }
    __syncthreads();
  }
}

// Pass 1 works on a set of columns closed under k -> M - k: column 0,
// column M1/2, or the pair (k1, M1 - k1).  Each spectral bin X_j is drawn
// once; every Z_k is built from X_k and X_{M-k} held in LDS, two at a time
// (e^{2 pi i (M-k)/N} = -conj e^{2 pi i k/N}).
// Per-stage twiddle tables for transforms of length 2^lg: entry m lies in
// the stage of half-length h = 2^floor(log2(m + 1)) and holds
// e^{2 pi i (m - h + 1) / 2h}.
__global__ void k_pink_tables(float2* tw1, int lg1, float2* tw2, int lg2) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int n1 = (1 << lg1) - 1, n2 = (1 << lg2) - 1;
  if (m < n1 || m < n2) {
    const int lh = 31 - __clz(m + 1);      // log2 h
    const uint32_t pos = (uint32_t)(m + 1 - (1 << lh));
    const float2 v = twiddle(pos, lh + 1);
    if (m < n1) tw1[m] = v;
    if (m < n2) tw2[m] = v;
  }
}

__global__ __launch_bounds__(256) void k_pink_pass1(PinkArgs a) {
  __shared__ float2 buf[2][kLdsC];
  const int grp = blockIdx.x;
  const int sl = blockIdx.y;
  const int64_t series = a.s0 + sl;
  const int p = (int)(series / a.K);
  const int k = (int)(series % a.K);
  const float sc = a.scale[k];
  const float halpha = -0.5f * a.alpha[k];
  const float fstep = (float)(a.fs / (double)a.N);
  const int M1 = a.M1, M2 = a.M2;
  const int lgN = a.lgM1 + a.lgM2 + 1;
  // columns of this group: kind 0 = {0}, 1 = {M1/2}, 2 = {k1, M1 - k1}
  int kind, col[2], ncol;
  if (grp == 0) { kind = 0; col[0] = 0; ncol = 1; }
  else if (grp == 1) { kind = 1; col[0] = M1 / 2; ncol = 1; }
  else { kind = 2; col[0] = grp - 1; col[1] = M1 - (grp - 1); ncol = 2; }
  col[1] = (ncol == 2) ? col[1] : col[0];

  // draw X for every bin of the group's columns (natural order)
  for (int idx = threadIdx.x; idx < (ncol << a.lgM2); idx += blockDim.x) {
    const int c = idx >> a.lgM2, k2 = idx & (M2 - 1);
    const int64_t j = col[c] + (int64_t)M1 * k2;
    float2 x = make_float2(0.f, 0.f);
    if (j > 0 && j < a.M) {
      const u32x4 o = philox10(u32x4{(uint32_t)j, (uint32_t)k, (uint32_t)(a.pix0 + p), 1u},
                               a.key0, a.key1);
      float zc, zs;
      box_muller(o.x, o.y, &zc, &zs);
      const float cj = sc * exp2f(halpha * log2f((float)j * fstep));
      x = make_float2(cj * zc, cj * zs);
    }
    buf[c][k2] = x;
  }
  __syncthreads();
  // Z in place, one pair (k, M - k) per work item
  const int U = kind == 0 ? M2 / 2 + 1 : (kind == 1 ? M2 / 2 : M2);
  for (int u = threadIdx.x; u < U; u += blockDim.x) {
    int ca, ra, cb, rb;   // (column slot, row) of k and of M - k
    bool nyq = false;
    if (kind == 0) {
      ca = 0; ra = (u == M2 / 2 && M2 > 1) ? M2 / 2 : u;
      if (u == 0 || M2 == 1) { nyq = true; cb = 0; rb = 0; }
      else { cb = 0; rb = M2 - ra; }
    } else if (kind == 1) {
      ca = 0; ra = u; cb = 0; rb = M2 - 1 - u;
    } else {
      ca = 0; ra = u; cb = 1; rb = M2 - 1 - u;
    }
    const float2 xa = buf[ca][ra];
    const float2 xb = nyq ? make_float2(0.f, 0.f) : buf[cb][rb];
    const int64_t kk = col[ca] + (int64_t)M1 * ra;
    const float2 w = twiddle((uint32_t)kk, lgN);
    // Z_k = (X_k + conj X_{M-k}) + i w (X_k - conj X_{M-k})
    const float2 ev = make_float2(xa.x + xb.x, xa.y - xb.y);
    const float2 od = make_float2(xa.x - xb.x, xa.y + xb.y);
    const float2 wo = cmul(w, od);
    const float2 za = make_float2(ev.x - wo.y, ev.y + wo.x);
    if (nyq || (ca == cb && ra == rb)) {
      buf[ca][ra] = za;
    } else {
      // Z_{M-k} with twiddle -conj(w): E' = conj(E), O' = -conj(O)
      const float2 wb = make_float2(-w.x, w.y);
      const float2 evb = make_float2(ev.x, -ev.y);
      const float2 odb = make_float2(-od.x, od.y);
      const float2 wob = cmul(wb, odb);
      buf[ca][ra] = za;
      buf[cb][rb] = make_float2(evb.x - wob.y, evb.y + wob.x);
    }
  }
  __syncthreads();
  lds_dif(&buf[0][0], a.tw1, a.lgM2);
  if (ncol == 2) lds_dif(&buf[1][0], a.tw1, a.lgM2);
  const int lgM = a.lgM1 + a.lgM2;
  for (int c = 0; c < ncol; ++c) {
    const int k1 = col[c];
    if (M1 == 1) {
      for (int m2 = threadIdx.x; m2 < M2; m2 += blockDim.x)
        store_out(a, series, m2, buf[c][bitrev(m2, a.lgM2)]);
    } else {
      float2* dst = a.scratch + ((int64_t)sl * M1 + k1) * M2;
      for (int m2 = threadIdx.x; m2 < M2; m2 += blockDim.x) {
        const uint32_t e = (uint32_t)(((uint64_t)k1 * m2) & ((1ull << lgM) - 1));
        dst[m2] = cmul(buf[c][bitrev(m2, a.lgM2)], twiddle(e, lgM));
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_pink_pass2(PinkArgs a) {
  __shared__ float2 buf[kLdsC];
  const int nb = blockIdx.x;
  const int sl = blockIdx.y;
  const int64_t series = a.s0 + sl;
  const int M2 = a.M2, lgB2 = a.lgB2, B2 = 1 << lgB2;
  const int m20 = nb << lgB2;
  const float2* src = a.scratch + ((int64_t)sl << (a.lgM1 + a.lgM2));
  const int n = 1 << (a.lgM1 + lgB2);
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const int k1 = idx >> lgB2, bb = idx & (B2 - 1);
    buf[(bb << a.lgM1) + bitrev(k1, a.lgM1)] = src[(int64_t)k1 * M2 + m20 + bb];
  }
  __syncthreads();
  lds_dit(buf, a.tw2, a.lgM1, lgB2);
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const int m1 = idx >> lgB2, bb = idx & (B2 - 1);
    store_out(a, series, (int64_t)m1 * M2 + m20 + bb, buf[(bb << a.lgM1) + m1]);
  }
}

void launch_pink_tables(const PinkArgs& a, hipStream_t s) {
  const int n = 1 << std::max(a.lgM1, a.lgM2);
  hipLaunchKernelGGL(k_pink_tables, dim3((n + 255) / 256), dim3(256), 0, s, a.tw1,
                     a.lgM2, a.tw2, a.lgM1);
}

void launch_pink_pass1(const PinkArgs& a, hipStream_t s) {
  const int groups = a.M1 == 1 ? 1 : a.M1 / 2 + 1;
  hipLaunchKernelGGL(k_pink_pass1, dim3(groups, a.n_series), dim3(256), 0, s, a);
}

void launch_pink_pass2(const PinkArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_pink_pass2, dim3(a.M2 >> a.lgB2, a.n_series), dim3(256), 0,
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
