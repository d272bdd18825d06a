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
// With M1 = 1 pass 1 writes the output directly.
//
// Each DFT runs in LDS as self-sorting (Stockham) passes of radix 16, then
// one of radix 2, 4 or 8 for the remaining factor: a thread loads the R
// inputs j + r L/R of one group into registers, multiplies them by
// e^{2 pi i r (j mod S) / (S R)} (S = product of the radices before),
// does the length-R DFT in registers and stores output s at
// (j div S) S R + (j mod S) + s S.  Input and output are in natural order.
// Pass twiddles come from one table of e^{2 pi i m / 4096} in global
// memory (evaluated with sincospi on exact arguments): a pass loads w, w^2,
// w^4, w^8 for its group and forms the other powers as products of at
// most four of them.  The in-register DFTs use the constants cos, sin(2 pi
// m / 16).  The real-to-complex and four-step twiddles of a thread's 16
// elements are a geometric sequence, taken as w0 times products of at most
// four sincospi factors.  Pass 1 keeps its one or
// two transforms contiguous in LDS with one float2 of padding after every
// 16, so that the stride-16 stores of the first pass hit distinct banks;
// pass 2 interleaves its B2 transforms (element i of transform t at
// i B2 + t, t fastest across lanes), which makes every access consecutive.
// All index arithmetic is shifts and masks (lengths are powers of two).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gtod_internal.h"
#include "philox.h"

namespace gtod {

namespace {

constexpr int kLdsC = 4096;   // complex values per transform set

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ float2 csub(float2 a, float2 b) {
  return make_float2(a.x - b.x, a.y - b.y);
}

__device__ __forceinline__ float2 twiddle(uint32_t num, int lg_den) {
  // e^{2 pi i num / 2^lg_den}, num < 2^lg_den <= 2^24
  const float x = ldexpf((float)num, 1 - lg_den);  // 2 num / den, exact
  float s, c;
  sincospif(x, &s, &c);
  return make_float2(c, s);
}

// e^{2 pi i (e0 + i d) / 2^lg} for i = 0 .. 15: w0 times the product of the
// factors e^{2 pi i 2^b d / 2^lg} for the set bits b of i, each evaluated
// with sincospi on an exact argument (at most five roundings in all).
struct GeoTwiddle {
  float2 w0, f[4];
  __device__ GeoTwiddle(uint32_t e0, uint32_t d, int lg) {
    const uint32_t mask = (1u << lg) - 1;
    w0 = twiddle(e0 & mask, lg);
#pragma unroll
    for (int b = 0; b < 4; ++b) f[b] = twiddle((d << b) & mask, lg);
  }
  __device__ float2 operator()(int i) const {
    float2 w = w0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if ((i >> b) & 1) w = cmul(w, f[b]);
    return w;
  }
};

// cos and sin of 2 pi m / 16, m = 0 .. 7, rounded to float
__device__ constexpr float kCos16[8] = {
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f};
__device__ constexpr float kSin16[8] = {
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f};

// a e^{2 pi i m / 16}; m is a constant once the callers are unrolled
__device__ __forceinline__ float2 mul_w16(float2 a, int m) {
  if (m == 0) return a;
  if (m == 4) return make_float2(-a.y, a.x);
  return make_float2(a.x * kCos16[m] - a.y * kSin16[m],
                     a.x * kSin16[m] + a.y * kCos16[m]);
}

constexpr int brev_c(int x, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((x >> b) & 1) << (bits - 1 - b);
  return r;
}

// In-register inverse DFT of length 2^LGR (<= 16), natural order in and
// out: bit-reversed copy, then radix-2 decimation in time.
template <int LGR>
__device__ __forceinline__ void dft_inv(float2 (&v)[1 << LGR]) {
  constexpr int R = 1 << LGR;
  float2 u[R];
#pragma unroll
  for (int r = 0; r < R; ++r) u[brev_c(r, LGR)] = v[r];
#pragma unroll
  for (int s = 1; s <= LGR; ++s) {
    const int half = 1 << (s - 1);
#pragma unroll
    for (int b = 0; b < R / 2; ++b) {
      const int pos = b & (half - 1);
      const int i = ((b >> (s - 1)) << s) + pos;
      const float2 x = u[i];
      const float2 y = mul_w16(u[i + half], pos << (4 - s));
      u[i] = cadd(x, y);
      u[i + half] = csub(x, y);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = u[r];
}

// Element i of transform t: pass 1 keeps transforms contiguous with one
// float2 of padding after every 16; pass 2 interleaves them.
struct AddrPadded {
  int lgL;
  __device__ int operator()(int t, int i) const {
    const int x = (t << lgL) + i;
    return x + (x >> 4);
  }
};
struct AddrInterleaved {
  int lgT;
  __device__ int operator()(int t, int i) const { return (i << lgT) + t; }
};

// One Stockham pass of radix 2^LGR over the 2^lgT transforms of length
// 2^lgL in buf, after passes whose radices multiply to 2^lgNs.  EMAX is
// the largest element count of any caller (groups per thread <= EMAX /
// (256 R)).  Transform t and group j of group g: t slowest for contiguous
// transforms (TFAST = false), fastest for interleaved ones.
template <int LGR, int EMAX, bool TFAST, class Addr>
__device__ __forceinline__ void stockham_pass(float2* buf, Addr addr, int lgL, int lgT,
                                              int lgNs, const float2* __restrict__ tab) {
  constexpr int R = 1 << LGR;
  constexpr int GM = (EMAX / 256 / R) > 0 ? EMAX / 256 / R : 1;
  const int lgJ = lgL - LGR;                     // log2 of the groups per transform
  const int nG = 1 << (lgT + lgJ);
  float2 v[GM][R];
#pragma unroll
  for (int gi = 0; gi < GM; ++gi) {
    const int g = threadIdx.x + gi * 256;
    if (g < nG) {
      const int t = TFAST ? (g & ((1 << lgT) - 1)) : (g >> lgJ);
      const int j = TFAST ? (g >> lgT) : (g & ((1 << lgJ) - 1));
#pragma unroll
      for (int r = 0; r < R; ++r) v[gi][r] = buf[addr(t, j + (r << lgJ))];
      if (lgNs > 0) {
        // w^r for w = e^{2 pi i k / (S R)}: w^1, w^2, w^4, w^8 from the
        // table, the other powers as products of at most four of them
        const int k = j & ((1 << lgNs) - 1);
        const int sh = 12 - lgNs - LGR;
        float2 wp[R];
        wp[0] = make_float2(1.f, 0.f);
#pragma unroll
        for (int b = 0; b < LGR; ++b) wp[1 << b] = tab[(k << b) << sh];
#pragma unroll
        for (int r = 3; r < R; ++r)
          if (r & (r - 1)) wp[r] = cmul(wp[r & (r - 1)], wp[r & -r]);
#pragma unroll
        for (int r = 1; r < R; ++r) v[gi][r] = cmul(v[gi][r], wp[r]);
      }
      dft_inv<LGR>(v[gi]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int gi = 0; gi < GM; ++gi) {
    const int g = threadIdx.x + gi * 256;
    if (g < nG) {
      const int t = TFAST ? (g & ((1 << lgT) - 1)) : (g >> lgJ);
      const int j = TFAST ? (g >> lgT) : (g & ((1 << lgJ) - 1));
      const int k = j & ((1 << lgNs) - 1);
      const int d = ((j >> lgNs) << (lgNs + LGR)) + k;
#pragma unroll
      for (int s = 0; s < R; ++s) buf[addr(t, d + (s << lgNs))] = v[gi][s];
    }
  }
  __syncthreads();
}

// In-place inverse DFTs (natural order in and out) of the 2^lgT
// transforms of length 2^lgL (<= 4096) in buf.
template <int EMAX, bool TFAST, class Addr>
__device__ __forceinline__ void fft_inv(float2* buf, Addr addr, int lgL, int lgT,
                                        const float2* __restrict__ tab) {
  int lgNs = 0;
  while (lgL - lgNs >= 4) {
    stockham_pass<4, EMAX, TFAST>(buf, addr, lgL, lgT, lgNs, tab);
    lgNs += 4;
  }
  switch (lgL - lgNs) {
    case 1: stockham_pass<1, EMAX, TFAST>(buf, addr, lgL, lgT, lgNs, tab); break;
    case 2: stockham_pass<2, EMAX, TFAST>(buf, addr, lgL, lgT, lgNs, tab); break;
    case 3: stockham_pass<3, EMAX, TFAST>(buf, addr, lgL, lgT, lgNs, tab); break;
    default: break;
  }
}

// Samples 2m and 2m + 1 of a series: one 8-byte access where the pair is
// 8-byte aligned (even row pitch, aligned output), so that a run of lanes
// covers whole cache lines in one store; else two 4-byte accesses.
__device__ __forceinline__ void store_out(const PinkArgs& a, int64_t series,
                                          int64_t m, float2 z) {
  const int64_t t = 2 * m;
  float* dst = a.tod + series * a.out_ld;
  const bool pairs = ((a.out_ld & 1) == 0) && ((reinterpret_cast<uintptr_t>(a.tod) & 7) == 0);
  if (pairs && t + 1 < a.t_total) {
    float2* d2 = reinterpret_cast<float2*>(dst + t);
    if (a.accumulate) {
      float2 o = *d2;
      o.x += z.x;
      o.y += z.y;
      *d2 = o;
    } else {
      *d2 = z;
    }
    return;
  }
  if (t < a.t_total) {
    if (a.accumulate) dst[t] += z.x; else dst[t] = z.x;
  }
  if (t + 1 < a.t_total) {
    if (a.accumulate) dst[t + 1] += z.y; else dst[t + 1] = z.y;
  }
}


}  // namespace

// Twiddle table: entry m holds e^{2 pi i m / 4096}.
__global__ void k_pink_tables(float2* tab) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < kLdsC) tab[m] = twiddle((uint32_t)m, 12);
}

// Pass 1 works on a set of columns closed under k -> M - k: column 0,
// column M1/2, or the pair (k1, M1 - k1).  Each spectral bin X_j is drawn
// once; every Z_k is built from X_k and X_{M-k} held in LDS, two at a time
// (e^{2 pi i (M-k)/N} = -conj e^{2 pi i k/N}).
// Dynamic LDS: one or two padded transforms of M2 values; EMAX bounds the
// values per workgroup.  LGM2 > 0 fixes lg M2 at compile time (the length
// every two-pass series uses), so that the transform's index arithmetic
// folds into constants; LGM2 = 0 takes it from the arguments.
template <int EMAX, int LGM2>
__global__ __launch_bounds__(256) void k_pink_pass1(PinkArgs a) {
  extern __shared__ float2 buf[];
  const int lgM2 = LGM2 > 0 ? LGM2 : a.lgM2;
  const AddrPadded at{lgM2};
  const int grp = blockIdx.x;
  const int sl = blockIdx.y;
  const int64_t series = a.s0 + sl;
  const int p = (int)(series / a.K);
  const int k = (int)(series % a.K);
  const float sc = a.scale[k];
  const float halpha = -0.5f * a.alpha[k];
  const float fstep = (float)(a.fs / (double)a.N);
  const int M1 = a.M1, M2 = 1 << lgM2;
  const int lgN = a.lgM1 + lgM2 + 1;
  // columns of this group: kind 0 = {0}, 1 = {M1/2}, 2 = {k1, M1 - k1}
  int kind, col[2], ncol;
  if (grp == 0) { kind = 0; col[0] = 0; ncol = 1; }
  else if (grp == 1) { kind = 1; col[0] = M1 / 2; ncol = 1; }
  else { kind = 2; col[0] = grp - 1; col[1] = M1 - (grp - 1); ncol = 2; }
  col[1] = (ncol == 2) ? col[1] : col[0];

  // draw X for every bin of the group's columns (natural order)
  for (int idx = threadIdx.x; idx < (ncol << lgM2); idx += blockDim.x) {
    const int c = idx >> lgM2, k2 = idx & (M2 - 1);
    const int64_t j = col[c] + (int64_t)M1 * k2;
    float2 x = make_float2(0.f, 0.f);
    if (j > 0 && j < a.M) {
      const u32x4 o = philox10(u32x4{(uint32_t)j, (uint32_t)k, (uint32_t)(a.pix0 + p), 1u},
                               a.key0, a.key1);
      float zc, zs;
      box_muller(o.x, o.y, &zc, &zs);
      // power law from the hardware log2 and exp2 (about one ulp each)
      const float cj = sc * __builtin_amdgcn_exp2f(halpha * __builtin_amdgcn_logf((float)j * fstep));
      x = make_float2(cj * zc, cj * zs);
    }
    buf[at(c, k2)] = x;
  }
  __syncthreads();
  // Z in place, one pair (k, M - k) per work item
  const int U = kind == 0 ? M2 / 2 + 1 : (kind == 1 ? M2 / 2 : M2);
  // e^{2 pi i k / N} at k = col + M1 u, u = threadIdx.x + 256 i
  const GeoTwiddle wz((uint32_t)(col[0] + (int64_t)M1 * threadIdx.x),
                      (uint32_t)((int64_t)M1 * 256), lgN);
  for (int u = threadIdx.x, iu = 0; u < U; u += 256, ++iu) {
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
    const float2 xa = buf[at(ca, ra)];
    const float2 xb = nyq ? make_float2(0.f, 0.f) : buf[at(cb, rb)];
    const float2 w = wz(iu);
    // Z_k = (X_k + conj X_{M-k}) + i w (X_k - conj X_{M-k})
    const float2 ev = make_float2(xa.x + xb.x, xa.y - xb.y);
    const float2 od = make_float2(xa.x - xb.x, xa.y + xb.y);
    const float2 wo = cmul(w, od);
    const float2 za = make_float2(ev.x - wo.y, ev.y + wo.x);
    if (nyq || (ca == cb && ra == rb)) {
      buf[at(ca, ra)] = za;
    } else {
      // Z_{M-k} with twiddle -conj(w): E' = conj(E), O' = -conj(O)
      const float2 wb = make_float2(-w.x, w.y);
      const float2 evb = make_float2(ev.x, -ev.y);
      const float2 odb = make_float2(-od.x, od.y);
      const float2 wob = cmul(wb, odb);
      buf[at(ca, ra)] = za;
      buf[at(cb, rb)] = make_float2(evb.x - wob.y, evb.y + wob.x);
    }
  }
  __syncthreads();
  if constexpr (LGM2 > 0) {
    if (ncol == 2) fft_inv<EMAX, false>(buf, at, LGM2, 1, a.tab);
    else fft_inv<EMAX, false>(buf, at, LGM2, 0, a.tab);
  } else {
    fft_inv<EMAX, false>(buf, at, lgM2, ncol - 1, a.tab);
  }
  const int lgM = a.lgM1 + lgM2;
  for (int c = 0; c < ncol; ++c) {
    const int k1 = col[c];
    if (M1 == 1) {
      for (int m2 = threadIdx.x; m2 < M2; m2 += blockDim.x)
        store_out(a, series, m2, buf[at(c, m2)]);
    } else {
      float2* dst = a.scratch + ((int64_t)sl * M1 + k1) * M2;
      // e^{2 pi i k1 m2 / M} at m2 = threadIdx.x + 256 i
      const GeoTwiddle ws((uint32_t)((uint64_t)k1 * threadIdx.x),
                          (uint32_t)((uint64_t)k1 * 256), lgM);
      for (int m2 = threadIdx.x, im = 0; m2 < M2; m2 += 256, ++im)
        dst[m2] = cmul(buf[at(c, m2)], ws(im));
    }
  }
}

// Pass 2 for at most EMAX = 2^(lgM1 + lgB2) elements per workgroup, held
// in dynamic LDS of exactly that size (small blocks keep many workgroups
// per CU, which is what this memory-bound pass needs).
// LGM1 > 0 fixes lg M1 at compile time for series whose columns are
// 2048 long (lg M2 = 11), so that the index arithmetic folds; LGM1 = 0
// takes the lengths from the arguments.
template <int EMAX, int LGM1>
__global__ __launch_bounds__(256) void k_pink_pass2(PinkArgs a) {
  extern __shared__ float2 buf[];
  const int nb = blockIdx.x;
  const int sl = blockIdx.y;
  const int64_t series = a.s0 + sl;
  constexpr int kLgB2 = LGM1 > 0 ? (12 - LGM1 < kPinkLgB2 ? 12 - LGM1 : kPinkLgB2) : 0;
  const int lgM1 = LGM1 > 0 ? LGM1 : a.lgM1;
  const int lgM2 = LGM1 > 0 ? kPinkLgM2 : a.lgM2;
  const int M2 = 1 << lgM2, lgB2 = LGM1 > 0 ? kLgB2 : a.lgB2, B2 = 1 << lgB2;
  const int m20 = nb << lgB2;
  const float2* src = a.scratch + ((int64_t)sl << (lgM1 + lgM2));
  const int n = 1 << (lgM1 + lgB2);
  // element k1 of transform bb at k1 B2 + bb: both sides consecutive
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const int k1 = idx >> lgB2, bb = idx & (B2 - 1);
    buf[idx] = src[(int64_t)k1 * M2 + m20 + bb];
  }
  __syncthreads();
  fft_inv<EMAX, true>(buf, AddrInterleaved{lgB2}, lgM1, lgB2, a.tab);
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const int m1 = idx >> lgB2, bb = idx & (B2 - 1);
    store_out(a, series, (int64_t)m1 * M2 + m20 + bb, buf[idx]);
  }
}

void launch_pink_tables(const PinkArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_pink_tables, dim3(kLdsC / 256), dim3(256), 0, s, a.tab_w);
}

void launch_pink_pass1(const PinkArgs& a, hipStream_t s) {
  const int groups = a.M1 == 1 ? 1 : a.M1 / 2 + 1;
  const int e = (a.M1 == 1 ? 1 : 2) << a.lgM2;   // values per workgroup
  const size_t lds = (size_t)(e + (e >> 4)) * sizeof(float2);
  const dim3 grid(groups, a.n_series);
  if (e <= kLdsC && a.lgM2 == kPinkLgM2)
    hipLaunchKernelGGL((k_pink_pass1<kLdsC, kPinkLgM2>), grid, dim3(256), lds, s, a);
  else if (e <= kLdsC)
    hipLaunchKernelGGL((k_pink_pass1<kLdsC, 0>), grid, dim3(256), lds, s, a);
  else
    hipLaunchKernelGGL((k_pink_pass1<2 * kLdsC, 0>), grid, dim3(256), lds, s, a);
}

void launch_pink_pass2(const PinkArgs& a, hipStream_t s) {
  const dim3 grid(a.M2 >> a.lgB2, a.n_series);
  const int e = 1 << (a.lgM1 + a.lgB2);
  const size_t lds = (size_t)e * sizeof(float2);
#define GTOD_PASS2(EM, L) hipLaunchKernelGGL((k_pink_pass2<EM, L>), grid, dim3(256), lds, s, a)
  if (a.lgM2 == kPinkLgM2 && a.lgB2 == std::min(kPinkLgB2, 12 - a.lgM1)) {
    switch (a.lgM1) {   // e = 2^(lgM1 + lgB2) <= 4096
      case 1: GTOD_PASS2(kLdsC / 2, 1); return;
      case 2: GTOD_PASS2(kLdsC / 2, 2); return;
      case 3: GTOD_PASS2(kLdsC / 2, 3); return;
      case 4: GTOD_PASS2(kLdsC / 2, 4); return;
      case 5: GTOD_PASS2(kLdsC / 2, 5); return;
      case 6: GTOD_PASS2(kLdsC / 2, 6); return;
      case 7: GTOD_PASS2(kLdsC / 2, 7); return;
      case 8: GTOD_PASS2(kLdsC, 8); return;
      default: break;
    }
  }
  if (e <= kLdsC / 2) GTOD_PASS2(kLdsC / 2, 0);
  else GTOD_PASS2(kLdsC, 0);
#undef GTOD_PASS2
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
