// Brightness-temperature scale by a simulated skydip (section 2.7), FP64.
//
// The sky brightness is varied through the zenith PWV at a fixed elevation
// while the noise-free channel power is recorded; per channel, a
// least-squares line P = a + b T_b maps power to the line-of-sight
// brightness temperature
//   T_b,k = T_atm sum_j B0_jk (1 - eta_atm,j) / sum_j B0_jk,  B0 = w eta.
// Row powers use the collapsed cascade P = E + (1 - eta_atm) D (no source).
// Three small kernels: sweep rows, contraction against B0, per-channel fit.
// This is a calibration call, run once per spectral setup and elevation;
// everything stays in FP64 so that the scale carries no FP32 rounding into
// the Kelvin output.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gtod_internal.h"

namespace gtod {

namespace {

constexpr int kSdCh = 64;      // channels per contraction block (one wave)
constexpr int kSdPhases = 4;   // waves splitting the frequency axis
constexpr int kSdRows = 8;     // sweep rows per contraction block
constexpr int kSdFit = 256;    // threads of the fit block

}  // namespace

// Row i, bin j: zenith optical depth interpolated linearly in PWV with the
// PWV clamped to the table axis, sky emissivity 1 - eta_atm and power.
__global__ __launch_bounds__(128) void k_skydip_rows(SkydipArgs a) {
  const int j = blockIdx.x * 128 + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= a.F) return;
  const double step = (a.pwv_hi - a.pwv_lo) / (double)(a.n - 1);
  const double pwv = (i == a.n - 1) ? a.pwv_hi : a.pwv_lo + i * step;
  double g = (pwv - a.pwv0) / a.dpwv;
  g = fmin(fmax(g, 0.0), (double)(a.n_pwv - 1));
  int ci = (int)floor(g);
  if (ci > a.n_pwv - 2) ci = a.n_pwv - 2;
  const double wg = g - ci;
  const double tz = (1.0 - wg) * a.tau64[(int64_t)ci * a.F + j] +
                    wg * a.tau64[(int64_t)(ci + 1) * a.F + j];
  const double xi = -expm1(-a.csc * tz);
  a.Pm[(int64_t)i * a.F + j] = a.E64[j] + xi * a.D64[j];
  a.Xm[(int64_t)i * a.F + j] = xi;
}

// Block: kSdCh channels x kSdRows sweep rows; wave w sums bins j = w mod
// kSdPhases, then the phases are added in a fixed order.
__global__ __launch_bounds__(kSdCh * kSdPhases) void k_skydip_contract(SkydipArgs a) {
  __shared__ double red[kSdPhases][2 * kSdRows + 1][kSdCh];
  const int kl = threadIdx.x % kSdCh, ph = threadIdx.x / kSdCh;
  const int k = blockIdx.x * kSdCh + kl;
  const int i0 = blockIdx.y * kSdRows;
  double sp[kSdRows], sx[kSdRows], sw = 0.0;
#pragma unroll
  for (int r = 0; r < kSdRows; ++r) sp[r] = sx[r] = 0.0;
  int64_t rowoff[kSdRows];
#pragma unroll
  for (int r = 0; r < kSdRows; ++r)
    rowoff[r] = (int64_t)min(i0 + r, a.n - 1) * a.F;
  if (k < a.K) {
    for (int j = ph; j < a.F; j += kSdPhases) {
      const double bk = a.B0[(int64_t)j * a.K + k];
      sw += bk;
#pragma unroll
      for (int r = 0; r < kSdRows; ++r) {
        sp[r] += a.Pm[rowoff[r] + j] * bk;
        sx[r] += a.Xm[rowoff[r] + j] * bk;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kSdRows; ++r) {
    red[ph][r][kl] = sp[r];
    red[ph][kSdRows + r][kl] = sx[r];
  }
  red[ph][2 * kSdRows][kl] = sw;
  __syncthreads();
  if (ph != 0 || k >= a.K) return;
  double w = 0.0;
  for (int q = 0; q < kSdPhases; ++q) w += red[q][2 * kSdRows][kl];
  for (int r = 0; r < kSdRows; ++r) {
    const int i = i0 + r;
    if (i >= a.n) break;
    double p = 0.0, x = 0.0;
    for (int q = 0; q < kSdPhases; ++q) {
      p += red[q][r][kl];
      x += red[q][kSdRows + r][kl];
    }
    a.p_kid[(int64_t)i * a.K + k] = p;
    a.t_b[(int64_t)i * a.K + k] = (w > 0.0) ? a.t_atm * x / w : NAN;
  }
}

namespace {

__device__ double block_sum(double v, double* s) {
  s[threadIdx.x] = v;
  __syncthreads();
  for (int st = kSdFit / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  const double r = s[0];
  __syncthreads();
  return r;
}

}  // namespace

// One block per channel: means, then centred moments (two passes), with a
// fixed-order tree reduction.  No scale (NaN) for a channel whose T_b is
// undefined or constant over the sweep.
__global__ __launch_bounds__(kSdFit) void k_skydip_fit(SkydipArgs a) {
  __shared__ double s[kSdFit];
  const int k = blockIdx.x;
  double sx = 0.0, sy = 0.0, bad = 0.0;
  for (int i = threadIdx.x; i < a.n; i += kSdFit) {
    const double x = a.t_b[(int64_t)i * a.K + k];
    if (!isfinite(x)) bad = 1.0;
    sx += x;
    sy += a.p_kid[(int64_t)i * a.K + k];
  }
  const double nbad = block_sum(bad, s);
  const double mx = block_sum(sx, s) / a.n;
  const double my = block_sum(sy, s) / a.n;
  double sxx = 0.0, sxy = 0.0;
  if (nbad == 0.0) {
    for (int i = threadIdx.x; i < a.n; i += kSdFit) {
      const double dx = a.t_b[(int64_t)i * a.K + k] - mx;
      sxx += dx * dx;
      sxy += dx * (a.p_kid[(int64_t)i * a.K + k] - my);
    }
  }
  const double Sxx = block_sum(sxx, s);
  const double Sxy = block_sum(sxy, s);
  if (threadIdx.x != 0) return;
  if (nbad != 0.0 || !(Sxx > 0.0)) {
    a.a[k] = a.b[k] = a.ib[k] = NAN;
    return;
  }
  const double b = Sxy / Sxx;
  a.b[k] = b;
  a.a[k] = my - b * mx;
  a.ib[k] = 1.0 / b;
}

void launch_skydip(const SkydipArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_skydip_rows, dim3((a.F + 127) / 128, a.n), dim3(128),
                     0, s, a);
  hipLaunchKernelGGL(k_skydip_contract,
                     dim3((a.K + kSdCh - 1) / kSdCh, (a.n + kSdRows - 1) / kSdRows),
                     dim3(kSdCh * kSdPhases), 0, s, a);
  hipLaunchKernelGGL(k_skydip_fit, dim3(a.K), dim3(kSdFit), 0, s, a);
}

}  // namespace gtod
