// Common-mode atmosphere subtraction (section 4.3, Eqs. common_mode and
// Sj) and inverse-variance gridding of a brightness-temperature TOD, FP64
// arithmetic on FP32 data.
//
//   eta_z,k   = sum_j B0_jk eta_z,j(PWV_mean) / sum_j B0_jk
//   eta_i     = eta_z,k ^ (1 / sin(theta(t) + theta0 + dtheta_i))
//   M(t, k)   = (1 / N_out) sum_{j off source} T_b,j / (1 - eta_j)
//   T*_i      = T_b,i / eta_i - (1 - eta_i) / eta_i M(t, k)
// with 1 - eta = -expm1(ln eta) so that transparent channels keep their
// relative precision.  Gridding bins T*_i(t, k) of spaxel i at (phi(t) +
// dphi_i, theta(t) + dtheta_i) to the nearest node of an n x n grid; per
// (spaxel, channel, cell) the mean and the variance of the samples give a
// weight m / s^2, and the cells of all spaxels are combined with it.
//
// Kernels: setup (scan table, mean PWV, channel transmission), common (one
// thread per sample and 16 channels: M and optionally T*), grid (one block
// per (spaxel, channel): cell sums in LDS), combine (one thread per
// (channel, cell)).  The common and grid kernels each stream the TOD once;
// per sample they evaluate one FP64 expm1 (eta = 1 + expm1(ln eta), so
// 1 - eta keeps its relative precision), with the cosecant shared by the
// channels of a thread in the common kernel.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gtod_internal.h"
#include "scan.h"

namespace gtod {

namespace {

constexpr int kRdThreads = 256;

__device__ double block_sum_256(double v, double* s) {
  s[threadIdx.x] = v;
  __syncthreads();
  for (int st = kRdThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  const double r = s[0];
  __syncthreads();
  return r;
}

__device__ inline int map_cell(const ReduceArgs& a, double x, double y) {
  const double gx = floor((x + a.half) / a.dcell + 0.5);
  const double gy = floor((y + a.half) / a.dcell + 0.5);
  if (!(gx >= 0.0 && gx < (double)a.map_n && gy >= 0.0 && gy < (double)a.map_n))
    return -1;
  return (int)gy * a.map_n + (int)gx;
}

}  // namespace

__global__ __launch_bounds__(kRdThreads) void k_rd_scan(ReduceArgs a) {
  const int64_t t = (int64_t)blockIdx.x * kRdThreads + threadIdx.x;
  if (t >= a.T) return;
  double phi, th;
  scan_offsets(a.scan_kind, a.r_petal, a.omega, a.Omega, a.traj, a.t0 + t,
               a.f_s, &phi, &th);
  a.scan_tab[t] = make_double2(phi, th);
}

// Mean zenith PWV (one block, fixed-order sums), then ln eta_z,k (one
// block per channel).
__global__ __launch_bounds__(kRdThreads) void k_rd_pwv_mean(ReduceArgs a) {
  __shared__ double s[kRdThreads];
  double acc = 0.0;
  if (a.pwv) {
    const int64_t n = (int64_t)a.P * a.pwv_len;
    for (int64_t i = threadIdx.x; i < n; i += kRdThreads) {
      const int64_t p = i / a.pwv_len, t = i % a.pwv_len;
      acc += (double)a.pwv[p * a.pwv_ld + t];
    }
  }
  const double tot = block_sum_256(acc, s);
  if (threadIdx.x == 0)
    a.pwv_mean[0] = a.pwv ? tot / ((double)a.P * (double)a.pwv_len) : a.pwv_host;
}

__global__ __launch_bounds__(kRdThreads) void k_rd_channel(ReduceArgs a) {
  __shared__ double s[kRdThreads];
  const int k = blockIdx.x;
  double g = (a.pwv_mean[0] - a.pwv0) / a.dpwv;
  g = fmin(fmax(g, 0.0), (double)(a.n_pwv - 1));
  int ci = (int)floor(g);
  if (ci > a.n_pwv - 2) ci = a.n_pwv - 2;
  const double wg = g - ci;
  double num = 0.0, den = 0.0;
  for (int j = threadIdx.x; j < a.F; j += kRdThreads) {
    const double tz = (1.0 - wg) * a.tau64[(int64_t)ci * a.F + j] +
                      wg * a.tau64[(int64_t)(ci + 1) * a.F + j];
    const double b = a.B0[(int64_t)j * a.K + k];
    num += b * exp(-tz);
    den += b;
  }
  const double N = block_sum_256(num, s);
  const double D = block_sum_256(den, s);
  if (threadIdx.x == 0) a.lnz[k] = (D > 0.0) ? log(N / D) : NAN;
}

// One thread per sample t and kRdChan channels of the group: the cosecant
// of each spaxel is evaluated once per (spaxel, sample) and used for every
// channel; eta and 1 - eta both come from one expm1.
constexpr int kRdChan = 16;
__global__ __launch_bounds__(kRdThreads) void k_rd_common(ReduceArgs a) {
  const int64_t t = (int64_t)blockIdx.x * kRdThreads + threadIdx.x;
  const int kl0 = blockIdx.y * kRdChan;
  if (t >= a.T) return;
  const int nk = min(kRdChan, a.kg - kl0);
  double lz[kRdChan], sum[kRdChan];
#pragma unroll
  for (int q = 0; q < kRdChan; ++q) {
    lz[q] = q < nk ? a.lnz[a.k0 + kl0 + q] : 0.0;
    sum[q] = 0.0;
  }
  const double th = a.scan_tab[t].y + a.theta0;
  const int64_t rowK = a.ld;                      // stride between channels
  for (int p = 0; p < a.P; ++p) {
    if (!a.off[p]) continue;
    const double csc = 1.0 / sin(th + a.dtheta[p]);
    const float* src = a.tod + ((int64_t)p * a.K + a.k0 + kl0) * a.ld + t;
#pragma unroll
    for (int q = 0; q < kRdChan; ++q)
      if (q < nk) sum[q] += (double)src[q * rowK] / -expm1(lz[q] * csc);
  }
#pragma unroll
  for (int q = 0; q < kRdChan; ++q) {
    sum[q] /= (double)a.n_out;
    if (q < nk && a.M) a.M[(int64_t)(kl0 + q) * a.T + t] = sum[q];
  }
  if (!a.t_star || a.map_n > 0) return;
  for (int p = 0; p < a.P; ++p) {
    const double csc = 1.0 / sin(th + a.dtheta[p]);
    const int64_t o = ((int64_t)p * a.K + a.k0 + kl0) * a.ld + t;
#pragma unroll
    for (int q = 0; q < kRdChan; ++q) {
      if (q < nk) {
        const double em = expm1(lz[q] * csc);     // eta - 1
        a.t_star[o + q * rowK] =
            (float)(((double)a.tod[o + q * rowK] + em * sum[q]) / (1.0 + em));
      }
    }
  }
}

// One block per (spaxel, kRdGridChan channels of the group), spaxel
// fastest so that the blocks sharing those channels' M rows run together.
// The sample's cosecant and cell are evaluated once for all its channels;
// cell count (common to the channels), and per channel the sums of v =
// T* - shift (shift = the channel's first sample) and v^2, accumulate in
// LDS; the variance is (S2 - S1^2 / m) / (m - 1).  When T* is requested
// with maps, this kernel also stores it (for every sample, in or out of
// the map).
constexpr int kRdGridChan = 4;
__global__ __launch_bounds__(kRdThreads) void k_rd_grid(ReduceArgs a) {
  extern __shared__ double gsm[];
  const int C = a.map_n * a.map_n;
  double* s1 = gsm;                                   // [G][C]
  double* s2 = gsm + kRdGridChan * C;                 // [G][C]
  unsigned* cnt = (unsigned*)(gsm + 2 * kRdGridChan * C);   // [C]
  const int p = blockIdx.x % a.P;
  const int kl0 = (blockIdx.x / a.P) * kRdGridChan;
  const int nk = min(kRdGridChan, a.kg - kl0);
  for (int c = threadIdx.x; c < C; c += kRdThreads) {
    cnt[c] = 0u;
#pragma unroll
    for (int q = 0; q < kRdGridChan; ++q) {
      s1[q * C + c] = 0.0;
      s2[q * C + c] = 0.0;
    }
  }
  const double dth = a.theta0 + a.dtheta[p];
  const double dph = a.dphi[p];
  double lz[kRdGridChan], shift[kRdGridChan];
  const float* row[kRdGridChan];
  const double* Mr[kRdGridChan];
  const double csc0 = 1.0 / sin(a.scan_tab[0].y + dth);
#pragma unroll
  for (int q = 0; q < kRdGridChan; ++q) {
    const int kq = min(kl0 + q, a.kg - 1);     // dead slots repeat the last channel
    lz[q] = a.lnz[a.k0 + kq];
    row[q] = a.tod + ((int64_t)p * a.K + a.k0 + kq) * a.ld;
    Mr[q] = a.M + (int64_t)kq * a.T;
    const double em = expm1(lz[q] * csc0);
    shift[q] = ((double)row[q][0] + em * Mr[q][0]) / (1.0 + em);
  }
  float* out_ts = a.t_star ? a.t_star + ((int64_t)p * a.K + a.k0 + kl0) * a.ld : nullptr;
  __syncthreads();
  for (int64_t t = threadIdx.x; t < a.T; t += kRdThreads) {
    const double2 sc = a.scan_tab[t];
    const int c = map_cell(a, sc.x + dph, sc.y + a.dtheta[p]);
    if (c < 0 && !out_ts) continue;
    const double csc = 1.0 / sin(sc.y + dth);
    if (c >= 0) atomicAdd(&cnt[c], 1u);
#pragma unroll
    for (int q = 0; q < kRdGridChan; ++q) {
      if (q < nk) {
        const double em = expm1(lz[q] * csc);     // eta - 1
        const double ts = ((double)row[q][t] + em * Mr[q][t]) / (1.0 + em);
        if (out_ts) out_ts[q * a.ld + t] = (float)ts;
        if (c >= 0) {
          const double v = ts - shift[q];
          atomicAdd(&s1[q * C + c], v);
          atomicAdd(&s2[q * C + c], v * v);
        }
      }
    }
  }
  __syncthreads();
  for (int q = 0; q < nk; ++q) {
    double2* out = a.stats + ((int64_t)p * a.kg + kl0 + q) * C;
    for (int c = threadIdx.x; c < C; c += kRdThreads) {
      const double m = (double)cnt[c];
      double w = 0.0, mean = 0.0;
      if (m >= 2.0) {
        const double S1 = s1[q * C + c], S2 = s2[q * C + c];
        const double var = (S2 - S1 * S1 / m) / (m - 1.0);
        if (var > 0.0) {
          w = m / var;
          mean = S1 / m + shift[q];
        }
      }
      out[c] = make_double2(w, mean);
    }
  }
}

__global__ __launch_bounds__(kRdThreads) void k_rd_combine(ReduceArgs a) {
  const int C = a.map_n * a.map_n;
  const int c = blockIdx.x * kRdThreads + threadIdx.x;
  const int kl = blockIdx.y;
  if (c >= C) return;
  double ws = 0.0, num = 0.0;
  for (int p = 0; p < a.P; ++p) {
    const double2 st = a.stats[((int64_t)p * a.kg + kl) * C + c];
    if (st.x > 0.0) {
      ws += st.x;
      num += st.x * st.y;
    }
  }
  const int64_t o = (int64_t)(a.k0 + kl) * C + c;
  a.map[o] = ws > 0.0 ? num / ws : NAN;
  a.weight[o] = ws;
}

void launch_reduce_setup(const ReduceArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_rd_scan, dim3((unsigned)((a.T + kRdThreads - 1) / kRdThreads)),
                     dim3(kRdThreads), 0, s, a);
  hipLaunchKernelGGL(k_rd_pwv_mean, dim3(1), dim3(kRdThreads), 0, s, a);
  hipLaunchKernelGGL(k_rd_channel, dim3(a.K), dim3(kRdThreads), 0, s, a);
}

void launch_reduce_common(const ReduceArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_rd_common,
                     dim3((unsigned)((a.T + kRdThreads - 1) / kRdThreads),
                          (a.kg + kRdChan - 1) / kRdChan),
                     dim3(kRdThreads), 0, s, a);
}

int launch_reduce_grid(const ReduceArgs& a, hipStream_t s) {
  const int C = a.map_n * a.map_n;
  const size_t lds = (size_t)C * (2 * kRdGridChan * sizeof(double) + sizeof(unsigned));
  if (hipFuncSetAttribute((const void*)k_rd_grid,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 1;
  const int groups = (a.kg + kRdGridChan - 1) / kRdGridChan;
  hipLaunchKernelGGL(k_rd_grid, dim3((unsigned)(a.P * groups)), dim3(kRdThreads), lds, s, a);
  return 0;
}

void launch_reduce_combine(const ReduceArgs& a, hipStream_t s) {
  const int C = a.map_n * a.map_n;
  hipLaunchKernelGGL(k_rd_combine, dim3((C + kRdThreads - 1) / kRdThreads, a.kg),
                     dim3(kRdThreads), 0, s, a);
}

}  // namespace gtod
