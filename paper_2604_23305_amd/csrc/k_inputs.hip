// Input preparation (section 2.2): far-field pattern of the Gaussian-tapered
// aperture, source-beam convolution (Eq. convolve_src) and footprint
// smoothing of the PWV screen.
//
// Aperture (Eq. aper_dist): A(r) = 10^(t_edge (r / R)^2 / 20) for r < R.
// Far field: F = |FT{A}|^2 / peak.  For a circularly symmetric field the
// two-dimensional transform is the Hankel transform
//   H(rho) = int_0^R A(r) J0(2 pi rho r / lambda) r dr,   F = (H / H(0))^2,
// evaluated with Gauss-Legendre quadrature on [0, R] (the node count is
// chosen by the runtime from the largest 2 pi rho R / lambda of the grid).
// Source: P(i, j) = A_p daz del sum_{i', j'} I(i', j') cos(el_j') F(rho),
// rho = sqrt(((i - i') daz)^2 + ((j - j') del)^2): one block per (frequency,
// 32x32 output tile) holding the frequency's weighted intensity plane and
// its far-field table F[|dj|][|di|] in LDS; each thread sums 2x2 outputs
// in FP64.  Screen: weights A(r) normalised to 1 over the cells within R;
// one block per 32x64 output tile with its halo in LDS, edges clamped.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gtod_internal.h"

namespace gtod {

namespace {

constexpr double kC = 299792458.0;
constexpr double kPi = 3.14159265358979323846;

__device__ inline double aperture(double r, double R, double t_edge_db) {
  if (r >= R) return 0.0;
  const double q = r / R;
  return exp10(t_edge_db * q * q / 20.0);
}

}  // namespace

// Gauss-Legendre nodes and weights on [0, 1]: Newton on P_n from the
// Chebyshev-like initial guess, one thread per node.
__global__ void k_gauss_legendre(double* x, double* w, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double z = cos(kPi * (i + 0.75) / (n + 0.5));
  double dp = 1.0;
  for (int it = 0; it < 100; ++it) {
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    const double dz = p1 / dp;
    z -= dz;
    if (fabs(dz) < 1e-16) break;
  }
  x[i] = 0.5 * (1.0 - z);
  w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
}

// One thread per (a, b, frequency).
__global__ __launch_bounds__(256) void k_beam_table(BeamArgs a) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t per = (int64_t)a.n_a * a.n_b;
  if (id >= per * a.F) return;
  const int f = (int)(id / per);
  const int rem = (int)(id % per);
  const int ib = rem / a.n_a, ia = rem % a.n_a;
  const double lam = kC / a.nu[f];
  const double rho = sqrt((ia * a.da) * (ia * a.da) + (ib * a.db) * (ib * a.db));
  const double k = 2.0 * kPi * rho / lam;
  double h = 0.0, h0 = 0.0;
  for (int n = 0; n < a.n_nodes; ++n) {
    const double r = a.r_tel * a.gl_x[n];
    const double g = a.gl_w[n] * aperture(r, a.r_tel, a.t_edge_db) * r;
    h0 += g;
    h += g * j0(k * r);
  }
  const double q = h / h0;
  a.table[id] = (float)(q * q);
}

// Block: frequency f0 + blockIdx.y, output tile blockIdx.x (32x32).
__global__ __launch_bounds__(256) void k_source_conv(SrcConvArgs a) {
  extern __shared__ float dyn[];
  const int nn = a.n_az * a.n_el;
  float* sI = dyn;          // [n_el][n_az] I cos(el)
  float* sF = dyn + nn;     // [n_el][n_az] F(|dj|, |di|)
  const int fl = blockIdx.y, f = a.f0 + fl;
  const int tiles_x = (a.n_az + 31) / 32;
  const int ti = (blockIdx.x % tiles_x) * 32, tj = (blockIdx.x / tiles_x) * 32;
  const float* tab = a.table + (int64_t)fl * nn;
  for (int q = threadIdx.x; q < nn; q += 256) {
    const int j = q / a.n_az;
    sI[q] = (float)((double)a.in[(int64_t)q * a.ld_in + f] * cos(a.el0 + j * a.del));
    sF[q] = tab[q];
  }
  __syncthreads();
  const int i0 = ti + (threadIdx.x & 15), j0_ = tj + (threadIdx.x >> 4);
  const int i1 = i0 + 16, j1 = j0_ + 16;
  double acc00 = 0.0, acc01 = 0.0, acc10 = 0.0, acc11 = 0.0;
  for (int jp = 0; jp < a.n_el; ++jp) {
    const float* rI = sI + jp * a.n_az;
    // rows beyond the grid only occur for outputs outside it (not stored);
    // clamping keeps their reads inside the table
    const float* rF0 = sF + min(abs(j0_ - jp), a.n_el - 1) * a.n_az;
    const float* rF1 = sF + min(abs(j1 - jp), a.n_el - 1) * a.n_az;
    for (int ip = 0; ip < a.n_az; ++ip) {
      const float v = rI[ip];
      const int e0 = min(abs(i0 - ip), a.n_az - 1), e1 = min(abs(i1 - ip), a.n_az - 1);
      acc00 += (double)(v * rF0[e0]);
      acc01 += (double)(v * rF0[e1]);
      acc10 += (double)(v * rF1[e0]);
      acc11 += (double)(v * rF1[e1]);
    }
  }
  auto put = [&](int i, int j, double acc) {
    if (i < a.n_az && j < a.n_el)
      a.out[((int64_t)j * a.n_az + i) * a.ld_out + f] = (float)(a.scale * acc);
  };
  put(i0, j0_, acc00);
  put(i1, j0_, acc01);
  put(i0, j1, acc10);
  put(i1, j1, acc11);
}

// Footprint weights A(r) over [2ry+1][2rx+1] cells, normalised to 1 (one
// block; fixed-order sum).
__global__ __launch_bounds__(256) void k_screen_weights(ScreenConvArgs a) {
  __shared__ double s[256];
  const int wx = 2 * a.rx + 1, n = wx * (2 * a.ry + 1);
  double acc = 0.0;
  for (int q = threadIdx.x; q < n; q += 256) {
    const double x = (q % wx - a.rx) * a.dx, y = (q / wx - a.ry) * a.dy;
    const double v = aperture(sqrt(x * x + y * y), a.r_tel, a.t_edge_db);
    a.w[q] = v;
    acc += v;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  const double inv = 1.0 / s[0];
  for (int q = threadIdx.x; q < n; q += 256) a.w[q] *= inv;
}

// Block: 32 x 64 outputs; thread (tx, ty) computes rows ty + 4r, r < 8,
// of column tx.
__global__ __launch_bounds__(256) void k_screen_conv(ScreenConvArgs a) {
  extern __shared__ double dsm[];
  const int wx = 2 * a.rx + 1, wy = 2 * a.ry + 1;
  const int TW = kScreenTileX + 2 * a.rx, TH = kScreenTileY + 2 * a.ry;
  double* sw = dsm;               // [wy][wx]
  double* st = dsm + wx * wy;     // [TH][TW]
  const int64_t tiles_x = (a.nx + kScreenTileX - 1) / kScreenTileX;
  const int64_t x0 = (blockIdx.x % tiles_x) * kScreenTileX;
  const int64_t y0 = (blockIdx.x / tiles_x) * kScreenTileY;
  for (int q = threadIdx.x; q < wx * wy; q += 256) sw[q] = a.w[q];
  for (int q = threadIdx.x; q < TW * TH; q += 256) {
    const int ty = q / TW, tx = q % TW;
    int64_t gy = y0 - a.ry + ty, gx = x0 - a.rx + tx;
    gy = gy < 0 ? 0 : (gy >= a.ny ? a.ny - 1 : gy);
    gx = gx < 0 ? 0 : (gx >= a.nx ? a.nx - 1 : gx);
    st[q] = a.in[gy * a.nx + gx];
  }
  __syncthreads();
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  double acc[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) acc[r] = 0.0;
  for (int dy = 0; dy < wy; ++dy) {
    for (int dx = 0; dx < wx; ++dx) {
      const double w = sw[dy * wx + dx];
      if (w == 0.0) continue;
      const double* col = st + (ty + dy) * TW + tx + dx;
#pragma unroll
      for (int r = 0; r < 8; ++r) acc[r] += w * col[4 * r * TW];
    }
  }
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int64_t y = y0 + ty + 4 * r, x = x0 + tx;
    if (y < a.ny && x < a.nx) a.out[y * a.nx + x] = acc[r];
  }
}

void launch_gauss_legendre(double* x, double* w, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_gauss_legendre, dim3((n + 127) / 128), dim3(128), 0, s, x, w, n);
}

void launch_beam_table(const BeamArgs& a, hipStream_t s) {
  const int64_t n = (int64_t)a.n_a * a.n_b * a.F;
  hipLaunchKernelGGL(k_beam_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
}

int launch_source_conv(const SrcConvArgs& a, hipStream_t s) {
  const size_t lds = (size_t)2 * a.n_az * a.n_el * sizeof(float);
  if (hipFuncSetAttribute((const void*)k_source_conv,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 1;
  const int tiles = ((a.n_az + 31) / 32) * ((a.n_el + 31) / 32);
  hipLaunchKernelGGL(k_source_conv, dim3(tiles, a.nf), dim3(256), lds, s, a);
  return 0;
}

void launch_screen_weights(const ScreenConvArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_screen_weights, dim3(1), dim3(256), 0, s, a);
}

int launch_screen_conv(const ScreenConvArgs& a, hipStream_t s) {
  const int wx = 2 * a.rx + 1, wy = 2 * a.ry + 1;
  const size_t lds = sizeof(double) * ((size_t)wx * wy +
                     (size_t)(kScreenTileX + 2 * a.rx) * (kScreenTileY + 2 * a.ry));
  if (hipFuncSetAttribute((const void*)k_screen_conv,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 1;
  const int64_t tiles = ((a.nx + kScreenTileX - 1) / kScreenTileX) *
                        ((a.ny + kScreenTileY - 1) / kScreenTileY);
  hipLaunchKernelGGL(k_screen_conv, dim3((unsigned)tiles), dim3(256), lds, s, a);
  return 0;
}

}  // namespace gtod
