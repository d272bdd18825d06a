// Panel kernel: per (row, nu) spectral power deviation dP = P - Pref.
//
// Per row (one pixel at one time sample), in FP64 (section 2.4):
//   t = n / f_sample; scan offsets (phi, theta) from the pattern;
//   screen position x = h tan(phi + dphi) + u_w t, y = h tan(theta + dtheta)
//   (Eq. xy_atm) -> bilinear PWV on the screen; table row and weight of
//   that PWV; cosecant of the elevation theta + theta0 + dtheta (Eq.
//   airmass); source cell and weights at the full pointing (zero outside).
// Per (row, nu), in FP32, coalesced along nu:
//   tau_z = (1-w) tau[i][nu] + w tau[i+1][nu]    optical-depth interpolation
//   xi    = -expm1(-csc tau_z)                     1 - eta_z^csc
//   P     = E + xi D + (1 - xi) W P_src            collapsed cascade
//   dP    = P - Pref
// A workgroup handles kPanelRows rows; threads stride over nu so that every
// table, cube and panel access is a contiguous run along nu.
#include <hip/hip_runtime.h>

#include "gtod_internal.h"
#include "scan.h"

namespace gtod {

namespace {

struct RowInfo {
  int valid;
  int li;          // table row below the PWV
  float lw;        // weight of the row above
  float csc;
  int src;         // pointing inside the source grid
  float wa, we;    // source weights along az / el
  int64_t sbase;   // offset of corner (el, az) in the cube
};

__device__ inline void clamp_cell(double g, int64_t n, int64_t* cell,
                                  double* w, bool* clamped) {
  const double gc = fmin(fmax(g, 0.0), (double)(n - 1));
  *clamped = (gc != g);
  int64_t c = (int64_t)floor(gc);
  if (c > n - 2) c = n - 2;
  *cell = c;
  *w = gc - (double)c;
}

}  // namespace

__global__ __launch_bounds__(256) void k_panel(PanelArgs a) {
  __shared__ RowInfo ri[kPanelRows];
  const int64_t row0 = (int64_t)blockIdx.x * kPanelRows;

  if (threadIdx.x < kPanelRows) {
    RowInfo q{};
    const int64_t r = row0 + threadIdx.x;
    const int pl = (int)(r / a.Tpad);
    const int tl = (int)(r % a.Tpad);
    q.valid = (pl < a.n_pix) && (tl < a.Tc);
    if (q.valid) {
      const int p = a.p0 + pl;
      const int64_t n = a.t0 + tl;
      const double t = (double)n / a.f_s;
      double phi, th;
      scan_offsets(a.scan_kind, a.r_petal, a.omega, a.Omega, a.traj, n, a.f_s,
                   &phi, &th);
      const double x = a.h * tan(phi + a.dphi[p]) + a.wind * t;
      const double y = a.h * tan(th + a.dtheta[p]);
      int64_t cx, cy;
      double wx, wy;
      bool ox, oy;
      clamp_cell(x / a.dx + a.ix0, a.nx, &cx, &wx, &ox);
      clamp_cell(y / a.dy + a.iy0, a.ny, &cy, &wy, &oy);
      const double* s0 = a.scr + cy * a.nx + cx;
      const double pwv = (1.0 - wx) * (1.0 - wy) * s0[0] + wx * (1.0 - wy) * s0[1] +
                         (1.0 - wx) * wy * s0[a.nx] + wx * wy * s0[a.nx + 1];
      if (ox || oy) atomicAdd(&a.counters[0], 1ull);
      if (a.pwv_out) a.pwv_out[(int64_t)p * a.out_ld + (n - a.out_t0)] = (float)pwv;
      int64_t li;
      double lw;
      bool ol;
      clamp_cell((pwv - a.pwv0) / a.dpwv, a.n_pwv, &li, &lw, &ol);
      if (ol) atomicAdd(&a.counters[1], 1ull);
      q.li = (int)li;
      q.lw = (float)lw;
      const double el = th + a.theta0 + a.dtheta[p];
      q.csc = (float)(1.0 / sin(el));
      q.src = 0;
      if (a.cube) {
        const double az = phi + a.phi0 + a.dphi[p];
        const double ga = (az - a.az0) / a.daz;
        const double ge = (el - a.el0) / a.del;
        if (ga >= 0.0 && ga <= (double)(a.n_az - 1) && ge >= 0.0 &&
            ge <= (double)(a.n_el - 1)) {
          int64_t ca, ce;
          double wa, we;
          bool d0, d1;
          clamp_cell(ga, a.n_az, &ca, &wa, &d0);
          clamp_cell(ge, a.n_el, &ce, &we, &d1);
          q.src = 1;
          q.wa = (float)wa;
          q.we = (float)we;
          q.sbase = (ce * a.n_az + ca) * a.cube_ld;
        }
      }
    }
    ri[threadIdx.x] = q;
  }
  __syncthreads();

  const int64_t Fp = a.Fp;
  for (int j = threadIdx.x; j < a.Fp; j += blockDim.x) {
    const bool inF = j < a.F;
    const float E = a.E[j], D = a.D[j], W = a.W[j], Pr = a.Pref[j];
#pragma unroll 2
    for (int rr = 0; rr < kPanelRows; ++rr) {
      const RowInfo& q = ri[rr];
      float dP = 0.f;
      if (q.valid && inF) {
        const float t0v = a.tau[(int64_t)q.li * Fp + j];
        const float t1v = a.tau[(int64_t)(q.li + 1) * Fp + j];
        const float tz = (1.f - q.lw) * t0v + q.lw * t1v;
        const float xi = -expm1f(-q.csc * tz);
        float P = E + xi * D;
        if (q.src) {
          const float* c = a.cube + q.sbase + j;
          const int64_t ld = a.cube_ld, row = (int64_t)a.n_az * a.cube_ld;
          const float ps = (1.f - q.wa) * (1.f - q.we) * c[0] +
                           q.wa * (1.f - q.we) * c[ld] +
                           (1.f - q.wa) * q.we * c[row] + q.wa * q.we * c[row + ld];
          P += (1.f - xi) * (W * ps);
        }
        dP = P - Pr;
      }
      a.panel[(row0 + rr) * Fp + j] = dP;
    }
  }
}

void launch_panel(const PanelArgs& a, hipStream_t s) {
  const int64_t rows = (int64_t)a.n_pix * a.Tpad;
  const int64_t blocks = rows / kPanelRows;
  hipLaunchKernelGGL(k_panel, dim3((unsigned)blocks), dim3(256), 0, s, a);
}

}  // namespace gtod
