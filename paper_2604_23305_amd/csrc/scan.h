// Scan pattern offsets (phi(t), theta(t)) at absolute sample n (section
// 2.4): stare (0, 0); daisy (Eq. daisy) with t = n / f_s; a user
// trajectory traj[n] = (phi, theta).  FP64.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gtod {

__device__ inline void scan_offsets(int kind, double r_petal, double omega,
                                    double Omega, const double* traj,
                                    int64_t n, double f_s, double* phi,
                                    double* th) {
  *phi = 0.0;
  *th = 0.0;
  if (kind == 1) {
    const double t = (double)n / f_s;
    const double sw = sin(omega * t);
    *phi = r_petal * cos(Omega * t) * sw;
    *th = r_petal * sin(Omega * t) * sw;
  } else if (kind == 2) {
    *phi = traj[2 * n];
    *th = traj[2 * n + 1];
  }
}

}  // namespace gtod
