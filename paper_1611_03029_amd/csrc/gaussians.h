// The analytic solution of the smooth-solution example (device code).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace mfl {

// The solution of the smooth-solution example (Sec. 4.3, eq. pois_analytic): three Gaussians
// of width alpha = 1/5, u = (alpha sqrt(2 pi))^-3 sum_j exp(-|x - x_j|^2 / alpha^2).
// Returns u, grad u and Laplace u (in 3D, Laplace exp(-r^2/a^2) = (4 r^2/a^4 - 6/a^2) exp).
__device__ inline void gaussians(const double x[3], double &u, double g[3], double &lap) {
  const double alpha = 0.2, ia2 = 1.0 / (alpha * alpha);
  const double centres[3][3] = {{-0.5, 0.5, 0.25}, {-0.6, -0.5, -0.125}, {0.5, -0.5, 0.5}};
  const double s = 1.0 / (alpha * sqrt(2.0 * M_PI)), scale = s * s * s;
  u = 0.0;
  lap = 0.0;
  g[0] = g[1] = g[2] = 0.0;
  for (int j = 0; j < 3; ++j) {
    const double d0 = x[0] - centres[j][0], d1 = x[1] - centres[j][1], d2 = x[2] - centres[j][2];
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    const double e = exp(-r2 * ia2);
    u += e;
    g[0] -= 2.0 * ia2 * d0 * e;
    g[1] -= 2.0 * ia2 * d1 * e;
    g[2] -= 2.0 * ia2 * d2 * e;
    lap += (4.0 * r2 * ia2 * ia2 - 6.0 * ia2) * e;
  }
  u *= scale;
  lap *= scale;
  g[0] *= scale;
  g[1] *= scale;
  g[2] *= scale;
}

}  // namespace mfl
