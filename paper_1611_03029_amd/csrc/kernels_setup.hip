// Setup kernels of the continuous Q_k operator (FP64): per-quadrature-point metric of
// curved cells, the matrix diagonal for the Jacobi smoother, and the right-hand sides of
// the sine problem and of the three-Gaussian example (Sec. 4.3, eq. pois_analytic).
#include <cmath>

#include "device_common.h"
#include "gaussians.h"

namespace mfl {

namespace {

constexpr int kBlock = 256;


// The strongly varying coefficient of Sec. 4.3, eq. (diffusivity_shell), with each cosine
// factor squared so that it is positive: 1 + amp prod_e cos^2(2 pi x_e + 0.1 e), e = 1..3.
__device__ __forceinline__ double cosine_field(const double x[3], double amp) {
  double p = 1.0;
  for (int e = 0; e < 3; ++e) {
    const double c = cos(2.0 * M_PI * x[e] + 0.1 * (e + 1));
    p *= c * c;
  }
  return 1.0 + amp * p;
}

// Per cell and Gauss point: node positions of the isoparametric map (Gauss-Lobatto
// support points of x + a sin(pi x) sin(pi y) sin(pi z) (1,1,1)), J_q = sum_i x_i (x)
// grad phi_i(xi_q), and G_q = w_q det J_q J_q^{-1} J_q^{-T}, stored [cell][6][q] in FP64
// and FP32 (components 00, 11, 22, 01, 02, 12).  With kfield the position-dependent
// coefficient at the image x_q = sum_i x_i phi_i(xi_q) of the Gauss point is folded into
// G_q.  A det J_q that is not positive raises kFlagDetJ in *flag.
template <int K>
__global__ void __launch_bounds__(kBlock)
metric_kernel(double *__restrict__ m64, float *__restrict__ m32, int Nc, double h, double amp,
              int kfield, double kamp, int *__restrict__ flag, Tab<K + 1, double> tb) {
  constexpr int n = K + 1, n3 = n * n * n;
  __shared__ double S[n * n], Sd[n * n], gll[n], w[n];
  for (int i = threadIdx.x; i < n * n; i += kBlock) {
    S[i] = tb.S[i];
    Sd[i] = tb.Sd[i];
  }
  if (threadIdx.x < n) {
    gll[threadIdx.x] = tb.gll[threadIdx.x];
    w[threadIdx.x] = tb.w[threadIdx.x];
  }
  __syncthreads();
  const int64_t total = int64_t(Nc) * Nc * Nc * n3;
  for (int64_t id = blockIdx.x * int64_t(kBlock) + threadIdx.x; id < total;
       id += int64_t(gridDim.x) * kBlock) {
    const int64_t cell = id / n3;
    const int q = int(id - cell * n3), q0 = q % n, q1 = (q / n) % n, q2 = q / (n * n);
    const int c[3] = {int(cell % Nc), int((cell / Nc) % Nc), int(cell / (int64_t(Nc) * Nc))};
    double X[3][n], s1[3][n];
    for (int d = 0; d < 3; ++d)
      for (int i = 0; i < n; ++i) {
        X[d][i] = (c[d] + gll[i]) * h;
        s1[d][i] = sin(M_PI * X[d][i]);
      }
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, xq[3] = {0, 0, 0};
    for (int i2 = 0; i2 < n; ++i2)
      for (int i1 = 0; i1 < n; ++i1)
        for (int i0 = 0; i0 < n; ++i0) {
          const double disp = amp * s1[0][i0] * s1[1][i1] * s1[2][i2];
          const double xn[3] = {X[0][i0] + disp, X[1][i1] + disp, X[2][i2] + disp};
          const double phi = S[q0 * n + i0] * S[q1 * n + i1] * S[q2 * n + i2];
          const double dphi[3] = {Sd[q0 * n + i0] * S[q1 * n + i1] * S[q2 * n + i2],
                                  S[q0 * n + i0] * Sd[q1 * n + i1] * S[q2 * n + i2],
                                  S[q0 * n + i0] * S[q1 * n + i1] * Sd[q2 * n + i2]};
          for (int a = 0; a < 3; ++a) {
            xq[a] += xn[a] * phi;
            for (int b = 0; b < 3; ++b) J[a][b] += xn[a] * dphi[b];
          }
        }
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(det > 0.0) || !isfinite(det)) atomicOr(flag, int(kFlagDetJ));
    double Ji[3][3];
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    const double wd = w[q0] * w[q1] * w[q2] * det * (kfield ? cosine_field(xq, kamp) : 1.0);
    const int cc[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    for (int e = 0; e < 6; ++e) {
      const int a = cc[e][0], b = cc[e][1];
      const double v = wd * (Ji[a][0] * Ji[b][0] + Ji[a][1] * Ji[b][1] + Ji[a][2] * Ji[b][2]);
      m64[cell * (6 * n3) + e * n3 + q] = v;
      m32[cell * (6 * n3) + e * n3 + q] = float(v);
    }
  }
}

// diag(A) contributions of Cartesian cells: kappa h (K_aa M_bb M_ll + M_aa K_bb M_ll +
// M_aa M_bb K_ll); assembled with atomics (Dirichlet DoFs skipped, set by the finalize).
template <int K>
__global__ void __launch_bounds__(kBlock)
diag_cart_kernel(double *__restrict__ diag, const double *__restrict__ kappa, int Nc, int N1,
                 double h, int dmask, Tab<K + 1, double> tb) {
  constexpr int n = K + 1, n3 = n * n * n;
  __shared__ double Md[n], Kd[n];
  if (threadIdx.x < n) {
    Md[threadIdx.x] = tb.M[threadIdx.x * n + threadIdx.x];
    Kd[threadIdx.x] = tb.K[threadIdx.x * n + threadIdx.x];
  }
  __syncthreads();
  const int64_t total = int64_t(Nc) * Nc * Nc * n3;
  const int64_t plane = int64_t(N1) * N1;
  for (int64_t id = blockIdx.x * int64_t(kBlock) + threadIdx.x; id < total;
       id += int64_t(gridDim.x) * kBlock) {
    const int64_t cell = id / n3;
    const int i = int(id - cell * n3), a = i % n, b = (i / n) % n, l = i / (n * n);
    const int gx = int(cell % Nc) * K + a, gy = int((cell / Nc) % Nc) * K + b,
              gz = int(cell / (int64_t(Nc) * Nc)) * K + l;
    if (dirichlet_dof(gx, gy, gz, N1, dmask)) continue;
    const double v = kappa[cell] * h *
                     (Kd[a] * Md[b] * Md[l] + Md[a] * Kd[b] * Md[l] + Md[a] * Md[b] * Kd[l]);
    atomic_add(diag + gx + N1 * int64_t(gy) + plane * gz, v);
  }
}

// diag(A) contributions of curved cells: sum_q kappa grad phi_i(q) . G_q grad phi_i(q).
template <int K>
__global__ void __launch_bounds__(kBlock)
diag_curved_kernel(double *__restrict__ diag, const double *__restrict__ kappa,
                   const double *__restrict__ metric, int Nc, int N1, int dmask,
                   Tab<K + 1, double> tb) {
  constexpr int n = K + 1, n3 = n * n * n;
  __shared__ double S[n * n], Sd[n * n];
  for (int i = threadIdx.x; i < n * n; i += kBlock) {
    S[i] = tb.S[i];
    Sd[i] = tb.Sd[i];
  }
  __syncthreads();
  const int64_t total = int64_t(Nc) * Nc * Nc * n3;
  const int64_t plane = int64_t(N1) * N1;
  for (int64_t id = blockIdx.x * int64_t(kBlock) + threadIdx.x; id < total;
       id += int64_t(gridDim.x) * kBlock) {
    const int64_t cell = id / n3;
    const int i = int(id - cell * n3), a = i % n, b = (i / n) % n, l = i / (n * n);
    const int gx = int(cell % Nc) * K + a, gy = int((cell / Nc) % Nc) * K + b,
              gz = int(cell / (int64_t(Nc) * Nc)) * K + l;
    if (dirichlet_dof(gx, gy, gz, N1, dmask)) continue;
    const double *G = metric + cell * (6 * n3);
    double acc = 0;
    for (int q = 0; q < n3; ++q) {
      const int q0 = q % n, q1 = (q / n) % n, q2 = q / (n * n);
      const double d0 = Sd[q0 * n + a] * S[q1 * n + b] * S[q2 * n + l];
      const double d1 = S[q0 * n + a] * Sd[q1 * n + b] * S[q2 * n + l];
      const double d2 = S[q0 * n + a] * S[q1 * n + b] * Sd[q2 * n + l];
      acc += G[q] * d0 * d0 + G[n3 + q] * d1 * d1 + G[2 * n3 + q] * d2 * d2 +
             2.0 * (G[3 * n3 + q] * d0 * d1 + G[4 * n3 + q] * d0 * d2 + G[5 * n3 + q] * d1 * d2);
    }
    atomic_add(diag + gx + N1 * int64_t(gy) + plane * gz, kappa[cell] * acc);
  }
}

// Node displacements d = amp sin(pi x) sin(pi y) sin(pi z) of the curved map x = X + d (1,1,1)
// at the CG nodes of a level (node coordinates and product order of metric_kernel), in FP64
// and FP32: the geometry data of the on-the-fly metric.
template <int K>
__global__ void __launch_bounds__(kBlock)
disp_kernel(double *__restrict__ d64, float *__restrict__ d32, int Nc, int N1, double h, double amp,
            Tab<K + 1, double> tb) {
  const int64_t total = int64_t(N1) * N1 * N1;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < total; i += int64_t(gridDim.x) * kBlock) {
    const int g[3] = {int(i % N1), int((i / N1) % N1), int(i / (int64_t(N1) * N1))};
    double sn[3];
    for (int e = 0; e < 3; ++e) {
      const int c = min(g[e] / K, Nc - 1);
      sn[e] = sin(M_PI * ((c + tb.gll[g[e] - c * K]) * h));
    }
    const double v = amp * sn[0] * sn[1] * sn[2];
    d64[i] = v;
    d32[i] = float(v);
  }
}

// Setup-time metric of one cell from its node displacements (one work-group per cell, direct
// tensor sums): with g = grad d at Gauss point q and s = g . (1,1,1), J = h I + (1,1,1) g^T,
// det J = h^2 (h + s) and G = w [(h + s) I - (1 g^T + g 1^T) + |g|^2 / (h + s) 1 1^T], stored to
// G[e n^3 + q] (e: 00, 11, 22, 01, 02, 12).  Raises kFlagDetJ for a determinant that is not
// positive or not finite.  dl: the cell's n^3 displacements (local lexicographic).
template <int K>
__device__ void otf_cell_metric(const double *dl, double *G, const double *S, const double *Sd, const double *w,
                                double h, int *flag) {
  constexpr int n = K + 1, n3 = n * n * n;
  for (int q = threadIdx.x; q < n3; q += kBlock) {
    const int q0 = q % n, q1 = (q / n) % n, q2 = q / (n * n);
    double g[3] = {0, 0, 0};
    for (int i2 = 0; i2 < n; ++i2)
      for (int i1 = 0; i1 < n; ++i1)
        for (int i0 = 0; i0 < n; ++i0) {
          const double di = dl[i0 + n * (i1 + n * i2)];
          g[0] += di * Sd[q0 * n + i0] * S[q1 * n + i1] * S[q2 * n + i2];
          g[1] += di * S[q0 * n + i0] * Sd[q1 * n + i1] * S[q2 * n + i2];
          g[2] += di * S[q0 * n + i0] * S[q1 * n + i1] * Sd[q2 * n + i2];
        }
    const double hs = h + (g[0] + g[1] + g[2]);
    const double det = h * h * hs;
    if (!(det > 0.0) || !isfinite(det)) atomicOr(flag, int(kFlagDetJ));
    const double t = (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) / hs;
    const double wq = w[q0] * w[q1] * w[q2];
    G[0 * n3 + q] = wq * (hs - 2.0 * g[0] + t);
    G[1 * n3 + q] = wq * (hs - 2.0 * g[1] + t);
    G[2 * n3 + q] = wq * (hs - 2.0 * g[2] + t);
    G[3 * n3 + q] = wq * (t - g[0] - g[1]);
    G[4 * n3 + q] = wq * (t - g[0] - g[2]);
    G[5 * n3 + q] = wq * (t - g[1] - g[2]);
  }
}

// One work-group per curved cell with the on-the-fly metric: the Jacobian check at setup
// (diag == nullptr) or, in addition, the cell's contributions to diag(A) as in
// diag_curved_kernel.
template <int K>
__global__ void __launch_bounds__(kBlock)
otf_cell_kernel(double *__restrict__ diag, const double *__restrict__ kappa, const double *__restrict__ disp,
                int Nc, int N1, double h, int dmask, int *__restrict__ flag, Tab<K + 1, double> tb) {
  constexpr int n = K + 1, n3 = n * n * n;
  __shared__ double S[n * n], Sd[n * n], w[n], dl[n3], G[6 * n3];
  for (int i = threadIdx.x; i < n * n; i += kBlock) {
    S[i] = tb.S[i];
    Sd[i] = tb.Sd[i];
  }
  if (threadIdx.x < n) w[threadIdx.x] = tb.w[threadIdx.x];
  const int64_t cell = blockIdx.x;
  const int cx = int(cell % Nc), cy = int((cell / Nc) % Nc), cz = int(cell / (int64_t(Nc) * Nc));
  const int64_t plane = int64_t(N1) * N1;
  for (int i = threadIdx.x; i < n3; i += kBlock) {
    const int a = i % n, b = (i / n) % n, l = i / (n * n);
    dl[i] = disp[(cx * K + a) + N1 * int64_t(cy * K + b) + plane * (cz * K + l)];
  }
  __syncthreads();
  otf_cell_metric<K>(dl, G, S, Sd, w, h, flag);
  if (!diag) return;
  __syncthreads();
  for (int i = threadIdx.x; i < n3; i += kBlock) {
    const int a = i % n, b = (i / n) % n, l = i / (n * n);
    const int gx = cx * K + a, gy = cy * K + b, gz = cz * K + l;
    if (dirichlet_dof(gx, gy, gz, N1, dmask)) continue;
    double acc = 0;
    for (int q = 0; q < n3; ++q) {
      const int q0 = q % n, q1 = (q / n) % n, q2 = q / (n * n);
      const double d0 = Sd[q0 * n + a] * S[q1 * n + b] * S[q2 * n + l];
      const double d1 = S[q0 * n + a] * Sd[q1 * n + b] * S[q2 * n + l];
      const double d2 = S[q0 * n + a] * S[q1 * n + b] * Sd[q2 * n + l];
      acc += G[q] * d0 * d0 + G[n3 + q] * d1 * d1 + G[2 * n3 + q] * d2 * d2 +
             2.0 * (G[3 * n3 + q] * d0 * d1 + G[4 * n3 + q] * d0 * d2 + G[5 * n3 + q] * d1 * d2);
    }
    atomic_add(diag + gx + N1 * int64_t(gy) + plane * gz, kappa[cell] * acc);
  }
}

// f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z): the forcing of u = sin sin sin.
struct SineForcing {
  __device__ double operator()(const double x[3]) const {
    return 3.0 * M_PI * M_PI * sin(M_PI * x[0]) * sin(M_PI * x[1]) * sin(M_PI * x[2]);
  }
};

// f = -Laplace(u) of the three-Gaussian solution.
struct GaussianForcing {
  __device__ double operator()(const double x[3]) const {
    double u, g[3], lap;
    gaussians(x, u, g, lap);
    return -lap;
  }
};

// Right-hand side b_i = sum_q w_q det J_q f(x_q) phi_i(xi_q), with x_q the isoparametric
// image of the Gauss point (cells of [lo, lo + Nc h]^3).  DoFs on Dirichlet faces are
// skipped.  One work-group per cell.
template <int K, class F>
__global__ void __launch_bounds__(kBlock)
rhs_kernel(double *__restrict__ b, int Nc, int N1, double h, double lo, double amp, int dmask,
           Tab<K + 1, double> tb) {
  constexpr int n = K + 1, n3 = n * n * n;
  __shared__ double S[n * n], Sd[n * n], gll[n], w[n], fw[n3];
  for (int i = threadIdx.x; i < n * n; i += kBlock) {
    S[i] = tb.S[i];
    Sd[i] = tb.Sd[i];
  }
  if (threadIdx.x < n) {
    gll[threadIdx.x] = tb.gll[threadIdx.x];
    w[threadIdx.x] = tb.w[threadIdx.x];
  }
  __syncthreads();
  const int64_t cell = blockIdx.x;
  const int c[3] = {int(cell % Nc), int((cell / Nc) % Nc), int(cell / (int64_t(Nc) * Nc))};
  for (int q = threadIdx.x; q < n3; q += kBlock) {
    const int q0 = q % n, q1 = (q / n) % n, q2 = q / (n * n);
    if (amp == 0.0) {
      // affine cell: x_q = lo + (c + xi_q) h, det J = h^3
      const double xq[3] = {lo + (c[0] + tb.xg[q0]) * h, lo + (c[1] + tb.xg[q1]) * h, lo + (c[2] + tb.xg[q2]) * h};
      fw[q] = w[q0] * w[q1] * w[q2] * h * h * h * F()(xq);
      continue;
    }
    double X[3][n], s1[3][n];
    for (int d = 0; d < 3; ++d)
      for (int i = 0; i < n; ++i) {
        X[d][i] = lo + (c[d] + gll[i]) * h;
        s1[d][i] = sin(M_PI * X[d][i]);
      }
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, xq[3] = {0, 0, 0};
    for (int i2 = 0; i2 < n; ++i2)
      for (int i1 = 0; i1 < n; ++i1)
        for (int i0 = 0; i0 < n; ++i0) {
          const double disp = amp * s1[0][i0] * s1[1][i1] * s1[2][i2];
          const double xn[3] = {X[0][i0] + disp, X[1][i1] + disp, X[2][i2] + disp};
          const double phi = S[q0 * n + i0] * S[q1 * n + i1] * S[q2 * n + i2];
          const double dphi[3] = {Sd[q0 * n + i0] * S[q1 * n + i1] * S[q2 * n + i2],
                                  S[q0 * n + i0] * Sd[q1 * n + i1] * S[q2 * n + i2],
                                  S[q0 * n + i0] * S[q1 * n + i1] * Sd[q2 * n + i2]};
          for (int a = 0; a < 3; ++a) {
            xq[a] += xn[a] * phi;
            for (int bb = 0; bb < 3; ++bb) J[a][bb] += xn[a] * dphi[bb];
          }
        }
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    fw[q] = w[q0] * w[q1] * w[q2] * det * F()(xq);
  }
  __syncthreads();
  const int64_t plane = int64_t(N1) * N1;
  for (int i = threadIdx.x; i < n3; i += kBlock) {
    const int a = i % n, bb = (i / n) % n, l = i / (n * n);
    const int gx = c[0] * K + a, gy = c[1] * K + bb, gz = c[2] * K + l;
    if (dirichlet_dof(gx, gy, gz, N1, dmask)) continue;
    double s = 0;
    for (int q = 0; q < n3; ++q) {
      const int q0 = q % n, q1 = (q / n) % n, q2 = q / (n * n);
      s += S[q0 * n + a] * S[q1 * n + bb] * S[q2 * n + l] * fw[q];
    }
    atomic_add(b + gx + N1 * int64_t(gy) + plane * gz, s);
  }
}

// Neumann loads int_F g_N phi_i, g_N = grad u . n of the three-Gaussian solution (n the
// outward normal), on the boundary faces without Dirichlet conditions of a Cartesian mesh
// of [lo, lo + Nc h]^3.  One work-group per (domain face, cell face on it); k+1 Gauss
// points per tangential direction; the face basis functions are products of the
// tangential GLL bases.  Block b: face f = b / Nc^2 (direction f % 3, side f / 3).
template <int K>
__global__ void __launch_bounds__(kBlock)
neumann_face_kernel(double *__restrict__ b, int Nc, int N1, double h, double lo, int dmask,
                    Tab<K + 1, double> tb) {
  constexpr int n = K + 1;
  __shared__ double gw[n * n];
  const int64_t per_face = int64_t(Nc) * Nc;
  const int face = int(blockIdx.x / per_face);
  const int e = face % 3, side = face / 3;
  if ((dmask >> side) & 1) return;   // Dirichlet face: no load (uniform per work-group)
  const int64_t r = blockIdx.x - face * per_face;
  const int ta = e == 0 ? 1 : 0, tb2 = e == 2 ? 1 : 2;   // tangential directions
  int c[3];
  c[e] = side ? Nc - 1 : 0;
  c[ta] = int(r % Nc);
  c[tb2] = int(r / Nc);
  for (int q = threadIdx.x; q < n * n; q += kBlock) {
    const int q1 = q % n, q2 = q / n;
    double x[3], u, g[3], lap;
    x[e] = lo + (c[e] + side) * h;
    x[ta] = lo + (c[ta] + tb.xg[q1]) * h;
    x[tb2] = lo + (c[tb2] + tb.xg[q2]) * h;
    gaussians(x, u, g, lap);
    gw[q] = tb.w[q1] * tb.w[q2] * h * h * (side ? g[e] : -g[e]);
  }
  __syncthreads();
  const int64_t plane = int64_t(N1) * N1;
  for (int i = threadIdx.x; i < n * n; i += kBlock) {
    const int i1 = i % n, i2 = i / n;
    int gi[3];
    gi[e] = c[e] * K + (side ? K : 0);
    gi[ta] = c[ta] * K + i1;
    gi[tb2] = c[tb2] * K + i2;
    if (dirichlet_dof(gi[0], gi[1], gi[2], N1, dmask)) continue;
    double s = 0;
    for (int q = 0; q < n * n; ++q) s += tb.S[(q % n) * n + i1] * tb.S[(q / n) * n + i2] * gw[q];
    atomic_add(b + gi[0] + N1 * int64_t(gi[1]) + plane * gi[2], s);
  }
}

// x0 = u (three-Gaussian solution) interpolated at the Dirichlet DoFs of a Cartesian mesh,
// 0 elsewhere.  Grid line g lies at lo + (c + gll[g - c K]) h, c = min(g / K, Nc - 1).
template <int K>
__global__ void __launch_bounds__(kBlock)
gaussian_dirichlet_kernel(double *__restrict__ x0, int Nc, int N1, double h, double lo, int dmask,
                          Tab<K + 1, double> tb) {
  const int64_t nd = int64_t(N1) * N1 * N1;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < nd; i += int64_t(gridDim.x) * kBlock) {
    const int g[3] = {int(i % N1), int((i / N1) % N1), int(i / (int64_t(N1) * N1))};
    double v = 0.0;
    if (dirichlet_dof(g[0], g[1], g[2], N1, dmask)) {
      double x[3], gr[3], lap;
      for (int d = 0; d < 3; ++d) {
        const int c = min(g[d] / K, Nc - 1);
        x[d] = lo + (c + tb.gll[g[d] - c * K]) * h;
      }
      gaussians(x, v, gr, lap);
    }
    x0[i] = v;
  }
}

// b = x0 on Dirichlet DoFs, b - a0 elsewhere (a0 = A0 x0, the lifting of the Dirichlet data).
__global__ void __launch_bounds__(kBlock)
lift_kernel(double *__restrict__ b, const double *__restrict__ x0, const double *__restrict__ a0, int N1,
            int dmask) {
  const int64_t nd = int64_t(N1) * N1 * N1;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < nd; i += int64_t(gridDim.x) * kBlock) {
    const int x = int(i % N1), y = int((i / N1) % N1), z = int(i / (int64_t(N1) * N1));
    b[i] = dirichlet_dof(x, y, z, N1, dmask) ? x0[i] : b[i] - a0[i];
  }
}

inline int grid_for(int64_t items, int cap = 65536) {
  int64_t g = (items + kBlock - 1) / kBlock;
  return int(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_metric_setup(const Context &c, const Level &L, hipStream_t s) {
  const int64_t items = L.ncells * int64_t(c.n) * c.n * c.n;
  if (metric_on_the_fly(c.p)) {
    // node displacements, then the Jacobian check of every cell
#define CASE(K)                                                                                  \
  disp_kernel<K><<<grid_for(L.ndofs), kBlock, 0, s>>>(L.disp64, L.disp32, L.Nc, L.N1, L.h, c.p.curve_amp, \
                                                      shrink_tab<K + 1, double>(c.tab64));       \
  otf_cell_kernel<K><<<int(L.ncells), kBlock, 0, s>>>(nullptr, nullptr, L.disp64, L.Nc, L.N1, L.h, 0, c.flags, \
                                                      shrink_tab<K + 1, double>(c.tab64));       \
  break
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
    return hipGetLastError();
  }
#define CASE(K)                                                                                \
  metric_kernel<K><<<grid_for(items), kBlock, 0, s>>>(                                          \
      L.metric64, L.metric32, L.Nc, L.h, c.p.curve_amp, c.p.kappa_field == MFL_KAPPA_COSINE,        \
      c.p.kappa_field_amp, c.flags, shrink_tab<K + 1, double>(c.tab64));                            \
  break
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipGetLastError();
}

hipError_t launch_cg_diagonal(const Context &c, const Level &L, hipStream_t s) {
  const int64_t items = L.ncells * int64_t(c.n) * c.n * c.n;
  const int dir = dirichlet_mask(c.p);
  hipError_t e = launch_fill(L.diag64, MFL_F64, L.ndofs, 0.0, s);
  if (e != hipSuccess) return e;
  if (c.p.geometry == MFL_GEOM_CURVED && metric_on_the_fly(c.p)) {
#define CASE(K)                                                                                  \
  otf_cell_kernel<K><<<int(L.ncells), kBlock, 0, s>>>(L.diag64, L.kappa64, L.disp64, L.Nc, L.N1, L.h, dir, \
                                                      c.flags, shrink_tab<K + 1, double>(c.tab64)); \
  break
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  } else if (c.p.geometry == MFL_GEOM_CURVED) {
#define CASE(K)                                                                                  \
  diag_curved_kernel<K><<<grid_for(items), kBlock, 0, s>>>(L.diag64, L.kappa64, L.metric64, L.Nc, \
                                                           L.N1, dir, shrink_tab<K + 1, double>(c.tab64)); \
  break
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  } else {
#define CASE(K)                                                                               \
  diag_cart_kernel<K><<<grid_for(items), kBlock, 0, s>>>(L.diag64, L.kappa64, L.Nc, L.N1, L.h,  \
                                                         dir, shrink_tab<K + 1, double>(c.tab64)); \
  break
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_diag_finalize(c, L, s);
}

hipError_t launch_rhs_sine(const Context &c, const Level &L, double *b, hipStream_t s) {
  hipError_t e = launch_fill(b, MFL_F64, L.ndofs, 0.0, s);
  if (e != hipSuccess) return e;
  const double amp = c.p.geometry == MFL_GEOM_CURVED ? c.p.curve_amp : 0.0;
#define CASE(K)                                                                              \
  rhs_kernel<K, SineForcing><<<int(L.ncells), kBlock, 0, s>>>(                                \
      b, L.Nc, L.N1, L.h, c.p.domain_lo, amp, dirichlet_mask(c.p), shrink_tab<K + 1, double>(c.tab64)); \
  break
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipGetLastError();
}

hipError_t launch_rhs_gaussians(const Context &c, const Level &L, double *b, hipStream_t s) {
  hipError_t e = launch_fill(b, MFL_F64, L.ndofs, 0.0, s);
  if (e != hipSuccess) return e;
  const int dm = dirichlet_mask(c.p);
  const int64_t faces = 6 * int64_t(L.Nc) * L.Nc;
#define CASE(K)                                                                              \
  rhs_kernel<K, GaussianForcing><<<int(L.ncells), kBlock, 0, s>>>(                            \
      b, L.Nc, L.N1, L.h, c.p.domain_lo, 0.0, dm, shrink_tab<K + 1, double>(c.tab64));        \
  neumann_face_kernel<K><<<int(faces), kBlock, 0, s>>>(b, L.Nc, L.N1, L.h, c.p.domain_lo, dm, \
                                                       shrink_tab<K + 1, double>(c.tab64));   \
  break
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipGetLastError();
}

hipError_t launch_gaussian_dirichlet(const Context &c, const Level &L, double *x0, hipStream_t s) {
  const int dm = dirichlet_mask(c.p);
#define CASE(K)                                                                              \
  gaussian_dirichlet_kernel<K><<<grid_for(L.ndofs, 16384), kBlock, 0, s>>>(                   \
      x0, L.Nc, L.N1, L.h, c.p.domain_lo, dm, shrink_tab<K + 1, double>(c.tab64));             \
  break
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipGetLastError();
}

hipError_t launch_lift(const Context &c, const Level &L, double *b, const double *x0, const double *a0,
                       hipStream_t s) {
  lift_kernel<<<grid_for(L.ndofs, 16384), kBlock, 0, s>>>(b, x0, a0, L.N1, dirichlet_mask(c.p));
  return hipGetLastError();
}

}  // namespace mfl
