// Continuous Q_k Laplacian on hexahedra: matrix-free cell kernels (Sec. 3, eq. mf_eval).
//
// Thread layout shared by the cell kernels: a work-group of 256 lanes holds
// CPB = floor(256 / n^2) cells, n^2 lanes per cell (n = k+1).  Each lane owns one line
// of n points of its cell and keeps it in registers; the 1D contractions along that line
// run on registers with the 1D matrices as uniform (scalar) operands.  Between
// contraction directions the cell's n^3 values are transposed through LDS, so every LDS
// value is written once and read once per direction change.  Lanes are reinterpreted per
// phase as (x, y) owners of z-lines, (x, z) owners of y-lines or (y, z) owners of
// x-lines.  LDS index of point (x, y, z) of a cell: z n^2 + y n + x.
//
// The CG vector is gathered from and scattered to the lexicographic grid directly
// (indices are computed, no index table); contributions of cells sharing a DoF are
// combined with hardware FP64/FP32 atomic adds into a destination that the
// boundary-initialization kernel cleared first.  Dirichlet DoFs are read as zero
// (eliminated columns) and never written by the cell kernels (identity rows are set by
// the initialization kernel).
#include <cmath>

#include "device_common.h"

namespace mfl {

namespace {

constexpr int kBlock = 256;

template <int K>
struct Shape {
  static constexpr int n = K + 1, n2 = n * n, n3 = n2 * n, cpb = kBlock / n2;
};

// ---------------------------------------------------------------------------------------
// Cartesian cells: constant Jacobian h I, so with exact Gauss quadrature the element
// operator of eq. (mf_eval) factors into the Kronecker sum
//   A_e = kappa_e h (K (x) M (x) M + M (x) K (x) M + M (x) M (x) K)
// of the reference 1D mass M and stiffness K of the GLL basis (the same numbers as the
// quadrature form, re-associated).  Three contraction directions, 7 n^4 FMA per cell.
// GRAD: instead of scattering, reduce lambda_c^T A_c^{(kappa=1)} u_c per cell.
template <int K, typename T, bool GRAD>
__global__ void __launch_bounds__(kBlock)
cart_kernel(const T *__restrict__ src, T *__restrict__ dst, const T *__restrict__ kappa,
            const T *__restrict__ lam, T *__restrict__ grad, int Nc, int N1, T h, int dirichlet,
            Tab<K + 1, T> tb) {
  using S = Shape<K>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, CPB = S::cpb;
  __shared__ T sm[4][CPB * n3];
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int t = threadIdx.x, lc = t / n2, p = t - lc * n2, i0 = p % n, i1 = p / n;
  const int64_t ncell = int64_t(Nc) * Nc * Nc;
  const int64_t cell = int64_t(blk) * CPB + lc;
  const bool inblk = lc < CPB;
  const bool active = inblk && cell < ncell;
  int cx = 0, cy = 0, cz = 0;
  if (active) {
    cx = int(cell % Nc);
    cy = int((cell / Nc) % Nc);
    cz = int(cell / (int64_t(Nc) * Nc));
  }
  const int gx = cx * K + i0, gy = cy * K + i1;
  const bool bxy = dirichlet && (on_boundary(gx, N1) || on_boundary(gy, N1));
  const int64_t plane = int64_t(N1) * N1;
  const int64_t base = gx + int64_t(N1) * gy + plane * (int64_t(cz) * K);
  T *A = sm[0] + lc * n3, *B = sm[1] + lc * n3, *C = sm[2] + lc * n3, *D = sm[3] + lc * n3;

  // phase 1: z-lines (x = i0, y = i1): gather, then M and K along z
  if (inblk) {
    T u[n];
#pragma unroll
    for (int l = 0; l < n; ++l) {
      const bool bnd = bxy || (dirichlet && on_boundary(cz * K + l, N1));
      u[l] = (active && !bnd) ? src[base + plane * l] : T(0);
    }
#pragma unroll
    for (int q = 0; q < n; ++q) {
      T a = 0, b = 0;
#pragma unroll
      for (int l = 0; l < n; ++l) {
        a += tb.M[q * n + l] * u[l];
        b += tb.K[q * n + l] * u[l];
      }
      A[q * n2 + p] = a;
      B[q * n2 + p] = b;
    }
  }
  __syncthreads();
  // phase 2: y-lines (x = i0, z = i1): P = M_y (M_z u), S = K_y (M_z u) + M_y (K_z u)
  if (inblk) {
    T a1[n], a2[n];
#pragma unroll
    for (int b = 0; b < n; ++b) {
      a1[b] = A[i1 * n2 + b * n + i0];
      a2[b] = B[i1 * n2 + b * n + i0];
    }
#pragma unroll
    for (int q = 0; q < n; ++q) {
      T pp = 0, ss = 0;
#pragma unroll
      for (int b = 0; b < n; ++b) {
        pp += tb.M[q * n + b] * a1[b];
        ss += tb.K[q * n + b] * a1[b] + tb.M[q * n + b] * a2[b];
      }
      C[i1 * n2 + q * n + i0] = pp;
      D[i1 * n2 + q * n + i0] = ss;
    }
  }
  __syncthreads();
  // phase 3: x-lines (y = i0, z = i1): y = K_x P + M_x S, scaled by kappa h
  if (inblk) {
    T pa[n], sa[n];
#pragma unroll
    for (int a = 0; a < n; ++a) {
      pa[a] = C[i1 * n2 + i0 * n + a];
      sa[a] = D[i1 * n2 + i0 * n + a];
    }
    const T scale = GRAD ? h : (active ? kappa[cell] * h : T(0));
#pragma unroll
    for (int q = 0; q < n; ++q) {
      T y = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) y += tb.K[q * n + a] * pa[a] + tb.M[q * n + a] * sa[a];
      A[i1 * n2 + i0 * n + q] = y * scale;
    }
  }
  __syncthreads();
  // phase 4: z-lines again: scatter-add (or the per-cell gradient reduction)
  T partial = 0;
  if (active) {
#pragma unroll
    for (int l = 0; l < n; ++l) {
      const bool bnd = bxy || (dirichlet && on_boundary(cz * K + l, N1));
      const T v = A[l * n2 + p];
      if (!bnd) {
        if constexpr (GRAD)
          partial += v * lam[base + plane * l];
        else
          atomic_add(dst + base + plane * l, v);
      }
    }
  }
  if constexpr (GRAD) {
    if (inblk) B[p] = partial;
    __syncthreads();
    if (active && p == 0) {
      T s = 0;
      for (int j = 0; j < n2; ++j) s += B[j];
      grad[cell] = -s;
    }
  }
}

// ---------------------------------------------------------------------------------------
// Curved cells (general isoparametric geometry): the per-quadrature-point tensor
// G_q = w_q det J_q J_q^{-1} J_q^{-T} (6 unique entries, computed at setup and streamed
// from HBM; kappa_c applied on the fly).  Sum factorization in the collocation form:
// values at the Gauss points v = (S (x) S (x) S) u, reference gradient by the Gauss-point
// collocation derivative D in each direction, q = kappa G grad v, then the transposed
// sequence.  12 n^4 + 9 n^3 FMA per cell, 8 LDS transposes, 3 LDS buffers per cell.
template <int K, typename T, bool GRAD>
__global__ void __launch_bounds__(kBlock)
curved_kernel(const T *__restrict__ src, T *__restrict__ dst, const T *__restrict__ kappa,
              const T *__restrict__ metric, const T *__restrict__ lam, T *__restrict__ grad,
              int Nc, int N1, int dirichlet, Tab<K + 1, T> tb) {
  using S = Shape<K>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, CPB = S::cpb;
  __shared__ T sm[3][CPB * n3];
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int t = threadIdx.x, lc = t / n2, p = t - lc * n2, i0 = p % n, i1 = p / n;
  const int64_t ncell = int64_t(Nc) * Nc * Nc;
  const int64_t cell = int64_t(blk) * CPB + lc;
  const bool inblk = lc < CPB;
  const bool active = inblk && cell < ncell;
  int cx = 0, cy = 0, cz = 0;
  if (active) {
    cx = int(cell % Nc);
    cy = int((cell / Nc) % Nc);
    cz = int(cell / (int64_t(Nc) * Nc));
  }
  const int gx = cx * K + i0, gy = cy * K + i1;
  const bool bxy = dirichlet && (on_boundary(gx, N1) || on_boundary(gy, N1));
  const int64_t plane = int64_t(N1) * N1;
  const int64_t base = gx + int64_t(N1) * gy + plane * (int64_t(cz) * K);
  T *A = sm[0] + lc * n3, *B = sm[1] + lc * n3, *C = sm[2] + lc * n3;

  T g[6][n];
  T kap = 0;
  // F1: z-lines (x = i0, y = i1): gather, S along z; issue the metric loads early
  if (inblk) {
    T u[n];
#pragma unroll
    for (int l = 0; l < n; ++l) {
      const bool bnd = bxy || (dirichlet && on_boundary(cz * K + l, N1));
      u[l] = (active && !bnd) ? src[base + plane * l] : T(0);
    }
    const T *gm = metric + (active ? cell : 0) * (6 * n3) + p;
#pragma unroll
    for (int c = 0; c < 6; ++c)
#pragma unroll
      for (int l = 0; l < n; ++l) g[c][l] = active ? gm[c * n3 + l * n2] : T(0);
    kap = GRAD ? T(1) : (active ? kappa[cell] : T(0));
#pragma unroll
    for (int q = 0; q < n; ++q) {
      T a = 0;
#pragma unroll
      for (int l = 0; l < n; ++l) a += tb.S[q * n + l] * u[l];
      A[q * n2 + p] = a;
    }
  }
  __syncthreads();
  // F2: y-lines (x = i0, z = i1): S along y
  if (inblk) {
    T r[n];
#pragma unroll
    for (int b = 0; b < n; ++b) r[b] = A[i1 * n2 + b * n + i0];
#pragma unroll
    for (int q = 0; q < n; ++q) {
      T a = 0;
#pragma unroll
      for (int b = 0; b < n; ++b) a += tb.S[q * n + b] * r[b];
      B[i1 * n2 + q * n + i0] = a;
    }
  }
  __syncthreads();
  // F3: x-lines (y = i0, z = i1): S along x -> values v at Gauss points; D along x -> gx
  if (inblk) {
    T r[n], v[n];
#pragma unroll
    for (int a = 0; a < n; ++a) r[a] = B[i1 * n2 + i0 * n + a];
#pragma unroll
    for (int q = 0; q < n; ++q) {
      T a = 0;
#pragma unroll
      for (int j = 0; j < n; ++j) a += tb.S[q * n + j] * r[j];
      v[q] = a;
    }
#pragma unroll
    for (int q = 0; q < n; ++q) {
      T a = 0;
#pragma unroll
      for (int j = 0; j < n; ++j) a += tb.D[q * n + j] * v[j];
      A[i1 * n2 + i0 * n + q] = v[q];
      C[i1 * n2 + i0 * n + q] = a;
    }
  }
  __syncthreads();
  // F4: y-lines (x = i0, z = i1): D along y -> gy
  if (inblk) {
    T r[n];
#pragma unroll
    for (int b = 0; b < n; ++b) r[b] = A[i1 * n2 + b * n + i0];
#pragma unroll
    for (int q = 0; q < n; ++q) {
      T a = 0;
#pragma unroll
      for (int b = 0; b < n; ++b) a += tb.D[q * n + b] * r[b];
      B[i1 * n2 + q * n + i0] = a;
    }
  }
  __syncthreads();
  // F5 + B1: z-lines (x = i0, y = i1): D along z -> gz; quadrature-point operation;
  // first transposed derivative (along z).  Each lane rewrites only its own z-line.
  if (inblk) {
    T r[n], gz[n], fx[n], fy[n], fz[n];
#pragma unroll
    for (int l = 0; l < n; ++l) r[l] = A[l * n2 + p];
#pragma unroll
    for (int q = 0; q < n; ++q) {
      T a = 0;
#pragma unroll
      for (int l = 0; l < n; ++l) a += tb.D[q * n + l] * r[l];
      gz[q] = a;
    }
#pragma unroll
    for (int l = 0; l < n; ++l) {
      const T ux = C[l * n2 + p], uy = B[l * n2 + p], uz = gz[l];
      // metric components: 00, 11, 22, 01, 02, 12
      fx[l] = kap * (g[0][l] * ux + g[3][l] * uy + g[4][l] * uz);
      fy[l] = kap * (g[3][l] * ux + g[1][l] * uy + g[5][l] * uz);
      fz[l] = kap * (g[4][l] * ux + g[5][l] * uy + g[2][l] * uz);
    }
#pragma unroll
    for (int l = 0; l < n; ++l) {
      T a = 0;
#pragma unroll
      for (int q = 0; q < n; ++q) a += tb.D[q * n + l] * fz[q];
      A[l * n2 + p] = a;
      C[l * n2 + p] = fx[l];
      B[l * n2 + p] = fy[l];
    }
  }
  __syncthreads();
  // B2: y-lines (x = i0, z = i1): acc += D^T along y of fy
  if (inblk) {
    T f[n];
#pragma unroll
    for (int b = 0; b < n; ++b) f[b] = B[i1 * n2 + b * n + i0];
#pragma unroll
    for (int b = 0; b < n; ++b) {
      T a = A[i1 * n2 + b * n + i0];
#pragma unroll
      for (int q = 0; q < n; ++q) a += tb.D[q * n + b] * f[q];
      A[i1 * n2 + b * n + i0] = a;
    }
  }
  __syncthreads();
  // B3: x-lines (y = i0, z = i1): acc += D^T along x of fx; S^T along x
  if (inblk) {
    T f[n], acc[n];
#pragma unroll
    for (int a = 0; a < n; ++a) f[a] = C[i1 * n2 + i0 * n + a];
#pragma unroll
    for (int a = 0; a < n; ++a) {
      T s = A[i1 * n2 + i0 * n + a];
#pragma unroll
      for (int q = 0; q < n; ++q) s += tb.D[q * n + a] * f[q];
      acc[a] = s;
    }
#pragma unroll
    for (int i = 0; i < n; ++i) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < n; ++q) s += tb.S[q * n + i] * acc[q];
      B[i1 * n2 + i0 * n + i] = s;
    }
  }
  __syncthreads();
  // B4: y-lines (x = i0, z = i1): S^T along y
  if (inblk) {
    T r[n];
#pragma unroll
    for (int b = 0; b < n; ++b) r[b] = B[i1 * n2 + b * n + i0];
#pragma unroll
    for (int i = 0; i < n; ++i) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < n; ++q) s += tb.S[q * n + i] * r[q];
      A[i1 * n2 + i * n + i0] = s;
    }
  }
  __syncthreads();
  // B5: z-lines (x = i0, y = i1): S^T along z, then scatter-add (or gradient reduction)
  T partial = 0;
  if (active) {
    T r[n];
#pragma unroll
    for (int l = 0; l < n; ++l) r[l] = A[l * n2 + p];
#pragma unroll
    for (int i = 0; i < n; ++i) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < n; ++q) s += tb.S[q * n + i] * r[q];
      const bool bnd = bxy || (dirichlet && on_boundary(cz * K + i, N1));
      if (!bnd) {
        if constexpr (GRAD)
          partial += s * lam[base + plane * i];
        else
          atomic_add(dst + base + plane * i, s);
      }
    }
  }
  if constexpr (GRAD) {
    if (inblk) C[p] = partial;
    __syncthreads();
    if (active && p == 0) {
      T s = 0;
      for (int j = 0; j < n2; ++j) s += C[j];
      grad[cell] = -s;
    }
  }
}

// dst = src on Dirichlet DoFs, 0 elsewhere (the cell kernels then add into dst).
template <typename T>
__global__ void __launch_bounds__(kBlock)
boundary_init_kernel(const T *__restrict__ src, T *__restrict__ dst, int N1, int dirichlet) {
  const int64_t n = int64_t(N1) * N1 * N1;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const int x = int(i % N1), y = int((i / N1) % N1), z = int(i / (int64_t(N1) * N1));
    const bool bnd = dirichlet && (on_boundary(x, N1) || on_boundary(y, N1) || on_boundary(z, N1));
    dst[i] = bnd ? src[i] : T(0);
  }
}

// ---------------------------------------------------------------------------------------
// Setup kernels (FP64).

// Per cell and Gauss point: node positions of the isoparametric map (Gauss-Lobatto
// support points of x + a sin(pi x) sin(pi y) sin(pi z) (1,1,1)), J_q = sum_i x_i (x)
// grad phi_i(xi_q), and G_q = w_q det J_q J_q^{-1} J_q^{-T}, stored [cell][6][q] in FP64
// and FP32 (components 00, 11, 22, 01, 02, 12).
template <int K>
__global__ void __launch_bounds__(kBlock)
metric_kernel(double *__restrict__ m64, float *__restrict__ m32, int Nc, double h, double amp,
              Tab<K + 1, double> tb) {
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
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int i2 = 0; i2 < n; ++i2)
      for (int i1 = 0; i1 < n; ++i1)
        for (int i0 = 0; i0 < n; ++i0) {
          const double disp = amp * s1[0][i0] * s1[1][i1] * s1[2][i2];
          const double xn[3] = {X[0][i0] + disp, X[1][i1] + disp, X[2][i2] + disp};
          const double dphi[3] = {Sd[q0 * n + i0] * S[q1 * n + i1] * S[q2 * n + i2],
                                  S[q0 * n + i0] * Sd[q1 * n + i1] * S[q2 * n + i2],
                                  S[q0 * n + i0] * S[q1 * n + i1] * Sd[q2 * n + i2]};
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) J[a][b] += xn[a] * dphi[b];
        }
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
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
    const double wd = w[q0] * w[q1] * w[q2] * det;
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
                 double h, int dirichlet, Tab<K + 1, double> tb) {
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
    if (dirichlet && (on_boundary(gx, N1) || on_boundary(gy, N1) || on_boundary(gz, N1))) continue;
    const double v = kappa[cell] * h *
                     (Kd[a] * Md[b] * Md[l] + Md[a] * Kd[b] * Md[l] + Md[a] * Md[b] * Kd[l]);
    atomic_add(diag + gx + N1 * int64_t(gy) + plane * gz, v);
  }
}

// diag(A) contributions of curved cells: sum_q kappa grad phi_i(q) . G_q grad phi_i(q).
template <int K>
__global__ void __launch_bounds__(kBlock)
diag_curved_kernel(double *__restrict__ diag, const double *__restrict__ kappa,
                   const double *__restrict__ metric, int Nc, int N1, int dirichlet,
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
    if (dirichlet && (on_boundary(gx, N1) || on_boundary(gy, N1) || on_boundary(gz, N1))) continue;
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

// Right-hand side b_i = sum_q w_q det J_q f(x_q) phi_i(xi_q), f = 3 pi^2 sin sin sin, with
// x_q the isoparametric image of the Gauss point.  One work-group per cell.
template <int K>
__global__ void __launch_bounds__(kBlock)
rhs_kernel(double *__restrict__ b, int Nc, int N1, double h, double amp, Tab<K + 1, double> tb) {
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
            for (int bb = 0; bb < 3; ++bb) J[a][bb] += xn[a] * dphi[bb];
          }
        }
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    const double f = 3.0 * M_PI * M_PI * sin(M_PI * xq[0]) * sin(M_PI * xq[1]) * sin(M_PI * xq[2]);
    fw[q] = w[q0] * w[q1] * w[q2] * det * f;
  }
  __syncthreads();
  const int64_t plane = int64_t(N1) * N1;
  for (int i = threadIdx.x; i < n3; i += kBlock) {
    const int a = i % n, bb = (i / n) % n, l = i / (n * n);
    const int gx = c[0] * K + a, gy = c[1] * K + bb, gz = c[2] * K + l;
    if (on_boundary(gx, N1) || on_boundary(gy, N1) || on_boundary(gz, N1)) continue;
    double s = 0;
    for (int q = 0; q < n3; ++q) {
      const int q0 = q % n, q1 = (q / n) % n, q2 = q / (n * n);
      s += S[q0 * n + a] * S[q1 * n + bb] * S[q2 * n + l] * fw[q];
    }
    atomic_add(b + gx + N1 * int64_t(gy) + plane * gz, s);
  }
}

inline int grid_for(int64_t items, int cap = 65536) {
  int64_t g = (items + kBlock - 1) / kBlock;
  return int(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_boundary_init(const Context &c, const Level &L, int dtype, const void *src,
                                void *dst, hipStream_t s) {
  const int dir = c.p.bc == MFL_BC_DIRICHLET;
  const int grid = grid_for(L.ndofs, 8192);
  if (dtype == MFL_F64)
    boundary_init_kernel<double><<<grid, kBlock, 0, s>>>((const double *)src, (double *)dst, L.N1, dir);
  else
    boundary_init_kernel<float><<<grid, kBlock, 0, s>>>((const float *)src, (float *)dst, L.N1, dir);
  return hipGetLastError();
}

template <int K, typename T>
static hipError_t cg_apply_k(const Context &c, const Level &L, const Tab<kMaxN, T> &tab,
                             const T *kappa, const T *metric, const T *src, T *dst, hipStream_t s) {
  constexpr int CPB = Shape<K>::cpb;
  const int grid = int((L.ncells + CPB - 1) / CPB);
  const int dir = c.p.bc == MFL_BC_DIRICHLET;
  const Tab<K + 1, T> tb = shrink_tab<K + 1, T>(tab);
  if (c.p.geometry == MFL_GEOM_CURVED)
    curved_kernel<K, T, false><<<grid, kBlock, 0, s>>>(src, dst, kappa, metric, nullptr, nullptr,
                                                      L.Nc, L.N1, dir, tb);
  else
    cart_kernel<K, T, false><<<grid, kBlock, 0, s>>>(src, dst, kappa, nullptr, nullptr, L.Nc, L.N1,
                                                    T(L.h), dir, tb);
  return hipGetLastError();
}

hipError_t launch_cg_apply(const Context &c, const Level &L, int dtype, const void *src, void *dst,
                           hipStream_t s) {
  hipError_t e = launch_boundary_init(c, L, dtype, src, dst, s);
  if (e != hipSuccess) return e;
  if (dtype == MFL_F64) {
#define CASE(K) return cg_apply_k<K, double>(c, L, c.tab64, L.kappa64, L.metric64, (const double *)src, (double *)dst, s)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  } else {
#define CASE(K) return cg_apply_k<K, float>(c, L, c.tab32, L.kappa32, L.metric32, (const float *)src, (float *)dst, s)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  }
  return hipErrorInvalidValue;
}

template <int K>
static hipError_t kappa_grad_k(const Context &c, const Level &L, const double *u, const double *lam,
                               double *grad, hipStream_t s) {
  constexpr int CPB = Shape<K>::cpb;
  const int grid = int((L.ncells + CPB - 1) / CPB);
  const int dir = c.p.bc == MFL_BC_DIRICHLET;
  const Tab<K + 1, double> tb = shrink_tab<K + 1, double>(c.tab64);
  if (c.p.geometry == MFL_GEOM_CURVED)
    curved_kernel<K, double, true><<<grid, kBlock, 0, s>>>(u, nullptr, L.kappa64, L.metric64, lam,
                                                          grad, L.Nc, L.N1, dir, tb);
  else
    cart_kernel<K, double, true><<<grid, kBlock, 0, s>>>(u, nullptr, L.kappa64, lam, grad, L.Nc,
                                                        L.N1, L.h, dir, tb);
  return hipGetLastError();
}

hipError_t launch_cg_kappa_grad(const Context &c, const Level &L, const double *u, const double *lam,
                                double *grad, hipStream_t s) {
#define CASE(K) return kappa_grad_k<K>(c, L, u, lam, grad, s)
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipErrorInvalidValue;
}

hipError_t launch_metric_setup(const Context &c, const Level &L, hipStream_t s) {
  const int64_t items = L.ncells * int64_t(c.n) * c.n * c.n;
#define CASE(K)                                                                                \
  metric_kernel<K><<<grid_for(items), kBlock, 0, s>>>(L.metric64, L.metric32, L.Nc, L.h,        \
                                                      c.p.curve_amp, shrink_tab<K + 1, double>(c.tab64)); \
  break
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipGetLastError();
}

hipError_t launch_cg_diagonal(const Context &c, const Level &L, hipStream_t s) {
  const int64_t items = L.ncells * int64_t(c.n) * c.n * c.n;
  const int dir = c.p.bc == MFL_BC_DIRICHLET;
  hipError_t e = launch_fill(L.diag64, MFL_F64, L.ndofs, 0.0, s);
  if (e != hipSuccess) return e;
  if (c.p.geometry == MFL_GEOM_CURVED) {
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
  rhs_kernel<K><<<int(L.ncells), kBlock, 0, s>>>(b, L.Nc, L.N1, L.h, amp,                     \
                                                  shrink_tab<K + 1, double>(c.tab64));        \
  break
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipGetLastError();
}

}  // namespace mfl
