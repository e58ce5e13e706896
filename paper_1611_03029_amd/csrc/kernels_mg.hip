// Multigrid transfer, Chebyshev smoother updates and PCG vector kernels (Sec. 4.1).
//
// All vector kernels stream their operands once (grid-stride loops); reductions are
// deterministic: fixed-size block partials followed by a one-block finalize kernel that
// also forms the CG scalars on the device, so the host reads only the residual norm.
#include "device_common.h"

namespace mfl {

namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t items, int cap = 16384) {
  int64_t g = (items + kBlock - 1) / kBlock;
  return int(g < 1 ? 1 : (g > cap ? cap : g));
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < (n); i += int64_t(gridDim.x) * kBlock)

template <typename T>
__global__ void __launch_bounds__(kBlock) fill_kernel(T *d, int64_t n, T v) {
  GRID_STRIDE(i, n) d[i] = v;
}

template <typename A, typename B>
__global__ void __launch_bounds__(kBlock) cast_kernel(const A *s, B *d, int64_t n) {
  GRID_STRIDE(i, n) d[i] = B(s[i]);
}

__global__ void __launch_bounds__(kBlock) check_positive_kernel(const double *v, int64_t n, int *flag, int bit) {
  bool bad = false;
  GRID_STRIDE(i, n) {
    const double x = v[i];
    bad = bad || !(x > 0.0) || !isfinite(x);
  }
  if (bad) atomicOr(flag, bit);
}

__global__ void __launch_bounds__(kBlock)
coarsen_kappa_kernel(const double *__restrict__ fine, double *__restrict__ c64, float *__restrict__ c32,
                     int Ncc) {
  const int64_t nc = int64_t(Ncc) * Ncc * Ncc;
  const int Nf = 2 * Ncc;
  GRID_STRIDE(i, nc) {
    const int x = int(i % Ncc), y = int((i / Ncc) % Ncc), z = int(i / (int64_t(Ncc) * Ncc));
    double s = 0;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx)
          s += fine[(2 * x + dx) + int64_t(Nf) * ((2 * y + dy) + int64_t(Nf) * (2 * z + dz))];
    c64[i] = 0.125 * s;
    c32[i] = float(0.125 * s);
  }
}

// Dirichlet DoFs get diagonal 1 (identity rows); inverse and FP32 copies.
__global__ void __launch_bounds__(kBlock)
diag_finalize_kernel(double *__restrict__ d64, double *__restrict__ i64, float *__restrict__ d32,
                     float *__restrict__ i32, int N1, int dmask) {
  const int64_t n = int64_t(N1) * N1 * N1;
  GRID_STRIDE(i, n) {
    const int x = int(i % N1), y = int((i / N1) % N1), z = int(i / (int64_t(N1) * N1));
    double v = d64[i];
    if (dirichlet_dof(x, y, z, N1, dmask)) v = 1.0;
    d64[i] = v;
    i64[i] = 1.0 / v;
    d32[i] = float(v);
    i32[i] = float(1.0 / v);
  }
}

// Inverse and FP32 copies of a diagonal without identity rows (SIPG).
__global__ void __launch_bounds__(kBlock)
diag_invert_kernel(const double *__restrict__ d64, double *__restrict__ i64, float *__restrict__ d32,
                   float *__restrict__ i32, int64_t n) {
  GRID_STRIDE(i, n) {
    const double v = d64[i];
    i64[i] = 1.0 / v;
    d32[i] = float(v);
    i32[i] = float(1.0 / v);
  }
}

// First Chebyshev update from a zero initial guess: d = D^{-1} b / theta, x = d.
// b_in may be of another precision than the level (the FP64 residual entering an FP32
// cycle); it is stored converted in b_store for the residuals of the later steps.
template <typename A, typename T>
__global__ void __launch_bounds__(kBlock)
cheb_first_kernel(const A *__restrict__ b_in, T *__restrict__ b_store, const T *__restrict__ dinv,
                  T *__restrict__ d, T *__restrict__ x, int64_t n, T inv_theta) {
  GRID_STRIDE(i, n) {
    const T b = T(b_in[i]);
    if (b_store) b_store[i] = b;
    const T v = dinv[i] * b * inv_theta;
    d[i] = v;
    x[i] = v;
  }
}

// One Chebyshev update: d = c1 d + c2 D^{-1} (b - A x); x += d.  The residual is never
// stored.  x64_out (optional) receives x in FP64 (exit of an FP32 cycle).
template <typename T>
__global__ void __launch_bounds__(kBlock)
cheb_step_kernel(const T *__restrict__ b, const T *__restrict__ ax, const T *__restrict__ dinv,
                 T *__restrict__ d, T *__restrict__ x, double *__restrict__ x64, int64_t n, T c1,
                 T c2) {
  GRID_STRIDE(i, n) {
    const T dn = c1 * d[i] + c2 * dinv[i] * (b[i] - ax[i]);
    const T xn = x[i] + dn;
    d[i] = dn;
    x[i] = xn;
    if (x64) x64[i] = double(xn);
  }
}

// ---- transfers between continuous Q_k levels (Sec. 4.1) ------------------------------
// Prolongation is the embedding P = P1 (x) P1 (x) P1 of the coarse Q_k space in the fine one,
// restriction its transpose, both with the rows and columns of Dirichlet DoFs removed.  P1 is
// applied as a gather, so that every output value is written once (no atomics, no clearing
// pass) and every pass streams whole rows: restriction in x and y per fine z-plane, then in
// z; prolongation in z, then in x and y per fine z-plane.  T holds the intermediate
// [fine z][coarse y][coarse x] (N1f N1c^2 values).
//
// 1D embedding: fine line f lies in fine cell min(f / K, Nf - 1), whose coarse parent is
// pc = that / 2, at the fl = f - 2K pc -th of the 2K+1 fine lines of pc, so
// P1[f][I] = P[fl][I - K pc] (the coarse basis of pc at that line) when 0 <= I - K pc <= K and
// 0 otherwise.  The fine lines where coarse line I = K c + a is nonzero lie in
// [2I - 2K, 2I + 2K] (in [2K c, 2K (c+1)] for 0 < a < K, plus cell c - 1 for a = 0).
template <int K>
__device__ __forceinline__ int embed_parent(int f, int Nf) {
  return min(f / K, Nf - 1) / 2;
}

template <int K>
__device__ __forceinline__ double embed_weight(const double *P, int Nf, int f, int I) {
  const int pc = embed_parent<K>(f, Nf), a = I - K * pc;
  return (a >= 0 && a <= K) ? P[(f - 2 * K * pc) * (K + 1) + a] : 0.0;
}

constexpr int kRestrictTX = 32, kRestrictTY = 16;   // coarse x, y DoFs of a restriction tile
constexpr int kProlongTX = 64, kProlongTY = 16;     // fine x, y DoFs of a prolongation tile

// T[fz][J][I] = sum_{fy, fx} P1[fy][J] P1[fx][I] r[fz][fy][fx] with r = b_f - A x_f (axf ==
// nullptr: r = b_f), zero on Dirichlet DoFs.  Work-group = one tile of kRestrictTX x
// kRestrictTY coarse (x, y) DoFs of one fine z-plane (blockIdx.y): the x sums of the fine
// rows the tile needs go to LDS, then the y sums to T.
template <int K, typename TF>
__global__ void __launch_bounds__(kBlock)
restrict_xy_kernel(const TF *__restrict__ bf, const TF *__restrict__ axf, TF *__restrict__ T, int Ncc, int dmask,
                   TransferTab tt) {
  constexpr int n = K + 1, TX = kRestrictTX, TY = kRestrictTY, FY = 2 * TY + 4 * K - 1;
  __shared__ double P[(2 * K + 1) * n];
  __shared__ TF U[FY * TX];
  for (int i = threadIdx.x; i < (2 * K + 1) * n; i += kBlock) P[i] = tt.P[i];
  const int N1c = K * Ncc + 1, N1f = 2 * K * Ncc + 1, Nf = 2 * Ncc;
  const int ntx = (N1c + TX - 1) / TX;
  const int tx = int(blockIdx.x) % ntx, ty = int(blockIdx.x) / ntx, fz = int(blockIdx.y);
  const int I0 = tx * TX, J0 = ty * TY, fy0 = 2 * J0 - 2 * K;
  const bool zbnd = on_dirichlet(fz, N1f, dmask);
  const int64_t plane = int64_t(fz) * N1f * N1f;
  __syncthreads();
  for (int idx = threadIdx.x; idx < FY * TX; idx += kBlock) {
    const int r = idx / TX, i = idx - r * TX, I = I0 + i, fy = fy0 + r;
    TF acc = 0;
    if (!zbnd && I < N1c && fy >= 0 && fy < N1f && !on_dirichlet(fy, N1f, dmask)) {
      const int64_t row = plane + int64_t(fy) * N1f;
#pragma unroll
      for (int d = -2 * K; d <= 2 * K; ++d) {
        const int f = 2 * I + d;
        if (f < 0 || f >= N1f || on_dirichlet(f, N1f, dmask)) continue;
        const double w = embed_weight<K>(P, Nf, f, I);
        if (w != 0.0) acc += TF(w) * (axf ? bf[row + f] - axf[row + f] : bf[row + f]);
      }
    }
    U[idx] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < TY * TX; idx += kBlock) {
    const int j = idx / TX, i = idx - j * TX, I = I0 + i, J = J0 + j;
    if (I >= N1c || J >= N1c) continue;
    TF acc = 0;
#pragma unroll
    for (int d = -2 * K; d <= 2 * K; ++d) {
      const int fy = 2 * J + d;
      if (fy < 0 || fy >= N1f) continue;
      acc += TF(embed_weight<K>(P, Nf, fy, J)) * U[(fy - fy0) * TX + i];
    }
    T[(int64_t(fz) * N1c + J) * N1c + I] = acc;
  }
}

// bc[Iz][J][I] = sum_fz P1[fz][Iz] T[fz][J][I]; zero on the coarse Dirichlet DoFs.
template <int K, typename TF, typename TC>
__global__ void __launch_bounds__(kBlock)
restrict_z_kernel(const TF *__restrict__ T, TC *__restrict__ bc, int Ncc, int dmask, TransferTab tt) {
  constexpr int n = K + 1;
  __shared__ double P[(2 * K + 1) * n];
  for (int i = threadIdx.x; i < (2 * K + 1) * n; i += kBlock) P[i] = tt.P[i];
  __syncthreads();
  const int N1c = K * Ncc + 1, N1f = 2 * K * Ncc + 1, Nf = 2 * Ncc;
  const int64_t pc2 = int64_t(N1c) * N1c, total = pc2 * N1c;
  GRID_STRIDE(idx, total) {
    const int I = int(idx % N1c), J = int((idx / N1c) % N1c), Iz = int(idx / pc2);
    TF acc = 0;
    if (!dirichlet_dof(I, J, Iz, N1c, dmask)) {
      const int64_t col = int64_t(J) * N1c + I;
#pragma unroll
      for (int d = -2 * K; d <= 2 * K; ++d) {
        const int fz = 2 * Iz + d;
        if (fz < 0 || fz >= N1f) continue;
        const double w = embed_weight<K>(P, Nf, fz, Iz);
        if (w != 0.0) acc += TF(w) * T[int64_t(fz) * pc2 + col];
      }
    }
    bc[idx] = TC(acc);
  }
}

// T[fz][J][I] = sum_Iz P1[fz][Iz] xc[Iz][J][I] (coarse Dirichlet DoFs taken as zero).
template <int K, typename TC, typename TF>
__global__ void __launch_bounds__(kBlock)
prolong_z_kernel(const TC *__restrict__ xc, TF *__restrict__ T, int Ncc, int dmask, TransferTab tt) {
  constexpr int n = K + 1;
  __shared__ double P[(2 * K + 1) * n];
  for (int i = threadIdx.x; i < (2 * K + 1) * n; i += kBlock) P[i] = tt.P[i];
  __syncthreads();
  const int N1c = K * Ncc + 1, N1f = 2 * K * Ncc + 1, Nf = 2 * Ncc;
  const int64_t pc2 = int64_t(N1c) * N1c, total = pc2 * N1f;
  GRID_STRIDE(idx, total) {
    const int I = int(idx % N1c), J = int((idx / N1c) % N1c), fz = int(idx / pc2);
    TF acc = 0;
    if (!on_dirichlet(I, N1c, dmask) && !on_dirichlet(J, N1c, dmask)) {
      const int pc = embed_parent<K>(fz, Nf), fl = fz - 2 * K * pc;
#pragma unroll
      for (int a = 0; a <= K; ++a) {
        const int Iz = K * pc + a;
        if (on_dirichlet(Iz, N1c, dmask)) continue;
        acc += TF(P[fl * n + a]) * TF(xc[int64_t(Iz) * pc2 + int64_t(J) * N1c + I]);
      }
    }
    T[idx] = acc;
  }
}

// xf[fz][fy][fx] += sum_{J, I} P1[fy][J] P1[fx][I] T[fz][J][I] on the non-Dirichlet fine DoFs.
// Work-group = one tile of kProlongTX x kProlongTY fine (x, y) DoFs of one fine z-plane: the
// coarse (x, y) block of T the tile needs goes to LDS, then its x sums, then the y sums are
// added to xf.
template <int K, typename TF>
__global__ void __launch_bounds__(kBlock)
prolong_xy_kernel(const TF *__restrict__ T, TF *__restrict__ xf, int Ncc, int dmask, TransferTab tt) {
  constexpr int n = K + 1, FX = kProlongTX, FYT = kProlongTY;
  // coarse lines a tile of F fine lines touches: K (parent(last) - parent(first)) + K + 1 <=
  // F / 2 + 2K + 1 (parents of lines F - 1 apart differ by at most (F - 1) / (2K) + 1)
  constexpr int CX = FX / 2 + 2 * K + 2, CY = FYT / 2 + 2 * K + 2;
  __shared__ double P[(2 * K + 1) * n];
  __shared__ TF Tc[CY * CX];
  __shared__ TF V[CY * FX];
  const int N1c = K * Ncc + 1, N1f = 2 * K * Ncc + 1, Nf = 2 * Ncc;
  const int fz = int(blockIdx.y);
  if (on_dirichlet(fz, N1f, dmask)) return;   // the same for the whole work-group
  for (int i = threadIdx.x; i < (2 * K + 1) * n; i += kBlock) P[i] = tt.P[i];
  const int ntx = (N1f + FX - 1) / FX;
  const int fx0 = (int(blockIdx.x) % ntx) * FX, fy0 = (int(blockIdx.x) / ntx) * FYT;
  const int fx1 = min(fx0 + FX, N1f) - 1, fy1 = min(fy0 + FYT, N1f) - 1;
  const int cx0 = K * embed_parent<K>(fx0, Nf), cy0 = K * embed_parent<K>(fy0, Nf);
  const int wx = K * embed_parent<K>(fx1, Nf) + K + 1 - cx0, wy = K * embed_parent<K>(fy1, Nf) + K + 1 - cy0;
  const int64_t tplane = int64_t(fz) * N1c * N1c;
  for (int idx = threadIdx.x; idx < wy * wx; idx += kBlock) {
    const int cy = idx / wx, cx = idx - cy * wx;
    Tc[cy * CX + cx] = T[tplane + int64_t(cy0 + cy) * N1c + cx0 + cx];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < wy * FX; idx += kBlock) {
    const int cy = idx / FX, i = idx - cy * FX, fx = fx0 + i;
    TF acc = 0;
    if (fx < N1f) {
      const int pc = embed_parent<K>(fx, Nf), fl = fx - 2 * K * pc, o = K * pc - cx0;
#pragma unroll
      for (int a = 0; a <= K; ++a) acc += TF(P[fl * n + a]) * Tc[cy * CX + o + a];
    }
    V[cy * FX + i] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < FYT * FX; idx += kBlock) {
    const int j = idx / FX, i = idx - j * FX, fx = fx0 + i, fy = fy0 + j;
    if (fx >= N1f || fy >= N1f || on_dirichlet(fx, N1f, dmask) || on_dirichlet(fy, N1f, dmask)) continue;
    const int pc = embed_parent<K>(fy, Nf), fl = fy - 2 * K * pc, o = K * pc - cy0;
    TF acc = 0;
#pragma unroll
    for (int b = 0; b <= K; ++b) acc += TF(P[fl * n + b]) * V[(o + b) * FX + i];
    xf[(int64_t(fz) * N1f + fy) * N1f + fx] += acc;
  }
}

__global__ void __launch_bounds__(kBlock)
dot_partial_kernel(const double *__restrict__ a, const double *__restrict__ b, int64_t n,
                   double *__restrict__ partials) {
  __shared__ double sc[kBlock];
  double s = 0;
  GRID_STRIDE(i, n) s += a[i] * b[i];
  s = block_sum(s, sc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock)
finalize_kernel(const double *__restrict__ partials, double *__restrict__ sc, int which, int op) {
  __shared__ double red[kBlock];
  double s = 0;
  for (int i = threadIdx.x; i < kReduceBlocks; i += kBlock) s += partials[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    if (op == kFinSum) {
      sc[which] = s;
    } else if (op == kFinAlpha) {
      // a non-positive or non-finite p^T A p is a breakdown: skip the update (alpha = 0)
      sc[kPQ] = s;
      sc[kAlpha] = (s > 0.0 && isfinite(s)) ? sc[kRZ] / s : 0.0;
    } else {
      sc[kRZnew] = s;
      sc[kBeta] = s / sc[kRZ];
      sc[kRZ] = s;
    }
  }
}

__global__ void __launch_bounds__(kBlock)
pcg_update_xr_kernel(double *__restrict__ x, double *__restrict__ r, const double *__restrict__ p,
                     const double *__restrict__ q, const double *__restrict__ sc, int64_t n,
                     double *__restrict__ partials) {
  __shared__ double red[kBlock];
  const double alpha = sc[kAlpha];
  double s = 0;
  GRID_STRIDE(i, n) {
    x[i] += alpha * p[i];
    const double rn = r[i] - alpha * q[i];
    r[i] = rn;
    s += rn * rn;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock)
pcg_update_p_kernel(double *__restrict__ p, const double *__restrict__ z, const double *__restrict__ sc,
                    int64_t n) {
  const double beta = sc[kBeta];
  GRID_STRIDE(i, n) p[i] = z[i] + beta * p[i];
}

// SplitMix64 counter stream (Steele, Lea, Flood 2014): value i of stream `key` is the
// finalizer applied to key + (i+1) * 0x9E3779B97F4A7C15, mapped to [-1, 1).
__global__ void __launch_bounds__(kBlock)
random_start_kernel(double *__restrict__ v, int64_t n, int N1, uint64_t key, int dmask) {
  GRID_STRIDE(i, n) {
    uint64_t z = key + uint64_t(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    const double u = 2.0 * double(z >> 11) * 0x1.0p-53 - 1.0;
    // dmask = 0 (no Dirichlet rows, e.g. the DG layout): the grid coordinates are unused
    const int x = int(i % N1), y = int((i / N1) % N1), zz = int(i / (int64_t(N1) * N1));
    const bool bnd = dmask != 0 && dirichlet_dof(x, y, zz, N1, dmask);
    v[i] = bnd ? 0.0 : u;
  }
}

__global__ void __launch_bounds__(kBlock)
jacobi_kernel(const double *__restrict__ dinv, const double *__restrict__ r, double *__restrict__ z,
              int64_t n) {
  GRID_STRIDE(i, n) z[i] = dinv[i] * r[i];
}

__global__ void __launch_bounds__(kBlock) zero_boundary_kernel(double *__restrict__ v, int N1, int dmask) {
  const int64_t n = int64_t(N1) * N1 * N1;
  GRID_STRIDE(i, n) {
    const int x = int(i % N1), y = int((i / N1) % N1), z = int(i / (int64_t(N1) * N1));
    if (dirichlet_dof(x, y, z, N1, dmask)) v[i] = 0.0;
  }
}

}  // namespace

hipError_t launch_fill(void *dst, int dtype, int64_t n, double value, hipStream_t s) {
  if (dtype == MFL_F64)
    fill_kernel<double><<<grid_for(n), kBlock, 0, s>>>((double *)dst, n, value);
  else
    fill_kernel<float><<<grid_for(n), kBlock, 0, s>>>((float *)dst, n, float(value));
  return hipGetLastError();
}

hipError_t launch_cast(const void *src, int sd, void *dst, int dd, int64_t n, hipStream_t s) {
  const int g = grid_for(n);
  if (sd == MFL_F64 && dd == MFL_F32)
    cast_kernel<double, float><<<g, kBlock, 0, s>>>((const double *)src, (float *)dst, n);
  else if (sd == MFL_F32 && dd == MFL_F64)
    cast_kernel<float, double><<<g, kBlock, 0, s>>>((const float *)src, (double *)dst, n);
  else if (sd == MFL_F64)
    cast_kernel<double, double><<<g, kBlock, 0, s>>>((const double *)src, (double *)dst, n);
  else
    cast_kernel<float, float><<<g, kBlock, 0, s>>>((const float *)src, (float *)dst, n);
  return hipGetLastError();
}

hipError_t launch_check_positive(const double *v, int64_t n, int *flag, int bit, hipStream_t s) {
  check_positive_kernel<<<grid_for(n, 1024), kBlock, 0, s>>>(v, n, flag, bit);
  return hipGetLastError();
}

hipError_t launch_coarsen_kappa(const Level &coarse, const Level &fine, hipStream_t s) {
  coarsen_kappa_kernel<<<grid_for(coarse.ncells), kBlock, 0, s>>>(fine.kappa64, coarse.kappa64,
                                                                  coarse.kappa32, coarse.Nc);
  return hipGetLastError();
}

hipError_t launch_diag_finalize(const Context &c, const Level &L, hipStream_t s) {
  diag_finalize_kernel<<<grid_for(L.ndofs), kBlock, 0, s>>>(L.diag64, L.dinv64, L.diag32, L.dinv32,
                                                            L.N1, dirichlet_mask(c.p));
  return hipGetLastError();
}

hipError_t launch_diag_invert(const Level &L, hipStream_t s) {
  diag_invert_kernel<<<grid_for(L.ndofs), kBlock, 0, s>>>(L.diag64, L.dinv64, L.diag32, L.dinv32, L.ndofs);
  return hipGetLastError();
}

hipError_t launch_cheb_first(const void *b_in, int in_dtype, void *b_store, const void *dinv,
                             void *d, void *x, int dtype, int64_t n, double inv_theta, hipStream_t s) {
  const int g = grid_for(n);
  if (dtype == MFL_F64) {
    if (in_dtype != MFL_F64) return hipErrorInvalidValue;
    cheb_first_kernel<double, double><<<g, kBlock, 0, s>>>((const double *)b_in, (double *)b_store,
                                                           (const double *)dinv, (double *)d,
                                                           (double *)x, n, inv_theta);
  } else if (in_dtype == MFL_F64) {
    cheb_first_kernel<double, float><<<g, kBlock, 0, s>>>((const double *)b_in, (float *)b_store,
                                                          (const float *)dinv, (float *)d,
                                                          (float *)x, n, float(inv_theta));
  } else {
    cheb_first_kernel<float, float><<<g, kBlock, 0, s>>>((const float *)b_in, (float *)b_store,
                                                         (const float *)dinv, (float *)d, (float *)x,
                                                         n, float(inv_theta));
  }
  return hipGetLastError();
}

hipError_t launch_cheb_step(const void *b, const void *ax, const void *dinv, void *d, void *x,
                            double *x64_out, int dtype, int64_t n, double c1, double c2,
                            hipStream_t s) {
  const int g = grid_for(n);
  if (dtype == MFL_F64)
    cheb_step_kernel<double><<<g, kBlock, 0, s>>>((const double *)b, (const double *)ax,
                                                  (const double *)dinv, (double *)d, (double *)x,
                                                  x64_out, n, c1, c2);
  else
    cheb_step_kernel<float><<<g, kBlock, 0, s>>>((const float *)b, (const float *)ax,
                                                 (const float *)dinv, (float *)d, (float *)x, x64_out,
                                                 n, float(c1), float(c2));
  return hipGetLastError();
}

template <int K, typename TC, typename TF>
static hipError_t prolongate_kt(const Context &c, const Level &coarse, const Level &fine, const void *xc, void *xf,
                                hipStream_t s) {
  const int N1c = coarse.N1, N1f = fine.N1;
  TF *T = static_cast<TF *>(fine.tbuf);
  const int64_t nt = int64_t(N1f) * N1c * N1c;
  prolong_z_kernel<K, TC, TF><<<grid_for(nt), kBlock, 0, s>>>((const TC *)xc, T, coarse.Nc, dirichlet_mask(c.p),
                                                             c.transfer);
  const int tiles = ((N1f + kProlongTX - 1) / kProlongTX) * ((N1f + kProlongTY - 1) / kProlongTY);
  prolong_xy_kernel<K, TF><<<dim3(tiles, N1f), kBlock, 0, s>>>(T, (TF *)xf, coarse.Nc, dirichlet_mask(c.p),
                                                               c.transfer);
  return hipGetLastError();
}

template <int K>
static hipError_t prolongate_k(const Context &c, const Level &coarse, const Level &fine, const void *xc, int cd,
                               void *xf, int fd, hipStream_t s) {
  if (fd == MFL_F64 && cd == MFL_F64) return prolongate_kt<K, double, double>(c, coarse, fine, xc, xf, s);
  if (fd == MFL_F32 && cd == MFL_F64) return prolongate_kt<K, double, float>(c, coarse, fine, xc, xf, s);
  if (fd == MFL_F32 && cd == MFL_F32) return prolongate_kt<K, float, float>(c, coarse, fine, xc, xf, s);
  return hipErrorInvalidValue;
}

hipError_t launch_prolongate_add(const Context &c, const Level &coarse, const Level &fine,
                                 const void *xc, int cd, void *xf, int fd, hipStream_t s) {
  if (!fine.tbuf) return hipErrorInvalidValue;
#define CASE(K) return prolongate_k<K>(c, coarse, fine, xc, cd, xf, fd, s)
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipErrorInvalidValue;
}

template <int K, typename TF, typename TC>
static hipError_t restrict_kt(const Context &c, const Level &coarse, const Level &fine, const void *bf,
                              const void *axf, void *bc, hipStream_t s) {
  const int N1c = coarse.N1, N1f = fine.N1;
  TF *T = static_cast<TF *>(fine.tbuf);
  const int tiles = ((N1c + kRestrictTX - 1) / kRestrictTX) * ((N1c + kRestrictTY - 1) / kRestrictTY);
  restrict_xy_kernel<K, TF><<<dim3(tiles, N1f), kBlock, 0, s>>>((const TF *)bf, (const TF *)axf, T, coarse.Nc,
                                                                dirichlet_mask(c.p), c.transfer);
  restrict_z_kernel<K, TF, TC><<<grid_for(coarse.ndofs), kBlock, 0, s>>>(T, (TC *)bc, coarse.Nc,
                                                                         dirichlet_mask(c.p), c.transfer);
  return hipGetLastError();
}

template <int K>
static hipError_t restrict_k(const Context &c, const Level &coarse, const Level &fine, const void *bf,
                             const void *axf, int fd, void *bc, int cd, hipStream_t s) {
  if (fd == MFL_F64 && cd == MFL_F64) return restrict_kt<K, double, double>(c, coarse, fine, bf, axf, bc, s);
  if (fd == MFL_F32 && cd == MFL_F64) return restrict_kt<K, float, double>(c, coarse, fine, bf, axf, bc, s);
  if (fd == MFL_F32 && cd == MFL_F32) return restrict_kt<K, float, float>(c, coarse, fine, bf, axf, bc, s);
  return hipErrorInvalidValue;
}

hipError_t launch_restrict_residual(const Context &c, const Level &coarse, const Level &fine,
                                    const void *bf, const void *axf, int fd, void *bc, int cd,
                                    hipStream_t s) {
  if (!fine.tbuf) return hipErrorInvalidValue;
#define CASE(K) return restrict_k<K>(c, coarse, fine, bf, axf, fd, bc, cd, s)
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipErrorInvalidValue;
}

hipError_t launch_dot_partial(const double *a, const double *b, int64_t n, double *partials,
                              hipStream_t s) {
  dot_partial_kernel<<<kReduceBlocks, kBlock, 0, s>>>(a, b, n, partials);
  return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, double *scalars, int which, int op, hipStream_t s) {
  finalize_kernel<<<1, kBlock, 0, s>>>(partials, scalars, which, op);
  return hipGetLastError();
}

hipError_t launch_pcg_update_xr(double *x, double *r, const double *p, const double *q,
                                const double *scalars, int64_t n, double *partials, hipStream_t s) {
  pcg_update_xr_kernel<<<kReduceBlocks, kBlock, 0, s>>>(x, r, p, q, scalars, n, partials);
  return hipGetLastError();
}

hipError_t launch_pcg_update_p(double *p, const double *z, const double *scalars, int64_t n,
                               hipStream_t s) {
  pcg_update_p_kernel<<<grid_for(n), kBlock, 0, s>>>(p, z, scalars, n);
  return hipGetLastError();
}

hipError_t launch_random_start(double *v, const Level &L, uint64_t key, int dmask, hipStream_t s) {
  random_start_kernel<<<grid_for(L.ndofs), kBlock, 0, s>>>(v, L.ndofs, L.N1, key, dmask);
  return hipGetLastError();
}

hipError_t launch_jacobi(const double *dinv, const double *r, double *z, int64_t n, hipStream_t s) {
  jacobi_kernel<<<grid_for(n), kBlock, 0, s>>>(dinv, r, z, n);
  return hipGetLastError();
}

hipError_t launch_zero_boundary(double *v, const Level &L, int dmask, hipStream_t s) {
  zero_boundary_kernel<<<grid_for(L.ndofs), kBlock, 0, s>>>(v, L.N1, dmask);
  return hipGetLastError();
}

}  // namespace mfl
