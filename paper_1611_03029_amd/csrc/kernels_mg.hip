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

// bit: some value is not finite and positive; with prev, change_bit: some value differs
// from prev in its bits.
__global__ void __launch_bounds__(kBlock) check_positive_kernel(const double *v, int64_t n, int *flag, int bit,
                                                               const double *prev, int change_bit) {
  bool bad = false, changed = false;
  GRID_STRIDE(i, n) {
    const double x = v[i];
    bad = bad || !(x > 0.0) || !isfinite(x);
    if (prev) changed = changed || __double_as_longlong(x) != __double_as_longlong(prev[i]);
  }
  if (bad) atomicOr(flag, bit);
  if (changed) atomicOr(flag, change_bit);
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

// Quad form of cheb_first_kernel: four entries per lane in 16-byte accesses, the same
// arithmetic per entry; the n mod 4 trailing entries are done by the first work-group.
#define QUAD_STRIDE(c, nq) \
  for (int64_t c = blockIdx.x * int64_t(kBlock) + threadIdx.x; c < (nq); c += int64_t(gridDim.x) * kBlock)
#define QUAD_TAIL(i, n)   \
  if (blockIdx.x == 0)    \
    for (int64_t i = ((n) & ~int64_t(3)) + threadIdx.x; i < (n); i += kBlock)

template <typename A, typename T>
__global__ void __launch_bounds__(kBlock)
cheb_first_quad_kernel(const A *__restrict__ b_in, T *__restrict__ b_store, const T *__restrict__ dinv,
                       T *__restrict__ d, T *__restrict__ x, int64_t n, T inv_theta) {
  QUAD_STRIDE(c, n >> 2) {
    const Quad<A> bi = load_quad(b_in, 4 * c);
    const Quad<T> di = load_quad(dinv, 4 * c);
    Quad<T> bt, v;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bt.v[j] = T(bi.v[j]);
      v.v[j] = di.v[j] * bt.v[j] * inv_theta;
    }
    if (b_store) store_quad(b_store, 4 * c, bt);
    store_quad(d, 4 * c, v);
    store_quad(x, 4 * c, v);
  }
  QUAD_TAIL(i, n) {
    const T b = T(b_in[i]);
    if (b_store) b_store[i] = b;
    const T v = dinv[i] * b * inv_theta;
    d[i] = v;
    x[i] = v;
  }
}

// Coarse cells per work-group of the transfer kernels (a row along x): fine rows of up to
// about 65 values (2kR + 1), as far as a (2kR + 1)(2k + 1)^2 fine tile stays within LDS bytes.
// Fine rows then move in long contiguous segments, and the work-group's barriers are shared
// by R cells.  The restriction, whose load phase waits on two fine vectors, keeps a smaller
// tile for more resident work-groups.
#ifndef MFL_RESTRICT_LDS
#define MFL_RESTRICT_LDS 12288
#endif
constexpr int kProlongLds = 32768, kRestrictLds = MFL_RESTRICT_LDS;
template <int K, typename TF, int LDS>
constexpr int transfer_row() {
  constexpr int m = 2 * K + 1;
  constexpr int by_len = 32 / K;
  constexpr int by_lds = ((LDS / (m * m * int(sizeof(TF)))) - 1) / (2 * K);
  constexpr int r = by_len < by_lds ? by_len : by_lds;
  return r < 1 ? 1 : r;
}

// Work-group -> row of coarse cells (rx-th row of R cells along x of line (cy, cz)).
struct TransferRow {
  int cx0, nc, cy, cz;
  template <int R>
  __device__ static TransferRow at(int blk, int Ncc) {
    const int nrow = (Ncc + R - 1) / R;
    TransferRow t;
    const int rx = blk % nrow;
    t.cy = (blk / nrow) % Ncc;
    t.cz = blk / (nrow * Ncc);
    t.cx0 = rx * R;
    t.nc = min(R, Ncc - t.cx0);
    return t;
  }
};

// Work-groups of a transfer with rows of R coarse cells; a level whose rows would give fewer
// than kRowMinBlocks work-groups (coarse multigrid levels) uses one cell per work-group, so
// that it still spreads over the chip.
constexpr int kRowMinBlocks = 2048;
inline int transfer_blocks(int R, int Ncc) { return ((Ncc + R - 1) / R) * Ncc * Ncc; }
template <int R>
inline bool use_rows(int Ncc) { return R > 1 && transfer_blocks(R, Ncc) >= kRowMinBlocks; }

// fine += P coarse over a row of up to R coarse cells per work-group: embedding of the
// coarse Q_k basis at the fine nodes, applied direction by direction (z, y on the row's
// coarse points, then x to the fine points).  Each fine node is written by exactly one
// coarse cell (half-open ownership), so no atomics are needed.  Work-groups of one XCD take
// consecutive rows (xcd_block), so that the fine rows' cache lines that neighbouring rows
// share stay in that XCD's L2.
template <int K, typename TC, typename TF, int R>
__global__ void __launch_bounds__(kBlock)
prolongate_kernel(const TC *__restrict__ xc, TF *__restrict__ xf, int Ncc, int dmask, TransferTab tt) {
  constexpr int n = K + 1, m = 2 * K + 1, CX = K * R + 1, FX = 2 * K * R + 1;
  __shared__ double P[m * n];
  __shared__ TF b0[n * n * CX], b1[m * n * CX], b2[m * m * CX];   // [l][b][X], [L][b][X], [L][J][X]
  for (int i = threadIdx.x; i < m * n; i += kBlock) P[i] = tt.P[i];
  const TransferRow w = TransferRow::at<R>(xcd_block(blockIdx.x, gridDim.x), Ncc);
  const int N1c = K * Ncc + 1, N1f = 2 * K * Ncc + 1;
  const int cxn = K * w.nc + 1;   // coarse points of the row along x (the tiles hold CX)
  // (index decompositions use the compile-time extents; entries past the row stay unused)
  constexpr int NC = n * n * CX, IC = (NC + kBlock - 1) / kBlock;
  TC cv[IC];
#pragma unroll
  for (int it = 0; it < IC; ++it) {   // all coarse loads first; entries past the row read a valid address
    const int i = min(int(threadIdx.x) + it * kBlock, NC - 1);
    const int X = i % CX, bl = i / CX, b = bl % n, l = bl / n;
    const int gx = min(K * w.cx0 + X, N1c - 1), gy = w.cy * K + b, gz = w.cz * K + l;
    cv[it] = xc[gx + int64_t(N1c) * (gy + int64_t(N1c) * gz)];
  }
#pragma unroll
  for (int it = 0; it < IC; ++it) {
    const int i = int(threadIdx.x) + it * kBlock;
    if (i >= NC) break;
    const int X = i % CX, bl = i / CX, b = bl % n, l = bl / n;
    const int gx = K * w.cx0 + X, gy = w.cy * K + b, gz = w.cz * K + l;
    const bool bnd = X >= cxn || dirichlet_dof(gx, gy, gz, N1c, dmask);
    b0[i] = bnd ? TF(0) : TF(cv[it]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m * n * CX; i += kBlock) {   // z
    const int X = i % CX, Lb = i / CX, b = Lb % n, L = Lb / n;
    TF s = 0;
#pragma unroll
    for (int l = 0; l < n; ++l) s += TF(P[L * n + l]) * b0[(l * n + b) * CX + X];
    b1[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m * m * CX; i += kBlock) {   // y
    const int X = i % CX, LJ = i / CX, J = LJ % m, L = LJ / m;
    TF s = 0;
#pragma unroll
    for (int b = 0; b < n; ++b) s += TF(P[J * n + b]) * b1[(L * n + b) * CX + X];
    b2[i] = s;
  }
  __syncthreads();
  // x: the fine points of the row that it owns: below the next row's first point unless the
  // row ends the line, J and L below the cell's upper face unless it is the last cell in that
  // direction (half-open ownership)
  const int fxn = 2 * K * w.nc + (w.cx0 + w.nc == Ncc ? 1 : 0);
  for (int i = threadIdx.x; i < FX * m * m; i += kBlock) {
    const int I = i % FX, JL = i / FX, J = JL % m, L = JL / m;
    if (I >= fxn || (J == m - 1 && w.cy < Ncc - 1) || (L == m - 1 && w.cz < Ncc - 1)) continue;
    const int c = min(I / (2 * K), R - 1), Ic = I - 2 * K * c;   // cell of the row, local index
    const int fx = 2 * K * w.cx0 + I, fy = 2 * K * w.cy + J, fz = 2 * K * w.cz + L;
    if (dirichlet_dof(fx, fy, fz, N1f, dmask)) continue;
    TF s = 0;
#pragma unroll
    for (int a = 0; a < n; ++a) s += TF(P[Ic * n + a]) * b2[JL * CX + K * c + a];
    xf[fx + int64_t(N1f) * (fy + int64_t(N1f) * fz)] += s;
  }
}

// Restriction coarse = P^T (b_f - A x_f) (axf == nullptr: P^T b_f) in two kernels without
// atomics.  restrict_cell_kernel: a row of up to R coarse cells per work-group loads the
// row's fine tile once (fine nodes shared by several coarse cells weighted by
// 1/multiplicity, so that the sum over cells is P^T), applies the transposed embedding of
// each cell (x, y, z) and stores each cell's n^3 contributions contiguously in `cellbuf`.
// restrict_gather_kernel: each coarse DoF sums the contributions of the 1 to 8 cells that
// contain it, in a fixed order, and is written once (zero on Dirichlet DoFs).
template <int K, typename TF, int R>
__global__ void __launch_bounds__(kBlock)
restrict_cell_kernel(const TF *__restrict__ bf, const TF *__restrict__ axf, TF *__restrict__ cellbuf, int Ncc,
                     int dmask, TransferTab tt) {
  constexpr int n = K + 1, m = 2 * K + 1, FX = 2 * K * R + 1;
  constexpr int RS = FX * m * m > R * m * n * n ? FX * m * m : R * m * n * n;
  __shared__ double P[m * n];
  __shared__ TF r[RS], t1[R * m * m * n];   // r: [L][J][X], then [c][L][b][a]; t1: [c][L][J][a]
  for (int i = threadIdx.x; i < m * n; i += kBlock) P[i] = tt.P[i];
  const TransferRow w = TransferRow::at<R>(xcd_block(blockIdx.x, gridDim.x), Ncc);
  const int N1f = 2 * K * Ncc + 1;
  const int fxn = 2 * K * w.nc + 1;   // fine points of the row along x (the tile holds FX)
  // weight 1/2 per direction in which the fine node lies on a face shared by two coarse cells
  auto shared_half = [&](int f) { return f % (2 * K) == 0 && f > 0 && f < N1f - 1; };
  // (index decompositions use the compile-time extents; cells past the row are skipped)
  // All of a lane's tile loads are issued before the first is used: one round trip to
  // memory per work-group instead of one per tile entry of the lane.  Entries outside the
  // row read a valid address and are discarded.
  constexpr int NT = FX * m * m, IT = (NT + kBlock - 1) / kBlock;
  TF bv[IT], av[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int i = min(int(threadIdx.x) + it * kBlock, NT - 1);
    const int X = i % FX, JL = i / FX, J = JL % m, L = JL / m;
    const int fx = min(2 * K * w.cx0 + X, N1f - 1), fy = 2 * K * w.cy + J, fz = 2 * K * w.cz + L;
    const int64_t g = fx + int64_t(N1f) * (fy + int64_t(N1f) * fz);
    bv[it] = bf[g];
    av[it] = axf ? axf[g] : TF(0);
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int i = int(threadIdx.x) + it * kBlock;
    if (i >= NT) break;
    const int X = i % FX, JL = i / FX, J = JL % m, L = JL / m;
    const int fx = 2 * K * w.cx0 + X, fy = 2 * K * w.cy + J, fz = 2 * K * w.cz + L;
    TF v = 0;
    if (X < fxn && !dirichlet_dof(fx, fy, fz, N1f, dmask)) {
      TF wgt = 1;
      if (shared_half(fx)) wgt *= TF(0.5);
      if (shared_half(fy)) wgt *= TF(0.5);
      if (shared_half(fz)) wgt *= TF(0.5);
      v = wgt * (axf ? bv[it] - av[it] : bv[it]);
    }
    r[i] = v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R * m * m * n; i += kBlock) {   // x: [c][L][J][a]
    const int a = i % n, cLJ = i / n, LJ = cLJ % (m * m), c = cLJ / (m * m);
    TF s = 0;
#pragma unroll
    for (int I = 0; I < m; ++I) s += TF(P[I * n + a]) * r[LJ * FX + 2 * K * c + I];
    t1[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R * m * n * n; i += kBlock) {   // y: [c][L][b][a] (reuses r)
    const int a = i % n, b = (i / n) % n, cL = i / (n * n);   // cL = c m + L
    TF s = 0;
#pragma unroll
    for (int J = 0; J < m; ++J) s += TF(P[J * n + b]) * t1[(cL * m + J) * n + a];
    r[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R * n * n * n; i += kBlock) {   // z: coarse DoF (a, b, l) of cell c
    const int ab = i % (n * n), l = (i / (n * n)) % n, c = i / (n * n * n);
    if (c >= w.nc) continue;
    TF s = 0;
#pragma unroll
    for (int L = 0; L < m; ++L) s += TF(P[L * n + l]) * r[(c * m + L) * n * n + ab];
    const int64_t cell = (w.cx0 + c) + int64_t(Ncc) * (w.cy + int64_t(Ncc) * w.cz);
    cellbuf[cell * (n * n * n) + l * n * n + ab] = s;
  }
}

// Cells containing coarse grid line g of Nc cells along one direction, with the line's
// local index in each: (g / K, g % K) inside a cell; at a cell vertex also (g / K - 1, K);
// the last line only in the last cell.  Returns the count (1 or 2).
template <int K>
__device__ __forceinline__ int line_cells(int g, int Nc, int (&c)[2], int (&a)[2]) {
  const int q = g / K, r = g - q * K;
  if (q == Nc) {
    c[0] = Nc - 1;
    a[0] = K;
    return 1;
  }
  c[0] = q;
  a[0] = r;
  if (r == 0 && q > 0) {
    c[1] = q - 1;
    a[1] = K;
    return 2;
  }
  return 1;
}

template <int K, typename TF, typename TC>
__global__ void __launch_bounds__(kBlock)
restrict_gather_kernel(const TF *__restrict__ cellbuf, TC *__restrict__ bc, int Ncc, int dmask) {
  constexpr int n = K + 1, n3 = n * n * n;
  const int N1c = K * Ncc + 1;
  const int64_t total = int64_t(N1c) * N1c * N1c;
  GRID_STRIDE(i, total) {
    const int gx = int(i % N1c), gy = int((i / N1c) % N1c), gz = int(i / (int64_t(N1c) * N1c));
    TF s = 0;
    if (!dirichlet_dof(gx, gy, gz, N1c, dmask)) {
      int cx[2], ax[2], cy[2], ay[2], cz[2], az[2];
      const int nx = line_cells<K>(gx, Ncc, cx, ax), ny = line_cells<K>(gy, Ncc, cy, ay),
                nz = line_cells<K>(gz, Ncc, cz, az);
      for (int tz = 0; tz < nz; ++tz)
        for (int ty = 0; ty < ny; ++ty)
          for (int tx = 0; tx < nx; ++tx) {
            const int64_t cell = cx[tx] + int64_t(Ncc) * (cy[ty] + int64_t(Ncc) * cz[tz]);
            s += cellbuf[cell * n3 + ax[tx] + n * (ay[ty] + n * az[tz])];
          }
    }
    bc[i] = TC(s);
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
finalize_kernel(const double *__restrict__ partials, double *__restrict__ sc, int which, int op, int np) {
  __shared__ double red[kBlock];
  double s = 0;
  for (int i = threadIdx.x; i < np; i += kBlock) s += partials[i];
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

hipError_t launch_check_positive(const double *v, int64_t n, int *flag, int bit, hipStream_t s, const double *prev,
                                int change_bit) {
  check_positive_kernel<<<grid_for(n, 1024), kBlock, 0, s>>>(v, n, flag, bit, prev, change_bit);
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
  if (aligned16(b_in, b_store, dinv, d, x)) {
    const int g = grid_for(n / 4);
    if (dtype == MFL_F64) {
      if (in_dtype != MFL_F64) return hipErrorInvalidValue;
      cheb_first_quad_kernel<double, double><<<g, kBlock, 0, s>>>(
          (const double *)b_in, (double *)b_store, (const double *)dinv, (double *)d, (double *)x, n, inv_theta);
    } else if (in_dtype == MFL_F64) {
      cheb_first_quad_kernel<double, float><<<g, kBlock, 0, s>>>(
          (const double *)b_in, (float *)b_store, (const float *)dinv, (float *)d, (float *)x, n, float(inv_theta));
    } else {
      cheb_first_quad_kernel<float, float><<<g, kBlock, 0, s>>>(
          (const float *)b_in, (float *)b_store, (const float *)dinv, (float *)d, (float *)x, n, float(inv_theta));
    }
    return hipGetLastError();
  }
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

// prolongation rows: measured faster up to k = 4 on the fine levels, slower above
template <int K, typename TC, typename TF>
static void prolongate_kt(const Context &c, const Level &coarse, const void *xc, void *xf, hipStream_t s) {
  constexpr int R = K <= 4 ? transfer_row<K, TF, kProlongLds>() : 1;
  const int Ncc = coarse.Nc, dm = dirichlet_mask(c.p);
  if (use_rows<R>(Ncc))
    prolongate_kernel<K, TC, TF, R><<<transfer_blocks(R, Ncc), kBlock, 0, s>>>((const TC *)xc, (TF *)xf, Ncc, dm,
                                                                               c.transfer);
  else
    prolongate_kernel<K, TC, TF, 1><<<transfer_blocks(1, Ncc), kBlock, 0, s>>>((const TC *)xc, (TF *)xf, Ncc, dm,
                                                                               c.transfer);
}

template <int K>
static hipError_t prolongate_k(const Context &c, const Level &coarse, const void *xc, int cd,
                               void *xf, int fd, hipStream_t s) {
  if (cd == MFL_F64 && fd == MFL_F64)
    prolongate_kt<K, double, double>(c, coarse, xc, xf, s);
  else if (cd == MFL_F64 && fd == MFL_F32)
    prolongate_kt<K, double, float>(c, coarse, xc, xf, s);
  else if (cd == MFL_F32 && fd == MFL_F32)
    prolongate_kt<K, float, float>(c, coarse, xc, xf, s);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_prolongate_add(const Context &c, const Level &coarse, const Level &fine,
                                 const void *xc, int cd, void *xf, int fd, hipStream_t s) {
  (void)fine;
#define CASE(K) return prolongate_k<K>(c, coarse, xc, cd, xf, fd, s)
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipErrorInvalidValue;
}

template <int K, typename TF, typename TC>
static hipError_t restrict_kt(const Context &c, const Level &coarse, const Level &fine, const void *bf,
                              const void *axf, void *bc, hipStream_t s) {
  TF *cellbuf = static_cast<TF *>(fine.tbuf);
  constexpr int R = transfer_row<K, TF, kRestrictLds>();
  const int Ncc = coarse.Nc, dm = dirichlet_mask(c.p);
  if (use_rows<R>(Ncc))
    restrict_cell_kernel<K, TF, R><<<transfer_blocks(R, Ncc), kBlock, 0, s>>>((const TF *)bf, (const TF *)axf,
                                                                              cellbuf, Ncc, dm, c.transfer);
  else
    restrict_cell_kernel<K, TF, 1><<<transfer_blocks(1, Ncc), kBlock, 0, s>>>((const TF *)bf, (const TF *)axf,
                                                                              cellbuf, Ncc, dm, c.transfer);
  restrict_gather_kernel<K, TF, TC><<<grid_for(coarse.ndofs), kBlock, 0, s>>>(cellbuf, (TC *)bc, coarse.Nc,
                                                                              dirichlet_mask(c.p));
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

hipError_t launch_finalize(const double *partials, double *scalars, int which, int op, hipStream_t s,
                           int n_partials) {
  finalize_kernel<<<1, kBlock, 0, s>>>(partials, scalars, which, op, n_partials);
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
