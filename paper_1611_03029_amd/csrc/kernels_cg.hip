// Continuous Q_k Laplacian on hexahedra: matrix-free operator kernels (Sec. 3, eq. mf_eval).
//
// Cell computation.  n^2 lanes per cell (n = k+1); each lane owns one line of n points
// of its cell in registers and applies the 1D matrices along that line in even-odd form
// (Sec. 3: about half the products; the coefficients are compile-time constants, see
// ct_tables.h).  Between contraction directions the cell's n^3 values are transposed
// through LDS.  Lanes are reinterpreted per phase as (x, y) owners of z-lines, (x, z)
// owners of y-lines or (y, z) owners of x-lines.  LDS index of point (x, y, z) of a cell:
// z n^2 + y n + x.  Where n^2 <= 64 every cell lies inside one wavefront and the phases
// are separated by wavefront-level synchronization only.
//
// Assembly without global atomics.  A work-group owns a brick of cells (a few chunks of
// CX x BY x BZ cells along x).  The last contraction of every cell adds its n^3 results
// into the brick's DoF tile in LDS (FP64 LDS atomics; cells share faces).  Every grid DoF
// is owned by exactly one brick (half-open ranges per direction, the last brick also
// owning the domain's upper plane).  After its cells the work-group stores the owned DoFs
// of the tile (Dirichlet DoFs get the identity-row value src) and writes the tile's upper
// faces, which belong to neighbouring bricks, to the brick's halo record.  A second
// kernel adds the halo records into the lower faces of each brick.  No global atomics and
// no clearing pass.  A DoF shared by cells of one brick sums their contributions with LDS
// atomics in whatever order the wavefronts reach them, so results agree between runs to
// rounding, not bitwise.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "ct_tables.h"
#include "device_common.h"

namespace mfl {

namespace {

constexpr int kBlock = 256;


template <int K>
struct Shape {
  static constexpr int n = K + 1, n2 = n * n, n3 = n2 * n, cpb = kBlock / n2;
};

// Cells per chunk in x, y, z for degree K, chunks per brick along x (chunks), y (ny) and z
// (nz), and the lane layout:
// wave = true places every cell's n^2 lanes inside one wavefront (64 / n^2 cells per
// wavefront, four wavefronts per work-group), so the phases of a cell need no work-group
// barrier; wave = false packs the cells densely over the work-group (cells may straddle
// wavefronts; required for n^2 > 64).
template <int K> struct Brick;
template <> struct Brick<1> { static constexpr int x = 4, y = 4, z = 4, chunks = 1, ny = 1, nz = 1; static constexpr bool wave = true; };
template <> struct Brick<2> { static constexpr int x = 3, y = 3, z = 3, chunks = 1, ny = 1, nz = 1; static constexpr bool wave = true; };
template <> struct Brick<3> { static constexpr int x = 4, y = 2, z = 2, chunks = 2, ny = 1, nz = 1; static constexpr bool wave = true; };
template <> struct Brick<4> { static constexpr int x = 2, y = 2, z = 2, chunks = 4, ny = 1, nz = 1; static constexpr bool wave = true; };
template <> struct Brick<5> { static constexpr int x = 3, y = 2, z = 1, chunks = 2, ny = 1, nz = 1; static constexpr bool wave = false; };
template <> struct Brick<6> { static constexpr int x = 2, y = 2, z = 1, chunks = 2, ny = 1, nz = 1; static constexpr bool wave = true; };
template <> struct Brick<7> { static constexpr int x = 2, y = 2, z = 1, chunks = 2, ny = 1, nz = 1; static constexpr bool wave = true; };
template <> struct Brick<8> { static constexpr int x = 3, y = 1, z = 1, chunks = 2, ny = 1, nz = 1; static constexpr bool wave = false; };

// Taller brick shapes for degree K, precision T and geometry where they were measured faster
// on large meshes.  On Cartesian cells (no metric stream) the operator costs little per DoF
// and the halo of the brick faces takes a large share at low degree; bricks that also span
// two chunks in y (and z) cut it (measured on 64^3 cells, operator plus halo addition: Q2
// -18% / -20% (FP64 / FP32), Q3 -9% / -3%, Q5 and Q6 FP64 -10% and -7%; slower for Q4 and
// for FP32 at Q5 and Q6).  They give a mesh fewer work-groups, so a level uses them only
// when at least kTallMinBricks of them fill it (coarse multigrid levels keep Brick<K>).
template <int K, typename T, bool CURVED>
struct TallShape : Brick<K> {
  static constexpr bool tall = false;
};
template <> struct TallShape<2, float, false> : Brick<2> { static constexpr int chunks = 4, ny = 2, nz = 2; static constexpr bool tall = true; };
template <> struct TallShape<2, double, false> : Brick<2> { static constexpr int chunks = 2, ny = 2, nz = 2; static constexpr bool tall = true; };
template <> struct TallShape<3, float, false> : Brick<3> { static constexpr int chunks = 2, ny = 2, nz = 1; static constexpr bool tall = true; };
template <> struct TallShape<3, double, false> : Brick<3> { static constexpr int chunks = 2, ny = 2, nz = 1; static constexpr bool tall = true; };
template <> struct TallShape<5, double, false> : Brick<5> { static constexpr int chunks = 2, ny = 2, nz = 1; static constexpr bool tall = true; };
template <> struct TallShape<6, double, false> : Brick<6> { static constexpr int chunks = 2, ny = 2, nz = 1; static constexpr bool tall = true; };
#ifndef MFL_TALL_MIN_BRICKS
#define MFL_TALL_MIN_BRICKS 512
#endif
constexpr int kTallMinBricks = MFL_TALL_MIN_BRICKS;

// One-chunk bricks for coarse multigrid levels.  A work-group walks the chunks of its brick
// one after another, so on a level with few default bricks (fewer than kShortMaxBricks
// work-groups on 256 compute units) the chip is mostly idle and the time is the length of
// that chain; one-chunk bricks give the level more, shorter work-groups (continuous
// levels, Cartesian and curved; degrees whose default brick has several chunks).
template <int K>
struct ShortShape : Brick<K> {
  static constexpr int chunks = 1, ny = 1, nz = 1;
};
constexpr int kShortMaxBricks = 256;

// Brick shape S of a level: 0 Brick<K>, 1 TallShape, 2 ShortShape.
enum { kShapeDefault = 0, kShapeTall = 1, kShapeShort = 2 };
template <int K, typename T, bool CURVED, int S>
using ShapeOf = typename std::conditional<
    S == kShapeTall, TallShape<K, T, CURVED>,
    typename std::conditional<S == kShapeShort, ShortShape<K>, Brick<K>>::type>::type;

struct CellCtx {
  int i0, i1;        // lane coordinates within the cell
  int cz;            // cell coordinate in z (x, y enter through gx, gy)
  bool inblk;        // lane belongs to a cell slot of the work-group
  bool active;       // ... and that cell exists
  bool bxy;          // lane's z-line lies on a Dirichlet x- or y-face
  int64_t base;      // grid index of the lane's z-line start
  int64_t plane;     // N1^2
  int N1, K, dmask;
};

__device__ __forceinline__ CellCtx make_ctx(int K, int n, int p, bool inblk, bool active, int cx, int cy,
                                            int cz, int N1, int dmask) {
  CellCtx c;
  c.i0 = p % n;
  c.i1 = p / n;
  c.cz = cz;
  c.inblk = inblk;
  c.active = active;
  const int gx = cx * K + c.i0, gy = cy * K + c.i1;
  c.bxy = on_dirichlet(gx, N1, dmask) || on_dirichlet(gy, N1, dmask);
  c.plane = int64_t(N1) * N1;
  c.base = gx + int64_t(N1) * gy + c.plane * (int64_t(cz) * K);
  c.N1 = N1;
  c.K = K;
  c.dmask = dmask;
  return c;
}

__device__ __forceinline__ bool z_bnd(const CellCtx &c, int l) {
  return c.bxy || on_dirichlet(c.cz * c.K + l, c.N1, c.dmask);
}

// The lane's z-line of src (Dirichlet DoFs and inactive lanes read as zero: the columns of
// the Dirichlet DoFs are eliminated).
template <int N, typename T>
__device__ __forceinline__ void gather_zline(const CellCtx &cc, const T *__restrict__ src, T (&u)[N]) {
#pragma unroll
  for (int l = 0; l < N; ++l) u[l] = (cc.active && !z_bnd(cc, l)) ? src[cc.base + cc.plane * l] : T(0);
}

// The metric of the lane's z-line of Gauss points (layout [6][q] per cell).  The metric is
// streamed once per application; with NT the loads are non-temporal so that they do not
// displace the src lines that neighbouring bricks re-read from L2 (measured: 4-10% faster
// for the FP64 kernels up to k = 4, slower for FP32 and higher degrees).
template <int N, bool NT, typename T>
__device__ __forceinline__ void load_metric(bool active, const T *__restrict__ gm, int p, T (&g)[6][N]) {
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int l = 0; l < N; ++l) {
      const T *a = gm + c * N * N * N + l * N * N + p;
      if constexpr (NT)
        g[c][l] = active ? __builtin_nontemporal_load(a) : T(0);
      else
        g[c][l] = active ? *a : T(0);
    }
}

template <int K, typename T>
constexpr bool kStreamMetric = sizeof(T) == 8 && K <= 4;

struct NoOp {
  __device__ void operator()() const {}
};

// ---------------------------------------------------------------------------------------
// Cartesian cell: constant Jacobian h I, so with exact Gauss quadrature the element
// operator of eq. (mf_eval) factors into the Kronecker sum
//   A_e = scale (K (x) M (x) M + M (x) K (x) M + M (x) M (x) K),  scale = kappa_e h,
// of the reference 1D mass M and stiffness K of the GLL basis (the same numbers as the
// quadrature form, re-associated).  Seven 1D applications per line set.
// u: the lane's gathered z-line.  Buffers A..D: n^3 each; C and D may alias A and B (every
// phase reads only the lines its lane then rewrites).  TXS == 0: y_e ends in A;
// TXS > 0: y_e is added (LDS atomics) into `tile` (row stride TXS, plane stride
// TXS * TYS, this cell's origin at `tile`).  after_gather() runs once u is consumed (it may
// overwrite u with the next cell's line).  Contains 3 cell barriers.
template <int K, typename T, int TXS = 0, int TYS = 0, bool WL = false, class AfterGather = NoOp>
__device__ __forceinline__ void cart_cell(const CellCtx &cc, const T (&u)[K + 1], T scale, T *A, T *B, T *C,
                                          T *D, const EOTab<K + 1, T> &eo, double *tile = nullptr,
                                          AfterGather after_gather = {}) {
  constexpr int n = K + 1, n2 = n * n;
  const int i0 = cc.i0, i1 = cc.i1, p = i0 + n * i1;
  // z-lines (x = i0, y = i1): M and K along z
  if (cc.inblk) {
    T a[n], b[n];
    eo_apply<n, 1>(eo.M, u, a);
    eo_apply<n, 1>(eo.K, u, b);
#pragma unroll
    for (int q = 0; q < n; ++q) {
      A[q * n2 + p] = a[q];
      B[q * n2 + p] = b[q];
    }
  }
  after_gather();
  cell_sync<WL>();
  // y-lines (x = i0, z = i1): P = M_y (M_z u), S = K_y (M_z u) + M_y (K_z u)
  if (cc.inblk) {
    T a1[n], a2[n], pp[n], s1[n], s2[n];
#pragma unroll
    for (int b = 0; b < n; ++b) {
      a1[b] = A[i1 * n2 + b * n + i0];
      a2[b] = B[i1 * n2 + b * n + i0];
    }
    eo_apply<n, 1>(eo.M, a1, pp);
    eo_apply<n, 1>(eo.K, a1, s1);
    eo_apply<n, 1>(eo.M, a2, s2);
#pragma unroll
    for (int q = 0; q < n; ++q) {
      C[i1 * n2 + q * n + i0] = pp[q];
      D[i1 * n2 + q * n + i0] = s1[q] + s2[q];
    }
  }
  cell_sync<WL>();
  // x-lines (y = i0, z = i1): y = scale (K_x P + M_x S)
  if (cc.inblk) {
    T pa[n], sa[n], y1[n], y2[n];
#pragma unroll
    for (int a = 0; a < n; ++a) {
      pa[a] = C[i1 * n2 + i0 * n + a];
      sa[a] = D[i1 * n2 + i0 * n + a];
    }
    eo_apply<n, 1>(eo.K, pa, y1);
    eo_apply<n, 1>(eo.M, sa, y2);
#pragma unroll
    for (int q = 0; q < n; ++q) {
      const T y = (y1[q] + y2[q]) * scale;
      if constexpr (TXS > 0)
        lds_add(tile + i1 * (TXS * TYS) + i0 * TXS + q, double(y));
      else
        A[i1 * n2 + i0 * n + q] = y;
    }
  }
  cell_sync<WL>();
}

// ---------------------------------------------------------------------------------------
// Curved cell (general isoparametric geometry): the per-quadrature-point tensor
// G_q = w_q det J_q J_q^{-1} J_q^{-T} (6 unique entries, computed at setup and streamed
// from HBM, layout [cell][6][q]; kappa applied on the fly).  Collocation form of sum
// factorization: values at the Gauss points v = (S (x) S (x) S) u, reference gradient by
// the Gauss-point collocation derivative D per direction, q = kappa G grad v, then the
// transposed sequence.  u: the lane's gathered z-line; g: the metric of the lane's z-line
// of Gauss points.  Buffers A..C; y_e ends in A (TXS == 0) or is added into `tile` as for
// cart_cell.  after_gather() runs once u is consumed, after_metric() once g and kap are
// (both may overwrite them with the next cell's operands, so that those loads are in
// flight during the rest of this cell).  Contains 9 cell barriers.
template <int K, typename T, int TXS = 0, int TYS = 0, bool WL = false, class AfterGather = NoOp,
          class AfterMetric = NoOp>
__device__ __forceinline__ void curved_cell(const CellCtx &cc, const T (&u)[K + 1], const T (&g)[6][K + 1],
                                            const T &kap, T *A, T *B, T *C, const EOTab<K + 1, T> &eo,
                                            double *tile = nullptr, AfterGather after_gather = {},
                                            AfterMetric after_metric = {}) {
  constexpr int n = K + 1, n2 = n * n;
  const int i0 = cc.i0, i1 = cc.i1, p = i0 + n * i1;
  // F1: z-lines (x = i0, y = i1): S along z
  if (cc.inblk) {
    T t[n];
    eo_apply<n, 1>(eo.S, u, t);
#pragma unroll
    for (int q = 0; q < n; ++q) A[q * n2 + p] = t[q];
  }
  after_gather();
  cell_sync<WL>();
  // F2: y-lines (x = i0, z = i1): S along y
  if (cc.inblk) {
    T r[n], t[n];
#pragma unroll
    for (int b = 0; b < n; ++b) r[b] = A[i1 * n2 + b * n + i0];
    eo_apply<n, 1>(eo.S, r, t);
#pragma unroll
    for (int q = 0; q < n; ++q) B[i1 * n2 + q * n + i0] = t[q];
  }
  cell_sync<WL>();
  // F3: x-lines (y = i0, z = i1): S along x -> values v at the Gauss points; D -> dv/dx
  if (cc.inblk) {
    T r[n], v[n], d[n];
#pragma unroll
    for (int a = 0; a < n; ++a) r[a] = B[i1 * n2 + i0 * n + a];
    eo_apply<n, 1>(eo.S, r, v);
    eo_apply<n, -1>(eo.D, v, d);
#pragma unroll
    for (int q = 0; q < n; ++q) {
      A[i1 * n2 + i0 * n + q] = v[q];
      C[i1 * n2 + i0 * n + q] = d[q];
    }
  }
  cell_sync<WL>();
  // F4: y-lines (x = i0, z = i1): D along y -> dv/dy
  if (cc.inblk) {
    T r[n], d[n];
#pragma unroll
    for (int b = 0; b < n; ++b) r[b] = A[i1 * n2 + b * n + i0];
    eo_apply<n, -1>(eo.D, r, d);
#pragma unroll
    for (int q = 0; q < n; ++q) B[i1 * n2 + q * n + i0] = d[q];
  }
  cell_sync<WL>();
  // F5 + B1: z-lines (x = i0, y = i1): D along z -> dv/dz; quadrature-point operation;
  // transposed derivative along z.  Each lane rewrites only its own z-line.
  if (cc.inblk) {
    T r[n], gz[n], fx[n], fy[n], fz[n], acc[n];
#pragma unroll
    for (int l = 0; l < n; ++l) r[l] = A[l * n2 + p];
    eo_apply<n, -1>(eo.D, r, gz);
#pragma unroll
    for (int l = 0; l < n; ++l) {
      const T ux = C[l * n2 + p], uy = B[l * n2 + p], uz = gz[l];
      // metric components 00, 11, 22, 01, 02, 12
      fx[l] = kap * (g[0][l] * ux + g[3][l] * uy + g[4][l] * uz);
      fy[l] = kap * (g[3][l] * ux + g[1][l] * uy + g[5][l] * uz);
      fz[l] = kap * (g[4][l] * ux + g[5][l] * uy + g[2][l] * uz);
    }
    eo_apply_t<n, -1>(eo.D, fz, acc);
#pragma unroll
    for (int l = 0; l < n; ++l) {
      A[l * n2 + p] = acc[l];
      C[l * n2 + p] = fx[l];
      B[l * n2 + p] = fy[l];
    }
  }
  after_metric();
  cell_sync<WL>();
  // B2: y-lines (x = i0, z = i1): acc += D^T along y of fy
  if (cc.inblk) {
    T f[n], d[n];
#pragma unroll
    for (int b = 0; b < n; ++b) f[b] = B[i1 * n2 + b * n + i0];
    eo_apply_t<n, -1>(eo.D, f, d);
#pragma unroll
    for (int b = 0; b < n; ++b) A[i1 * n2 + b * n + i0] += d[b];
  }
  cell_sync<WL>();
  // B3: x-lines (y = i0, z = i1): acc += D^T along x of fx; S^T along x
  if (cc.inblk) {
    T f[n], d[n], acc[n], w[n];
#pragma unroll
    for (int a = 0; a < n; ++a) f[a] = C[i1 * n2 + i0 * n + a];
    eo_apply_t<n, -1>(eo.D, f, d);
#pragma unroll
    for (int a = 0; a < n; ++a) acc[a] = A[i1 * n2 + i0 * n + a] + d[a];
    eo_apply_t<n, 1>(eo.S, acc, w);
#pragma unroll
    for (int i = 0; i < n; ++i) B[i1 * n2 + i0 * n + i] = w[i];
  }
  cell_sync<WL>();
  // B4: y-lines (x = i0, z = i1): S^T along y
  if (cc.inblk) {
    T r[n], w[n];
#pragma unroll
    for (int b = 0; b < n; ++b) r[b] = B[i1 * n2 + b * n + i0];
    eo_apply_t<n, 1>(eo.S, r, w);
#pragma unroll
    for (int i = 0; i < n; ++i) A[i1 * n2 + i * n + i0] = w[i];
  }
  cell_sync<WL>();
  // B5: z-lines (x = i0, y = i1): S^T along z; y_e back into A (own z-line only) or into
  // the tile
  if (cc.inblk) {
    T r[n], w[n];
#pragma unroll
    for (int l = 0; l < n; ++l) r[l] = A[l * n2 + p];
    eo_apply_t<n, 1>(eo.S, r, w);
#pragma unroll
    for (int i = 0; i < n; ++i) {
      if constexpr (TXS > 0)
        lds_add(tile + i * (TXS * TYS) + i1 * TXS + i0, double(w[i]));
      else
        A[i * n2 + p] = w[i];
    }
  }
  cell_sync<WL>();
}

// ---------------------------------------------------------------------------------------
// Curved cells with the metric formed on the fly.  The isoparametric map of the curved
// meshes is x = X + d(X) (1,1,1) with X affine (cell size h) and d the Q_k interpolant of
// the node displacements, so J = h I + (1,1,1) (grad d)^T: a rank-one update of h I.  With
// g = grad d at a quadrature point and s = g_x + g_y + g_z, det J = h^2 (h + s) and
// (Sherman-Morrison) w det J J^{-1} J^{-T} = w [(h + s) I - (1 g^T + g 1^T) + |g|^2 / (h + s) 1 1^T],
// i.e. G_ab = w (h + s) delta_ab - w (g_a + g_b) + w |g|^2 / (h + s).
// otf_metric forms grad d at the Gauss points of the cell by the collocation scheme of
// curved_cell (S along z, y, x, then D along x, y, z: 6 one-dimensional applications per
// lane in 5 phases) from the lane's z-line d of node displacements, and returns the metric
// of the lane's z-line of Gauss points in the layout of load_metric (00, 11, 22, 01, 02, 12).
// Buffers A..C are free again when it returns.
// 1 / x from the hardware reciprocal estimate refined by Newton steps (two in FP64, one in
// FP32), each of which squares the relative error; within an ulp or two of the division.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// scale multiplies the metric (the cell's kappa, so that the operator phases take kappa 1).
template <int K, typename T, bool WL>
__device__ __forceinline__ void otf_metric(const CellCtx &cc, const T (&d)[K + 1], T *A, T *B, T *C,
                                           const EOTab<K + 1, T> &eo, T h, T scale, T (&g)[6][K + 1]) {
  constexpr int n = K + 1, n2 = n * n;
  constexpr const ct::DGTab<n, T> &gauss = ct::DGTables<n, T>::tab;   // Gauss weights w
  const int i0 = cc.i0, i1 = cc.i1, p = i0 + n * i1;
  if (cc.inblk) {   // z-lines: S along z
    T t[n];
    eo_apply<n, 1>(eo.S, d, t);
#pragma unroll
    for (int q = 0; q < n; ++q) A[q * n2 + p] = t[q];
  }
  cell_sync<WL>();
  if (cc.inblk) {   // y-lines: S along y
    T r[n], t[n];
#pragma unroll
    for (int b = 0; b < n; ++b) r[b] = A[i1 * n2 + b * n + i0];
    eo_apply<n, 1>(eo.S, r, t);
#pragma unroll
    for (int q = 0; q < n; ++q) B[i1 * n2 + q * n + i0] = t[q];
  }
  cell_sync<WL>();
  if (cc.inblk) {   // x-lines: S along x -> d at the Gauss points; D along x -> dd/dx
    T r[n], v[n], dd[n];
#pragma unroll
    for (int a = 0; a < n; ++a) r[a] = B[i1 * n2 + i0 * n + a];
    eo_apply<n, 1>(eo.S, r, v);
    eo_apply<n, -1>(eo.D, v, dd);
#pragma unroll
    for (int q = 0; q < n; ++q) {
      A[i1 * n2 + i0 * n + q] = v[q];
      C[i1 * n2 + i0 * n + q] = dd[q];
    }
  }
  cell_sync<WL>();
  if (cc.inblk) {   // y-lines: D along y -> dd/dy
    T r[n], dd[n];
#pragma unroll
    for (int b = 0; b < n; ++b) r[b] = A[i1 * n2 + b * n + i0];
    eo_apply<n, -1>(eo.D, r, dd);
#pragma unroll
    for (int q = 0; q < n; ++q) B[i1 * n2 + q * n + i0] = dd[q];
  }
  cell_sync<WL>();
  if (cc.inblk) {   // z-lines: D along z -> dd/dz, then the metric of the lane's points
    T r[n], gz[n];
#pragma unroll
    for (int l = 0; l < n; ++l) r[l] = A[l * n2 + p];
    eo_apply<n, -1>(eo.D, r, gz);
    const T w01 = gauss.w[i0] * gauss.w[i1] * scale;
#pragma unroll
    for (int l = 0; l < n; ++l) {
      const T gx = C[l * n2 + p], gy = B[l * n2 + p], gzl = gz[l];
      const T hs = h + (gx + gy + gzl);
      const T t = (gx * gx + gy * gy + gzl * gzl) * recip(hs);
      const T w = w01 * gauss.w[l];
      const T wx = w * gx, wy = w * gy, wz = w * gzl, wd = w * (hs + t), wt = w * t;
      g[0][l] = wd - T(2) * wx;
      g[1][l] = wd - T(2) * wy;
      g[2][l] = wd - T(2) * wz;
      g[3][l] = wt - wx - wy;
      g[4][l] = wt - wx - wz;
      g[5][l] = wt - wy - wz;
    }
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c)
#pragma unroll
      for (int l = 0; l < n; ++l) g[c][l] = T(0);
  }
  cell_sync<WL>();
}

// The lane's z-line of a field of node values without the Dirichlet mask (geometry data);
// inactive lanes read zero.
template <int N, typename T>
__device__ __forceinline__ void gather_zline_nodes(const CellCtx &cc, const T *__restrict__ v, T (&u)[N]) {
#pragma unroll
  for (int l = 0; l < N; ++l) u[l] = cc.active ? v[cc.base + cc.plane * l] : T(0);
}

// ---------------------------------------------------------------------------------------
// Brick apply kernel.

// Raw buffer resource at p (no stride, 2^31 - 1 bytes in range, 32-bit data format).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t brick_rsrc(const void *p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, 0x7fffffff, 0x00020000);
}

// Buffer load at byte offset voff (per lane) + soff (the same in every lane: taken from the
// first lane, so that it is kept in a scalar register) from the resource.
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  soff = __builtin_amdgcn_readfirstlane(soff);
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

struct BrickGrid {
  int Nc, N1;
  int sx;              // cells per brick in x (multiple of the chunk width)
  int my, mz;          // brick extent in y and z in DoF intervals
  int nbx, nby, nbz;   // bricks per direction
  int dmask;           // Dirichlet face mask
  int off32;           // per-lane offsets within a brick fit in 31 bits (see brick_grid)
};

// Halo record of a brick (upper faces owned by neighbouring bricks), M = brick extent in
// DoF intervals: the x face (MY+1)(MZ+1) [Z][Y], then the y face without x = MX,
// MX (MZ+1) [Z][X], then the z face without x = MX and y = MY, MX MY [Y][X].  x is the
// fastest index of the y and z faces, so their reads and writes are coalesced.
__host__ __device__ __forceinline__ int halo_size(int MX, int MY, int MZ) {
  return (MY + 1) * (MZ + 1) + MX * (MZ + 1) + MX * MY;
}

__device__ __forceinline__ int halo_index(int X, int Y, int Z, int MX, int MY, int MZ) {
  const int fx = Z * (MY + 1) + Y;
  const int fy = (MY + 1) * (MZ + 1) + Z * MX + X;
  const int fz = (MY + 1) * (MZ + 1) + MX * (MZ + 1) + Y * MX + X;
  return X == MX ? fx : (Y == MY ? fy : fz);
}

// dst = A src for CG Q_K, one brick per work-group.  The work-group walks the chunks of its
// brick (x fastest, then y, then z; chunks outside the mesh are skipped); every lane holds
// the src line (and, on curved meshes, the metric and kappa) of its cell of the next chunk
// in registers, loaded while the current chunk is computed.
// OTF (curved only): `metric` holds the node displacements of the level (one value per DoF)
// and the metric is formed on the fly (otf_metric); otherwise the stored per-point metric.
template <int K, typename T, bool CURVED, int SHAPE, bool OTF = false>
__global__ void __launch_bounds__(kBlock)
apply_brick_kernel(const T *__restrict__ src, T *__restrict__ dst, T *__restrict__ halo,
                   const T *__restrict__ kappa, const T *__restrict__ metric, BrickGrid bg, T h) {
  constexpr const EOTab<K + 1, T> &eo = ct::Tables<K + 1, T>::eo;
  using S = Shape<K>;
  using Bk = ShapeOf<K, T, CURVED, SHAPE>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3;
  constexpr int CX = Bk::x, BY = Bk::y, BZ = Bk::z, CPB = CX * BY * BZ;
  constexpr int NCX = Bk::chunks, NCY = Bk::ny, NCZ = Bk::nz, NCH = NCX * NCY * NCZ;
  constexpr bool WL = Bk::wave;
  static_assert(WL ? (n2 <= 64 && CPB <= (kBlock / 64) * (64 / n2)) : CPB * n2 <= kBlock,
                "chunk does not fit the work-group");
  constexpr int MX = NCX * CX * K, MY = NCY * BY * K, MZ = NCZ * BZ * K;   // brick extent in DoF intervals
  constexpr int TX = MX + 1, TY = MY + 1, TZ = MZ + 1;
  constexpr int NBUF = CURVED ? 3 : 2;   // Cartesian: cart_cell runs in place in two buffers
  constexpr int ITEMS = TX * TY * TZ, ITERS = (ITEMS + kBlock - 1) / kBlock;
  __shared__ T sm[NBUF][CPB * n3];
  __shared__ double tile[ITEMS];   // FP64 accumulation also for T = float (ds_add_f32 is slow)

  const int brick = xcd_block(blockIdx.x, bg.nbx * bg.nby * bg.nbz);
  const int bx = brick % bg.nbx, by = (brick / bg.nbx) % bg.nby, bz = brick / (bg.nbx * bg.nby);
  const int t = threadIdx.x;
  const LaneMap<n2, WL> lm(t, CPB);
  const int lc = lm.used ? lm.slot : 0, p = lm.p;
  const int lx = lc % CX, ly = (lc / CX) % BY, lz = lc / (CX * BY);
  const bool inblk = lm.used;
  const int Nc = bg.Nc, N1 = bg.N1;
  const int cx0 = bx * NCX * CX, cy0 = by * NCY * BY, cz0 = bz * NCZ * BZ;
  // chunks per direction that hold cells of the mesh
  const int ncx = min(NCX, (Nc - cx0 + CX - 1) / CX), ncy = min(NCY, (Nc - cy0 + BY - 1) / BY),
            ncz = min(NCZ, (Nc - cz0 + BZ - 1) / BZ);
  T *A = sm[0] + lc * n3, *B = sm[1] + lc * n3, *C = sm[CURVED ? 2 : 0] + lc * n3;

  // the lane's cell in chunk (jx, jy, jz) (inactive for jx < 0: no chunk)
  auto cell_at = [&](int jx, int jy, int jz, CellCtx &cc, int64_t &cell) {
    const int cx = cx0 + jx * CX + lx, cy = cy0 + jy * BY + ly, cz = cz0 + jz * BZ + lz;
    const bool active = inblk && jx >= 0 && cx < Nc && cy < Nc && cz < Nc;
    cell = active ? cx + int64_t(Nc) * (cy + int64_t(Nc) * cz) : 0;
    cc = make_ctx(K, n, p, inblk, active, cx, cy, cz, N1, bg.dmask);
  };

#pragma unroll
  for (int it = 0; it < ITERS; ++it) {
    const int i = t + it * kBlock;
    if (ITEMS % kBlock == 0 || i < ITEMS) tile[i] = 0.0;
  }
  __syncthreads();

  const bool lastx = bx == bg.nbx - 1, lasty = by == bg.nby - 1, lastz = bz == bg.nbz - 1;
  const int64_t plane = int64_t(N1) * N1;
  const int gx0 = cx0 * K, gy0 = cy0 * K, gz0 = cz0 * K;
  const int64_t gbase = gx0 + int64_t(N1) * gy0 + plane * gz0;
  // interior bricks without Dirichlet DoFs and without cut-off cells need no per-item tests
  const bool plain = gx0 + MX < N1 - 1 && gy0 + MY < N1 - 1 && gz0 + MZ < N1 - 1 &&
                     !((bg.dmask & 1) && (gx0 == 0 || gy0 == 0 || gz0 == 0));

  // Cartesian interior bricks take a walk without tests; the others the general walk.  (The
  // same walk on curved cells, with the metric read through a buffer resource as well, was
  // measured 4% slower at k = 4.)
  const bool fast = !CURVED && plain && bg.off32;
  if constexpr (!CURVED) {
    if (fast) {
      // Interior brick: every cell of every chunk exists and reads no Dirichlet DoF, so the
      // walk has no per-lane tests, and each operand is read through a buffer resource at the
      // brick (a base common to the work-group), a byte offset of the lane fixed for the whole
      // walk and a uniform byte offset of the chunk and line.  All offsets stay below 2^31
      // (checked on the host), so no lane does 64-bit address arithmetic.
      const int i0 = p % n, i1 = p / n;
      const uint32_t so = inblk ? uint32_t(sizeof(T)) * uint32_t((lx * K + i0) + N1 * (ly * K + i1) +
                                                                 uint32_t(plane) * uint32_t(lz * K))
                                : 0u;
      const uint32_t ko = inblk ? uint32_t(sizeof(T)) * uint32_t(lx + Nc * (ly + Nc * lz)) : 0u;
      const int64_t cell0 = cx0 + int64_t(Nc) * (cy0 + int64_t(Nc) * cz0);
      const auto rs = brick_rsrc(src + gbase), rk = brick_rsrc(kappa + cell0);
      // operands of chunk j: the src z-line and kappa of the lane's cell
      auto load = [&](int j, T(&u)[n], T &kap) {
        const int jx = j % NCX, jy = (j / NCX) % NCY, jz = j / (NCX * NCY);
        const uint32_t sc = uint32_t(jx * CX * K) + uint32_t(N1) * uint32_t(jy * BY * K) +
                            uint32_t(plane) * uint32_t(jz * BZ * K);
#pragma unroll
        for (int l = 0; l < n; ++l) u[l] = buf_load<T>(rs, so, uint32_t(sizeof(T)) * (sc + uint32_t(plane) * l));
        const uint32_t kc = uint32_t(jx * CX) + uint32_t(Nc) * (uint32_t(jy * BY) + uint32_t(Nc) * uint32_t(jz * BZ));
        kap = buf_load<T>(rk, ko, uint32_t(sizeof(T)) * kc);
      };
      CellCtx cc;
      cc.i0 = i0;
      cc.i1 = i1;
      cc.inblk = inblk;
      T u[n];
      T kap;
      load(0, u, kap);
#pragma unroll
      for (int j = 0; j < NCH; ++j) {
        const int jx = j % NCX, jy = (j / NCX) % NCY, jz = j / (NCX * NCY);
        double *ctile = tile + ((jz * BZ + lz) * K) * (TX * TY) + ((jy * BY + ly) * K) * TX + (jx * CX + lx) * K;
        T kn = kap;
        cart_cell<K, T, TX, TY, WL>(cc, u, kap * h, A, B, A, B, eo, ctile, [&] {
          if (j + 1 < NCH) load(j + 1, u, kn);
        });
        kap = kn;
      }
    }
  }
  if (!fast) {
  CellCtx cc;
  int64_t cell;
  cell_at(0, 0, 0, cc, cell);
  T u[n];
  T g[6][CURVED ? n : 1];
  T dz[OTF ? n : 1];   // on the fly: the node displacements of the lane's z-line
  gather_zline(cc, src, u);
  if constexpr (CURVED && OTF)
    gather_zline_nodes(cc, metric, dz);
  else if constexpr (CURVED)
    load_metric<n, kStreamMetric<K, T>>(cc.active, metric + cell * (6 * n3), p, g);
  T kap = cc.active ? kappa[cell] : T(0);

#pragma unroll
  for (int j = 0; j < NCH; ++j) {
    const int jx = j % NCX, jy = (j / NCX) % NCY, jz = j / (NCX * NCY);
    if (jx >= ncx || jy >= ncy || jz >= ncz) continue;
    // the next chunk of the walk that holds cells
    const int nx = jx + 1 < ncx ? jx + 1 : (jy + 1 < ncy || jz + 1 < ncz ? 0 : -1);
    const int ny = jx + 1 < ncx ? jy : (jy + 1 < ncy ? jy + 1 : 0);
    const int nz = jx + 1 < ncx || jy + 1 < ncy ? jz : jz + 1;
    CellCtx cn;
    int64_t celln;
    cell_at(nx, ny, nz, cn, celln);
    double *ctile = tile + ((jz * BZ + lz) * K) * (TX * TY) + ((jy * BY + ly) * K) * TX + (jx * CX + lx) * K;
    if constexpr (CURVED && OTF) {
      otf_metric<K, T, WL>(cc, dz, A, B, C, eo, h, kap, g);   // kappa folded into the metric
      const T one = T(1);
      curved_cell<K, T, TX, TY, WL>(
          cc, u, g, one, A, B, C, eo, ctile, [&] { gather_zline(cn, src, u); },
          [&] {
            gather_zline_nodes(cn, metric, dz);
            kap = cn.active ? kappa[celln] : T(0);
          });
    } else if constexpr (CURVED) {
      curved_cell<K, T, TX, TY, WL>(
          cc, u, g, kap, A, B, C, eo, ctile, [&] { gather_zline(cn, src, u); },
          [&] {
            load_metric<n, kStreamMetric<K, T>>(cn.active, metric + celln * (6 * n3), p, g);
            kap = cn.active ? kappa[celln] : T(0);
          });
    } else {
      T kn = 0;
      cart_cell<K, T, TX, TY, WL>(cc, u, kap * h, A, B, A, B, eo, ctile, [&] {
        gather_zline(cn, src, u);
        kn = cn.active ? kappa[celln] : T(0);
      });
      kap = kn;
    }
    cc = cn;
    cell = celln;
  }
  }
  __syncthreads();

  // Stores.  Tile items with X < MX, Y < MY, Z < MZ are owned by this brick; items on the
  // upper faces are owned by a neighbouring brick (-> halo record) unless the brick is the
  // last one in every direction in which the item lies on its upper face (-> dst).
  // Dirichlet DoFs get the identity-row value src.
  constexpr int OWN = MX * MY * MZ, ITO = (OWN + kBlock - 1) / kBlock;
  constexpr int HS = (MY + 1) * (MZ + 1) + MX * (MZ + 1) + MX * MY, ITH = (HS + kBlock - 1) / kBlock;
  T *hrec = halo + int64_t(brick) * HS;
  // tile position of halo record item i (layout of halo_index)
  auto halo_item = [&](int i, int &X, int &Y, int &Z) {
    if (i < (MY + 1) * (MZ + 1)) {
      X = MX;
      Y = i % (MY + 1);
      Z = i / (MY + 1);
    } else if (i < (MY + 1) * (MZ + 1) + MX * (MZ + 1)) {
      const int q = i - (MY + 1) * (MZ + 1);
      X = q % MX;
      Y = MY;
      Z = q / MX;
    } else {
      const int q = i - (MY + 1) * (MZ + 1) - MX * (MZ + 1);
      X = q % MX;
      Y = q / MX;
      Z = MZ;
    }
  };
  if (plain) {
    // Interior brick: every owned item goes to dst and every face item to the halo record.
    // These loops hold stores only; a load in the same loop (the Dirichlet values below)
    // makes the compiler wait for every store to complete before the next item.
#pragma unroll
    for (int it = 0; it < ITO; ++it) {
      const int i = t + it * kBlock;
      if (OWN % kBlock == 0 || i < OWN) {
        const int X = i % MX, Y = (i / MX) % MY, Z = i / (MX * MY);
        dst[gbase + (X + N1 * Y) + plane * Z] = T(tile[X + TX * (Y + TY * Z)]);
      }
    }
#pragma unroll
    for (int it = 0; it < ITH; ++it) {
      const int i = t + it * kBlock;
      if (HS % kBlock == 0 || i < HS) {
        int X, Y, Z;
        halo_item(i, X, Y, Z);
        hrec[i] = T(tile[X + TX * (Y + TY * Z)]);
      }
    }
    return;
  }
  // Boundary brick: items outside the mesh are skipped and Dirichlet DoFs take the value of
  // src.  Those src values are loaded first, in loops without stores, so that the stores do
  // not wait one by one.
  T so[ITO], sh[ITH];
#pragma unroll
  for (int it = 0; it < ITO; ++it) {
    const int i = t + it * kBlock;
    const int X = i % MX, Y = (i / MX) % MY, Z = i / (MX * MY);
    const int gx = gx0 + X, gy = gy0 + Y, gz = gz0 + Z;
    const bool in = (OWN % kBlock == 0 || i < OWN) && gx < N1 && gy < N1 && gz < N1;
    so[it] = (in && dirichlet_dof(gx, gy, gz, N1, bg.dmask)) ? src[gbase + (X + N1 * Y) + plane * Z] : T(0);
  }
#pragma unroll
  for (int it = 0; it < ITH; ++it) {
    const int i = t + it * kBlock;
    int X, Y, Z;
    halo_item(i, X, Y, Z);
    const int gx = gx0 + X, gy = gy0 + Y, gz = gz0 + Z;
    const bool in = (HS % kBlock == 0 || i < HS) && gx < N1 && gy < N1 && gz < N1;
    sh[it] = (in && dirichlet_dof(gx, gy, gz, N1, bg.dmask)) ? src[gbase + (X + N1 * Y) + plane * Z] : T(0);
  }
#pragma unroll
  for (int it = 0; it < ITO; ++it) {
    const int i = t + it * kBlock;
    if (OWN % kBlock == 0 || i < OWN) {
      const int X = i % MX, Y = (i / MX) % MY, Z = i / (MX * MY);
      const int gx = gx0 + X, gy = gy0 + Y, gz = gz0 + Z;
      if (gx < N1 && gy < N1 && gz < N1) {
        const T v = T(tile[X + TX * (Y + TY * Z)]);
        dst[gbase + (X + N1 * Y) + plane * Z] = dirichlet_dof(gx, gy, gz, N1, bg.dmask) ? so[it] : v;
      }
    }
  }
#pragma unroll
  for (int it = 0; it < ITH; ++it) {
    const int i = t + it * kBlock;
    if (HS % kBlock == 0 || i < HS) {
      int X, Y, Z;
      halo_item(i, X, Y, Z);
      const int gx = gx0 + X, gy = gy0 + Y, gz = gz0 + Z;
      if (gx < N1 && gy < N1 && gz < N1) {
        const T v = T(tile[X + TX * (Y + TY * Z)]);
        const bool is_halo = (X == MX && !lastx) || (Y == MY && !lasty) || (Z == MZ && !lastz);
        if (is_halo)
          hrec[i] = v;
        else
          dst[gbase + (X + N1 * Y) + plane * Z] = dirichlet_dof(gx, gy, gz, N1, bg.dmask) ? sh[it] : v;
      }
    }
  }
}

// dst += halo contributions on the lower faces of every brick (DoFs whose index is a
// positive multiple of the brick extent M in some direction).  Each such DoF is visited
// once (x faces, then y faces off x faces, then z faces off both; x is the fastest index
// within the y and z faces) and sums, in a fixed order, the upper-face values of the 1, 3
// or 7 lower bricks sharing it.  A thread takes kHaloPer face positions kBlock apart and
// issues the loads of all of them before the first store; 32-bit index arithmetic with
// multiply-shift divisions (sizes checked on the host).
constexpr int kHaloPer = 4;
struct HaloDiv {
  FastDiv plane, n1, mx, my, mz;
};

template <int K, typename T>
__global__ void __launch_bounds__(kBlock)
halo_add_kernel(T *__restrict__ dst, const T *__restrict__ halo, BrickGrid bg, HaloDiv hv) {
  const int MX = bg.sx * K, MY = bg.my, MZ = bg.mz;
  const unsigned N1 = bg.N1, P = N1 * N1;
  const unsigned fx = unsigned(bg.nbx - 1) * P, fy = unsigned(bg.nby - 1) * P,
                 fz = unsigned(bg.nbz - 1) * P;
  const unsigned total = fx + fy + fz;
  const int hs = halo_size(MX, MY, MZ);
  const int M[3] = {MX, MY, MZ}, NB[3] = {bg.nbx, bg.nby, bg.nbz};
  const unsigned stride = gridDim.x * kBlock * kHaloPer;
  for (unsigned base = blockIdx.x * kBlock * kHaloPer + threadIdx.x; base < total; base += stride) {
    bool ok[kHaloPer];
    uint32_t gi[kHaloPer];
    int b[kHaloPer][3], X[kHaloPer][3];
    uint8_t sh[kHaloPer];
    T d[kHaloPer], s[kHaloPer];
#pragma unroll
    for (int j = 0; j < kHaloPer; ++j) {
      const unsigned id = base + j * kBlock;
      int g[3] = {0, 0, 0};
      bool skip = id >= total;
      if (!skip) {
        // face f of the direction, position r within the face plane
        const unsigned q = id < fx ? id : (id < fx + fy ? id - fx : id - fx - fy);
        const unsigned f = hv.plane.div(q), r = q - f * P, hi = hv.n1.div(r), lo = r - hi * N1;
        if (id < fx) {
          g[0] = int(f + 1) * MX;
          g[1] = int(lo);
          g[2] = int(hi);
        } else if (id < fx + fy) {
          g[0] = int(lo);
          g[1] = int(f + 1) * MY;
          g[2] = int(hi);
        } else {
          g[0] = int(lo);
          g[1] = int(hi);
          g[2] = int(f + 1) * MZ;
        }
        const unsigned qx = hv.mx.div(unsigned(g[0])), qy = hv.my.div(unsigned(g[1]));
        const bool onx = g[0] == int(qx) * MX && qx >= 1 && int(qx) < bg.nbx;
        const bool ony = g[1] == int(qy) * MY && qy >= 1 && int(qy) < bg.nby;
        skip = (id >= fx && onx) || (id >= fx + fy && ony) || dirichlet_dof(g[0], g[1], g[2], N1, bg.dmask);
      }
      ok[j] = !skip;
      const int qg[3] = {int(hv.mx.div(unsigned(g[0]))), int(hv.my.div(unsigned(g[1]))), int(hv.mz.div(unsigned(g[2])))};
      uint8_t m = 0;
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        b[j][e] = min(qg[e], NB[e] - 1);
        X[j][e] = g[e] - b[j][e] * M[e];
        if (X[j][e] == 0 && b[j][e] > 0) m |= uint8_t(1 << e);
      }
      sh[j] = m;
      gi[j] = unsigned(g[0]) + N1 * (unsigned(g[1]) + N1 * unsigned(g[2]));
    }
    // record entry of the lower brick across the shared directions in mask m
    auto entry = [&](int j, int m) {
      const int ob0 = b[j][0] - (m & 1), ob1 = b[j][1] - ((m >> 1) & 1), ob2 = b[j][2] - ((m >> 2) & 1);
      const int tx = (m & 1) ? MX : X[j][0], ty = (m & 2) ? MY : X[j][1], tz = (m & 4) ? MZ : X[j][2];
      const int64_t ob = ob0 + int64_t(bg.nbx) * (ob1 + int64_t(bg.nby) * ob2);
      return ob * hs + halo_index(tx, ty, tz, MX, MY, MZ);
    };
    // dst and the first record entry (every visited DoF lies on at least one face)
#pragma unroll
    for (int j = 0; j < kHaloPer; ++j) {
      if (ok[j]) {
        d[j] = dst[gi[j]];
        s[j] = halo[entry(j, (sh[j] & 1) ? 1 : ((sh[j] & 2) ? 2 : 4))];
      }
    }
    // edges and corners (3 and 7 entries) add the others in increasing m
#pragma unroll
    for (int j = 0; j < kHaloPer; ++j) {
      if (ok[j] && (sh[j] & (sh[j] - 1))) {
        const int m0 = (sh[j] & 1) ? 1 : ((sh[j] & 2) ? 2 : 4);
        for (int m = m0 + 1; m < 8; ++m)
          if ((m & sh[j]) == m) s[j] += halo[entry(j, m)];
      }
    }
#pragma unroll
    for (int j = 0; j < kHaloPer; ++j)
      if (ok[j]) dst[gi[j]] = d[j] + s[j];
  }
}

// Chebyshev update of the smoother fused with the halo addition (continuous Q_k), one DoF per
// thread in memory order: ax = the brick kernel's value plus, on the lower faces of a brick,
// the record entries of the 1, 3 or 7 lower bricks sharing the DoF (summed in the order of
// halo_add_kernel), then d = c1 d + c2 dinv (b - ax) and x += d (and the FP64 copy of x when
// x64 is given), as the plain Chebyshev update.  The face DoFs are no longer read and written
// by a pass of their own.  32-bit DoF indices (checked on the host).
struct DofDiv {
  FastDiv n1, mx, my, mz;
};

// A x at DoF (gx, gy, gz): the brick kernel's value a plus the halo record entries of the
// lower bricks sharing the DoF, in the order of halo_add_kernel.
template <int K, typename T>
__device__ __forceinline__ T cheb_halo_ax(T a, int gx, int gy, int gz, const T *__restrict__ halo, const BrickGrid &bg,
                                          const DofDiv &dv, int hs) {
  const int MX = bg.sx * K, MY = bg.my, MZ = bg.mz;
  const int g[3] = {gx, gy, gz};
  const int q[3] = {int(dv.mx.div(gx)), int(dv.my.div(gy)), int(dv.mz.div(gz))};
  const int M[3] = {MX, MY, MZ}, NB[3] = {bg.nbx, bg.nby, bg.nbz};
  int bb[3], X[3];
  bool sh[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    bb[e] = min(q[e], NB[e] - 1);
    X[e] = g[e] - bb[e] * M[e];
    sh[e] = X[e] == 0 && bb[e] > 0;
  }
  if (!(sh[0] || sh[1] || sh[2]) || dirichlet_dof(gx, gy, gz, bg.N1, bg.dmask)) return a;
  auto entry = [&](int m) {
    const int ob0 = bb[0] - (m & 1), ob1 = bb[1] - ((m >> 1) & 1), ob2 = bb[2] - ((m >> 2) & 1);
    const int tx = (m & 1) ? MX : X[0], ty = (m & 2) ? MY : X[1], tz = (m & 4) ? MZ : X[2];
    const int64_t ob = ob0 + int64_t(bg.nbx) * (ob1 + int64_t(bg.nby) * ob2);
    return ob * hs + halo_index(tx, ty, tz, MX, MY, MZ);
  };
  const int m0 = sh[0] ? 1 : (sh[1] ? 2 : 4);
  T sum = halo[entry(m0)];
  for (int m = m0 + 1; m < 8; ++m) {
    if (((m & 1) && !sh[0]) || ((m & 2) && !sh[1]) || ((m & 4) && !sh[2])) continue;
    sum += halo[entry(m)];
  }
  return a + sum;
}

template <int K, typename T>
__global__ void __launch_bounds__(kBlock)
cheb_halo_kernel(const T *__restrict__ ax, const T *__restrict__ halo, const T *__restrict__ b,
                 const T *__restrict__ dinv, T *__restrict__ d, T *__restrict__ x,
                 double *__restrict__ x64, BrickGrid bg, DofDiv dv, T c1, T c2) {
  const int N1 = bg.N1;
  const uint32_t n = uint32_t(N1) * uint32_t(N1) * uint32_t(N1);
  const int hs = halo_size(bg.sx * K, bg.my, bg.mz);
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const uint32_t r = dv.n1.div(i), gz = dv.n1.div(r);
    const int gx = int(i - r * uint32_t(N1)), gy = int(r - gz * uint32_t(N1));
    const T a = cheb_halo_ax<K, T>(ax[i], gx, gy, int(gz), halo, bg, dv, hs);
    const T dn = c1 * d[i] + c2 * dinv[i] * (b[i] - a);
    const T xn = x[i] + dn;
    d[i] = dn;
    x[i] = xn;
    if (x64) x64[i] = double(xn);
  }
}

// Quad form of cheb_halo_kernel: four consecutive DoFs per lane, b, A x, D^{-1}, d and x
// moved in 16-byte accesses (the vectors are 16-byte aligned, checked on the host).  The
// grid coordinates of the first DoF come from two divisions; the other three follow by
// stepping along x (at most one of them wraps to the next row).  The halo entries are added
// per DoF exactly as in cheb_halo_kernel, so the results are the same bit for bit.  The
// N1^3 mod 4 trailing DoFs are done by the first work-group.
template <int K, typename T>
__global__ void __launch_bounds__(kBlock)
cheb_halo_quad_kernel(const T *__restrict__ ax, const T *__restrict__ halo, const T *__restrict__ b,
                      const T *__restrict__ dinv, T *__restrict__ d, T *__restrict__ x,
                      double *__restrict__ x64, BrickGrid bg, DofDiv dv, T c1, T c2) {
  const int N1 = bg.N1;
  const uint32_t n = uint32_t(N1) * uint32_t(N1) * uint32_t(N1), nq = n >> 2;
  const int hs = halo_size(bg.sx * K, bg.my, bg.mz);
  auto update = [&](T a, T bi, T di, T dd, T xx, T &dn, T &xn) {
    dn = c1 * dd + c2 * di * (bi - a);
    xn = xx + dn;
  };
  for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < nq; c += gridDim.x * kBlock) {
    const uint32_t i0 = 4 * c;
    const Quad<T> aq = load_quad(ax, i0), bq = load_quad(b, i0), iq = load_quad(dinv, i0),
                  dq = load_quad(d, i0), xq = load_quad(x, i0);
    const uint32_t r = dv.n1.div(i0), gz0 = dv.n1.div(r);
    const int gx0 = int(i0 - r * uint32_t(N1)), gy0 = int(r - gz0 * uint32_t(N1));
    Quad<T> dn, xn;
    Quad<double> x8;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int gx = gx0 + j, gy = gy0, gz = int(gz0);
      if (gx >= N1) {
        gx -= N1;
        if (++gy == N1) {
          gy = 0;
          ++gz;
        }
      }
      update(cheb_halo_ax<K, T>(aq.v[j], gx, gy, gz, halo, bg, dv, hs), bq.v[j], iq.v[j], dq.v[j], xq.v[j], dn.v[j],
             xn.v[j]);
      x8.v[j] = double(xn.v[j]);
    }
    store_quad(d, i0, dn);
    store_quad(x, i0, xn);
    if (x64) store_quad(x64, i0, x8);
  }
  if (blockIdx.x == 0)
    for (uint32_t i = 4 * nq + threadIdx.x; i < n; i += kBlock) {
      const uint32_t r = dv.n1.div(i), gz = dv.n1.div(r);
      const int gx = int(i - r * uint32_t(N1)), gy = int(r - gz * uint32_t(N1));
      T dn, xn;
      update(cheb_halo_ax<K, T>(ax[i], gx, gy, int(gz), halo, bg, dv, hs), b[i], dinv[i], d[i], x[i], dn, xn);
      d[i] = dn;
      x[i] = xn;
      if (x64) x64[i] = double(xn);
    }
}

// ---------------------------------------------------------------------------------------
// Per-cell gradient kernel: g_c = -lambda_c^T A_c^{(kappa=1)} u_c (CPB cells per group).
// OTF: `metric` holds the node displacements and the metric is formed on the fly.
template <int K, typename T, bool CURVED, bool OTF = false>
__global__ void __launch_bounds__(kBlock)
kappa_grad_kernel(const T *__restrict__ u, const T *__restrict__ lam, T *__restrict__ grad,
                  const T *__restrict__ metric, int Nc, int N1, T h, int dmask) {
  constexpr const EOTab<K + 1, T> &eo = ct::Tables<K + 1, T>::eo;
  using S = Shape<K>;
  constexpr int n = S::n, n2 = S::n2, n3 = S::n3, CPB = S::cpb;
  constexpr int NBUF = CURVED ? 3 : 2;   // Cartesian: cart_cell runs in place in two buffers
  __shared__ T sm[NBUF][CPB * n3];
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int t = threadIdx.x, lc = t / n2, p = t - lc * n2;
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
  const CellCtx cc = make_ctx(K, n, p, inblk, active, cx, cy, cz, N1, dmask);
  const int slot = inblk ? lc : 0;
  T *A = sm[0] + slot * n3, *B = sm[1] + slot * n3, *C = sm[CURVED ? 2 : 0] + slot * n3;
  T ul[n];
  gather_zline(cc, u, ul);
  if constexpr (CURVED) {
    T g[6][n];
    if constexpr (OTF) {
      T dz[n];
      gather_zline_nodes(cc, metric, dz);
      otf_metric<K, T, false>(cc, dz, A, B, C, eo, h, T(1), g);
    } else {
      load_metric<n, false>(active, metric + (active ? cell : 0) * (6 * n3), p, g);
    }
    curved_cell<K, T>(cc, ul, g, T(1), A, B, C, eo);
  } else {
    cart_cell<K, T>(cc, ul, active ? h : T(0), A, B, A, B, eo);
  }
  T partial = 0;
  if (active) {
#pragma unroll
    for (int l = 0; l < n; ++l)
      if (!z_bnd(cc, l)) partial += A[l * n2 + p] * lam[cc.base + cc.plane * l];
  }
  if (inblk) B[p] = partial;   // B is not used after the cell computation
  __syncthreads();
  if (active && p == 0) {
    T s = 0;
    for (int j = 0; j < n2; ++j) s += B[j];
    grad[cell] = -s;
  }
}

// dst = src on Dirichlet DoFs, 0 elsewhere.
template <typename T>
__global__ void __launch_bounds__(kBlock)
boundary_init_kernel(const T *__restrict__ src, T *__restrict__ dst, int N1, int dmask) {
  const int64_t n = int64_t(N1) * N1 * N1;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const int x = int(i % N1), y = int((i / N1) % N1), z = int(i / (int64_t(N1) * N1));
    const bool bnd = dirichlet_dof(x, y, z, N1, dmask);
    dst[i] = bnd ? src[i] : T(0);
  }
}

inline int grid_for(int64_t items, int cap = 65536) {
  int64_t g = (items + kBlock - 1) / kBlock;
  return int(g < 1 ? 1 : (g > cap ? cap : g));
}

// Bricks: chunk shape from Brick<K>; the x extent is a multiple of the chunk width chosen so
// that there are about MFL_TARGET_BRICKS bricks (enough work-groups to fill the chip) when
// the mesh allows, which keeps the strided x-face halos to a few planes.
template <int K, typename T, bool CURVED, int SHAPE>
BrickGrid brick_grid(int Nc, int N1, int dmask) {
  using Bk = ShapeOf<K, T, CURVED, SHAPE>;
  BrickGrid bg;
  bg.Nc = Nc;
  bg.N1 = N1;
  bg.sx = Bk::x * Bk::chunks;
  bg.my = Bk::y * Bk::ny * K;
  bg.mz = Bk::z * Bk::nz * K;
  bg.nbx = (Nc + bg.sx - 1) / bg.sx;
  bg.nby = (Nc + Bk::y * Bk::ny - 1) / (Bk::y * Bk::ny);
  bg.nbz = (Nc + Bk::z * Bk::nz - 1) / (Bk::z * Bk::nz);
  bg.dmask = dmask;
  // byte offsets of the interior walk from the brick's first DoF and first cell: src within
  // the brick's mz + 1 planes of DoFs, kappa within its planes of cells
  constexpr double lim = 2147483648.0;
  const double plane = double(N1) * N1, cplane = double(Nc) * Nc;
  bg.off32 = sizeof(T) * plane * (bg.mz + 1) < lim && sizeof(T) * cplane * (Bk::z * Bk::nz + 1) < lim;
  return bg;
}

template <int K, typename T, bool CURVED, int SHAPE>
int64_t brick_count(int Nc) {
  const BrickGrid bg = brick_grid<K, T, CURVED, SHAPE>(Nc, K * Nc + 1, 0);
  return int64_t(bg.nbx) * bg.nby * bg.nbz;
}

template <int K>
constexpr bool kHasShort = Brick<K>::chunks > 1;

// The brick shape of a level: the tall shape when it exists and still gives the mesh
// kTallMinBricks work-groups; one-chunk bricks on levels with fewer than kShortMaxBricks
// default bricks; Brick<K> otherwise.
template <int K, typename T, bool CURVED>
int level_shape(int Nc) {
  if constexpr (TallShape<K, T, CURVED>::tall) {
    if (brick_count<K, T, CURVED, kShapeTall>(Nc) >= kTallMinBricks) return kShapeTall;
  }
  if constexpr (kHasShort<K>) {
    if (brick_count<K, T, CURVED, kShapeDefault>(Nc) < kShortMaxBricks) return kShapeShort;
  }
  return kShapeDefault;
}

// The brick grid of a level (shape chosen by level_shape).
template <int K, typename T, bool CURVED>
BrickGrid level_grid(int Nc, int N1, int dmask) {
  switch (level_shape<K, T, CURVED>(Nc)) {
    case kShapeTall: return brick_grid<K, T, CURVED, kShapeTall>(Nc, N1, dmask);
    case kShapeShort: return brick_grid<K, T, CURVED, kShapeShort>(Nc, N1, dmask);
    default: return brick_grid<K, T, CURVED, kShapeDefault>(Nc, N1, dmask);
  }
}

template <int K, typename T, bool CURVED>
int64_t halo_elements(int Nc) {
  const BrickGrid bg = level_grid<K, T, CURVED>(Nc, K * Nc + 1, 3);
  return int64_t(bg.nbx) * bg.nby * bg.nbz * halo_size(bg.sx * K, bg.my, bg.mz);
}

}  // namespace

int64_t cg_halo_elements(int k, int Nc, bool curved) {
#define CASE(K)                                                                                \
  return curved ? std::max(halo_elements<K, double, true>(Nc), halo_elements<K, float, true>(Nc)) \
                : std::max(halo_elements<K, double, false>(Nc), halo_elements<K, float, false>(Nc))
  switch (k) {
    case 1: CASE(1);
    case 2: CASE(2);
    case 3: CASE(3);
    case 4: CASE(4);
    case 5: CASE(5);
    case 6: CASE(6);
    case 7: CASE(7);
    case 8: CASE(8);
    default: return 0;
  }
#undef CASE
}

hipError_t launch_boundary_init(const Context &c, const Level &L, int dtype, const void *src,
                                void *dst, hipStream_t s) {
  const int dir = dirichlet_mask(c.p);
  const int grid = grid_for(L.ndofs, 8192);
  if (dtype == MFL_F64)
    boundary_init_kernel<double><<<grid, kBlock, 0, s>>>((const double *)src, (double *)dst, L.N1, dir);
  else
    boundary_init_kernel<float><<<grid, kBlock, 0, s>>>((const float *)src, (float *)dst, L.N1, dir);
  return hipGetLastError();
}

template <int K, typename T>
static hipError_t cg_apply_k(const Context &c, const Level &L, const Tab<kMaxN, T> &tab, const T *kappa,
                             const T *metric, const T *src, T *dst, T *halo, hipStream_t s, int dmask,
                             const LaunchEvents *ev) {
  const int dm = dmask < 0 ? dirichlet_mask(c.p) : dmask;
  (void)tab;
  const T *none = nullptr;
  if (c.p.geometry == MFL_GEOM_CURVED) {
    auto curved = [&](auto shape) {
      constexpr int S = decltype(shape)::value;
      const BrickGrid bg = brick_grid<K, T, true, S>(L.Nc, L.N1, dm);
      if (metric_on_the_fly(c.p))
        launch_timed(apply_brick_kernel<K, T, true, S, true>, bg.nbx * bg.nby * bg.nbz, kBlock, s, ev, src, dst, halo,
                     kappa, metric, bg, T(L.h));
      else
        launch_timed(apply_brick_kernel<K, T, true, S>, bg.nbx * bg.nby * bg.nbz, kBlock, s, ev, src, dst, halo,
                     kappa, metric, bg, T(L.h));
    };
    if constexpr (kHasShort<K>) {
      if (level_shape<K, T, true>(L.Nc) == kShapeShort) {
        curved(std::integral_constant<int, kShapeShort>{});
        return hipGetLastError();
      }
    }
    curved(std::integral_constant<int, kShapeDefault>{});
  } else {
    const int shape = level_shape<K, T, false>(L.Nc);
    if constexpr (TallShape<K, T, false>::tall) {
      if (shape == kShapeTall) {
        const BrickGrid bg = brick_grid<K, T, false, kShapeTall>(L.Nc, L.N1, dm);
        launch_timed(apply_brick_kernel<K, T, false, kShapeTall>, bg.nbx * bg.nby * bg.nbz, kBlock, s, ev, src,
                     dst, halo, kappa, none, bg, T(L.h));
        return hipGetLastError();
      }
    }
    if constexpr (kHasShort<K>) {
      if (shape == kShapeShort) {
        const BrickGrid bg = brick_grid<K, T, false, kShapeShort>(L.Nc, L.N1, dm);
        launch_timed(apply_brick_kernel<K, T, false, kShapeShort>, bg.nbx * bg.nby * bg.nbz, kBlock, s, ev, src,
                     dst, halo, kappa, none, bg, T(L.h));
        return hipGetLastError();
      }
    }
    const BrickGrid bg = brick_grid<K, T, false, kShapeDefault>(L.Nc, L.N1, dm);
    launch_timed(apply_brick_kernel<K, T, false, kShapeDefault>, bg.nbx * bg.nby * bg.nbz, kBlock, s, ev, src,
                 dst, halo, kappa, none, bg, T(L.h));
  }
  return hipGetLastError();
}

template <int K, typename T>
static hipError_t cg_halo_k(const Context &c, const Level &L, T *dst, const T *halo, hipStream_t s,
                            int dmask) {
  const int dm = dmask < 0 ? dirichlet_mask(c.p) : dmask;
  const BrickGrid bg = c.p.geometry == MFL_GEOM_CURVED ? level_grid<K, T, true>(L.Nc, L.N1, dm)
                                                       : level_grid<K, T, false>(L.Nc, L.N1, dm);
  const int64_t total = int64_t(bg.nbx - 1 + bg.nby - 1 + bg.nbz - 1) * L.N1 * L.N1;
  if (total == 0) return hipSuccess;
  // 32-bit face positions and DoF indices
  if (total >= (int64_t(1) << 31) || int64_t(L.N1) * L.N1 * L.N1 >= (int64_t(1) << 32)) return hipErrorInvalidValue;
  const HaloDiv hv{FastDiv(uint32_t(L.N1) * uint32_t(L.N1)), FastDiv(uint32_t(L.N1)), FastDiv(uint32_t(bg.sx * K)),
                   FastDiv(uint32_t(bg.my)), FastDiv(uint32_t(bg.mz))};
  halo_add_kernel<K, T><<<grid_for((total + kHaloPer - 1) / kHaloPer, 16384), kBlock, 0, s>>>(dst, halo, bg, hv);
  return hipGetLastError();
}

template <int K, typename T>
static hipError_t cg_cheb_halo_k(const Context &c, const Level &L, const T *b, const T *ax, const T *dinv,
                                 T *d, T *x, double *x64, double c1, double c2, hipStream_t s) {
  const int dm = dirichlet_mask(c.p);
  const BrickGrid bg = c.p.geometry == MFL_GEOM_CURVED ? level_grid<K, T, true>(L.Nc, L.N1, dm)
                                                       : level_grid<K, T, false>(L.Nc, L.N1, dm);
  if (L.ndofs >= (int64_t(1) << 31)) return hipErrorInvalidValue;   // 32-bit DoF index space
  const DofDiv dv{FastDiv(uint32_t(L.N1)), FastDiv(uint32_t(bg.sx * K)), FastDiv(uint32_t(bg.my)),
                  FastDiv(uint32_t(bg.mz))};
  // four DoFs per lane where the grid stays full (8192 work-groups); on smaller levels, whose
  // kernels are latency-bound, one DoF per lane spreads the halo additions over more lanes
  if (L.ndofs >= int64_t(4) * 8192 * kBlock && aligned16(ax, b, dinv, d, x, x64))
    cheb_halo_quad_kernel<K, T><<<grid_for(L.ndofs / 4, 8192), kBlock, 0, s>>>(ax, (const T *)L.halo, b, dinv, d, x,
                                                                               x64, bg, dv, T(c1), T(c2));
  else
    cheb_halo_kernel<K, T><<<grid_for(L.ndofs, 8192), kBlock, 0, s>>>(ax, (const T *)L.halo, b, dinv, d, x, x64, bg,
                                                                      dv, T(c1), T(c2));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Coarse-grid solve of the multigrid (Sec. 4.1) on a small continuous level in one
// work-group: all `steps` updates of the Chebyshev iteration from x = 0 over [lo, hi] of the
// Jacobi-scaled operator (theta = (lo + hi) / 2, delta = (hi - lo) / 2), with x and A x in
// LDS and b, D^{-1} and d in registers.  Each update applies the operator cell by cell (the
// Kronecker-sum cell of cart_cell or the curved cell, added into A x with LDS atomics; identity rows on
// Dirichlet DoFs), then d = c1 d + c2 D^{-1} (b - A x), x += d.  The coarsest level holds a
// few hundred to a few thousand DoFs: there the operator and update kernels of every
// update are bound by launch and memory latency, while here one launch does all updates.
// The loop count is `steps`, the same in every thread, so every barrier is reached.
// Curved levels (GEOM 1: stored metric, 2: metric formed from the node displacements) take
// the curved cell in three buffers; there every lane holds one cell for the whole solve
// (NPASS = 1), so its geometry factors are formed once, before the updates.
template <int K, int NC, int GEOM>
struct CoarseShape {
  static constexpr int n = K + 1, n2 = n * n, n3 = n2 * n;
  static constexpr int N1 = K * NC + 1, N = N1 * N1 * N1, NPT = (N + kBlock - 1) / kBlock;
  static constexpr int CELLS = NC * NC * NC, CPP = kBlock / n2, NPASS = (CELLS + CPP - 1) / CPP;
  static constexpr int NBUF = GEOM == 0 ? 2 : 3;
  static constexpr long lds = long(sizeof(double)) * (2L * N + long(NBUF) * CPP * n3);
  static constexpr bool fits = lds <= 150L * 1024 && NPT <= 32 && (GEOM == 0 || NPASS == 1);
};

template <int K, int NC, int GEOM>
__global__ void __launch_bounds__(kBlock)
coarse_cheb_kernel(const double *__restrict__ b, const double *__restrict__ dinv,
                   const double *__restrict__ kappa, const double *__restrict__ geo, double *__restrict__ x_out,
                   double *__restrict__ x64, double h, int dmask, int steps, double theta,
                   double delta) {
  using CS = CoarseShape<K, NC, GEOM>;
  constexpr const EOTab<K + 1, double> &eo = ct::Tables<K + 1, double>::eo;
  constexpr int n = CS::n, n2 = CS::n2, n3 = CS::n3, N1 = CS::N1, N = CS::N, NPT = CS::NPT;
  constexpr int CELLS = CS::CELLS, CPP = CS::CPP, NPASS = CS::NPASS;
  __shared__ double xs[N], ax[N], buf[CS::NBUF][CPP * n3];
  const int t = threadIdx.x;
  const int slot = t / n2, p = t % n2;
  const bool used = slot < CPP;
  double *A = buf[0] + (used ? slot : 0) * n3, *B = buf[1] + (used ? slot : 0) * n3;
  double *C = buf[CS::NBUF - 1] + (used ? slot : 0) * n3;
  double bb[NPT], di[NPT], d[NPT];
  bool dir[NPT];
  const double inv_theta = 1.0 / theta;
  // curved: the metric of the lane's z-line of Gauss points in its (only) cell, with kappa
  // folded in when it is formed on the fly
  double g[6][GEOM == 0 ? 1 : n];
  double kcell = 1.0;
  if constexpr (GEOM != 0) {
    const int cell = slot;
    const bool active = used && cell < CELLS;
    const int cx = active ? cell % NC : 0, cy = active ? (cell / NC) % NC : 0, cz = active ? cell / (NC * NC) : 0;
    const CellCtx cc = make_ctx(K, n, p, used, active, cx, cy, cz, N1, dmask);
    const double kap = active ? kappa[cell] : 0.0;
    if constexpr (GEOM == 2) {
      double dz[n];
      gather_zline_nodes(cc, geo, dz);
      otf_metric<K, double, false>(cc, dz, A, B, C, eo, h, kap, g);
    } else {
      load_metric<n, false>(active, geo + (active ? cell : 0) * (6 * n3), p, g);
      kcell = kap;
    }
  }
  // the thread's DoFs i = t + j kBlock: b, D^{-1}, and the first update from x = 0
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int i = t + j * kBlock;
    const bool in = N % kBlock == 0 || i < N;
    bb[j] = in ? b[i] : 0.0;
    di[j] = in ? dinv[i] : 0.0;
    dir[j] = in && dirichlet_dof(i % N1, (i / N1) % N1, i / (N1 * N1), N1, dmask);
    d[j] = di[j] * bb[j] * inv_theta;
    if (in) xs[i] = d[j];
  }
  __syncthreads();
  double rho = delta > 0.0 ? delta / theta : 0.0;   // 1 / sigma_1
  for (int st = 1; st < steps; ++st) {
    const double rho_new = 1.0 / (2.0 * theta / delta - rho);
    const double c1 = rho_new * rho, c2 = 2.0 * rho_new / delta;
    rho = rho_new;
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
      const int i = t + j * kBlock;
      if (N % kBlock == 0 || i < N) ax[i] = 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int pass = 0; pass < NPASS; ++pass) {
      const int cell = pass * CPP + slot;
      const bool active = used && cell < CELLS;
      const int cx = active ? cell % NC : 0, cy = active ? (cell / NC) % NC : 0, cz = active ? cell / (NC * NC) : 0;
      const CellCtx cc = make_ctx(K, n, p, used, active, cx, cy, cz, N1, dmask);
      double u[n];
#pragma unroll
      for (int l = 0; l < n; ++l) u[l] = (active && !z_bnd(cc, l)) ? xs[cc.base + cc.plane * l] : 0.0;
      if constexpr (GEOM == 0) {
        const double scale = active ? kappa[cell] * h : 0.0;
        cart_cell<K, double, 0, 0, false>(cc, u, scale, A, B, A, B, eo);
      } else {
        curved_cell<K, double, 0, 0, false>(cc, u, g, kcell, A, B, C, eo);
      }
      // y_e of the lane's x-line (y = i0, z = i1) is in A after the cell's last barrier (both
      // cell forms leave it in the layout z n^2 + y n + x)
      if (active) {
        const int g0 = (cz * K + cc.i1) * N1 * N1 + (cy * K + cc.i0) * N1 + cx * K;
#pragma unroll
        for (int q = 0; q < n; ++q) lds_add(ax + g0 + q, A[cc.i1 * n2 + cc.i0 * n + q]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
      const int i = t + j * kBlock;
      if (N % kBlock == 0 || i < N) {
        const double axv = dir[j] ? xs[i] : ax[i];
        d[j] = c1 * d[j] + c2 * di[j] * (bb[j] - axv);
        xs[i] += d[j];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int i = t + j * kBlock;
    if (N % kBlock == 0 || i < N) {
      x_out[i] = xs[i];
      if (x64) x64[i] = xs[i];
    }
  }
}

// GEOM of a context: 0 Cartesian, 1 curved with the stored metric, 2 curved with the metric
// formed on the fly.
inline int coarse_geom(const Context &c) {
  if (c.p.geometry != MFL_GEOM_CURVED) return 0;
  return metric_on_the_fly(c.p) ? 2 : 1;
}

template <int K, int NC, int GEOM>
static hipError_t coarse_cheb_launch_g(const Context &c, const Level &L, const double *b, double *x,
                                       double *x64_out, int steps, double theta, double delta, hipStream_t s) {
  if constexpr (CoarseShape<K, NC, GEOM>::fits) {
    const double *geo = GEOM == 2 ? L.disp64 : (GEOM == 1 ? L.metric64 : nullptr);
    coarse_cheb_kernel<K, NC, GEOM><<<1, kBlock, 0, s>>>(b, L.dinv64, L.kappa64, geo, x, x64_out, L.h,
                                                         dirichlet_mask(c.p), steps, theta, delta);
    return hipGetLastError();
  }
  return hipErrorNotSupported;
}

template <int K, int NC>
static hipError_t coarse_cheb_launch(const Context &c, const Level &L, const double *b, double *x,
                                     double *x64_out, int steps, double theta, double delta, hipStream_t s) {
  switch (coarse_geom(c)) {
    case 0: return coarse_cheb_launch_g<K, NC, 0>(c, L, b, x, x64_out, steps, theta, delta, s);
    case 1: return coarse_cheb_launch_g<K, NC, 1>(c, L, b, x, x64_out, steps, theta, delta, s);
    default: return coarse_cheb_launch_g<K, NC, 2>(c, L, b, x, x64_out, steps, theta, delta, s);
  }
}

template <int K, int GEOM>
static bool coarse_cheb_fits_g(int Nc) {
  return (Nc == 1 && CoarseShape<K, 1, GEOM>::fits) || (Nc == 2 && CoarseShape<K, 2, GEOM>::fits) ||
         (Nc == 3 && CoarseShape<K, 3, GEOM>::fits);
}

template <int K>
static bool coarse_cheb_fits(int Nc, int geom) {
  return geom == 0 ? coarse_cheb_fits_g<K, 0>(Nc) : (geom == 1 ? coarse_cheb_fits_g<K, 1>(Nc) : coarse_cheb_fits_g<K, 2>(Nc));
}

bool cg_coarse_cheb_supported(const Context &c, const Level &L) {
  if (c.p.disc != MFL_DISC_CG || L.mg_f32) return false;
  const int geom = coarse_geom(c);
  switch (c.k) {
    case 1: return coarse_cheb_fits<1>(L.Nc, geom);
    case 2: return coarse_cheb_fits<2>(L.Nc, geom);
    case 3: return coarse_cheb_fits<3>(L.Nc, geom);
    case 4: return coarse_cheb_fits<4>(L.Nc, geom);
    case 5: return coarse_cheb_fits<5>(L.Nc, geom);
    case 6: return coarse_cheb_fits<6>(L.Nc, geom);
    case 7: return coarse_cheb_fits<7>(L.Nc, geom);
    case 8: return coarse_cheb_fits<8>(L.Nc, geom);
    default: return false;
  }
}

hipError_t launch_cg_coarse_cheb(const Context &c, const Level &L, const double *b, double *x, double *x64_out,
                                 int steps, double theta, double delta, hipStream_t s) {
  if (!cg_coarse_cheb_supported(c, L) || steps < 1) return hipErrorInvalidValue;
#define CASE(K)                                                                         \
  switch (L.Nc) {                                                                       \
    case 1: return coarse_cheb_launch<K, 1>(c, L, b, x, x64_out, steps, theta, delta, s); \
    case 2: return coarse_cheb_launch<K, 2>(c, L, b, x, x64_out, steps, theta, delta, s); \
    default: return coarse_cheb_launch<K, 3>(c, L, b, x, x64_out, steps, theta, delta, s); \
  }
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipErrorInvalidValue;
}

hipError_t launch_cg_cheb_halo(const Context &c, const Level &L, const void *b, const void *ax,
                               const void *dinv, void *d, void *x, double *x64_out, int dtype, double c1,
                               double c2, hipStream_t s) {
  if (dtype == MFL_F64) {
#define CASE(K) return cg_cheb_halo_k<K, double>(c, L, (const double *)b, (const double *)ax, (const double *)dinv, (double *)d, (double *)x, x64_out, c1, c2, s)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  } else {
#define CASE(K) return cg_cheb_halo_k<K, float>(c, L, (const float *)b, (const float *)ax, (const float *)dinv, (float *)d, (float *)x, x64_out, c1, c2, s)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_cg_apply(const Context &c, const Level &L, int dtype, const void *src, void *dst,
                           hipStream_t s, int dmask, const LaunchEvents *ev) {
  if (dtype == MFL_F64) {
#define CASE(K) return cg_apply_k<K, double>(c, L, c.tab64, L.kappa64, metric_on_the_fly(c.p) ? L.disp64 : L.metric64, (const double *)src, (double *)dst, (double *)L.halo, s, dmask, ev)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  } else {
#define CASE(K) return cg_apply_k<K, float>(c, L, c.tab32, L.kappa32, metric_on_the_fly(c.p) ? L.disp32 : L.metric32, (const float *)src, (float *)dst, (float *)L.halo, s, dmask, ev)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_cg_halo_add(const Context &c, const Level &L, int dtype, void *dst, hipStream_t s,
                              int dmask) {
  if (dtype == MFL_F64) {
#define CASE(K) return cg_halo_k<K, double>(c, L, (double *)dst, (const double *)L.halo, s, dmask)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  } else {
#define CASE(K) return cg_halo_k<K, float>(c, L, (float *)dst, (const float *)L.halo, s, dmask)
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
  const int dir = dirichlet_mask(c.p);
  if (c.p.geometry == MFL_GEOM_CURVED && metric_on_the_fly(c.p))
    kappa_grad_kernel<K, double, true, true><<<grid, kBlock, 0, s>>>(u, lam, grad, L.disp64, L.Nc, L.N1, L.h, dir);
  else if (c.p.geometry == MFL_GEOM_CURVED)
    kappa_grad_kernel<K, double, true><<<grid, kBlock, 0, s>>>(u, lam, grad, L.metric64, L.Nc, L.N1, L.h, dir);
  else
    kappa_grad_kernel<K, double, false><<<grid, kBlock, 0, s>>>(u, lam, grad, nullptr, L.Nc, L.N1, L.h, dir);
  return hipGetLastError();
}

hipError_t launch_cg_kappa_grad(const Context &c, const Level &L, const double *u, const double *lam,
                                double *grad, hipStream_t s) {
#define CASE(K) return kappa_grad_k<K>(c, L, u, lam, grad, s)
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipErrorInvalidValue;
}

}  // namespace mfl
