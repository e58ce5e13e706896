// Symmetric interior penalty DG Laplacian on Cartesian cells (Sec. 2.2, eq. poisson_dgsip,
// boundary values of eq. bc_dgsip), kappa = 1, penalty sigma = c (k+1)^2 / h.
//
// With the Lagrange basis in the k+1 Gauss points the 1D DG mass is diagonal (h w) and the
// face quadrature points coincide with the tangential basis nodes, so on a Cartesian mesh
// the operator is the Kronecker sum of one 1D SIPG operator A1 per direction,
//   A = sum_d (h w) (x) (h w) (x) A1  (tangential weights times A1 along direction d),
// where A1 on a line of cells has the cell block K_g / h and, per face, the terms
// -{u'}[v] - {v'}[u] + sigma [u][v] built from the end-point values and derivatives.
// Each face therefore needs only the neighbouring cell's line along the face normal.
//
// Element-centric kernel: n^2 lanes per cell, one line per lane; phase z (lanes own
// z-lines), phase y, phase x (transposes through LDS); each phase reads the neighbour
// cells' lines across its two faces from global memory (mostly L2 hits: neighbours in x
// are in the same or an adjacent work-group, the XCD remap keeps y/z neighbours on one
// XCD).  Every DoF is written once by its own cell: no atomics.
#include <initializer_list>

#include "ct_tables.h"
#include "device_common.h"
#include "gaussians.h"

namespace mfl {

namespace {

constexpr int kBlock = 256;

// Lane layout of the cell kernels: cells inside one wavefront (phases without work-group
// barriers) where that fills the wavefront (k <= 3: 64, 63 and 64 lanes); denser packing
// over the work-group otherwise (measured faster for k = 4 and 6).
template <int K>
struct DGLanes {
  static constexpr int n2 = (K + 1) * (K + 1);
  static constexpr bool wave = K <= 3;
  static constexpr int cpb = wave ? (kBlock / 64) * (64 / n2) : kBlock / n2;   // cells per block
};

// LDS layout of a cell's n^3 values in the operator kernel: point (x, y, z) at z PS + y n + x
// of the cell's block of CS values.  The padded plane and cell strides spread the lanes of a
// phase over the LDS banks: with the unpadded strides n^2 and n^3 (powers of two for odd k)
// the lanes of the cells of one wavefront that read the same point of their cells hit the
// same bank (measured 11.4 conflict cycles per LDS instruction at k = 3).  Chosen with a
// model of 64 four-byte banks serving 32 lanes per cycle; k = 2, 4, 8 need no padding.
template <int K>
struct DGLds {
  static constexpr int n = K + 1;
  static constexpr int pp = K == 1 ? 2 : K == 3 ? 3 : K == 5 ? 1 : K == 6 ? 3 : K == 7 ? 5 : 0;
  static constexpr int cp = K == 3 ? 4 : K == 5 ? 6 : K == 6 ? 5 : 0;
  static constexpr int PS = n * n + pp, CS = n * PS + cp;
};

// out = scale * A1-part of one line: the cell term K_g u / h plus the two faces of the cell
// along this direction (face 0 at xi = 0 with outward normal -1, face 1 at xi = 1 with +1).
// Per face, with own and neighbour end-point values v-, v+ and derivatives d-, d+:
//   jump = v- - v+,  avg = sign (d- + d+) / (2h),
//   cv = -avg + sigma jump (tests by value),  cg = -sign jump / (2h) (tests by derivative),
//   t_i += cv psi_i(face) + cg psi_i'(face).
// uL / uR: the neighbour cells' lines (used when hasL / hasR); without a neighbour the face
// is a boundary face: Dirichlet mirror u+ = -u-, grad u+ = grad u- (jump 2 v-, average
// derivative = own derivative), or homogeneous Neumann (no contribution).
// The cell term and both faces are evaluated in even-odd form: by the symmetry of the Gauss
// points the own end-point values of the two faces are E +- O of one even and one odd sum
// over u_i +- u_{N-1-i}, and the face updates split the same way, so that they add to the
// even and odd parts of K_g u before those are recombined.
template <int N, typename T>
__device__ __forceinline__ void sipg_line(const ct::DGTab<N, T> &tb, const T *u, const T *uL, bool hasL,
                                          const T *uR, bool hasR, T inv_h, T sigma, int dmask,
                                          T scale, T *out) {
  constexpr int H = N / 2;
  constexpr bool ODD = N & 1;
  T e[H], o[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    e[i] = u[i] + u[N - 1 - i];
    o[i] = u[i] - u[N - 1 - i];
  }
  // own end-point values (vm0, vm1) and derivatives (dm0, dm1) at xi = 0, 1
  T VE = ODD ? tb.fv0[H] * u[H] : T(0), DE = ODD ? tb.fd0[H] * u[H] : T(0), VO = 0, DO = 0;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    VE += tb.fe[i] * e[i];
    VO += tb.fo[i] * o[i];
    DE += tb.de[i] * e[i];
    DO += tb.dd[i] * o[i];
  }
  const T vm0 = VE + VO, vm1 = VE - VO, dm0 = DE + DO, dm1 = DO - DE;
  // neighbour end-point values at the shared faces: the left neighbour's xi = 1, the right
  // neighbour's xi = 0
  T vp0 = 0, dp0 = 0, vp1 = 0, dp1 = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    vp0 += tb.fv0[N - 1 - i] * uL[i];
    dp0 -= tb.fd0[N - 1 - i] * uL[i];
    vp1 += tb.fv0[i] * uR[i];
    dp1 += tb.fd0[i] * uR[i];
  }
  const T hh = T(0.5) * inv_h;
  T j0, a0, j1, a1;   // jumps and average normal derivatives (sign included)
  if (hasL) {
    j0 = vm0 - vp0;
    a0 = -hh * (dm0 + dp0);
  } else if (dmask & 1) {
    j0 = T(2) * vm0;
    a0 = -inv_h * dm0;
  } else {
    j0 = 0;
    a0 = 0;
  }
  if (hasR) {
    j1 = vm1 - vp1;
    a1 = hh * (dm1 + dp1);
  } else if (dmask & 2) {
    j1 = T(2) * vm1;
    a1 = inv_h * dm1;
  } else {
    j1 = 0;
    a1 = 0;
  }
  const T cv0 = sigma * j0 - a0, cv1 = sigma * j1 - a1;
  const T cg0 = hh * j0, cg1 = -hh * j1;
  // scaled even / odd coefficients of the face updates
  const T pe = scale * (cv0 + cv1), qe = scale * (cg0 - cg1);
  const T po = scale * (cv0 - cv1), qo = scale * (cg0 + cg1);
  const T sk = scale * inv_h;
#pragma unroll
  for (int q = 0; q < H; ++q) {
    T ev = ODD ? tb.Kg.ec[q] * u[H] : T(0), od = 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      ev += tb.Kg.ep[q * H + i] * e[i];
      od += tb.Kg.op[q * H + i] * o[i];
    }
    const T EV = sk * ev + pe * tb.fe[q] + qe * tb.de[q];
    const T OD = sk * od + po * tb.fo[q] + qo * tb.dd[q];
    out[q] = EV + OD;
    out[N - 1 - q] = EV - OD;
  }
  if constexpr (ODD) {
    T m = tb.Kg.mid[H] * u[H];
#pragma unroll
    for (int i = 0; i < H; ++i) m += tb.Kg.mid[i] * e[i];
    out[H] = sk * m + pe * tb.fv0[H] + qe * tb.fd0[H];
  }
}

// Cell order of the SIPG kernel.  A cell reads its neighbours' lines across all six faces;
// in plain x-fastest order the z neighbours are a whole plane of cells apart (7 MB for Q5 on
// 64^3 cells, more than one XCD's 4 MB L2), so both z neighbours missed L2 and src was
// fetched about three times (measured).  Instead the x-y plane is split into 2 x 4 column
// tiles, one per XCD (work-groups are dispatched round-robin over the 8 XCDs), and each XCD
// walks its column plane by plane, x fastest: the z neighbours are one tile plane apart and
// stay in that XCD's L2.  Only the lines read across tile boundaries come from further out.
struct ColumnOrder {
  static constexpr int SX = 2, SY = 4;   // tiles per direction, SX * SY = number of XCDs
  static int blocks_per_xcd(int Nc, int cpb) {
    const int tx = (Nc + SX - 1) / SX, ty = (Nc + SY - 1) / SY;
    return (tx * ty * Nc + cpb - 1) / cpb;
  }
  // cell coordinates of position t of the XCD's traversal; false past its last cell
  __device__ static bool cell(int xcd, int t, int Nc, int &cx, int &cy, int &cz) {
    const int ix = xcd % SX, iy = xcd / SX;
    const int x0 = ix * Nc / SX, x1 = (ix + 1) * Nc / SX, y0 = iy * Nc / SY, y1 = (iy + 1) * Nc / SY;
    const int tx = x1 - x0, area = tx * (y1 - y0);
    if (t >= area * Nc) return false;   // also for an empty tile (area 0)
    cz = t / area;
    const int r = t - cz * area;
    cy = y0 + r / tx;
    cx = x0 + r - (r / tx) * tx;
    return true;
  }
  // the x range [x0, x1) of the XCD's tile: consecutive positions of the traversal are
  // x-neighbours unless a row of the tile ends between them
  __device__ static void xrange(int xcd, int Nc, int &x0, int &x1) {
    const int ix = xcd % SX;
    x0 = ix * Nc / SX;
    x1 = (ix + 1) * Nc / SX;
  }
};

// Whether the x-neighbour of the cell in slot lc lies in slot lc - 1 (left) or lc + 1
// (right) of the same work-group, so that its values can be read from the work-group's LDS
// copy after the first phase (the phases are separated by work-group barriers).  Used where
// cells straddle wavefronts (not WL): measured 3-6% faster there (k = 4, 5); with
// wavefront-local cells (k <= 3) the neighbour would have to lie in the lane's wavefront,
// and the branches cost more than the loads they save (k = 3 FP32 5% slower).
template <bool WL>
__device__ __forceinline__ void lds_x_neighbours(bool active, int lc, int cpb, int cx, int Nc, bool &lin,
                                                 bool &rin) {
  if constexpr (WL) {
    lin = rin = false;
  } else {
    int x0, x1;
    ColumnOrder::xrange(blockIdx.x % 8, Nc, x0, x1);
    lin = active && lc > 0 && cx > x0;
    rin = active && lc + 1 < cpb && cx + 1 < x1;
  }
}

// A lane's x-line of a DG vector: its n values are contiguous (local lexicographic order,
// x fastest).  For even n every x-line starts at an even element offset, so on 16-byte
// aligned vectors (checked by the launchers) the line moves in 16-byte (FP64, FP32 with
// 4 | n) or 8-byte (other FP32) accesses: n / 2 or n / 4 memory instructions instead of n,
// which halves the address work of the x phase in the texture pipeline.  Measured: the
// fused SIPG smoother step gains 5-13% per DG-SIP solve; the operator kernel alone does not
// change in FP64 and was up to 9% slower in FP32 at k = 3, so it uses them for FP64 only
// (VEC = false keeps one access per value).
template <int N, bool VEC = true, typename T>
__device__ __forceinline__ void load_xline(const T *__restrict__ p, T (&v)[N]) {
  if constexpr (!VEC) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = p[i];
  } else if constexpr (sizeof(T) == 8 && N % 2 == 0) {
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      const double2 w = reinterpret_cast<const double2 *>(p)[i];
      v[2 * i] = w.x;
      v[2 * i + 1] = w.y;
    }
  } else if constexpr (sizeof(T) == 4 && N % 4 == 0) {
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      const float4 w = reinterpret_cast<const float4 *>(p)[i];
      v[4 * i] = w.x;
      v[4 * i + 1] = w.y;
      v[4 * i + 2] = w.z;
      v[4 * i + 3] = w.w;
    }
  } else if constexpr (sizeof(T) == 4 && N % 2 == 0) {
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      const float2 w = reinterpret_cast<const float2 *>(p)[i];
      v[2 * i] = w.x;
      v[2 * i + 1] = w.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = p[i];
  }
}

template <int N, bool VEC = true, typename T>
__device__ __forceinline__ void store_xline(T *__restrict__ p, const T (&v)[N]) {
  if constexpr (!VEC) {
#pragma unroll
    for (int i = 0; i < N; ++i) p[i] = v[i];
  } else if constexpr (sizeof(T) == 8 && N % 2 == 0) {
#pragma unroll
    for (int i = 0; i < N / 2; ++i) reinterpret_cast<double2 *>(p)[i] = make_double2(v[2 * i], v[2 * i + 1]);
  } else if constexpr (sizeof(T) == 4 && N % 4 == 0) {
#pragma unroll
    for (int i = 0; i < N / 4; ++i)
      reinterpret_cast<float4 *>(p)[i] = make_float4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]);
  } else if constexpr (sizeof(T) == 4 && N % 2 == 0) {
#pragma unroll
    for (int i = 0; i < N / 2; ++i) reinterpret_cast<float2 *>(p)[i] = make_float2(v[2 * i], v[2 * i + 1]);
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) p[i] = v[i];
  }
}

// Whether the vectors meet the alignment that load_xline / store_xline assume for degree K.
template <int K>
inline bool xline_aligned(std::initializer_list<const void *> ptrs) {
  if ((K + 1) % 2) return true;
  for (const void *q : ptrs)
    if (reinterpret_cast<uintptr_t>(q) % 16) return false;
  return true;
}

// DOT: also the work-group's partial sum of src . dst over its cells, written to
// partials[blockIdx.x] (the conjugate-gradient product p . A p without a pass of its own; a
// cell's A p is complete inside the kernel).
template <int K, typename T, bool DOT = false>
__global__ void __launch_bounds__(kBlock)
sipg_kernel(const T *__restrict__ src, T *__restrict__ dst, int Nc, T h, T sigma, int dmask,
            double *__restrict__ partials = nullptr) {
  constexpr int n = K + 1, n2 = n * n, n3 = n2 * n, CPB = DGLanes<K>::cpb;
  constexpr int PS = DGLds<K>::PS, CS = DGLds<K>::CS;
  constexpr bool WL = DGLanes<K>::wave;
  constexpr const ct::DGTab<n, T> &tb = ct::DGTables<n, T>::tab;
  __shared__ T U[CPB * CS], R[CPB * CS];
  const LaneMap<n2, WL> lm(threadIdx.x, CPB);
  const int lc = lm.slot, p = lm.p, i0 = p % n, i1 = p / n;
  const bool inblk = lm.used;
  int cx = 0, cy = 0, cz = 0;
  const bool active = inblk && ColumnOrder::cell(blockIdx.x % 8, (blockIdx.x / 8) * CPB + lc, Nc, cx, cy, cz);
  const int64_t cell = active ? cx + int64_t(Nc) * (cy + int64_t(Nc) * cz) : 0;
  const T inv_h = T(1) / h;
  const T scale = h * h * tb.w[i0] * tb.w[i1];   // tangential weights of every phase
  const int slot = inblk ? lc : 0;
  T *Uc = U + slot * CS, *Rc = R + slot * CS;
  const T *uc = src + cell * n3;
  const int64_t plane = int64_t(Nc) * Nc;
  // Loads are unconditional: every pointer below addresses a cell of src (an inactive lane
  // reads cell 0, a missing neighbour the cell itself), and sipg_line ignores the neighbour
  // line of a boundary face.  Guarded loads would become one branch each.

  // phase z: lanes own z-lines (x = i0, y = i1)
  if (inblk) {
    T u[n], ul[n], ur[n], out[n];
    const bool hasL = cz > 0, hasR = cz < Nc - 1;
    const T *pl = src + (hasL ? cell - plane : cell) * n3, *pr = src + (hasR ? cell + plane : cell) * n3;
#pragma unroll
    for (int l = 0; l < n; ++l) {
      u[l] = uc[l * n2 + p];
      ul[l] = pl[l * n2 + p];
      ur[l] = pr[l * n2 + p];
    }
    sipg_line<n, T>(tb, u, ul, hasL, ur, hasR, inv_h, sigma, dmask, scale, out);
#pragma unroll
    for (int l = 0; l < n; ++l) {
      Uc[l * PS + p] = u[l];
      Rc[l * PS + p] = out[l];
    }
  }
  cell_sync<WL>();
  // phase y: lanes own y-lines (x = i0, z = i1)
  if (inblk) {
    T u[n], ul[n], ur[n], out[n];
    const bool hasL = cy > 0, hasR = cy < Nc - 1;
    const T *pl = src + (hasL ? cell - Nc : cell) * n3, *pr = src + (hasR ? cell + Nc : cell) * n3;
#pragma unroll
    for (int b = 0; b < n; ++b) {
      const int o = i1 * n2 + b * n + i0;
      u[b] = Uc[i1 * PS + b * n + i0];
      ul[b] = pl[o];
      ur[b] = pr[o];
    }
    sipg_line<n, T>(tb, u, ul, hasL, ur, hasR, inv_h, sigma, dmask, scale, out);
#pragma unroll
    for (int b = 0; b < n; ++b) Rc[i1 * PS + b * n + i0] += out[b];
  }
  cell_sync<WL>();
  // phase x: lanes own x-lines (y = i0, z = i1); the sum of the three directions is stored
  double pq = 0;   // DOT: the lane's x-line of src . dst
  if (inblk) {
    T u[n], ul[n], ur[n], out[n];
    const bool hasL = cx > 0, hasR = cx < Nc - 1;
    const int o = i1 * n2 + i0 * n, ol = i1 * PS + i0 * n;
    const T *pl = src + (hasL ? cell - 1 : cell) * n3 + o, *pr = src + (hasR ? cell + 1 : cell) * n3 + o;
    constexpr bool VX = sizeof(T) == 8;
    bool lin, rin;
    lds_x_neighbours<WL>(active, lc, CPB, cx, Nc, lin, rin);
    if (lin) {
#pragma unroll
      for (int a = 0; a < n; ++a) ul[a] = U[(slot - 1) * CS + ol + a];
    } else {
      load_xline<n, VX>(pl, ul);
    }
    if (rin) {
#pragma unroll
      for (int a = 0; a < n; ++a) ur[a] = U[(slot + 1) * CS + ol + a];
    } else {
      load_xline<n, VX>(pr, ur);
    }
#pragma unroll
    for (int a = 0; a < n; ++a) u[a] = Uc[ol + a];
    sipg_line<n, T>(tb, u, ul, hasL, ur, hasR, inv_h, sigma, dmask, scale, out);
    if (active) {
#pragma unroll
      for (int a = 0; a < n; ++a) out[a] += Rc[ol + a];
      store_xline<n, VX>(dst + cell * n3 + o, out);
      if constexpr (DOT) {
#pragma unroll
        for (int a = 0; a < n; ++a) pq += double(u[a]) * double(out[a]);
      }
    }
  }
  if constexpr (DOT) {
    __shared__ double red[kBlock];
    pq = block_sum(pq, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = pq;
  }
}

template <int K, typename T>
hipError_t sipg_k(const Context &c, const Level &L, const T *src, T *dst, hipStream_t s, const LaunchEvents *ev) {
  constexpr int CPB = DGLanes<K>::cpb;
  const int grid = 8 * ColumnOrder::blocks_per_xcd(L.Nc, CPB);
  const double sigma = c.p.penalty_factor * (K + 1) * (K + 1) / L.h;
  if (!xline_aligned<K>({src, dst})) return hipErrorInvalidValue;
  launch_timed(sipg_kernel<K, T>, grid, kBlock, s, ev, src, dst, L.Nc, T(L.h), T(sigma), dirichlet_mask(c.p),
               static_cast<double *>(nullptr));
  return hipGetLastError();
}

template <int K>
hipError_t sipg_dot_k(const Context &c, const Level &L, const double *src, double *dst, double *partials, int *n,
                      hipStream_t s) {
  constexpr int CPB = DGLanes<K>::cpb;
  const int grid = 8 * ColumnOrder::blocks_per_xcd(L.Nc, CPB);
  const double sigma = c.p.penalty_factor * (K + 1) * (K + 1) / L.h;
  if (!xline_aligned<K>({src, dst})) return hipErrorInvalidValue;
  sipg_kernel<K, double, true><<<grid, kBlock, 0, s>>>(src, dst, L.Nc, L.h, sigma, dirichlet_mask(c.p), partials);
  *n = grid;
  return hipGetLastError();
}

// Own-cell diagonal of the 1D line operator at index a for a cell at position cpos of Nc
// along the line: K_g[a][a] / h plus, per face, the coefficient of u_a in the face terms of
// sipg_line with the neighbour's line zero (interior face: sigma fv^2 - sign fv fd / h;
// Dirichlet mirror: twice that; Neumann: nothing).
template <int N>
__device__ __forceinline__ double sipg_line_diag(const ct::DGTab<N, double> &tb, int a, int cpos, int Nc,
                                                 double h, double sigma, int dmask) {
  double v = tb.kgd[a] / h;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const bool has = s ? cpos < Nc - 1 : cpos > 0;
    const double fvo = s ? tb.fv0[N - 1 - a] : tb.fv0[a];
    const double fdo = s ? -tb.fd0[N - 1 - a] : tb.fd0[a];
    const double sign = s ? 1.0 : -1.0;
    const double term = sigma * fvo * fvo - sign * fvo * fdo / h;
    if (has)
      v += term;
    else if ((dmask >> s) & 1)
      v += 2.0 * term;
  }
  return v;
}

// diag(A): per DoF the sum over the three directions of the tangential weights h^2 w w times
// the own-cell diagonal of that direction's line operator (the operator is a Kronecker sum).
template <int K>
__global__ void __launch_bounds__(kBlock)
sipg_diag_kernel(double *__restrict__ d, int Nc, double h, double sigma, int dmask) {
  constexpr int n = K + 1, n3 = n * n * n;
  constexpr const ct::DGTab<n, double> &tb = ct::DGTables<n, double>::tab;
  const int64_t total = int64_t(Nc) * Nc * Nc * n3;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < total; i += int64_t(gridDim.x) * kBlock) {
    const int64_t cell = i / n3;
    const int r = int(i - cell * n3), a = r % n, b = (r / n) % n, c = r / (n * n);
    const int cx = int(cell % Nc), cy = int((cell / Nc) % Nc), cz = int(cell / (int64_t(Nc) * Nc));
    d[i] = h * h * (tb.w[b] * tb.w[c] * sipg_line_diag<n>(tb, a, cx, Nc, h, sigma, dmask) +
                    tb.w[a] * tb.w[c] * sipg_line_diag<n>(tb, b, cy, Nc, h, sigma, dmask) +
                    tb.w[a] * tb.w[b] * sipg_line_diag<n>(tb, c, cz, Nc, h, sigma, dmask));
  }
}

// Embedding of the coarse DG space in the fine one, one work-group per coarse cell:
// xf(child) += (E_sz (x) E_sy (x) E_sx) xc(cell) for the 8 children (sx, sy, sz), where
// E_s[f][c] = coarse basis c at the f-th Gauss point of child s.  Fine cells belong to
// exactly one coarse cell, so no atomics.
template <int K, typename TC, typename TF>
__global__ void __launch_bounds__(kBlock)
dg_prolongate_kernel(const TC *__restrict__ xc, TF *__restrict__ xf, int Ncc, TransferTab tt) {
  constexpr int n = K + 1, n2 = n * n, n3 = n2 * n;
  __shared__ double E[2 * n2];
  __shared__ TF u[n3], t1[2 * n3], t2[4 * n3];
  for (int i = threadIdx.x; i < 2 * n2; i += kBlock) E[i] = tt.E[i];
  const int64_t cell = blockIdx.x;
  const int cx = int(cell % Ncc), cy = int((cell / Ncc) % Ncc), cz = int(cell / (int64_t(Ncc) * Ncc));
  const int Nf = 2 * Ncc;
  // fine value i of the children, in the order (sz, sy, sx) of the z phase below
  auto fine_index = [&](int i) {
    const int sz = i / (4 * n3), rest = i - sz * 4 * n3, sy = rest / (2 * n3), rest2 = rest - sy * 2 * n3;
    const int sx = rest2 / n3, r = rest2 - sx * n3;
    const int64_t fc = (2 * cx + sx) + int64_t(Nf) * ((2 * cy + sy) + int64_t(Nf) * (2 * cz + sz));
    return fc * n3 + r;
  };
  // the lane's fine values are loaded first, so that those loads are in flight during the
  // three phases instead of each waiting before its own update
  constexpr int NF = 8 * n3, IF = (NF + kBlock - 1) / kBlock;
  TF xv[IF];
#pragma unroll
  for (int it = 0; it < IF; ++it) xv[it] = xf[fine_index(min(int(threadIdx.x) + it * kBlock, NF - 1))];
  for (int i = threadIdx.x; i < n3; i += kBlock) u[i] = TF(xc[cell * n3 + i]);
  __syncthreads();
  for (int i = threadIdx.x; i < 2 * n3; i += kBlock) {   // x: [sx][c][b][a]
    const int sx = i / n3, r = i - sx * n3, a = r % n, bc = r / n;
    TF v = 0;
    for (int j = 0; j < n; ++j) v += TF(E[(sx * n + a) * n + j]) * u[bc * n + j];
    t1[i] = v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 4 * n3; i += kBlock) {   // y: [sy][sx][c][b][a]
    const int sy = i / (2 * n3), rest = i - sy * 2 * n3, sx = rest / n3, r = rest - sx * n3;
    const int a = r % n, b = (r / n) % n, c = r / n2;
    TF v = 0;
    for (int j = 0; j < n; ++j) v += TF(E[(sy * n + b) * n + j]) * t1[sx * n3 + c * n2 + j * n + a];
    t2[i] = v;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IF; ++it) {   // z: fine cell (sx, sy, sz)
    const int i = int(threadIdx.x) + it * kBlock;
    if (i >= NF) break;
    const int sz = i / (4 * n3), rest = i - sz * 4 * n3, sy = rest / (2 * n3), rest2 = rest - sy * 2 * n3;
    const int sx = rest2 / n3, r = rest2 - sx * n3, a = r % n, b = (r / n) % n, c = r / n2;
    TF v = 0;
    for (int j = 0; j < n; ++j) v += TF(E[(sz * n + c) * n + j]) * t2[(sy * 2 + sx) * n3 + j * n2 + b * n + a];
    xf[fine_index(i)] = xv[it] + v;
  }
}

// coarse = P^T (b_f - A x_f) (axf == nullptr: P^T b_f), one work-group per coarse cell:
// the transposed embedding of the 8 children summed; every coarse value is written once.
template <int K, typename TF, typename TC>
__global__ void __launch_bounds__(kBlock)
dg_restrict_kernel(const TF *__restrict__ bf, const TF *__restrict__ axf, TC *__restrict__ bc, int Ncc,
                   TransferTab tt) {
  constexpr int n = K + 1, n2 = n * n, n3 = n2 * n;
  __shared__ double E[2 * n2];
  __shared__ TF r8[8 * n3], t2[4 * n3], t1[2 * n3];
  for (int i = threadIdx.x; i < 2 * n2; i += kBlock) E[i] = tt.E[i];
  const int64_t cell = blockIdx.x;
  const int cx = int(cell % Ncc), cy = int((cell / Ncc) % Ncc), cz = int(cell / (int64_t(Ncc) * Ncc));
  const int Nf = 2 * Ncc;
  // children in order (sz, sy, sx); all of a lane's loads are issued before the first is used
  constexpr int NR = 8 * n3, IR = (NR + kBlock - 1) / kBlock;
  TF bv[IR], av[IR];
#pragma unroll
  for (int it = 0; it < IR; ++it) {
    const int i = min(int(threadIdx.x) + it * kBlock, NR - 1);
    const int ch = i / n3, r = i - ch * n3, sx = ch & 1, sy = (ch >> 1) & 1, sz = ch >> 2;
    const int64_t fc = (2 * cx + sx) + int64_t(Nf) * ((2 * cy + sy) + int64_t(Nf) * (2 * cz + sz));
    const int64_t g = fc * n3 + r;
    bv[it] = bf[g];
    av[it] = axf ? axf[g] : TF(0);
  }
#pragma unroll
  for (int it = 0; it < IR; ++it) {
    const int i = int(threadIdx.x) + it * kBlock;
    if (i >= NR) break;
    r8[i] = axf ? bv[it] - av[it] : bv[it];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 4 * n3; i += kBlock) {   // z: [sy][sx][c'][b][a]
    const int sy = i / (2 * n3), rest = i - sy * 2 * n3, sx = rest / n3, r = rest - sx * n3;
    const int a = r % n, b = (r / n) % n, c = r / n2;
    TF v = 0;
    for (int sz = 0; sz < 2; ++sz)
      for (int j = 0; j < n; ++j)
        v += TF(E[(sz * n + j) * n + c]) * r8[(sz * 4 + sy * 2 + sx) * n3 + j * n2 + b * n + a];
    t2[i] = v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2 * n3; i += kBlock) {   // y: [sx][c'][b'][a]
    const int sx = i / n3, r = i - sx * n3, a = r % n, b = (r / n) % n, c = r / n2;
    TF v = 0;
    for (int sy = 0; sy < 2; ++sy)
      for (int j = 0; j < n; ++j)
        v += TF(E[(sy * n + j) * n + b]) * t2[(sy * 2 + sx) * n3 + c * n2 + j * n + a];
    t1[i] = v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n3; i += kBlock) {       // x: coarse (a', b', c')
    const int a = i % n, bc2 = i / n;
    TF v = 0;
    for (int sx = 0; sx < 2; ++sx)
      for (int j = 0; j < n; ++j) v += TF(E[(sx * n + j) * n + a]) * t1[sx * n3 + bc2 * n + j];
    bc[cell * n3 + i] = TC(v);
  }
}

// Right-hand side of the three-Gaussian example for SIPG on [lo, lo + Nc h]^3, Gauss-point
// basis: (f, psi_i) with the (k+1)^3 Gauss rule (= w w w h^3 f at the DoF's own point), plus
// on each boundary face of the DoF's cell the data terms of the mirror extension (Sec. 2.2,
// eq. bc_dgsip): Dirichlet int (2 sigma g psi_i - g n . grad psi_i), Neumann
// int (n . grad u) psi_i, face Gauss points = the tangential Gauss points.
template <int K>
__global__ void __launch_bounds__(kBlock)
sipg_rhs_gaussians_kernel(double *__restrict__ b, int Nc, double h, double lo, double sigma, int dmask) {
  constexpr int n = K + 1, n3 = n * n * n;
  constexpr const ct::DGTab<n, double> &tb = ct::DGTables<n, double>::tab;
  const int64_t total = int64_t(Nc) * Nc * Nc * n3;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < total; i += int64_t(gridDim.x) * kBlock) {
    const int64_t cell = i / n3;
    const int r = int(i - cell * n3);
    const int idx[3] = {r % n, (r / n) % n, r / (n * n)};
    const int cc[3] = {int(cell % Nc), int((cell / Nc) % Nc), int(cell / (int64_t(Nc) * Nc))};
    double x[3], u, g[3], lap;
    for (int d = 0; d < 3; ++d) x[d] = lo + (cc[d] + tb.xg[idx[d]]) * h;
    gaussians(x, u, g, lap);
    double v = tb.w[idx[0]] * tb.w[idx[1]] * tb.w[idx[2]] * h * h * h * (-lap);
    for (int d = 0; d < 3; ++d) {
      const int a = idx[d];
      const double W = tb.w[idx[(d + 1) % 3]] * tb.w[idx[(d + 2) % 3]] * h * h;
      for (int s = 0; s < 2; ++s) {
        if (cc[d] != (s ? Nc - 1 : 0)) continue;
        const double fvo = s ? tb.fv0[n - 1 - a] : tb.fv0[a];
        const double fdo = s ? -tb.fd0[n - 1 - a] : tb.fd0[a];
        const double sign = s ? 1.0 : -1.0;
        double xf[3] = {x[0], x[1], x[2]}, uf, gf[3], lf;
        xf[d] = lo + (cc[d] + s) * h;
        gaussians(xf, uf, gf, lf);
        if ((dmask >> s) & 1)
          v += W * (2.0 * sigma * uf * fvo - uf * sign * fdo / h);
        else
          v += W * sign * gf[d] * fvo;
      }
    }
    b[i] = v;
  }
}

// D'^{-1}, D' = diagonal of the SIPG operator in the GLL-Lagrange basis of each cell.  With
// T = S (x) S (x) S the operator there is sum_d (h M) (x) (h M) (x) S^T A1_d S, whose line
// part has the own-cell diagonal K[a][a] / h plus, for the end node a of a face (GLL nodes
// lie on the faces), f (sigma + d0 / h) with f = 1 (interior), 2 (Dirichlet), 0 (Neumann).
template <int K>
__global__ void __launch_bounds__(kBlock)
sipg_gll_jacobi_diag_kernel(double *__restrict__ i64, float *__restrict__ i32, int Nc, double h,
                            double sigma, int dmask) {
  constexpr int n = K + 1, n3 = n * n * n;
  constexpr const ct::GLLDiag<n, double> &g = ct::GLLDiagTables<n, double>::tab;
  const int64_t total = int64_t(Nc) * Nc * Nc * n3;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < total; i += int64_t(gridDim.x) * kBlock) {
    const int64_t cell = i / n3;
    const int r = int(i - cell * n3);
    const int idx[3] = {r % n, (r / n) % n, r / (n * n)};
    const int cc[3] = {int(cell % Nc), int((cell / Nc) % Nc), int(cell / (int64_t(Nc) * Nc))};
    double line[3];
    for (int d = 0; d < 3; ++d) {
      const int a = idx[d];
      double v = g.k[a] / h;
      for (int s = 0; s < 2; ++s) {
        if (a != (s ? K : 0)) continue;
        const bool has = s ? cc[d] < Nc - 1 : cc[d] > 0;
        const double f = has ? 1.0 : (((dmask >> s) & 1) ? 2.0 : 0.0);
        v += f * (sigma + g.d0 / h);
      }
      line[d] = v;
    }
    const double dv = h * h * (g.m[idx[1]] * g.m[idx[2]] * line[0] + g.m[idx[0]] * g.m[idx[2]] * line[1] +
                               g.m[idx[0]] * g.m[idx[1]] * line[2]);
    i64[i] = 1.0 / dv;
    i32[i] = float(1.0 / dv);
  }
}

// Jacobi step of the GLL-Lagrange basis applied to Gauss-basis vectors, per cell
// C w = T (D'^{-1} (T^T w)), fused with the smoother updates:
//   MODE 0 (first Chebyshev update): w = b_in; d = C w * c1; x = d; b_store = b_in if given
//   MODE 1 (Chebyshev update):      w = b - ax; d = c1 d + c2 C w; x += d; x64 = x if given
//   MODE 2 (Jacobi step):           d = C w, w = b_in
// n^2 lanes per cell, one line each; five phases with LDS transposes: S^T along z, y, x;
// D'^{-1}; S along x, y, z.  The lane's z-line of w is read and its z-line of the result
// written, so global accesses of consecutive lanes are contiguous within a cell.
template <int K, typename A, typename T, int MODE>
__global__ void __launch_bounds__(kBlock)
dg_gll_jacobi_kernel(const A *__restrict__ b_in, T *__restrict__ b_store, const T *__restrict__ ax,
                     const T *__restrict__ dpinv, T *__restrict__ d, T *__restrict__ x,
                     double *__restrict__ x64, int64_t ncells, T c1, T c2) {
  constexpr int n = K + 1, n2 = n * n, n3 = n2 * n, CPB = DGLanes<K>::cpb;
  constexpr bool WL = DGLanes<K>::wave;
  constexpr const EOTab<n, T> &eo = ct::Tables<n, T>::eo;
  __shared__ T U[CPB * n3], V[CPB * n3];
  const LaneMap<n2, WL> lm(threadIdx.x, CPB);
  const int lc = lm.slot, p = lm.p, i0 = p % n, i1 = p / n;
  const int64_t cell = int64_t(xcd_block(blockIdx.x, gridDim.x)) * CPB + lc;
  const bool inblk = lm.used;
  const bool active = inblk && cell < ncells;
  const int slot = inblk ? lc : 0;
  T *Uc = U + slot * n3, *Vc = V + slot * n3;
  const int64_t base = (active ? cell : 0) * n3;
  // phase 1: z-lines (x = i0, y = i1): w, S^T along z
  if (inblk) {
    T w[n], r[n];
#pragma unroll
    for (int l = 0; l < n; ++l) {
      const int64_t gi = base + l * n2 + p;
      T v = 0;
      if (active) {
        v = T(b_in[gi]);
        if (MODE == 1) v -= ax[gi];
      }
      w[l] = v;
    }
    // stored after all loads: a load after a store would wait for the store
    if (MODE == 0 && b_store && active) {
#pragma unroll
      for (int l = 0; l < n; ++l) b_store[base + l * n2 + p] = w[l];
    }
    eo_apply_t<n, 1>(eo.S, w, r);
#pragma unroll
    for (int l = 0; l < n; ++l) Uc[l * n2 + p] = r[l];
  }
  cell_sync<WL>();
  // phase 2: y-lines (x = i0, z = i1): S^T along y
  if (inblk) {
    T w[n], r[n];
#pragma unroll
    for (int b = 0; b < n; ++b) w[b] = Uc[i1 * n2 + b * n + i0];
    eo_apply_t<n, 1>(eo.S, w, r);
#pragma unroll
    for (int b = 0; b < n; ++b) Vc[i1 * n2 + b * n + i0] = r[b];
  }
  cell_sync<WL>();
  // phase 3: x-lines (y = i0, z = i1): S^T along x, D'^{-1}, S along x
  if (inblk) {
    T w[n], r[n];
#pragma unroll
    for (int a = 0; a < n; ++a) w[a] = Vc[i1 * n2 + i0 * n + a];
    eo_apply_t<n, 1>(eo.S, w, r);
#pragma unroll
    for (int a = 0; a < n; ++a) r[a] *= active ? dpinv[base + i1 * n2 + i0 * n + a] : T(0);
    eo_apply<n, 1>(eo.S, r, w);
#pragma unroll
    for (int a = 0; a < n; ++a) Uc[i1 * n2 + i0 * n + a] = w[a];
  }
  cell_sync<WL>();
  // phase 4: y-lines: S along y
  if (inblk) {
    T w[n], r[n];
#pragma unroll
    for (int b = 0; b < n; ++b) w[b] = Uc[i1 * n2 + b * n + i0];
    eo_apply<n, 1>(eo.S, w, r);
#pragma unroll
    for (int b = 0; b < n; ++b) Vc[i1 * n2 + b * n + i0] = r[b];
  }
  cell_sync<WL>();
  // phase 5: z-lines: S along z, then the update of the lane's z-line
  if (active) {
    T w[n], cw[n];
#pragma unroll
    for (int l = 0; l < n; ++l) w[l] = Vc[l * n2 + p];
    eo_apply<n, 1>(eo.S, w, cw);
#pragma unroll
    for (int l = 0; l < n; ++l) {
      const int64_t gi = base + l * n2 + p;
      if (MODE == 0) {
        const T v = cw[l] * c1;
        d[gi] = v;
        x[gi] = v;
      } else if (MODE == 1) {
        const T dn = c1 * d[gi] + c2 * cw[l];
        const T xn = x[gi] + dn;
        d[gi] = dn;
        x[gi] = xn;
        if (x64) x64[gi] = double(xn);
      } else {
        d[gi] = cw[l];
      }
    }
  }
}

// One Chebyshev update of the SIPG smoother fused with the operator application:
//   w = b - A x,  d = c1 d + c2 C w,  x_out = x + d  (x64 = x_out when given),
// with the point Jacobi step of the GLL-Lagrange basis C = T D'^{-1} T^T (T = S (x) S (x) S,
// applied here along x, y, z and back, which the Kronecker form allows).  A x of a cell is
// complete after the three phases of sipg_kernel (no halo), so the cell continues with the
// five phases of the Jacobi step without writing A x out: per DoF x, b, D'^{-1} and d are
// read and d and x_out written (the separate kernels also write and read A x).  x_out must
// not alias x: neighbouring cells read x.  Lane layout and cell order of sipg_kernel.
template <int K, typename T>
__global__ void __launch_bounds__(kBlock)
sipg_cheb_kernel(const T *__restrict__ src, const T *__restrict__ b, const T *__restrict__ dpinv,
                 T *__restrict__ d, T *__restrict__ x_out, double *__restrict__ x64, int Nc, T h, T sigma,
                 int dmask, T c1, T c2) {
  constexpr int n = K + 1, n2 = n * n, n3 = n2 * n, CPB = DGLanes<K>::cpb;
  constexpr bool WL = DGLanes<K>::wave;
  constexpr const ct::DGTab<n, T> &tb = ct::DGTables<n, T>::tab;
  constexpr const EOTab<n, T> &eo = ct::Tables<n, T>::eo;
  __shared__ T U[CPB * n3], R[CPB * n3];
  const LaneMap<n2, WL> lm(threadIdx.x, CPB);
  const int lc = lm.slot, p = lm.p, i0 = p % n, i1 = p / n;
  const bool inblk = lm.used;
  int cx = 0, cy = 0, cz = 0;
  const bool active = inblk && ColumnOrder::cell(blockIdx.x % 8, (blockIdx.x / 8) * CPB + lc, Nc, cx, cy, cz);
  const int64_t cell = active ? cx + int64_t(Nc) * (cy + int64_t(Nc) * cz) : 0;
  const T inv_h = T(1) / h;
  const T scale = h * h * tb.w[i0] * tb.w[i1];
  const int slot = inblk ? lc : 0;
  T *Uc = U + slot * n3, *Rc = R + slot * n3;
  const T *uc = src + cell * n3;
  const int64_t plane = int64_t(Nc) * Nc;
  const int64_t xl0 = cell * n3 + i1 * n2 + i0 * n;   // the lane's x-line (y = i0, z = i1)
  // Loads are unconditional (see sipg_kernel).
  T v[n];   // the cell's values on the lane's x-line, kept for the final update
  // In FP32 the lane's own lines of b, D'^{-1} and d, read in the later phases, are loaded
  // first, so that those loads are in flight during the operator phases (15 more VGPRs, the
  // same 8 waves per SIMD at k = 4; in FP64 the registers would cost occupancy).
  constexpr bool PRE = sizeof(T) == 4;
  T bq[n], dpq[n], dq[n];
  if constexpr (PRE) {
    load_xline<n>(b + xl0, bq);
#pragma unroll
    for (int l = 0; l < n; ++l) dpq[l] = dpinv[cell * n3 + l * n2 + p];
    load_xline<n>(d + xl0, dq);
  }

  // operator, phase z
  if (inblk) {
    T u[n], ul[n], ur[n], out[n];
    const bool hasL = cz > 0, hasR = cz < Nc - 1;
    const T *pl = src + (hasL ? cell - plane : cell) * n3, *pr = src + (hasR ? cell + plane : cell) * n3;
#pragma unroll
    for (int l = 0; l < n; ++l) {
      u[l] = uc[l * n2 + p];
      ul[l] = pl[l * n2 + p];
      ur[l] = pr[l * n2 + p];
    }
    sipg_line<n, T>(tb, u, ul, hasL, ur, hasR, inv_h, sigma, dmask, scale, out);
#pragma unroll
    for (int l = 0; l < n; ++l) {
      Uc[l * n2 + p] = u[l];
      Rc[l * n2 + p] = out[l];
    }
  }
  cell_sync<WL>();
  // operator, phase y
  if (inblk) {
    T u[n], ul[n], ur[n], out[n];
    const bool hasL = cy > 0, hasR = cy < Nc - 1;
    const T *pl = src + (hasL ? cell - Nc : cell) * n3, *pr = src + (hasR ? cell + Nc : cell) * n3;
#pragma unroll
    for (int j = 0; j < n; ++j) {
      const int o = i1 * n2 + j * n + i0;
      u[j] = Uc[o];
      ul[j] = pl[o];
      ur[j] = pr[o];
    }
    sipg_line<n, T>(tb, u, ul, hasL, ur, hasR, inv_h, sigma, dmask, scale, out);
#pragma unroll
    for (int j = 0; j < n; ++j) Rc[i1 * n2 + j * n + i0] += out[j];
  }
  cell_sync<WL>();
  // operator, phase x, then w = b - A x and S^T along x
  if (inblk) {
    T ul[n], ur[n], out[n], w[n], r[n];
    const bool hasL = cx > 0, hasR = cx < Nc - 1;
    const int o = i1 * n2 + i0 * n;
    const T *pl = src + (hasL ? cell - 1 : cell) * n3 + o, *pr = src + (hasR ? cell + 1 : cell) * n3 + o;
    bool lin, rin;
    lds_x_neighbours<WL>(active, lc, CPB, cx, Nc, lin, rin);
    if (lin) {
#pragma unroll
      for (int a = 0; a < n; ++a) ul[a] = U[(slot - 1) * n3 + o + a];
    } else {
      load_xline<n>(pl, ul);
    }
    if (rin) {
#pragma unroll
      for (int a = 0; a < n; ++a) ur[a] = U[(slot + 1) * n3 + o + a];
    } else {
      load_xline<n>(pr, ur);
    }
    if constexpr (PRE) {
#pragma unroll
      for (int a = 0; a < n; ++a) w[a] = bq[a];
    } else {
      load_xline<n>(b + xl0, w);
    }
#pragma unroll
    for (int a = 0; a < n; ++a) v[a] = Uc[o + a];
    sipg_line<n, T>(tb, v, ul, hasL, ur, hasR, inv_h, sigma, dmask, scale, out);
#pragma unroll
    for (int a = 0; a < n; ++a) w[a] -= Rc[i1 * n2 + i0 * n + a] + out[a];
    eo_apply_t<n, 1>(eo.S, w, r);
    // into R (the lane's own x-line, read above): U keeps the cell's values for the
    // x-neighbours that read them in this phase
#pragma unroll
    for (int a = 0; a < n; ++a) Rc[i1 * n2 + i0 * n + a] = r[a];
  }
  cell_sync<WL>();
  // S^T along y
  if (inblk) {
    T w[n], r[n];
#pragma unroll
    for (int j = 0; j < n; ++j) w[j] = Rc[i1 * n2 + j * n + i0];
    eo_apply_t<n, 1>(eo.S, w, r);
#pragma unroll
    for (int j = 0; j < n; ++j) Uc[i1 * n2 + j * n + i0] = r[j];
  }
  cell_sync<WL>();
  // S^T along z, D'^{-1}, S along z
  if (inblk) {
    T w[n], r[n], dp[n];
#pragma unroll
    for (int l = 0; l < n; ++l) {
      w[l] = Uc[l * n2 + p];
      dp[l] = PRE ? dpq[l] : dpinv[cell * n3 + l * n2 + p];
    }
    eo_apply_t<n, 1>(eo.S, w, r);
#pragma unroll
    for (int l = 0; l < n; ++l) r[l] *= dp[l];
    eo_apply<n, 1>(eo.S, r, w);
#pragma unroll
    for (int l = 0; l < n; ++l) Rc[l * n2 + p] = w[l];
  }
  cell_sync<WL>();
  // S along y
  if (inblk) {
    T w[n], r[n];
#pragma unroll
    for (int j = 0; j < n; ++j) w[j] = Rc[i1 * n2 + j * n + i0];
    eo_apply<n, 1>(eo.S, w, r);
#pragma unroll
    for (int j = 0; j < n; ++j) Uc[i1 * n2 + j * n + i0] = r[j];
  }
  cell_sync<WL>();
  // S along x and the update of the lane's x-line (d is read in full before any store: a
  // load after a store of the same array would wait for that store)
  if (active) {
    T w[n], cw[n], dn[n], xn[n];
#pragma unroll
    for (int a = 0; a < n; ++a) w[a] = Uc[i1 * n2 + i0 * n + a];
    if constexpr (PRE) {
#pragma unroll
      for (int a = 0; a < n; ++a) dn[a] = dq[a];
    } else {
      load_xline<n>(d + xl0, dn);
    }
    eo_apply<n, 1>(eo.S, w, cw);
#pragma unroll
    for (int a = 0; a < n; ++a) {
      dn[a] = c1 * dn[a] + c2 * cw[a];
      xn[a] = v[a] + dn[a];
    }
    store_xline<n>(d + xl0, dn);
    store_xline<n>(x_out + xl0, xn);
    if (x64) {
#pragma unroll
      for (int a = 0; a < n; ++a) x64[xl0 + a] = double(xn[a]);
    }
  }
}

inline int grid_for(int64_t items, int cap = 16384) {
  int64_t g = (items + kBlock - 1) / kBlock;
  return int(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_sipg_apply(const Context &c, const Level &L, int dtype, const void *src, void *dst,
                             hipStream_t s, const LaunchEvents *ev) {
  if (dtype == MFL_F64) {
#define CASE(K) return sipg_k<K, double>(c, L, (const double *)src, (double *)dst, s, ev)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  } else {
#define CASE(K) return sipg_k<K, float>(c, L, (const float *)src, (float *)dst, s, ev)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sipg_apply_dot(const Context &c, const Level &L, const double *src, double *dst,
                                 double *partials, int *n, hipStream_t s) {
#define CASE(K) return sipg_dot_k<K>(c, L, src, dst, partials, n, s)
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipErrorInvalidValue;
}

int sipg_apply_blocks(int k, int Nc) {
#define CASE(K) return 8 * ColumnOrder::blocks_per_xcd(Nc, DGLanes<K>::cpb)
  MFL_DISPATCH_K(k, CASE)
#undef CASE
  return 0;
}

hipError_t launch_sipg_diagonal(const Context &c, const Level &L, hipStream_t s) {
  const double sigma = c.p.penalty_factor * (c.k + 1) * (c.k + 1) / L.h;
  const int dm = dirichlet_mask(c.p);
#define CASE(K) sipg_diag_kernel<K><<<grid_for(L.ndofs), kBlock, 0, s>>>(L.diag64, L.Nc, L.h, sigma, dm); break
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_diag_invert(L, s);
}

template <int K>
static hipError_t dg_prolongate_k(const Context &c, const Level &coarse, const void *xc, int cd, void *xf,
                                  int fd, hipStream_t s) {
  const int grid = int(coarse.ncells);
  if (cd == MFL_F64 && fd == MFL_F64)
    dg_prolongate_kernel<K, double, double><<<grid, kBlock, 0, s>>>((const double *)xc, (double *)xf, coarse.Nc, c.transfer);
  else if (cd == MFL_F64 && fd == MFL_F32)
    dg_prolongate_kernel<K, double, float><<<grid, kBlock, 0, s>>>((const double *)xc, (float *)xf, coarse.Nc, c.transfer);
  else if (cd == MFL_F32 && fd == MFL_F32)
    dg_prolongate_kernel<K, float, float><<<grid, kBlock, 0, s>>>((const float *)xc, (float *)xf, coarse.Nc, c.transfer);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_dg_prolongate_add(const Context &c, const Level &coarse, const void *xc, int cd, void *xf,
                                    int fd, hipStream_t s) {
#define CASE(K) return dg_prolongate_k<K>(c, coarse, xc, cd, xf, fd, s)
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipErrorInvalidValue;
}

template <int K>
static hipError_t dg_restrict_k(const Context &c, const Level &coarse, const void *bf, const void *axf, int fd,
                                void *bc, int cd, hipStream_t s) {
  const int grid = int(coarse.ncells);
  if (fd == MFL_F64 && cd == MFL_F64)
    dg_restrict_kernel<K, double, double><<<grid, kBlock, 0, s>>>((const double *)bf, (const double *)axf, (double *)bc, coarse.Nc, c.transfer);
  else if (fd == MFL_F32 && cd == MFL_F64)
    dg_restrict_kernel<K, float, double><<<grid, kBlock, 0, s>>>((const float *)bf, (const float *)axf, (double *)bc, coarse.Nc, c.transfer);
  else if (fd == MFL_F32 && cd == MFL_F32)
    dg_restrict_kernel<K, float, float><<<grid, kBlock, 0, s>>>((const float *)bf, (const float *)axf, (float *)bc, coarse.Nc, c.transfer);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_dg_restrict(const Context &c, const Level &coarse, const void *bf, const void *axf, int fd,
                              void *bc, int cd, hipStream_t s) {
#define CASE(K) return dg_restrict_k<K>(c, coarse, bf, axf, fd, bc, cd, s)
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipErrorInvalidValue;
}

hipError_t launch_sipg_gll_jacobi_diag(const Context &c, const Level &L, hipStream_t s) {
  const double sigma = c.p.penalty_factor * (c.k + 1) * (c.k + 1) / L.h;
  const int dm = dirichlet_mask(c.p);
#define CASE(K)                                                                                  \
  sipg_gll_jacobi_diag_kernel<K><<<grid_for(L.ndofs), kBlock, 0, s>>>(L.dinv64, L.dinv32, L.Nc, L.h, \
                                                                      sigma, dm);                  \
  break
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipGetLastError();
}

template <int K, typename A, typename T, int MODE>
static hipError_t dg_gll_k(const Level &L, const void *b_in, void *b_store, const void *ax, const void *dpinv,
                           void *d, void *x, double *x64, double c1, double c2, hipStream_t s) {
  constexpr int CPB = DGLanes<K>::cpb;
  const int grid = int((L.ncells + CPB - 1) / CPB);
  dg_gll_jacobi_kernel<K, A, T, MODE><<<grid, kBlock, 0, s>>>(
      (const A *)b_in, (T *)b_store, (const T *)ax, (const T *)dpinv, (T *)d, (T *)x, x64, L.ncells, T(c1), T(c2));
  return hipGetLastError();
}

hipError_t launch_dg_gll_cheb_first(const Context &c, const Level &L, const void *b_in, int in_dtype,
                                    void *b_store, void *d, void *x, int dtype, double inv_theta,
                                    hipStream_t s) {
  if (dtype == MFL_F64) {
    if (in_dtype != MFL_F64) return hipErrorInvalidValue;
#define CASE(K) return dg_gll_k<K, double, double, 0>(L, b_in, b_store, nullptr, L.dinv64, d, x, nullptr, inv_theta, 0.0, s)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  } else if (in_dtype == MFL_F64) {
#define CASE(K) return dg_gll_k<K, double, float, 0>(L, b_in, b_store, nullptr, L.dinv32, d, x, nullptr, inv_theta, 0.0, s)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  } else {
#define CASE(K) return dg_gll_k<K, float, float, 0>(L, b_in, b_store, nullptr, L.dinv32, d, x, nullptr, inv_theta, 0.0, s)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_dg_gll_cheb_step(const Context &c, const Level &L, const void *b, const void *ax, void *d,
                                   void *x, double *x64_out, int dtype, double c1, double c2, hipStream_t s) {
  if (dtype == MFL_F64) {
#define CASE(K) return dg_gll_k<K, double, double, 1>(L, b, nullptr, ax, L.dinv64, d, x, x64_out, c1, c2, s)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  } else {
#define CASE(K) return dg_gll_k<K, float, float, 1>(L, b, nullptr, ax, L.dinv32, d, x, x64_out, c1, c2, s)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  }
  return hipErrorInvalidValue;
}

template <int K, typename T>
static hipError_t sipg_cheb_k(const Context &c, const Level &L, const T *x, const T *b, const T *dpinv, T *d,
                              T *x_out, double *x64, double c1, double c2, hipStream_t s) {
  constexpr int CPB = DGLanes<K>::cpb;
  const int grid = 8 * ColumnOrder::blocks_per_xcd(L.Nc, CPB);
  const double sigma = c.p.penalty_factor * (K + 1) * (K + 1) / L.h;
  if (!xline_aligned<K>({x, b, d, x_out})) return hipErrorInvalidValue;
  sipg_cheb_kernel<K, T><<<grid, kBlock, 0, s>>>(x, b, dpinv, d, x_out, x64, L.Nc, T(L.h), T(sigma),
                                                 dirichlet_mask(c.p), T(c1), T(c2));
  return hipGetLastError();
}

hipError_t launch_sipg_cheb(const Context &c, const Level &L, const void *x, const void *b, void *d, void *x_out,
                            double *x64_out, int dtype, double c1, double c2, hipStream_t s) {
  if (dtype == MFL_F64) {
#define CASE(K) return sipg_cheb_k<K, double>(c, L, (const double *)x, (const double *)b, L.dinv64, (double *)d, (double *)x_out, x64_out, c1, c2, s)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  } else {
#define CASE(K) return sipg_cheb_k<K, float>(c, L, (const float *)x, (const float *)b, L.dinv32, (float *)d, (float *)x_out, x64_out, c1, c2, s)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_dg_gll_jacobi(const Context &c, const Level &L, const double *r, double *z, hipStream_t s) {
#define CASE(K) return dg_gll_k<K, double, double, 2>(L, r, nullptr, nullptr, L.dinv64, z, nullptr, nullptr, 0.0, 0.0, s)
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipErrorInvalidValue;
}

hipError_t launch_sipg_rhs_gaussians(const Context &c, const Level &L, double *b, hipStream_t s) {
  const double sigma = c.p.penalty_factor * (c.k + 1) * (c.k + 1) / L.h;
  const int dm = dirichlet_mask(c.p);
#define CASE(K)                                                                                   \
  sipg_rhs_gaussians_kernel<K><<<grid_for(L.ndofs), kBlock, 0, s>>>(b, L.Nc, L.h, c.p.domain_lo,   \
                                                                    sigma, dm);                    \
  break
  MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  return hipGetLastError();
}

}  // namespace mfl
