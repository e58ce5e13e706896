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
#include "ct_tables.h"
#include "device_common.h"

namespace mfl {

namespace {

constexpr int kBlock = 256;

// t = scale * A1-part of one line: cell term K_g u / h plus the two faces of the cell along
// this direction (face 0 at xi = 0 with outward normal -1, face 1 at xi = 1 with +1).
// uL / uR: the neighbour cells' lines (used when hasL / hasR); without a neighbour the face
// is a boundary face: Dirichlet mirror u+ = -u-, grad u+ = grad u- (jump 2u-, average
// derivative = own derivative), or homogeneous Neumann (no contribution).
template <int N, typename T>
__device__ __forceinline__ void sipg_line(const ct::DGTab<N, T> &tb, const T *u, const T *uL, bool hasL,
                                          const T *uR, bool hasR, T inv_h, T sigma, int dmask,
                                          T scale, T *out) {
  T t[N];
  eo_apply<N, 1>(tb.Kg, u, t);
#pragma unroll
  for (int i = 0; i < N; ++i) t[i] *= inv_h;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const T sign = s ? T(1) : T(-1);
    const bool has = s ? hasR : hasL;
    const T *un = s ? uR : uL;
    // own end-point value and derivative at xi = s; neighbour's at xi = 1 - s
    T vm = 0, dm = 0, vp = 0, dp = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const T fvo = s ? tb.fv0[N - 1 - i] : tb.fv0[i];
      const T fdo = s ? -tb.fd0[N - 1 - i] : tb.fd0[i];
      const T fvn = s ? tb.fv0[i] : tb.fv0[N - 1 - i];
      const T fdn = s ? tb.fd0[i] : -tb.fd0[N - 1 - i];
      vm += fvo * u[i];
      dm += fdo * u[i];
      vp += fvn * un[i];
      dp += fdn * un[i];
    }
    T jump, avg;
    if (has) {
      jump = vm - vp;
      avg = T(0.5) * sign * (dm + dp) * inv_h;
    } else if ((dmask >> s) & 1) {
      jump = T(2) * vm;
      avg = sign * dm * inv_h;
    } else {
      jump = 0;
      avg = 0;
    }
    // test by value: -{n.grad u} + sigma [u];  test by normal derivative: -[u]/2
    const T cv = -avg + sigma * jump;
    const T cg = T(-0.5) * jump * sign * inv_h;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const T fvo = s ? tb.fv0[N - 1 - i] : tb.fv0[i];
      const T fdo = s ? -tb.fd0[N - 1 - i] : tb.fd0[i];
      t[i] += cv * fvo + cg * fdo;
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) out[i] = scale * t[i];
}

template <int K, typename T>
__global__ void __launch_bounds__(kBlock)
sipg_kernel(const T *__restrict__ src, T *__restrict__ dst, int Nc, T h, T sigma, int dmask) {
  constexpr int n = K + 1, n2 = n * n, n3 = n2 * n, CPB = kBlock / n2;
  constexpr const ct::DGTab<n, T> &tb = ct::DGTables<n, T>::tab;
  __shared__ T U[CPB * n3], R[CPB * n3];
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
  const T inv_h = T(1) / h;
  const T scale = h * h * tb.w[i0] * tb.w[i1];   // tangential weights of every phase
  const int slot = inblk ? lc : 0;
  T *Uc = U + slot * n3, *Rc = R + slot * n3;
  const T *uc = src + cell * n3;
  const int64_t plane = int64_t(Nc) * Nc;

  // phase z: lanes own z-lines (x = i0, y = i1)
  if (inblk) {
    T u[n], ul[n], ur[n], out[n];
    const bool hasL = cz > 0, hasR = cz < Nc - 1;
    const T *pl = src + (hasL ? cell - plane : cell) * n3, *pr = src + (hasR ? cell + plane : cell) * n3;
#pragma unroll
    for (int l = 0; l < n; ++l) {
      u[l] = active ? uc[l * n2 + p] : T(0);
      ul[l] = (active && hasL) ? pl[l * n2 + p] : T(0);
      ur[l] = (active && hasR) ? pr[l * n2 + p] : T(0);
    }
    sipg_line<n, T>(tb, u, ul, hasL, ur, hasR, inv_h, sigma, dmask, scale, out);
#pragma unroll
    for (int l = 0; l < n; ++l) {
      Uc[l * n2 + p] = u[l];
      Rc[l * n2 + p] = out[l];
    }
  }
  __syncthreads();
  // phase y: lanes own y-lines (x = i0, z = i1)
  if (inblk) {
    T u[n], ul[n], ur[n], out[n];
    const bool hasL = cy > 0, hasR = cy < Nc - 1;
    const T *pl = src + (hasL ? cell - Nc : cell) * n3, *pr = src + (hasR ? cell + Nc : cell) * n3;
#pragma unroll
    for (int b = 0; b < n; ++b) {
      const int o = i1 * n2 + b * n + i0;
      u[b] = Uc[o];
      ul[b] = (active && hasL) ? pl[o] : T(0);
      ur[b] = (active && hasR) ? pr[o] : T(0);
    }
    sipg_line<n, T>(tb, u, ul, hasL, ur, hasR, inv_h, sigma, dmask, scale, out);
#pragma unroll
    for (int b = 0; b < n; ++b) Rc[i1 * n2 + b * n + i0] += out[b];
  }
  __syncthreads();
  // phase x: lanes own x-lines (y = i0, z = i1); the sum of the three directions is stored
  if (inblk) {
    T u[n], ul[n], ur[n], out[n];
    const bool hasL = cx > 0, hasR = cx < Nc - 1;
    const T *pl = src + (hasL ? cell - 1 : cell) * n3, *pr = src + (hasR ? cell + 1 : cell) * n3;
#pragma unroll
    for (int a = 0; a < n; ++a) {
      const int o = i1 * n2 + i0 * n + a;
      u[a] = Uc[o];
      ul[a] = (active && hasL) ? pl[o] : T(0);
      ur[a] = (active && hasR) ? pr[o] : T(0);
    }
    sipg_line<n, T>(tb, u, ul, hasL, ur, hasR, inv_h, sigma, dmask, scale, out);
    if (active) {
      T *d = dst + cell * n3 + i1 * n2 + i0 * n;
#pragma unroll
      for (int a = 0; a < n; ++a) d[a] = Rc[i1 * n2 + i0 * n + a] + out[a];
    }
  }
}

template <int K, typename T>
hipError_t sipg_k(const Context &c, const Level &L, const T *src, T *dst, hipStream_t s) {
  constexpr int CPB = kBlock / ((K + 1) * (K + 1));
  const int grid = int((L.ncells + CPB - 1) / CPB);
  const double sigma = c.p.penalty_factor * (K + 1) * (K + 1) / L.h;
  sipg_kernel<K, T><<<grid, kBlock, 0, s>>>(src, dst, L.Nc, T(L.h), T(sigma),
                                           dirichlet_mask(c.p));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sipg_apply(const Context &c, const Level &L, int dtype, const void *src, void *dst,
                             hipStream_t s) {
  if (dtype == MFL_F64) {
#define CASE(K) return sipg_k<K, double>(c, L, (const double *)src, (double *)dst, s)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  } else {
#define CASE(K) return sipg_k<K, float>(c, L, (const float *)src, (float *)dst, s)
    MFL_DISPATCH_K(c.k, CASE)
#undef CASE
  }
  return hipErrorInvalidValue;
}

}  // namespace mfl
