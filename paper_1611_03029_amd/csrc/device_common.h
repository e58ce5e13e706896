// Device helpers shared by the kernels of the library.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mfl_internal.h"

namespace mfl {

// Workgroups are dispatched round-robin over the 8 XCDs of the chip.  Remapping the
// hardware block index so that each XCD receives one contiguous range of logical
// blocks keeps neighbouring cells (which share DoFs) inside one XCD's L2.
__device__ __forceinline__ int xcd_block(int bid, int nblk) {
  const int q = nblk / 8, r = nblk % 8, x = bid % 8, j = bid / 8;
  return (x < r) ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

// kernel<<<grid, block, 0, s>>>(args...), with the launch timed by ev when ev is given.
template <typename... Params, typename... Args>
inline void launch_timed(void (*kernel)(Params...), int grid, int block, hipStream_t s, const LaunchEvents *ev,
                         Args... args) {
  if (ev)
    hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, ev->start, ev->stop, 0, Params(args)...);
  else
    kernel<<<grid, block, 0, s>>>(Params(args)...);
}

__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }

// Four consecutive vector entries moved with 16-byte accesses (one for FP32, two for FP64).
// With one entry per lane a streaming kernel keeps too few bytes in flight per wavefront to
// cover the HBM latency; four per lane reach the streaming rate.  The pointer plus the
// index must be 16-byte aligned.
template <typename T>
struct alignas(16) Quad {
  T v[4];
};

template <typename T>
__device__ __forceinline__ Quad<T> load_quad(const T *p, int64_t i) {
  return *reinterpret_cast<const Quad<T> *>(p + i);
}

template <typename T>
__device__ __forceinline__ void store_quad(T *p, int64_t i, const Quad<T> &q) {
  *reinterpret_cast<Quad<T> *>(p + i) = q;
}

// Host check for the quad kernels: every non-null pointer 16-byte aligned.
inline bool aligned16() { return true; }
template <typename P, typename... R>
inline bool aligned16(P p, R... rest) {
  return reinterpret_cast<uintptr_t>(p) % 16 == 0 && aligned16(rest...);
}

// LDS atomic add without return (ds_add_f64 / ds_add_f32)
template <typename T>
__device__ __forceinline__ void lds_add(T *p, T v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Division of 31-bit unsigned values by an invariant divisor d >= 1 with one 64-bit multiply
// and a shift (division by invariant integers, Granlund and Montgomery 1994): with
// L = ceil(log2 d) and m = ceil(2^(32+L) / d), q = floor(n m / 2^(32+L)) is exact for n < 2^31
// because the rounding error of m times n stays below 2^(32+L) / d.
struct FastDiv {
  uint32_t d;
  int shift;   // 32 + L
  uint64_t m;
  FastDiv() = default;
  __host__ explicit FastDiv(uint32_t div) : d(div) {
    int L = 0;
    while ((uint64_t(1) << L) < div) ++L;
    shift = 32 + L;
    m = ((uint64_t(1) << shift) + div - 1) / div;
  }
  __device__ __forceinline__ uint32_t div(uint32_t n) const { return uint32_t((uint64_t(n) * m) >> shift); }
};

__device__ __forceinline__ bool on_boundary(int g, int N1) { return g == 0 || g == N1 - 1; }

// Grid index g (0..N1-1) along one direction lies on a face with Dirichlet conditions:
// dmask bit 0 marks the lower faces (g = 0), bit 1 the upper faces (g = N1 - 1).
__device__ __forceinline__ bool on_dirichlet(int g, int N1, int dmask) {
  return ((dmask & 1) && g == 0) || ((dmask & 2) && g == N1 - 1);
}

__device__ __forceinline__ bool dirichlet_dof(int x, int y, int z, int N1, int dmask) {
  return on_dirichlet(x, N1, dmask) || on_dirichlet(y, N1, dmask) || on_dirichlet(z, N1, dmask);
}

// Synchronization point among the lanes of one wavefront for data exchanged through LDS.
// A wavefront's LDS instructions execute in issue order, so only the compiler has to be
// kept from moving LDS accesses across this point; no instruction is emitted.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Barrier between the phases of a cell computation: a wavefront barrier when every cell
// lies inside one wavefront (WAVE), a work-group barrier otherwise.
template <bool WAVE>
__device__ __forceinline__ void cell_sync() {
  if constexpr (WAVE)
    wave_sync();
  else
    __syncthreads();
}

// Lane -> (cell slot, lane within the cell) of a work-group.  WAVE: every cell's N2 lanes
// lie inside one wavefront (64 / N2 cells per wavefront); otherwise cells are packed densely
// over the work-group and may straddle wavefronts.
template <int N2, bool WAVE>
struct LaneMap {
  int slot, p;
  bool used;   // lane belongs to a cell slot below `slots`
  __device__ __forceinline__ LaneMap(int t, int slots) {
    if constexpr (WAVE) {
      constexpr int CPW = 64 / N2;
      const int w = t / 64, ln = t % 64, s = ln / N2;
      slot = w * CPW + s;
      p = ln - s * N2;
      used = s < CPW && slot < slots;
    } else {
      slot = t / N2;
      p = t - slot * N2;
      used = slot < slots;
    }
  }
};

// Copy of the first N*N entries of the kMaxN-sized host tables (rows of length N).
template <int N, typename T>
Tab<N, T> shrink_tab(const Tab<kMaxN, T> &t) {
  Tab<N, T> o{};
  for (int i = 0; i < N * N; ++i) {
    o.S[i] = t.S[i];
    o.Sd[i] = t.Sd[i];
    o.D[i] = t.D[i];
    o.M[i] = t.M[i];
    o.K[i] = t.K[i];
  }
  for (int i = 0; i < 2 * N; ++i) {
    o.Fv[i] = t.Fv[i];
    o.Fd[i] = t.Fd[i];
  }
  for (int i = 0; i < N; ++i) {
    o.w[i] = t.w[i];
    o.gll[i] = t.gll[i];
    o.xg[i] = t.xg[i];
  }
  return o;
}

template <int N, typename T>
EOTab<N, T> make_eotab(const Tab<kMaxN, T> &t) {
  // the dense tables have rows of length N; rebuild them in double for the even-odd split
  double M[N * N], K[N * N], S[N * N], D[N * N];
  for (int i = 0; i < N * N; ++i) {
    M[i] = double(t.M[i]);
    K[i] = double(t.K[i]);
    S[i] = double(t.S[i]);
    D[i] = double(t.D[i]);
  }
  EOTab<N, T> e;
  e.M = make_eo<N, T>(M);
  e.K = make_eo<N, T>(K);
  e.S = make_eo<N, T>(S);
  e.D = make_eo<N, T>(D);
  return e;
}

// out = A u with A in even-odd form; SG = +1 (centro-symmetric) or -1 (antisymmetric).
// N^2/2 + O(N) multiply-adds instead of N^2.
template <int N, int SG, typename T>
__host__ __device__ __forceinline__ void eo_apply(const EO<N, T> &a, const T *u, T *out) {
  constexpr int H = N / 2;
  constexpr bool ODD = N & 1;
  T e[H], o[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    e[i] = u[i] + u[N - 1 - i];
    o[i] = u[i] - u[N - 1 - i];
  }
#pragma unroll
  for (int q = 0; q < H; ++q) {
    T ev = ODD ? a.ec[q] * u[H] : T(0), od = 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      ev += a.ep[q * H + i] * e[i];
      od += a.op[q * H + i] * o[i];
    }
    out[q] = ev + od;
    out[N - 1 - q] = SG > 0 ? ev - od : od - ev;
  }
  if constexpr (ODD) {
    T m = SG > 0 ? a.mid[H] * u[H] : T(0);   // the middle entry vanishes if antisymmetric
#pragma unroll
    for (int i = 0; i < H; ++i) m += a.mid[i] * (SG > 0 ? e[i] : o[i]);
    out[H] = m;
  }
}

// out = A^T u with the same even-odd coefficients.
template <int N, int SG, typename T>
__host__ __device__ __forceinline__ void eo_apply_t(const EO<N, T> &a, const T *u, T *out) {
  constexpr int H = N / 2;
  constexpr bool ODD = N & 1;
  T e[H], o[H];
#pragma unroll
  for (int q = 0; q < H; ++q) {
    e[q] = SG > 0 ? u[q] + u[N - 1 - q] : u[q] - u[N - 1 - q];
    o[q] = SG > 0 ? u[q] - u[N - 1 - q] : u[q] + u[N - 1 - q];
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    T ev = 0, od = 0;
#pragma unroll
    for (int q = 0; q < H; ++q) {
      ev += a.ep[q * H + i] * e[q];
      od += a.op[q * H + i] * o[q];
    }
    const T mc = ODD ? a.mid[i] * u[H] : T(0);
    out[i] = ev + od + mc;
    out[N - 1 - i] = SG > 0 ? ev - od + mc : ev - od - mc;
  }
  if constexpr (ODD) {
    T m = SG > 0 ? a.mid[H] * u[H] : T(0);
#pragma unroll
    for (int q = 0; q < H; ++q) m += a.ec[q] * e[q];
    out[H] = m;
  }
}

// Sum over a block of `nthreads` (<= 1024) threads, deterministic order; result valid in
// thread 0.  `scratch` holds blockDim.x values.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *scratch) {
  const int t = threadIdx.x;
  scratch[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) scratch[t] += scratch[t + s];
    __syncthreads();
  }
  return scratch[0];
}

#define MFL_DISPATCH_K(k, MACRO) \
  switch (k) {                   \
    case 1: MACRO(1); break;     \
    case 2: MACRO(2); break;     \
    case 3: MACRO(3); break;     \
    case 4: MACRO(4); break;     \
    case 5: MACRO(5); break;     \
    case 6: MACRO(6); break;     \
    case 7: MACRO(7); break;     \
    case 8: MACRO(8); break;     \
    default: return hipErrorInvalidValue; \
  }

}  // namespace mfl
