// Device helpers shared by the kernels of the library.
#pragma once

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

__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }

__device__ __forceinline__ bool on_boundary(int g, int N1) { return g == 0 || g == N1 - 1; }

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
  }
  return o;
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
