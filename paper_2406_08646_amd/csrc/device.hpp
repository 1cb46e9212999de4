// Device-side building blocks: wave/block reductions, XCD-aware block
// order and the deterministic "last workgroup finishes the reduction"
// pattern used by the fused solver kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spx {

// Sum over the 64 lanes of a wave; every lane receives the total.  The
// butterfly order is fixed, so the result is reproducible.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over aligned groups of L lanes (L a power of two <= 64); every lane of
// the group receives the group total.
template <int L, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = L / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, L);
  return v;
}

// Block-wide sum for blockDim.x == BLOCK; the result is valid in thread 0.
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v, double* lds) {
  static_assert(BLOCK % 64 == 0, "block must be whole waves");
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < BLOCK / 64; ++i) r += lds[i];
  }
  __syncthreads();
  return r;
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b lands on
// XCD b % 8).  Renumber them so every XCD walks one contiguous range of
// logical blocks, which keeps neighbouring rows (and the x entries they
// share) in one L2.  Bijective for any block count.
__device__ __forceinline__ int64_t xcd_logical_block(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, r = nb & 7;
  const int64_t x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// Loads that bypass the L2 allocation policy for streamed matrix data.
template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
  return __builtin_nontemporal_load(p);
}

}  // namespace spx
