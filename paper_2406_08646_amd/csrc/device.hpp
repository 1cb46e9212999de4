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

// Called by every thread after thread 0 has stored this block's partial
// results.  Returns true in the one block that arrives last; that block
// then sees every other block's partials.  The ticket is reset for reuse.
__device__ __forceinline__ bool arrive_last(uint32_t* ticket) {
  __shared__ int last;
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t t =
        __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = (t == gridDim.x - 1);
    if (last) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  const bool is_last = last != 0;
  if (is_last) __threadfence();
  return is_last;
}

// Deterministic sum of nparts values by one block (fixed strided split,
// fixed tree), result valid in thread 0.
template <int BLOCK>
__device__ __forceinline__ double reduce_partials(const double* parts, int64_t nparts, double* lds) {
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += BLOCK) s += parts[i];
  return block_sum<BLOCK>(s, lds);
}

// Loads that bypass the L2 allocation policy for streamed matrix data.
template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
  return __builtin_nontemporal_load(p);
}

}  // namespace spx
