// The per-row inner loop shared by the product and solver kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"

namespace spx {

// Partial dot product of one CSR row handled by lane `lane` of an aligned
// L-lane group: lane l takes entries t0 + l, t0 + l + L, ...  The caller
// finishes with group_sum<L>.  VT: stored value type, XT: vector type, ACC:
// accumulator type.
template <int L, typename VT, typename XT, typename ACC>
__device__ __forceinline__ ACC row_partial(const int32_t* __restrict__ rowptr,
                                           const int32_t* __restrict__ col,
                                           const VT* __restrict__ val, const XT* __restrict__ x,
                                           int64_t row, int lane) {
  const int32_t t0 = rowptr[row], t1 = rowptr[row + 1];
  ACC acc = ACC(0);
  int32_t t = t0 + lane;
  // two independent loads in flight per lane before the gathers
  for (; t + L < t1; t += 2 * L) {
    const VT a0 = stream_load(val + t);
    const VT a1 = stream_load(val + t + L);
    const int32_t c0 = stream_load(col + t);
    const int32_t c1 = stream_load(col + t + L);
    acc += (ACC)a0 * (ACC)x[c0];
    acc += (ACC)a1 * (ACC)x[c1];
  }
  if (t < t1) acc += (ACC)stream_load(val + t) * (ACC)x[stream_load(col + t)];
  return acc;
}

}  // namespace spx
