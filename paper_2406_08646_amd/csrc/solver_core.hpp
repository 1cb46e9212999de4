// Device building blocks shared by the single-system and batched solvers:
// work shares, cross-workgroup partial sums and the row walk used by the
// SpMV-shaped kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"
#include "device.hpp"
#include "spmv_core.hpp"

namespace spx {
namespace solver {

constexpr int kBlock = 256;
// LDS of a solver kernel's reductions: a wave sum and a result for each of
// up to three sums at once.
constexpr int kLds = 3 * (kBlock / 64) + 3;

struct Range {
  int64_t lo, hi;
};

__device__ __forceinline__ Range block_range(int64_t total, int64_t b, int64_t nb) {
  const int64_t per = (total + nb - 1) / nb;
  int64_t lo = b * per;
  if (lo > total) lo = total;
  int64_t hi = lo + per;
  if (hi > total) hi = total;
  return {lo, hi};
}

// Sums of N arrays of nparts partials each (parts[k][0 .. nparts)); every
// workgroup gets the same values (fixed strided split, fixed tree: each
// thread adds its partials in index order, each wave its threads, thread 0
// the waves in order).  A thread loads its partials of all N arrays in
// groups of kReduceGroup before the first add (a partial past the end
// loads partial 0 and is not added), at one round trip per group: one load
// and add at a time paid a round trip per partial, at the start of every
// kernel that reads the previous one's partials.  The N sums share three
// barriers.  lds: kLds doubles.
constexpr int kReduceGroup = 8;
constexpr int kReduceMax = 3;
template <int N>
__device__ __forceinline__ void reduce_all_n(const double* const (&parts)[N], int64_t nparts,
                                             double* lds, double (&out)[N]) {
  static_assert(N >= 1 && N <= kReduceMax, "lds holds kReduceMax sums");
  constexpr int W = kBlock / 64;
  double s[N];
#pragma unroll
  for (int k = 0; k < N; ++k) s[k] = 0.0;
  if (nparts <= kBlock) {  // one partial per thread at most: no groups
    if (threadIdx.x < nparts) {
#pragma unroll
      for (int k = 0; k < N; ++k) s[k] += parts[k][threadIdx.x];
    }
  } else {
    for (int64_t i0 = threadIdx.x; i0 < nparts; i0 += (int64_t)kReduceGroup * kBlock) {
      double v[N][kReduceGroup];
#pragma unroll
      for (int k = 0; k < N; ++k)
#pragma unroll
        for (int u = 0; u < kReduceGroup; ++u) {
          const int64_t i = i0 + (int64_t)u * kBlock;
          v[k][u] = parts[k][i < nparts ? i : 0];
        }
#pragma unroll
      for (int k = 0; k < N; ++k)
#pragma unroll
        for (int u = 0; u < kReduceGroup; ++u)
          if (i0 + (int64_t)u * kBlock < nparts) s[k] += v[k][u];
    }
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    s[k] = wave_sum(s[k]);
    if (lane == 0) lds[k * W + w] = s[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double r = 0.0;
#pragma unroll
      for (int i = 0; i < W; ++i) r += lds[k * W + i];
      lds[N * W + k] = r;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) out[k] = lds[N * W + k];
  __syncthreads();
}

__device__ __forceinline__ double reduce_all(const double* parts, int64_t nparts, double* lds) {
  const double* const pp[1] = {parts};
  double out[1];
  reduce_all_n<1>(pp, nparts, lds, out);
  return out[0];
}

// Two or three sums at once (see reduce_all_n).
__device__ __forceinline__ void reduce_all(const double* pa, const double* pb, int64_t nparts,
                                           double* lds, double& a, double& b) {
  const double* const pp[2] = {pa, pb};
  double out[2];
  reduce_all_n<2>(pp, nparts, lds, out);
  a = out[0];
  b = out[1];
}
__device__ __forceinline__ void reduce_all(const double* pa, const double* pb, const double* pc,
                                           int64_t nparts, double* lds, double& a, double& b,
                                           double& c) {
  const double* const pp[3] = {pa, pb, pc};
  double out[3];
  reduce_all_n<3>(pp, nparts, lds, out);
  a = out[0];
  b = out[1];
  c = out[2];
}

// PIPE: 0 for the plain stream walk, else the per-thread register depth U
// of the pipelined walk (a tile then holds at most kBlock * U entries).
template <int V, int L, bool NT, bool VEC = false, int PIPE = 0>
struct Shape {
  static constexpr int variant = V;
  static constexpr int lanes = L;
  static constexpr bool nt = NT;
  static constexpr bool vec = VEC;
  static constexpr int pipe = PIPE;
};

// Loads one tile's values and columns (cnt <= kBlock * U entries from t0)
// and this thread's row bounds into registers.
template <int U, typename VT, bool NT>
__device__ __forceinline__ void pipe_load(const int32_t* __restrict__ rowptr,
                                          const int32_t* __restrict__ col,
                                          const VT* __restrict__ val, int64_t r0, int64_t r1,
                                          int32_t t0, int32_t cnt, VT (&a)[U], int32_t (&c)[U],
                                          int32_t& rs, int32_t& re) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int32_t i = u * kBlock + threadIdx.x;
    if (i < cnt) {
      a[u] = mload<NT>(val + t0 + i);
      c[u] = mload<NT>(col + t0 + i);
    }
  }
  if (threadIdx.x < r1 - r0) {
    rs = rowptr[r0 + threadIdx.x];
    re = rowptr[r0 + threadIdx.x + 1];
  }
}

// The stream walk over a share of tiles with the next tile's loads issued
// before the current tile's gathers and row sums, so each workgroup keeps
// its matrix loads in flight across tiles.  Requires every tile to hold at
// most kBlock * U entries.  Same results as the plain stream walk.
template <int U, typename VT, typename XT, typename ACC, bool NT, typename Epi>
__device__ __forceinline__ void stream_tiles_pipelined(int64_t n, const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ col,
                                                       const VT* __restrict__ val,
                                                       const XT* __restrict__ x, int rows,
                                                       int64_t first, int64_t end, int64_t step,
                                                       ACC* prod, Epi&& epi) {
  if (first >= end) return;
  int64_t rb = first;
  int64_t r0 = rb * rows;
  int64_t r1 = r0 + rows < n ? r0 + rows : n;
  int32_t t0 = rowptr[r0];
  int32_t cnt = rowptr[r1] - t0;
  VT a[U];
  int32_t c[U];
  int32_t rs = 0, re = 0;
  pipe_load<U, VT, NT>(rowptr, col, val, r0, r1, t0, cnt, a, c, rs, re);
  for (;;) {
    const int64_t nrb = rb + step;
    const bool more = nrb < end;
    int64_t nr0 = 0, nr1 = 0;
    int32_t nt0 = 0, ncnt = 0;
    VT an[U];
    int32_t cn[U];
    int32_t nrs = 0, nre = 0;
    if (more) {
      nr0 = nrb * rows;
      nr1 = nr0 + rows < n ? nr0 + rows : n;
      nt0 = rowptr[nr0];
      ncnt = rowptr[nr1] - nt0;
      pipe_load<U, VT, NT>(rowptr, col, val, nr0, nr1, nt0, ncnt, an, cn, nrs, nre);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t i = u * kBlock + threadIdx.x;
      if (i < cnt) prod[i] = (ACC)a[u] * (ACC)x[c[u]];
    }
    __syncthreads();
    ACC sum = ACC(0);
    const bool owner = threadIdx.x < r1 - r0;
    if (owner)
      for (int32_t i = rs - t0; i < re - t0; ++i) sum += prod[i];
    __syncthreads();
    if (owner) epi(r0 + threadIdx.x, sum);
    if (!more) break;
    rb = nrb;
    r0 = nr0;
    r1 = nr1;
    t0 = nt0;
    cnt = ncnt;
    rs = nrs;
    re = nre;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a[u] = an[u];
      c[u] = cn[u];
    }
  }
}

// Share of `total` work items of logical workgroup lb out of nb: the items
// are cut into 8 contiguous regions, one per XCD (the workgroups of XCD x
// are the x-th contiguous group of logical numbers), and each region is
// dealt out grid-stride to its group.  The XCD then sweeps its region as
// one narrow band, so the x entries the band gathers stay in its L2.
struct Share {
  int64_t first, end, step;
};

__device__ __forceinline__ Share xcd_share(int64_t total, int64_t lb, int64_t nb) {
  if (nb < 8) return {lb, total, nb};
  const int64_t q = nb >> 3, rem = nb & 7;
  const int64_t x = lb < (q + 1) * rem ? lb / (q + 1) : rem + (lb - (q + 1) * rem) / q;
  const int64_t j = lb - (x * q + (x < rem ? x : rem));
  const int64_t size = q + (x < rem ? 1 : 0);
  const int64_t lo = total * x / 8, hi = total * (x + 1) / 8;
  return {lo + j, hi, size};
}

// Calls epi(row, value) on the thread that owns each row of this
// workgroup's share, value = sum_t val[t] x[col[t]] over the row.
// The DMA walk over a share of tiles, double-buffered: while a tile's rows
// are being added, the next tile's direct loads are already in flight.
// `lds` holds two staging buffers for tiles of up to `tile` entries.
template <typename VT, typename XT, typename ACC, typename Epi>
__device__ __forceinline__ void dma_tiles(int64_t n, const int32_t* __restrict__ rowptr,
                                          const int32_t* __restrict__ col,
                                          const VT* __restrict__ val, const XT* __restrict__ x,
                                          int rows, int64_t tile, int64_t first, int64_t end,
                                          int64_t step, char* lds, Epi&& epi) {
  if (first >= end) return;
  const int64_t capc = (tile + 8 + 3) & ~int64_t(3);
  const size_t buf = (dma_buffer_bytes(tile, sizeof(VT)) + 15) & ~size_t(15);
  int32_t* lc[2] = {reinterpret_cast<int32_t*>(lds), reinterpret_cast<int32_t*>(lds + buf)};
  VT* lv[2] = {reinterpret_cast<VT*>(lds + 4 * capc), reinterpret_cast<VT*>(lds + buf + 4 * capc)};
  int64_t rb = first;
  int64_t r0 = rb * rows;
  int64_t r1 = r0 + rows < n ? r0 + rows : n;
  int32_t t0 = rowptr[r0], t1 = rowptr[r1];
  dma_issue<kBlock, VT>(col, val, t0, t1, lc[0], lv[0]);
  int cur = 0;
  for (;;) {
    const bool owner = threadIdx.x < r1 - r0;
    int32_t rs = 0, re = 0;
    if (owner) {
      rs = rowptr[r0 + threadIdx.x];
      re = rowptr[r0 + threadIdx.x + 1];
    }
    dma_products<kBlock, VT, XT, ACC>(x, t0, t1, lc[cur], lv[cur]);
    const int64_t nrb = rb + step;
    const bool more = nrb < end;
    int64_t nr0 = 0, nr1 = 0;
    int32_t nt0 = 0, nt1 = 0;
    if (more) {
      nr0 = nrb * rows;
      nr1 = nr0 + rows < n ? nr0 + rows : n;
      nt0 = rowptr[nr0];
      nt1 = rowptr[nr1];
      dma_issue<kBlock, VT>(col, val, nt0, nt1, lc[cur ^ 1], lv[cur ^ 1]);
    }
    if (owner) epi(r0 + threadIdx.x, dma_row_sum<VT, ACC>(lv[cur], t0, rs, re));
    if (!more) break;
    rb = nrb;
    r0 = nr0;
    r1 = nr1;
    t0 = nt0;
    t1 = nt1;
    cur ^= 1;
  }
}

template <class SH, typename VT, typename XT, typename ACC, typename Epi>
__device__ __forceinline__ void for_rows(int64_t n, const int32_t* __restrict__ rowptr,
                                         const int32_t* __restrict__ col,
                                         const VT* __restrict__ val, const XT* __restrict__ x,
                                         int rows, int64_t lb, int64_t nb, ACC* prod, Epi&& epi,
                                         int64_t tile = 0, const WinView& win = WinView{}) {
  if constexpr (SH::variant == kVariantWindow) {
    static_assert(kBlock == kWinRows, "one thread per row of a window tile");
    static_assert(sizeof(VT) == sizeof(ACC) && sizeof(XT) == sizeof(ACC),
                  "the window walk's LDS is sized for one element type");
    const Share sh = xcd_share(ceil_div(n, kWinRows), lb, nb);
    for (int64_t rb = sh.first; rb < sh.end; rb += sh.step) {
      const int64_t r0 = rb * kWinRows;
      const int64_t r1 = r0 + kWinRows < n ? r0 + kWinRows : n;
      const ACC s = window_rows<win_u_solver<VT>(), win_v<VT>(), kBlock, VT, XT, ACC, SH::nt>(
          rowptr, col, val, x, n, win, rb, r0, r1, prod);
      if (threadIdx.x < r1 - r0) epi(r0 + threadIdx.x, s);
    }
  } else if constexpr (SH::variant == kVariantDma) {
    const Share sh = xcd_share(ceil_div(n, rows), lb, nb);
    dma_tiles<VT, XT, ACC>(n, rowptr, col, val, x, rows, tile, sh.first, sh.end, sh.step,
                           reinterpret_cast<char*>(prod), epi);
  } else if constexpr (SH::variant == kVariantStream && SH::pipe) {
    const Share sh = xcd_share(ceil_div(n, rows), lb, nb);
    stream_tiles_pipelined<SH::pipe, VT, XT, ACC, SH::nt>(n, rowptr, col, val, x, rows, sh.first,
                                                          sh.end, sh.step, prod, epi);
  } else if constexpr (SH::variant == kVariantStream) {
    const Share sh = xcd_share(ceil_div(n, rows), lb, nb);
    for (int64_t rb = sh.first; rb < sh.end; rb += sh.step) {
      const int64_t r0 = rb * rows;
      const int64_t r1 = r0 + rows < n ? r0 + rows : n;
      ACC s;
      if constexpr (SH::vec)
        s = stream_rows_v4<kBlock, 2, VT, XT, ACC, SH::nt>(rowptr, col, val, x, r0, r1, prod);
      else
        s = stream_rows<kBlock, 8, VT, XT, ACC, SH::nt>(rowptr, col, val, x, r0, r1, prod);
      if (threadIdx.x < r1 - r0) epi(r0 + threadIdx.x, s);
    }
  } else {
    constexpr int L = SH::lanes;
    constexpr int RPB = kBlock / L;
    const Share sh = xcd_share(ceil_div(n, RPB), lb, nb);
    const int lane = threadIdx.x % L;
    for (int64_t g = sh.first; g < sh.end; g += sh.step) {
      const int64_t row = g * RPB + threadIdx.x / L;
      if (row < n) {
        const ACC s = group_sum<L>(row_partial<L, VT, XT, ACC, SH::nt>(rowptr, col, val, x, row, lane));
        if (lane == 0) epi(row, s);
      }
    }
  }
}

__device__ __forceinline__ int64_t logical_block(int remap) {
  return remap ? xcd_logical_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
}


// Calls f with the compile-time Shape of sh.  Only callers whose kernels
// receive the window index (WIN) may be handed the window walk.
template <bool WIN = false, typename F>
inline int with_shape(const SpmvShape& sh, F&& f) {
  if (sh.variant == kVariantWindow) {
    if constexpr (WIN)
      return sh.nt ? f(Shape<kVariantWindow, 1, true>()) : f(Shape<kVariantWindow, 1, false>());
    else
      return set_error(SPX_INVALID_ARG, "this kernel has no window walk");
  }
  if (sh.variant == kVariantDma) return f(Shape<kVariantDma, 1, false>());
  if (sh.variant == kVariantStream) {
    if (sh.pipe == 8)
      return sh.nt ? f(Shape<kVariantStream, 1, true, false, 8>())
                   : f(Shape<kVariantStream, 1, false, false, 8>());
    if (sh.pipe == 16)
      return sh.nt ? f(Shape<kVariantStream, 1, true, false, 16>())
                   : f(Shape<kVariantStream, 1, false, false, 16>());
    if (sh.vec)
      return sh.nt ? f(Shape<kVariantStream, 1, true, true>())
                   : f(Shape<kVariantStream, 1, false, true>());
    return sh.nt ? f(Shape<kVariantStream, 1, true>()) : f(Shape<kVariantStream, 1, false>());
  }
  switch (sh.lanes) {
#define SPX_LANES_CASE(LL) \
  case LL:                 \
    return sh.nt ? f(Shape<kVariantVector, LL, true>()) : f(Shape<kVariantVector, LL, false>());
    SPX_LANES_CASE(1)
    SPX_LANES_CASE(2)
    SPX_LANES_CASE(4)
    SPX_LANES_CASE(8)
    SPX_LANES_CASE(16)
    SPX_LANES_CASE(32)
    SPX_LANES_CASE(64)
#undef SPX_LANES_CASE
    default:
      return set_error(SPX_INVALID_ARG, "unsupported lane count %d", sh.lanes);
  }
}


}  // namespace solver
}  // namespace spx
