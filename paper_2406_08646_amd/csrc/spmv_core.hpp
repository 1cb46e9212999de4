// The per-row inner loops shared by the product and solver kernels.
//
// Two ways to walk a CSR matrix on a 64-wide wavefront:
//  * vector: an aligned group of L lanes owns one row (any row length);
//  * stream: a workgroup owns R consecutive rows; it streams their entire
//    contiguous run of (value, column) pairs with every lane reading
//    consecutive entries (fully coalesced, U independent loads in flight per
//    lane), stages the products a*x[col] in LDS, then one lane per row adds
//    its row's products in order.  Used when rows are short and regular.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"
#include "device.hpp"

namespace spx {

template <bool NT, typename T>
__device__ __forceinline__ T mload(const T* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

// Partial dot product of one CSR row handled by lane `lane` of an aligned
// L-lane group: lane l takes entries t0 + l, t0 + l + L, ...  The caller
// finishes with group_sum<L>.  VT: stored value type, XT: vector type, ACC:
// accumulator type.
template <int L, typename VT, typename XT, typename ACC, bool NT = false>
__device__ __forceinline__ ACC row_partial(const int32_t* __restrict__ rowptr,
                                           const int32_t* __restrict__ col,
                                           const VT* __restrict__ val, const XT* __restrict__ x,
                                           int64_t row, int lane) {
  const int32_t t0 = rowptr[row], t1 = rowptr[row + 1];
  ACC acc = ACC(0);
  int32_t t = t0 + lane;
  // two independent loads in flight per lane before the gathers
  for (; t + L < t1; t += 2 * L) {
    const VT a0 = mload<NT>(val + t);
    const VT a1 = mload<NT>(val + t + L);
    const int32_t c0 = mload<NT>(col + t);
    const int32_t c1 = mload<NT>(col + t + L);
    acc += (ACC)a0 * (ACC)x[c0];
    acc += (ACC)a1 * (ACC)x[c1];
  }
  if (t < t1) acc += (ACC)mload<NT>(val + t) * (ACC)x[mload<NT>(col + t)];
  return acc;
}

// K members of a chunk of the stream walk per thread (member u of thread t
// is entry base + u * BLOCK + t): values and columns, then the gathers of
// x, then the products into prod.  Every load is issued, a member past the
// tile loading the tile's last entry again (unused): a gather left under a
// data-dependent branch waited for every load before it, one round trip
// per member.  K is the number of members the chunk reaches, so whole
// waves past the tile issue nothing.
template <int K, int BLOCK, typename VT, typename XT, typename ACC, bool NT>
__device__ __forceinline__ void stream_chunk(const int32_t* __restrict__ col,
                                             const VT* __restrict__ val,
                                             const XT* __restrict__ x, int32_t t0, int32_t cnt,
                                             int32_t base, ACC* prod) {
  const int tid = threadIdx.x;
  VT a[K];
  int32_t c[K];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int32_t i = base + u * BLOCK + tid, ic = i < cnt ? i : cnt - 1;
    a[u] = mload<NT>(val + t0 + ic);
    c[u] = mload<NT>(col + t0 + ic);
  }
  XT xv[K];
#pragma unroll
  for (int u = 0; u < K; ++u) xv[u] = x[c[u]];
  // all gathers in registers here: one sunk into the branch of its store
  // would wait for the loads before it again
#pragma unroll
  for (int u = 0; u < K; ++u) asm volatile("" : "+v"(xv[u]));
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int32_t i = base + u * BLOCK + tid;
    if (i < cnt) prod[i] = (ACC)a[u] * (ACC)xv[u];
  }
}

// stream_chunk with K = k (1 <= k <= KMAX, the same in every thread).
template <int KMAX, int BLOCK, typename VT, typename XT, typename ACC, bool NT>
__device__ __forceinline__ void stream_chunk_k(int k, const int32_t* __restrict__ col,
                                               const VT* __restrict__ val,
                                               const XT* __restrict__ x, int32_t t0,
                                               int32_t cnt, int32_t base, ACC* prod) {
  if constexpr (KMAX >= 1) {
    if (k == KMAX)
      stream_chunk<KMAX, BLOCK, VT, XT, ACC, NT>(col, val, x, t0, cnt, base, prod);
    else
      stream_chunk_k<KMAX - 1, BLOCK, VT, XT, ACC, NT>(k, col, val, x, t0, cnt, base, prod);
  }
}

// Rows [r0, r1) of one workgroup of BLOCK threads (r1 - r0 <= BLOCK); the
// products of the rows' entries are staged in `prod` (LDS, at least
// rowptr[r1] - rowptr[r0] elements).  Returns, in thread t < r1 - r0, the
// sum of row r0 + t (entries added in order); other threads get 0.
// EAGER: every load of a chunk issued together (stream_chunk).  It makes
// the one-workgroup solvers' iterations faster; the grid kernels (MatMult
// on small patterns, the solvers' persistent SpMV kernels) measured as
// fast or slower with it, so they keep the plain form.
template <int BLOCK, int U, typename VT, typename XT, typename ACC, bool NT = false,
          bool EAGER = false>
__device__ __forceinline__ ACC stream_rows(const int32_t* __restrict__ rowptr,
                                           const int32_t* __restrict__ col,
                                           const VT* __restrict__ val, const XT* __restrict__ x,
                                           int64_t r0, int64_t r1, ACC* prod) {
  const int tid = threadIdx.x;
  const int32_t t0 = rowptr[r0];
  const int32_t cnt = rowptr[r1] - t0;
  if constexpr (EAGER) {
    // this thread's row bounds, loaded with the tile's (held in registers so
    // that their loads are not left until after the barrier), and every
    // chunk's loads issued together (stream_chunk)
    const bool own = tid < r1 - r0;
    const int64_t ri = own ? r0 + tid : r0;
    int32_t ra = rowptr[ri], re = rowptr[ri + 1];
    asm volatile("" : "+v"(ra), "+v"(re));
    for (int32_t base = 0; base < cnt; base += BLOCK * U) {
      const int32_t left = cnt - base;
      stream_chunk_k<U, BLOCK, VT, XT, ACC, NT>(
          left >= BLOCK * U ? U : (int)((left + BLOCK - 1) / BLOCK), col, val, x, t0, cnt, base,
          prod);
    }
    __syncthreads();
    ACC s = ACC(0);
    if (own) {
      for (int32_t i = ra - t0; i < re - t0; ++i) s += prod[i];
    }
    __syncthreads();  // prod is reused by the caller's next tile
    return s;
  } else {
    for (int32_t base = 0; base < cnt; base += BLOCK * U) {
      VT a[U];
      int32_t c[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t i = base + u * BLOCK + tid;
        if (i < cnt) {
          a[u] = mload<NT>(val + t0 + i);
          c[u] = mload<NT>(col + t0 + i);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t i = base + u * BLOCK + tid;
        if (i < cnt) prod[i] = (ACC)a[u] * (ACC)x[c[u]];
      }
    }
    __syncthreads();
    ACC s = ACC(0);
    if (tid < r1 - r0) {
      const int32_t a = rowptr[r0 + tid] - t0, e = rowptr[r0 + tid + 1] - t0;
      for (int32_t i = a; i < e; ++i) s += prod[i];
    }
    __syncthreads();  // prod is reused by the caller's next tile
    return s;
  }
}

// Vector types for 16-byte loads.
typedef double dbl2_t __attribute__((ext_vector_type(2)));
typedef float flt4_t __attribute__((ext_vector_type(4)));
typedef int32_t int4_t __attribute__((ext_vector_type(4)));

// Four consecutive values at a 16-byte aligned address.
template <bool NT>
__device__ __forceinline__ void load4(const double* p, double (&v)[4]) {
  const dbl2_t a = mload<NT>(reinterpret_cast<const dbl2_t*>(p));
  const dbl2_t b = mload<NT>(reinterpret_cast<const dbl2_t*>(p + 2));
  v[0] = a.x;
  v[1] = a.y;
  v[2] = b.x;
  v[3] = b.y;
}
__device__ __forceinline__ void store4(double* p, const double (&v)[4]) {
  dbl2_t a, b;
  a.x = v[0];
  a.y = v[1];
  b.x = v[2];
  b.y = v[3];
  *reinterpret_cast<dbl2_t*>(p) = a;
  *reinterpret_cast<dbl2_t*>(p + 2) = b;
}
__device__ __forceinline__ void store4(float* p, const float (&v)[4]) {
  flt4_t a;
  a.x = v[0];
  a.y = v[1];
  a.z = v[2];
  a.w = v[3];
  *reinterpret_cast<flt4_t*>(p) = a;
}
template <bool NT>
__device__ __forceinline__ void load4(const float* p, float (&v)[4]) {
  const flt4_t a = mload<NT>(reinterpret_cast<const flt4_t*>(p));
  v[0] = a.x;
  v[1] = a.y;
  v[2] = a.z;
  v[3] = a.w;
}

// Same contract as stream_rows, reading the run in aligned quads: every
// lane issues one 16-byte column load and 16 (fp32) or 2 x 16 (fp64) bytes
// of values per quad and stores its four products with 16-byte LDS writes
// at quad-aligned positions (prod[idx - ta], ta = t0 rounded down to 4), so
// neither the global loads nor the LDS writes conflict.  The entries of the
// first and last quad that lie outside [t0, t1) get a zero product without
// touching x.  The value and column arrays carry at least three entries of
// padding so the last quad stays inside the allocation; `prod` needs
// t1 - ta + 3 elements.
template <int BLOCK, int U, typename VT, typename XT, typename ACC, bool NT = false>
__device__ __forceinline__ ACC stream_rows_v4(const int32_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ col,
                                              const VT* __restrict__ val,
                                              const XT* __restrict__ x, int64_t r0, int64_t r1,
                                              ACC* prod) {
  const int tid = threadIdx.x;
  const int32_t t0 = rowptr[r0];
  const int32_t t1 = rowptr[r1];
  const int32_t ta = t0 & ~3;
  const int32_t nq = (t1 - ta + 3) >> 2;
  for (int32_t qb = 0; qb < nq; qb += BLOCK * U) {
    VT a[U][4];
    int4_t c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t q = qb + u * BLOCK + tid;
      if (q < nq) {
        const int32_t e = ta + 4 * q;
        c[u] = mload<NT>(reinterpret_cast<const int4_t*>(col + e));
        load4<NT>(val + e, a[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t q = qb + u * BLOCK + tid;
      if (q < nq) {
        const int32_t e = ta + 4 * q;
        const int32_t cc[4] = {c[u].x, c[u].y, c[u].z, c[u].w};
        ACC pr[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int32_t idx = e + j;
          pr[j] = (idx >= t0 && idx < t1) ? (ACC)a[u][j] * (ACC)x[cc[j]] : ACC(0);
        }
        store4(prod + 4 * q, pr);
      }
    }
  }
  __syncthreads();
  ACC s = ACC(0);
  if (tid < r1 - r0) {
    const int32_t a = rowptr[r0 + tid] - ta, e = rowptr[r0 + tid + 1] - ta;
    for (int32_t i = a; i < e; ++i) s += prod[i];
  }
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------- DMA walk
// gfx950 loads global memory straight into LDS (global_load_lds_dwordx4:
// lane l of a wave writes its 16 bytes at the wave's LDS base + 16 l), so a
// tile's columns and values can be staged without passing through
// registers.  Columns are moved in aligned quads (ca = t0 rounded down to
// 4), values in aligned 16-byte groups (va = t0 rounded down to 16 /
// sizeof(VT)); the few entries outside [t0, t1) that ride along are never
// used.  The value and column arrays carry padding so the last group stays
// inside the allocation.
typedef __attribute__((address_space(3))) void lds_void_t;
typedef const __attribute__((address_space(1))) void glb_void_t;

__device__ __forceinline__ int32_t dma_col_base(int32_t t0) { return t0 & ~3; }
template <typename VT>
__device__ __forceinline__ int32_t dma_val_base(int32_t t0) {
  return t0 & ~(int32_t)(16 / sizeof(VT) - 1);
}

// Issues the direct loads of entries [t0, t1) into lcol / lval.
template <int BLOCK, typename VT>
__device__ __forceinline__ void dma_issue(const int32_t* __restrict__ col,
                                          const VT* __restrict__ val, int32_t t0, int32_t t1,
                                          int32_t* lcol, VT* lval) {
  constexpr int EV = 16 / sizeof(VT);
  const int32_t ca = dma_col_base(t0), nq = (t1 - ca + 3) >> 2;
  const int32_t va = dma_val_base<VT>(t0), nv = (t1 - va + EV - 1) / EV;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  for (int32_t qb = w * 64; qb < nq; qb += BLOCK)
    if (qb + l < nq)
      __builtin_amdgcn_global_load_lds((glb_void_t*)(col + ca + 4 * (qb + l)),
                                       (lds_void_t*)(lcol + 4 * qb), 16, 0, 0);
  for (int32_t vb = w * 64; vb < nv; vb += BLOCK)
    if (vb + l < nv)
      __builtin_amdgcn_global_load_lds((glb_void_t*)(val + va + EV * (vb + l)),
                                       (lds_void_t*)(lval + EV * vb), 16, 0, 0);
}

// Waits for the tile's direct loads, forms the products in place
// (lval[i - va] = val * x[col]), and returns in thread t < r1 - r0 the sum
// of row r0 + t in entry order (rs / re: that row's bounds, loaded by the
// caller).  Leaves the workgroup synchronised.
template <int BLOCK, typename VT, typename XT, typename ACC>
__device__ __forceinline__ void dma_products(const XT* __restrict__ x, int32_t t0, int32_t t1,
                                             const int32_t* lcol, VT* lval) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const int32_t ca = dma_col_base(t0), va = dma_val_base<VT>(t0);
  for (int32_t i = t0 + threadIdx.x; i < t1; i += BLOCK)
    lval[i - va] = (ACC)lval[i - va] * (ACC)x[lcol[i - ca]];
  __syncthreads();
}

template <typename VT, typename ACC>
__device__ __forceinline__ ACC dma_row_sum(const VT* lval, int32_t t0, int32_t rs, int32_t re) {
  const int32_t va = dma_val_base<VT>(t0);
  ACC s = ACC(0);
  for (int32_t i = rs - va; i < re - va; ++i) s += (ACC)lval[i];
  return s;
}

// LDS bytes of one staging buffer for tiles of up to `tile` entries.
__host__ __device__ inline size_t dma_buffer_bytes(int64_t tile, size_t vbytes) {
  const int64_t capc = (tile + 8 + 3) & ~int64_t(3);
  const int64_t capv = tile + 16;
  return 4 * (size_t)capc + vbytes * (size_t)capv;
}

// -------------------------------------------------------------- window walk
// Each thread takes V consecutive entries per step (one vector load of
// values, one of columns) and U = 2 steps per chunk.  fp64: V = 2 (16-byte
// value loads); on the 27-point operator that is 20,480 bytes of LDS, and
// eight workgroups per CU fit exactly once the solver's SpMV kernel keeps
// its workgroup sums in that LDS instead of a static array (with U = 1 and
// 16 KB the kernel took 0.121 ms, with U = 2 0.115).  fp32: V = 4 (16-byte
// value loads), 14 KB.
constexpr int kWinUProduct = 2;
template <typename VT>
__host__ __device__ constexpr int win_v() {
  return sizeof(VT) == 8 ? 2 : 4;
}
template <typename VT>
__host__ __device__ constexpr int win_u_solver() {
  return 2;
}

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};

// V consecutive values or column indices in one load.
template <typename T, int V>
struct VecN {
  typedef T type __attribute__((ext_vector_type(V)));
};

// Copies blocks blk[k0 .. k0 + nbk) of x (n entries; entries at n and
// beyond read as 0) into xs, block i at xs + i * kWinBlock, with 16-byte
// loads when x is 16-byte aligned.  x is read through the caches: each
// block serves several neighbouring tiles.
//
// EAGER: a thread loads all its block numbers, then all its pieces of x,
// then stores them; otherwise it loads and stores one piece at a time.
// Loads left under data-dependent branches each wait for every load before
// them, a round trip per piece, which the eager form avoids: threads past
// the window load its last piece again, and a piece that runs past n loads
// 16 bytes of the block list instead (unused) and is read entry by entry
// once the others are in flight.  One tile per workgroup (MatMult) gains
// from it; the solver's persistent walk measured slower with it, so it
// keeps the plain loop.
template <int BLOCK, typename XT, bool EAGER>
__device__ __forceinline__ void load_window(const XT* __restrict__ x, int64_t n,
                                            const int32_t* __restrict__ blk, int32_t k0,
                                            int32_t nbk, XT* xs) {
  constexpr int PER = 16 / sizeof(XT);
  constexpr int LPB = kWinBlock / PER;
  constexpr int PRE = 4;  // pieces per thread in flight together
  typedef typename Vec16<XT>::type V;
  const int cnt = nbk * LPB;
  if (!EAGER || (reinterpret_cast<uintptr_t>(x) & 15) != 0) {
    const bool aligned = (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    for (int q = threadIdx.x; q < cnt; q += BLOCK) {
      const int i = q / LPB, e = (q % LPB) * PER;
      const int64_t g = (int64_t)blk[k0 + i] * kWinBlock + e;
      XT* d = xs + i * kWinBlock + e;
      if (aligned && g + PER <= n) {
        *reinterpret_cast<V*>(d) = *reinterpret_cast<const V*>(x + g);
      } else {
#pragma unroll
        for (int j = 0; j < PER; ++j) d[j] = g + j < n ? x[g + j] : XT(0);
      }
    }
    return;
  }
  for (int q0 = 0; q0 < cnt; q0 += PRE * BLOCK) {
    int32_t bq[PRE];
#pragma unroll
    for (int u = 0; u < PRE; ++u) {
      const int q = q0 + threadIdx.x + u * BLOCK;
      bq[u] = blk[k0 + (q < cnt ? q : cnt - 1) / LPB];
    }
    V v[PRE];
#pragma unroll
    for (int u = 0; u < PRE; ++u) {
      const int q = q0 + threadIdx.x + u * BLOCK;
      const int64_t g = (int64_t)bq[u] * kWinBlock + ((q < cnt ? q : cnt - 1) % LPB) * PER;
      v[u] = *(g + PER <= n ? reinterpret_cast<const V*>(x + g) : reinterpret_cast<const V*>(blk));
    }
    // all pieces in registers here: a load sunk into the branch of its
    // store would wait for every load before it
#pragma unroll
    for (int u = 0; u < PRE; ++u) asm volatile("" : "+v"(v[u]));
#pragma unroll
    for (int u = 0; u < PRE; ++u) {
      const int q = q0 + threadIdx.x + u * BLOCK;
      if (q < cnt) {
        const int i = q / LPB, e = (q % LPB) * PER;
        const int64_t g = (int64_t)bq[u] * kWinBlock + e;
        XT* d = xs + i * kWinBlock + e;
        if (g + PER <= n) {
          *reinterpret_cast<V*>(d) = v[u];
        } else {
#pragma unroll
          for (int j = 0; j < PER; ++j) d[j] = g + j < n ? x[g + j] : XT(0);
        }
      }
    }
  }
}

// The chunk loop of one tile of the window walk.  WIN: x is read from the
// tile's window (blocks blk[k0 .. k0 + nbk), staged into xs before the
// first barrier while the first chunk's values and indices are in flight)
// through the 16-bit window columns `cidx`; otherwise straight from memory
// through the 32-bit columns.  The entries are walked V at a time from the
// multiple of V at or below the tile's first entry t0; members outside
// [t0, t1) are loaded (the arrays carry tail padding) but never used.
// Thread i owns the row whose entries are [ra, re) relative to that entry ta.
template <bool WIN, bool EAGER, int U, int V, int BLOCK, typename VT, typename XT, typename ACC,
          bool NT, typename CT>
__device__ __forceinline__ ACC window_chunks(const CT* __restrict__ cidx, const VT* __restrict__ val,
                                             const XT* __restrict__ x, int64_t n,
                                             const int32_t* __restrict__ blk, int32_t k0,
                                             int32_t nbk, int32_t t0, int32_t t1, int32_t ra,
                                             int32_t re, ACC* prod) {
  constexpr int32_t C = BLOCK * U * V;
  typedef typename VecN<VT, V>::type VV;
  typedef typename VecN<CT, V>::type CV;
  XT* xs = reinterpret_cast<XT*>(prod + C);
  const int tid = threadIdx.x;
  const int32_t ta = t0 & ~(V - 1);
  const int32_t cnt = t1 - ta, skip = t0 - ta;
  // EAGER: members past the tile load its first group again (unused), so
  // that no load sits under a data-dependent branch
  VV a[U];
  CV c[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int32_t e = (u * BLOCK + tid) * V;
    if constexpr (EAGER) {
      const int32_t ec = e < cnt ? e : 0;
      a[u] = mload<NT>(reinterpret_cast<const VV*>(val + ta + ec));
      c[u] = mload<NT>(reinterpret_cast<const CV*>(cidx + ta + ec));
    } else if (e < cnt) {
      a[u] = mload<NT>(reinterpret_cast<const VV*>(val + ta + e));
      c[u] = mload<NT>(reinterpret_cast<const CV*>(cidx + ta + e));
    }
  }
  if constexpr (WIN) load_window<BLOCK, XT, EAGER>(x, n, blk, k0, nbk, xs);
  __syncthreads();
  ACC s = ACC(0);
  for (int32_t base = 0; base < cnt; base += C) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t e = base + (u * BLOCK + tid) * V;
#pragma unroll
      for (int j = 0; j < V; ++j) {
        if (e + j >= skip && e + j < cnt) {
          const int32_t cj = (int32_t)c[u][j];
          XT xv;
          if constexpr (WIN)
            xv = xs[cj];
          else
            xv = x[cj];
          prod[(u * BLOCK + tid) * V + j] = (ACC)a[u][j] * (ACC)xv;
        }
      }
    }
    const int32_t next = base + C;
    if (next < cnt) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t e = next + (u * BLOCK + tid) * V;
        if constexpr (EAGER) {
          const int32_t ec = e < cnt ? e : next;
          a[u] = mload<NT>(reinterpret_cast<const VV*>(val + ta + ec));
          c[u] = mload<NT>(reinterpret_cast<const CV*>(cidx + ta + ec));
        } else if (e < cnt) {
          a[u] = mload<NT>(reinterpret_cast<const VV*>(val + ta + e));
          c[u] = mload<NT>(reinterpret_cast<const CV*>(cidx + ta + e));
        }
      }
    }
    __syncthreads();
    const int32_t lo = ra > base ? ra : base, hi = re < next ? re : next;
    for (int32_t i = lo; i < hi; ++i) s += prod[i - base];
    __syncthreads();
  }
  return s;
}

// One tile of the window walk: tile number `tile` covers rows [r0, r1)
// (r1 - r0 <= kWinRows == BLOCK) and thread i owns row r0 + i.  The tile's
// entries are taken in chunks of BLOCK * U * V: the chunk's products
// val[t] * x[col[t]] go to prod (x read from the tile's window, staged in
// LDS behind prod, or directly from memory for a tile without a window),
// then every thread adds its own row's products of the chunk in entry
// order, carrying its sum from chunk to chunk.  Each row's sum is thus
// formed in exactly the order of stream_rows, with LDS use independent of
// the tile's length.  The next chunk's values and columns are loaded before
// the current chunk's sums.  LDS: BLOCK * U * V ACC products, then the
// largest window's x entries.  Returns the row sum in its owner thread and
// leaves the workgroup synchronised.
template <int U, int V, int BLOCK, typename VT, typename XT, typename ACC, bool NT,
          bool EAGER = false>
__device__ __forceinline__ ACC window_rows(const int32_t* __restrict__ rowptr,
                                           const int32_t* __restrict__ col,
                                           const VT* __restrict__ val, const XT* __restrict__ x,
                                           int64_t n, const WinView& w, int64_t tile, int64_t r0,
                                           int64_t r1, ACC* prod) {
  static_assert(BLOCK == kWinRows, "one thread per row of a window tile");
  const int tid = threadIdx.x;
  const int32_t t0 = rowptr[r0], t1 = rowptr[r1];
  const int32_t ta = t0 & ~(V - 1);
  const int32_t k0 = w.ptr[tile], nbk = w.ptr[tile + 1] - k0;
  const bool own = tid < r1 - r0;
  int32_t ra, re;
  if constexpr (EAGER) {
    const int64_t ri = own ? r0 + tid : r0;  // loaded either way: no branch
    const int32_t ra0 = rowptr[ri], re0 = rowptr[ri + 1];
    ra = own ? ra0 - ta : 0;
    re = own ? re0 - ta : 0;
  } else {
    ra = own ? rowptr[r0 + tid] - ta : 0;
    re = own ? rowptr[r0 + tid + 1] - ta : 0;
  }
  if (nbk > 0)
    return window_chunks<true, EAGER, U, V, BLOCK, VT, XT, ACC, NT>(w.lcol, val, x, n, w.blk, k0,
                                                                    nbk, t0, t1, ra, re, prod);
  return window_chunks<false, EAGER, U, V, BLOCK, VT, XT, ACC, NT>(col, val, x, n, w.blk, k0, nbk,
                                                                   t0, t1, ra, re, prod);
}

// LDS bytes of the window walk with chunks of kWinRows * per_thread
// entries, for elements of `bytes` bytes.
__host__ __device__ inline size_t window_lds_bytes(int64_t max_blocks, size_t bytes,
                                                   int per_thread) {
  return ((size_t)kWinRows * per_thread + (size_t)max_blocks * kWinBlock) * bytes;
}

}  // namespace spx
