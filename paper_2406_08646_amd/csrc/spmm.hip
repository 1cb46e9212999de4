// Y = A X for 16 contiguous right-hand sides (multi-RHS product of the
// batched forms, paper Sec. 7) with each tile's rows of X staged in LDS.
//
// A 16-column row of X is 128 bytes, and on a stencil operator the 27
// entries of a row and the entries of the rows next to it name mostly the
// same rows of X: a tile of 32 consecutive rows of the 3-D 27-point
// operator has 864 entries but only 306 distinct columns.  Gathering a row
// of X per entry (the pair kernels in spmv.hip) moves 3.5 KB per matrix row
// from L2 to the compute units; staging the tile's distinct rows once, with
// coalesced 128-byte loads, moves 1.2 KB, and the products then read X from
// LDS.  The distinct columns of every tile and each entry's position among
// them (16 bits, 2 bytes per entry where the column index takes 4) are
// built once per pattern on the first such product.
//
// Each row's products are added in entry order from +0.0, as the pair
// kernels do, so the results are bitwise theirs, at every tile height
// (16, 32 or 64 rows; SPX_OPT_SPMM_TILE_ROWS, 32 by default).
#include <algorithm>

#include <utility>

#include "common.hpp"
#include "device.hpp"

namespace spx {
namespace {

// Tile shapes: entries a tile may hold (the index builder sorts that many
// columns in LDS) and distinct columns it may stage (kMax rows of X and a
// row of zeros: 24, 40 and 80 KB of LDS).
template <int ROWS>
struct RsShape;
template <>
struct RsShape<16> {
  static constexpr int kCap = 1024, kMax = 191, kWaves = 6;
};
template <>
struct RsShape<32> {
  static constexpr int kCap = 1024, kMax = 319, kWaves = 8;
};
template <>
struct RsShape<64> {
  static constexpr int kCap = 2048, kMax = 639, kWaves = 8;
};

constexpr int kRsBlock = 256;  // threads of the index builder

// The tile's columns (m <= CAP of them, from entry e0) in LDS, sorted
// ascending; the slots after m hold INT32_MAX.
template <int CAP>
__device__ __forceinline__ void rs_sorted_columns(const int32_t* __restrict__ col, int32_t e0,
                                                  int m, int32_t* keys) {
  for (int i = threadIdx.x; i < CAP; i += kRsBlock) keys[i] = i < m ? col[e0 + i] : INT32_MAX;
  __syncthreads();
  // bitonic network over CAP keys
  for (int k = 2; k <= CAP; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < CAP; i += kRsBlock) {
        const int p = i ^ j;
        if (p > i) {
          const int32_t a = keys[i], b = keys[p];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            keys[i] = b;
            keys[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ bool rs_first(const int32_t* keys, int i) {
  return keys[i] != INT32_MAX && (i == 0 || keys[i] != keys[i - 1]);
}

// The list of tile b (count, then the distinct columns) at ucol + b *
// (kMax + 1) and every entry's position in it; the count -1 for a tile that
// is gathered instead.
template <int ROWS>
__global__ __launch_bounds__(kRsBlock) void k_rs_build(int64_t n, const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ col,
                                                       int32_t* __restrict__ ucol,
                                                       uint16_t* __restrict__ lidx) {
  constexpr int CAP = RsShape<ROWS>::kCap, MAX = RsShape<ROWS>::kMax;
  static_assert(CAP % kRsBlock == 0, "whole sort steps");
  constexpr int IPT = CAP / kRsBlock;
  __shared__ int32_t keys[CAP];
  __shared__ int32_t list[MAX];
  __shared__ int32_t wsum[kRsBlock / 64];
  const int64_t b = blockIdx.x, r0 = b * ROWS;
  const int64_t r1 = r0 + ROWS < n ? r0 + ROWS : n;
  int32_t* out = ucol + b * (MAX + 1);
  const int32_t e0 = rowptr[r0];
  const int m = rowptr[r1] - e0;
  if (m > CAP) {
    if (threadIdx.x == 0) out[0] = -1;
    return;
  }
  rs_sorted_columns<CAP>(col, e0, m, keys);
  // rank of every first occurrence: thread t owns IPT consecutive keys
  const int i0 = threadIdx.x * IPT;
  int firsts = 0;
#pragma unroll
  for (int u = 0; u < IPT; ++u) firsts += rs_first(keys, i0 + u) ? 1 : 0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int inc = firsts;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int d = 0, rank = inc - firsts;
  for (int ww = 0; ww < kRsBlock / 64; ++ww) {
    if (ww < w) rank += wsum[ww];
    d += wsum[ww];
  }
  if (d > MAX) {
    if (threadIdx.x == 0) out[0] = -1;
    return;
  }
  if (threadIdx.x == 0) out[0] = d;
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    if (rs_first(keys, i0 + u)) {
      list[rank] = keys[i0 + u];
      out[1 + rank] = keys[i0 + u];
      ++rank;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += kRsBlock) {
    const int32_t c = col[e0 + i];
    int lo = 0, hi = d;  // list[lo] == c at the end
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (list[mid] <= c)
        lo = mid;
      else
        hi = mid;
    }
    lidx[e0 + i] = (uint16_t)lo;
  }
}

// The product: tile b of ROWS rows, 16 lanes per row, lane c computing
// column c.  A staged tile first loads its rows of X into registers (every
// load of a thread issued before any of its stores) and copies them to LDS,
// after them one row of zeros (kMax + 1 rows of 128 bytes).  It then walks
// each row's entries in chunks of 32: lanes l and 16 + l of the chunk hold
// entry l and 16 + l as a value and the byte offset of its row of X in LDS,
// and entry j reaches the whole row by a DPP broadcast within the 16-lane
// row (row_newbcast), which the compiler folds into the address add; the
// value takes one 64-bit DPP move.  So the entries never pass through LDS
// and X is the only LDS traffic: one conflict-free 128-byte read per row
// and entry.  The slots of a chunk past the row's end hold the value 0 and
// the zero row, and add +0.0 to a sum that is never -0.0, so they change
// nothing.  A gathered tile (count -1) reads columns and X directly.
constexpr int kRpLanes = 16;
constexpr int kRpRow = kRpLanes * 8;  // bytes of a row of X
typedef double rs_d2 __attribute__((ext_vector_type(2)));

template <int J>
__device__ __forceinline__ int rs_bcast(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x150 + J, 0xf, 0xf, true);
}
template <int J>
__device__ __forceinline__ double rs_bcast(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + J, 0xf, 0xf, true);
}

template <int J>
__device__ __forceinline__ int rs_bcast_i(int v) {
  return rs_bcast<J>(v);
}
template <int J>
__device__ __forceinline__ double rs_bcast_d(double v) {
  return rs_bcast<J>(v);
}

// Entries J..J+3 of a chunk into s, in entry order.
template <int J>
__device__ __forceinline__ void rs_entries(double va, int ca, double vb, int cb,
                                           const char* __restrict__ xl, double& s) {
  double x[4], v[4];
  x[0] = *reinterpret_cast<const double*>(xl + (J < 16 ? rs_bcast<J & 15>(ca) : rs_bcast<J & 15>(cb)));
  x[1] = *reinterpret_cast<const double*>(xl + (J + 1 < 16 ? rs_bcast<(J + 1) & 15>(ca) : rs_bcast<(J + 1) & 15>(cb)));
  x[2] = *reinterpret_cast<const double*>(xl + (J + 2 < 16 ? rs_bcast<(J + 2) & 15>(ca) : rs_bcast<(J + 2) & 15>(cb)));
  x[3] = *reinterpret_cast<const double*>(xl + (J + 3 < 16 ? rs_bcast<(J + 3) & 15>(ca) : rs_bcast<(J + 3) & 15>(cb)));
  v[0] = J < 16 ? rs_bcast<J & 15>(va) : rs_bcast<J & 15>(vb);
  v[1] = J + 1 < 16 ? rs_bcast<(J + 1) & 15>(va) : rs_bcast<(J + 1) & 15>(vb);
  v[2] = J + 2 < 16 ? rs_bcast<(J + 2) & 15>(va) : rs_bcast<(J + 2) & 15>(vb);
  v[3] = J + 3 < 16 ? rs_bcast<(J + 3) & 15>(va) : rs_bcast<(J + 3) & 15>(vb);
  s += v[0] * x[0];
  s += v[1] * x[1];
  s += v[2] * x[2];
  s += v[3] * x[3];
}

// The m <= 32 entries of a chunk, in groups of four.
template <int J>
__device__ __forceinline__ void rs_chunk(int m, double va, int ca, double vb, int cb,
                                         const char* __restrict__ xl, double& s) {
  if constexpr (J < 32) {
    if (J < m) {
      rs_entries<J>(va, ca, vb, cb, xl, s);
      rs_chunk<J + 4>(m, va, ca, vb, cb, xl, s);
    }
  }
}

// Entries J..J+7 of a chunk into s, in entry order: eight LDS reads in
// flight before the first add, for the pipelined form's fewer waves.
template <int J, int... K>
__device__ __forceinline__ void rs_entries8_(double va, int ca, double vb, int cb,
                                             const char* __restrict__ xl, double& s,
                                             std::integer_sequence<int, K...>) {
  const double x[8] = {*reinterpret_cast<const double*>(
      xl + ((J + K < 16) ? rs_bcast_i<(J + K) & 15>(ca) : rs_bcast_i<(J + K) & 15>(cb)))...};
  const double v[8] = {((J + K < 16) ? rs_bcast_d<(J + K) & 15>(va)
                                     : rs_bcast_d<(J + K) & 15>(vb))...};
#pragma unroll
  for (int k = 0; k < 8; ++k) s += v[k] * x[k];
}
template <int J>
__device__ __forceinline__ void rs_entries8(double va, int ca, double vb, int cb,
                                            const char* __restrict__ xl, double& s) {
  rs_entries8_<J>(va, ca, vb, cb, xl, s, std::make_integer_sequence<int, 8>{});
}

template <int J>
__device__ __forceinline__ void rs_chunk8(int m, double va, int ca, double vb, int cb,
                                          const char* __restrict__ xl, double& s) {
  if constexpr (J < 32) {
    if (J < m) {
      rs_entries8<J>(va, ca, vb, cb, xl, s);
      rs_chunk8<J + 8>(m, va, ca, vb, cb, xl, s);
    }
  }
}

// Entries base + lane and base + 16 + lane of a row: value and byte offset
// of the entry's row of X in LDS, or 0 and the zero row (row zrow) past the
// row's end.
__device__ __forceinline__ void rs_load_chunk(const double* __restrict__ val,
                                              const uint16_t* __restrict__ lidx, int32_t t0,
                                              int len, int base, int lane, int zrow, double& va,
                                              int& ca, double& vb, int& cb) {
  va = vb = 0.0;
  ca = cb = zrow * kRpRow;
  if (base + lane < len) {
    va = stream_load(val + t0 + base + lane);
    ca = (int)lidx[t0 + base + lane] * kRpRow;
  }
  if (base + kRpLanes + lane < len) {
    vb = stream_load(val + t0 + base + kRpLanes + lane);
    cb = (int)lidx[t0 + base + kRpLanes + lane] * kRpRow;
  }
}

template <int ROWS>
__global__ __launch_bounds__(ROWS * kRpLanes) __attribute__((amdgpu_waves_per_eu(RsShape<ROWS>::kWaves, 8))) void k_spmm_rowset(
    int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const int32_t* __restrict__ ucol,
    const uint16_t* __restrict__ lidx, const double* __restrict__ X, double* __restrict__ Y) {
  constexpr int MAX = RsShape<ROWS>::kMax;
  constexpr int BLOCK = ROWS * kRpLanes;
  constexpr int XQ = (MAX * 8 + BLOCK - 1) / BLOCK;  // 16-byte pieces per thread
  static_assert(XQ * BLOCK == (MAX + 1) * 8, "the pieces past the list cover the zero row");
  __shared__ rs_d2 xs2[(MAX + 1) * 8];
  const int64_t b = blockIdx.x, r0 = b * ROWS;
  const int64_t row = r0 + threadIdx.x / kRpLanes;
  const int lane = threadIdx.x % kRpLanes;
  const int64_t rr = row < n ? row : n - 1;
  const int32_t t0 = rowptr[rr], t1 = rowptr[rr + 1];
  const int len = row < n ? t1 - t0 : 0;
  // the list and its count in one go: the list's place is fixed
  const int32_t* list = ucol + b * (MAX + 1);
  const int d = list[0];
  int32_t lst[XQ];
#pragma unroll
  for (int u = 0; u < XQ; ++u) {
    const int q = threadIdx.x + u * BLOCK;
    lst[u] = list[1 + (q < MAX * 8 ? q : MAX * 8 - 1) / 8];
  }
  // the whole list in registers here, its loads in flight with the row's
  // bounds: a load of it left for later would hold back the loads of X
#pragma unroll
  for (int u = 0; u < XQ; ++u) asm volatile("" : "+v"(lst[u]));
  if (d >= 0) {
    // Every load of the staging is issued, where its result goes unused
    // from a valid address near the ones in use (the row's first entry,
    // which the tail padding keeps inside the arrays even for an empty last
    // row; a row of X of the tile's own rows), so that none has to wait for
    // another: loads under data-dependent branches each waited for all the
    // loads before them.  The chain is list, then X, then the barrier.  The
    // first chunk of the row's entries comes with them.
    const bool ha = lane < len, hb = kRpLanes + lane < len;
    const int32_t ia = ha ? t0 + lane : t0, ib = hb ? t0 + kRpLanes + lane : t0;
    double va0 = stream_load(val + ia), vb0 = stream_load(val + ib);
    int pa = lidx[ia], pb = lidx[ib];
    const rs_d2* X2 = reinterpret_cast<const rs_d2*>(X);
    rs_d2 xv[XQ];
#pragma unroll
    for (int u = 0; u < XQ; ++u) {
      const int q = threadIdx.x + u * BLOCK;
      const int64_t own = r0 + (q / 8) % ROWS;
      xv[u] = X2[(q < d * 8 ? (int64_t)lst[u] : own < n ? own : n - 1) * 8 + q % 8];
    }
    // pieces past the list write zeros into the zero row (row MAX), which
    // they cover whole since XQ * BLOCK == (MAX + 1) * 8
#pragma unroll
    for (int u = 0; u < XQ; ++u) {
      const int q = threadIdx.x + u * BLOCK;
      const bool in = q < d * 8;
      xs2[in ? q : MAX * 8 + q % 8] = in ? xv[u] : rs_d2{0.0, 0.0};
    }
    // the entries are needed here, so their loads stay ahead of the barrier
    asm volatile("" : "+v"(va0), "+v"(vb0), "+v"(pa), "+v"(pb));
    double va = ha ? va0 : 0.0, vb = hb ? vb0 : 0.0;
    int ca = (ha ? pa : MAX) * kRpRow, cb = (hb ? pb : MAX) * kRpRow;
    __syncthreads();
    if (row >= n) return;
    const char* xl = reinterpret_cast<const char*>(xs2) + lane * 8;
    double s = 0.0;
    for (int base = 0;;) {
      rs_chunk<0>(len - base, va, ca, vb, cb, xl, s);
      base += 2 * kRpLanes;
      if (base >= len) break;
      rs_load_chunk(val, lidx, t0, len, base, lane, MAX, va, ca, vb, cb);
    }
    Y[row * 16 + lane] = s;
    return;
  }
  if (row >= n) return;
  double s = 0.0;
  for (int32_t t = t0; t < t0 + len; ++t) s += val[t] * X[(int64_t)col[t] * 16 + lane];
  Y[row * 16 + lane] = s;
}

// The pipelined form of the product (32-row tiles): a persistent grid of
// two workgroups per CU, each with two LDS buffers of the tile's rows of X.
// While a workgroup forms the products of one tile from one buffer, the
// next tile's rows of X are already loading into the other by direct
// global-to-LDS loads (lane l of a wave writes 16 bytes at the wave's base +
// 16 l, so they take no registers), with that tile's first chunk of entries
// and the list and row bounds of the tile after it.  The two buffers are
// separate arrays, so the products' LDS reads wait only for LDS; they go
// eight at a time (rs_chunk8) for the fewer waves.  Every tile's products
// are those of k_spmm_rowset, bitwise (tested).  On the 128^3-node operator
// 0.337-0.342 ms against 0.353 for k_spmm_rowset at 32-row tiles (which
// keeps the 16- and 64-row tiles: at 64 rows a second 80 KB buffer would
// leave one workgroup per CU, at 16 rows three instead of six).
struct RsNext {      // list and row bounds of a tile whose X is still to load
  int d;
  int32_t t0, t1;
  int32_t lst[(RsShape<32>::kMax * 8 + 511) / 512];
};
struct RsCur {       // a tile whose X is loading or loaded
  int d;
  int32_t t0;
  int len;
  double va, vb;
  int pa, pb;
};

// Loads (issues) the list and this thread's row bounds of tile b; d = -2
// when there is no tile b.  Every load is unconditional (tile and row
// clamped to the last), so none of them is held back by a branch and the
// results need no copies at a join, which would wait for them.
template <int ROWS>
__device__ __forceinline__ void rsp_next(int64_t n, const int32_t* __restrict__ rowptr,
                                         const int32_t* __restrict__ ucol, int64_t b,
                                         int64_t tiles, RsNext& nx) {
  constexpr int MAX = RsShape<ROWS>::kMax;
  constexpr int BLOCK = ROWS * kRpLanes;
  constexpr int XQ = (MAX * 8 + BLOCK - 1) / BLOCK;
  const int64_t bc = b < tiles ? b : tiles - 1;
  const int32_t* list = ucol + bc * (MAX + 1);
  const int d = list[0];
  nx.d = b < tiles ? d : -2;
#pragma unroll
  for (int u = 0; u < XQ; ++u) {
    const int q = threadIdx.x + u * BLOCK;
    nx.lst[u] = list[1 + (q < MAX * 8 ? q : MAX * 8 - 1) / 8];
  }
  const int64_t row = bc * ROWS + threadIdx.x / kRpLanes;
  const int64_t rr = row < n ? row : n - 1;
  const int32_t t0 = rowptr[rr], t1 = rowptr[rr + 1];
  nx.t0 = t0;
  nx.t1 = row < n ? t1 : t0;
}

// Issues the direct loads of tile nx's rows of X into buf (a staged tile)
// and the loads of its first chunk of entries into cu (always, from valid
// addresses).
template <int ROWS>
__device__ __forceinline__ void rsp_issue(const RsNext& nx, const double* __restrict__ val,
                                          const uint16_t* __restrict__ lidx,
                                          const double* __restrict__ X, rs_d2* buf, RsCur& cu) {
  constexpr int MAX = RsShape<ROWS>::kMax;
  constexpr int BLOCK = ROWS * kRpLanes;
  constexpr int XQ = (MAX * 8 + BLOCK - 1) / BLOCK;
  const int lane = threadIdx.x % kRpLanes;
  cu.d = nx.d;
  cu.t0 = nx.t0;
  cu.len = nx.t1 - nx.t0;
  const rs_d2* X2 = reinterpret_cast<const rs_d2*>(X);
  const int wv = threadIdx.x >> 6;
  const int nq = nx.d > 0 ? nx.d * 8 : 0;
#pragma unroll
  for (int u = 0; u < XQ; ++u) {
    const int q = threadIdx.x + u * BLOCK;
    if (q < nq)
      __builtin_amdgcn_global_load_lds(
          (const __attribute__((address_space(1))) void*)(X2 + (int64_t)nx.lst[u] * 8 + q % 8),
          (__attribute__((address_space(3))) void*)(buf + u * BLOCK + wv * 64), 16, 0, 0);
  }
  const bool ha = lane < cu.len, hb = kRpLanes + lane < cu.len;
  const int32_t ia = ha ? cu.t0 + lane : cu.t0, ib = hb ? cu.t0 + kRpLanes + lane : cu.t0;
  cu.va = stream_load(val + ia);
  cu.vb = stream_load(val + ib);
  cu.pa = lidx[ia];
  cu.pb = lidx[ib];
}

// The products of tile b (state cu, rows of X in buf when staged).
template <int ROWS>
__device__ __forceinline__ void rsp_products(int64_t n, int64_t b, const RsCur& cu,
                                             const int32_t* __restrict__ col,
                                             const double* __restrict__ val,
                                             const uint16_t* __restrict__ lidx,
                                             const double* __restrict__ X,
                                             double* __restrict__ Y, const rs_d2* buf) {
  constexpr int MAX = RsShape<ROWS>::kMax;
  const int64_t row = b * ROWS + threadIdx.x / kRpLanes;
  const int lane = threadIdx.x % kRpLanes;
  if (row >= n) return;
  double s = 0.0;
  if (cu.d >= 0) {
    const int len = cu.len;
    const bool ha = lane < len, hb = kRpLanes + lane < len;
    double va = ha ? cu.va : 0.0, vb = hb ? cu.vb : 0.0;
    int ca = (ha ? cu.pa : MAX) * kRpRow, cb = (hb ? cu.pb : MAX) * kRpRow;
    const char* xl = reinterpret_cast<const char*>(buf) + lane * 8;
    for (int base = 0;;) {
      rs_chunk8<0>(len - base, va, ca, vb, cb, xl, s);
      base += 2 * kRpLanes;
      if (base >= len) break;
      rs_load_chunk(val, lidx, cu.t0, len, base, lane, MAX, va, ca, vb, cb);
    }
  } else {
    for (int32_t t = cu.t0; t < cu.t0 + cu.len; ++t)
      s += val[t] * X[(int64_t)col[t] * 16 + lane];
  }
  Y[row * 16 + lane] = s;
}

// One step of the pipeline for tile b, whose rows of X the step before
// issued into cur (state cu) with the list of tile b + step (nx): wait for
// them, issue tile b + step's rows of X into nxt (state cn) and the list of
// tile b + 2 step (into nn), then form b's products from cur.  The kernel
// alternates two sets of state so that none is copied while its loads are
// in flight.
template <int ROWS>
__device__ __forceinline__ void rsp_step(int64_t n, const int32_t* __restrict__ rowptr,
                                         const int32_t* __restrict__ col,
                                         const double* __restrict__ val,
                                         const int32_t* __restrict__ ucol,
                                         const uint16_t* __restrict__ lidx,
                                         const double* __restrict__ X, double* __restrict__ Y,
                                         int64_t b, int64_t step, int64_t tiles, const RsCur& cu,
                                         RsCur& cn, const RsNext& nx, RsNext& nn,
                                         const rs_d2* cur, rs_d2* nxt) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();  // b's X in cur; every thread done with nxt's last tile
  rsp_issue<ROWS>(nx, val, lidx, X, nxt, cn);
  rsp_next<ROWS>(n, rowptr, ucol, b + 2 * step, tiles, nn);
  rsp_products<ROWS>(n, b, cu, col, val, lidx, X, Y, cur);
}

template <int ROWS>
__global__ __launch_bounds__(ROWS * kRpLanes) void k_spmm_rowset_pipe(
    int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const int32_t* __restrict__ ucol,
    const uint16_t* __restrict__ lidx, const double* __restrict__ X, double* __restrict__ Y) {
  constexpr int MAX = RsShape<ROWS>::kMax;
  static_assert(ROWS == 32, "the pipelined form is built for 32-row tiles");
  __shared__ rs_d2 xa[(MAX + 1) * 8];
  __shared__ rs_d2 xb[(MAX + 1) * 8];
  const int64_t tiles = ceil_div(n, ROWS), step = gridDim.x;
  if (threadIdx.x < 8) {
    xa[MAX * 8 + threadIdx.x] = rs_d2{0.0, 0.0};
    xb[MAX * 8 + threadIdx.x] = rs_d2{0.0, 0.0};
  }
  RsNext na, nb;
  RsCur ca, cb;
  // workgroup w takes tiles b0, b0 + step, ... with b0 its XCD-grouped
  // number: at any time the grid works on one stretch of step tiles, and
  // each XCD on a contiguous part of it, so neighbouring lines' tiles share
  // an L2 (0.336-0.338 ms against 0.341-0.342 in workgroup order)
  int64_t b = xcd_logical_block(blockIdx.x, gridDim.x);
  rsp_next<ROWS>(n, rowptr, ucol, b, tiles, na);
  __builtin_amdgcn_s_waitcnt(0);
  rsp_issue<ROWS>(na, val, lidx, X, xa, ca);
  rsp_next<ROWS>(n, rowptr, ucol, b + step, tiles, nb);
  for (;;) {
    if (b >= tiles) break;
    rsp_step<ROWS>(n, rowptr, col, val, ucol, lidx, X, Y, b, step, tiles, ca, cb, nb, na, xa, xb);
    b += step;
    if (b >= tiles) break;
    rsp_step<ROWS>(n, rowptr, col, val, ucol, lidx, X, Y, b, step, tiles, cb, ca, na, nb, xb, xa);
    b += step;
  }
}

template <int ROWS>
int build_rowset_t(Csr& A, hipStream_t s) {
  RowSet& R = A.rs;
  const int64_t tiles = ceil_div(A.n, ROWS);
  int st = SPX_OK;
  do {
    if ((st = dalloc_n(&R.col, (size_t)(tiles * (RsShape<ROWS>::kMax + 1)))) != SPX_OK) break;
    if ((st = dalloc_n(&R.lidx, (size_t)std::max<int64_t>(A.nnz, 1))) != SPX_OK) break;
    hipLaunchKernelGGL(k_rs_build<ROWS>, dim3((unsigned)tiles), dim3(kRsBlock), 0, s, A.n,
                       A.rowptr, A.col, R.col, R.lidx);
    if (hipGetLastError() != hipSuccess) {
      st = set_error(SPX_HIP_ERROR, "spmm: row-set index: launch failed");
      break;
    }
  } while (false);
  return st;
}

}  // namespace

int build_rowset(Csr& A, int rows, hipStream_t s) {
  RowSet& R = A.rs;
  if (rows != 16 && rows != 32 && rows != 64)
    return set_error(SPX_INVALID_ARG, "spmm: tile height %d is not 16, 32 or 64", rows);
  if (A.n == 0 || (R.built && R.rows == rows)) return SPX_OK;
  // a new tile height: the lists are built again
  dfree(R.col);
  dfree(R.lidx);
  R = RowSet();
  const int st = rows == 16   ? build_rowset_t<16>(A, s)
                 : rows == 32 ? build_rowset_t<32>(A, s)
                              : build_rowset_t<64>(A, s);
  if (st != SPX_OK) {
    dfree(R.col);
    dfree(R.lidx);
    R = RowSet();
    return st;
  }
  R.rows = rows;
  R.built = true;
  return SPX_OK;
}

int launch_spmm_rowset(const Csr& A, const double* X, double* Y, hipStream_t s) {
  const RowSet& R = A.rs;
  if (A.n == 0) return SPX_OK;
  auto go = [&](auto k, int rows) {
    hipLaunchKernelGGL(k, dim3((unsigned)ceil_div(A.n, rows)), dim3(rows * kRpLanes), 0, s, A.n,
                       A.rowptr, A.col, A.val, R.col, R.lidx, X, Y);
  };
  if (R.rows == 16) {
    go(k_spmm_rowset<16>, 16);
  } else if (R.rows == 64) {
    go(k_spmm_rowset<64>, 64);
  } else {
    // 32-row tiles: the pipelined form, a persistent grid of the workgroups
    // that fit at once (two per CU with its two 40 KB buffers; asked once)
    static const int fit = [] {
      int f = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
              &f, reinterpret_cast<const void*>(&k_spmm_rowset_pipe<32>), 32 * kRpLanes, 0) !=
              hipSuccess ||
          f < 1)
        f = 1;
      (void)hipGetLastError();
      return f;
    }();
    const int64_t grid = std::min<int64_t>(ceil_div(A.n, 32), (int64_t)fit * cu_count());
    hipLaunchKernelGGL(k_spmm_rowset_pipe<32>, dim3((unsigned)grid), dim3(32 * kRpLanes), 0, s,
                       A.n, A.rowptr, A.col, A.val, R.col, R.lidx, X, Y);
  }
  return SPX_OK;
}

}  // namespace spx
