// COO -> CSR assembly on the device (paper Sec. 5, "Portable matrix assembly
// on GPUs"): a symbolic stage that turns the index arrays into a CSR pattern
// plus the jmap/perm maps, and a numeric stage in which one thread owns one
// stored entry and sums its contributions in input order (no atomics).
#include <algorithm>
#include <new>

#include "common.hpp"
#include "device.hpp"

namespace spx {

namespace {

constexpr int kBlock = 256;
constexpr int kIpt = 8;
constexpr int64_t kTile = kBlock * kIpt;

__device__ __forceinline__ uint32_t block_exscan(uint32_t v, uint32_t* lds_wave, uint32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  if (lane == 63) lds_wave[w] = inc;
  __syncthreads();
  uint32_t wave_off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) {
    uint32_t c = lds_wave[i];
    if (i < w) wave_off += c;
    tot += c;
  }
  __syncthreads();
  if (total) *total = tot;
  return wave_off + inc - v;
}

__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t value) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = value;
}

__global__ void k_fill_u32_local(uint32_t* p, int64_t count, uint32_t value) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = value;
}

__global__ void k_fill_f64(double* p, int64_t count, double value) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = value;
}

__global__ void k_iota_u32(uint32_t* p, int64_t count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = (uint32_t)t;
}

// Per tile of kTile triplets: number of kept triplets; flags indices >= n.
__global__ __launch_bounds__(kBlock) void k_coo_count(const int32_t* __restrict__ i,
                                                      const int32_t* __restrict__ j,
                                                      int64_t ncoo, int64_t n,
                                                      uint32_t* __restrict__ tilecnt,
                                                      int32_t* __restrict__ err) {
  __shared__ uint32_t lds[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  uint32_t c = 0;
  bool bad = false;
#pragma unroll
  for (int s = 0; s < kIpt; ++s) {
    const int64_t k = base + (int64_t)s * kBlock + threadIdx.x;
    if (k < ncoo) {
      const int32_t a = i[k], b = j[k];
      if (a >= 0 && b >= 0) {
        if (a >= n || b >= n)
          bad = true;
        else
          ++c;
      }
    }
  }
  if (bad) atomicOr(err, 1);
  uint32_t tot;
  (void)block_exscan(c, lds, &tot);
  if (threadIdx.x == 0) tilecnt[blockIdx.x] = tot;
}

// Stable compaction of the kept triplets into (key, k) pairs with
// key = row << cb | col (ROW_ONLY: key = row).  Wave w of a tile owns the contiguous items
// [w*512, (w+1)*512) and walks them in 64-item steps (coalesced loads); the
// write position of an item is its wave's offset plus the number of kept
// items before it, counted with ballots, so input order is preserved.
template <typename K, bool ROW_ONLY = false>
__global__ __launch_bounds__(kBlock) void k_coo_compact(const int32_t* __restrict__ i,
                                                        const int32_t* __restrict__ j,
                                                        int64_t ncoo, int64_t n, int cb,
                                                        const uint32_t* __restrict__ tileoff,
                                                        K* __restrict__ keys,
                                                        uint32_t* __restrict__ vals) {
  __shared__ uint32_t wcount[kBlock / 64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)w * (kIpt * 64);
  const uint64_t lt = (1ull << lane) - 1ull;
  int32_t a[kIpt], b[kIpt];
  bool keep[kIpt];
  uint32_t cnt = 0;
#pragma unroll
  for (int s = 0; s < kIpt; ++s) {
    const int64_t k = base + s * 64 + lane;
    a[s] = k < ncoo ? i[k] : -1;
    b[s] = k < ncoo ? j[k] : -1;
    keep[s] = a[s] >= 0 && b[s] >= 0 && a[s] < n && b[s] < n;
    cnt += (uint32_t)__popcll(__ballot(keep[s]));
  }
  if (lane == 0) wcount[w] = cnt;
  __syncthreads();
  uint32_t pos = tileoff[blockIdx.x];
  for (int ww = 0; ww < w; ++ww) pos += wcount[ww];
#pragma unroll
  for (int s = 0; s < kIpt; ++s) {
    const uint64_t m = __ballot(keep[s]);
    if (keep[s]) {
      const uint32_t at = pos + (uint32_t)__popcll(m & lt);
      if constexpr (ROW_ONLY)
        keys[at] = (K)(uint32_t)a[s];
      else
        keys[at] = ((K)(uint32_t)a[s] << cb) | (K)(uint32_t)b[s];
      vals[at] = (uint32_t)(base + s * 64 + lane);
    }
    pos += (uint32_t)__popcll(m);
  }
}

// Second stage of the two-stage order: the kept items sorted stably by row
// alone (increasing k within a row) are re-sorted by column inside each row
// in LDS, ties keeping their order, which gives the (row, column, k) order
// of the full sort.  Tile b takes the whole rows whose first item lies in
// [b kRowTile, (b + 1) kRowTile); when those rows hold more than kRowCap
// items, *overflow is set and the caller sorts the full keys instead.
// Output: key row << cb | col and k at the item's final position.
constexpr int64_t kRowTile = 512;  // 1024 measured slower (5.55 vs 5.3 ms at 131M items)
constexpr int kRowCap = 1024;
constexpr int kRowPosBits = 10;  // positions in a tile, in the rank key
static_assert(kRowCap <= (1 << kRowPosBits), "tile positions must fit the rank key");
constexpr int kRowColBits = 32 - kRowPosBits;  // columns of the rank key (n up to 2^22)
constexpr int kRowIpt = kRowCap / kBlock;  // items per thread

// The tile's range [q0, q1): q0 is the first row start in [b0, end0) (end0
// if none), q1 the first at or after end0, searched up to
// lim1 = end0 + kRowCap + 1 (q1 = lim1 when none is found there, which is
// more than kRowCap past any q0; q1 = count when lim1 reaches count).  Both
// searches run in the same steps; every thread gets both answers.
__device__ __forceinline__ void tile_rows(const uint32_t* __restrict__ rk, int64_t count,
                                          int64_t b0, int64_t end0, unsigned long long* slot,
                                          int64_t* q0, int64_t* q1) {
  const int64_t lim1 = end0 + kRowCap + 1 < count ? end0 + kRowCap + 1 : count;
  if (threadIdx.x == 0) {
    slot[0] = (unsigned long long)end0;
    slot[1] = (unsigned long long)lim1;
  }
  __syncthreads();
  for (int64_t off = 0;; off += kBlock) {
    const int64_t qa = b0 + off + threadIdx.x, qb = end0 + off + threadIdx.x;
    if (qa < end0 && (qa == 0 || rk[qa] != rk[qa - 1])) atomicMin(&slot[0], (unsigned long long)qa);
    if (qb < lim1 && rk[qb] != rk[qb - 1]) atomicMin(&slot[1], (unsigned long long)qb);
    __syncthreads();
    const bool done0 = slot[0] < (unsigned long long)end0 || b0 + off + kBlock >= end0;
    const bool done1 = slot[1] < (unsigned long long)lim1 || end0 + off + kBlock >= lim1;
    __syncthreads();
    if (done0 && done1) break;
  }
  *q0 = (int64_t)slot[0];
  *q1 = (int64_t)slot[1];
}

// The tile's rows are found with one block-wide scan: item l starts a row
// when its row key differs from item l - 1's; the inclusive count of starts
// numbers the rows, and each start records its position, so an item's row
// spans [start[row], start[row + 1]).  Its rank there is the number of the
// row's items with a smaller column, or an equal column and a smaller
// position (the row sort left equal columns in increasing k): one compare
// of col << kRowPosBits | position.  Thread t
// loads and ranks items t, t + kBlock, ...; the row numbering walks
// contiguous runs of kRowIpt items per thread.
__global__ __launch_bounds__(kBlock) void k_rowtile_sort(const uint32_t* __restrict__ rk,
                                                         const uint32_t* __restrict__ rv,
                                                         int64_t count,
                                                         const int32_t* __restrict__ j, int cb,
                                                         uint64_t* __restrict__ okeys,
                                                         uint32_t* __restrict__ ovals,
                                                         uint32_t* __restrict__ overflow) {
  __shared__ uint32_t srow[kRowCap];
  __shared__ uint32_t scol[kRowCap];
  __shared__ int32_t start[kRowCap + 1];
  __shared__ int16_t srid[kRowCap];
  __shared__ uint32_t wtot[kBlock / 64];
  __shared__ unsigned long long slot[2];
  const int64_t b0 = (int64_t)blockIdx.x * kRowTile;
  const int64_t end0 = b0 + kRowTile < count ? b0 + kRowTile : count;
  int64_t q0, q1;
  tile_rows(rk, count, b0, end0, slot, &q0, &q1);
  if (q0 >= end0) return;  // no row starts here
  if (q1 - q0 > kRowCap) {
    if (threadIdx.x == 0) atomicOr(overflow, 1u);
    return;
  }
  const int L = (int)(q1 - q0);
  uint32_t kv[kRowIpt];
#pragma unroll
  for (int u = 0; u < kRowIpt; ++u) {
    const int l = threadIdx.x + u * kBlock;
    if (l < L) {
      kv[u] = rv[q0 + l];
      srow[l] = rk[q0 + l];
    }
  }
#pragma unroll
  for (int u = 0; u < kRowIpt; ++u) {
    const int l = threadIdx.x + u * kBlock;
    if (l < L) scol[l] = ((uint32_t)j[kv[u]] << kRowPosBits) | (uint32_t)l;
  }
  __syncthreads();
  const int l0 = threadIdx.x * kRowIpt;
  uint32_t heads = 0;
#pragma unroll
  for (int u = 0; u < kRowIpt; ++u) {
    const int l = l0 + u;
    if (l < L && (l == 0 || srow[l] != srow[l - 1])) ++heads;
  }
  uint32_t tot;
  uint32_t run = block_exscan(heads, wtot, &tot);
#pragma unroll
  for (int u = 0; u < kRowIpt; ++u) {
    const int l = l0 + u;
    if (l < L) {
      if (l == 0 || srow[l] != srow[l - 1]) {
        start[run] = l;
        ++run;
      }
      srid[l] = (int16_t)(run - 1);
    }
  }
  if (threadIdx.x == 0) start[tot] = L;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kRowIpt; ++u) {
    const int l = threadIdx.x + u * kBlock;
    if (l < L) {
      const int rid = srid[l];
      const int rs = start[rid], re = start[rid + 1];
      const uint32_t key = scol[l];
      int rank = 0;
      // sixteen keys per step, their loads issued together
      int m = rs;
      for (; m + 16 <= re; m += 16) {
        uint32_t km[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) km[u] = scol[m + u];
#pragma unroll
        for (int u = 0; u < 16; ++u) rank += km[u] < key ? 1 : 0;
      }
      for (; m < re; ++m) rank += scol[m] < key ? 1 : 0;
      const int64_t at = q0 + rs + rank;
      okeys[at] = ((uint64_t)srow[l] << cb) | (uint64_t)(key >> kRowPosBits);
      ovals[at] = kv[u];
    }
  }
}

// Number of run heads (first element of each distinct key) per tile.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_heads_count(const K* __restrict__ keys,
                                                        int64_t count,
                                                        uint32_t* __restrict__ tilecnt) {
  __shared__ uint32_t lds[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  uint32_t c = 0;
#pragma unroll
  for (int s = 0; s < kIpt; ++s) {
    const int64_t q = base + (int64_t)s * kBlock + threadIdx.x;
    if (q < count && (q == 0 || keys[q] != keys[q - 1])) ++c;
  }
  uint32_t tot;
  (void)block_exscan(c, lds, &tot);
  if (threadIdx.x == 0) tilecnt[blockIdx.x] = tot;
}

// For each run head q (entry t): jmap[t] = q, col[t], diagonal position,
// and rowptr for every row that starts at t (empty rows included).  Same
// wave-ordered walk as the compaction: entry numbers are the tile offset
// plus the heads before q, counted with ballots.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_heads_emit(const K* __restrict__ keys, int64_t count,
                                                       int cb, const uint32_t* __restrict__ tileoff,
                                                       int32_t* __restrict__ jmap,
                                                       int32_t* __restrict__ col,
                                                       int32_t* __restrict__ rowptr,
                                                       int32_t* __restrict__ dpos) {
  __shared__ uint32_t wcount[kBlock / 64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)w * (kIpt * 64);
  const K cmask = cb >= (int)(8 * sizeof(K)) ? ~K(0) : ((K(1) << cb) - K(1));
  const uint64_t lt = (1ull << lane) - 1ull;
  K cur[kIpt], prev[kIpt];
  bool head[kIpt];
  uint32_t cnt = 0;
#pragma unroll
  for (int s = 0; s < kIpt; ++s) {
    const int64_t q = base + s * 64 + lane;
    cur[s] = q < count ? keys[q] : K(0);
    prev[s] = (q > 0 && q < count) ? keys[q - 1] : K(0);
    head[s] = q < count && (q == 0 || cur[s] != prev[s]);
    cnt += (uint32_t)__popcll(__ballot(head[s]));
  }
  if (lane == 0) wcount[w] = cnt;
  __syncthreads();
  uint32_t pos = tileoff[blockIdx.x];
  for (int ww = 0; ww < w; ++ww) pos += wcount[ww];
#pragma unroll
  for (int s = 0; s < kIpt; ++s) {
    const uint64_t m = __ballot(head[s]);
    if (head[s]) {
      const int64_t q = base + s * 64 + lane;
      const uint32_t t = pos + (uint32_t)__popcll(m & lt);
      const int64_t r = (int64_t)(cur[s] >> cb);
      const int32_t cc = (int32_t)(cur[s] & cmask);
      jmap[t] = (int32_t)q;
      col[t] = cc;
      if (r == cc) dpos[r] = (int32_t)t;
      const int64_t pr = q == 0 ? -1 : (int64_t)(prev[s] >> cb);
      for (int64_t rr = pr + 1; rr <= r; ++rr) rowptr[rr] = (int32_t)t;
    }
    pos += (uint32_t)__popcll(m);
  }
}

// rowptr of the rows after the last stored row, and the closing jmap entry.
template <typename K>
__global__ void k_rowptr_tail(const K* __restrict__ keys, int64_t count, int cb, int64_t n,
                              const uint32_t* __restrict__ nnz_dev, int32_t* __restrict__ rowptr,
                              int32_t* __restrict__ jmap) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t last = count > 0 ? (int64_t)(keys[count - 1] >> cb) : -1;
  const int32_t nnz = (int32_t)*nnz_dev;
  if (r <= n && r > last) rowptr[r] = nnz;
  if (r == 0 && jmap) jmap[nnz] = (int32_t)count;
}

// Longest row: wave max, then workgroup max in LDS, one atomic per workgroup.
__global__ __launch_bounds__(256) void k_max_row(const int32_t* __restrict__ rowptr, int64_t n,
                                                 int32_t* __restrict__ out) {
  __shared__ int32_t wmax[4];
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t len = r < n ? rowptr[r + 1] - rowptr[r] : 0;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) len = max(len, __shfl_xor(len, off, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = len;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(out, max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3])));
}

// Tiled numeric stage: a workgroup owns `ents` consecutive entries.
// Their contributions form one contiguous run of perm, which the workgroup
// reads coalesced while gathering v into LDS, kSvBatch values per thread at
// a time with all of a batch's gathers in flight before any is stored; then
// each thread adds its entries' contributions from LDS in order, from +0.0
// (bitwise the same sums as one thread walking perm).  The gather is bound
// by latency, not bytes, so the batches and a small LDS footprint (more
// workgroups per CU) are what set the rate.  A tile whose run exceeds kSvCap
// values is summed straight from memory, each thread issuing up to kSvBatch
// gathers of its own run before adding them in order.
constexpr int kSvBatch = 4;
constexpr int kSvCap = 2048;

// Entries per workgroup: the largest of 512, 256 and 128 whose tiles
// typically (1.5x the mean contributions per entry) fit in kSvCap values.
int sv_entries(int64_t nvalid, int64_t nnz) {
  const double per = nnz > 0 ? (double)nvalid / (double)nnz : 0.0;
  for (int e : {512, 256, 128})
    if (1.5 * per * e <= kSvCap) return e;
  return 64;
}

__global__ __launch_bounds__(256) void k_set_values_tiled(const int32_t* __restrict__ jmap,
                                                          const int32_t* __restrict__ perm,
                                                          const double* __restrict__ v,
                                                          int64_t nnz, int mode, int ents,
                                                          double* __restrict__ val) {
  __shared__ double lv[kSvCap];
  const int64_t e0 = (int64_t)blockIdx.x * ents;
  const int64_t e1 = e0 + ents < nnz ? e0 + ents : nnz;
  const int32_t q0 = jmap[e0], q1 = jmap[e1];
  if (q1 - q0 > kSvCap) {
    for (int64_t t = e0 + threadIdx.x; t < e1; t += 256) {
      const int32_t qe = jmap[t + 1];
      double s = 0.0;
      for (int32_t q = jmap[t]; q < qe; q += kSvBatch) {
        double x[kSvBatch];
#pragma unroll
        for (int k = 0; k < kSvBatch; ++k) x[k] = q + k < qe ? v[perm[q + k]] : 0.0;
#pragma unroll
        for (int k = 0; k < kSvBatch; ++k)
          if (q + k < qe) s += x[k];
      }
      val[t] = mode ? val[t] + s : s;
    }
    return;
  }
  for (int32_t base = q0; base < q1; base += 256 * kSvBatch) {
    int32_t p[kSvBatch];
#pragma unroll
    for (int k = 0; k < kSvBatch; ++k) {
      const int32_t q = base + k * 256 + (int32_t)threadIdx.x;
      p[k] = q < q1 ? perm[q] : -1;
    }
    double x[kSvBatch];
#pragma unroll
    for (int k = 0; k < kSvBatch; ++k) x[k] = p[k] >= 0 ? v[p[k]] : 0.0;
#pragma unroll
    for (int k = 0; k < kSvBatch; ++k) {
      const int32_t q = base + k * 256 + (int32_t)threadIdx.x;
      if (q < q1) lv[q - q0] = x[k];
    }
  }
  __syncthreads();
  for (int64_t t = e0 + threadIdx.x; t < e1; t += 256) {
    double s = 0.0;
    for (int32_t q = jmap[t]; q < jmap[t + 1]; ++q) s += lv[q - q0];
    val[t] = mode ? val[t] + s : s;
  }
}

__global__ void k_expand_rows(const int32_t* __restrict__ rowptr, int64_t n,
                              int32_t* __restrict__ rowidx) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int32_t t = rowptr[r]; t < rowptr[r + 1]; ++t) rowidx[t] = (int32_t)r;
}

// Explicit transpose from the column-sorted entries: tmap[tt] = entry of A.
__global__ void k_transpose_emit(const uint32_t* __restrict__ ckeys,
                                 const uint32_t* __restrict__ tmap, const int32_t* __restrict__ rowidx,
                                 int64_t nnz, int32_t* __restrict__ rowptrT,
                                 int32_t* __restrict__ colT, int32_t* __restrict__ dposT) {
  const int64_t tt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tt >= nnz) return;
  const int64_t c = ckeys[tt];
  const int32_t r = rowidx[tmap[tt]];
  colT[tt] = r;
  if (r == c) dposT[c] = (int32_t)tt;
  const int64_t pc = tt == 0 ? -1 : (int64_t)ckeys[tt - 1];
  for (int64_t cc = pc + 1; cc <= c; ++cc) rowptrT[cc] = (int32_t)tt;
}

__global__ void k_transpose_tail(const uint32_t* __restrict__ ckeys, int64_t nnz, int64_t n,
                                 int32_t* __restrict__ rowptrT) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t last = nnz > 0 ? (int64_t)ckeys[nnz - 1] : -1;
  if (r <= n && r > last) rowptrT[r] = (int32_t)nnz;
}

__global__ void k_gather_vals(const int32_t* __restrict__ tmap, const double* __restrict__ val,
                              int64_t nnz, double* __restrict__ valT) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nnz) valT[t] = val[tmap[t]];
}

__global__ void k_to_f32(const double* __restrict__ a, int64_t count, float* __restrict__ b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) b[t] = (float)a[t];
}

__global__ void k_kslot(const int32_t* __restrict__ jmap, const int32_t* __restrict__ perm,
                        int64_t nnz, int32_t* __restrict__ kslot) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nnz) return;
  for (int32_t q = jmap[t]; q < jmap[t + 1]; ++q) kslot[perm[q]] = (int32_t)t;
}

__global__ void k_coo_gather(const int32_t* __restrict__ kslot, const double* __restrict__ G,
                             int64_t ncoo, double* __restrict__ gv) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ncoo) return;
  const int32_t t = kslot[k];
  gv[k] = t >= 0 ? G[t] : 0.0;
}

__global__ void k_coo_gather_blocks(const int32_t* __restrict__ kslot,
                                    const double* __restrict__ G, const double* __restrict__ w,
                                    int64_t nblocks, int64_t block, double* __restrict__ ge) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nblocks) return;
  double s = 0.0;
  for (int64_t k = e * block; k < (e + 1) * block; ++k) {
    const int32_t t = kslot[k];
    const double g = t >= 0 ? G[t] : 0.0;
    s += g * w[k];
  }
  ge[e] = s;
}

inline unsigned grid_for(int64_t count, int block) {
  return (unsigned)std::max<int64_t>(1, ceil_div(count, block));
}

template <typename K>
int symbolic(spx_matrix* h, const int32_t* i, const int32_t* j, hipStream_t s) {
  const int64_t n = h->n, ncoo = h->ncoo;
  const int cb = h->colbits;
  const int bits = 2 * cb;
  const int64_t ntiles = std::max<int64_t>(1, ceil_div(ncoo, kTile));
  // misc: [0] err, [1] nvalid, [2] nnz, [3] maxrow, [4] row-tile overflow
  uint32_t* misc = nullptr;
  uint32_t* tilecnt = nullptr;
  K* keys = nullptr;
  // two separate value buffers: the one the sort leaves its result in
  // becomes perm as it is
  uint32_t* vals = nullptr;
  uint32_t* vals_alt = nullptr;
  int st = SPX_OK;
  uint32_t host_misc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t scratch_n = scan_scratch_elems(ntiles);
  if ((st = dalloc_n(&misc, 64)) != SPX_OK) return st;
  if ((st = dalloc_n(&tilecnt, (size_t)(ntiles + scratch_n))) != SPX_OK) {
    dfree(misc);
    return st;
  }
  uint32_t* scratch = tilecnt + ntiles;
  const int64_t cap = std::max<int64_t>(ncoo, 1);
  if ((st = dalloc(reinterpret_cast<void**>(&keys), sizeof(K) * (size_t)cap * 2 + 64)) != SPX_OK ||
      (st = dalloc_n(&vals, (size_t)cap)) != SPX_OK ||
      (st = dalloc_n(&vals_alt, (size_t)cap)) != SPX_OK) {
    dfree(keys);
    dfree(vals);
    dfree(tilecnt);
    dfree(misc);
    return st;
  }
  K* keys_alt = keys + cap;
  K* skeys = keys;
  uint32_t* svals = vals;
  int64_t nvalid = 0, nnz = 0;

  do {
    hipLaunchKernelGGL(k_fill_u32_local, dim3(1), dim3(64), 0, s, misc, (int64_t)64, 0u);
    hipLaunchKernelGGL(k_coo_count, dim3((unsigned)ntiles), dim3(kBlock), 0, s, i, j, ncoo, n,
                       tilecnt, (int32_t*)misc);
    if ((st = exclusive_scan_u32(tilecnt, tilecnt, ntiles, misc + 1, scratch, s)) != SPX_OK) break;
    // Keys wider than 32 bits take the two-stage order (up to 2^22 rows): a
    // stable sort by row alone (32-bit keys, half the passes of the full
    // key), then each tile's whole rows re-sorted by column in LDS.  The row keys and their
    // alternate buffer live in the first half of `keys`; the full keys come
    // out in the second half.
    bool two_stage = sizeof(K) == 8 && cb <= kRowColBits;
    if (hipMemcpyAsync(host_misc, misc, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = set_error(SPX_HIP_ERROR, "coo_preallocate: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
    if (host_misc[0]) {
      st = set_error(SPX_INDEX_OUT_OF_RANGE, "coo_preallocate: a COO index is >= n (%lld)",
                     (long long)n);
      break;
    }
    nvalid = host_misc[1];
    // With every triplet kept the row sort reads the caller's rows and takes
    // the triplet numbers as its values: no compaction.
    const bool all_kept = nvalid == ncoo;
    if (two_stage && !all_kept)
      hipLaunchKernelGGL((k_coo_compact<uint32_t, true>), dim3((unsigned)ntiles), dim3(kBlock), 0,
                         s, i, j, ncoo, n, cb, tilecnt, reinterpret_cast<uint32_t*>(keys), vals);
    else if (!two_stage)
      hipLaunchKernelGGL(k_coo_compact<K>, dim3((unsigned)ntiles), dim3(kBlock), 0, s, i, j, ncoo,
                         n, cb, tilecnt, keys, vals);
    if (two_stage) {
      uint32_t* rk = reinterpret_cast<uint32_t*>(keys);
      uint32_t *rk_out = nullptr, *rv_out = nullptr;
      if ((st = radix_sort_pairs_u32(rk, rk + cap, vals, vals_alt, nvalid, cb, s, &rk_out, &rv_out,
                                     all_kept ? reinterpret_cast<const uint32_t*>(i) : nullptr,
                                     all_kept)) != SPX_OK)
        break;
      K* ok = keys + cap;
      uint32_t* ov = rv_out == vals ? vals_alt : vals;
      if (nvalid > 0)
        hipLaunchKernelGGL(k_rowtile_sort, dim3((unsigned)ceil_div(nvalid, kRowTile)),
                           dim3(kBlock), 0, s, rk_out, rv_out, nvalid, j, cb,
                           reinterpret_cast<uint64_t*>(ok), ov, misc + 4);
      if (hipMemcpyAsync(host_misc + 4, misc + 4, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        st = set_error(SPX_HIP_ERROR, "coo_preallocate: %s", hipGetErrorString(hipGetLastError()));
        break;
      }
      if (host_misc[4] == 0) {
        skeys = ok;
        svals = ov;
      } else {
        // rows too long for a tile: the full keys, compacted again
        two_stage = false;
        hipLaunchKernelGGL(k_coo_compact<K>, dim3((unsigned)ntiles), dim3(kBlock), 0, s, i, j,
                           ncoo, n, cb, tilecnt, keys, vals);
      }
    }
    if (!two_stage &&
        (st = (sizeof(K) == 8
                   ? radix_sort_pairs_u64((uint64_t*)keys, (uint64_t*)keys_alt, vals, vals_alt,
                                          nvalid, bits, s, (uint64_t**)&skeys, &svals)
                   : radix_sort_pairs_u32((uint32_t*)keys, (uint32_t*)keys_alt, vals, vals_alt,
                                          nvalid, bits, s, (uint32_t**)&skeys, &svals))) != SPX_OK)
      break;
    const int64_t vt = std::max<int64_t>(1, ceil_div(nvalid, kTile));
    hipLaunchKernelGGL(k_heads_count<K>, dim3((unsigned)vt), dim3(kBlock), 0, s, skeys, nvalid,
                       tilecnt);
    if ((st = exclusive_scan_u32(tilecnt, tilecnt, vt, misc + 2, scratch, s)) != SPX_OK) break;
    if (hipMemcpyAsync(host_misc, misc, 16, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = set_error(SPX_HIP_ERROR, "coo_preallocate: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
    nnz = host_misc[2];
    h->nvalid = nvalid;
    h->A.n = n;
    h->A.nnz = nnz;
    if ((st = dalloc_n(&h->A.rowptr, (size_t)n + 1)) != SPX_OK) break;
    if ((st = dalloc_n(&h->A.dpos, (size_t)n)) != SPX_OK) break;
    if ((st = dalloc_n(&h->A.col, (size_t)std::max<int64_t>(nnz, 1))) != SPX_OK) break;
    if ((st = dalloc_n(&h->A.val, (size_t)std::max<int64_t>(nnz, 1))) != SPX_OK) break;
    if ((st = dalloc_n(&h->jmap, (size_t)nnz + 1)) != SPX_OK) break;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, s, h->A.dpos, n, -1);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(nnz, 256)), dim3(256), 0, s, h->A.val, nnz, 0.0);
    hipLaunchKernelGGL(k_heads_emit<K>, dim3((unsigned)vt), dim3(kBlock), 0, s, skeys, nvalid, cb,
                       tilecnt, h->jmap, h->A.col, h->A.rowptr, h->A.dpos);
    hipLaunchKernelGGL(k_rowptr_tail<K>, dim3(grid_for(n + 1, 256)), dim3(256), 0, s, skeys,
                       nvalid, cb, n, misc + 2, h->A.rowptr, h->jmap);
    hipLaunchKernelGGL(k_max_row, dim3(grid_for(n, 256)), dim3(256), 0, s, h->A.rowptr, n,
                       (int32_t*)(misc + 3));
    // The sorted values are perm; keep that buffer, release the rest.
    if (hipMemcpyAsync(host_misc, misc, 16, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = set_error(SPX_HIP_ERROR, "coo_preallocate: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
    h->A.max_row = host_misc[3];
    if ((st = compute_tiles(h->A, s)) != SPX_OK) break;
    if ((st = build_window(h->A, s)) != SPX_OK) break;
    h->perm = reinterpret_cast<int32_t*>(svals);
    if (svals == vals)
      vals = nullptr;
    else
      vals_alt = nullptr;
    if (hipStreamSynchronize(s) != hipSuccess) {
      st = set_error(SPX_HIP_ERROR, "coo_preallocate: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
  } while (false);

  dfree(keys);
  dfree(vals);
  dfree(vals_alt);
  dfree(tilecnt);
  dfree(misc);
  return st;
}

}  // namespace

int ensure_transpose(spx_matrix* h, hipStream_t s) {
  const int64_t n = h->n, nnz = h->A.nnz;
  if (!h->has_t) {
    uint32_t *keys = nullptr, *vals = nullptr;
    int32_t* rowidx = nullptr;
    const int64_t cap = std::max<int64_t>(nnz, 1);
    int st = SPX_OK;
    do {
      if ((st = dalloc_n(&keys, (size_t)cap * 2)) != SPX_OK) break;
      if ((st = dalloc_n(&vals, (size_t)cap * 2)) != SPX_OK) break;
      if ((st = dalloc_n(&rowidx, (size_t)cap)) != SPX_OK) break;
      if ((st = dalloc_n(&h->At.rowptr, (size_t)n + 1)) != SPX_OK) break;
      if ((st = dalloc_n(&h->At.col, (size_t)cap)) != SPX_OK) break;
      if ((st = dalloc_n(&h->At.val, (size_t)cap)) != SPX_OK) break;
      if ((st = dalloc_n(&h->At.dpos, (size_t)n)) != SPX_OK) break;
      if ((st = dalloc_n(&h->tmap, (size_t)cap)) != SPX_OK) break;
      hipLaunchKernelGGL(k_expand_rows, dim3(grid_for(n, 256)), dim3(256), 0, s, h->A.rowptr, n,
                         rowidx);
      if (nnz > 0) {
        SPX_CHECK_HIP(hipMemcpyAsync(keys, h->A.col, sizeof(int32_t) * (size_t)nnz,
                                     hipMemcpyDeviceToDevice, s));
      }
      hipLaunchKernelGGL(k_iota_u32, dim3(grid_for(nnz, 256)), dim3(256), 0, s, vals, nnz);
      uint32_t *sk = nullptr, *sv = nullptr;
      if ((st = radix_sort_pairs_u32(keys, keys + cap, vals, vals + cap, nnz, h->colbits, s, &sk,
                                     &sv)) != SPX_OK)
        break;
      hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, s, h->At.dpos, n, -1);
      hipLaunchKernelGGL(k_transpose_emit, dim3(grid_for(nnz, 256)), dim3(256), 0, s, sk, sv,
                         rowidx, nnz, h->At.rowptr, h->At.col, h->At.dpos);
      hipLaunchKernelGGL(k_transpose_tail, dim3(grid_for(n + 1, 256)), dim3(256), 0, s, sk, nnz, n,
                         h->At.rowptr);
      if (nnz > 0)
        SPX_CHECK_HIP(hipMemcpyAsync(h->tmap, sv, sizeof(int32_t) * (size_t)nnz,
                                     hipMemcpyDeviceToDevice, s));
      // row lengths of A^T
      int32_t* mx = rowidx;  // reuse as scratch after the emit kernels
      SPX_CHECK_HIP(hipStreamSynchronize(s));
      hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, mx, (int64_t)1, 0);
      hipLaunchKernelGGL(k_max_row, dim3(grid_for(n, 256)), dim3(256), 0, s, h->At.rowptr, n, mx);
      int32_t host_mx = 0;
      SPX_CHECK_HIP(hipMemcpyAsync(&host_mx, mx, 4, hipMemcpyDeviceToHost, s));
      SPX_CHECK_HIP(hipStreamSynchronize(s));
      h->At.max_row = host_mx;
      h->At.n = n;
      h->At.nnz = nnz;
      if ((st = compute_tiles(h->At, s)) != SPX_OK) break;
      if ((st = build_window(h->At, s)) != SPX_OK) break;
    } while (false);
    dfree(keys);
    dfree(vals);
    dfree(rowidx);
    if (st != SPX_OK) return st;
    h->has_t = true;
    h->valT_fresh = false;
  }
  if (!h->valT_fresh) {
    hipLaunchKernelGGL(k_gather_vals, dim3(grid_for(nnz, 256)), dim3(256), 0, s, h->tmap, h->A.val,
                       nnz, h->At.val);
    h->valT_fresh = true;
    h->valT32_fresh = false;
  }
  return SPX_OK;
}

int ensure_val32(spx_matrix* h, hipStream_t s) {
  if (!h->A.val32) SPX_TRY(dalloc_n(&h->A.val32, (size_t)std::max<int64_t>(h->A.nnz, 1)));
  if (!h->val32_fresh) {
    hipLaunchKernelGGL(k_to_f32, dim3(grid_for(h->A.nnz, 256)), dim3(256), 0, s, h->A.val,
                       h->A.nnz, h->A.val32);
    h->val32_fresh = true;
  }
  return SPX_OK;
}

int ensure_kslot(spx_matrix* h, hipStream_t s) {
  if (h->kslot) return SPX_OK;
  SPX_TRY(dalloc_n(&h->kslot, (size_t)std::max<int64_t>(h->ncoo, 1)));
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(h->ncoo, 256)), dim3(256), 0, s, h->kslot, h->ncoo,
                     -1);
  hipLaunchKernelGGL(k_kslot, dim3(grid_for(h->A.nnz, 256)), dim3(256), 0, s, h->jmap, h->perm,
                     h->A.nnz, h->kslot);
  return SPX_OK;
}

}  // namespace spx

using namespace spx;

extern "C" int spx_coo_preallocate(int64_t n, int64_t ncoo, const int32_t* i, const int32_t* j,
                                   void* stream, spx_handle* out) {
  clear_error();
  if (!out) return set_error(SPX_INVALID_ARG, "coo_preallocate: out is NULL");
  *out = nullptr;
  if (n <= 0 || n > INT32_MAX - 1)
    return set_error(SPX_INVALID_ARG, "coo_preallocate: n = %lld out of [1, 2^31-2]", (long long)n);
  if (ncoo < 0 || ncoo > INT32_MAX - 1)
    return set_error(SPX_INVALID_ARG, "coo_preallocate: ncoo = %lld out of [0, 2^31-2]",
                     (long long)ncoo);
  if (ncoo > 0 && (!i || !j)) return set_error(SPX_INVALID_ARG, "coo_preallocate: i or j is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  spx_matrix* h = new (std::nothrow) spx_matrix();
  if (!h) return set_error(SPX_OUT_OF_MEMORY, "coo_preallocate: host allocation failed");
  SPX_CHECK_HIP(hipGetDevice(&h->device));
  h->n = n;
  h->ncoo = ncoo;
  int cb = 0;
  while (cb < 31 && ((int64_t)1 << cb) < n) ++cb;  // bits of n-1
  h->colbits = cb;
  const int st = (2 * cb <= 32) ? symbolic<uint32_t>(h, i, j, s) : symbolic<uint64_t>(h, i, j, s);
  if (st != SPX_OK) {
    spx_destroy(h);
    return st;
  }
  *out = h;
  return SPX_OK;
}

namespace spx {
int set_values_into(spx_handle h, const double* v, int mode, double* out, hipStream_t s) {
  const int64_t nnz = h->A.nnz;
  if (nnz > 0) {
    const int ents = sv_entries(h->nvalid, nnz);
    hipLaunchKernelGGL(k_set_values_tiled, dim3(grid_for(nnz, ents)), dim3(256), 0, s, h->jmap,
                       h->perm, v, nnz, mode, ents, out);
  }
  SPX_CHECK_HIP(hipGetLastError());
  return SPX_OK;
}
}  // namespace spx

extern "C" int spx_set_values_coo(spx_handle h, const double* v, int mode, void* stream) {
  clear_error();
  if (!h) return set_error(SPX_INVALID_ARG, "set_values_coo: NULL handle");
  if (mode != SPX_INSERT_VALUES && mode != SPX_ADD_VALUES)
    return set_error(SPX_INVALID_ARG, "set_values_coo: mode %d is not INSERT(0) or ADD(1)", mode);
  if (h->nvalid > 0 && !v) return set_error(SPX_INVALID_ARG, "set_values_coo: v is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t nnz = h->A.nnz;
  if (nnz > 0) {
    const int ents = sv_entries(h->nvalid, nnz);
    hipLaunchKernelGGL(k_set_values_tiled, dim3(grid_for(nnz, ents)), dim3(256), 0, s, h->jmap,
                       h->perm, v, nnz, mode, ents, h->A.val);
  }
  h->valT_fresh = false;
  h->val32_fresh = false;
  h->valT32_fresh = false;
  SPX_CHECK_HIP(hipGetLastError());
  return SPX_OK;
}

extern "C" int spx_get_info(spx_handle h, int64_t* n, int64_t* nnz, int64_t* nvalid,
                            int64_t* ncoo) {
  clear_error();
  if (!h) return set_error(SPX_INVALID_ARG, "get_info: NULL handle");
  if (n) *n = h->n;
  if (nnz) *nnz = h->A.nnz;
  if (nvalid) *nvalid = h->nvalid;
  if (ncoo) *ncoo = h->ncoo;
  return SPX_OK;
}

extern "C" int spx_get_csr(spx_handle h, int32_t transpose, int32_t* rowptr, int32_t* col,
                           double* val, void* stream) {
  clear_error();
  if (!h) return set_error(SPX_INVALID_ARG, "get_csr: NULL handle");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (transpose) SPX_TRY(ensure_transpose(h, s));
  const Csr& M = transpose ? h->At : h->A;
  if (rowptr)
    SPX_CHECK_HIP(hipMemcpyAsync(rowptr, M.rowptr, sizeof(int32_t) * (size_t)(h->n + 1),
                                 hipMemcpyDeviceToDevice, s));
  if (col && M.nnz)
    SPX_CHECK_HIP(hipMemcpyAsync(col, M.col, sizeof(int32_t) * (size_t)M.nnz,
                                 hipMemcpyDeviceToDevice, s));
  if (val && M.nnz)
    SPX_CHECK_HIP(hipMemcpyAsync(val, M.val, sizeof(double) * (size_t)M.nnz,
                                 hipMemcpyDeviceToDevice, s));
  return SPX_OK;
}

extern "C" int spx_get_coo_maps(spx_handle h, int32_t* jmap, int32_t* perm, void* stream) {
  clear_error();
  if (!h) return set_error(SPX_INVALID_ARG, "get_coo_maps: NULL handle");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (jmap)
    SPX_CHECK_HIP(hipMemcpyAsync(jmap, h->jmap, sizeof(int32_t) * (size_t)(h->A.nnz + 1),
                                 hipMemcpyDeviceToDevice, s));
  if (perm && h->nvalid)
    SPX_CHECK_HIP(hipMemcpyAsync(perm, h->perm, sizeof(int32_t) * (size_t)h->nvalid,
                                 hipMemcpyDeviceToDevice, s));
  return SPX_OK;
}

extern "C" int spx_coo_gather(spx_handle h, const double* G, double* grad_v, void* stream) {
  clear_error();
  if (!h || (h->ncoo > 0 && (!G || !grad_v)))
    return set_error(SPX_INVALID_ARG, "coo_gather: NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  SPX_TRY(ensure_kslot(h, s));
  if (h->ncoo > 0)
    hipLaunchKernelGGL(k_coo_gather, dim3(grid_for(h->ncoo, 256)), dim3(256), 0, s, h->kslot, G,
                       h->ncoo, grad_v);
  SPX_CHECK_HIP(hipGetLastError());
  return SPX_OK;
}

extern "C" int spx_coo_gather_blocks(spx_handle h, const double* G, const double* w,
                                     int64_t block, double* grad_e, void* stream) {
  clear_error();
  if (!h || block <= 0 || (h->ncoo > 0 && (!G || !w || !grad_e)))
    return set_error(SPX_INVALID_ARG, "coo_gather_blocks: bad argument");
  if (h->ncoo % block != 0)
    return set_error(SPX_INVALID_ARG, "coo_gather_blocks: ncoo %lld is not a multiple of %lld",
                     (long long)h->ncoo, (long long)block);
  hipStream_t s = static_cast<hipStream_t>(stream);
  SPX_TRY(ensure_kslot(h, s));
  const int64_t nb = h->ncoo / block;
  if (nb > 0)
    hipLaunchKernelGGL(k_coo_gather_blocks, dim3(grid_for(nb, 256)), dim3(256), 0, s, h->kslot, G,
                       w, nb, block, grad_e);
  SPX_CHECK_HIP(hipGetLastError());
  return SPX_OK;
}
