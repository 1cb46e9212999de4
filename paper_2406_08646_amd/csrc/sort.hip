// Device scan and stable LSD radix sort of (key, value) pairs for gfx950.
//
// The COO symbolic stage orders the kept triplets by (row, column) and must
// keep equal keys in input order, so that duplicate contributions are later
// summed in increasing triplet index.  A least-significant-digit radix sort
// is stable by construction as long as every scatter pass is stable; the
// scatter below ranks keys inside a tile with wave ballots (64-lane match of
// equal digits) and per-wave counters in LDS, then stages the tile in LDS in
// digit order so that global writes go out in contiguous runs.
#include <algorithm>

#include "common.hpp"
#include "device.hpp"

namespace spx {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanIpt = 8;
constexpr int64_t kScanTile = kScanBlock * kScanIpt;

constexpr int kSortBlock = 256;
constexpr int kSortWaves = kSortBlock / 64;
constexpr int kSortSteps = 8;  // 64-item steps per wave
constexpr int64_t kSortTile = kSortBlock * kSortSteps;
constexpr int kMaxDigitBits = 8;
constexpr int kMaxBins = 1 << kMaxDigitBits;

// Exclusive scan of one value per thread over a block of kScanBlock threads.
__device__ __forceinline__ uint32_t block_exclusive_scan_u32(uint32_t v, uint32_t* lds_wave,
                                                             uint32_t* block_total) {
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
  for (int i = 0; i < kScanBlock / 64; ++i) {
    uint32_t c = lds_wave[i];
    if (i < w) wave_off += c;
    tot += c;
  }
  __syncthreads();
  if (block_total) *block_total = tot;
  return wave_off + inc - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const uint32_t* __restrict__ in,
                                                            int64_t count,
                                                            uint32_t* __restrict__ bsum) {
  __shared__ uint32_t lds[kScanBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIpt;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanIpt; ++k)
    if (base + k < count) s += in[base + k];
  uint32_t tot;
  (void)block_exclusive_scan_u32(s, lds, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const uint32_t* in, uint32_t* out,
                                                           int64_t count,
                                                           const uint32_t* __restrict__ boff,
                                                           uint32_t* __restrict__ total) {
  __shared__ uint32_t lds[kScanBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIpt;
  uint32_t v[kScanIpt];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanIpt; ++k) {
    v[k] = (base + k < count) ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t run = block_exclusive_scan_u32(s, lds, nullptr) + (boff ? boff[blockIdx.x] : 0u);
#pragma unroll
  for (int k = 0; k < kScanIpt; ++k) {
    if (base + k < count) {
      out[base + k] = run;
      if (total && base + k == count - 1) *total = run + v[k];
    }
    run += v[k];
  }
}

__global__ void k_fill_u32(uint32_t* p, int64_t count, uint32_t value) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = value;
}

// ------------------------------------------------------------ radix sort

// Digits of equal value among the active lanes of a wave: returns the mask
// of lanes holding the same digit as this lane.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int dbits, uint64_t active) {
  uint64_t peers = active;
  for (int b = 0; b < dbits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

template <typename K>
__global__ __launch_bounds__(kSortBlock) void k_radix_hist(const K* __restrict__ keys,
                                                           int64_t count, int shift, int dbits,
                                                           uint32_t* __restrict__ hist,
                                                           int64_t ntiles) {
  __shared__ uint32_t cnt[kMaxBins];
  const int nb = 1 << dbits;
  for (int d = threadIdx.x; d < kMaxBins; d += kSortBlock) cnt[d] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const uint32_t mask = (uint32_t)nb - 1u;
  const int lane = threadIdx.x & 63;
  const uint64_t lt = (1ull << lane) - 1ull;
  K k[kSortSteps];
#pragma unroll
  for (int s = 0; s < kSortSteps; ++s) {
    const int64_t idx = base + (int64_t)s * kSortBlock + threadIdx.x;
    k[s] = idx < count ? keys[idx] : K(0);
  }
#pragma unroll
  for (int s = 0; s < kSortSteps; ++s) {
    const int64_t idx = base + (int64_t)s * kSortBlock + threadIdx.x;
    const bool valid = idx < count;
    const uint32_t d = (uint32_t)(k[s] >> shift) & mask;
    const uint64_t peers = match_digit(d, dbits, __ballot(valid));
    if (valid && (peers & lt) == 0) atomicAdd(&cnt[d], (uint32_t)__popcll(peers));
  }
  __syncthreads();
  for (int d = threadIdx.x; d < nb; d += kSortBlock) hist[(int64_t)d * ntiles + blockIdx.x] = cnt[d];
}

template <typename K>
__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(
    const K* __restrict__ keys, const uint32_t* __restrict__ vals, K* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, int64_t count, int shift, int dbits,
    const uint32_t* __restrict__ hist_scan, int64_t ntiles) {
  __shared__ K skey[kSortTile];
  __shared__ uint32_t sval[kSortTile];
  __shared__ uint32_t wcnt[kSortWaves][kMaxBins];
  __shared__ uint32_t toff[kMaxBins];
  __shared__ uint32_t gbase[kMaxBins];
  __shared__ uint32_t scan_lds[kSortBlock / 64];

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int nb = 1 << dbits;
  const uint32_t mask = (uint32_t)nb - 1u;
  for (int d = tid; d < kMaxBins; d += kSortBlock)
#pragma unroll
    for (int ww = 0; ww < kSortWaves; ++ww) wcnt[ww][d] = 0;
  __syncthreads();

  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const int64_t rem = count - base;
  const int tile_n = (int)(rem < kSortTile ? rem : kSortTile);
  const uint64_t lt = (1ull << lane) - 1ull;

  // Each wave owns a contiguous quarter of the tile and walks it in order,
  // so ranks follow input order: stability.
  K k[kSortSteps];
  uint32_t v[kSortSteps];
  uint32_t rank[kSortSteps];
#pragma unroll
  for (int s = 0; s < kSortSteps; ++s) {
    const int local = w * (kSortSteps * 64) + s * 64 + lane;
    if (local < tile_n) {
      k[s] = keys[base + local];
      v[s] = vals ? vals[base + local] : (uint32_t)(base + local);
    } else {
      k[s] = K(0);
      v[s] = 0;
    }
  }
#pragma unroll
  for (int s = 0; s < kSortSteps; ++s) {
    const int local = w * (kSortSteps * 64) + s * 64 + lane;
    const bool valid = local < tile_n;
    const uint32_t d = (uint32_t)(k[s] >> shift) & mask;
    const uint64_t peers = match_digit(d, dbits, __ballot(valid));
    rank[s] = 0;
    if (valid) {
      const uint32_t before = wcnt[w][d];
      const uint64_t below = peers & lt;
      rank[s] = before + (uint32_t)__popcll(below);
      if (below == 0) wcnt[w][d] = before + (uint32_t)__popcll(peers);
    }
  }
  __syncthreads();

  uint32_t tot = 0;
  if (tid < nb) {
    uint32_t run = 0;
#pragma unroll
    for (int ww = 0; ww < kSortWaves; ++ww) {
      const uint32_t c = wcnt[ww][tid];
      wcnt[ww][tid] = run;
      run += c;
    }
    tot = run;
    gbase[tid] = hist_scan[(int64_t)tid * ntiles + blockIdx.x];
  }
  const uint32_t ex = block_exclusive_scan_u32(tot, scan_lds, nullptr);
  if (tid < nb) toff[tid] = ex;
  __syncthreads();

#pragma unroll
  for (int s = 0; s < kSortSteps; ++s) {
    const int local = w * (kSortSteps * 64) + s * 64 + lane;
    if (local < tile_n) {
      const uint32_t d = (uint32_t)(k[s] >> shift) & mask;
      const uint32_t lp = toff[d] + wcnt[w][d] + rank[s];
      skey[lp] = k[s];
      sval[lp] = v[s];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < tile_n; idx += kSortBlock) {
    const K kk = skey[idx];
    const uint32_t d = (uint32_t)(kk >> shift) & mask;
    const int64_t pos = (int64_t)gbase[d] + (idx - (int64_t)toff[d]);
    keys_out[pos] = kk;
    vals_out[pos] = sval[idx];
  }
}

// first_keys (optional): the first pass reads its keys there instead of in
// keys, and with iota_vals its values are the item indices (vals is then
// only written); keys and vals are overwritten either way.
template <typename K>
int radix_sort_impl(K* keys, K* keys_alt, uint32_t* vals, uint32_t* vals_alt, int64_t count,
                    int bits, hipStream_t s, K** keys_out, uint32_t** vals_out,
                    const K* first_keys = nullptr, bool iota_vals = false) {
  *keys_out = keys;
  *vals_out = vals;
  if (count <= 1 || bits <= 0) {
    if (first_keys || iota_vals) {
      // nothing to order: the output is the input
      if (count == 1 && first_keys)
        SPX_CHECK_HIP(hipMemcpyAsync(keys, first_keys, sizeof(K), hipMemcpyDeviceToDevice, s));
      if (count == 1 && iota_vals)
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, vals, (int64_t)1, 0u);
    }
    return SPX_OK;
  }
  if (bits > (int)(8 * sizeof(K)))
    return set_error(SPX_INVALID_ARG, "radix sort: %d bits exceed the key width", bits);
  const int passes = (bits + kMaxDigitBits - 1) / kMaxDigitBits;
  const int dbits = (bits + passes - 1) / passes;
  const int nb = 1 << dbits;
  const int64_t ntiles = ceil_div(count, kSortTile);
  const int64_t hist_n = (int64_t)nb * ntiles;
  if (hist_n >= (int64_t)UINT32_MAX || count >= (int64_t)UINT32_MAX)
    return set_error(SPX_INVALID_ARG, "radix sort: %lld items is too many",
                     (long long)count);
  uint32_t* hist = nullptr;
  const int64_t scratch_n = scan_scratch_elems(hist_n);
  SPX_TRY(dalloc_n(&hist, (size_t)(hist_n + scratch_n)));
  uint32_t* scratch = hist + hist_n;
  // pass p reads (ck, cv) and writes (ak, av); with first_keys the first
  // pass reads the caller's keys and writes keys_alt, so the passes after
  // it alternate between keys_alt and keys
  const K* ck = first_keys ? first_keys : keys;
  K* ak = keys_alt;
  const uint32_t* cv = iota_vals ? nullptr : vals;
  uint32_t* av = vals_alt;
  K* next_k = keys;
  uint32_t* next_v = vals;
  int st = SPX_OK;
  for (int p = 0; p < passes && st == SPX_OK; ++p) {
    const int shift = p * dbits;
    hipLaunchKernelGGL(k_radix_hist<K>, dim3((unsigned)ntiles), dim3(kSortBlock), 0, s, ck, count,
                       shift, dbits, hist, ntiles);
    st = exclusive_scan_u32(hist, hist, hist_n, nullptr, scratch, s);
    if (st != SPX_OK) break;
    hipLaunchKernelGGL(k_radix_scatter<K>, dim3((unsigned)ntiles), dim3(kSortBlock), 0, s, ck,
                       cv, ak, av, count, shift, dbits, hist, ntiles);
    // the buffer just written is the next input; the other one takes the
    // next output
    K* wk = ak;
    uint32_t* wv = av;
    ak = next_k;
    av = next_v;
    next_k = wk;
    next_v = wv;
    ck = wk;
    cv = wv;
  }
  hipError_t e = hipGetLastError();
  // The free below waits for the passes; preallocation is synchronous.
  hipError_t e2 = hipStreamSynchronize(s);
  dfree(hist);
  if (st != SPX_OK) return st;
  if (e != hipSuccess) return set_error(SPX_HIP_ERROR, "radix sort launch: %s", hipGetErrorString(e));
  if (e2 != hipSuccess)
    return set_error(SPX_HIP_ERROR, "radix sort: %s", hipGetErrorString(e2));
  *keys_out = const_cast<K*>(ck);
  *vals_out = const_cast<uint32_t*>(cv);
  return SPX_OK;
}

}  // namespace

int64_t scan_scratch_elems(int64_t count) {
  int64_t total = 0;
  int64_t c = count;
  while (c > kScanTile) {
    c = ceil_div(c, kScanTile);
    total += c + 64;
  }
  return total + 64;
}

int exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t count, uint32_t* total,
                       uint32_t* scratch, hipStream_t s) {
  if (count <= 0) {
    if (total) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, total, (int64_t)1, 0u);
    return SPX_OK;
  }
  const int64_t nt = ceil_div(count, kScanTile);
  if (nt == 1) {
    hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kScanBlock), 0, s, in, out, count,
                       (const uint32_t*)nullptr, total);
    return SPX_OK;
  }
  uint32_t* bsum = scratch;
  uint32_t* next = scratch + ((nt + 64) & ~int64_t(63));
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nt), dim3(kScanBlock), 0, s, in, count, bsum);
  SPX_TRY(exclusive_scan_u32(bsum, bsum, nt, nullptr, next, s));
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nt), dim3(kScanBlock), 0, s, in, out, count,
                     (const uint32_t*)bsum, total);
  return SPX_OK;
}

int radix_sort_pairs_u64(uint64_t* keys, uint64_t* keys_alt, uint32_t* vals, uint32_t* vals_alt,
                         int64_t count, int bits, hipStream_t s, uint64_t** keys_out,
                         uint32_t** vals_out) {
  return radix_sort_impl<uint64_t>(keys, keys_alt, vals, vals_alt, count, bits, s, keys_out,
                                   vals_out);
}

int radix_sort_pairs_u32(uint32_t* keys, uint32_t* keys_alt, uint32_t* vals, uint32_t* vals_alt,
                         int64_t count, int bits, hipStream_t s, uint32_t** keys_out,
                         uint32_t** vals_out, const uint32_t* first_keys, bool iota_vals) {
  return radix_sort_impl<uint32_t>(keys, keys_alt, vals, vals_alt, count, bits, s, keys_out,
                                   vals_out, first_keys, iota_vals);
}

}  // namespace spx
