// Window index of a CSR pattern for the window walk of the products: per
// tile of kWinRows rows, the ascending list of the kWinBlock-entry blocks of
// x that its columns fall in, and each entry's position in that list.
// Built on the device once per pattern (after the symbolic assembly, and for
// the explicit transpose when it is built): one pass marks each tile's
// blocks in an LDS bitmap and counts them, a scan turns the counts into
// offsets, and a second pass writes the block lists and the 16-bit window
// columns.  Values are never touched, so set_values_coo keeps it valid.
#include <algorithm>
#include <climits>

#include "common.hpp"
#include "device.hpp"

namespace spx {

namespace {

constexpr int kWinWords = kWinSpan / 32;  // bitmap words of one tile
static_assert(kWinWords == kWinRows, "one bitmap word per thread");
static_assert(kWinMaxBlocks * kWinBlock <= 65536, "window columns fit in 16 bits");

__device__ __forceinline__ int32_t wg_min(int32_t v, int32_t* red) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  __syncthreads();  // earlier readers of red are done
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return min(min(red[0], red[1]), min(red[2], red[3]));
}

__device__ __forceinline__ int32_t wg_max(int32_t v, int32_t* red) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return max(max(red[0], red[1]), max(red[2], red[3]));
}

__device__ __forceinline__ int32_t wg_sum(int32_t v, int32_t* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// Marks the blocks of entries [t0, t1) in bits (relative to block lo).
__device__ __forceinline__ void mark_blocks(const int32_t* __restrict__ col, int32_t t0, int32_t t1,
                                            int32_t lo, uint32_t* bits) {
  bits[threadIdx.x] = 0;
  __syncthreads();
  for (int32_t e = t0 + (int32_t)threadIdx.x; e < t1; e += kWinRows) {
    const int32_t d = col[e] / kWinBlock - lo;
    atomicOr(&bits[d >> 5], 1u << (d & 31));
  }
  __syncthreads();
}

// Per tile: blocks in its window (0 if it gets none) and its lowest block.
// stats[0] += entries of tiles without a window; stats[1] = largest window.
__global__ __launch_bounds__(kWinRows) void k_win_count(int64_t n, const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        uint32_t* __restrict__ cnt,
                                                        int32_t* __restrict__ lo_out,
                                                        unsigned long long* __restrict__ stats) {
  __shared__ uint32_t bits[kWinWords];
  __shared__ int32_t red[kWinRows / 64];
  const int64_t t = blockIdx.x;
  const int64_t r0 = t * kWinRows;
  const int64_t r1 = r0 + kWinRows < n ? r0 + kWinRows : n;
  const int32_t t0 = rowptr[r0], t1 = rowptr[r1];
  if (t0 == t1) {
    if (threadIdx.x == 0) {
      cnt[t] = 0;
      lo_out[t] = 0;
    }
    return;
  }
  int32_t lo = INT_MAX, hi = -1;
  for (int32_t e = t0 + (int32_t)threadIdx.x; e < t1; e += kWinRows) {
    const int32_t b = col[e] / kWinBlock;
    lo = min(lo, b);
    hi = max(hi, b);
  }
  lo = wg_min(lo, red);
  hi = wg_max(hi, red);
  int32_t c = 0;
  if (hi - lo < kWinSpan) {
    mark_blocks(col, t0, t1, lo, bits);
    c = wg_sum(__popc(bits[threadIdx.x]), red);
    if (c > kWinMaxBlocks) c = 0;
  }
  if (threadIdx.x == 0) {
    cnt[t] = (uint32_t)c;
    lo_out[t] = lo;
    if (c == 0)
      atomicAdd(&stats[0], (unsigned long long)(t1 - t0));
    else
      atomicMax(&stats[1], (unsigned long long)c);
  }
}

// Per tile with a window: blk[ptr[t] ..] = its blocks ascending, and
// lcol[e] = (rank of e's block) * kWinBlock + col[e] % kWinBlock.
__global__ __launch_bounds__(kWinRows) void k_win_emit(int64_t n, const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ col,
                                                       const int32_t* __restrict__ ptr,
                                                       const int32_t* __restrict__ lo_in,
                                                       int32_t* __restrict__ blk,
                                                       uint16_t* __restrict__ lcol) {
  __shared__ uint32_t bits[kWinWords];
  __shared__ uint32_t incl[kWinWords];
  const int64_t t = blockIdx.x;
  const int32_t k0 = ptr[t];
  if (ptr[t + 1] == k0) return;
  const int64_t r0 = t * kWinRows;
  const int64_t r1 = r0 + kWinRows < n ? r0 + kWinRows : n;
  const int32_t t0 = rowptr[r0], t1 = rowptr[r1];
  const int32_t lo = lo_in[t];
  const int tid = threadIdx.x;
  mark_blocks(col, t0, t1, lo, bits);
  const uint32_t w = bits[tid];
  incl[tid] = __popc(w);
  __syncthreads();
  for (int o = 1; o < kWinWords; o <<= 1) {
    const uint32_t v = tid >= o ? incl[tid - o] : 0u;
    __syncthreads();
    incl[tid] += v;
    __syncthreads();
  }
  uint32_t rank = incl[tid] - __popc(w);
  for (uint32_t m = w; m != 0; m &= m - 1) blk[k0 + rank++] = lo + tid * 32 + (__ffs(m) - 1);
  for (int32_t e = t0 + tid; e < t1; e += kWinRows) {
    const int32_t c = col[e];
    const int32_t d = c / kWinBlock - lo;
    const uint32_t word = bits[d >> 5];
    const uint32_t r = incl[d >> 5] - __popc(word) + __popc(word & ((1u << (d & 31)) - 1u));
    lcol[e] = (uint16_t)(r * kWinBlock + c % kWinBlock);
  }
}

__global__ void k_win_zero(unsigned long long* p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0;
}

void release(Window& w) {
  dfree(w.lcol);
  dfree(w.ptr);
  dfree(w.blk);
  w = Window();
}

}  // namespace

// Builds A.win, or leaves it empty when the window walk would not pay: the
// staged windows would hold more than two x entries per matrix entry, or
// more than one entry in eight would sit in tiles without a window.  Out of
// device memory for the index also leaves it empty (the products then take
// another walk); other failures are reported.
int build_window(Csr& A, hipStream_t s) {
  release(A.win);
  if (A.n == 0 || A.nnz == 0) return SPX_OK;
  const int64_t tiles = ceil_div(A.n, kWinRows);
  uint32_t* cnt = nullptr;
  int32_t* lo = nullptr;
  int32_t* ptr = nullptr;
  uint32_t* scratch = nullptr;
  unsigned long long* stats = nullptr;
  int st = SPX_OK;
  do {
    if ((st = dalloc_n(&cnt, (size_t)tiles)) != SPX_OK) break;
    if ((st = dalloc_n(&lo, (size_t)tiles)) != SPX_OK) break;
    if ((st = dalloc_n(&ptr, (size_t)tiles + 1)) != SPX_OK) break;
    if ((st = dalloc_n(&scratch, (size_t)scan_scratch_elems(tiles))) != SPX_OK) break;
    if ((st = dalloc_n(&stats, 2)) != SPX_OK) break;
    hipLaunchKernelGGL(k_win_zero, dim3(1), dim3(64), 0, s, stats);
    hipLaunchKernelGGL(k_win_count, dim3((unsigned)tiles), dim3(kWinRows), 0, s, A.n, A.rowptr,
                       A.col, cnt, lo, stats);
    if ((st = exclusive_scan_u32(cnt, reinterpret_cast<uint32_t*>(ptr), tiles,
                                 reinterpret_cast<uint32_t*>(ptr) + tiles, scratch, s)) != SPX_OK)
      break;
    unsigned long long hs[2] = {0, 0};
    int32_t total = 0;
    hipError_t e = hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&total, ptr + tiles, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      st = set_error(SPX_HIP_ERROR, "window index: %s", hipGetErrorString(e));
      break;
    }
    const bool pays = hs[1] > 0 && (int64_t)total * kWinBlock <= 2 * A.nnz &&
                      (int64_t)hs[0] * 8 <= A.nnz;
    if (!pays) break;
    Window w;
    w.ptr = ptr;
    w.max_blocks = (int64_t)hs[1];
    w.total_blocks = total;
    w.gather_entries = (int64_t)hs[0];
    if ((st = dalloc_n(&w.lcol, (size_t)A.nnz)) != SPX_OK ||
        (st = dalloc_n(&w.blk, (size_t)std::max<int32_t>(total, 1))) != SPX_OK) {
      ptr = nullptr;  // released with w
      release(w);
      break;
    }
    hipLaunchKernelGGL(k_win_emit, dim3((unsigned)tiles), dim3(kWinRows), 0, s, A.n, A.rowptr, A.col,
                       ptr, lo, w.blk, w.lcol);
    if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess) {
      ptr = nullptr;
      release(w);
      st = set_error(SPX_HIP_ERROR, "window index: %s", hipGetErrorString(e));
      break;
    }
    A.win = w;
    ptr = nullptr;  // owned by A.win
  } while (false);
  (void)hipStreamSynchronize(s);
  dfree(cnt);
  dfree(lo);
  dfree(ptr);
  dfree(scratch);
  dfree(stats);
  if (st == SPX_OUT_OF_MEMORY) {
    clear_error();
    return SPX_OK;
  }
  return st;
}

}  // namespace spx

using namespace spx;

extern "C" int spx_get_window(spx_handle h, int32_t transpose, int64_t* stats, int32_t* ptr,
                              int32_t* blk, uint16_t* lcol, void* stream) {
  clear_error();
  if (!h || !stats) return set_error(SPX_INVALID_ARG, "get_window: NULL handle or stats");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (transpose) SPX_TRY(ensure_transpose(h, s));
  const Csr& M = transpose ? h->At : h->A;
  const Window& w = M.win;
  stats[0] = w.lcol ? 1 : 0;
  stats[1] = w.max_blocks;
  stats[2] = w.total_blocks;
  stats[3] = w.gather_entries;
  if (!w.lcol) return SPX_OK;
  const int64_t tiles = ceil_div(M.n, kWinRows);
  if (ptr)
    SPX_CHECK_HIP(hipMemcpyAsync(ptr, w.ptr, sizeof(int32_t) * (size_t)(tiles + 1),
                                 hipMemcpyDeviceToDevice, s));
  if (blk && w.total_blocks)
    SPX_CHECK_HIP(hipMemcpyAsync(blk, w.blk, sizeof(int32_t) * (size_t)w.total_blocks,
                                 hipMemcpyDeviceToDevice, s));
  if (lcol && M.nnz)
    SPX_CHECK_HIP(hipMemcpyAsync(lcol, w.lcol, sizeof(uint16_t) * (size_t)M.nnz,
                                 hipMemcpyDeviceToDevice, s));
  return SPX_OK;
}
