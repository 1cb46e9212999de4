// CSR products for gfx950: y = A x, y = A^T x (on the explicit transpose)
// and Y = A X for a row-major block of right-hand sides.
//
// A row is handled by an aligned group of L lanes of a 64-wide wave: the
// group reads the row's values and column indices as one contiguous run
// (coalesced, non-temporal so the streamed matrix does not evict x from
// L2), gathers x, and reduces with a fixed butterfly.  L is chosen from the
// mean row length.  Blocks are renumbered so each XCD walks a contiguous row
// range, which keeps the x entries shared by neighbouring rows in that XCD's
// L2.  No MFMA: SpMV moves ~6 bytes per flop, far below the matrix-core
// ridge point, so the kernel is bound by HBM bandwidth.
//
// Where the pattern has a window index, the default walk is the window
// walk: a workgroup per tile of kWinRows rows stages the x blocks its
// columns touch in LDS and streams values with 16-bit window columns, so
// the x gather becomes an LDS read and each entry moves 10 bytes instead of
// 12; its row sums are bitwise those of the stream walk.
#include <algorithm>

#include "common.hpp"
#include "device.hpp"
#include "spmv_core.hpp"

namespace spx {

namespace {

template <int L, int BLOCK, bool NT>
__global__ __launch_bounds__(BLOCK) void k_spmv(int64_t n, const int32_t* __restrict__ rowptr,
                                                const int32_t* __restrict__ col,
                                                const double* __restrict__ val,
                                                const double* __restrict__ x,
                                                double* __restrict__ y, int remap) {
  constexpr int RPB = BLOCK / L;
  const int64_t b = remap ? xcd_logical_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
  const int64_t row = b * RPB + threadIdx.x / L;
  const int lane = threadIdx.x % L;
  if (row >= n) return;
  double s = row_partial<L, double, double, double, NT>(rowptr, col, val, x, row, lane);
  s = group_sum<L>(s);
  if (lane == 0) y[row] = s;
}

template <int BLOCK, int U, bool NT, bool VEC>
__global__ __launch_bounds__(BLOCK) void k_spmv_stream(int64_t n, const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ col,
                                                       const double* __restrict__ val,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ y, int rows,
                                                       int remap) {
  extern __shared__ __align__(16) char smem[];
  double* prod = reinterpret_cast<double*>(smem);
  const int64_t b = remap ? xcd_logical_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
  const int64_t r0 = b * rows;
  const int64_t r1 = r0 + rows < n ? r0 + rows : n;
  double s;
  if constexpr (VEC)
    s = stream_rows_v4<BLOCK, U, double, double, double, NT>(rowptr, col, val, x, r0, r1, prod);
  else
    s = stream_rows<BLOCK, U, double, double, double, NT>(rowptr, col, val, x, r0, r1, prod);
  if (threadIdx.x < r1 - r0) y[r0 + threadIdx.x] = s;
}

template <bool NT>
__global__ __launch_bounds__(kWinRows) void k_spmv_window(int64_t n, const int32_t* __restrict__ rowptr,
                                                          const int32_t* __restrict__ col,
                                                          const double* __restrict__ val,
                                                          const double* __restrict__ x,
                                                          double* __restrict__ y, WinView w,
                                                          int remap) {
  extern __shared__ __align__(16) char smem[];
  const int64_t b = remap ? xcd_logical_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
  const int64_t r0 = b * kWinRows;
  const int64_t r1 = r0 + kWinRows < n ? r0 + kWinRows : n;
  const double s =
      window_rows<kWinUProduct, win_v<double>(), kWinRows, double, double, double, NT, true>(
          rowptr, col, val, x, n, w, b, r0, r1, reinterpret_cast<double*>(smem));
  if (threadIdx.x < r1 - r0) y[r0 + threadIdx.x] = s;
}

__global__ void k_zero_i32(int32_t* p, int64_t count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = 0;
}

// One tile per workgroup, its columns and values staged by direct loads.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_spmv_dma(int64_t n, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ y, int rows, int remap,
                                                    int64_t tile) {
  extern __shared__ __align__(16) char smem[];
  const int64_t capc = (tile + 8 + 3) & ~int64_t(3);
  int32_t* lcol = reinterpret_cast<int32_t*>(smem);
  double* lval = reinterpret_cast<double*>(smem + 4 * capc);
  const int64_t b = remap ? xcd_logical_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
  const int64_t r0 = b * rows;
  const int64_t r1 = r0 + rows < n ? r0 + rows : n;
  const int32_t t0 = rowptr[r0], t1 = rowptr[r1];
  dma_issue<BLOCK, double>(col, val, t0, t1, lcol, lval);
  const bool owner = threadIdx.x < r1 - r0;
  int32_t rs = 0, re = 0;
  if (owner) {
    rs = rowptr[r0 + threadIdx.x];
    re = rowptr[r0 + threadIdx.x + 1];
  }
  dma_products<BLOCK, double, double, double>(x, t0, t1, lcol, lval);
  if (owner) y[r0 + threadIdx.x] = dma_row_sum<double, double>(lval, t0, rs, re);
}

// Largest entry count of any block of 32, 64, 128 and 256 consecutive rows.
__global__ void k_tile_nnz(const int32_t* __restrict__ rowptr, int64_t n, int32_t* __restrict__ out) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // index of a 32-row block
  const int64_t nb32 = (n + 31) / 32;
  if (b >= nb32) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t R = 32 << k;
    if ((b * 32) % R != 0) continue;
    const int64_t r0 = b * 32;
    const int64_t r1 = r0 + R < n ? r0 + R : n;
    atomicMax(&out[k], rowptr[r1] - rowptr[r0]);
  }
}

template <int L, bool NT>
int launch_vector_l(const Csr& A, const double* x, double* y, int remap, hipStream_t s) {
  constexpr int BLOCK = 256;
  constexpr int RPB = BLOCK / L;
  const int64_t nb = ceil_div(A.n, RPB);
  hipLaunchKernelGGL((k_spmv<L, BLOCK, NT>), dim3((unsigned)nb), dim3(BLOCK), 0, s, A.n, A.rowptr,
                     A.col, A.val, x, y, remap);
  return SPX_OK;
}

template <bool NT>
int launch_vector(const Csr& A, int lanes, const double* x, double* y, int remap, hipStream_t s) {
  switch (lanes) {
    case 1: return launch_vector_l<1, NT>(A, x, y, remap, s);
    case 2: return launch_vector_l<2, NT>(A, x, y, remap, s);
    case 4: return launch_vector_l<4, NT>(A, x, y, remap, s);
    case 8: return launch_vector_l<8, NT>(A, x, y, remap, s);
    case 16: return launch_vector_l<16, NT>(A, x, y, remap, s);
    case 32: return launch_vector_l<32, NT>(A, x, y, remap, s);
    case 64: return launch_vector_l<64, NT>(A, x, y, remap, s);
    default: return set_error(SPX_INVALID_ARG, "spmv: unsupported lane count %d", lanes);
  }
}

// Y[r, c] for c < nrhs; a group of G lanes per row, lane c owns column c
// (and c + G, ...).  The row's (value, column) pair is loaded once per lane
// group and the 8*G contiguous bytes of X per nonzero are one transaction;
// each lane keeps 8 such gathers in flight and adds them in entry order.
template <int G, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_spmm(int64_t n, const int32_t* __restrict__ rowptr,
                                                const int32_t* __restrict__ col,
                                                const double* __restrict__ val, int64_t nrhs,
                                                const double* __restrict__ X, int64_t ldx,
                                                double* __restrict__ Y, int64_t ldy, int remap) {
  constexpr int RPB = BLOCK / G;
  const int64_t b = remap ? xcd_logical_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
  const int64_t row = b * RPB + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (row >= n) return;
  const int32_t t0 = rowptr[row], t1 = rowptr[row + 1];
  constexpr int U = 8;  // independent gathers in flight per lane
  for (int64_t c0 = 0; c0 < nrhs; c0 += G) {
    const int64_t c = c0 + lane;
    double acc = 0.0;
    if (c < nrhs) {
      int32_t t = t0;
      for (; t + U <= t1; t += U) {
        double a[U], xv[U];
        int64_t cc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          a[u] = stream_load(val + t + u);
          cc[u] = stream_load(col + t + u);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = X[cc[u] * ldx + c];
#pragma unroll
        for (int u = 0; u < U; ++u) acc += a[u] * xv[u];
      }
      for (; t < t1; ++t) {
        const double a = stream_load(val + t);
        const int64_t cc = stream_load(col + t);
        acc += a * X[cc * ldx + c];
      }
      Y[row * ldy + c] = acc;
    }
  }
}

// The same product with each lane owning a pair of right-hand sides (c, c+1)
// read with one 16-byte load per entry, so a row of X takes G/2 lanes and a
// wave covers twice the rows per gather.  Needs X and Y 16-byte aligned and
// ldx, ldy even; an odd last column is read on its own.  Each column is
// accumulated in entry order exactly as in k_spmm, so the results are the
// same bits.  FULL: nrhs == ldx == ldy == 2 G (contiguous blocks, one pass,
// compile-time strides).
template <int G, int BLOCK, bool FULL>
__global__ __launch_bounds__(BLOCK) void k_spmm_pairs(int64_t n, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col,
                                                      const double* __restrict__ val, int64_t nrhs,
                                                      const double* __restrict__ X, int64_t ldx,
                                                      double* __restrict__ Y, int64_t ldy, int remap) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  constexpr int RPB = BLOCK / G;
  constexpr int U = 8;  // independent gathers in flight per lane
  const int64_t b = remap ? xcd_logical_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
  const int64_t row = b * RPB + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (row >= n) return;
  if constexpr (FULL) {
    ldx = ldy = nrhs = 2 * G;
  }
  const int32_t t0 = rowptr[row], t1 = rowptr[row + 1];
  for (int64_t c0 = 0; c0 < nrhs; c0 += 2 * G) {
    const int64_t c = c0 + 2 * lane;
    if (c >= nrhs) continue;
    if (FULL || c + 1 < nrhs) {
      d2 acc = {0.0, 0.0};
      int32_t t = t0;
      for (; t + U <= t1; t += U) {
        double a[U];
        int64_t cc[U];
        d2 xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          a[u] = stream_load(val + t + u);
          cc[u] = stream_load(col + t + u);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = *reinterpret_cast<const d2*>(X + cc[u] * ldx + c);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          acc.x += a[u] * xv[u].x;
          acc.y += a[u] * xv[u].y;
        }
      }
      for (; t < t1; ++t) {
        const double a = stream_load(val + t);
        const d2 xv = *reinterpret_cast<const d2*>(X + (int64_t)stream_load(col + t) * ldx + c);
        acc.x += a * xv.x;
        acc.y += a * xv.y;
      }
      *reinterpret_cast<d2*>(Y + row * ldy + c) = acc;
    } else {
      double acc = 0.0;
      int32_t t = t0;
      for (; t + U <= t1; t += U) {
        double a[U], xv[U];
        int64_t cc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          a[u] = stream_load(val + t + u);
          cc[u] = stream_load(col + t + u);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = X[cc[u] * ldx + c];
#pragma unroll
        for (int u = 0; u < U; ++u) acc += a[u] * xv[u];
      }
      for (; t < t1; ++t) acc += stream_load(val + t) * X[(int64_t)stream_load(col + t) * ldx + c];
      Y[row * ldy + c] = acc;
    }
  }
}

// The paired-column product for wide blocks of right-hand sides, with the
// block's run of (value, column) pairs staged in LDS first.  R = BLOCK / GP
// rows per block: the run of their entries is loaded once, coalesced,
// instead of once per lane of each row, and each lane then issues its X
// gathers U entries at a time with a predicated tail.  What bounds the
// kernel is the number of resident waves, not the gathers in flight per
// lane (2 to 8 per round measured the same at equal occupancy), so U is
// small and the register budget is held to 8 waves per SIMD.
// A block whose run exceeds CAP entries reads the pairs from global memory.
// Each column is accumulated in entry order as in k_spmm_pairs (same bits).
template <int GP, int BLOCK, bool FULL, int CAP>
__global__ __launch_bounds__(BLOCK, 8) void k_spmm_tile(int64_t n, const int32_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ val, int64_t nrhs,
                                                     const double* __restrict__ X, int64_t ldx,
                                                     double* __restrict__ Y, int64_t ldy) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  constexpr int R = BLOCK / GP;
  constexpr int U = 4;
  __shared__ double s_val[CAP];
  __shared__ int32_t s_col[CAP];
  if constexpr (FULL) {
    ldx = ldy = nrhs = 2 * GP;
  }
  const int64_t row0 = (int64_t)blockIdx.x * R;
  const int64_t rend = row0 + R < n ? row0 + R : n;
  const int64_t row = row0 + threadIdx.x / GP;
  const int lane = threadIdx.x % GP;
  // the row's bounds are read before the barrier (a clamped row past n)
  const int64_t rr = row < n ? row : n - 1;
  const int32_t t0 = rowptr[rr], t1 = rowptr[rr + 1];
  const int32_t e0 = rowptr[row0];
  const int32_t cnt = rowptr[rend] - e0;
  const bool staged = cnt <= CAP;
  if (staged) {
    for (int i = threadIdx.x; i < cnt; i += BLOCK) {
      s_val[i] = stream_load(val + e0 + i);
      s_col[i] = stream_load(col + e0 + i);
    }
  }
  __syncthreads();
  if (row >= n) return;
  auto pair_at = [&](int32_t t, double& a, int64_t& c) {
    if (staged) {
      a = s_val[t - e0];
      c = s_col[t - e0];
    } else {
      a = stream_load(val + t);
      c = stream_load(col + t);
    }
  };
  for (int64_t c0 = 0; c0 < nrhs; c0 += 2 * GP) {
    const int64_t c = c0 + 2 * lane;
    if (c >= nrhs) continue;
    if (FULL || c + 1 < nrhs) {
      d2 acc = {0.0, 0.0};
      for (int32_t t = t0; t < t1; t += U) {
        double a[U];
        d2 xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (t + u < t1) {
            int64_t cc;
            pair_at(t + u, a[u], cc);
            xv[u] = *reinterpret_cast<const d2*>(X + cc * ldx + c);
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (t + u < t1) {
            acc.x += a[u] * xv[u].x;
            acc.y += a[u] * xv[u].y;
          }
        }
      }
      *reinterpret_cast<d2*>(Y + row * ldy + c) = acc;
    } else {
      double acc = 0.0;
      for (int32_t t = t0; t < t1; t += U) {
        double a[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (t + u < t1) {
            int64_t cc;
            pair_at(t + u, a[u], cc);
            xv[u] = X[cc * ldx + c];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (t + u < t1) acc += a[u] * xv[u];
      }
      Y[row * ldy + c] = acc;
    }
  }
}

// Bandwidth references: the whole grid sweeps the array in lockstep, one
// 16-byte non-temporal access per lane per step (measured to be the
// pattern HBM serves best on this chip).
typedef double stream_dbl2 __attribute__((ext_vector_type(2)));
constexpr int kStreamBlocks = 2048;

__global__ __launch_bounds__(256) void k_stream_copy(const stream_dbl2* __restrict__ x,
                                                     stream_dbl2* __restrict__ y, int64_t n2,
                                                     const double* __restrict__ xs,
                                                     double* __restrict__ ys, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(x + i), y + i);
  if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) ys[n - 1] = xs[n - 1];
}

__global__ __launch_bounds__(256) void k_stream_sum(const stream_dbl2* __restrict__ x, int64_t n2,
                                                    const double* __restrict__ xs, int64_t n,
                                                    double* __restrict__ partials) {
  __shared__ double lds[4];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) {
    const stream_dbl2 v = __builtin_nontemporal_load(x + i);
    s += v.x + v.y;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) s += xs[n - 1];
  s = block_sum<256>(s, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// G[t] = -lam[row t] * u[col t] on the stored pattern.
template <int L, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_sddmm(int64_t n, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col,
                                                 const double* __restrict__ lam,
                                                 const double* __restrict__ u,
                                                 double* __restrict__ G) {
  constexpr int RPB = BLOCK / L;
  const int64_t row = (int64_t)blockIdx.x * RPB + threadIdx.x / L;
  const int lane = threadIdx.x % L;
  if (row >= n) return;
  const double nl = -lam[row];
  for (int32_t t = rowptr[row] + lane; t < rowptr[row + 1]; t += L) G[t] = nl * u[col[t]];
}

template <int L>
int launch_sddmm_l(const Csr& A, const double* lam, const double* u, double* G, hipStream_t s) {
  constexpr int BLOCK = 256;
  const int64_t nb = ceil_div(A.n, BLOCK / L);
  hipLaunchKernelGGL((k_sddmm<L, BLOCK>), dim3((unsigned)nb), dim3(BLOCK), 0, s, A.n, A.rowptr,
                     A.col, lam, u, G);
  return SPX_OK;
}

template <int G>
int launch_spmm_g(const Csr& A, int64_t nrhs, const double* X, int64_t ldx, double* Y,
                  int64_t ldy, hipStream_t s) {
  constexpr int BLOCK = 256;
  const bool pairs = G >= 2 && ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) &
                                15) == 0 && ldx % 2 == 0 && ldy % 2 == 0;
  if (pairs) {
    constexpr int GP = G >= 2 ? G / 2 : 1;  // a lane per pair of columns
    const int64_t nb = ceil_div(A.n, BLOCK / GP);
    if constexpr (G >= 8) {
      // staged runs: room for 32 entries per row on average (12 KB at 16
      // columns), plain block order (measured faster than the XCD order)
      constexpr int CAP = 32 * (BLOCK / GP);
      if (nrhs == G && ldx == G && ldy == G)
        hipLaunchKernelGGL((k_spmm_tile<GP, BLOCK, true, CAP>), dim3((unsigned)nb), dim3(BLOCK), 0, s,
                           A.n, A.rowptr, A.col, A.val, nrhs, X, ldx, Y, ldy);
      else
        hipLaunchKernelGGL((k_spmm_tile<GP, BLOCK, false, CAP>), dim3((unsigned)nb), dim3(BLOCK), 0,
                           s, A.n, A.rowptr, A.col, A.val, nrhs, X, ldx, Y, ldy);
      return SPX_OK;
    }
    if (nrhs == G && ldx == G && ldy == G)
      hipLaunchKernelGGL((k_spmm_pairs<GP, BLOCK, true>), dim3((unsigned)nb), dim3(BLOCK), 0, s, A.n,
                         A.rowptr, A.col, A.val, nrhs, X, ldx, Y, ldy, 1);
    else
      hipLaunchKernelGGL((k_spmm_pairs<GP, BLOCK, false>), dim3((unsigned)nb), dim3(BLOCK), 0, s,
                         A.n, A.rowptr, A.col, A.val, nrhs, X, ldx, Y, ldy, 1);
    return SPX_OK;
  }
  constexpr int RPB = BLOCK / G;
  const int64_t nb = ceil_div(A.n, RPB);
  hipLaunchKernelGGL((k_spmm<G, BLOCK>), dim3((unsigned)nb), dim3(BLOCK), 0, s, A.n, A.rowptr,
                     A.col, A.val, nrhs, X, ldx, Y, ldy, 1);
  return SPX_OK;
}

}  // namespace

int pick_lanes(const Csr& A, int opt) {
  if (opt > 0) return opt;
  const double mean = A.n > 0 ? (double)A.nnz / (double)A.n : 0.0;
  // smallest power of two that covers about half a mean row per lane
  int L = 1;
  while (L < 64 && 2.0 * L < mean) L <<= 1;
  return L;
}

int compute_tiles(Csr& A, hipStream_t s) {
  int32_t* d = nullptr;
  SPX_TRY(dalloc_n(&d, 4));
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, d, (int64_t)4);
  const int64_t nb32 = ceil_div(A.n, 32);
  if (nb32 > 0)
    hipLaunchKernelGGL(k_tile_nnz, dim3((unsigned)ceil_div(nb32, 256)), dim3(256), 0, s, A.rowptr,
                       A.n, d);
  int32_t hostv[4] = {0, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(hostv, d, sizeof(hostv), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dfree(d);
  if (e != hipSuccess) return set_error(SPX_HIP_ERROR, "tile sizes: %s", hipGetErrorString(e));
  for (int k = 0; k < 4; ++k) A.tile_nnz[k] = hostv[k];
  return SPX_OK;
}

namespace {
constexpr size_t kStreamLdsCap = 40 * 1024;  // keeps >= 3 workgroups per CU
constexpr size_t kStreamLdsMax = 64 * 1024;
int rows_index(int rows) { return rows == 32 ? 0 : rows == 64 ? 1 : rows == 128 ? 2 : 3; }
}  // namespace

namespace {
// The window walk's shape when A has a window index and the options leave
// the choice to the library (or ask for it).  Left to itself the library
// takes it for patterns with enough 256-row tiles per compute unit (below
// that the stream walk's smaller tiles fill the chip better): 12 when rows
// average more than 16 entries, 7 for shorter rows, whose gather costs the
// stream walk more; and whose rows average at most 64 entries in every tile
// (one thread adds each row).  It needs no tile in LDS, so it also takes
// patterns whose tiles exceed the stream walk's limit.
// MatMult's own kernel (one tile per workgroup, a tile's loads issued
// together) gains from the window walk from fewer tiles: 2.5 per compute
// unit (measured crossover between 1.7 and 2.7 on 27-point patterns, about
// 2 on 9-point ones).
constexpr int64_t kWinAutoTilesPerCu = 12;
constexpr int64_t kWinAutoTilesPerCuShortRows = 7;
constexpr int64_t kWinAutoHalfTilesPerCuMatMult = 5;
bool window_shape(const spx_matrix* h, const Csr& A, bool allow, bool matmult, SpmvShape& sh) {
  if (!allow || !A.win.lcol) return false;
  const int want = h ? h->variant_opt : 0;
  const bool tuned = h && (h->rows_opt || h->vec_opt || h->pipe_opt);
  const int64_t per_cu = A.nnz <= 16 * A.n ? kWinAutoTilesPerCuShortRows : kWinAutoTilesPerCu;
  const int64_t tiles = ceil_div(A.n, kWinRows);
  const bool large = matmult ? 2 * tiles >= kWinAutoHalfTilesPerCuMatMult * cu_count()
                             : tiles >= per_cu * cu_count();
  if (want == kVariantWindow || (want == kVariantAuto && !tuned && large &&
                                 A.tile_nnz[3] <= 64 * (int64_t)kWinRows)) {
    sh.variant = kVariantWindow;
    sh.rows = kWinRows;
    sh.tile = A.win.max_blocks * kWinBlock;
    // the fp64 solver kernels' LDS (the fp32 ones compute theirs from tile)
    sh.lds = window_lds_bytes(A.win.max_blocks, sizeof(double),
                              win_u_solver<double>() * win_v<double>());
    return true;
  }
  return false;
}
}  // namespace

SpmvShape spmv_shape(const spx_matrix* h, const Csr& A) { return spmv_shape_for(h, A, true); }

SpmvShape matmult_shape(const spx_matrix* h, const Csr& A) {
  return spmv_shape_for(h, A, true, true);
}

SpmvShape spmv_shape_for(const spx_matrix* h, const Csr& A, bool allow_window, bool matmult) {
  SpmvShape sh;
  sh.lanes = pick_lanes(A, h ? h->lanes_opt : 0);
  sh.nt = h ? h->nt_opt : 1;
  sh.vec = h ? h->vec_opt : 0;
  sh.pipe = 0;
  sh.rows = 0;
  sh.lds = 0;
  sh.variant = kVariantVector;
  sh.tile = 0;
  const int want = h ? h->variant_opt : 0;
  if (want == kVariantVector) return sh;
  if (window_shape(h, A, allow_window, matmult, sh)) return sh;
  const int rows_opt = h ? h->rows_opt : 0;
  if (want == kVariantDma) {
    // two staging buffers per workgroup in the solver kernels
    for (int rows : {64, 32, 128, 256}) {
      if (rows_opt && rows != rows_opt) continue;
      const int64_t tile = A.tile_nnz[rows_index(rows)];
      if (2 * dma_buffer_bytes(tile, sizeof(double)) + 64 <= kStreamLdsMax) {
        sh.variant = kVariantDma;
        sh.rows = rows;
        sh.tile = tile;
        sh.lds = dma_buffer_bytes(tile, sizeof(double));
        return sh;
      }
    }
    return sh;
  }
  if (rows_opt) {
    const size_t lds = (size_t)(A.tile_nnz[rows_index(rows_opt)] + 8) * sizeof(double);
    if (lds <= kStreamLdsMax) {
      sh.variant = kVariantStream;
      sh.rows = rows_opt;
      sh.lds = lds;
      sh.tile = A.tile_nnz[rows_index(rows_opt)];
    }
    return sh;
  }
  // Automatic: stream when some row count keeps the tile small and rows
  // are not much longer than 64 entries on average.
  for (int rows : {64, 128, 32, 256}) {
    const int64_t tile = A.tile_nnz[rows_index(rows)];
    const size_t lds = (size_t)(tile + 8) * sizeof(double);
    if (lds <= kStreamLdsCap && tile <= 64 * (int64_t)rows) {
      sh.variant = kVariantStream;
      sh.rows = rows;
      sh.lds = lds;
      sh.tile = tile;
      return sh;
    }
  }
  if (want == kVariantStream) {
    const size_t lds = (size_t)(A.tile_nnz[0] + 8) * sizeof(double);
    if (lds <= kStreamLdsMax) {
      sh.variant = kVariantStream;
      sh.rows = 32;
      sh.lds = lds;
      sh.tile = A.tile_nnz[0];
    }
  }
  return sh;
}

namespace {
// The pipelined walk holds a whole tile in registers.
void set_pipe(const spx_matrix* h, const Csr& A, SpmvShape& sh) {
  sh.pipe = 0;
  if (!(h ? h->pipe_opt : 0) || sh.variant != kVariantStream || sh.vec) return;
  const int64_t tile = A.tile_nnz[rows_index(sh.rows)];
  if (tile <= 256 * 8)
    sh.pipe = 8;
  else if (tile <= 256 * 16)
    sh.pipe = 16;
}
}  // namespace

// Shape of the fp32 copy (mixed-precision inner solve): fp32 products take
// half the LDS, so the tile doubles when it still fits.
SpmvShape spmv_shape32(const spx_matrix* h, const Csr& A) {
  SpmvShape sh = spmv_shape_for(h, A, !(h && h->rows32_opt));
  if (sh.variant == kVariantWindow) return sh;
  if (sh.variant == kVariantDma) {
    const int want = h && h->rows32_opt ? h->rows32_opt : sh.rows;
    const int64_t tile = A.tile_nnz[rows_index(want)];
    if (2 * dma_buffer_bytes(tile, sizeof(float)) + 64 <= kStreamLdsMax) {
      sh.rows = want;
      sh.tile = tile;
    }
    return sh;
  }
  if (sh.variant != kVariantStream) return sh;
  int want = h && h->rows32_opt ? h->rows32_opt : (h && h->rows_opt ? h->rows_opt : 2 * sh.rows);
  if (want > 256) want = 256;
  const size_t lds = (size_t)(A.tile_nnz[rows_index(want)] + 8) * sizeof(double);
  if (lds / 2 <= kStreamLdsMax) {
    sh.rows = want;
    sh.lds = lds;
    sh.tile = A.tile_nnz[rows_index(want)];
  }
  set_pipe(h, A, sh);
  return sh;
}

SpmvShape solver_shape(const spx_matrix* h, const Csr& A) {
  SpmvShape sh = spmv_shape(h, A);
  set_pipe(h, A, sh);
  return sh;
}

int launch_spmv(const Csr& A, const SpmvShape& sh, const double* x, double* y, int remap,
                hipStream_t s) {
  if (A.n == 0) return SPX_OK;
  if (sh.variant == kVariantWindow) {
    const int64_t nb = ceil_div(A.n, kWinRows);
    const size_t lds =
        window_lds_bytes(A.win.max_blocks, sizeof(double), kWinUProduct * win_v<double>());
    if (sh.nt)
      hipLaunchKernelGGL(k_spmv_window<true>, dim3((unsigned)nb), dim3(kWinRows), lds, s, A.n,
                         A.rowptr, A.col, A.val, x, y, win_view(A), remap);
    else
      hipLaunchKernelGGL(k_spmv_window<false>, dim3((unsigned)nb), dim3(kWinRows), lds, s, A.n,
                         A.rowptr, A.col, A.val, x, y, win_view(A), remap);
    return SPX_OK;
  }
  if (sh.variant == kVariantDma) {
    const int64_t nb = ceil_div(A.n, sh.rows);
    hipLaunchKernelGGL((k_spmv_dma<256>), dim3((unsigned)nb), dim3(256),
                       dma_buffer_bytes(sh.tile, sizeof(double)), s, A.n, A.rowptr, A.col, A.val,
                       x, y, sh.rows, remap, sh.tile);
    return SPX_OK;
  }
  if (sh.variant == kVariantStream) {
    const int64_t nb = ceil_div(A.n, sh.rows);
    const size_t lds = sh.lds > 0 ? sh.lds : 16;
#define SPX_STREAM_LAUNCH(NT, VEC, U)                                                        \
  hipLaunchKernelGGL((k_spmv_stream<256, U, NT, VEC>), dim3((unsigned)nb), dim3(256), lds, s, A.n, \
                     A.rowptr, A.col, A.val, x, y, sh.rows, remap)
    if (sh.vec) {
      if (sh.nt)
        SPX_STREAM_LAUNCH(true, true, 2);
      else
        SPX_STREAM_LAUNCH(false, true, 2);
    } else {
      if (sh.nt)
        SPX_STREAM_LAUNCH(true, false, 8);
      else
        SPX_STREAM_LAUNCH(false, false, 8);
    }
#undef SPX_STREAM_LAUNCH
    return SPX_OK;
  }
  return sh.nt ? launch_vector<true>(A, sh.lanes, x, y, remap, s)
               : launch_vector<false>(A, sh.lanes, x, y, remap, s);
}

int launch_spmm(const Csr& A, int64_t nrhs, const double* X, int64_t ldx, double* Y, int64_t ldy,
                hipStream_t s) {
  if (A.n == 0 || nrhs == 0) return SPX_OK;
  if (nrhs <= 4) return launch_spmm_g<4>(A, nrhs, X, ldx, Y, ldy, s);
  if (nrhs <= 8) return launch_spmm_g<8>(A, nrhs, X, ldx, Y, ldy, s);
  if (nrhs <= 16) return launch_spmm_g<16>(A, nrhs, X, ldx, Y, ldy, s);
  if (nrhs <= 32) return launch_spmm_g<32>(A, nrhs, X, ldx, Y, ldy, s);
  return launch_spmm_g<64>(A, nrhs, X, ldx, Y, ldy, s);
}

}  // namespace spx

using namespace spx;

extern "C" int spx_matmult(spx_handle h, const double* x, double* y, void* stream) {
  clear_error();
  if (!h || !x || !y) return set_error(SPX_INVALID_ARG, "matmult: NULL argument");
  if (x == y) return set_error(SPX_INVALID_ARG, "matmult: x and y must not alias");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const SpmvShape sh = matmult_shape(h, h->A);
  SPX_TRY(launch_spmv(h->A, sh, x, y, remap_for(h, sh), s));
  SPX_CHECK_HIP(hipGetLastError());
  return SPX_OK;
}

extern "C" int spx_matmult_transpose(spx_handle h, const double* x, double* y, void* stream) {
  clear_error();
  if (!h || !x || !y) return set_error(SPX_INVALID_ARG, "matmult_transpose: NULL argument");
  if (x == y) return set_error(SPX_INVALID_ARG, "matmult_transpose: x and y must not alias");
  hipStream_t s = static_cast<hipStream_t>(stream);
  SPX_TRY(ensure_transpose(h, s));
  const SpmvShape sh = matmult_shape(h, h->At);
  SPX_TRY(launch_spmv(h->At, sh, x, y, remap_for(h, sh), s));
  SPX_CHECK_HIP(hipGetLastError());
  return SPX_OK;
}

extern "C" int spx_sddmm(spx_handle h, const double* lam, const double* u, double* G,
                         void* stream) {
  clear_error();
  if (!h || !lam || !u || (h->A.nnz > 0 && !G))
    return set_error(SPX_INVALID_ARG, "sddmm: NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int L = pick_lanes(h->A, h->lanes_opt);
  int st;
  switch (L) {
    case 1: st = launch_sddmm_l<1>(h->A, lam, u, G, s); break;
    case 2: st = launch_sddmm_l<2>(h->A, lam, u, G, s); break;
    case 4: st = launch_sddmm_l<4>(h->A, lam, u, G, s); break;
    case 8: st = launch_sddmm_l<8>(h->A, lam, u, G, s); break;
    case 16: st = launch_sddmm_l<16>(h->A, lam, u, G, s); break;
    case 32: st = launch_sddmm_l<32>(h->A, lam, u, G, s); break;
    default: st = launch_sddmm_l<64>(h->A, lam, u, G, s); break;
  }
  SPX_TRY(st);
  SPX_CHECK_HIP(hipGetLastError());
  return SPX_OK;
}

extern "C" int spx_spmm(spx_handle h, int64_t nrhs, const double* X, int64_t ldx, double* Y,
                        int64_t ldy, void* stream) {
  clear_error();
  if (!h || nrhs < 0 || (nrhs > 0 && (!X || !Y)) || ldx < nrhs || ldy < nrhs)
    return set_error(SPX_INVALID_ARG, "spmm: bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // 16 contiguous, 16-byte aligned columns: each tile's rows of X staged in
  // LDS (spmm.hip), the index built on the first call
  const bool rowset = nrhs == 16 && ldx == 16 && ldy == 16 &&
                      ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) & 15) == 0;
  if (rowset) {
    SPX_TRY(build_rowset(h->A, h->spmm_rows_opt ? h->spmm_rows_opt : 32, s));
    SPX_TRY(launch_spmm_rowset(h->A, X, Y, s));
  } else {
    SPX_TRY(launch_spmm(h->A, nrhs, X, ldx, Y, ldy, s));
  }
  SPX_CHECK_HIP(hipGetLastError());
  return SPX_OK;
}

extern "C" int spx_stream_copy(const double* x, double* y, int64_t n, void* stream) {
  clear_error();
  if (n < 0 || (n > 0 && (!x || !y))) return set_error(SPX_INVALID_ARG, "stream_copy: bad argument");
  if (((uintptr_t)x | (uintptr_t)y) & 15)
    return set_error(SPX_INVALID_ARG, "stream_copy: x and y must be 16-byte aligned");
  if (n == 0) return SPX_OK;
  hipLaunchKernelGGL(k_stream_copy, dim3(kStreamBlocks), dim3(256), 0,
                     static_cast<hipStream_t>(stream), reinterpret_cast<const stream_dbl2*>(x),
                     reinterpret_cast<stream_dbl2*>(y), n / 2, x, y, n);
  SPX_CHECK_HIP(hipGetLastError());
  return SPX_OK;
}

extern "C" int spx_stream_sum(const double* x, int64_t n, double* partials, void* stream) {
  clear_error();
  if (n < 0 || !partials || (n > 0 && !x)) return set_error(SPX_INVALID_ARG, "stream_sum: bad argument");
  if ((uintptr_t)x & 15) return set_error(SPX_INVALID_ARG, "stream_sum: x must be 16-byte aligned");
  hipLaunchKernelGGL(k_stream_sum, dim3(kStreamBlocks), dim3(256), 0,
                     static_cast<hipStream_t>(stream), reinterpret_cast<const stream_dbl2*>(x), n / 2,
                     x, n, partials);
  SPX_CHECK_HIP(hipGetLastError());
  return SPX_OK;
}
