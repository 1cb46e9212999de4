// Limited-memory BFGS product p = H_k g in the paper's intermediate dense
// form (Sec. 8, dense reformulations):
//   H_k g = [I, -S R^-T] [I 0; Y^T I] diag(H0, D) [I Y; 0 I] [I; -R^-1 S^T] g
// with R = triu(S^T Y), D = diag(S^T Y) and a diagonal base operator H0
// that may change from call to call.  Evaluated right to left:
//   c = -R^-1 (S^T g);  a = h0 (g + Y c);  f = Y^T a + D c;  e = R^-T f;
//   p = a - S e.
//
// Design for gfx950.  The history is a ring of m column slots, S and Y
// column-major (slot j's pair contiguous at j*n), so every pass walks rows
// with coalesced loads of each column and a new pair overwrites one column
// with contiguous stores.  The m x m matrix of pair products s_a.y_b is kept
// by slot; R = triu(S^T Y) in time order only ever reads s_a.y_b with pair a
// no newer than pair b, so an update fills the new slot's column
// (s_b.y_new for every held b, the diagonal included) from one pass over S
// and never reads Y.  One apply is three passes over the rows (S^T g; then
// a and Y^T a in one pass over Y, long histories staging row blocks of Y
// in LDS; then p from S), separated by the two reductions the formula needs; each
// pass kernel re-adds the per-workgroup partials of the previous one, so
// no workgroup waits for another and no fence is needed.  The two m x m
// triangular solves are done by every workgroup of the pass that needs
// their result (m <= 64: a few thousand flops from L2).
#include <algorithm>
#include <cmath>
#include <new>

#include "common.hpp"
#include "device.hpp"
#include "solver_core.hpp"

struct spx_lbfgs {
  int device = 0;
  int64_t n = 0;
  int m = 0;
  int count = 0;  // pairs held
  int start = 0;  // slot of the oldest pair
  int G = 0;      // workgroups of the pass kernels
  int Gy = 0;     // workgroups of the staged a / Y^T a pass (long histories)
  double* S = nullptr;
  double* Y = nullptr;
  double* SY = nullptr;  // SY[a*m + b] = s_a . y_b, by slot
  double* P = nullptr;   // partials [2m][G]
  double* red = nullptr; // reduced vectors: q[m] | c[m] | f[m] | e[m] | spare
  double* a = nullptr;   // n
};

namespace spx {
namespace {

using namespace solver;

constexpr int kMaxHistory = 64;
constexpr int kLB = 256;
constexpr int kJB = 8;      // columns per unrolled step of the row passes
constexpr int kJT = 16;     // columns per accumulator chunk of the transposed products
constexpr int kFused = 16;  // up to this many pairs, a and Y^T a share one pass
// The transposed products hold their registers to 8 waves per SIMD (they
// stream the history; resident waves, not loads in flight per wave, set
// their rate: 0.72 vs 0.76 ms for 50 columns of 10^7 rows).
constexpr int kGemvtWaves = 8;

// Rows are walked V at a time (V = 2: 16-byte loads of every column and
// vector, taken when n is even and the caller's vectors are 16-byte
// aligned; otherwise V = 1).
template <int V>
struct Vd;
template <>
struct Vd<1> {
  typedef double type;
};
template <>
struct Vd<2> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <int V>
__device__ __forceinline__ typename Vd<V>::type ldv(const double* p) {
  return *reinterpret_cast<const typename Vd<V>::type*>(p);
}
template <int V>
__device__ __forceinline__ double el(const typename Vd<V>::type& v, int j) {
  if constexpr (V == 1)
    return v;
  else
    return v[j];
}

// The ring: logical pair b (oldest first) lives in slot start + b (mod m).
struct Ring {
  int m, start, cnt;
  __device__ __forceinline__ int64_t slot(int b) const {
    const int s = start + b;
    return s >= m ? s - m : s;
  }
};

// Row range of workgroup b of G over n rows (contiguous, balanced), with
// both ends multiples of V (n is a multiple of V).
template <int V>
__device__ __forceinline__ void rows_of(int64_t n, int b, int G, int64_t* lo, int64_t* hi) {
  *lo = (n * b / G) & ~(int64_t)(V - 1);
  *hi = (n * (b + 1) / G) & ~(int64_t)(V - 1);
}

// Workgroup sums of the first cnt of NA per-thread accumulators; the totals
// land in out[0..cnt).
template <int NA>
__device__ __forceinline__ void block_sums(const double (&acc)[NA], int cnt, double* lds,
                                           double* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    if (j < cnt) {
      const double v = wave_sum(acc[j]);
      if (lane == 0) lds[w * NA + j] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < cnt) {
    double s = 0.0;
    for (int q = 0; q < kLB / 64; ++q) s += lds[q * NA + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Partials of d_b = sum_i col_b[i] w[i] over the workgroup's rows, for the
// ring's cnt columns, into P[(row0 + b) * G + workgroup].  Columns go in
// chunks of kJT accumulators (each element of the history read once; w
// re-read per chunk, from cache).
template <int V>
__device__ __forceinline__ void gemvt_partials(int64_t n, const double* __restrict__ base,
                                               Ring R, const double* __restrict__ w,
                                               double* __restrict__ P, int row0, double* lds,
                                               double* tot) {
  typedef typename Vd<V>::type VD;
  int64_t lo, hi;
  rows_of<V>(n, blockIdx.x, gridDim.x, &lo, &hi);
  for (int jb = 0; jb < R.cnt; jb += kJT) {
    const int nc = R.cnt - jb < kJT ? R.cnt - jb : kJT;
    const double* cp[kJT];
#pragma unroll
    for (int u = 0; u < kJT; ++u) cp[u] = base + (u < nc ? R.slot(jb + u) : 0) * n;
    double acc[kJT];
#pragma unroll
    for (int u = 0; u < kJT; ++u) acc[u] = 0.0;
    for (int64_t i = lo + V * (int64_t)threadIdx.x; i < hi; i += V * kLB) {
      const VD wv = ldv<V>(w + i);
#pragma unroll
      for (int u = 0; u < kJT; ++u)
        if (u < nc) {
          const VD c = ldv<V>(cp[u] + i);
#pragma unroll
          for (int j = 0; j < V; ++j) acc[u] += el<V>(c, j) * el<V>(wv, j);
        }
    }
    block_sums<kJT>(acc, nc, lds, tot);
    if (threadIdx.x < nc)
      P[(int64_t)(row0 + jb + threadIdx.x) * gridDim.x + blockIdx.x] = tot[threadIdx.x];
  }
}

// Partials of d_b = col_b . w1 (into row row1 + b of P) and e_b = col_b . w2
// (row row2 + b) in one pass over the columns: half as many columns per
// chunk, two accumulators each.  Every column's products are added in the
// same per-thread row order as in gemvt_partials, so each total has the
// bits of the single-vector pass.
constexpr int kJT2 = kJT / 2;
template <int V>
__device__ __forceinline__ void gemvt2_partials(int64_t n, const double* __restrict__ base,
                                                Ring R, const double* __restrict__ w1,
                                                const double* __restrict__ w2,
                                                double* __restrict__ P, int row1, int row2,
                                                double* lds, double* tot) {
  typedef typename Vd<V>::type VD;
  int64_t lo, hi;
  rows_of<V>(n, blockIdx.x, gridDim.x, &lo, &hi);
  for (int jb = 0; jb < R.cnt; jb += kJT2) {
    const int nc = R.cnt - jb < kJT2 ? R.cnt - jb : kJT2;
    const double* cp[kJT2];
#pragma unroll
    for (int u = 0; u < kJT2; ++u) cp[u] = base + (u < nc ? R.slot(jb + u) : 0) * n;
    double acc[kJT2], acc2[kJT2];
#pragma unroll
    for (int u = 0; u < kJT2; ++u) acc[u] = acc2[u] = 0.0;
    for (int64_t i = lo + V * (int64_t)threadIdx.x; i < hi; i += V * kLB) {
      const VD wv = ldv<V>(w1 + i);
      const VD wv2 = ldv<V>(w2 + i);
#pragma unroll
      for (int u = 0; u < kJT2; ++u)
        if (u < nc) {
          const VD c = ldv<V>(cp[u] + i);
#pragma unroll
          for (int j = 0; j < V; ++j) {
            acc[u] += el<V>(c, j) * el<V>(wv, j);
            acc2[u] += el<V>(c, j) * el<V>(wv2, j);
          }
        }
    }
    block_sums<kJT2>(acc, nc, lds, tot);
    if (threadIdx.x < nc)
      P[(int64_t)(row1 + jb + threadIdx.x) * gridDim.x + blockIdx.x] = tot[threadIdx.x];
    block_sums<kJT2>(acc2, nc, lds, tot);
    if (threadIdx.x < nc)
      P[(int64_t)(row2 + jb + threadIdx.x) * gridDim.x + blockIdx.x] = tot[threadIdx.x];
  }
}

// The row passes t_i = init_i + sign * sum_j col_j[i] coef_j over the
// workgroup's rows, then out_i = fin(i, t_i).  Rows go in blocks of
// kRowSteps steps of V * kLB: each thread keeps its kRowSteps values in
// registers while the columns go past kJB at a time, so every column is
// read as one contiguous stretch per block rather than all columns at once
// per row step (the fused step at m = 50, n = 10^7: 4.28 to 4.21 ms; two
// steps per block keep 47-54 VGPRs, four spill at 8 waves per SIMD).  Each
// row sees the same operations in the same order as the plain loop
// (t = init; for each column in order: t += or -= col * coef).
constexpr int kRowSteps = 2;
template <int V, bool SUB, typename Init, typename Fin>
__device__ __forceinline__ void row_blocks(int64_t n, const double* __restrict__ base, Ring R,
                                           const double* coef, Init init, Fin fin) {
  typedef typename Vd<V>::type VD;
  constexpr int64_t STEP = V * kLB;
  int64_t lo, hi;
  rows_of<V>(n, blockIdx.x, gridDim.x, &lo, &hi);
  const int cnt = R.cnt;
  for (int64_t b0 = lo; b0 < hi; b0 += STEP * kRowSteps) {
    VD t[kRowSteps];
#pragma unroll
    for (int r = 0; r < kRowSteps; ++r) {
      const int64_t i = b0 + STEP * r + V * (int64_t)threadIdx.x;
      if (i < hi) t[r] = init(i);
    }
    for (int jb = 0; jb < cnt; jb += kJB) {
      const int nc = cnt - jb < kJB ? cnt - jb : kJB;
      const double* cp[kJB];
      double e[kJB];
#pragma unroll
      for (int u = 0; u < kJB; ++u) {
        cp[u] = base + (u < nc ? R.slot(jb + u) : 0) * n;
        e[u] = u < nc ? coef[jb + u] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < kRowSteps; ++r) {
        const int64_t i = b0 + STEP * r + V * (int64_t)threadIdx.x;
        if (i < hi) {
#pragma unroll
          for (int u = 0; u < kJB; ++u)
            if (u < nc) {
              if constexpr (SUB)
                t[r] -= ldv<V>(cp[u] + i) * e[u];
              else
                t[r] += ldv<V>(cp[u] + i) * e[u];
            }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kRowSteps; ++r) {
      const int64_t i = b0 + STEP * r + V * (int64_t)threadIdx.x;
      if (i < hi) fin(i, t[r]);
    }
  }
}

// ---------------------------------------------------------------- update
__global__ void k_lb_put(int64_t n, const double* __restrict__ s, const double* __restrict__ y,
                         double* __restrict__ Snew, double* __restrict__ Ynew) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    Snew[i] = s[i];
    Ynew[i] = y[i];
  }
}

// Partials of v_b = s_b . y_new (rows kMaxHistory + b) for every held pair,
// the new one (already in its slot, logical cnt - 1) included.
template <int V>
__global__ __launch_bounds__(kLB, kGemvtWaves) void k_lb_update(int64_t n, const double* __restrict__ S,
                                                   const double* __restrict__ Y, Ring R,
                                                   double* __restrict__ P) {
  __shared__ double lds[(kLB / 64) * kJT];
  __shared__ double tot[kJT];
  const int64_t cur = R.slot(R.cnt - 1) * n;
  gemvt_partials<V>(n, S, R, Y + cur, P, kMaxHistory, lds, tot);
}

// The update's pass with the apply's first one folded in: the pass over S
// also takes the partials of q_b = s_b . g (rows 2 kMaxHistory + b).
template <int V>
__global__ __launch_bounds__(kLB, kGemvtWaves) void k_lb_update_g(int64_t n, const double* __restrict__ S,
                                                     const double* __restrict__ Y, Ring R,
                                                     const double* __restrict__ g,
                                                     double* __restrict__ P) {
  __shared__ double lds[(kLB / 64) * kJT];
  __shared__ double tot[kJT];
  const int64_t cur = R.slot(R.cnt - 1) * n;
  gemvt2_partials<V>(n, S, R, Y + cur, g, P, kMaxHistory, 2 * kMaxHistory, lds, tot);
}

// one workgroup per logical index b: SY column of the new slot, s_b . y_new
__global__ __launch_bounds__(kLB) void k_lb_update_finish(const double* __restrict__ P, int G,
                                                          Ring R, int slot,
                                                          double* __restrict__ SY) {
  __shared__ double lds[kLds];
  const int b = blockIdx.x;
  const double t = reduce_all(P + (int64_t)(kMaxHistory + b) * G, G, lds);
  if (threadIdx.x == 0) SY[R.slot(b) * R.m + slot] = t;
}

// ----------------------------------------------------------------- apply
// pass 1: partials of q_b = s_b . g
template <int V>
__global__ __launch_bounds__(kLB, kGemvtWaves) void k_lb_sg(int64_t n, const double* __restrict__ S, Ring R,
                                               const double* __restrict__ g,
                                               double* __restrict__ P) {
  __shared__ double lds[(kLB / 64) * kJT];
  __shared__ double tot[kJT];
  gemvt_partials<V>(n, S, R, g, P, 0, lds, tot);
}

// one workgroup per logical index: out[b] = sum of the G partials of b
__global__ __launch_bounds__(kLB) void k_lb_reduce(const double* __restrict__ P, int G,
                                                   double* __restrict__ out) {
  __shared__ double lds[kLds];
  const double t = reduce_all(P + (int64_t)blockIdx.x * G, G, lds);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// R_ab (a <= b, logical) = s_a . y_b
__device__ __forceinline__ double rmat(const double* SY, const Ring& R, int a, int b) {
  return SY[R.slot(a) * R.m + R.slot(b)];
}

// The two triangular solves of the apply, R = triu(S^T Y) in the ring's
// logical order: c = -R^-1 q (WHICH 0, into red[m..]) after the first
// pass, e = R^-T (f + D c) (WHICH 1, into red[3m..]) after the second.
// One workgroup stages R in LDS, then one wave sweeps the columns: lane x
// holds row x's running sum, and at step y every lane takes the finished
// unknown y by a shuffle and lanes still open subtract their entry of
// column y times it (cnt <= 64 lanes).
template <int WHICH>
__global__ __launch_bounds__(kLB) void k_lb_solve(const double* __restrict__ SY, Ring R,
                                                  double* __restrict__ red) {
  __shared__ double rl[kMaxHistory * kMaxHistory];
  const int cnt = R.cnt;
  for (int i = threadIdx.x; i < cnt * cnt; i += kLB) {
    const int a = i / cnt, b = i % cnt;
    rl[i] = a <= b ? rmat(SY, R, a, b) : 0.0;
  }
  __syncthreads();
  if (threadIdx.x >= 64) return;
  const int x = threadIdx.x;
  double out = 0.0;
  if constexpr (WHICH == 0) {
    double t = x < cnt ? -red[x] : 0.0;
    for (int y = cnt - 1; y >= 0; --y) {
      const double uy = __shfl(t, y, 64) / rl[y * cnt + y];
      if (x == y) out = uy;
      if (x < y) t -= rl[x * cnt + y] * uy;
    }
    if (x < cnt) red[kMaxHistory + x] = out;
  } else {
    const double* c = red + kMaxHistory;
    const double* f = red + 2 * kMaxHistory;
    double t = x < cnt ? f[x] + rl[x * cnt + x] * c[x] : 0.0;
    for (int y = 0; y < cnt; ++y) {
      const double uy = __shfl(t, y, 64) / rl[y * cnt + y];
      if (x == y) out = uy;
      if (x > y) t -= rl[y * cnt + x] * uy;
    }
    if (x < cnt) red[3 * kMaxHistory + x] = out;
  }
}

// pass 2 for histories of at most kFused pairs: a = h0 (g + Y c) with c
// from red[m..], and the partials of f_b = y_b . a, each row's history
// values held in registers
template <int V>
__global__ __launch_bounds__(kLB, 1) void k_lb_ya(int64_t n, const double* __restrict__ Y, Ring R,
                                               const double* __restrict__ g,
                                               const double* __restrict__ h0,
                                               const double* __restrict__ SY,
                                               double* __restrict__ red,
                                               double* __restrict__ a_out,
                                               double* __restrict__ P) {
  typedef typename Vd<V>::type VD;
  __shared__ double lds[(kLB / 64) * kFused];
  __shared__ double tot[kFused];
  __shared__ double cs[kMaxHistory];
  const int cnt = R.cnt;
  if (threadIdx.x < cnt) cs[threadIdx.x] = red[kMaxHistory + threadIdx.x];
  __syncthreads();
  int64_t lo, hi;
  rows_of<V>(n, blockIdx.x, gridDim.x, &lo, &hi);
  {
    const double* cp[kFused];
    double c[kFused], f[kFused];
#pragma unroll
    for (int b = 0; b < kFused; ++b) {
      cp[b] = Y + (b < cnt ? R.slot(b) : 0) * n;
      c[b] = b < cnt ? cs[b] : 0.0;
      f[b] = 0.0;
    }
    for (int64_t i = lo + V * (int64_t)threadIdx.x; i < hi; i += V * kLB) {
      VD yv[kFused];
      VD t = ldv<V>(g + i);
#pragma unroll
      for (int b = 0; b < kFused; ++b)
        if (b < cnt) {
          yv[b] = ldv<V>(cp[b] + i);
          t += yv[b] * c[b];
        }
      const VD ai = h0 ? ldv<V>(h0 + i) * t : t;
      *reinterpret_cast<VD*>(a_out + i) = ai;
#pragma unroll
      for (int b = 0; b < kFused; ++b)
        if (b < cnt) {
#pragma unroll
          for (int j = 0; j < V; ++j) f[b] += el<V>(yv[b], j) * el<V>(ai, j);
        }
    }
    block_sums<kFused>(f, cnt, lds, tot);
    if (threadIdx.x < cnt) P[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = tot[threadIdx.x];
  }
}

// pass 2 for histories longer than kFused: a and the partials of
// f_b = y_b . a from ONE pass over Y.  Each block of kYRows rows
// is staged in LDS (kYRows x cnt, column stride kYRows + 1 so that the
// column-wise reads below hit distinct banks): thread r < kYRows forms
// a_r = h0_r (g_r + sum_b y_b[r] c_b) with the columns in order (its g_r
// and h0_r loaded with the block's elements of Y); then
// thread t adds y_b[r] a_r for column b = t % 64 over its quarter of the
// block's rows.  Every element of Y is read from memory once; the next
// block's elements are loaded into registers (kYPer per thread, all issued
// together) while the current block is used.  (Measured at n = 10^7,
// m = 50: one block ahead 2.9 ms for the fused step; two blocks ahead, in
// 64- or 32-row blocks, 3.3-3.5 ms; 128-row blocks of 512 threads, apply
// 3.0 ms against 2.45; (Y c)_r split over the four waves, no change.)
constexpr int kYRows = 64;
constexpr int kYStride = kYRows + 1;
constexpr int kYPer = kMaxHistory * kYRows / kLB;
__global__ __launch_bounds__(kLB) void k_lb_ya_staged(int64_t n, const double* __restrict__ Y,
                                                      Ring R, const double* __restrict__ g,
                                                      const double* __restrict__ h0,
                                                      const double* __restrict__ SY,
                                                      double* __restrict__ red,
                                                      double* __restrict__ a_out,
                                                      double* __restrict__ P) {
  __shared__ double tile[kMaxHistory * kYStride];
  __shared__ double as[kYRows];
  __shared__ double cs[kMaxHistory];
  __shared__ int64_t cols[kMaxHistory];
  const int cnt = R.cnt;
  if (threadIdx.x < cnt) {
    cs[threadIdx.x] = red[kMaxHistory + threadIdx.x];
    cols[threadIdx.x] = R.slot(threadIdx.x) * n;
  }
  __syncthreads();
  int64_t lo, hi;
  rows_of<1>(n, blockIdx.x, gridDim.x, &lo, &hi);
  // element k of this thread in a block: column eb + k kBStep, row er
  const int er = threadIdx.x % kYRows, eb = threadIdx.x / kYRows;
  constexpr int kBStep = kLB / kYRows;
  double v[kYPer];
  double gn = 0.0, hn = 1.0;  // g and h0 of row er of the block, for threads below kYRows
  auto load = [&](int64_t r0) {
    const bool in = r0 + er < hi;
#pragma unroll
    for (int k = 0; k < kYPer; ++k) {
      const int b = eb + k * kBStep;
      if (in && b < cnt) v[k] = Y[cols[b] + r0 + er];
    }
    if (in && threadIdx.x < kYRows) {
      gn = g[r0 + er];
      if (h0) hn = h0[r0 + er];
    }
  };
  const int fb = threadIdx.x & 63;  // column of this thread's f accumulator
  const int fq = threadIdx.x >> 6;  // its quarter of each block's rows
  constexpr int kQ = kYRows / (kLB / 64);
  double f = 0.0;
  if (lo < hi) load(lo);
  for (int64_t r0 = lo; r0 < hi; r0 += kYRows) {
    const int nr = hi - r0 < kYRows ? (int)(hi - r0) : kYRows;
#pragma unroll
    for (int k = 0; k < kYPer; ++k) {
      const int b = eb + k * kBStep;
      if (er < nr && b < cnt) tile[b * kYStride + er] = v[k];
    }
    const double gc = gn, hc = hn;
    __syncthreads();
    if (r0 + kYRows < hi) load(r0 + kYRows);
    if (threadIdx.x < nr) {
      const int r = threadIdx.x;
      double t = gc;
      for (int b = 0; b < cnt; ++b) t += tile[b * kYStride + r] * cs[b];
      const double ar = h0 ? hc * t : t;
      a_out[r0 + r] = ar;
      as[r] = ar;
    }
    __syncthreads();
    if (fb < cnt) {
      const int rl = fq * kQ, rh = rl + kQ < nr ? rl + kQ : nr;
      for (int r = rl; r < rh; ++r) f += tile[fb * kYStride + r] * as[r];
    }
    __syncthreads();
  }
  // the workgroup's f: the four quarters of each column, added in order
  double* fs = tile;
  fs[threadIdx.x] = f;
  __syncthreads();
  if (threadIdx.x < cnt) {
    double t = 0.0;
    for (int q = 0; q < kLB / 64; ++q) t += fs[q * 64 + threadIdx.x];
    P[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
}

// pass 3: p = a - S e, e from red[3m..]
template <int V>
__global__ __launch_bounds__(kLB, kGemvtWaves) void k_lb_p(int64_t n, const double* __restrict__ S, Ring R,
                                              const double* __restrict__ a,
                                              const double* __restrict__ SY,
                                              const double* __restrict__ red,
                                              double* __restrict__ p) {
  typedef typename Vd<V>::type VD;
  __shared__ double es[kMaxHistory];
  const int cnt = R.cnt;
  if (threadIdx.x < cnt) es[threadIdx.x] = red[3 * kMaxHistory + threadIdx.x];
  __syncthreads();
  row_blocks<V, true>(
      n, S, R, es, [&](int64_t i) { return ldv<V>(a + i); },
      [&](int64_t i, const VD& t) { *reinterpret_cast<VD*>(p + i) = t; });
}

__global__ void k_lb_scale(int64_t n, const double* __restrict__ g, const double* __restrict__ h0,
                           double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (h0 ? h0[i] : 1.0) * g[i];
}


}  // namespace
}  // namespace spx

using namespace spx;
using namespace spx::solver;

namespace {
// The apply's passes with rows taken V at a time.
// With have_q the partials of S^T g are already in rows 2 kMaxHistory + b of
// the workspace (left there by the fused update).
template <int V>
int apply_passes(spx_lbfgs* h, const double* g, const double* h0, double* p, hipStream_t st,
                 bool have_q = false) {
  const int64_t n = h->n;
  const int cnt = h->count;
  const int G = h->G;
  const Ring R{h->m, h->start, cnt};
  if (have_q) {
    hipLaunchKernelGGL(k_lb_reduce, dim3(cnt), dim3(kLB), 0, st,
                       h->P + (int64_t)2 * kMaxHistory * G, G, h->red);
  } else {
    hipLaunchKernelGGL(k_lb_sg<V>, dim3(G), dim3(kLB), 0, st, n, h->S, R, g, h->P);
    hipLaunchKernelGGL(k_lb_reduce, dim3(cnt), dim3(kLB), 0, st, h->P, G, h->red);
  }
  hipLaunchKernelGGL(k_lb_solve<0>, dim3(1), dim3(kLB), 0, st, h->SY, R, h->red);
  int Gf = G;  // workgroups whose partials of f the reduction adds
  if (cnt <= kFused) {
    hipLaunchKernelGGL(k_lb_ya<V>, dim3(G), dim3(kLB), 0, st, n, h->Y, R, g, h0, h->SY,
                       h->red, h->a, h->P);
  } else {
    Gf = h->Gy;
    hipLaunchKernelGGL(k_lb_ya_staged, dim3(Gf), dim3(kLB), 0, st, n, h->Y, R, g, h0, h->SY,
                       h->red, h->a, h->P);
  }
  hipLaunchKernelGGL(k_lb_reduce, dim3(cnt), dim3(kLB), 0, st, h->P, Gf, h->red + 2 * kMaxHistory);
  hipLaunchKernelGGL(k_lb_solve<1>, dim3(1), dim3(kLB), 0, st, h->SY, R, h->red);
  hipLaunchKernelGGL(k_lb_p<V>, dim3(G), dim3(kLB), 0, st, n, h->S, R, h->a, h->SY, h->red, p);
  return SPX_OK;
}
}  // namespace

extern "C" int spx_lbfgs_create(int64_t n, int32_t m, void* stream, spx_lbfgs_handle* out) {
  clear_error();
  if (!out) return set_error(SPX_INVALID_ARG, "lbfgs_create: out is NULL");
  *out = nullptr;
  if (n <= 0 || m < 1 || m > kMaxHistory)
    return set_error(SPX_INVALID_ARG, "lbfgs_create: need n > 0 and 1 <= m <= %d", kMaxHistory);
  (void)stream;
  spx_lbfgs* h = new (std::nothrow) spx_lbfgs();
  if (!h) return set_error(SPX_OUT_OF_MEMORY, "lbfgs_create: host allocation failed");
  (void)hipGetDevice(&h->device);
  h->n = n;
  h->m = m;
  const int64_t rows_per_wg = 4 * kLB;
  // histories longer than kFused run the passes over S (the update's and
  // p's) at 8 waves per SIMD with 8 workgroups per CU; shorter ones run the
  // register-held a / Y^T a pass (184 VGPRs), which keeps 4 (measured: 0.58
  // vs 0.57 ms at m = 5, 4.28 vs 4.44 ms at m = 50, n = 10^7)
  const int per_cu = m > kFused ? 8 : 4;
  h->G = (int)std::max<int64_t>(1, std::min<int64_t>(cu_count() * per_cu, ceil_div(n, rows_per_wg)));
  // the staged pass runs as many workgroups as are resident at once (its
  // LDS allows four per CU)
  int fit = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, reinterpret_cast<const void*>(&k_lb_ya_staged),
                                                   kLB, 0) != hipSuccess || fit <= 0)
    fit = 4;
  (void)hipGetLastError();
  h->Gy = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)cu_count() * fit,
                                                      ceil_div(n, rows_per_wg)));
  int st = SPX_OK;
  do {
    if ((st = dalloc_n(&h->S, (size_t)n * m)) != SPX_OK) break;
    if ((st = dalloc_n(&h->Y, (size_t)n * m)) != SPX_OK) break;
    if ((st = dalloc_n(&h->SY, (size_t)m * m)) != SPX_OK) break;
    if ((st = dalloc_n(&h->P, (size_t)3 * kMaxHistory * h->G)) != SPX_OK) break;
    if ((st = dalloc_n(&h->red, (size_t)5 * kMaxHistory)) != SPX_OK) break;
    if ((st = dalloc_n(&h->a, (size_t)n)) != SPX_OK) break;
  } while (false);
  if (st != SPX_OK) {
    spx_lbfgs_destroy(h);
    return st;
  }
  *out = h;
  return SPX_OK;
}

extern "C" int spx_lbfgs_destroy(spx_lbfgs_handle h) {
  clear_error();
  if (!h) return SPX_OK;
  dfree(h->S);
  dfree(h->Y);
  dfree(h->SY);
  dfree(h->P);
  dfree(h->red);
  dfree(h->a);
  delete h;
  return SPX_OK;
}

extern "C" int spx_lbfgs_reset(spx_lbfgs_handle h) {
  clear_error();
  if (!h) return set_error(SPX_INVALID_ARG, "lbfgs_reset: NULL handle");
  h->count = 0;
  h->start = 0;
  return SPX_OK;
}

extern "C" int spx_lbfgs_get_info(spx_lbfgs_handle h, int64_t* n, int32_t* m, int32_t* count) {
  clear_error();
  if (!h) return set_error(SPX_INVALID_ARG, "lbfgs_get_info: NULL handle");
  if (n) *n = h->n;
  if (m) *m = h->m;
  if (count) *count = h->count;
  return SPX_OK;
}

namespace {
// The update; with g (non-NULL) the pass over S also leaves the partials of
// S^T g for the apply that follows (the caller has checked that g's row
// width matches the update's).
int update_impl(spx_lbfgs* h, const double* s, const double* y, const double* g,
                hipStream_t st) {
  int slot, start, cnt;
  if (h->count < h->m) {
    slot = (h->start + h->count) % h->m;
    start = h->start;
    cnt = h->count + 1;
  } else {
    slot = h->start;  // the oldest pair leaves
    start = (h->start + 1) % h->m;
    cnt = h->m;
  }
  const int G = h->G;
  const Ring R{h->m, start, cnt};
  hipLaunchKernelGGL(k_lb_put, dim3((unsigned)ceil_div(h->n, 256)), dim3(256), 0, st, h->n, s, y,
                     h->S + (int64_t)slot * h->n, h->Y + (int64_t)slot * h->n);
  if (g) {
    if (h->n % 2 == 0)
      hipLaunchKernelGGL(k_lb_update_g<2>, dim3(G), dim3(kLB), 0, st, h->n, h->S, h->Y, R, g, h->P);
    else
      hipLaunchKernelGGL(k_lb_update_g<1>, dim3(G), dim3(kLB), 0, st, h->n, h->S, h->Y, R, g, h->P);
  } else if (h->n % 2 == 0) {
    hipLaunchKernelGGL(k_lb_update<2>, dim3(G), dim3(kLB), 0, st, h->n, h->S, h->Y, R, h->P);
  } else {
    hipLaunchKernelGGL(k_lb_update<1>, dim3(G), dim3(kLB), 0, st, h->n, h->S, h->Y, R, h->P);
  }
  hipLaunchKernelGGL(k_lb_update_finish, dim3(cnt), dim3(kLB), 0, st, h->P, G, R, slot, h->SY);
  SPX_CHECK_HIP(hipGetLastError());
  h->start = start;
  h->count = cnt;
  return SPX_OK;
}

// Rows go two at a time when n is even and g, h0, p are 16-byte aligned.
bool wide_rows(const spx_lbfgs* h, const double* g, const double* h0, const double* p) {
  return h->n % 2 == 0 && ((reinterpret_cast<uintptr_t>(g) | reinterpret_cast<uintptr_t>(h0) |
                            reinterpret_cast<uintptr_t>(p)) & 15) == 0;
}
}  // namespace

extern "C" int spx_lbfgs_update(spx_lbfgs_handle h, const double* s, const double* y,
                                void* stream) {
  clear_error();
  if (!h || !s || !y) return set_error(SPX_INVALID_ARG, "lbfgs_update: NULL argument");
  return update_impl(h, s, y, nullptr, static_cast<hipStream_t>(stream));
}

extern "C" int spx_lbfgs_update_apply(spx_lbfgs_handle h, const double* s, const double* y,
                                      const double* g, const double* h0, double* p,
                                      void* stream) {
  clear_error();
  if (!h || !s || !y || !g || !p)
    return set_error(SPX_INVALID_ARG, "lbfgs_update_apply: NULL argument");
  if (p == g) return set_error(SPX_INVALID_ARG, "lbfgs_update_apply: p must not alias g");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool wide = wide_rows(h, g, h0, p);
  // the folded pass walks rows as the update does (two at a time for even
  // n); when the apply would walk them otherwise, the two run separately so
  // that the result is the same either way
  const bool fold = wide == (h->n % 2 == 0);
  SPX_TRY(update_impl(h, s, y, fold ? g : nullptr, st));
  SPX_TRY(wide ? apply_passes<2>(h, g, h0, p, st, fold) : apply_passes<1>(h, g, h0, p, st, fold));
  SPX_CHECK_HIP(hipGetLastError());
  return SPX_OK;
}

extern "C" int spx_lbfgs_apply(spx_lbfgs_handle h, const double* g, const double* h0, double* p,
                               void* stream) {
  clear_error();
  if (!h || !g || !p) return set_error(SPX_INVALID_ARG, "lbfgs_apply: NULL argument");
  if (p == g) return set_error(SPX_INVALID_ARG, "lbfgs_apply: p must not alias g");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t n = h->n;
  const int cnt = h->count;
  if (cnt == 0) {
    hipLaunchKernelGGL(k_lb_scale, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, n, g, h0, p);
    SPX_CHECK_HIP(hipGetLastError());
    return SPX_OK;
  }
  const bool wide = wide_rows(h, g, h0, p);
  SPX_TRY(wide ? apply_passes<2>(h, g, h0, p, st) : apply_passes<1>(h, g, h0, p, st));
  SPX_CHECK_HIP(hipGetLastError());
  return SPX_OK;
}
