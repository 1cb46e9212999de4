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
// by slot and grows by one row and one column per update.  One apply is
// three passes over the rows (S^T g; then a and Y^T a in one pass over Y;
// then p from S), separated by the two reductions the formula needs; each
// pass kernel re-adds the per-workgroup partials of the previous one, so
// no workgroup waits for another and no fence is needed.  The two m x m
// triangular solves are done by every workgroup of the pass that needs
// their result (m <= 64: a few thousand flops from L2).
#include <algorithm>
#include <cmath>
#include <new>
#include <type_traits>

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
  double* S = nullptr;
  double* Y = nullptr;
  double* SY = nullptr;  // SY[a*m + b] = s_a . y_b, by slot
  double* P = nullptr;   // partials [2m][G]
  double* red = nullptr; // reduced vectors: q[m] | c[m] | f[m] | u[m] | v[m]
  double* a = nullptr;   // n
};

namespace spx {
namespace {

using namespace solver;

constexpr int kMaxHistory = 64;
constexpr int kLB = 256;

// Column pointers of the pairs in use, oldest first (a kernel argument, so
// the walk needs no slot arithmetic).
struct Cols {
  const double* p[kMaxHistory];
};

// Row range of workgroup b of G over n rows (contiguous, balanced).
__device__ __forceinline__ void rows_of(int64_t n, int b, int G, int64_t* lo, int64_t* hi) {
  *lo = n * b / G;
  *hi = n * (b + 1) / G;
}

// Sum over the workgroup of MM per-thread accumulators; thread 0 of the
// workgroup gets the totals in out[0..cnt).
template <int MM>
__device__ __forceinline__ void block_sums(double (&acc)[MM], int cnt, double* lds, double* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int j = 0; j < cnt; ++j) {
    double v = acc[j];
    v = wave_sum(v);
    if (lane == 0) lds[w * MM + j] = v;
  }
  __syncthreads();
  if (threadIdx.x < cnt) {
    double s = 0.0;
    for (int q = 0; q < kLB / 64; ++q) s += lds[q * MM + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- update
// Writes the new pair into its slot (Snew, Ynew) and forms partials of
// u_b = s_new . y_b and v_b = s_b . y_new over the `cnt` pairs in use,
// oldest first; logical index cnt - 1 is the new pair, whose values come
// straight from s and y.
template <int MM>
__global__ __launch_bounds__(kLB) void k_lb_update(int64_t n, double* __restrict__ Snew,
                                                   double* __restrict__ Ynew,
                                                   const double* __restrict__ s,
                                                   const double* __restrict__ y, Cols Sc, Cols Yc,
                                                   int cnt, double* __restrict__ P) {
  __shared__ double lds[(kLB / 64) * MM];
  __shared__ double tot[MM];
  int64_t lo, hi;
  rows_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  double u[MM], v[MM];
#pragma unroll
  for (int b = 0; b < MM; ++b) u[b] = v[b] = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kLB) {
    const double si = s[i], yi = y[i];
    Snew[i] = si;
    Ynew[i] = yi;
#pragma unroll
    for (int b = 0; b < MM; ++b) {
      if (b < cnt) {
        const bool last = b == cnt - 1;
        const double yb = last ? yi : Yc.p[b][i];
        const double sbv = last ? si : Sc.p[b][i];
        u[b] += si * yb;
        v[b] += sbv * yi;
      }
    }
  }
  const int G = gridDim.x;
  block_sums<MM>(u, cnt, lds, tot);
  if (threadIdx.x < cnt) P[(int64_t)threadIdx.x * G + blockIdx.x] = tot[threadIdx.x];
  block_sums<MM>(v, cnt, lds, tot);
  if (threadIdx.x < cnt) P[(int64_t)(MM + threadIdx.x) * G + blockIdx.x] = tot[threadIdx.x];
}

// one workgroup per (logical index, kind): SY row and column of the new
// slot; workgroups past the pairs in use leave SY alone
template <int MM>
__global__ __launch_bounds__(kLB) void k_lb_update_finish(int m, const double* __restrict__ P,
                                                          int G, int slot, int start, int cnt,
                                                          double* __restrict__ SY) {
  __shared__ double lds[kLds];
  const int b = blockIdx.x % MM, kind = blockIdx.x / MM;
  if (b >= cnt) return;
  const double t = reduce_all(P + (int64_t)(kind * MM + b) * G, G, lds);
  if (threadIdx.x == 0) {
    const int sb = (start + b) % m;
    if (kind == 0)
      SY[slot * m + sb] = t;  // s_new . y_b
    else
      SY[sb * m + slot] = t;  // s_b . y_new
  }
}

// ----------------------------------------------------------------- apply
// pass 1: partials of q_b = s_b . g
template <int MM>
__global__ __launch_bounds__(kLB) void k_lb_sg(int64_t n, Cols Sc, const double* __restrict__ g,
                                               int cnt, double* __restrict__ P) {
  __shared__ double lds[(kLB / 64) * MM];
  __shared__ double tot[MM];
  int64_t lo, hi;
  rows_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  double q[MM];
#pragma unroll
  for (int b = 0; b < MM; ++b) q[b] = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kLB) {
    const double gi = g[i];
#pragma unroll
    for (int b = 0; b < MM; ++b)
      if (b < cnt) q[b] += Sc.p[b][i] * gi;
  }
  block_sums<MM>(q, cnt, lds, tot);
  if (threadIdx.x < cnt) P[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = tot[threadIdx.x];
}

// one workgroup per logical index: out[b] = sum of the G partials of b
__global__ __launch_bounds__(kLB) void k_lb_reduce(const double* __restrict__ P, int G,
                                                   double* __restrict__ out) {
  __shared__ double lds[kLds];
  const double t = reduce_all(P + (int64_t)blockIdx.x * G, G, lds);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// R_ab (a <= b, logical) = s_a . y_b
__device__ __forceinline__ double rmat(const double* SY, int m, int start, int a, int b) {
  return SY[((start + a) % m) * m + (start + b) % m];
}

// pass 2: c = -R^-1 q (every workgroup; workgroup 0 stores it);
// a = h0 (g + Y c); partials of f_b = y_b . a
template <int MM>
__global__ __launch_bounds__(kLB) void k_lb_ya(int64_t n, int m, Cols Yc,
                                               const double* __restrict__ g,
                                               const double* __restrict__ h0,
                                               const double* __restrict__ SY, int start, int cnt,
                                               double* __restrict__ red,
                                               double* __restrict__ a_out,
                                               double* __restrict__ P) {
  __shared__ double lds[(kLB / 64) * MM];
  __shared__ double tot[MM];
  __shared__ double cs[MM];
  if (threadIdx.x == 0) {
    const double* q = red;
    for (int x = cnt - 1; x >= 0; --x) {
      double t = -q[x];
      for (int y = x + 1; y < cnt; ++y) t -= rmat(SY, m, start, x, y) * cs[y];
      cs[x] = t / rmat(SY, m, start, x, x);
    }
    if (blockIdx.x == 0)
      for (int x = 0; x < cnt; ++x) red[MM + x] = cs[x];
  }
  __syncthreads();
  double c[MM];
#pragma unroll
  for (int b = 0; b < MM; ++b) c[b] = b < cnt ? cs[b] : 0.0;
  int64_t lo, hi;
  rows_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  double f[MM];
#pragma unroll
  for (int b = 0; b < MM; ++b) f[b] = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kLB) {
    double t = g[i];
#pragma unroll
    for (int b = 0; b < MM; ++b)
      if (b < cnt) t += Yc.p[b][i] * c[b];
    const double ai = (h0 ? h0[i] : 1.0) * t;
    a_out[i] = ai;
#pragma unroll
    for (int b = 0; b < MM; ++b)
      if (b < cnt) f[b] += Yc.p[b][i] * ai;
  }
  block_sums<MM>(f, cnt, lds, tot);
  if (threadIdx.x < cnt) P[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = tot[threadIdx.x];
}

// pass 3: e = R^-T (f + D c) (every workgroup); p = a - S e
template <int MM>
__global__ __launch_bounds__(kLB) void k_lb_p(int64_t n, int m, Cols Sc,
                                              const double* __restrict__ a,
                                              const double* __restrict__ SY, int start, int cnt,
                                              const double* __restrict__ red,
                                              double* __restrict__ p) {
  __shared__ double es[MM];
  if (threadIdx.x == 0) {
    const double* c = red + MM;
    const double* f = red + 2 * MM;
    for (int x = 0; x < cnt; ++x) {
      double t = f[x] + rmat(SY, m, start, x, x) * c[x];
      for (int y = 0; y < x; ++y) t -= rmat(SY, m, start, y, x) * es[y];
      es[x] = t / rmat(SY, m, start, x, x);
    }
  }
  __syncthreads();
  double e[MM];
#pragma unroll
  for (int b = 0; b < MM; ++b) e[b] = b < cnt ? es[b] : 0.0;
  int64_t lo, hi;
  rows_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kLB) {
    double t = a[i];
#pragma unroll
    for (int b = 0; b < MM; ++b)
      if (b < cnt) t -= Sc.p[b][i] * e[b];
    p[i] = t;
  }
}

__global__ void k_lb_scale(int64_t n, const double* __restrict__ g, const double* __restrict__ h0,
                           double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (h0 ? h0[i] : 1.0) * g[i];
}

template <typename F>
int with_mm(int m, F&& f) {
  if (m <= 8) return f(std::integral_constant<int, 8>());
  if (m <= 16) return f(std::integral_constant<int, 16>());
  if (m <= 32) return f(std::integral_constant<int, 32>());
  return f(std::integral_constant<int, 64>());
}

Cols columns(const double* base, int64_t n, int m, int start, int cnt) {
  Cols c = {};
  for (int b = 0; b < cnt; ++b) c.p[b] = base + (int64_t)((start + b) % m) * n;
  return c;
}

int cu_count_lb() {
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  return cus;
}

}  // namespace
}  // namespace spx

using namespace spx;
using namespace spx::solver;

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
  h->G = (int)std::max<int64_t>(1, std::min<int64_t>(cu_count_lb() * 4, ceil_div(n, rows_per_wg)));
  int st = SPX_OK;
  do {
    if ((st = dalloc_n(&h->S, (size_t)n * m)) != SPX_OK) break;
    if ((st = dalloc_n(&h->Y, (size_t)n * m)) != SPX_OK) break;
    if ((st = dalloc_n(&h->SY, (size_t)m * m)) != SPX_OK) break;
    if ((st = dalloc_n(&h->P, (size_t)2 * kMaxHistory * h->G)) != SPX_OK) break;
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

extern "C" int spx_lbfgs_update(spx_lbfgs_handle h, const double* s, const double* y,
                                void* stream) {
  clear_error();
  if (!h || !s || !y) return set_error(SPX_INVALID_ARG, "lbfgs_update: NULL argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
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
  const Cols Sc = columns(h->S, h->n, h->m, start, cnt);
  const Cols Yc = columns(h->Y, h->n, h->m, start, cnt);
  SPX_TRY(with_mm(cnt, [&](auto mmc) {
    constexpr int MM = decltype(mmc)::value;
    hipLaunchKernelGGL((k_lb_update<MM>), dim3(G), dim3(kLB), 0, st, h->n,
                       h->S + (int64_t)slot * h->n, h->Y + (int64_t)slot * h->n, s, y, Sc, Yc, cnt,
                       h->P);
    hipLaunchKernelGGL((k_lb_update_finish<MM>), dim3(2 * MM), dim3(kLB), 0, st, h->m, h->P, G,
                       slot, start, cnt, h->SY);
    return SPX_OK;
  }));
  SPX_CHECK_HIP(hipGetLastError());
  h->start = start;
  h->count = cnt;
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
  const int G = h->G;
  const Cols Sc = columns(h->S, n, h->m, h->start, cnt);
  const Cols Yc = columns(h->Y, n, h->m, h->start, cnt);
  SPX_TRY(with_mm(cnt, [&](auto mmc) {
    constexpr int MM = decltype(mmc)::value;
    hipLaunchKernelGGL((k_lb_sg<MM>), dim3(G), dim3(kLB), 0, st, n, Sc, g, cnt, h->P);
    hipLaunchKernelGGL(k_lb_reduce, dim3(cnt), dim3(kLB), 0, st, h->P, G, h->red);
    hipLaunchKernelGGL((k_lb_ya<MM>), dim3(G), dim3(kLB), 0, st, n, h->m, Yc, g, h0, h->SY,
                       h->start, cnt, h->red, h->a, h->P);
    hipLaunchKernelGGL(k_lb_reduce, dim3(cnt), dim3(kLB), 0, st, h->P, G, h->red + 2 * MM);
    hipLaunchKernelGGL((k_lb_p<MM>), dim3(G), dim3(kLB), 0, st, n, h->m, Sc, h->a, h->SY,
                       h->start, cnt, h->red, p);
    return SPX_OK;
  }));
  SPX_CHECK_HIP(hipGetLastError());
  return SPX_OK;
}
