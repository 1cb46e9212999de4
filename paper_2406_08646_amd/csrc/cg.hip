// Jacobi-preconditioned CG with device-resident scalars (paper Sec. 6, the
// CG -> CGAsync redesign): every scalar (rho, alpha, beta, the residual
// norm, the convergence flag) lives in device memory and is produced by the
// last workgroup of the kernel that reduces it, so the host only enqueues
// kernels and polls the flag every `check_every` iterations.
//
// One iteration is three kernels, each fused around its memory traffic:
//   K1  q = A p and the partial p.q; the last workgroup forms alpha
//   K2  x += alpha p, r -= alpha q, z = D^-1 r, partial r.z and r.r; the last
//       workgroup counts the iteration, tests ||r|| <= rtol ||b|| and forms
//       beta
//   K3  p = D^-1 r + beta p
// Kernels return at once when the flag is set, so work queued past
// convergence costs only the launches.  Dot products are reduced in a fixed
// order (lanes, waves, workgroups by index), so results are reproducible.
//
// The same kernels, instantiated for float, run the inner solve of the
// mixed-precision refinement (paper Sec. 2 multiprecision plan): fp32
// matrix copy, vectors and SpMV; fp64 products and sums in every dot.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "device.hpp"
#include "spmv_core.hpp"

namespace spx {

namespace {

constexpr int kBlock = 256;

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

__global__ void k_scal_reset(CgScalars* st, int32_t maxit) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    CgScalars z = {};
    z.maxit = maxit;
    *st = z;
  }
}

// dinv[r] = 1 / a_rr (and its fp32 rounding); a missing or zero diagonal
// marks the run with SPX_ZERO_DIAGONAL.
__global__ void k_dinv(int64_t n, const double* __restrict__ val, const int32_t* __restrict__ dpos,
                       double* __restrict__ dinv, float* __restrict__ dinv32, CgScalars* st) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int32_t t = dpos[r];
  const double d = t >= 0 ? val[t] : 0.0;
  double inv = 0.0;
  if (d == 0.0)
    __hip_atomic_store(&st->status, (int32_t)SPX_ZERO_DIAGONAL, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  else
    inv = 1.0 / d;
  dinv[r] = inv;
  if (dinv32) dinv32[r] = (float)inv;
}

// r = b - A x, z = D^-1 r, p = z, and the dots r.z, r.r, b.b.
template <int L>
__global__ __launch_bounds__(kBlock) void k_cg_init(int64_t n, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ r, double* __restrict__ p,
                                                    const double* __restrict__ dinv, CgScalars* st,
                                                    double* __restrict__ partials, double rtol,
                                                    int remap) {
  __shared__ double lds[kBlock / 64];
  constexpr int RPB = kBlock / L;
  const int64_t nb = gridDim.x;
  const int64_t bl = remap ? xcd_logical_block(blockIdx.x, nb) : (int64_t)blockIdx.x;
  const Range rg = block_range(ceil_div(n, RPB), bl, nb);
  const int lane = threadIdx.x % L;
  double rz = 0.0, rr = 0.0, bb = 0.0;
  for (int64_t g = rg.lo; g < rg.hi; ++g) {
    const int64_t row = g * RPB + threadIdx.x / L;
    if (row < n) {
      const double ax = group_sum<L>(row_partial<L, double, double, double>(rowptr, col, val, x, row, lane));
      if (lane == 0) {
        const double bi = b[row];
        const double ri = bi - ax;
        const double zi = dinv[row] * ri;
        r[row] = ri;
        p[row] = zi;
        rz += ri * zi;
        rr += ri * ri;
        bb += bi * bi;
      }
    }
  }
  rz = block_sum<kBlock>(rz, lds);
  rr = block_sum<kBlock>(rr, lds);
  bb = block_sum<kBlock>(bb, lds);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = rz;
    partials[nb + blockIdx.x] = rr;
    partials[2 * nb + blockIdx.x] = bb;
  }
  if (arrive_last(&st->ticket[0])) {
    const double trz = reduce_partials<kBlock>(partials, nb, lds);
    const double trr = reduce_partials<kBlock>(partials + nb, nb, lds);
    const double tbb = reduce_partials<kBlock>(partials + 2 * nb, nb, lds);
    if (threadIdx.x == 0) {
      st->bb = tbb;
      st->bnorm = sqrt(tbb);
      st->thresh = rtol * st->bnorm;
      st->rr = trr;
      st->rho = trz;
      st->iters = 0;
      if (st->status != SPX_OK) {
        st->done = 1;
      } else if (sqrt(trr) <= st->thresh) {
        st->done = 1;
      } else if (st->maxit <= 0) {
        st->done = 1;
        st->status = SPX_NOT_CONVERGED;
      } else {
        st->done = 0;
      }
    }
  }
}

// K1: q = A p, alpha = rho / p.q
template <int L, typename VT>
__global__ __launch_bounds__(kBlock) void k_cg_spmv_dot(int64_t n, const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const VT* __restrict__ val,
                                                        const VT* __restrict__ p,
                                                        VT* __restrict__ q, CgScalars* st,
                                                        double* __restrict__ partials, int remap) {
  __shared__ double lds[kBlock / 64];
  if (st->done) return;
  constexpr int RPB = kBlock / L;
  const int64_t nb = gridDim.x;
  const int64_t bl = remap ? xcd_logical_block(blockIdx.x, nb) : (int64_t)blockIdx.x;
  const Range rg = block_range(ceil_div(n, RPB), bl, nb);
  const int lane = threadIdx.x % L;
  double dot = 0.0;
  for (int64_t g = rg.lo; g < rg.hi; ++g) {
    const int64_t row = g * RPB + threadIdx.x / L;
    if (row < n) {
      const VT s = group_sum<L>(row_partial<L, VT, VT, VT>(rowptr, col, val, p, row, lane));
      if (lane == 0) {
        q[row] = s;
        dot += (double)p[row] * (double)s;
      }
    }
  }
  dot = block_sum<kBlock>(dot, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = dot;
  if (arrive_last(&st->ticket[1])) {
    const double pq = reduce_partials<kBlock>(partials, nb, lds);
    if (threadIdx.x == 0) {
      st->pq = pq;
      if (!(pq > 0.0) || !isfinite(pq)) {
        st->status = SPX_BREAKDOWN;
        st->done = 1;
      } else {
        st->alpha = st->rho / pq;
      }
    }
  }
}

// K2: x += alpha p; r -= alpha q; z = D^-1 r; r.z, r.r; convergence; beta
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_cg_update(int64_t n, VT* __restrict__ x,
                                                      VT* __restrict__ r,
                                                      const VT* __restrict__ p,
                                                      const VT* __restrict__ q,
                                                      const VT* __restrict__ dinv, CgScalars* st,
                                                      double* __restrict__ partials) {
  __shared__ double lds[kBlock / 64];
  if (st->done) return;
  const VT a = (VT)st->alpha;
  const int64_t nb = gridDim.x;
  const Range rg = block_range(n, blockIdx.x, nb);
  double rz = 0.0, rr = 0.0;
  for (int64_t i = rg.lo + threadIdx.x; i < rg.hi; i += kBlock) {
    const VT xi = x[i] + a * p[i];
    const VT ri = r[i] - a * q[i];
    const VT zi = dinv[i] * ri;
    x[i] = xi;
    r[i] = ri;
    rz += (double)ri * (double)zi;
    rr += (double)ri * (double)ri;
  }
  rz = block_sum<kBlock>(rz, lds);
  rr = block_sum<kBlock>(rr, lds);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = rz;
    partials[nb + blockIdx.x] = rr;
  }
  if (arrive_last(&st->ticket[2])) {
    const double trz = reduce_partials<kBlock>(partials, nb, lds);
    const double trr = reduce_partials<kBlock>(partials + nb, nb, lds);
    if (threadIdx.x == 0) {
      const int32_t it = st->iters + 1;
      st->iters = it;
      st->rr = trr;
      if (sqrt(trr) <= st->thresh) {
        st->done = 1;
        st->status = SPX_OK;
      } else if (it >= st->maxit) {
        st->done = 1;
        st->status = SPX_NOT_CONVERGED;
      } else {
        st->beta = trz / st->rho;
        st->rho = trz;
      }
    }
  }
}

// K3: p = D^-1 r + beta p
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_cg_pupdate(int64_t n, VT* __restrict__ p,
                                                       const VT* __restrict__ r,
                                                       const VT* __restrict__ dinv,
                                                       const CgScalars* st) {
  if (st->done) return;
  const VT bt = (VT)st->beta;
  const Range rg = block_range(n, blockIdx.x, gridDim.x);
  for (int64_t i = rg.lo + threadIdx.x; i < rg.hi; i += kBlock) p[i] = dinv[i] * r[i] + bt * p[i];
}

// ||b - A x||^2 into st->rr_true
template <int L>
__global__ __launch_bounds__(kBlock) void k_resnorm(int64_t n, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ x, CgScalars* st,
                                                    double* __restrict__ partials, int remap) {
  __shared__ double lds[kBlock / 64];
  constexpr int RPB = kBlock / L;
  const int64_t nb = gridDim.x;
  const int64_t bl = remap ? xcd_logical_block(blockIdx.x, nb) : (int64_t)blockIdx.x;
  const Range rg = block_range(ceil_div(n, RPB), bl, nb);
  const int lane = threadIdx.x % L;
  double rr = 0.0;
  for (int64_t g = rg.lo; g < rg.hi; ++g) {
    const int64_t row = g * RPB + threadIdx.x / L;
    if (row < n) {
      const double ax = group_sum<L>(row_partial<L, double, double, double>(rowptr, col, val, x, row, lane));
      if (lane == 0) {
        const double ri = b[row] - ax;
        rr += ri * ri;
      }
    }
  }
  rr = block_sum<kBlock>(rr, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = rr;
  if (arrive_last(&st->ticket[3])) {
    const double t = reduce_partials<kBlock>(partials, nb, lds);
    if (threadIdx.x == 0) st->rr_true = t;
  }
}

// ---------------------------------------------------- mixed precision

// ||b||^2 -> outer scalars and the outer threshold
__global__ __launch_bounds__(kBlock) void k_norm2(int64_t n, const double* __restrict__ b,
                                                  CgScalars* st, double* __restrict__ partials,
                                                  double rtol) {
  __shared__ double lds[kBlock / 64];
  const int64_t nb = gridDim.x;
  const Range rg = block_range(n, blockIdx.x, nb);
  double s = 0.0;
  for (int64_t i = rg.lo + threadIdx.x; i < rg.hi; i += kBlock) s += b[i] * b[i];
  s = block_sum<kBlock>(s, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
  if (arrive_last(&st->ticket[0])) {
    const double t = reduce_partials<kBlock>(partials, nb, lds);
    if (threadIdx.x == 0) {
      st->bb = t;
      st->bnorm = sqrt(t);
      st->thresh = rtol * st->bnorm;
    }
  }
}

// Outer fp64 residual r = b - A x with its norm, rounded to fp32, and the
// start of the inner solve: d = 0, z = D32^-1 r32, p = z, rho, ||r32||.
template <int L>
__global__ __launch_bounds__(kBlock) void k_ir_residual(
    int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ b, const double* __restrict__ x,
    const float* __restrict__ dinv32, float* __restrict__ r32, float* __restrict__ d32,
    float* __restrict__ p32, CgScalars* so, CgScalars* si, double* __restrict__ partials,
    double rtol_inner, int remap) {
  __shared__ double lds[kBlock / 64];
  constexpr int RPB = kBlock / L;
  const int64_t nb = gridDim.x;
  const int64_t bl = remap ? xcd_logical_block(blockIdx.x, nb) : (int64_t)blockIdx.x;
  const Range rg = block_range(ceil_div(n, RPB), bl, nb);
  const int lane = threadIdx.x % L;
  double rr64 = 0.0, rz = 0.0, rr32 = 0.0;
  for (int64_t g = rg.lo; g < rg.hi; ++g) {
    const int64_t row = g * RPB + threadIdx.x / L;
    if (row < n) {
      const double ax = group_sum<L>(row_partial<L, double, double, double>(rowptr, col, val, x, row, lane));
      if (lane == 0) {
        const double ri = b[row] - ax;
        rr64 += ri * ri;
        const float rf = (float)ri;
        const float zf = dinv32[row] * rf;
        r32[row] = rf;
        d32[row] = 0.0f;
        p32[row] = zf;
        rz += (double)rf * (double)zf;
        rr32 += (double)rf * (double)rf;
      }
    }
  }
  rr64 = block_sum<kBlock>(rr64, lds);
  rz = block_sum<kBlock>(rz, lds);
  rr32 = block_sum<kBlock>(rr32, lds);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = rr64;
    partials[nb + blockIdx.x] = rz;
    partials[2 * nb + blockIdx.x] = rr32;
  }
  if (arrive_last(&so->ticket[1])) {
    const double t64 = reduce_partials<kBlock>(partials, nb, lds);
    const double trz = reduce_partials<kBlock>(partials + nb, nb, lds);
    const double t32 = reduce_partials<kBlock>(partials + 2 * nb, nb, lds);
    if (threadIdx.x == 0) {
      so->rr = t64;
      so->rr_true = t64;
      if (so->status == SPX_OK && sqrt(t64) <= so->thresh) so->done = 1;
      si->rho = trz;
      si->r0norm = sqrt(t32);
      si->thresh = rtol_inner * si->r0norm;
      si->rr = t32;
      si->iters = 0;
      si->status = SPX_OK;
      si->done = (so->done || so->status != SPX_OK) ? 1 : 0;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_ir_update(int64_t n, double* __restrict__ x,
                                                      const float* __restrict__ d32) {
  const Range rg = block_range(n, blockIdx.x, gridDim.x);
  for (int64_t i = rg.lo + threadIdx.x; i < rg.hi; i += kBlock) x[i] = x[i] + (double)d32[i];
}

// ------------------------------------------------------------ dispatch

template <typename F>
int with_lanes(int L, F&& f) {
  switch (L) {
    case 1: return f(std::integral_constant<int, 1>());
    case 2: return f(std::integral_constant<int, 2>());
    case 4: return f(std::integral_constant<int, 4>());
    case 8: return f(std::integral_constant<int, 8>());
    case 16: return f(std::integral_constant<int, 16>());
    case 32: return f(std::integral_constant<int, 32>());
    case 64: return f(std::integral_constant<int, 64>());
    default: return set_error(SPX_INVALID_ARG, "unsupported lane count %d", L);
  }
}

int ensure_solver(spx_matrix* h) {
  const int64_t n = h->n;
  if (!h->work) {
    SPX_TRY(dalloc_n(&h->work, (size_t)n * 4));
    SPX_TRY(dalloc_n(&h->dinv, (size_t)n));
  }
  if (!h->scal) {
    SPX_TRY(dalloc_n(&h->scal, 2));
    SPX_CHECK_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->scal_host), sizeof(CgScalars) * 4,
                                hipHostMallocDefault));
    SPX_CHECK_HIP(hipEventCreateWithFlags(&h->ev[0], hipEventDisableTiming));
    SPX_CHECK_HIP(hipEventCreateWithFlags(&h->ev[1], hipEventDisableTiming));
    SPX_CHECK_HIP(hipMemset(h->scal, 0, sizeof(CgScalars) * 2));
  }
  const int64_t cap = (int64_t)fused_blocks() * 4;
  if (h->partial_cap < cap) {
    dfree(h->partials);
    h->partials = nullptr;
    SPX_TRY(dalloc_n(&h->partials, (size_t)cap));
    h->partial_cap = cap;
  }
  return SPX_OK;
}

int ensure_solver32(spx_matrix* h) {
  if (!h->work32) {
    SPX_TRY(dalloc_n(&h->work32, (size_t)h->n * 4));
    SPX_TRY(dalloc_n(&h->dinv32, (size_t)h->n));
  }
  return SPX_OK;
}

inline unsigned grid1(int64_t count) {
  return (unsigned)std::max<int64_t>(1, ceil_div(count, 256));
}

// Enqueues `count` CG iterations (K1, K2, K3) on the given operator.  With
// `evs` (6 events per iteration) every kernel is bracketed by events.
template <typename VT>
int enqueue_iterations(int L, int64_t n, const int32_t* rowptr, const int32_t* col, const VT* val,
                       VT* x, VT* r, VT* p, VT* q, const VT* dinv, CgScalars* st,
                       double* partials, int remap, int64_t count, hipStream_t s,
                       hipEvent_t* evs) {
  const unsigned nb = (unsigned)fused_blocks();
  return with_lanes(L, [&](auto Lc) {
    constexpr int LL = decltype(Lc)::value;
    for (int64_t k = 0; k < count; ++k) {
      hipEvent_t* e = evs ? evs + 6 * k : nullptr;
      if (e) (void)hipEventRecord(e[0], s);
      hipLaunchKernelGGL((k_cg_spmv_dot<LL, VT>), dim3(nb), dim3(kBlock), 0, s, n, rowptr, col, val,
                         p, q, st, partials, remap);
      if (e) (void)hipEventRecord(e[1], s);
      if (e) (void)hipEventRecord(e[2], s);
      hipLaunchKernelGGL((k_cg_update<VT>), dim3(nb), dim3(kBlock), 0, s, n, x, r, p, q, dinv, st,
                         partials);
      if (e) (void)hipEventRecord(e[3], s);
      if (e) (void)hipEventRecord(e[4], s);
      hipLaunchKernelGGL((k_cg_pupdate<VT>), dim3(nb), dim3(kBlock), 0, s, n, p, r, dinv, st);
      if (e) (void)hipEventRecord(e[5], s);
    }
    return SPX_OK;
  });
}

int ensure_prof_events(spx_matrix* h, int64_t need) {
  if (h->prof_ev_n >= need) return SPX_OK;
  hipEvent_t* ev = new hipEvent_t[need];
  for (int64_t k = 0; k < h->prof_ev_n; ++k) ev[k] = h->prof_ev[k];
  for (int64_t k = h->prof_ev_n; k < need; ++k) SPX_CHECK_HIP(hipEventCreate(&ev[k]));
  delete[] h->prof_ev;
  h->prof_ev = ev;
  h->prof_ev_n = need;
  return SPX_OK;
}

// Adds the event-timed durations of iterations [first, first+count) of a
// finished chunk, counting only launches that did work (iterations up to
// `iters`; the p update of the last iteration is skipped by the kernel).
void accumulate_profile(spx_matrix* h, hipEvent_t* evs, int64_t first, int64_t count,
                        int64_t iters, int kind0) {
  for (int64_t k = 0; k < count; ++k) {
    const int64_t it = first + k + 1;
    for (int j = 0; j < 3; ++j) {
      const bool ran = (j < 2) ? it <= iters : it < iters;
      if (!ran) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, evs[6 * k + 2 * j], evs[6 * k + 2 * j + 1]) == hipSuccess) {
        h->prof_ms[kind0 + j] += ms;
        h->prof_cnt[kind0 + j] += 1;
      }
    }
  }
}

// Runs iterations until the device flag is set, keeping one chunk of
// `check_every` iterations queued ahead of the one being polled.  Returns
// the last polled state in *final.
template <typename VT>
int run_until_done(spx_matrix* h, int L, int64_t n, const int32_t* rowptr, const int32_t* col,
                   const VT* val, VT* x, VT* r, VT* p, VT* q, const VT* dinv, CgScalars* st,
                   int64_t maxit, int32_t check_every, hipStream_t s, CgScalars* final) {
  int64_t launched = 0;
  CgScalars* host = h->scal_host;
  const bool prof = h->profile != 0;
  const int kind0 = sizeof(VT) == 8 ? 0 : 3;
  if (prof) SPX_TRY(ensure_prof_events(h, 2 * 6 * (int64_t)check_every));
  int64_t first[2] = {0, 0}, cnt[2] = {0, 0};
  auto chunk = [&](int slot) -> int {
    const int64_t m = std::min<int64_t>(check_every, maxit - launched);
    hipEvent_t* evs = prof ? h->prof_ev + slot * 6 * (int64_t)check_every : nullptr;
    SPX_TRY(enqueue_iterations<VT>(L, n, rowptr, col, val, x, r, p, q, dinv, st, h->partials,
                                   h->xcd_remap, m, s, evs));
    first[slot] = launched;
    cnt[slot] = m;
    launched += m;
    SPX_CHECK_HIP(hipMemcpyAsync(&host[slot], st, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
    SPX_CHECK_HIP(hipEventRecord(h->ev[slot], s));
    return SPX_OK;
  };
  auto harvest = [&](int slot, int64_t iters) {
    if (prof && cnt[slot] > 0)
      accumulate_profile(h, h->prof_ev + slot * 6 * (int64_t)check_every, first[slot], cnt[slot],
                         iters, kind0);
    cnt[slot] = 0;
  };
  // state before any iteration (init may already have converged)
  SPX_CHECK_HIP(hipMemcpyAsync(&host[0], st, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
  SPX_CHECK_HIP(hipStreamSynchronize(s));
  if (host[0].done || maxit <= 0) {
    *final = host[0];
    return SPX_OK;
  }
  SPX_TRY(chunk(0));
  int cur = 0;
  for (;;) {
    const bool more = launched < maxit;
    if (more) SPX_TRY(chunk(cur ^ 1));
    SPX_CHECK_HIP(hipEventSynchronize(h->ev[cur]));
    if (host[cur].done || !more) {
      *final = host[cur];
      break;
    }
    harvest(cur, host[cur].iters);
    cur ^= 1;
  }
  SPX_CHECK_HIP(hipStreamSynchronize(s));
  harvest(0, final->iters);
  harvest(1, final->iters);
  return SPX_OK;
}

int cg_solve_impl(spx_matrix* h, const Csr& A, const double* b, double* x, double rtol,
                  int64_t maxit, int32_t check_every, hipStream_t s, int64_t* iters_out,
                  double* relres_out) {
  if (!b || !x) return set_error(SPX_INVALID_ARG, "cg_solve: b or x is NULL");
  if (maxit < 0 || check_every < 1 || !(rtol >= 0.0))
    return set_error(SPX_INVALID_ARG, "cg_solve: bad maxit/check_every/rtol");
  if (maxit > INT32_MAX) maxit = INT32_MAX;
  SPX_TRY(ensure_solver(h));
  const int64_t n = A.n;
  double* r = h->work;
  double* p = h->work + n;
  double* q = h->work + 2 * n;
  CgScalars* st = h->scal;
  const unsigned nb = (unsigned)fused_blocks();
  const int L = pick_lanes(A, h->lanes_opt);
  hipLaunchKernelGGL(k_scal_reset, dim3(1), dim3(64), 0, s, st, (int32_t)maxit);
  hipLaunchKernelGGL(k_dinv, dim3(grid1(n)), dim3(256), 0, s, n, A.val, A.dpos, h->dinv,
                     (float*)nullptr, st);
  SPX_TRY(with_lanes(L, [&](auto Lc) {
    constexpr int LL = decltype(Lc)::value;
    hipLaunchKernelGGL((k_cg_init<LL>), dim3(nb), dim3(kBlock), 0, s, n, A.rowptr, A.col, A.val, b,
                       x, r, p, h->dinv, st, h->partials, rtol, h->xcd_remap);
    return SPX_OK;
  }));
  SPX_CHECK_HIP(hipGetLastError());
  CgScalars fin;
  SPX_TRY(run_until_done<double>(h, L, n, A.rowptr, A.col, A.val, x, r, p, q, h->dinv, st, maxit,
                                 check_every, s, &fin));
  SPX_TRY(with_lanes(L, [&](auto Lc) {
    constexpr int LL = decltype(Lc)::value;
    hipLaunchKernelGGL((k_resnorm<LL>), dim3(nb), dim3(kBlock), 0, s, n, A.rowptr, A.col, A.val, b,
                       x, st, h->partials, h->xcd_remap);
    return SPX_OK;
  }));
  SPX_CHECK_HIP(hipMemcpyAsync(&h->scal_host[2], st, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
  SPX_CHECK_HIP(hipStreamSynchronize(s));
  const CgScalars& f = h->scal_host[2];
  if (iters_out) *iters_out = f.iters;
  if (relres_out) *relres_out = f.bnorm > 0.0 ? sqrt(f.rr_true) / f.bnorm : sqrt(f.rr_true);
  if (f.status == SPX_ZERO_DIAGONAL)
    return set_error(SPX_ZERO_DIAGONAL, "cg_solve: zero or missing diagonal entry");
  if (f.status == SPX_BREAKDOWN)
    return set_error(SPX_BREAKDOWN, "cg_solve: breakdown (p.Ap = %g) at iteration %d", f.pq,
                     f.iters + 1);
  if (f.status == SPX_NOT_CONVERGED || !f.done)
    return set_error(SPX_NOT_CONVERGED, "cg_solve: %d iterations, ||r||/||b|| = %g", f.iters,
                     f.bnorm > 0 ? sqrt(f.rr) / f.bnorm : sqrt(f.rr));
  return SPX_OK;
}

}  // namespace

int fused_blocks() {
  static int cached[64] = {0};
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev < 0 || dev >= 64) dev = 0;
  if (!cached[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cached[dev] = cus * 8;
  }
  return cached[dev];
}

}  // namespace spx

using namespace spx;

extern "C" int spx_cg_solve(spx_handle h, const double* b, double* x, double rtol, int64_t maxit,
                            int32_t check_every, void* stream, int64_t* iters_out,
                            double* relres_out) {
  clear_error();
  if (!h) return set_error(SPX_INVALID_ARG, "cg_solve: NULL handle");
  return cg_solve_impl(h, h->A, b, x, rtol, maxit, check_every, static_cast<hipStream_t>(stream),
                       iters_out, relres_out);
}

extern "C" int spx_cg_solve_transpose(spx_handle h, const double* b, double* x, double rtol,
                                      int64_t maxit, int32_t check_every, void* stream,
                                      int64_t* iters_out, double* relres_out) {
  clear_error();
  if (!h) return set_error(SPX_INVALID_ARG, "cg_solve_transpose: NULL handle");
  hipStream_t s = static_cast<hipStream_t>(stream);
  SPX_TRY(ensure_transpose(h, s));
  return cg_solve_impl(h, h->At, b, x, rtol, maxit, check_every, s, iters_out, relres_out);
}

extern "C" int spx_cg_solve_mixed(spx_handle h, const double* b, double* x, double rtol_outer,
                                  double rtol_inner, int64_t maxit_outer, int64_t maxit_inner,
                                  int32_t check_every, void* stream, int64_t* outer_out,
                                  int64_t* inner_out, double* relres_out) {
  clear_error();
  if (!h || !b || !x) return set_error(SPX_INVALID_ARG, "cg_solve_mixed: NULL argument");
  if (maxit_outer < 0 || maxit_inner < 1 || check_every < 1 || !(rtol_outer >= 0.0) ||
      !(rtol_inner > 0.0))
    return set_error(SPX_INVALID_ARG, "cg_solve_mixed: bad iteration limits or tolerances");
  if (maxit_inner > INT32_MAX) maxit_inner = INT32_MAX;
  hipStream_t s = static_cast<hipStream_t>(stream);
  SPX_TRY(ensure_solver(h));
  SPX_TRY(ensure_solver32(h));
  SPX_TRY(ensure_val32(h, s));
  const Csr& A = h->A;
  const int64_t n = A.n;
  float* r32 = h->work32;
  float* d32 = h->work32 + n;
  float* p32 = h->work32 + 2 * n;
  float* q32 = h->work32 + 3 * n;
  CgScalars* so = h->scal;
  CgScalars* si = h->scal + 1;
  const unsigned nb = (unsigned)fused_blocks();
  const int L = pick_lanes(A, h->lanes_opt);
  hipLaunchKernelGGL(k_scal_reset, dim3(1), dim3(64), 0, s, so, (int32_t)0);
  hipLaunchKernelGGL(k_scal_reset, dim3(1), dim3(64), 0, s, si, (int32_t)maxit_inner);
  hipLaunchKernelGGL(k_dinv, dim3(grid1(n)), dim3(256), 0, s, n, A.val, A.dpos, h->dinv, h->dinv32,
                     so);
  hipLaunchKernelGGL(k_norm2, dim3(nb), dim3(kBlock), 0, s, n, b, so, h->partials, rtol_outer);
  SPX_CHECK_HIP(hipGetLastError());
  int64_t outer = 0, inner = 0;
  int status = SPX_OK;
  for (;;) {
    SPX_TRY(with_lanes(L, [&](auto Lc) {
      constexpr int LL = decltype(Lc)::value;
      hipLaunchKernelGGL((k_ir_residual<LL>), dim3(nb), dim3(kBlock), 0, s, n, A.rowptr, A.col,
                         A.val, b, x, h->dinv32, r32, d32, p32, so, si, h->partials, rtol_inner,
                         h->xcd_remap);
      return SPX_OK;
    }));
    SPX_CHECK_HIP(hipMemcpyAsync(&h->scal_host[2], so, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
    SPX_CHECK_HIP(hipStreamSynchronize(s));
    const CgScalars o = h->scal_host[2];
    if (o.status != SPX_OK) {
      status = o.status;
      break;
    }
    if (o.done) break;
    if (outer >= maxit_outer) {
      status = SPX_NOT_CONVERGED;
      break;
    }
    ++outer;
    CgScalars fin;
    SPX_TRY(run_until_done<float>(h, L, n, A.rowptr, A.col, A.val32, d32, r32, p32, q32, h->dinv32,
                                  si, maxit_inner, check_every, s, &fin));
    inner += fin.iters;
    hipLaunchKernelGGL(k_ir_update, dim3(nb), dim3(kBlock), 0, s, n, x, d32);
    if (fin.status == SPX_BREAKDOWN) {
      status = SPX_BREAKDOWN;
      break;
    }
  }
  SPX_TRY(with_lanes(L, [&](auto Lc) {
    constexpr int LL = decltype(Lc)::value;
    hipLaunchKernelGGL((k_resnorm<LL>), dim3(nb), dim3(kBlock), 0, s, n, A.rowptr, A.col, A.val, b,
                       x, so, h->partials, h->xcd_remap);
    return SPX_OK;
  }));
  SPX_CHECK_HIP(hipMemcpyAsync(&h->scal_host[2], so, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
  SPX_CHECK_HIP(hipStreamSynchronize(s));
  const CgScalars& f = h->scal_host[2];
  if (outer_out) *outer_out = outer;
  if (inner_out) *inner_out = inner;
  if (relres_out) *relres_out = f.bnorm > 0.0 ? sqrt(f.rr_true) / f.bnorm : sqrt(f.rr_true);
  if (status == SPX_ZERO_DIAGONAL)
    return set_error(status, "cg_solve_mixed: zero or missing diagonal entry");
  if (status == SPX_BREAKDOWN) return set_error(status, "cg_solve_mixed: inner breakdown");
  if (status == SPX_NOT_CONVERGED)
    return set_error(status, "cg_solve_mixed: %lld outer steps, relres %g", (long long)outer,
                     f.bnorm > 0.0 ? sqrt(f.rr_true) / f.bnorm : 0.0);
  return SPX_OK;
}
