// Batched Jacobi-CG over many independent systems (paper Sec. 7), on the
// team machinery of batch.hpp: each CG phase is one launch for the whole
// batch, the grid re-split among the running systems at every poll.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "batch.hpp"
#include "cg_one.hpp"
#include "common.hpp"
#include "device.hpp"
#include "solver_core.hpp"
#include "spmv_core.hpp"

namespace spx {
namespace {

using namespace solver;
using namespace batch;

// r = b - A x, p = D^-1 r; partials of r.z, r.r, b.b
template <class SH>
__global__ __launch_bounds__(kBlock) void k_b_init(const BatchSys* __restrict__ sys, PlanView pl,
                                                   const double* __restrict__ b,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ r, double* __restrict__ p,
                                                   const double* __restrict__ dinv,
                                                   double* __restrict__ P, int rows) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double lds[kLds];
  const int s = pl.sys(blockIdx.x);
  if (s < 0) return;
  const BatchSys S = sys[s];
  const int64_t o = S.off;
  double rz = 0.0, rr = 0.0, bb = 0.0;
  for_rows<SH, double, double, double>(S.n, S.rowptr, S.col, S.val, x + o, rows,
                                       blockIdx.x - pl.start(s), pl.size(s),
                                       reinterpret_cast<double*>(smem), [&](int64_t row, double ax) {
                                         const double bi = b[o + row];
                                         const double ri = bi - ax;
                                         const double zi = dinv[o + row] * ri;
                                         r[o + row] = ri;
                                         p[o + row] = zi;
                                         rz += ri * zi;
                                         rr += ri * ri;
                                         bb += bi * bi;
                                       }, 0, S.win);
  rz = block_sum<kBlock>(rz, lds);
  rr = block_sum<kBlock>(rr, lds);
  bb = block_sum<kBlock>(bb, lds);
  if (threadIdx.x == 0) {
    P[blockIdx.x] = rz;
    P[pl.G + blockIdx.x] = rr;
    P[2 * pl.G + blockIdx.x] = bb;
  }
}

template <class SH>
__global__ __launch_bounds__(kBlock) void k_b_spmv(const BatchSys* __restrict__ sys, PlanView pl,
                                                   const double* __restrict__ p,
                                                   double* __restrict__ q,
                                                   const CgScalars* __restrict__ st,
                                                   double* __restrict__ P1, int rows) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double lds[kLds];
  const int s = pl.sys(blockIdx.x);
  if (s < 0 || st[s].done) return;
  const BatchSys S = sys[s];
  const int64_t o = S.off;
  double dot = 0.0;
  for_rows<SH, double, double, double>(S.n, S.rowptr, S.col, S.val, p + o, rows,
                                       blockIdx.x - pl.start(s), pl.size(s),
                                       reinterpret_cast<double*>(smem), [&](int64_t row, double v) {
                                         q[o + row] = v;
                                         dot += p[o + row] * v;
                                       }, 0, S.win);
  dot = block_sum<kBlock>(dot, lds);
  if (threadIdx.x == 0) P1[blockIdx.x] = dot;
}

__global__ __launch_bounds__(kBlock) void k_b_update(const BatchSys* __restrict__ sys, PlanView pl,
                                                     double* __restrict__ x, double* __restrict__ r,
                                                     const double* __restrict__ p,
                                                     const double* __restrict__ q,
                                                     const double* __restrict__ dinv, CgScalars* st,
                                                     const double* __restrict__ P1,
                                                     double* __restrict__ P2, int64_t k) {
  __shared__ double lds[kLds];
  const int s = pl.sys(blockIdx.x);
  if (s < 0) return;
  // the system's flag, team and partials are loaded together, the flag
  // tested once the partials are in
  const auto done = st[s].done;
  const int a = pl.start(s), T = pl.size(s);
  const int64_t j = blockIdx.x - a;
  const double pq = reduce_all(P1 + a, T, lds);
  if (done) return;
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (j == 0 && threadIdx.x == 0) {
      st[s].pq = pq;
      st[s].status = SPX_BREAKDOWN;
      st[s].iters = (int32_t)(k - 1);
      st[s].done = 1;
    }
    return;
  }
  const double alpha = st[s].rho[(k - 1) & 1] / pq;
  const BatchSys S = sys[s];
  const int64_t o = S.off;
  const Range rg = block_range(S.n, j, T);
  double rz = 0.0, rr = 0.0;
  for (int64_t i = o + rg.lo + threadIdx.x; i < o + rg.hi; i += kBlock) {
    const double xi = x[i] + alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    const double zi = dinv[i] * ri;
    x[i] = xi;
    r[i] = ri;
    rz += ri * zi;
    rr += ri * ri;
  }
  rz = block_sum<kBlock>(rz, lds);
  rr = block_sum<kBlock>(rr, lds);
  if (threadIdx.x == 0) {
    P2[blockIdx.x] = rz;
    P2[pl.G + blockIdx.x] = rr;
  }
}

__global__ __launch_bounds__(kBlock) void k_b_pupdate(const BatchSys* __restrict__ sys, PlanView pl,
                                                      double* __restrict__ p,
                                                      const double* __restrict__ r,
                                                      const double* __restrict__ dinv,
                                                      CgScalars* st, const double* __restrict__ P2,
                                                      int64_t k) {
  __shared__ double lds[kLds];
  const int s = pl.sys(blockIdx.x);
  if (s < 0) return;
  const auto done = st[s].done;  // tested once the partials are in
  const int a = pl.start(s), T = pl.size(s);
  const int64_t j = blockIdx.x - a;
  double rz, rr;
  reduce_all(P2 + a, P2 + pl.G + a, T, lds, rz, rr);
  if (done) return;
  CgScalars& c = st[s];
  const bool conv = sqrt(rr) <= c.thresh;
  const bool stop = conv || k >= c.maxit;
  const double rho_prev = c.rho[(k - 1) & 1];
  if (j == 0 && threadIdx.x == 0) {
    c.rr = rr;
    c.iters = (int32_t)k;
    if (conv) {
      c.status = SPX_OK;
      c.done = 1;
    } else if (stop) {
      c.status = SPX_NOT_CONVERGED;
      c.done = 1;
    } else {
      c.rho[k & 1] = rz;
      c.beta = rz / rho_prev;
    }
  }
  if (stop) return;
  const double bt = rz / rho_prev;
  const BatchSys S = sys[s];
  const int64_t o = S.off;
  const Range rg = block_range(S.n, j, T);
  for (int64_t i = o + rg.lo + threadIdx.x; i < o + rg.hi; i += kBlock)
    p[i] = dinv[i] * r[i] + bt * p[i];
}

// One persistent launch for the whole batch: each workgroup takes the next
// system from a queue (largest first), runs its whole Jacobi-CG alone
// (cg_one.hpp: the K1..K3 recurrences, tests and statuses, workgroup sums
// for the dots), and takes another until the queue is empty.  A workgroup
// never waits for another; a system's vectors are touched by its own
// workgroup only.  Thread t owns rows t, t + BLOCK, ... of every pass, the
// D^-1 it writes included.  BLOCK = 256 for systems of at most 1024 rows
// (more systems in flight), 1024 above (each system faster); tiles of ROWS
// rows.
template <int BLOCK, int ROWS>
__global__ __launch_bounds__(BLOCK) void k_b_cg_persistent(
    const BatchSys* __restrict__ sys, int nsys, int32_t* __restrict__ queue,
    const double* __restrict__ bvec, double* __restrict__ x, double* __restrict__ r,
    double* __restrict__ p, double* __restrict__ q, double* __restrict__ dinv, CgScalars* st,
    double rtol) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double lds[BLOCK / 64];
  __shared__ int32_t pick, zero;
  for (;;) {
    if (threadIdx.x == 0) {
      pick = atomicAdd(queue, 1);
      zero = 0;
    }
    __syncthreads();
    const int32_t k = pick;
    if (k >= nsys) break;
    const int s = queue[1 + k];
    const BatchSys S = sys[s];
    const int64_t o = S.off;
    for (int64_t i = threadIdx.x; i < S.n; i += BLOCK) {
      const int32_t t = S.dpos[i];
      const double d = t >= 0 ? S.val[t] : 0.0;
      if (d == 0.0) zero = 1;
      dinv[o + i] = d == 0.0 ? 0.0 : 1.0 / d;
    }
    __syncthreads();
    one::cg_solve<BLOCK, ROWS, true>(S.n, S.rowptr, S.col, S.val, bvec + o, x + o, r + o, p + o, q + o,
                               dinv + o, zero ? SPX_ZERO_DIAGONAL : SPX_OK, st[s].maxit, rtol,
                               st + s, reinterpret_cast<double*>(smem), lds);
    __syncthreads();  // `pick` and `zero` read by every thread before thread 0 rewrites them
  }
}

}  // namespace
}  // namespace spx

using namespace spx;
using namespace spx::solver;

using namespace spx::batch;

namespace {
template <int BLOCK, int ROWS>
int launch_persistent(spx_batch* B, const PersistShape& ps, const double* bvec, double* x,
                      double* r, double* p, double* q, double* dinv, double rtol, hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&k_b_cg_persistent<BLOCK, ROWS>);
  int fit = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, fn, BLOCK, ps.lds) != hipSuccess || fit < 1)
    fit = 1;
  const int G = (int)std::min<int64_t>(B->nsys, (int64_t)cu_count() * fit);
  hipLaunchKernelGGL((k_b_cg_persistent<BLOCK, ROWS>), dim3((unsigned)G), dim3(BLOCK), ps.lds, s,
                     B->d_sys, B->nsys, B->d_queue, bvec, x, r, p, q, dinv, B->d_st, rtol);
  return SPX_OK;
}
}  // namespace

extern "C" int spx_batch_create(int32_t nsys, const spx_handle* hs, void* stream,
                                spx_batch_handle* out) {
  clear_error();
  if (!out) return set_error(SPX_INVALID_ARG, "batch_create: out is NULL");
  *out = nullptr;
  if (nsys <= 0 || !hs) return set_error(SPX_INVALID_ARG, "batch_create: no systems");
  hipStream_t s = static_cast<hipStream_t>(stream);
  spx_batch* B = new (std::nothrow) spx_batch();
  if (!B) return set_error(SPX_OUT_OF_MEMORY, "batch_create: host allocation failed");
  (void)hipGetDevice(&B->device);
  B->nsys = nsys;
  int64_t off = 0;
  for (int k = 0; k < nsys; ++k) {
    spx_handle h = hs[k];
    if (!h) {
      delete B;
      return set_error(SPX_INVALID_ARG, "batch_create: handle %d is NULL", k);
    }
    B->hs.push_back(h);
    BatchSys S;
    S.n = h->n;
    S.off = off;
    S.rowptr = h->A.rowptr;
    S.col = h->A.col;
    S.val = h->A.val;
    S.dpos = h->A.dpos;
    S.win = win_view(h->A);
    B->sys.push_back(S);
    B->win_blocks = h->A.win.lcol && B->win_blocks >= 0
                        ? std::max(B->win_blocks, h->A.win.max_blocks)
                        : -1;
    off += h->n;
    for (int t = 0; t < 4; ++t) B->max_tile[t] = std::max(B->max_tile[t], h->A.tile_nnz[t]);
    B->max_row = std::max(B->max_row, h->A.max_row);
    B->max_nnz_sys = std::max(B->max_nnz_sys, h->A.nnz);
  }
  B->total = off;
  int st = SPX_OK;
  do {
    if ((st = dalloc_n(&B->d_sys, (size_t)nsys)) != SPX_OK) break;
    if ((st = dalloc_n(&B->work, (size_t)B->total * 4)) != SPX_OK) break;
    if ((st = dalloc_n(&B->d_st, (size_t)nsys)) != SPX_OK) break;
    if ((st = dalloc_n(&B->d_queue, (size_t)nsys + 1)) != SPX_OK) break;
    if (hipHostMalloc(reinterpret_cast<void**>(&B->h_st), sizeof(CgScalars) * (size_t)nsys,
                      hipHostMallocDefault) != hipSuccess) {
      st = set_error(SPX_OUT_OF_MEMORY, "batch_create: pinned allocation failed");
      break;
    }
    // the persistent solve's queue: systems by decreasing entry count
    // (ties in system order), so the longest solves start first
    std::vector<int32_t> order(nsys + 1, 0);
    for (int k = 0; k < nsys; ++k) order[1 + k] = k;
    std::stable_sort(order.begin() + 1, order.end(), [&](int32_t a, int32_t b) {
      return B->hs[a]->A.nnz > B->hs[b]->A.nnz;
    });
    if (hipMemcpyAsync(B->d_sys, B->sys.data(), sizeof(BatchSys) * (size_t)nsys,
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(B->d_queue, order.data(), sizeof(int32_t) * (size_t)(nsys + 1),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = set_error(SPX_HIP_ERROR, "batch_create: descriptor upload failed");
      break;
    }
  } while (false);
  if (st != SPX_OK) {
    spx_batch_destroy(B);
    return st;
  }
  *out = B;
  return SPX_OK;
}

extern "C" int spx_batch_destroy(spx_batch_handle B) {
  clear_error();
  if (!B) return SPX_OK;
  dfree(B->d_sys);
  dfree(B->work);
  dfree(B->d_st);
  dfree(B->d_plan);
  dfree(B->partials);
  dfree(B->d_sysT);
  dfree(B->kwork);
  dfree(B->d_queue);
  if (B->h_st) (void)hipHostFree(B->h_st);
  if (B->h_plan) (void)hipHostFree(B->h_plan);
  delete B;
  return SPX_OK;
}

extern "C" int spx_batch_total_rows(spx_batch_handle B, int64_t* total) {
  clear_error();
  if (!B || !total) return set_error(SPX_INVALID_ARG, "batch_total_rows: NULL argument");
  *total = B->total;
  return SPX_OK;
}

extern "C" int spx_batch_cg(spx_batch_handle B, const double* bvec, double* x, double rtol,
                            int64_t maxit, const spx_batch_tuning* tuning, void* stream,
                            int64_t* iters_out, double* relres_out) {
  clear_error();
  if (!B || !bvec || !x) return set_error(SPX_INVALID_ARG, "batch_cg: NULL argument");
  if (maxit < 0 || !(rtol >= 0.0)) return set_error(SPX_INVALID_ARG, "batch_cg: bad maxit/rtol");
  if (maxit > INT32_MAX - 1) maxit = INT32_MAX - 1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ns = B->nsys;
  int32_t pmode = 0;
  SPX_TRY(persistent_mode(tuning, "batch_cg", &pmode));
  Run run;
  SPX_TRY(prepare(B, tuning, B->max_tile, B->max_row, B->win_blocks, 3, s, &run));
  const int G = run.G;
  const int64_t tot = B->total;
  double* r = B->work;
  double* p = B->work + tot;
  double* q = B->work + 2 * tot;
  double* dinv = B->work + 3 * tot;
  const PersistShape ps = persistent_shape(B, B->max_tile[3]);
  if (pmode == 1 || (pmode == 0 && persistent_by_default(B, ps))) {
    if (ps.lds == 0)
      return set_error(SPX_INVALID_ARG,
                       "batch_cg: a 256-row tile of a system exceeds the persistent solve's LDS");
    hipLaunchKernelGGL(k_b_reset, dim3((unsigned)ceil_div(ns, 64)), dim3(64), 0, s, B->d_st, ns,
                       (int32_t)maxit);
    hipLaunchKernelGGL(k_b_queue_reset, dim3(1), dim3(64), 0, s, B->d_queue);
    if (ps.block == 256)
      SPX_TRY((launch_persistent<256, 256>(B, ps, bvec, x, r, p, q, dinv, rtol, s)));
    else if (ps.rows == 1024)
      SPX_TRY((launch_persistent<1024, 1024>(B, ps, bvec, x, r, p, q, dinv, rtol, s)));
    else if (ps.rows == 512)
      SPX_TRY((launch_persistent<1024, 512>(B, ps, bvec, x, r, p, q, dinv, rtol, s)));
    else
      SPX_TRY((launch_persistent<1024, 256>(B, ps, bvec, x, r, p, q, dinv, rtol, s)));
    SPX_CHECK_HIP(hipGetLastError());
    SPX_TRY(true_residuals(B, run, bvec, x, s));
    return finish(B, s, iters_out, relres_out, "batch_cg");
  }
  double* P1 = B->partials;
  double* P2 = B->partials + G;
  const PlanView pl = run.pl;
  const SpmvShape sh = run.sh;
  const size_t lds = run.lds;

  hipLaunchKernelGGL(k_b_reset, dim3((unsigned)ceil_div(ns, 64)), dim3(64), 0, s, B->d_st, ns,
                     (int32_t)maxit);
  hipLaunchKernelGGL(k_b_dinv, dim3(G), dim3(kBlock), 0, s, B->d_sys, pl, dinv, B->d_st);
  SPX_TRY(with_shape<true>(sh, [&](auto shc) {
    using SH = decltype(shc);
    hipLaunchKernelGGL((k_b_init<SH>), dim3(G), dim3(kBlock), lds, s, B->d_sys, pl, bvec, x, r, p,
                       dinv, B->partials, sh.rows);
    return SPX_OK;
  }));
  hipLaunchKernelGGL(k_b_init_finish, dim3(ns), dim3(kBlock), 0, s, pl, B->d_st, B->partials, rtol);
  SPX_CHECK_HIP(hipGetLastError());

  SPX_TRY(poll_loop(B, run, maxit, s, [&](int64_t first, int64_t m) {
    return with_shape<true>(sh, [&](auto shc) {
      using SH = decltype(shc);
      for (int64_t c = 0; c < m; ++c) {
        const int64_t kk = first + c;
        hipLaunchKernelGGL((k_b_spmv<SH>), dim3(G), dim3(kBlock), lds, s, B->d_sys, pl, p, q,
                           B->d_st, P1, sh.rows);
        hipLaunchKernelGGL(k_b_update, dim3(G), dim3(kBlock), 0, s, B->d_sys, pl, x, r, p, q, dinv,
                           B->d_st, P1, P2, kk);
        hipLaunchKernelGGL(k_b_pupdate, dim3(G), dim3(kBlock), 0, s, B->d_sys, pl, p, r, dinv,
                           B->d_st, P2, kk);
      }
      return SPX_OK;
    });
  }));
  SPX_TRY(true_residuals(B, run, bvec, x, s));
  return finish(B, s, iters_out, relres_out, "batch_cg");
}
