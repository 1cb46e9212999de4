// Batched Jacobi-CG over many independent systems (paper Sec. 7: one
// batched Krylov solver with a diagonal preconditioner for many small
// systems, instead of one stacked "ensemble" system).
//
// Design for gfx950.  All systems advance together, one iteration at a
// time, and each CG phase is ONE launch for the whole batch: the grid's
// workgroups are split into teams, one team per still-running system, and
// a team walks its system exactly as the single-system kernels do (same
// row walk, same partial sums reduced by the next launch).  A system that
// has converged stops consuming bandwidth, and at every host poll the
// workgroups are re-split among the systems still running (team size of
// system s proportional to nnz_s^exponent), so the large, slow-converging
// systems get the whole chip once the small ones are done.  Workgroups of
// one kernel never wait for each other, so no agent-scope fence (an L2
// write-back on this chip) is ever needed, and nothing can deadlock.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "common.hpp"
#include "device.hpp"
#include "solver_core.hpp"
#include "spmv_core.hpp"

namespace spx {
namespace {

using namespace solver;

struct BatchSys {
  int64_t n, off;
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  const int32_t* dpos;
};

// plan layout (int32): wg_sys[G] | team_start[nsys] | team_size[nsys]
struct PlanView {
  const int32_t* p;
  int G, nsys;
  __device__ int sys(int b) const { return p[b]; }
  __device__ int start(int s) const { return p[G + s]; }
  __device__ int size(int s) const { return p[G + nsys + s]; }
};

__global__ void k_b_reset(CgScalars* st, int nsys, int32_t maxit) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nsys) {
    CgScalars z = {};
    z.maxit = maxit;
    st[s] = z;
  }
}

__global__ __launch_bounds__(kBlock) void k_b_dinv(const BatchSys* __restrict__ sys, PlanView pl,
                                                   double* __restrict__ dinv, CgScalars* st) {
  const int s = pl.sys(blockIdx.x);
  if (s < 0) return;
  const BatchSys S = sys[s];
  const Range rg = block_range(S.n, blockIdx.x - pl.start(s), pl.size(s));
  for (int64_t r = rg.lo + threadIdx.x; r < rg.hi; r += kBlock) {
    const int32_t t = S.dpos[r];
    const double d = t >= 0 ? S.val[t] : 0.0;
    if (d == 0.0) st[s].status = SPX_ZERO_DIAGONAL;
    dinv[S.off + r] = d == 0.0 ? 0.0 : 1.0 / d;
  }
}

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
                                       });
  rz = block_sum<kBlock>(rz, lds);
  rr = block_sum<kBlock>(rr, lds);
  bb = block_sum<kBlock>(bb, lds);
  if (threadIdx.x == 0) {
    P[blockIdx.x] = rz;
    P[pl.G + blockIdx.x] = rr;
    P[2 * pl.G + blockIdx.x] = bb;
  }
}

// one workgroup per system
__global__ __launch_bounds__(kBlock) void k_b_init_finish(PlanView pl, CgScalars* st,
                                                          const double* __restrict__ P,
                                                          double rtol) {
  __shared__ double lds[kLds];
  const int s = blockIdx.x;
  const int a = pl.start(s), T = pl.size(s);
  const double rz = reduce_all(P + a, T, lds);
  const double rr = reduce_all(P + pl.G + a, T, lds);
  const double bb = reduce_all(P + 2 * pl.G + a, T, lds);
  if (threadIdx.x == 0) {
    CgScalars& c = st[s];
    c.rho[0] = rz;
    c.bb = bb;
    c.bnorm = sqrt(bb);
    c.thresh = rtol * c.bnorm;
    c.rr = rr;
    c.iters = 0;
    if (c.status != SPX_OK) {
      c.done = 1;
    } else if (sqrt(rr) <= c.thresh) {
      c.done = 1;
    } else if (c.maxit <= 0) {
      c.done = 1;
      c.status = SPX_NOT_CONVERGED;
    } else {
      c.done = 0;
    }
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
                                       });
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
  if (s < 0 || st[s].done) return;
  const int a = pl.start(s), T = pl.size(s);
  const int64_t j = blockIdx.x - a;
  const double pq = reduce_all(P1 + a, T, lds);
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
  if (s < 0 || st[s].done) return;
  const int a = pl.start(s), T = pl.size(s);
  const int64_t j = blockIdx.x - a;
  const double rz = reduce_all(P2 + a, T, lds);
  const double rr = reduce_all(P2 + pl.G + a, T, lds);
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

template <class SH>
__global__ __launch_bounds__(kBlock) void k_b_resnorm(const BatchSys* __restrict__ sys, PlanView pl,
                                                      const double* __restrict__ b,
                                                      const double* __restrict__ x,
                                                      double* __restrict__ P, int rows) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double lds[kLds];
  const int s = pl.sys(blockIdx.x);
  if (s < 0) return;
  const BatchSys S = sys[s];
  const int64_t o = S.off;
  double rr = 0.0;
  for_rows<SH, double, double, double>(S.n, S.rowptr, S.col, S.val, x + o, rows,
                                       blockIdx.x - pl.start(s), pl.size(s),
                                       reinterpret_cast<double*>(smem), [&](int64_t row, double ax) {
                                         const double ri = b[o + row] - ax;
                                         rr += ri * ri;
                                       });
  rr = block_sum<kBlock>(rr, lds);
  if (threadIdx.x == 0) P[blockIdx.x] = rr;
}

__global__ __launch_bounds__(kBlock) void k_b_resnorm_finish(PlanView pl, CgScalars* st,
                                                             const double* __restrict__ P) {
  __shared__ double lds[kLds];
  const int s = blockIdx.x;
  const double rr = reduce_all(P + pl.start(s), pl.size(s), lds);
  if (threadIdx.x == 0) st[s].rr_true = rr;
}

}  // namespace
}  // namespace spx

using namespace spx;
using namespace spx::solver;

struct spx_batch {
  int device = 0;
  int nsys = 0;
  std::vector<spx_handle> hs;
  std::vector<BatchSys> sys;
  int64_t total = 0;
  int64_t max_tile[4] = {0, 0, 0, 0};
  int64_t max_row = 0, max_nnz_sys = 0;
  BatchSys* d_sys = nullptr;
  double* work = nullptr;  // r, p, q, dinv (4 * total)
  CgScalars* d_st = nullptr;
  CgScalars* h_st = nullptr;  // pinned
  int32_t* d_plan = nullptr;
  int32_t* h_plan = nullptr;  // pinned
  int plan_cap = 0;
  double* partials = nullptr;
  int partial_cap = 0;
};

namespace {

int cu_count_b() {
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  return cus;
}

// Splits G workgroups among the active systems: team size proportional to
// nnz_s^gamma, at least one workgroup each, teams contiguous in system order.
void make_plan(const spx_batch* B, const std::vector<char>& active, int G, double gamma,
               int32_t* plan) {
  const int ns = B->nsys;
  std::vector<double> w(ns, 0.0);
  double wsum = 0.0;
  int nact = 0;
  for (int s = 0; s < ns; ++s)
    if (active[s]) {
      w[s] = std::pow((double)std::max<int64_t>(1, B->hs[s]->A.nnz), gamma);
      wsum += w[s];
      ++nact;
    }
  std::vector<int> T(ns, 0);
  int used = 0;
  for (int s = 0; s < ns; ++s)
    if (active[s]) {
      const int extra = G - nact;  // beyond the guaranteed one workgroup each
      T[s] = 1 + (int)std::floor(extra * w[s] / wsum);
      used += T[s];
    }
  // hand out the rounding remainder to the heaviest systems
  while (used < G && nact > 0) {
    int best = -1;
    for (int s = 0; s < ns; ++s)
      if (active[s] && (best < 0 || w[s] / T[s] > w[best] / T[best])) best = s;
    ++T[best];
    ++used;
  }
  int32_t* wg = plan;
  int32_t* start = plan + G;
  int32_t* size = plan + G + ns;
  int b = 0;
  for (int s = 0; s < ns; ++s) {
    start[s] = b;
    size[s] = T[s];
    for (int k = 0; k < T[s]; ++k) wg[b++] = s;
  }
  for (; b < G; ++b) wg[b] = -1;
}

SpmvShape batch_shape(const spx_batch* B, int rows_opt) {
  SpmvShape sh;
  sh.nt = 1;
  sh.vec = 0;
  sh.lanes = 1;
  sh.rows = 0;
  sh.lds = 0;
  sh.variant = kVariantVector;
  auto idx = [](int rows) { return rows == 32 ? 0 : rows == 64 ? 1 : rows == 128 ? 2 : 3; };
  const int cands[4] = {256, 128, 64, 32};
  for (int rows : cands) {
    if (rows_opt && rows != rows_opt) continue;
    const size_t lds = (size_t)(B->max_tile[idx(rows)] + 8) * sizeof(double);
    if (lds <= (rows_opt ? 64 * 1024 : 40 * 1024)) {
      sh.variant = kVariantStream;
      sh.rows = rows;
      sh.lds = lds;
      return sh;
    }
  }
  int L = 1;
  const double mean = 5.0;
  while (L < 64 && 2.0 * L < std::max<double>(mean, (double)B->max_row / 4)) L <<= 1;
  sh.lanes = L;
  return sh;
}

int upload_plan(spx_batch* B, int G, hipStream_t s) {
  const size_t bytes = sizeof(int32_t) * (size_t)(G + 2 * B->nsys);
  SPX_CHECK_HIP(hipMemcpyAsync(B->d_plan, B->h_plan, bytes, hipMemcpyHostToDevice, s));
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
    B->sys.push_back(S);
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
    if (hipHostMalloc(reinterpret_cast<void**>(&B->h_st), sizeof(CgScalars) * (size_t)nsys,
                      hipHostMallocDefault) != hipSuccess) {
      st = set_error(SPX_OUT_OF_MEMORY, "batch_create: pinned allocation failed");
      break;
    }
    if (hipMemcpyAsync(B->d_sys, B->sys.data(), sizeof(BatchSys) * (size_t)nsys,
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
  int G = (tuning && tuning->blocks > 0) ? tuning->blocks : cu_count_b() * 8;
  G = std::max(G, ns);
  const double gamma = (tuning && tuning->weight_exponent > 0.0) ? tuning->weight_exponent : 1.0;
  const int check_every = (tuning && tuning->check_every > 0) ? tuning->check_every : 20;
  const int rows_opt = tuning ? tuning->rows_per_tile : 0;
  if (rows_opt != 0 && rows_opt != 32 && rows_opt != 64 && rows_opt != 128 && rows_opt != 256)
    return set_error(SPX_INVALID_ARG, "batch_cg: rows_per_tile must be 0, 32, 64, 128 or 256");
  const SpmvShape sh = batch_shape(B, rows_opt);
  const size_t lds = sh.variant == kVariantStream ? sh.lds : 0;

  const int plan_n = G + 2 * ns;
  if (B->plan_cap < plan_n) {
    dfree(B->d_plan);
    B->d_plan = nullptr;
    if (B->h_plan) (void)hipHostFree(B->h_plan);
    B->h_plan = nullptr;
    SPX_TRY(dalloc_n(&B->d_plan, (size_t)plan_n));
    SPX_CHECK_HIP(hipHostMalloc(reinterpret_cast<void**>(&B->h_plan), sizeof(int32_t) * plan_n,
                                hipHostMallocDefault));
    B->plan_cap = plan_n;
  }
  if (B->partial_cap < 3 * G) {
    dfree(B->partials);
    B->partials = nullptr;
    SPX_TRY(dalloc_n(&B->partials, (size_t)3 * G));
    B->partial_cap = 3 * G;
  }
  const int64_t tot = B->total;
  double* r = B->work;
  double* p = B->work + tot;
  double* q = B->work + 2 * tot;
  double* dinv = B->work + 3 * tot;
  double* P1 = B->partials;
  double* P2 = B->partials + G;
  const PlanView pl{B->d_plan, G, ns};

  std::vector<char> active(ns, 1);
  make_plan(B, active, G, gamma, B->h_plan);
  SPX_TRY(upload_plan(B, G, s));
  hipLaunchKernelGGL(k_b_reset, dim3((unsigned)ceil_div(ns, 64)), dim3(64), 0, s, B->d_st, ns,
                     (int32_t)maxit);
  hipLaunchKernelGGL(k_b_dinv, dim3(G), dim3(kBlock), 0, s, B->d_sys, pl, dinv, B->d_st);
  SPX_TRY(with_shape(sh, [&](auto shc) {
    using SH = decltype(shc);
    hipLaunchKernelGGL((k_b_init<SH>), dim3(G), dim3(kBlock), lds, s, B->d_sys, pl, bvec, x, r, p,
                       dinv, B->partials, sh.rows);
    return SPX_OK;
  }));
  hipLaunchKernelGGL(k_b_init_finish, dim3(ns), dim3(kBlock), 0, s, pl, B->d_st, B->partials, rtol);
  SPX_CHECK_HIP(hipGetLastError());

  int64_t k = 0;
  for (;;) {
    SPX_CHECK_HIP(hipMemcpyAsync(B->h_st, B->d_st, sizeof(CgScalars) * ns, hipMemcpyDeviceToHost, s));
    SPX_CHECK_HIP(hipStreamSynchronize(s));
    std::vector<char> now(ns, 0);
    int nact = 0;
    for (int t = 0; t < ns; ++t) {
      now[t] = B->h_st[t].done ? 0 : 1;
      nact += now[t];
    }
    if (nact == 0 || k >= maxit) break;
    if (now != active) {
      active = now;
      make_plan(B, active, G, gamma, B->h_plan);
      SPX_TRY(upload_plan(B, G, s));
    }
    const int64_t m = std::min<int64_t>(check_every, maxit - k);
    SPX_TRY(with_shape(sh, [&](auto shc) {
      using SH = decltype(shc);
      for (int64_t c = 0; c < m; ++c) {
        const int64_t kk = k + c + 1;
        hipLaunchKernelGGL((k_b_spmv<SH>), dim3(G), dim3(kBlock), lds, s, B->d_sys, pl, p, q,
                           B->d_st, P1, sh.rows);
        hipLaunchKernelGGL(k_b_update, dim3(G), dim3(kBlock), 0, s, B->d_sys, pl, x, r, p, q, dinv,
                           B->d_st, P1, P2, kk);
        hipLaunchKernelGGL(k_b_pupdate, dim3(G), dim3(kBlock), 0, s, B->d_sys, pl, p, r, dinv,
                           B->d_st, P2, kk);
      }
      return SPX_OK;
    }));
    SPX_CHECK_HIP(hipGetLastError());
    k += m;
  }
  // true residuals with every system in the plan
  std::fill(active.begin(), active.end(), 1);
  make_plan(B, active, G, gamma, B->h_plan);
  SPX_TRY(upload_plan(B, G, s));
  SPX_TRY(with_shape(sh, [&](auto shc) {
    using SH = decltype(shc);
    hipLaunchKernelGGL((k_b_resnorm<SH>), dim3(G), dim3(kBlock), lds, s, B->d_sys, pl, bvec, x,
                       B->partials, sh.rows);
    return SPX_OK;
  }));
  hipLaunchKernelGGL(k_b_resnorm_finish, dim3(ns), dim3(kBlock), 0, s, pl, B->d_st, B->partials);
  SPX_CHECK_HIP(hipMemcpyAsync(B->h_st, B->d_st, sizeof(CgScalars) * ns, hipMemcpyDeviceToHost, s));
  SPX_CHECK_HIP(hipStreamSynchronize(s));
  int status = SPX_OK;
  for (int t = 0; t < ns; ++t) {
    const CgScalars& c = B->h_st[t];
    if (iters_out) iters_out[t] = c.iters;
    if (relres_out) relres_out[t] = c.bnorm > 0.0 ? sqrt(c.rr_true) / c.bnorm : sqrt(c.rr_true);
    int st_t = c.status;
    if (st_t == SPX_OK && !c.done) st_t = SPX_NOT_CONVERGED;
    if (st_t != SPX_OK && (status == SPX_OK || status == SPX_NOT_CONVERGED)) status = st_t;
  }
  if (status != SPX_OK)
    return set_error(status, "batch_cg: at least one system ended with status %d", status);
  return SPX_OK;
}
