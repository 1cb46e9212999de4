// Shared machinery of the batched solvers (paper Sec. 7: one batched Krylov
// solver with a diagonal preconditioner for many small systems, instead of
// one stacked "ensemble" system).
//
// All systems advance together, one iteration at a time, and each phase of
// an iteration is ONE launch for the whole batch: the grid's workgroups are
// split into teams, one team per still-running system, and a team walks its
// system exactly as the single-system kernels do (same row walk, same
// partial sums re-added by the next launch).  A system that has stopped
// stops consuming bandwidth, and at every host poll the workgroups are
// re-split among the systems still running (team size of system s
// proportional to nnz_s^exponent), so the large, slow-converging systems
// get the whole chip once the small ones are done.  Workgroups of one
// kernel never wait for each other: no agent-scope fence, no co-residency.
//
// The persistent form (below, and cg_one.hpp / krylov_one.hpp) launches
// once: each workgroup takes whole systems from a queue and runs the method
// on them alone, which pays off for many small systems.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "solver_core.hpp"

namespace spx {
namespace batch {

struct BatchSys {
  int64_t n, off;
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  const int32_t* dpos;
  WinView win;  // the system's window index (used when every system has one)
};

// plan layout (int32): wg_sys[G] | team_start[nsys] | team_size[nsys]
struct PlanView {
  const int32_t* p;
  int G, nsys;
  __device__ int sys(int b) const { return p[b]; }
  __device__ int start(int s) const { return p[G + s]; }
  __device__ int size(int s) const { return p[G + nsys + s]; }
};

}  // namespace batch
}  // namespace spx

struct spx_batch {
  int device = 0;
  int nsys = 0;
  std::vector<spx_handle> hs;
  std::vector<spx::batch::BatchSys> sys;
  int64_t total = 0;
  int64_t max_tile[4] = {0, 0, 0, 0};
  int64_t max_row = 0, max_nnz_sys = 0;
  int64_t win_blocks = 0;  // largest window of any system; -1 when one has no index
  spx::batch::BatchSys* d_sys = nullptr;
  double* work = nullptr;  // CG: r, p, q, dinv (4 * total)
  spx::CgScalars* d_st = nullptr;
  spx::CgScalars* h_st = nullptr;  // pinned
  int32_t* d_plan = nullptr;
  int32_t* h_plan = nullptr;  // pinned
  int plan_cap = 0;
  double* partials = nullptr;
  int partial_cap = 0;
  // non-symmetric solvers (lazy)
  spx::batch::BatchSys* d_sysT = nullptr;  // transposes, for BiCG
  int64_t max_tile_t[4] = {0, 0, 0, 0};
  int64_t max_row_t = 0;
  int64_t win_blocks_t = 0;
  double* kwork = nullptr;  // 8 * total
  // persistent solve: [0] the next queue position, [1 + k] the k-th system
  // to take (largest first)
  int32_t* d_queue = nullptr;
};

namespace spx {
namespace batch {

// Splits G workgroups among the active systems: team size proportional to
// nnz_s^gamma, at least one workgroup each, teams contiguous in system order.
inline void make_plan(const spx_batch* B, const std::vector<char>& active, int G, double gamma,
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

// Row walk of the batch: the window walk when every system (and, for BiCG,
// every transpose) has a window index (win_blocks > 0: the largest window)
// and no row count was asked for; else the stream walk with the largest
// tile that fits every system's tiles in LDS; else the lane walk.
inline SpmvShape batch_shape(const int64_t max_tile[4], int64_t max_row, int rows_opt,
                             int64_t win_blocks) {
  SpmvShape sh;
  sh.nt = 1;
  sh.vec = 0;
  sh.pipe = 0;
  sh.tile = 0;
  sh.lanes = 1;
  sh.rows = 0;
  sh.lds = 0;
  sh.variant = kVariantVector;
  if (win_blocks > 0 && rows_opt == 0) {
    sh.variant = kVariantWindow;
    sh.rows = kWinRows;
    sh.tile = win_blocks * kWinBlock;
    sh.lds = window_lds_bytes(win_blocks, sizeof(double),
                              win_u_solver<double>() * win_v<double>());
    return sh;
  }
  auto idx = [](int rows) { return rows == 32 ? 0 : rows == 64 ? 1 : rows == 128 ? 2 : 3; };
  const int cands[4] = {256, 128, 64, 32};
  for (int rows : cands) {
    if (rows_opt && rows != rows_opt) continue;
    const size_t lds = (size_t)(max_tile[idx(rows)] + 8) * sizeof(double);
    if (lds <= (rows_opt ? 64 * 1024 : 40 * 1024)) {
      sh.variant = kVariantStream;
      sh.rows = rows;
      sh.lds = lds;
      return sh;
    }
  }
  int L = 1;
  const double mean = 5.0;
  while (L < 64 && 2.0 * L < std::max<double>(mean, (double)max_row / 4)) L <<= 1;
  sh.lanes = L;
  return sh;
}

inline int upload_plan(spx_batch* B, int G, hipStream_t s) {
  const size_t bytes = sizeof(int32_t) * (size_t)(G + 2 * B->nsys);
  SPX_CHECK_HIP(hipMemcpyAsync(B->d_plan, B->h_plan, bytes, hipMemcpyHostToDevice, s));
  return SPX_OK;
}

// Launch parameters of one batched solve.
struct Run {
  int G = 0;
  double gamma = 1.0;
  int check_every = 20;
  SpmvShape sh;
  size_t lds = 0;
  PlanView pl;
};

// Validates the tuning, sizes the plan and `sets` partial arrays of G
// doubles, and uploads the plan with every system active.
inline int prepare(spx_batch* B, const spx_batch_tuning* tuning, const int64_t max_tile[4],
                   int64_t max_row, int64_t win_blocks, int sets, hipStream_t s, Run* run) {
  const int ns = B->nsys;
  int G = (tuning && tuning->blocks > 0) ? tuning->blocks : cu_count() * 8;
  G = std::max(G, ns);
  run->G = G;
  run->gamma = (tuning && tuning->weight_exponent > 0.0) ? tuning->weight_exponent : 1.0;
  run->check_every = (tuning && tuning->check_every > 0) ? tuning->check_every : 20;
  const int rows_opt = tuning ? tuning->rows_per_tile : 0;
  if (rows_opt != 0 && rows_opt != 32 && rows_opt != 64 && rows_opt != 128 && rows_opt != 256)
    return set_error(SPX_INVALID_ARG, "batch: rows_per_tile must be 0, 32, 64, 128 or 256");
  run->sh = batch_shape(max_tile, max_row, rows_opt, win_blocks);
  run->lds = (run->sh.variant == kVariantStream || run->sh.variant == kVariantWindow) ? run->sh.lds
                                                                                      : 0;
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
  if (B->partial_cap < sets * G) {
    dfree(B->partials);
    B->partials = nullptr;
    SPX_TRY(dalloc_n(&B->partials, (size_t)sets * G));
    B->partial_cap = sets * G;
  }
  run->pl = PlanView{B->d_plan, G, ns};
  std::vector<char> all(ns, 1);
  make_plan(B, all, G, run->gamma, B->h_plan);
  return upload_plan(B, G, s);
}

struct NoHook {
  int operator()(int64_t, bool*) const { return SPX_OK; }
};

// Polls the per-system state, re-splits the grid when the set of running
// systems changed, and enqueues chunks of `check_every` iterations with
// enq(first, count) (1-based iteration numbers) until every system is done
// or `max_iters` iterations were enqueued.  hook(k, &relaunched) runs at
// every poll on the freshly read state, k iterations in; when it enqueues
// work it sets relaunched and the state is read again.
template <typename Enq, typename Hook = NoHook>
int poll_loop(spx_batch* B, Run& run, int64_t max_iters, hipStream_t s, Enq&& enq,
              Hook&& hook = Hook()) {
  const int ns = B->nsys;
  std::vector<char> active(ns, 1);
  int64_t k = 0;
  for (;;) {
    SPX_CHECK_HIP(
        hipMemcpyAsync(B->h_st, B->d_st, sizeof(CgScalars) * ns, hipMemcpyDeviceToHost, s));
    SPX_CHECK_HIP(hipStreamSynchronize(s));
    bool relaunched = false;
    SPX_TRY(hook(k, &relaunched));
    if (relaunched) {
      SPX_CHECK_HIP(
          hipMemcpyAsync(B->h_st, B->d_st, sizeof(CgScalars) * ns, hipMemcpyDeviceToHost, s));
      SPX_CHECK_HIP(hipStreamSynchronize(s));
    }
    std::vector<char> now(ns, 0);
    int nact = 0;
    for (int t = 0; t < ns; ++t) {
      now[t] = B->h_st[t].done ? 0 : 1;
      nact += now[t];
    }
    if (nact == 0 || k >= max_iters) break;
    if (now != active) {
      active = now;
      make_plan(B, active, run.G, run.gamma, B->h_plan);
      SPX_TRY(upload_plan(B, run.G, s));
    }
    const int64_t m = std::min<int64_t>(run.check_every, max_iters - k);
    SPX_TRY(enq(k + 1, m));
    SPX_CHECK_HIP(hipGetLastError());
    k += m;
  }
  // every system back in the plan for the final residuals
  std::vector<char> all(ns, 1);
  make_plan(B, all, run.G, run.gamma, B->h_plan);
  return upload_plan(B, run.G, s);
}

// ------------------------------------------------------- persistent form
// Shape of the persistent solve (one launch, each workgroup solving whole
// systems from the queue): workgroup size, rows per tile and the dynamic LDS
// for the products of the largest such tile of any system.  tile256 bounds
// the entries of a 256-row tile of every matrix the solve walks; 512 and
// 1024 rows take 2 and 4 of them.  256 threads for systems of at most 1024
// rows (more systems in flight), 1024 above (each system faster); lds 0
// when not even a 256-row tile fits 64 KB.
struct PersistShape {
  int block = 256, rows = 256;
  size_t lds = 0;
};
inline PersistShape persistent_shape(const spx_batch* B, int64_t tile256) {
  PersistShape ps;
  int64_t max_n = 0;
  for (const BatchSys& S : B->sys) max_n = std::max(max_n, S.n);
  auto bytes = [&](int64_t tiles) { return (size_t)(tiles * tile256 + 8) * sizeof(double); };
  if (bytes(1) > 64 * 1024) return ps;
  if (max_n > 1024) {
    ps.block = 1024;
    ps.rows = bytes(4) <= 64 * 1024 ? 1024 : bytes(2) <= 64 * 1024 ? 512 : 256;
  }
  ps.lds = bytes(ps.rows / 256);
  return ps;
}

// The persistent solve pays off when there are enough systems to keep the
// workgroups busy and each is small enough for one workgroup: at least
// kPersistAutoSystems systems, none above kPersistAutoRows rows.  Measured
// with CG on 5-point batches (persistent vs one launch per phase): 4096
// systems of 16-256 rows 6.5x, 1024 of 64-1024 rows 2.0x, 2048 of 256-4096
// 1.8x, 256 of 1024-4096 1.2x, 1024 of 1024-8100 1.4x; 512 of 4096-16384
// 0.91x, and 64 of 1024-262144 0.05x (the largest system alone on one
// workgroup).
constexpr int kPersistAutoSystems = 256;
constexpr int64_t kPersistAutoRows = 8192;
inline bool persistent_by_default(const spx_batch* B, const PersistShape& ps) {
  if (B->nsys < kPersistAutoSystems || ps.lds == 0) return false;
  for (const BatchSys& S : B->sys)
    if (S.n > kPersistAutoRows) return false;
  return true;
}

inline int persistent_mode(const spx_batch_tuning* tuning, const char* what, int32_t* mode) {
  *mode = tuning ? tuning->persistent : 0;
  if (*mode < -1 || *mode > 1)
    return set_error(SPX_INVALID_ARG, "%s: persistent must be -1, 0 or 1", what);
  return SPX_OK;
}

// Copies the final state out and folds the per-system statuses.
inline int finish(spx_batch* B, hipStream_t s, int64_t* iters_out, double* relres_out,
                  const char* what) {
  const int ns = B->nsys;
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
    return set_error(status, "%s: at least one system ended with status %d", what, status);
  return SPX_OK;
}

// ---------------------------------------------------------------- kernels
// shared by every batched method (one copy per translation unit)
namespace {

__global__ void k_b_queue_reset(int32_t* queue) {
  if (threadIdx.x == 0) queue[0] = 0;
}

__global__ void k_b_reset(CgScalars* st, int nsys, int32_t maxit) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nsys) {
    CgScalars z = {};
    z.maxit = maxit;
    z.stop_pos = INT32_MAX;
    st[s] = z;
  }
}

__global__ __launch_bounds__(solver::kBlock) void k_b_dinv(const BatchSys* __restrict__ sys,
                                                           PlanView pl, double* __restrict__ dinv,
                                                           CgScalars* st) {
  using namespace solver;
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

// Start of a CG-type solve, one workgroup per system: rho_0 = r.z, the
// threshold rtol ||b||, and systems that need no iteration marked done.
__global__ __launch_bounds__(solver::kBlock) void k_b_init_finish(PlanView pl, CgScalars* st,
                                                          const double* __restrict__ P,
                                                          double rtol) {
  using namespace solver;
  __shared__ double lds[kLds];
  const int s = blockIdx.x;
  const int a = pl.start(s), T = pl.size(s);
  double rz, rr, bb;
  reduce_all(P + a, P + pl.G + a, P + 2 * pl.G + a, T, lds, rz, rr, bb);
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

// partials of ||b - A x||^2
template <class SH>
__global__ __launch_bounds__(solver::kBlock) void k_b_resnorm(const BatchSys* __restrict__ sys,
                                                              PlanView pl,
                                                              const double* __restrict__ b,
                                                              const double* __restrict__ x,
                                                              double* __restrict__ P, int rows) {
  using namespace solver;
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
                                       }, 0, S.win);
  rr = block_sum<kBlock>(rr, lds);
  if (threadIdx.x == 0) P[blockIdx.x] = rr;
}

__global__ __launch_bounds__(solver::kBlock) void k_b_resnorm_finish(PlanView pl, CgScalars* st,
                                                                     const double* __restrict__ P) {
  using namespace solver;
  __shared__ double lds[kLds];
  const int s = blockIdx.x;
  const double rr = reduce_all(P + pl.start(s), pl.size(s), lds);
  if (threadIdx.x == 0) st[s].rr_true = rr;
}

}  // namespace

// True residuals of every system (the plan must hold all of them).
inline int true_residuals(spx_batch* B, const Run& run, const double* bvec, const double* x,
                          hipStream_t s) {
  SPX_TRY(solver::with_shape<true>(run.sh, [&](auto shc) {
    using SH = decltype(shc);
    hipLaunchKernelGGL((k_b_resnorm<SH>), dim3(run.G), dim3(solver::kBlock), run.lds, s, B->d_sys,
                       run.pl, bvec, x, B->partials, run.sh.rows);
    return SPX_OK;
  }));
  hipLaunchKernelGGL(k_b_resnorm_finish, dim3(B->nsys), dim3(solver::kBlock), 0, s, run.pl,
                     B->d_st, B->partials);
  SPX_CHECK_HIP(hipGetLastError());
  return SPX_OK;
}

}  // namespace batch
}  // namespace spx
