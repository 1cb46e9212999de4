// Batched non-symmetric Krylov solvers with diagonal preconditioning
// (paper Sec. 7 names TFQMR and BiCG as the two batched methods), on the
// team machinery of batch.hpp: every phase of an iteration is one launch for
// the whole batch, re-split among the running systems at every poll.
//
// BiCG (left Jacobi, shadow residual started at r): 3 launches per
// iteration, q = A p and qh = A^T p-hat in one launch (the team walks its
// system's rows, then the rows of its explicit transpose).  On a symmetric
// system it performs the batched CG's arithmetic exactly.
//
// TFQMR (right Jacobi, x-space search direction): 4 launches per iteration
// of two half-steps, two of them row walks:
//   KA  au = A uh;  v = au + beta (t + beta v);  partials of rs.v
//   KB  alpha; w -= alpha au; d = uh + (theta^2 eta / alpha) d;
//       u -= alpha v; uh = D^-1 u;  partials of w.w
//   KC  theta, tau, eta of half-step 1; x += eta d; test;
//       d = uh + (theta^2 eta / alpha) d; t = A uh; w -= alpha t;
//       partials of w.w and rs.w
//   KD  theta, tau, eta of half-step 2; x += eta d; test; rho, beta;
//       u = w + beta u; uh = D^-1 u
// Scalars a launch reads while its first workgroup writes them live in
// alternating slots (rho, tau).  KC and KD update x after their stopping
// test, so a later workgroup of the same launch must not skip its rows when
// the first one has already marked the system done: launches compare the
// recorded stop position with their own instead of reading `done`.
// A cycle that ends on the method's residual bound is only a candidate: at
// the next host poll the true residual of x decides between done and a new
// cycle from x (the bound holds in exact arithmetic only, and the large
// intermediate residuals of this method can leave x far above it).
#include <algorithm>
#include <climits>
#include <cmath>
#include <type_traits>
#include <vector>

#include "batch.hpp"
#include "common.hpp"
#include "krylov_one.hpp"
#include "device.hpp"
#include "solver_core.hpp"
#include "spmv_core.hpp"

namespace spx {
namespace {

using namespace solver;
using namespace batch;

// ------------------------------------------------------------------ BiCG

// r = b - A x; rh = r; p = ph = D^-1 r; partials of r.z, r.r, b.b
template <class SH>
__global__ __launch_bounds__(kBlock) void k_bb_init(const BatchSys* __restrict__ sys, PlanView pl,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ r, double* __restrict__ rh,
                                                    double* __restrict__ p, double* __restrict__ ph,
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
                                         rh[o + row] = ri;
                                         p[o + row] = zi;
                                         ph[o + row] = zi;
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

// q = A p, qh = A^T ph; partials of ph.q
template <class SH>
__global__ __launch_bounds__(kBlock) void k_bb_spmv(const BatchSys* __restrict__ sys,
                                                    const BatchSys* __restrict__ sysT, PlanView pl,
                                                    const double* __restrict__ p,
                                                    const double* __restrict__ ph,
                                                    double* __restrict__ q, double* __restrict__ qh,
                                                    const CgScalars* __restrict__ st,
                                                    double* __restrict__ P1, int rows) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double lds[kLds];
  const int s = pl.sys(blockIdx.x);
  if (s < 0 || st[s].done) return;
  const BatchSys S = sys[s];
  const BatchSys T = sysT[s];
  const int64_t o = S.off;
  const int64_t lb = blockIdx.x - pl.start(s);
  double dot = 0.0;
  for_rows<SH, double, double, double>(S.n, S.rowptr, S.col, S.val, p + o, rows, lb, pl.size(s),
                                       reinterpret_cast<double*>(smem), [&](int64_t row, double v) {
                                         q[o + row] = v;
                                         dot += ph[o + row] * v;
                                       }, 0, S.win);
  __syncthreads();  // the staging area is reused by the second walk
  for_rows<SH, double, double, double>(T.n, T.rowptr, T.col, T.val, ph + o, rows, lb, pl.size(s),
                                       reinterpret_cast<double*>(smem),
                                       [&](int64_t row, double v) { qh[o + row] = v; }, 0, T.win);
  dot = block_sum<kBlock>(dot, lds);
  if (threadIdx.x == 0) P1[blockIdx.x] = dot;
}

// alpha = rho / ph.q; x += alpha p; r -= alpha q; rh -= alpha qh;
// partials of (D^-1 r).rh and r.r
__global__ __launch_bounds__(kBlock) void k_bb_update(const BatchSys* __restrict__ sys, PlanView pl,
                                                      double* __restrict__ x, double* __restrict__ r,
                                                      double* __restrict__ rh,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ q,
                                                      const double* __restrict__ qh,
                                                      const double* __restrict__ dinv,
                                                      CgScalars* st, const double* __restrict__ P1,
                                                      double* __restrict__ P2, int64_t k) {
  __shared__ double lds[kLds];
  const int s = pl.sys(blockIdx.x);
  if (s < 0) return;
  const auto done = st[s].done;  // tested once the partials are in
  const int a = pl.start(s), T = pl.size(s);
  const int64_t j = blockIdx.x - a;
  const double sigma = reduce_all(P1 + a, T, lds);
  if (done) return;
  if (sigma == 0.0 || !isfinite(sigma)) {
    if (j == 0 && threadIdx.x == 0) {
      st[s].pq = sigma;
      st[s].status = SPX_BREAKDOWN;
      st[s].iters = (int32_t)(k - 1);
      st[s].done = 1;
    }
    return;
  }
  const double alpha = st[s].rho[(k - 1) & 1] / sigma;
  const BatchSys S = sys[s];
  const int64_t o = S.off;
  const Range rg = block_range(S.n, j, T);
  double rz = 0.0, rr = 0.0;
  for (int64_t i = o + rg.lo + threadIdx.x; i < o + rg.hi; i += kBlock) {
    const double xi = x[i] + alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    const double rhi = rh[i] - alpha * qh[i];
    const double zi = dinv[i] * ri;
    x[i] = xi;
    r[i] = ri;
    rh[i] = rhi;
    rz += rhi * zi;
    rr += ri * ri;
  }
  rz = block_sum<kBlock>(rz, lds);
  rr = block_sum<kBlock>(rr, lds);
  if (threadIdx.x == 0) {
    P2[blockIdx.x] = rz;
    P2[pl.G + blockIdx.x] = rr;
  }
}

// test ||r||; beta = rho' / rho; p = D^-1 r + beta p; ph = D^-1 rh + beta ph
__global__ __launch_bounds__(kBlock) void k_bb_pupdate(const BatchSys* __restrict__ sys,
                                                       PlanView pl, double* __restrict__ p,
                                                       double* __restrict__ ph,
                                                       const double* __restrict__ r,
                                                       const double* __restrict__ rh,
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
  const bool broke = !conv && (rz == 0.0 || !isfinite(rz));
  const bool stop = conv || broke || k >= c.maxit;
  const double rho_prev = c.rho[(k - 1) & 1];
  if (j == 0 && threadIdx.x == 0) {
    c.rr = rr;
    c.iters = (int32_t)k;
    if (conv) {
      c.status = SPX_OK;
      c.done = 1;
    } else if (broke) {
      c.status = SPX_BREAKDOWN;
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
  for (int64_t i = o + rg.lo + threadIdx.x; i < o + rg.hi; i += kBlock) {
    p[i] = dinv[i] * r[i] + bt * p[i];
    ph[i] = dinv[i] * rh[i] + bt * ph[i];
  }
}

// ----------------------------------------------------------------- TFQMR

struct TqVecs {
  double *w, *u, *uh, *v, *au, *t, *d, *rs;
};

__device__ __forceinline__ bool tq_skip(const CgScalars& c, int64_t pos) {
  return (int64_t)c.stop_pos < pos;
}

// r0 = b - A x; w = u = rs = r0; uh = D^-1 r0; d = t = v = 0;
// partials of r0.r0 and b.b
template <class SH>
__global__ __launch_bounds__(kBlock) void k_tq_init(const BatchSys* __restrict__ sys, PlanView pl,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ x, TqVecs V,
                                                    const double* __restrict__ dinv,
                                                    double* __restrict__ P, int rows) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double lds[kLds];
  const int s = pl.sys(blockIdx.x);
  if (s < 0) return;
  const BatchSys S = sys[s];
  const int64_t o = S.off;
  double rr = 0.0, bb = 0.0;
  for_rows<SH, double, double, double>(S.n, S.rowptr, S.col, S.val, x + o, rows,
                                       blockIdx.x - pl.start(s), pl.size(s),
                                       reinterpret_cast<double*>(smem), [&](int64_t row, double ax) {
                                         const int64_t i = o + row;
                                         const double bi = b[i];
                                         const double ri = bi - ax;
                                         V.w[i] = ri;
                                         V.u[i] = ri;
                                         V.rs[i] = ri;
                                         V.uh[i] = dinv[i] * ri;
                                         V.d[i] = 0.0;
                                         V.t[i] = 0.0;
                                         V.v[i] = 0.0;
                                         rr += ri * ri;
                                         bb += bi * bi;
                                       }, 0, S.win);
  rr = block_sum<kBlock>(rr, lds);
  bb = block_sum<kBlock>(bb, lds);
  if (threadIdx.x == 0) {
    P[blockIdx.x] = rr;
    P[pl.G + blockIdx.x] = bb;
  }
}

// one workgroup per system: tau_0 = ||r0||, rho_0 = rs.r0 (= r0.r0)
__global__ __launch_bounds__(kBlock) void k_tq_init_finish(PlanView pl, CgScalars* st,
                                                           const double* __restrict__ P,
                                                           double rtol) {
  __shared__ double lds[kLds];
  const int s = blockIdx.x;
  const int a = pl.start(s), T = pl.size(s);
  double rr, bb;
  reduce_all(P + a, P + pl.G + a, T, lds, rr, bb);
  if (threadIdx.x == 0) {
    CgScalars& c = st[s];
    c.rho[0] = rr;
    c.tau[0] = sqrt(rr);
    c.theta = 0.0;
    c.eta = 0.0;
    c.beta = 0.0;
    c.bb = bb;
    c.bnorm = sqrt(bb);
    c.thresh = rtol * c.bnorm;
    c.rr = rr;
    c.iters = 0;
    bool done = true;
    if (c.status != SPX_OK) {
    } else if (c.tau[0] <= c.thresh) {
    } else if (c.maxit <= 0) {
      c.status = SPX_NOT_CONVERGED;
    } else {
      done = false;
    }
    c.done = done ? 1 : 0;
    c.stop_pos = done ? -1 : INT32_MAX;
  }
}

// KA(j): au = A uh; v = au + beta (t + beta v); partials of rs.v
template <class SH>
__global__ __launch_bounds__(kBlock) void k_tq_a(const BatchSys* __restrict__ sys, PlanView pl,
                                                 TqVecs V, const CgScalars* __restrict__ st,
                                                 double* __restrict__ P0, int rows, int64_t pos) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double lds[kLds];
  const int s = pl.sys(blockIdx.x);
  if (s < 0 || tq_skip(st[s], pos)) return;
  const BatchSys S = sys[s];
  const int64_t o = S.off;
  const double beta = st[s].beta;
  double sig = 0.0;
  for_rows<SH, double, double, double>(S.n, S.rowptr, S.col, S.val, V.uh + o, rows,
                                       blockIdx.x - pl.start(s), pl.size(s),
                                       reinterpret_cast<double*>(smem), [&](int64_t row, double a) {
                                         const int64_t i = o + row;
                                         const double vi = a + beta * (V.t[i] + beta * V.v[i]);
                                         V.au[i] = a;
                                         V.v[i] = vi;
                                         sig += V.rs[i] * vi;
                                       }, 0, S.win);
  sig = block_sum<kBlock>(sig, lds);
  if (threadIdx.x == 0) P0[blockIdx.x] = sig;
}

// KB(j): first half-step without its scalar update
__global__ __launch_bounds__(kBlock) void k_tq_b(const BatchSys* __restrict__ sys, PlanView pl,
                                                 TqVecs V, const double* __restrict__ dinv,
                                                 CgScalars* st, const double* __restrict__ P0,
                                                 double* __restrict__ P1, int64_t j, int64_t pos) {
  __shared__ double lds[kLds];
  const int s = pl.sys(blockIdx.x);
  if (s < 0) return;
  const bool skip = tq_skip(st[s], pos);  // tested once the partials are in
  const int a = pl.start(s), T = pl.size(s);
  const int64_t jb = blockIdx.x - a;
  CgScalars& c = st[s];
  const double sigma = reduce_all(P0 + a, T, lds);
  if (skip) return;
  if (sigma == 0.0 || !isfinite(sigma)) {
    if (jb == 0 && threadIdx.x == 0) {
      c.pq = sigma;
      c.status = SPX_BREAKDOWN;
      c.iters = (int32_t)(c.m0 + 2 * (j - c.j0));
      c.done = 1;
      c.stop_pos = (int32_t)pos;
    }
    return;
  }
  const double alpha = c.rho[j & 1] / sigma;
  const double coef = c.theta * c.theta * c.eta / alpha;
  if (jb == 0 && threadIdx.x == 0) {
    c.alpha = alpha;
    c.pq = sigma;
  }
  const BatchSys S = sys[s];
  const int64_t o = S.off;
  const Range rg = block_range(S.n, jb, T);
  double ww = 0.0;
  for (int64_t i = o + rg.lo + threadIdx.x; i < o + rg.hi; i += kBlock) {
    const double wi = V.w[i] - alpha * V.au[i];
    const double di = V.uh[i] + coef * V.d[i];
    const double ui = V.u[i] - alpha * V.v[i];
    V.w[i] = wi;
    V.d[i] = di;
    V.u[i] = ui;
    V.uh[i] = dinv[i] * ui;
    ww += wi * wi;
  }
  ww = block_sum<kBlock>(ww, lds);
  if (threadIdx.x == 0) P1[blockIdx.x] = ww;
}

// theta, c, tau, eta of one half-step from ||w||^2 and the previous tau
struct TqStep {
  double theta, tau, eta;
};
__device__ __forceinline__ TqStep tq_step(double ww, double tau_prev, double alpha) {
  TqStep r;
  r.theta = sqrt(ww) / tau_prev;
  const double c = 1.0 / sqrt(1.0 + r.theta * r.theta);
  r.tau = tau_prev * r.theta * c;
  r.eta = c * c * alpha;
  return r;
}

// KC(j): close half-step 2j+1, then the row walk of half-step 2j+2
template <class SH>
__global__ __launch_bounds__(kBlock) void k_tq_c(const BatchSys* __restrict__ sys, PlanView pl,
                                                 TqVecs V, double* __restrict__ x, CgScalars* st,
                                                 const double* __restrict__ P1,
                                                 double* __restrict__ P2, int rows, int64_t j,
                                                 int64_t pos) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double lds[kLds];
  const int s = pl.sys(blockIdx.x);
  if (s < 0) return;
  const bool skip = tq_skip(st[s], pos);  // tested once the partials are in
  const int a = pl.start(s), T = pl.size(s);
  const int64_t jb = blockIdx.x - a;
  CgScalars& c = st[s];
  const double ww = reduce_all(P1 + a, T, lds);
  if (skip) return;
  const double alpha = c.alpha;
  const TqStep h = tq_step(ww, c.tau[0], alpha);
  const int64_t ml = 2 * (j - c.j0) + 1;  // half-steps of this cycle
  const int64_t m = c.m0 + ml;
  const bool passed = sqrt((double)(ml + 1)) * h.tau <= c.thresh;
  const bool stop = passed || m >= c.maxit;
  if (jb == 0 && threadIdx.x == 0) {
    c.tau[1] = h.tau;
    c.theta = h.theta;
    c.eta = h.eta;
    c.iters = (int32_t)m;
    if (passed) {
      c.verify = 1;
      c.stop_pos = (int32_t)pos;
    } else if (stop) {
      c.status = SPX_NOT_CONVERGED;
      c.done = 1;
      c.stop_pos = (int32_t)pos;
    }
  }
  const BatchSys S = sys[s];
  const int64_t o = S.off;
  if (stop) {
    const Range rg = block_range(S.n, jb, T);
    for (int64_t i = o + rg.lo + threadIdx.x; i < o + rg.hi; i += kBlock)
      x[i] = x[i] + h.eta * V.d[i];
    return;
  }
  const double coef = h.theta * h.theta * h.eta / alpha;
  double w2 = 0.0, wr = 0.0;
  for_rows<SH, double, double, double>(S.n, S.rowptr, S.col, S.val, V.uh + o, rows, jb, T,
                                       reinterpret_cast<double*>(smem), [&](int64_t row, double y) {
                                         const int64_t i = o + row;
                                         const double d0 = V.d[i];
                                         x[i] = x[i] + h.eta * d0;
                                         V.d[i] = V.uh[i] + coef * d0;
                                         V.t[i] = y;
                                         const double wi = V.w[i] - alpha * y;
                                         V.w[i] = wi;
                                         w2 += wi * wi;
                                         wr += V.rs[i] * wi;
                                       }, 0, S.win);
  w2 = block_sum<kBlock>(w2, lds);
  wr = block_sum<kBlock>(wr, lds);
  if (threadIdx.x == 0) {
    P2[blockIdx.x] = w2;
    P2[pl.G + blockIdx.x] = wr;
  }
}

// KD(j): close half-step 2j+2; rho, beta; u = w + beta u; uh = D^-1 u
__global__ __launch_bounds__(kBlock) void k_tq_d(const BatchSys* __restrict__ sys, PlanView pl,
                                                 TqVecs V, double* __restrict__ x,
                                                 const double* __restrict__ dinv, CgScalars* st,
                                                 const double* __restrict__ P2, int64_t j,
                                                 int64_t pos) {
  __shared__ double lds[kLds];
  const int s = pl.sys(blockIdx.x);
  if (s < 0) return;
  const bool skip = tq_skip(st[s], pos);  // tested once the partials are in
  const int a = pl.start(s), T = pl.size(s);
  const int64_t jb = blockIdx.x - a;
  CgScalars& c = st[s];
  double ww, rho_new;
  reduce_all(P2 + a, P2 + pl.G + a, T, lds, ww, rho_new);
  if (skip) return;
  const double alpha = c.alpha;
  const TqStep h = tq_step(ww, c.tau[1], alpha);
  const int64_t ml = 2 * (j - c.j0) + 2;
  const int64_t m = c.m0 + ml;
  const bool passed = sqrt((double)(ml + 1)) * h.tau <= c.thresh;
  const bool limit = !passed && m >= c.maxit;
  const bool broke = !passed && !limit && (rho_new == 0.0 || !isfinite(rho_new));
  const bool stop = passed || limit || broke;
  const double rho_prev = c.rho[j & 1];
  if (jb == 0 && threadIdx.x == 0) {
    c.tau[0] = h.tau;
    c.theta = h.theta;
    c.eta = h.eta;
    c.iters = (int32_t)m;
    if (passed) {
      c.verify = 1;
      c.stop_pos = (int32_t)pos;
    } else if (stop) {
      c.status = limit ? SPX_NOT_CONVERGED : SPX_BREAKDOWN;
      c.done = 1;
      c.stop_pos = (int32_t)pos;
    } else {
      c.rho[(j + 1) & 1] = rho_new;
      c.beta = rho_new / rho_prev;
    }
  }
  const BatchSys S = sys[s];
  const int64_t o = S.off;
  const Range rg = block_range(S.n, jb, T);
  if (stop) {
    for (int64_t i = o + rg.lo + threadIdx.x; i < o + rg.hi; i += kBlock)
      x[i] = x[i] + h.eta * V.d[i];
    return;
  }
  const double beta = rho_new / rho_prev;
  for (int64_t i = o + rg.lo + threadIdx.x; i < o + rg.hi; i += kBlock) {
    x[i] = x[i] + h.eta * V.d[i];
    const double ui = V.w[i] + beta * V.u[i];
    V.u[i] = ui;
    V.uh[i] = dinv[i] * ui;
  }
}

// True residual of a system whose cycle ended on the bound, and the start of
// a new cycle from it: r = b - A x; w = u = rs = r; uh = D^-1 r;
// d = t = v = 0; partials of r.r.  Other systems are left alone.
template <class SH>
__global__ __launch_bounds__(kBlock) void k_tq_verify(const BatchSys* __restrict__ sys, PlanView pl,
                                                      const double* __restrict__ b,
                                                      const double* __restrict__ x, TqVecs V,
                                                      const double* __restrict__ dinv,
                                                      const CgScalars* __restrict__ st,
                                                      double* __restrict__ P, int rows) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double lds[kLds];
  const int s = pl.sys(blockIdx.x);
  if (s < 0 || !st[s].verify) return;
  const BatchSys S = sys[s];
  const int64_t o = S.off;
  double rr = 0.0;
  for_rows<SH, double, double, double>(S.n, S.rowptr, S.col, S.val, x + o, rows,
                                       blockIdx.x - pl.start(s), pl.size(s),
                                       reinterpret_cast<double*>(smem), [&](int64_t row, double ax) {
                                         const int64_t i = o + row;
                                         const double ri = b[i] - ax;
                                         V.w[i] = ri;
                                         V.u[i] = ri;
                                         V.rs[i] = ri;
                                         V.uh[i] = dinv[i] * ri;
                                         V.d[i] = 0.0;
                                         V.t[i] = 0.0;
                                         V.v[i] = 0.0;
                                         rr += ri * ri;
                                       }, 0, S.win);
  rr = block_sum<kBlock>(rr, lds);
  if (threadIdx.x == 0) P[blockIdx.x] = rr;
}

// one workgroup per system: done, or a new cycle from iteration jn
__global__ __launch_bounds__(kBlock) void k_tq_verify_finish(PlanView pl, CgScalars* st,
                                                             const double* __restrict__ P,
                                                             int64_t jn, int32_t max_restarts) {
  __shared__ double lds[kLds];
  const int s = blockIdx.x;
  if (!st[s].verify) return;
  const double rr = reduce_all(P + pl.start(s), pl.size(s), lds);
  if (threadIdx.x == 0) {
    CgScalars& c = st[s];
    c.verify = 0;
    c.rr = rr;
    const double tau = sqrt(rr);
    if (tau <= c.thresh) {
      c.status = SPX_OK;
      c.done = 1;
    } else if (c.restarts >= max_restarts || c.iters >= c.maxit) {
      c.status = SPX_NOT_CONVERGED;
      c.done = 1;
    } else {
      c.restarts += 1;
      c.rho[jn & 1] = rr;
      c.tau[0] = tau;
      c.theta = 0.0;
      c.eta = 0.0;
      c.beta = 0.0;
      c.j0 = (int32_t)jn;
      c.m0 = c.iters;
      c.stop_pos = INT32_MAX;
    }
  }
}

constexpr int32_t kTfqmrMaxRestarts = 8;

// ------------------------------------------------------- persistent form
// One launch for the whole batch: each workgroup takes the next system from
// the queue (largest first) and runs BiCG (METHOD 1) or TFQMR (METHOD 2) on
// it alone (krylov_one.hpp), D^-1 included; thread t owns rows t, t + BLOCK,
// ... of every pass.  No workgroup waits for another.
template <int METHOD, int BLOCK, int ROWS>
__global__ __launch_bounds__(BLOCK) void k_bk_persistent(
    const BatchSys* __restrict__ sys, const BatchSys* __restrict__ sysT, int nsys,
    int32_t* __restrict__ queue, const double* __restrict__ bvec, double* __restrict__ x,
    double* __restrict__ kw, int64_t tot, CgScalars* st, double rtol) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double lds[BLOCK / 64];
  __shared__ int32_t pick, zero;
  double* dinv = kw + (METHOD == 1 ? 6 : 8) * tot;
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
    const int32_t status0 = zero ? SPX_ZERO_DIAGONAL : SPX_OK;
    const one::Csr3 A{S.rowptr, S.col, S.val};
    double* prod = reinterpret_cast<double*>(smem);
    if constexpr (METHOD == 1) {
      const BatchSys T = sysT[s];
      one::bicg_solve<BLOCK, ROWS>(S.n, A, one::Csr3{T.rowptr, T.col, T.val}, bvec + o, x + o,
                                   kw + o, kw + tot + o, kw + 2 * tot + o, kw + 3 * tot + o,
                                   kw + 4 * tot + o, kw + 5 * tot + o, dinv + o, status0,
                                   st[s].maxit, rtol, st + s, prod, lds);
    } else {
      const one::TqVectors V{kw + o,           kw + tot + o,     kw + 2 * tot + o,
                             kw + 3 * tot + o, kw + 4 * tot + o, kw + 5 * tot + o,
                             kw + 6 * tot + o, kw + 7 * tot + o};
      one::tfqmr_solve<BLOCK, ROWS>(S.n, A, bvec + o, x + o, V, dinv + o, status0, st[s].maxit,
                                    kTfqmrMaxRestarts, rtol, st + s, prod, lds);
    }
    __syncthreads();  // `pick` and `zero` read by every thread before thread 0 rewrites them
  }
}

// Runs the persistent form of METHOD when the caller asks for it or the
// library picks it; *ran tells which.
template <int METHOD>
int maybe_persistent(spx_batch* B, const spx_batch_tuning* tuning, int64_t tile256,
                     const double* bvec, double* x, double rtol, int64_t maxit, hipStream_t s,
                     const char* what, bool* ran) {
  *ran = false;
  int32_t mode = 0;
  SPX_TRY(persistent_mode(tuning, what, &mode));
  const PersistShape ps = persistent_shape(B, tile256);
  if (!(mode == 1 || (mode == 0 && persistent_by_default(B, ps)))) return SPX_OK;
  if (ps.lds == 0)
    return set_error(SPX_INVALID_ARG,
                     "%s: a 256-row tile of a system exceeds the persistent solve's LDS", what);
  const int ns = B->nsys;
  hipLaunchKernelGGL(k_b_reset, dim3((unsigned)ceil_div(ns, 64)), dim3(64), 0, s, B->d_st, ns,
                     (int32_t)maxit);
  hipLaunchKernelGGL(k_b_queue_reset, dim3(1), dim3(64), 0, s, B->d_queue);
  auto launch = [&](auto blk, auto rws) {
    constexpr int BLOCK = decltype(blk)::value, ROWS = decltype(rws)::value;
    const void* fn = reinterpret_cast<const void*>(&k_bk_persistent<METHOD, BLOCK, ROWS>);
    int fit = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, fn, BLOCK, ps.lds) != hipSuccess ||
        fit < 1)
      fit = 1;
    const int G = (int)std::min<int64_t>(ns, (int64_t)cu_count() * fit);
    hipLaunchKernelGGL((k_bk_persistent<METHOD, BLOCK, ROWS>), dim3((unsigned)G), dim3(BLOCK),
                       ps.lds, s, B->d_sys, B->d_sysT, ns, B->d_queue, bvec, x, B->kwork,
                       B->total, B->d_st, rtol);
  };
  using I256 = std::integral_constant<int, 256>;
  using I512 = std::integral_constant<int, 512>;
  using I1024 = std::integral_constant<int, 1024>;
  if (ps.block == 256)
    launch(I256(), I256());
  else if (ps.rows == 1024)
    launch(I1024(), I1024());
  else if (ps.rows == 512)
    launch(I1024(), I512());
  else
    launch(I1024(), I256());
  SPX_CHECK_HIP(hipGetLastError());
  *ran = true;
  return SPX_OK;
}

// -------------------------------------------------------------- host side

int ensure_kwork(spx_batch* B) {
  if (!B->kwork) SPX_TRY(dalloc_n(&B->kwork, (size_t)B->total * 9));
  return SPX_OK;
}

int check_args(spx_batch* B, const double* bvec, double* x, double rtol, int64_t maxit,
               const char* what) {
  if (!B || !bvec || !x) return set_error(SPX_INVALID_ARG, "%s: NULL argument", what);
  if (maxit < 0 || !(rtol >= 0.0)) return set_error(SPX_INVALID_ARG, "%s: bad maxit/rtol", what);
  return SPX_OK;
}

}  // namespace
}  // namespace spx

using namespace spx;
using namespace spx::solver;
using namespace spx::batch;

extern "C" int spx_batch_bicg(spx_batch_handle B, const double* bvec, double* x, double rtol,
                              int64_t maxit, const spx_batch_tuning* tuning, void* stream,
                              int64_t* iters_out, double* relres_out) {
  clear_error();
  SPX_TRY(check_args(B, bvec, x, rtol, maxit, "batch_bicg"));
  if (maxit > INT32_MAX - 1) maxit = INT32_MAX - 1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ns = B->nsys;
  // explicit transposes, refreshed to the current values
  if (!B->d_sysT) SPX_TRY(dalloc_n(&B->d_sysT, (size_t)ns));
  std::vector<BatchSys> sysT(ns);
  int64_t tiles[4] = {B->max_tile[0], B->max_tile[1], B->max_tile[2], B->max_tile[3]};
  int64_t max_row = B->max_row;
  B->win_blocks_t = 0;
  for (int k = 0; k < ns; ++k) {
    spx_matrix* h = B->hs[k];
    SPX_TRY(ensure_transpose(h, s));
    sysT[k] = BatchSys{h->n, B->sys[k].off, h->At.rowptr, h->At.col, h->At.val, h->At.dpos,
                       win_view(h->At)};
    B->win_blocks_t = h->At.win.lcol && B->win_blocks_t >= 0
                          ? std::max(B->win_blocks_t, h->At.win.max_blocks)
                          : -1;
    for (int t = 0; t < 4; ++t) tiles[t] = std::max(tiles[t], h->At.tile_nnz[t]);
    max_row = std::max(max_row, h->At.max_row);
  }
  SPX_CHECK_HIP(hipMemcpyAsync(B->d_sysT, sysT.data(), sizeof(BatchSys) * (size_t)ns,
                               hipMemcpyHostToDevice, s));
  SPX_TRY(ensure_kwork(B));
  Run run;
  const int64_t wb = B->win_blocks > 0 && B->win_blocks_t > 0
                         ? std::max(B->win_blocks, B->win_blocks_t)
                         : -1;
  SPX_TRY(prepare(B, tuning, tiles, max_row, wb, 3, s, &run));
  bool ran = false;
  SPX_TRY(maybe_persistent<1>(B, tuning, tiles[3], bvec, x, rtol, maxit, s, "batch_bicg", &ran));
  if (ran) {
    SPX_TRY(true_residuals(B, run, bvec, x, s));
    return finish(B, s, iters_out, relres_out, "batch_bicg");
  }
  const int G = run.G;
  const int64_t tot = B->total;
  double* r = B->kwork;
  double* rh = B->kwork + tot;
  double* p = B->kwork + 2 * tot;
  double* ph = B->kwork + 3 * tot;
  double* q = B->kwork + 4 * tot;
  double* qh = B->kwork + 5 * tot;
  double* dinv = B->kwork + 6 * tot;
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
    hipLaunchKernelGGL((k_bb_init<SH>), dim3(G), dim3(kBlock), lds, s, B->d_sys, pl, bvec, x, r, rh,
                       p, ph, dinv, B->partials, sh.rows);
    return SPX_OK;
  }));
  hipLaunchKernelGGL(k_b_init_finish, dim3(ns), dim3(kBlock), 0, s, pl, B->d_st, B->partials, rtol);
  SPX_CHECK_HIP(hipGetLastError());
  SPX_TRY(poll_loop(B, run, maxit, s, [&](int64_t first, int64_t m) {
    return with_shape<true>(sh, [&](auto shc) {
      using SH = decltype(shc);
      for (int64_t c = 0; c < m; ++c) {
        const int64_t kk = first + c;
        hipLaunchKernelGGL((k_bb_spmv<SH>), dim3(G), dim3(kBlock), lds, s, B->d_sys, B->d_sysT, pl,
                           p, ph, q, qh, B->d_st, P1, sh.rows);
        hipLaunchKernelGGL(k_bb_update, dim3(G), dim3(kBlock), 0, s, B->d_sys, pl, x, r, rh, p, q,
                           qh, dinv, B->d_st, P1, P2, kk);
        hipLaunchKernelGGL(k_bb_pupdate, dim3(G), dim3(kBlock), 0, s, B->d_sys, pl, p, ph, r, rh,
                           dinv, B->d_st, P2, kk);
      }
      return SPX_OK;
    });
  }));
  SPX_TRY(true_residuals(B, run, bvec, x, s));
  return finish(B, s, iters_out, relres_out, "batch_bicg");
}

extern "C" int spx_batch_tfqmr(spx_batch_handle B, const double* bvec, double* x, double rtol,
                               int64_t maxit, const spx_batch_tuning* tuning, void* stream,
                               int64_t* iters_out, double* relres_out) {
  clear_error();
  SPX_TRY(check_args(B, bvec, x, rtol, maxit, "batch_tfqmr"));
  // half-steps; launch positions 4 j + phase stay within int32
  if (maxit > (int64_t)1 << 28) maxit = (int64_t)1 << 28;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ns = B->nsys;
  SPX_TRY(ensure_kwork(B));
  Run run;
  SPX_TRY(prepare(B, tuning, B->max_tile, B->max_row, B->win_blocks, 4, s, &run));
  bool ran = false;
  SPX_TRY(maybe_persistent<2>(B, tuning, B->max_tile[3], bvec, x, rtol, maxit, s, "batch_tfqmr",
                              &ran));
  if (ran) {
    SPX_TRY(true_residuals(B, run, bvec, x, s));
    return finish(B, s, iters_out, relres_out, "batch_tfqmr");
  }
  const int G = run.G;
  const int64_t tot = B->total;
  double* kw = B->kwork;
  const TqVecs V{kw, kw + tot, kw + 2 * tot, kw + 3 * tot, kw + 4 * tot, kw + 5 * tot,
                 kw + 6 * tot, kw + 7 * tot};
  double* dinv = kw + 8 * tot;
  double* P0 = B->partials;
  double* P1 = B->partials + G;
  double* P2 = B->partials + 2 * G;  // two sets
  const PlanView pl = run.pl;
  const SpmvShape sh = run.sh;
  const size_t lds = run.lds;

  hipLaunchKernelGGL(k_b_reset, dim3((unsigned)ceil_div(ns, 64)), dim3(64), 0, s, B->d_st, ns,
                     (int32_t)maxit);
  hipLaunchKernelGGL(k_b_dinv, dim3(G), dim3(kBlock), 0, s, B->d_sys, pl, dinv, B->d_st);
  SPX_TRY(with_shape<true>(sh, [&](auto shc) {
    using SH = decltype(shc);
    hipLaunchKernelGGL((k_tq_init<SH>), dim3(G), dim3(kBlock), lds, s, B->d_sys, pl, bvec, x, V,
                       dinv, P2, sh.rows);
    return SPX_OK;
  }));
  hipLaunchKernelGGL(k_tq_init_finish, dim3(ns), dim3(kBlock), 0, s, pl, B->d_st, P2, rtol);
  SPX_CHECK_HIP(hipGetLastError());
  // two half-steps per iteration, plus the polls a system may wait for
  // its true-residual check
  const int64_t iters = (maxit + 1) / 2 + (int64_t)(kTfqmrMaxRestarts + 1) * run.check_every;
  auto verify = [&](int64_t k, bool* relaunched) -> int {
    bool any = false;
    for (int t = 0; t < ns; ++t) any = any || (B->h_st[t].verify && !B->h_st[t].done);
    if (!any) return SPX_OK;
    SPX_TRY(with_shape<true>(sh, [&](auto shc) {
      using SH = decltype(shc);
      hipLaunchKernelGGL((k_tq_verify<SH>), dim3(G), dim3(kBlock), lds, s, B->d_sys, pl, bvec, x,
                         V, dinv, B->d_st, P2, sh.rows);
      return SPX_OK;
    }));
    hipLaunchKernelGGL(k_tq_verify_finish, dim3(ns), dim3(kBlock), 0, s, pl, B->d_st, P2, k,
                       kTfqmrMaxRestarts);
    SPX_CHECK_HIP(hipGetLastError());
    *relaunched = true;
    return SPX_OK;
  };
  SPX_TRY(poll_loop(B, run, iters, s, [&](int64_t first, int64_t m) {
    return with_shape<true>(sh, [&](auto shc) {
      using SH = decltype(shc);
      for (int64_t c = 0; c < m; ++c) {
        const int64_t j = first + c - 1;  // 0-based iteration
        const int64_t pos = 4 * j;
        hipLaunchKernelGGL((k_tq_a<SH>), dim3(G), dim3(kBlock), lds, s, B->d_sys, pl, V, B->d_st, P0,
                           sh.rows, pos);
        hipLaunchKernelGGL(k_tq_b, dim3(G), dim3(kBlock), 0, s, B->d_sys, pl, V, dinv, B->d_st, P0,
                           P1, j, pos + 1);
        hipLaunchKernelGGL((k_tq_c<SH>), dim3(G), dim3(kBlock), lds, s, B->d_sys, pl, V, x, B->d_st,
                           P1, P2, sh.rows, j, pos + 2);
        hipLaunchKernelGGL(k_tq_d, dim3(G), dim3(kBlock), 0, s, B->d_sys, pl, V, x, dinv, B->d_st,
                           P2, j, pos + 3);
      }
      return SPX_OK;
    });
  }, verify));
  SPX_TRY(true_residuals(B, run, bvec, x, s));
  return finish(B, s, iters_out, relres_out, "batch_tfqmr");
}
