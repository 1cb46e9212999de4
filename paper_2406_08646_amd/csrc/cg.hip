// Jacobi-preconditioned CG with device-resident scalars (paper Sec. 6, the
// CG -> CGAsync redesign): every scalar (rho, alpha, beta, the residual
// norm, the convergence flag) lives in device memory, so the host only
// enqueues kernels and polls the flag every `check_every` iterations.
//
// One iteration k is three kernels, each fused around its memory traffic:
//   K1  q = A p; per-workgroup partials of p.q
//   K2  every workgroup adds the p.q partials (same fixed order, same
//       result everywhere), alpha = rho_{k-1} / p.q; x += alpha p,
//       r -= alpha q, z = D^-1 r; partials of r.z and r.r
//   K3  every workgroup adds those partials: rho_k, ||r_k||; the test
//       ||r_k|| <= rtol ||b|| or k = maxit stops the run (workgroup 0 records
//       it); otherwise beta = rho_k / rho_{k-1} and p = D^-1 r + beta p
// Cross-workgroup results travel only through kernel boundaries: a
// workgroup never waits for another inside a kernel, and no agent-scope
// fence is issued (on gfx950 such a fence writes back the XCD's L2).  The
// kernels return at once when the flag is set, so work queued past
// convergence costs only the launches.  All sums use a fixed order, so runs
// are reproducible.
//
// The same kernels, instantiated for float, run the inner solve of the
// mixed-precision refinement (paper Sec. 2 multiprecision plan): fp32
// matrix copy, vectors and SpMV; fp64 products and sums in every dot.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "cg_one.hpp"
#include "common.hpp"
#include "device.hpp"
#include "solver_core.hpp"
#include "spmv_core.hpp"

namespace spx {

namespace {

using namespace solver;

__global__ void k_scal_reset(CgScalars* st, int32_t maxit) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    CgScalars z = {};
    z.maxit = maxit;
    z.stop_pos = INT32_MAX;
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
    st->status = SPX_ZERO_DIAGONAL;
  else
    inv = 1.0 / d;
  dinv[r] = inv;
  if (dinv32) dinv32[r] = (float)inv;
}

// r = b - A x, z = D^-1 r, p = z; partials of r.z, r.r, b.b.
template <class SH>
__global__ __launch_bounds__(kBlock) void k_cg_init(int64_t n, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ r, double* __restrict__ p,
                                                    const double* __restrict__ dinv,
                                                    double* __restrict__ P, int rows, int remap,
                                                    int64_t tile, WinView win) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double lds[kLds];
  const int64_t nb = gridDim.x;
  double rz = 0.0, rr = 0.0, bb = 0.0;
  for_rows<SH, double, double, double>(n, rowptr, col, val, x, rows, logical_block(remap), nb,
                                       reinterpret_cast<double*>(smem), [&](int64_t row, double ax) {
                                         const double bi = b[row];
                                         const double ri = bi - ax;
                                         const double zi = dinv[row] * ri;
                                         r[row] = ri;
                                         p[row] = zi;
                                         rz += ri * zi;
                                         rr += ri * ri;
                                         bb += bi * bi;
                                       }, tile, win);
  rz = block_sum<kBlock>(rz, lds);
  rr = block_sum<kBlock>(rr, lds);
  bb = block_sum<kBlock>(bb, lds);
  if (threadIdx.x == 0) {
    P[blockIdx.x] = rz;
    P[nb + blockIdx.x] = rr;
    P[2 * nb + blockIdx.x] = bb;
  }
}

__global__ __launch_bounds__(kBlock) void k_cg_init_finish(CgScalars* st, const double* P,
                                                           int64_t G, double rtol) {
  __shared__ double lds[kLds];
  double rz, rr, bb;
  reduce_all(P, P + G, P + 2 * G, G, lds, rz, rr, bb);
  if (threadIdx.x == 0) {
    st->rho[0] = rz;
    st->bb = bb;
    st->bnorm = sqrt(bb);
    st->thresh = rtol * st->bnorm;
    st->rr = rr;
    st->iters = 0;
    if (st->status != SPX_OK) {
      st->done = 1;
    } else if (sqrt(rr) <= st->thresh) {
      st->done = 1;
    } else if (st->maxit <= 0) {
      st->done = 1;
      st->status = SPX_NOT_CONVERGED;
    } else {
      st->done = 0;
    }
  }
}

// K1: q = A p; partials of p.q
// Scratch of the workgroup sums in a kernel with the LDS of SH's row walk:
// the window walk's own LDS (free between tiles' use and before the first
// one), so the kernel holds no static LDS and eight workgroups per CU fit
// with two 256-entry steps per chunk on the 27-point operator; a small
// static array for the other walks (whose LDS may be empty).  Callers
// synchronise before reusing it after the walk.
template <class SH>
__device__ __forceinline__ double* reduction_lds(char* smem) {
  if constexpr (SH::variant == kVariantWindow) {
    return reinterpret_cast<double*>(smem);
  } else {
    __shared__ double lds[kLds];
    return lds;
  }
}

template <class SH, typename VT>
__global__ __launch_bounds__(kBlock) void k_cg_spmv(int64_t n, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const VT* __restrict__ val,
                                                    const VT* __restrict__ p, VT* __restrict__ q,
                                                    const CgScalars* __restrict__ st,
                                                    double* __restrict__ P1, int rows, int remap,
                                                    int64_t tile, WinView win) {
  extern __shared__ __align__(16) char smem[];
  if (st->done) return;
  double dot = 0.0;
  for_rows<SH, VT, VT, VT>(n, rowptr, col, val, p, rows, logical_block(remap), gridDim.x,
                           reinterpret_cast<VT*>(smem), [&](int64_t row, VT s) {
                             q[row] = s;
                             dot += (double)p[row] * (double)s;
                           }, tile, win);
  __syncthreads();  // the walk's LDS may hold the reduction scratch
  dot = block_sum<kBlock>(dot, reduction_lds<SH>(smem));
  if (threadIdx.x == 0) P1[blockIdx.x] = dot;
}

// K2: alpha = rho_{k-1} / p.q; x += alpha p; r -= alpha q; partials of r.z, r.r
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_cg_update(int64_t n, VT* __restrict__ x,
                                                      VT* __restrict__ r,
                                                      const VT* __restrict__ p,
                                                      const VT* __restrict__ q,
                                                      const VT* __restrict__ dinv, CgScalars* st,
                                                      const double* __restrict__ P1, int64_t G1,
                                                      double* __restrict__ P2, int64_t k) {
  __shared__ double lds[kLds];
  // the flag is tested once the partials are in: both loads are in flight
  // together (after the solve stopped the partials are stale and unused)
  const auto done = st->done;
  const double pq = reduce_all(P1, G1, lds);
  if (done) return;
  if (k <= 0) k = (int64_t)st->iters + 1;  // replayed launch: the iteration count is on the device
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->pq = pq;
      st->status = SPX_BREAKDOWN;
      st->iters = (int32_t)(k - 1);
      st->done = 1;
    }
    return;
  }
  const double alpha = st->rho[(k - 1) & 1] / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->pq = pq;
    st->alpha = alpha;
    st->kcur = (int32_t)k;
  }
  const VT a = (VT)alpha;
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
    P2[blockIdx.x] = rz;
    P2[nb + blockIdx.x] = rr;
  }
}

// K3: rho_k, ||r_k||, stopping test; beta; p = D^-1 r + beta p
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_cg_pupdate(int64_t n, VT* __restrict__ p,
                                                       const VT* __restrict__ r,
                                                       const VT* __restrict__ dinv, CgScalars* st,
                                                       const double* __restrict__ P2, int64_t G2,
                                                       int64_t k) {
  __shared__ double lds[kLds];
  const auto done = st->done;  // tested once the partials are in
  double rz, rr;
  reduce_all(P2, P2 + G2, G2, lds, rz, rr);
  if (done) return;
  if (k <= 0) k = st->kcur;  // written by this iteration's update kernel
  const bool conv = sqrt(rr) <= st->thresh;
  const bool stop = conv || k >= st->maxit;
  const double rho_prev = st->rho[(k - 1) & 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rr = rr;
    st->iters = (int32_t)k;
    if (conv) {
      st->status = SPX_OK;
      st->done = 1;
    } else if (stop) {
      st->status = SPX_NOT_CONVERGED;
      st->done = 1;
    } else {
      st->rho[k & 1] = rz;
      st->beta = rz / rho_prev;
    }
  }
  if (stop) return;
  const VT bt = (VT)(rz / rho_prev);
  const Range rg = block_range(n, blockIdx.x, gridDim.x);
  for (int64_t i = rg.lo + threadIdx.x; i < rg.hi; i += kBlock) p[i] = dinv[i] * r[i] + bt * p[i];
}

// partials of ||b - A x||^2
template <class SH>
__global__ __launch_bounds__(kBlock) void k_resnorm(int64_t n, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ P, int rows, int remap,
                                                    int64_t tile, WinView win) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double lds[kLds];
  double rr = 0.0;
  for_rows<SH, double, double, double>(n, rowptr, col, val, x, rows, logical_block(remap), gridDim.x,
                                       reinterpret_cast<double*>(smem), [&](int64_t row, double ax) {
                                         const double ri = b[row] - ax;
                                         rr += ri * ri;
                                       }, tile, win);
  rr = block_sum<kBlock>(rr, lds);
  if (threadIdx.x == 0) P[blockIdx.x] = rr;
}

__global__ __launch_bounds__(kBlock) void k_resnorm_finish(CgScalars* st, const double* P,
                                                           int64_t G) {
  __shared__ double lds[kLds];
  const double rr = reduce_all(P, G, lds);
  if (threadIdx.x == 0) st->rr_true = rr;
}

// ------------------------------------------- single-reduction variant
// Chronopoulos-Gear form: two kernels per iteration and one reduction
// point.  KA(k) adds the delta partials of KB(k-1), forms alpha_k and
// updates x, r and u = D^-1 r with the partials of gamma_k = r.u and
// ||r||^2; KB(k) adds those, tests convergence, forms beta_k, computes
// w = A u and updates p = u + beta p, s = w + beta s with the partials of
// delta_k = w.u.  gamma_j lives in rho[j & 1], alpha_j in alpha_s[j & 1].

// w = A u, p = u, s = w; partials of delta_0 = w.u
template <class SH>
__global__ __launch_bounds__(kBlock) void k_sr_init(int64_t n, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ u,
                                                    double* __restrict__ p, double* __restrict__ s,
                                                    double* __restrict__ P, int rows, int remap,
                                                    int64_t tile, WinView win) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double lds[kLds];
  double delta = 0.0;
  for_rows<SH, double, double, double>(n, rowptr, col, val, u, rows, logical_block(remap), gridDim.x,
                                       reinterpret_cast<double*>(smem), [&](int64_t row, double w) {
                                         const double ur = u[row];
                                         p[row] = ur;
                                         s[row] = w;
                                         delta += w * ur;
                                       }, tile, win);
  delta = block_sum<kBlock>(delta, lds);
  if (threadIdx.x == 0) P[blockIdx.x] = delta;
}

// KA(k)
__global__ __launch_bounds__(kBlock) void k_sr_update(int64_t n, double* __restrict__ x,
                                                      double* __restrict__ r,
                                                      double* __restrict__ u,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ s,
                                                      const double* __restrict__ dinv,
                                                      CgScalars* st, const double* __restrict__ P1,
                                                      int64_t G1, double* __restrict__ P2,
                                                      int64_t k) {
  __shared__ double lds[kLds];
  const auto done = st->done;  // tested once the partials are in
  const double delta = reduce_all(P1, G1, lds);
  if (done) return;
  const double g1 = st->rho[(k - 1) & 1];
  double den = delta;
  if (k > 1) {
    const double beta = g1 / st->rho[k & 1];
    den = delta - beta * g1 / st->alpha_s[(k - 1) & 1];
  }
  if (!(den > 0.0) || !isfinite(den)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->pq = den;
      st->status = SPX_BREAKDOWN;
      st->iters = (int32_t)(k - 1);
      st->done = 1;
    }
    return;
  }
  const double alpha = g1 / den;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->alpha_s[k & 1] = alpha;
    st->alpha = alpha;
    st->pq = den;
  }
  const int64_t nb = gridDim.x;
  const Range rg = block_range(n, blockIdx.x, nb);
  double ru = 0.0, rr = 0.0;
  for (int64_t i = rg.lo + threadIdx.x; i < rg.hi; i += kBlock) {
    const double xi = x[i] + alpha * p[i];
    const double ri = r[i] - alpha * s[i];
    const double ui = dinv[i] * ri;
    x[i] = xi;
    r[i] = ri;
    u[i] = ui;
    ru += ri * ui;
    rr += ri * ri;
  }
  ru = block_sum<kBlock>(ru, lds);
  rr = block_sum<kBlock>(rr, lds);
  if (threadIdx.x == 0) {
    P2[blockIdx.x] = ru;
    P2[nb + blockIdx.x] = rr;
  }
}

// KB(k)
template <class SH>
__global__ __launch_bounds__(kBlock) void k_sr_spmv(int64_t n, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ u,
                                                    double* __restrict__ p, double* __restrict__ s,
                                                    CgScalars* st, const double* __restrict__ P2,
                                                    int64_t G2, double* __restrict__ P1, int rows,
                                                    int remap, int64_t tile, int64_t k, WinView win) {
  extern __shared__ __align__(16) char smem[];
  double* lds = reduction_lds<SH>(smem);
  const auto done = st->done;  // tested once the partials are in
  double gk, rr;
  reduce_all(P2, P2 + G2, G2, lds, gk, rr);
  if (done) return;
  const bool conv = sqrt(rr) <= st->thresh;
  const bool stop = conv || k >= st->maxit;
  const double gprev = st->rho[(k - 1) & 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rr = rr;
    st->iters = (int32_t)k;
    if (conv) {
      st->status = SPX_OK;
      st->done = 1;
    } else if (stop) {
      st->status = SPX_NOT_CONVERGED;
      st->done = 1;
    } else {
      st->rho[k & 1] = gk;
      st->beta = gk / gprev;
    }
  }
  if (stop) return;
  const double beta = gk / gprev;
  double delta = 0.0;
  for_rows<SH, double, double, double>(n, rowptr, col, val, u, rows, logical_block(remap), gridDim.x,
                                       reinterpret_cast<double*>(smem), [&](int64_t row, double w) {
                                         const double ur = u[row];
                                         p[row] = ur + beta * p[row];
                                         s[row] = w + beta * s[row];
                                         delta += w * ur;
                                       }, tile, win);
  __syncthreads();  // the walk's LDS may hold the reduction scratch
  delta = block_sum<kBlock>(delta, lds);
  if (threadIdx.x == 0) P1[blockIdx.x] = delta;
}

// ------------------------------------------------ pipelined variant
// Ghysels-Vanroose pipelined CG with M = D: the dots of iteration i
// (gamma_i = r.u, delta_i = w.u, ||r_i||) are formed by the update kernel
// that writes r_i, u_i, w_i, and reduced by the next update kernel, so the
// product between them (nv = A m) never waits for a reduction.  Per
// iteration k (1-based, i = k - 1):
//   KP(k)  nv = A m                                   (m = D^-1 w_i)
//   KU(k)  add the partials of KU(k-1): gamma_i, delta_i, ||r_i||; stop
//          when ||r_i|| <= rtol ||b|| (iters = i) or i = maxit; beta_i,
//          alpha_i; z = nv + beta z, q = m + beta q, s = w + beta s,
//          p = u + beta p (z = nv, ... at i = 0); x += alpha p,
//          r -= alpha s, u -= alpha q, w -= alpha z, m = D^-1 w; partials of
//          the next gamma, delta, ||r||.
// The partials alternate between two sets (KU(k) reads set (k-1) & 1 and
// writes set k & 1); gamma_i lives in rho[i & 1], alpha_i in alpha_s[i & 1].

// w = A u, m = D^-1 w; partials of gamma_0 = r.u, delta_0 = w.u, ||r_0||^2
template <class SH>
__global__ __launch_bounds__(kBlock) void k_pl_init(int64_t n, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ r,
                                                    const double* __restrict__ u,
                                                    double* __restrict__ w, double* __restrict__ m,
                                                    const double* __restrict__ dinv,
                                                    double* __restrict__ P, int rows, int remap,
                                                    int64_t tile, WinView win) {
  extern __shared__ __align__(16) char smem[];
  double* lds = reduction_lds<SH>(smem);
  double g = 0.0, dl = 0.0, rr = 0.0;
  for_rows<SH, double, double, double>(n, rowptr, col, val, u, rows, logical_block(remap), gridDim.x,
                                       reinterpret_cast<double*>(smem), [&](int64_t row, double wr) {
                                         const double ur = u[row], rv = r[row];
                                         w[row] = wr;
                                         m[row] = dinv[row] * wr;
                                         g += rv * ur;
                                         dl += wr * ur;
                                         rr += rv * rv;
                                       }, tile, win);
  __syncthreads();  // the walk's LDS may hold the reduction scratch
  const int64_t nb = gridDim.x;
  g = block_sum<kBlock>(g, lds);
  dl = block_sum<kBlock>(dl, lds);
  rr = block_sum<kBlock>(rr, lds);
  if (threadIdx.x == 0) {
    P[blockIdx.x] = g;
    P[nb + blockIdx.x] = dl;
    P[2 * nb + blockIdx.x] = rr;
  }
}

// KP(k): nv = A m
template <class SH>
__global__ __launch_bounds__(kBlock) void k_pl_spmv(int64_t n, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ m,
                                                    double* __restrict__ nv, const CgScalars* st,
                                                    int rows, int remap, int64_t tile, WinView win) {
  extern __shared__ __align__(16) char smem[];
  if (st->done) return;
  for_rows<SH, double, double, double>(n, rowptr, col, val, m, rows, logical_block(remap), gridDim.x,
                                       reinterpret_cast<double*>(smem),
                                       [&](int64_t row, double a) { nv[row] = a; }, tile, win);
}

// KU(k)
struct PlVectors {
  double *x, *r, *u, *w, *m, *nv, *z, *q, *s, *p;
  const double* dinv;
};

__global__ __launch_bounds__(kBlock) void k_pl_update(int64_t n, PlVectors v, CgScalars* st,
                                                      const double* __restrict__ Pin, int64_t Gin,
                                                      double* __restrict__ Pout, int64_t k) {
  __shared__ double lds[kLds];
  const auto done = st->done;  // tested once the partials are in
  double g, dl, rr;
  reduce_all(Pin, Pin + Gin, Pin + 2 * Gin, Gin, lds, g, dl, rr);
  if (done) return;
  const int64_t i = k - 1;
  const bool conv = sqrt(rr) <= st->thresh;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (conv || i >= st->maxit) {
    if (lead) {
      st->rr = rr;
      st->iters = (int32_t)i;
      st->status = conv ? SPX_OK : SPX_NOT_CONVERGED;
      st->done = 1;
    }
    return;
  }
  double beta = 0.0, den = dl;
  if (i > 0) {
    beta = g / st->rho[(i - 1) & 1];
    den = dl - beta * g / st->alpha_s[(i - 1) & 1];
  }
  if (!(den > 0.0) || !isfinite(den)) {
    if (lead) {
      st->rr = rr;
      st->pq = den;
      st->iters = (int32_t)i;
      st->status = SPX_BREAKDOWN;
      st->done = 1;
    }
    return;
  }
  const double alpha = g / den;
  if (lead) {
    st->rho[i & 1] = g;
    st->alpha_s[i & 1] = alpha;
    st->alpha = alpha;
    st->beta = beta;
    st->pq = den;
    st->rr = rr;
    st->iters = (int32_t)i;
  }
  const int64_t nb = gridDim.x;
  const Range rg = block_range(n, blockIdx.x, nb);
  double gn = 0.0, dn = 0.0, rn = 0.0;
  for (int64_t e = rg.lo + threadIdx.x; e < rg.hi; e += kBlock) {
    const double nve = v.nv[e], me = v.m[e], we = v.w[e], ue = v.u[e];
    double ze = nve, qe = me, se = we, pe = ue;
    if (i > 0) {
      ze = nve + beta * v.z[e];
      qe = me + beta * v.q[e];
      se = we + beta * v.s[e];
      pe = ue + beta * v.p[e];
    }
    const double xe = v.x[e] + alpha * pe;
    const double re = v.r[e] - alpha * se;
    const double u2 = ue - alpha * qe;
    const double w2 = we - alpha * ze;
    v.z[e] = ze;
    v.q[e] = qe;
    v.s[e] = se;
    v.p[e] = pe;
    v.x[e] = xe;
    v.r[e] = re;
    v.u[e] = u2;
    v.w[e] = w2;
    v.m[e] = v.dinv[e] * w2;
    gn += re * u2;
    dn += w2 * u2;
    rn += re * re;
  }
  gn = block_sum<kBlock>(gn, lds);
  dn = block_sum<kBlock>(dn, lds);
  rn = block_sum<kBlock>(rn, lds);
  if (threadIdx.x == 0) {
    Pout[blockIdx.x] = gn;
    Pout[nb + blockIdx.x] = dn;
    Pout[2 * nb + blockIdx.x] = rn;
  }
}

// ------------------------------------------------ one-workgroup solve
// Small systems: one workgroup of kOne threads runs the whole Jacobi-CG
// (cg_one.hpp), so no kernel is launched per iteration (the working set
// stays in L2); tiles of ROWS rows, as many as LDS holds (a lone workgroup
// may use all of a CU's).
constexpr int kOne = 1024;

template <int ROWS>
__global__ __launch_bounds__(kOne) void k_cg_one(int64_t n, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col,
                                                 const double* __restrict__ val,
                                                 const double* __restrict__ b,
                                                 double* __restrict__ x, double* __restrict__ r,
                                                 double* __restrict__ p, double* __restrict__ q,
                                                 const double* __restrict__ dinv, CgScalars* st,
                                                 double rtol) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double lds[kOne / 64];
  one::cg_solve<kOne, ROWS>(n, rowptr, col, val, b, x, r, p, q, dinv, st->status, st->maxit, rtol,
                            st, reinterpret_cast<double*>(smem), lds);
}

// ---------------------------------------------------- mixed precision

__global__ __launch_bounds__(kBlock) void k_norm2(int64_t n, const double* __restrict__ b,
                                                  double* __restrict__ P) {
  __shared__ double lds[kLds];
  const Range rg = block_range(n, blockIdx.x, gridDim.x);
  double s = 0.0;
  for (int64_t i = rg.lo + threadIdx.x; i < rg.hi; i += kBlock) s += b[i] * b[i];
  s = block_sum<kBlock>(s, lds);
  if (threadIdx.x == 0) P[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_norm2_finish(CgScalars* st, const double* P, int64_t G,
                                                         double rtol) {
  __shared__ double lds[kLds];
  const double bb = reduce_all(P, G, lds);
  if (threadIdx.x == 0) {
    st->bb = bb;
    st->bnorm = sqrt(bb);
    st->thresh = rtol * st->bnorm;
  }
}

// Outer fp64 residual r = b - A x with its norm, rounded to fp32, and the
// start of the inner solve: d = 0, z = D32^-1 r32, p = z; partials of
// ||r||^2 (fp64), r32.z and r32.r32.
template <class SH>
__global__ __launch_bounds__(kBlock) void k_ir_residual(
    int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ b, const double* __restrict__ x,
    const float* __restrict__ dinv32, float* __restrict__ r32, float* __restrict__ d32,
    float* __restrict__ p32, double* __restrict__ P, int rows, int remap, int64_t tile,
    WinView win) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double lds[kLds];
  const int64_t nb = gridDim.x;
  double rr64 = 0.0, rz = 0.0, rr32 = 0.0;
  for_rows<SH, double, double, double>(n, rowptr, col, val, x, rows, logical_block(remap), nb,
                                       reinterpret_cast<double*>(smem), [&](int64_t row, double ax) {
                                         const double ri = b[row] - ax;
                                         rr64 += ri * ri;
                                         const float rf = (float)ri;
                                         const float zf = dinv32[row] * rf;
                                         r32[row] = rf;
                                         d32[row] = 0.0f;
                                         p32[row] = zf;
                                         rz += (double)rf * (double)zf;
                                         rr32 += (double)rf * (double)rf;
                                       }, tile, win);
  rr64 = block_sum<kBlock>(rr64, lds);
  rz = block_sum<kBlock>(rz, lds);
  rr32 = block_sum<kBlock>(rr32, lds);
  if (threadIdx.x == 0) {
    P[blockIdx.x] = rr64;
    P[nb + blockIdx.x] = rz;
    P[2 * nb + blockIdx.x] = rr32;
  }
}

__global__ __launch_bounds__(kBlock) void k_ir_finish(CgScalars* so, CgScalars* si, const double* P,
                                                      int64_t G, double rtol_inner,
                                                      int early_exit) {
  __shared__ double lds[kLds];
  double t64, trz, t32;
  reduce_all(P, P + G, P + 2 * G, G, lds, t64, trz, t32);
  if (threadIdx.x == 0) {
    so->rr = t64;
    so->rr_true = t64;
    if (so->status == SPX_OK && sqrt(t64) <= so->thresh) so->done = 1;
    si->rho[0] = trz;
    si->r0norm = sqrt(t32);
    // the inner solve stops at rtol_inner relative to its right-hand side;
    // with early_exit also as soon as the outer target is in reach (this
    // shortens the last refinement step)
    si->thresh = early_exit ? fmax(rtol_inner * si->r0norm, 0.5 * so->thresh)
                            : rtol_inner * si->r0norm;
    si->rr = t32;
    si->iters = 0;
    si->status = SPX_OK;
    si->done = (so->done || so->status != SPX_OK) ? 1 : 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_ir_update(int64_t n, double* __restrict__ x,
                                                      const float* __restrict__ d32) {
  const Range rg = block_range(n, blockIdx.x, gridDim.x);
  for (int64_t i = rg.lo + threadIdx.x; i < rg.hi; i += kBlock) x[i] = x[i] + (double)d32[i];
}

// ------------------------------------------------------------ dispatch

// Vectors of n in the fp64 workspace: 4 (r, p, q and the single-reduction
// form's u) or 9 (the pipelined form).
int ensure_solver(spx_matrix* h, int nvec = 4) {
  const int64_t n = h->n;
  const size_t need = (size_t)n * (size_t)nvec;
  if (h->work_elems < need) {
    dfree(h->work);
    h->work = nullptr;
    h->work_elems = 0;
    SPX_TRY(dalloc_n(&h->work, need));
    h->work_elems = need;
  }
  if (!h->dinv) SPX_TRY(dalloc_n(&h->dinv, (size_t)n));
  if (!h->scal) {
    SPX_TRY(dalloc_n(&h->scal, 2));
    SPX_CHECK_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->scal_host), sizeof(CgScalars) * 4,
                                hipHostMallocDefault));
    SPX_CHECK_HIP(hipEventCreateWithFlags(&h->ev[0], hipEventDisableTiming));
    SPX_CHECK_HIP(hipEventCreateWithFlags(&h->ev[1], hipEventDisableTiming));
  }
  // two sets of three partials (the pipelined form), four for the others
  const int64_t cap = (int64_t)std::max(fused_blocks(h), vector_blocks(h)) * 6;
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

// The memory one fp64 solve works in: four vectors of n (r, p, q and the
// single-reduction form's u), the inverse diagonal, the workgroup partials,
// the device scalars and their host mirror.  With events, the host polls a
// chunk while the next one is queued; without, it polls by synchronising
// the stream.
struct Work {
  double* vec = nullptr;       // [4 n], [9 n] for the pipelined form
  double* dinv = nullptr;      // [n]
  double* partials = nullptr;  // [6 max(fused_blocks, vector_blocks)]
  CgScalars* scal = nullptr;   // device [2]
  CgScalars* host = nullptr;   // host [4]
  const hipEvent_t* ev = nullptr;  // 2 events or null
};

// The handle's own workspace (nvec vectors of n), allocated on first use.
int handle_work(spx_matrix* h, Work* w, int nvec = 4) {
  SPX_TRY(ensure_solver(h, nvec));
  w->vec = h->work;
  w->dinv = h->dinv;
  w->partials = h->partials;
  w->scal = h->scal;
  w->host = h->scal_host;
  w->ev = h->ev;
  return SPX_OK;
}

inline unsigned grid1(int64_t count) {
  return (unsigned)std::max<int64_t>(1, ceil_div(count, 256));
}

// The operator of one solve: a matrix in the precision VT plus its shape.
template <typename VT>
struct Op {
  int64_t n;
  const int32_t* rowptr;
  const int32_t* col;
  const VT* val;
  SpmvShape sh;
  WinView win;
};

// Dynamic LDS of the solver kernels for elements of type VT (sh.lds is
// sized for doubles).
template <typename VT>
size_t shape_lds(const SpmvShape& sh) {
  switch (sh.variant) {
    case kVariantDma:
      return 2 * ((dma_buffer_bytes(sh.tile, sizeof(VT)) + 15) & ~size_t(15));
    case kVariantStream:
      return sh.lds / sizeof(double) * sizeof(VT);
    case kVariantWindow:
      return window_lds_bytes(sh.tile / kWinBlock, sizeof(VT), win_u_solver<VT>() * win_v<VT>());
    default:
      return 0;  // the vector walk uses none
  }
}

// Enqueues iterations first .. first+count-1 (1-based k) of K1, K2, K3.
// With `evs` (6 events per iteration) every kernel is bracketed by events.
template <typename VT>
int enqueue_iterations(spx_matrix* h, const Work& w, const Op<VT>& A, VT* x, VT* r, VT* p, VT* q,
                       const VT* dinv, CgScalars* st, int64_t first, int64_t count, hipStream_t s,
                       hipEvent_t* evs, bool device_k = false) {
  const unsigned G1 = (unsigned)fused_blocks(h);
  const unsigned G2 = (unsigned)vector_blocks(h);
  double* P1 = w.partials;
  double* P2 = w.partials + G1;
  const size_t lds = shape_lds<VT>(A.sh);
  return with_shape<true>(A.sh, [&](auto shc) {
    using SH = decltype(shc);
    for (int64_t c = 0; c < count; ++c) {
      const int64_t k = device_k ? 0 : first + c;
      hipEvent_t* e = evs ? evs + 6 * c : nullptr;
      if (e) (void)hipEventRecord(e[0], s);
      hipLaunchKernelGGL((k_cg_spmv<SH, VT>), dim3(G1), dim3(kBlock), lds, s, A.n, A.rowptr, A.col,
                         A.val, p, q, st, P1, A.sh.rows, remap_for(h, A.sh), A.sh.tile, A.win);
      if (e) (void)hipEventRecord(e[1], s);
      if (e) (void)hipEventRecord(e[2], s);
      hipLaunchKernelGGL((k_cg_update<VT>), dim3(G2), dim3(kBlock), 0, s, A.n, x, r, p, q, dinv, st,
                         P1, (int64_t)G1, P2, k);
      if (e) (void)hipEventRecord(e[3], s);
      if (e) (void)hipEventRecord(e[4], s);
      hipLaunchKernelGGL((k_cg_pupdate<VT>), dim3(G2), dim3(kBlock), 0, s, A.n, p, r, dinv, st, P2,
                         (int64_t)G2, k);
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
// finished chunk (kinds[j] is the profile slot of the j-th of K kernels per
// iteration), counting only launches that did their full work: in the
// iteration that records the stop (`iters`) the kernels up to index
// `full_at`, the later ones (which return after the test) not at all.
void accumulate_profile(spx_matrix* h, hipEvent_t* evs, int64_t first, int64_t count,
                        int64_t iters, int K, const int* kinds, int full_at) {
  for (int64_t c = 0; c < count; ++c) {
    const int64_t it = first + c;
    for (int j = 0; j < K; ++j) {
      const bool ran = it < iters || (it == iters && j <= full_at);
      if (!ran || kinds[j] < 0) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, evs[2 * K * c + 2 * j], evs[2 * K * c + 2 * j + 1]) ==
          hipSuccess) {
        h->prof_ms[kinds[j]] += ms;
        h->prof_cnt[kinds[j]] += 1;
      }
    }
  }
}

// Runs iterations until the device flag is set, keeping one chunk of
// `check_every` iterations queued ahead of the one being polled.  The
// launch that records the stop is iteration iters + stop_offset (1 for
// the pipelined form, whose update kernel tests the previous iterate).  enq(first,
// count, events) enqueues iterations first .. first+count-1 (K kernels
// each, bracketed by 2K events when `events` is not null).  Returns the last
// polled state in *final.
template <typename Enq>
int run_until_done(spx_matrix* h, const Work& w, CgScalars* st, int64_t maxit,
                   int32_t check_every, hipStream_t s, int K, const int* kinds, int full_at,
                   Enq&& enq, CgScalars* final, int stop_offset = 0) {
  int64_t launched = 0;
  CgScalars* host = w.host;
  const bool prof = h->profile != 0 && w.ev;
  const int64_t per_chunk = 2 * K * (int64_t)check_every;
  if (prof) SPX_TRY(ensure_prof_events(h, 2 * per_chunk));
  int64_t first[2] = {0, 0}, cnt[2] = {0, 0};
  auto chunk = [&](int slot) -> int {
    const int64_t m = std::min<int64_t>(check_every, maxit - launched);
    hipEvent_t* evs = prof ? h->prof_ev + slot * per_chunk : nullptr;
    SPX_TRY(enq(launched + 1, m, evs));
    first[slot] = launched + 1;
    cnt[slot] = m;
    launched += m;
    SPX_CHECK_HIP(hipMemcpyAsync(&host[slot], st, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
    if (w.ev) SPX_CHECK_HIP(hipEventRecord(w.ev[slot], s));
    return SPX_OK;
  };
  auto harvest = [&](int slot, int64_t iters) {
    if (prof && cnt[slot] > 0)
      accumulate_profile(h, h->prof_ev + slot * per_chunk, first[slot], cnt[slot], iters, K, kinds,
                         full_at);
    cnt[slot] = 0;
  };
  // state before any iteration (the start may already satisfy the test)
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
    if (w.ev) {
      // queue the next chunk, then wait for this one's copy of the scalars
      if (more) SPX_TRY(chunk(cur ^ 1));
      SPX_CHECK_HIP(hipEventSynchronize(w.ev[cur]));
    } else {
      // no events: wait for this chunk, then queue the next one
      SPX_CHECK_HIP(hipStreamSynchronize(s));
      if (!host[cur].done && more) SPX_TRY(chunk(cur ^ 1));
    }
    if (host[cur].done || !more) {
      *final = host[cur];
      break;
    }
    harvest(cur, INT64_MAX);  // no stop in this chunk: every launch did its work
    cur ^= 1;
  }
  SPX_CHECK_HIP(hipStreamSynchronize(s));
  harvest(0, final->iters + stop_offset);
  harvest(1, final->iters + stop_offset);
  return SPX_OK;
}

// A graph of one full poll chunk (check_every iterations of K1, K2, K3 that
// take the iteration number from the device), captured on a private stream
// and kept while the operator, vectors and launch shape stay the same.
template <typename VT>
int chunk_graph(spx_matrix* h, const Work& w, const Op<VT>& A, VT* x, VT* r, VT* p, VT* q,
                const VT* dinv, CgScalars* st, int32_t check_every, hipGraphExec_t* out) {
  spx_matrix::GraphCache& gc = h->graph[sizeof(VT) == 8 ? 0 : 1];
  const uintptr_t key[16] = {(uintptr_t)A.rowptr, (uintptr_t)A.col, (uintptr_t)A.val,
                             (uintptr_t)x, (uintptr_t)r, (uintptr_t)p, (uintptr_t)q,
                             (uintptr_t)dinv, (uintptr_t)st, (uintptr_t)w.partials,
                             (uintptr_t)check_every, (uintptr_t)fused_blocks(h),
                             (uintptr_t)vector_blocks(h),
                             (uintptr_t)(A.sh.variant * 4096 + A.sh.rows * 8 + A.sh.nt * 2 + A.sh.vec),
                             (uintptr_t)(A.sh.tile * 64 + A.sh.lanes), (uintptr_t)(A.sh.pipe * 2 + remap_for(h, A.sh))};
  if (gc.exec && std::equal(key, key + 16, gc.key)) {
    *out = gc.exec;
    return SPX_OK;
  }
  if (gc.exec) {
    (void)hipGraphExecDestroy(gc.exec);
    gc.exec = nullptr;
  }
  if (!h->cap_stream) SPX_CHECK_HIP(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  SPX_CHECK_HIP(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  const int st_enq = enqueue_iterations<VT>(h, w, A, x, r, p, q, dinv, st, 0, check_every,
                                            h->cap_stream, nullptr, true);
  hipGraph_t graph = nullptr;
  const hipError_t e_end = hipStreamEndCapture(h->cap_stream, &graph);
  if (st_enq != SPX_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st_enq;
  }
  if (e_end != hipSuccess || !graph)
    return set_error(SPX_HIP_ERROR, "cg graph capture failed: %s", hipGetErrorString(e_end));
  hipGraphExec_t exec = nullptr;
  const hipError_t e_inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e_inst != hipSuccess)
    return set_error(SPX_HIP_ERROR, "cg graph instantiation failed: %s", hipGetErrorString(e_inst));
  gc.exec = exec;
  std::copy(key, key + 16, gc.key);
  *out = exec;
  return SPX_OK;
}

// The Hestenes-Stiefel iteration (K1, K2, K3) on operator A in precision VT.
// Graph replay needs the handle's workspace (a graph may outlive the call).
template <typename VT>
int run_hs(spx_matrix* h, const Work& w, const Op<VT>& A, VT* x, VT* r, VT* p, VT* q,
           const VT* dinv, CgScalars* st, int64_t maxit, int32_t check_every, hipStream_t s,
           CgScalars* final, bool allow_graph = true) {
  const int kinds64[3] = {0, 1, 2}, kinds32[3] = {3, 4, 5};
  hipGraphExec_t exec = nullptr;
  if (allow_graph && h->graph_opt && !h->profile)
    SPX_TRY(chunk_graph<VT>(h, w, A, x, r, p, q, dinv, st, check_every, &exec));
  return run_until_done(h, w, st, maxit, check_every, s, 3, sizeof(VT) == 8 ? kinds64 : kinds32, 1,
                        [&](int64_t first, int64_t count, hipEvent_t* evs) -> int {
                          if (exec && !evs && count == check_every) {
                            SPX_CHECK_HIP(hipGraphLaunch(exec, s));
                            return SPX_OK;
                          }
                          return enqueue_iterations<VT>(h, w, A, x, r, p, q, dinv, st, first,
                                                        count, s, evs);
                        },
                        final);
}

// The single-reduction iteration (KA, KB), fp64.
int run_sr(spx_matrix* h, const Work& w, const Op<double>& A, double* x, double* r, double* u,
           double* p, double* sv, CgScalars* st, int64_t maxit, int32_t check_every,
           hipStream_t s, CgScalars* final) {
  const unsigned G1 = (unsigned)fused_blocks(h);
  const unsigned G2 = (unsigned)vector_blocks(h);
  double* P1 = w.partials;
  double* P2 = w.partials + G1;
  const size_t lds = shape_lds<double>(A.sh);
  const int kinds[2] = {1, 0};  // KA is the vector kernel, KB the SpMV kernel
  return run_until_done(
      h, w, st, maxit, check_every, s, 2, kinds, 0,
      [&](int64_t first, int64_t count, hipEvent_t* evs) {
        return with_shape<true>(A.sh, [&](auto shc) {
          using SH = decltype(shc);
          for (int64_t c = 0; c < count; ++c) {
            const int64_t k = first + c;
            hipEvent_t* e = evs ? evs + 4 * c : nullptr;
            if (e) (void)hipEventRecord(e[0], s);
            hipLaunchKernelGGL(k_sr_update, dim3(G2), dim3(kBlock), 0, s, A.n, x, r, u, p, sv,
                               w.dinv, st, P1, (int64_t)G1, P2, k);
            if (e) (void)hipEventRecord(e[1], s);
            if (e) (void)hipEventRecord(e[2], s);
            hipLaunchKernelGGL((k_sr_spmv<SH>), dim3(G1), dim3(kBlock), lds, s, A.n, A.rowptr,
                               A.col, A.val, u, p, sv, st, P2, (int64_t)G2, P1, A.sh.rows,
                               remap_for(h, A.sh), A.sh.tile, k, A.win);
            if (e) (void)hipEventRecord(e[3], s);
          }
          return SPX_OK;
        });
      },
      final);
}

// The pipelined iteration (KP, KU), fp64.  KU(k) tests the residual of
// iteration k - 1, so a solve of at most maxit iterations launches up to
// maxit + 1 of them.
int run_pl(spx_matrix* h, const Work& w, const Op<double>& A, const PlVectors& v, CgScalars* st,
           int64_t maxit, int32_t check_every, hipStream_t s, CgScalars* final) {
  const unsigned G1 = (unsigned)fused_blocks(h);
  const unsigned G2 = (unsigned)vector_blocks(h);
  const int64_t set = 3 * (int64_t)std::max(G1, G2);  // one set of partials
  const size_t lds = shape_lds<double>(A.sh);
  const int kinds[2] = {0, 1};  // KP is the SpMV kernel, KU the vector kernel
  return run_until_done(
      h, w, st, maxit + 1, check_every, s, 2, kinds, 0,
      [&](int64_t first, int64_t count, hipEvent_t* evs) {
        return with_shape<true>(A.sh, [&](auto shc) {
          using SH = decltype(shc);
          for (int64_t c = 0; c < count; ++c) {
            const int64_t k = first + c;
            hipEvent_t* e = evs ? evs + 4 * c : nullptr;
            if (e) (void)hipEventRecord(e[0], s);
            hipLaunchKernelGGL((k_pl_spmv<SH>), dim3(G1), dim3(kBlock), lds, s, A.n, A.rowptr,
                               A.col, A.val, v.m, v.nv, st, A.sh.rows, remap_for(h, A.sh),
                               A.sh.tile, A.win);
            if (e) (void)hipEventRecord(e[1], s);
            if (e) (void)hipEventRecord(e[2], s);
            const double* Pin = w.partials + ((k - 1) & 1) * set;
            double* Pout = w.partials + (k & 1) * set;
            hipLaunchKernelGGL(k_pl_update, dim3(G2), dim3(kBlock), 0, s, A.n, v, st, Pin,
                               (int64_t)(k == 1 ? G1 : G2), Pout, k);
            if (e) (void)hipEventRecord(e[3], s);
          }
          return SPX_OK;
        });
      },
      final, 1);
}

// Launches the fp64 residual-norm kernels for b - A x into st->rr_true.
int enqueue_resnorm(spx_matrix* h, const Work& w, const Op<double>& A, const double* b,
                    const double* x, CgScalars* st, hipStream_t s) {
  const unsigned G = (unsigned)fused_blocks(h);
  SPX_TRY(with_shape<true>(A.sh, [&](auto shc) {
    using SH = decltype(shc);
    hipLaunchKernelGGL((k_resnorm<SH>), dim3(G), dim3(kBlock), shape_lds<double>(A.sh), s, A.n,
                       A.rowptr, A.col, A.val, b, x, w.partials, A.sh.rows, remap_for(h, A.sh),
                       A.sh.tile, A.win);
    return SPX_OK;
  }));
  hipLaunchKernelGGL(k_resnorm_finish, dim3(1), dim3(kBlock), 0, s, st, w.partials, (int64_t)G);
  return SPX_OK;
}

int finish_solve(spx_matrix* h, const Work& w, const Op<double>& A, const double* b,
                 const double* x, CgScalars* st, hipStream_t s, int64_t* iters_out,
                 double* relres_out);

// The one-workgroup solve: forced by SPX_OPT_SMALL_SOLVE = 2, chosen by the
// default 1 for systems of at most kOneAutoRows rows when no launch-shape
// option, profiling, graph replay or the single-reduction form asks for the
// multi-workgroup kernels; either way only if a 256-row tile fits in 64 KB.
constexpr int64_t kOneAutoRows = 2048;  // measured crossover with the launch-per-iteration path

// Without an explicit SPX_OPT_CG_VARIANT, systems of at most kSrAutoNnz
// entries take the single-reduction form: one launch and one reduction
// point fewer per iteration save about 2 us of each (11.7 vs 13.9 us at 36K
// entries, 15.5 vs 17.4 at 591K, 14.9 vs 16.7 at 831K; even at 2.4M; 36.3
// vs 35.7 at 6.9M).  Larger systems, and any solve with graph replay asked
// for (the captured chunk is the textbook iteration), take the textbook form.
constexpr int64_t kSrAutoNnz = 2000000;
constexpr int64_t kOneLds = 150 * 1024;  // dynamic LDS of the lone workgroup
bool use_one_workgroup(const spx_matrix* h, const Csr& M) {
  if (h->small_opt == 0 || h->cg_variant >= 1) return false;
  if ((M.tile_nnz[3] + 8) * (int64_t)sizeof(double) > 64 * 1024) return false;  // 256-row tiles fit
  if (h->small_opt == 2) return true;
  const bool shape_default = h->lanes_opt == 0 && h->variant_opt == 0 && h->rows_opt == 0 &&
                             h->rows32_opt == 0 && h->fused_opt == 0 && h->vec_blocks_opt == 0 &&
                             h->pipe_opt == 0 && h->vec_opt == 0 && h->nt_opt == 1;
  return shape_default && !h->profile && !h->graph_opt && M.n <= kOneAutoRows;
}

}  // namespace

int cg_form(const spx_matrix* h, const Csr& M) {
  if (h->cg_variant >= 0) return h->cg_variant;
  return !h->graph_opt && M.nnz <= kSrAutoNnz ? 1 : 0;
}

namespace {

// The fp64 solve on M in workspace w.  `scratch` marks the static scratch
// of spx_cg_solve_noalloc: no graph is captured (a graph would keep
// pointers into memory the next call reuses).
int cg_solve_impl(spx_matrix* h, const Work& w, const Csr& M, const double* b, double* x,
                  double rtol, int64_t maxit, int32_t check_every, hipStream_t s,
                  int64_t* iters_out, double* relres_out, bool scratch = false) {
  if (!b || !x) return set_error(SPX_INVALID_ARG, "cg_solve: b or x is NULL");
  if (maxit < 0 || check_every < 1 || !(rtol >= 0.0))
    return set_error(SPX_INVALID_ARG, "cg_solve: bad maxit/check_every/rtol");
  if (maxit > INT32_MAX - 1) maxit = INT32_MAX - 1;
  const int64_t n = M.n;
  const Op<double> A{n, M.rowptr, M.col, M.val, solver_shape(h, M), win_view(M)};
  const int form = cg_form(h, M);
  double* r = w.vec;
  double* p = w.vec + n;
  double* q = w.vec + 2 * n;
  CgScalars* st = w.scal;
  const unsigned G = (unsigned)fused_blocks(h);
  hipLaunchKernelGGL(k_scal_reset, dim3(1), dim3(64), 0, s, st, (int32_t)maxit);
  hipLaunchKernelGGL(k_dinv, dim3(grid1(n)), dim3(256), 0, s, n, M.val, M.dpos, w.dinv,
                     (float*)nullptr, st);
  CgScalars fin;
  if (form == 2) {
    // r, u = D^-1 r and the partials of gamma_0, ||r_0||, ||b||; then
    // w = A u, m = D^-1 w and the first set of KU partials
    const PlVectors v{x, w.vec, w.vec + n, w.vec + 2 * n, w.vec + 3 * n, w.vec + 4 * n,
                      w.vec + 5 * n, w.vec + 6 * n, w.vec + 7 * n, w.vec + 8 * n, w.dinv};
    SPX_TRY(with_shape<true>(A.sh, [&](auto shc) {
      using SH = decltype(shc);
      hipLaunchKernelGGL((k_cg_init<SH>), dim3(G), dim3(kBlock), shape_lds<double>(A.sh), s, n,
                         M.rowptr, M.col, M.val, b, x, v.r, v.u, w.dinv, w.partials, A.sh.rows,
                         remap_for(h, A.sh), A.sh.tile, A.win);
      return SPX_OK;
    }));
    hipLaunchKernelGGL(k_cg_init_finish, dim3(1), dim3(kBlock), 0, s, st, w.partials,
                       (int64_t)G, rtol);
    SPX_TRY(with_shape<true>(A.sh, [&](auto shc) {
      using SH = decltype(shc);
      hipLaunchKernelGGL((k_pl_init<SH>), dim3(G), dim3(kBlock), shape_lds<double>(A.sh), s, n,
                         M.rowptr, M.col, M.val, v.r, v.u, v.w, v.m, w.dinv, w.partials,
                         A.sh.rows, remap_for(h, A.sh), A.sh.tile, A.win);
      return SPX_OK;
    }));
    SPX_CHECK_HIP(hipGetLastError());
    SPX_TRY(run_pl(h, w, A, v, st, maxit, check_every, s, &fin));
    return finish_solve(h, w, A, b, x, st, s, iters_out, relres_out);
  }
  if (use_one_workgroup(h, M)) {
    // the largest tile whose products fit (4 and 2 tiles of 256 rows bound
    // the entries of 1024 and 512 consecutive rows)
    const int64_t t256 = M.tile_nnz[3];
    // a tile above 64 KB of LDS needs the kernel's limit raised first
    auto allow = [&](const void* fn, int64_t tiles) {
      const int64_t bytes = (tiles * t256 + 8) * (int64_t)sizeof(double);
      if (bytes > kOneLds) return false;
      return bytes <= 64 * 1024 ||
             hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) ==
                 hipSuccess;
    };
    const int rows = allow(reinterpret_cast<const void*>(&k_cg_one<1024>), 4)  ? 1024
                     : allow(reinterpret_cast<const void*>(&k_cg_one<512>), 2) ? 512
                                                                                : 256;
    (void)hipGetLastError();  // a refused attribute leaves no error behind
    const size_t lds = (size_t)((rows / 256) * t256 + 8) * sizeof(double);
    if (rows == 1024)
      hipLaunchKernelGGL(k_cg_one<1024>, dim3(1), dim3(kOne), lds, s, n, M.rowptr, M.col, M.val, b,
                         x, r, p, q, w.dinv, st, rtol);
    else if (rows == 512)
      hipLaunchKernelGGL(k_cg_one<512>, dim3(1), dim3(kOne), lds, s, n, M.rowptr, M.col, M.val, b,
                         x, r, p, q, w.dinv, st, rtol);
    else
      hipLaunchKernelGGL(k_cg_one<256>, dim3(1), dim3(kOne), lds, s, n, M.rowptr, M.col, M.val, b,
                         x, r, p, q, w.dinv, st, rtol);
    SPX_CHECK_HIP(hipGetLastError());
    return finish_solve(h, w, A, b, x, st, s, iters_out, relres_out);
  }
  SPX_TRY(with_shape<true>(A.sh, [&](auto shc) {
    using SH = decltype(shc);
    hipLaunchKernelGGL((k_cg_init<SH>), dim3(G), dim3(kBlock), shape_lds<double>(A.sh), s, n,
                       M.rowptr, M.col, M.val, b, x, r, p, w.dinv, w.partials, A.sh.rows,
                       remap_for(h, A.sh), A.sh.tile, A.win);
    return SPX_OK;
  }));
  hipLaunchKernelGGL(k_cg_init_finish, dim3(1), dim3(kBlock), 0, s, st, w.partials, (int64_t)G,
                     rtol);
  SPX_CHECK_HIP(hipGetLastError());
  if (form == 1) {
    // k_cg_init left u = D^-1 r in p; move it to its own vector and start
    // w = A u, p = u, s = w, delta_0
    double* u = w.vec + 3 * n;
    SPX_CHECK_HIP(hipMemcpyAsync(u, p, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
    SPX_TRY(with_shape<true>(A.sh, [&](auto shc) {
      using SH = decltype(shc);
      hipLaunchKernelGGL((k_sr_init<SH>), dim3(G), dim3(kBlock), shape_lds<double>(A.sh), s, n,
                         M.rowptr, M.col, M.val, u, p, q, w.partials, A.sh.rows, remap_for(h, A.sh),
                         A.sh.tile, A.win);
      return SPX_OK;
    }));
    SPX_CHECK_HIP(hipGetLastError());
    SPX_TRY(run_sr(h, w, A, x, r, u, p, q, st, maxit, check_every, s, &fin));
  } else {
    SPX_TRY(run_hs<double>(h, w, A, x, r, p, q, w.dinv, st, maxit, check_every, s, &fin,
                           !scratch));
  }
  return finish_solve(h, w, A, b, x, st, s, iters_out, relres_out);
}

// True residual of the returned x, the outputs and the status of a solve.
int finish_solve(spx_matrix* h, const Work& w, const Op<double>& A, const double* b,
                 const double* x, CgScalars* st, hipStream_t s, int64_t* iters_out,
                 double* relres_out) {
  SPX_TRY(enqueue_resnorm(h, w, A, b, x, st, s));
  SPX_CHECK_HIP(hipMemcpyAsync(&w.host[2], st, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
  SPX_CHECK_HIP(hipStreamSynchronize(s));
  const CgScalars& f = w.host[2];
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


// Workgroups of the solver's SpMV-shaped kernels (each walks a contiguous
// share of the rows) and of its vector kernels; every workgroup of the
// next kernel re-adds this many partials, so the counts stay moderate.
// Both shrink with the system: every workgroup of the next kernel re-adds
// all partials, so a small system with a full-chip grid would spend its
// iteration reading thousands of partials that hold zeros.
// Workgroups of the solver's row-walk kernels: 8 per CU, at least one
// 64-row tile each.  The window walk works on 256-row tiles and holds more
// LDS; its grid is cut to the workgroups that are resident at once (taken
// for the fp64 kernel, which needs the most), so no workgroup of the
// persistent grid waits for another to finish.
int fused_blocks(const spx_matrix* h) {
  if (h && h->fused_opt > 0) return h->fused_opt;
  if (!h) return 1;
  int64_t per_cu = 8;
  int64_t tiles = ceil_div(h->n, 64);
  const SpmvShape sh = solver_shape(h, h->A);
  if (sh.variant == kVariantWindow) {
    tiles = ceil_div(h->n, kWinRows);
    const void* fn =
        sh.nt ? reinterpret_cast<const void*>(&k_cg_spmv<Shape<kVariantWindow, 1, true>, double>)
              : reinterpret_cast<const void*>(&k_cg_spmv<Shape<kVariantWindow, 1, false>, double>);
    int fit = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, fn, kBlock, sh.lds) == hipSuccess &&
        fit > 0)
      per_cu = std::min<int64_t>(per_cu, fit);
    (void)hipGetLastError();
  }
  return (int)std::max<int64_t>(1, std::min<int64_t>(cu_count() * per_cu, tiles));
}

int vector_blocks(const spx_matrix* h) {
  if (h && h->vec_blocks_opt > 0) return h->vec_blocks_opt;
  const int64_t chunks = h ? ceil_div(h->n, 1024) : 1;  // at least 4 rows per thread
  return (int)std::max<int64_t>(1, std::min<int64_t>(cu_count() * 4, chunks));
}

}  // namespace spx

using namespace spx;

extern "C" int spx_cg_solve(spx_handle h, const double* b, double* x, double rtol, int64_t maxit,
                            int32_t check_every, void* stream, int64_t* iters_out,
                            double* relres_out) {
  clear_error();
  if (!h) return set_error(SPX_INVALID_ARG, "cg_solve: NULL handle");
  Work w;
  SPX_TRY(handle_work(h, &w, cg_form(h, h->A) == 2 ? 9 : 4));
  return cg_solve_impl(h, w, h->A, b, x, rtol, maxit, check_every,
                       static_cast<hipStream_t>(stream), iters_out, relres_out);
}

extern "C" int spx_cg_solve_transpose(spx_handle h, const double* b, double* x, double rtol,
                                      int64_t maxit, int32_t check_every, void* stream,
                                      int64_t* iters_out, double* relres_out) {
  clear_error();
  if (!h) return set_error(SPX_INVALID_ARG, "cg_solve_transpose: NULL handle");
  hipStream_t s = static_cast<hipStream_t>(stream);
  SPX_TRY(ensure_transpose(h, s));
  Work w;
  SPX_TRY(handle_work(h, &w, cg_form(h, h->At) == 2 ? 9 : 4));
  return cg_solve_impl(h, w, h->At, b, x, rtol, maxit, check_every, s, iters_out, relres_out);
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
  if (maxit_inner > INT32_MAX - 1) maxit_inner = INT32_MAX - 1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Work w;
  SPX_TRY(handle_work(h, &w));
  SPX_TRY(ensure_solver32(h));
  SPX_TRY(ensure_val32(h, s));
  const Csr& M = h->A;
  const int64_t n = M.n;
  const SpmvShape sh = solver_shape(h, M);
  const Op<double> A64{n, M.rowptr, M.col, M.val, sh, win_view(M)};
  const Op<float> A32{n, M.rowptr, M.col, M.val32, spmv_shape32(h, M), win_view(M)};
  float* r32 = h->work32;
  float* d32 = h->work32 + n;
  float* p32 = h->work32 + 2 * n;
  float* q32 = h->work32 + 3 * n;
  CgScalars* so = w.scal;
  CgScalars* si = w.scal + 1;
  const unsigned G = (unsigned)fused_blocks(h);
  hipLaunchKernelGGL(k_scal_reset, dim3(1), dim3(64), 0, s, so, (int32_t)0);
  hipLaunchKernelGGL(k_scal_reset, dim3(1), dim3(64), 0, s, si, (int32_t)maxit_inner);
  hipLaunchKernelGGL(k_dinv, dim3(grid1(n)), dim3(256), 0, s, n, M.val, M.dpos, w.dinv, h->dinv32,
                     so);
  hipLaunchKernelGGL(k_norm2, dim3(G), dim3(kBlock), 0, s, n, b, w.partials);
  hipLaunchKernelGGL(k_norm2_finish, dim3(1), dim3(kBlock), 0, s, so, w.partials, (int64_t)G,
                     rtol_outer);
  SPX_CHECK_HIP(hipGetLastError());
  int64_t outer = 0, inner = 0;
  int status = SPX_OK;
  for (;;) {
    SPX_TRY(with_shape<true>(sh, [&](auto shc) {
      using SH = decltype(shc);
      hipLaunchKernelGGL((k_ir_residual<SH>), dim3(G), dim3(kBlock), shape_lds<double>(sh), s, n,
                         M.rowptr, M.col, M.val, b, x, h->dinv32, r32, d32, p32, w.partials,
                         sh.rows, remap_for(h, sh), sh.tile, A64.win);
      return SPX_OK;
    }));
    hipLaunchKernelGGL(k_ir_finish, dim3(1), dim3(kBlock), 0, s, so, si, w.partials, (int64_t)G,
                       rtol_inner, h->ir_early_exit);
    SPX_CHECK_HIP(hipMemcpyAsync(&w.host[2], so, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
    SPX_CHECK_HIP(hipStreamSynchronize(s));
    const CgScalars o = w.host[2];
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
    SPX_TRY(run_hs<float>(h, w, A32, d32, r32, p32, q32, h->dinv32, si, maxit_inner, check_every, s,
                          &fin));
    inner += fin.iters;
    hipLaunchKernelGGL(k_ir_update, dim3(G), dim3(kBlock), 0, s, n, x, d32);
    if (fin.status == SPX_BREAKDOWN) {
      status = SPX_BREAKDOWN;
      break;
    }
  }
  SPX_TRY(enqueue_resnorm(h, w, A64, b, x, so, s));
  SPX_CHECK_HIP(hipMemcpyAsync(&w.host[2], so, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
  SPX_CHECK_HIP(hipStreamSynchronize(s));
  const CgScalars& f = w.host[2];
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

// ------------------------------------------------ solve without allocation
//
// spx_cg_solve_noalloc runs spx_cg_solve's kernels in the library's own
// device array `scratch` instead of the handle's lazily allocated workspace.
// Layout (doubles, every part 256-byte aligned): the two solver scalar
// blocks, the workgroup partials, r, p, q, u packed at stride n as in the
// handle's workspace, and the inverse diagonal after four times
// SPX_NOALLOC_MAX_ROWS (rounded up to 32).

namespace spx {
namespace {

constexpr int64_t kNoallocMaxBlocks = 4096;  // workgroups of a solver kernel
constexpr int64_t kScratchScal = 2 * ((sizeof(CgScalars) + 255) / 256) * 32;
constexpr int64_t kScratchPartials = 4 * kNoallocMaxBlocks;
constexpr int64_t kScratchStride = (SPX_NOALLOC_MAX_ROWS + 31) / 32 * 32;
constexpr int64_t kScratchDoubles = kScratchScal + kScratchPartials + 5 * kScratchStride;
constexpr int kScratchDevices = 64;

}  // namespace
}  // namespace spx

static __device__ __align__(256) double scratch[spx::kScratchDoubles];

namespace spx {
namespace {

std::mutex g_scratch_mu;
double* g_scratch_dev[kScratchDevices] = {};

// Device address of `scratch` on device `dev` (the current device), looked
// up on the first call there and kept: each GPU holds its own copy of the
// array at its own address, and host code must never use the array's name.
int scratch_on_device(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= kScratchDevices)
    return set_error(SPX_INVALID_ARG, "cg_solve_noalloc: device %d out of range", dev);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(SPX_HIP_ERROR, "cg_solve_noalloc: scratch address on device %d: %s", dev,
                       hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return SPX_OK;
}

}  // namespace
}  // namespace spx

extern "C" int spx_cg_solve_noalloc(spx_handle h, const double* b, double* x, double rtol,
                                    int64_t maxit, int32_t check_every, void* stream,
                                    int64_t* iters_out, double* relres_out) {
  clear_error();
  if (!h) return set_error(SPX_INVALID_ARG, "cg_solve_noalloc: NULL handle");
  const int64_t n = h->n;
  if (n > SPX_NOALLOC_MAX_ROWS)
    return set_error(SPX_INVALID_ARG, "cg_solve_noalloc: %lld rows exceed the limit of %d",
                     (long long)n, SPX_NOALLOC_MAX_ROWS);
  const int64_t G = std::max(fused_blocks(h), vector_blocks(h));
  if (G > kNoallocMaxBlocks)
    return set_error(SPX_INVALID_ARG,
                     "cg_solve_noalloc: %lld workgroups per solver kernel exceed the limit of %lld",
                     (long long)G, (long long)kNoallocMaxBlocks);
  if (cg_form(h, h->A) == 2)
    return set_error(SPX_INVALID_ARG,
                     "cg_solve_noalloc: the pipelined form needs nine vectors, the scratch holds four");
  int dev = -1;
  SPX_CHECK_HIP(hipGetDevice(&dev));
  if (dev != h->device)
    return set_error(SPX_INVALID_ARG,
                     "cg_solve_noalloc: the current device %d is not the handle's device %d", dev,
                     h->device);
  double* base = nullptr;
  SPX_TRY(scratch_on_device(dev, &base));
  Work w;
  w.scal = reinterpret_cast<CgScalars*>(base);
  w.partials = base + kScratchScal;
  w.vec = w.partials + kScratchPartials;
  w.dinv = w.vec + 4 * kScratchStride;
  CgScalars host[4];  // pageable: read only after the stream is synchronised
  w.host = host;
  w.ev = nullptr;
  return cg_solve_impl(h, w, h->A, b, x, rtol, maxit, check_every,
                       static_cast<hipStream_t>(stream), iters_out, relres_out, true);
}
