// The batched non-symmetric Krylov methods for one system run entirely by
// one workgroup of BLOCK threads: the persistent form of the batched
// solvers (paper Sec. 7: one team per system, one launch).  Same
// recurrences, tests and statuses as the launch-per-phase kernels of
// batched_krylov.hip (BiCG with left Jacobi and the shadow residual started
// at r; TFQMR with right Jacobi, cycles whose end on the residual bound is
// checked against the true residual and restarted from x when it fails);
// the dots are workgroup sums, so the iterates agree with those kernels'
// to rounding.  Products are the in-order stream walk over tiles of ROWS
// rows staged in `prod`.  Thread 0 stores the outcome in *st (done = 1).
#pragma once

#include <cmath>

#include "cg_one.hpp"
#include "common.hpp"
#include "spmv_core.hpp"

namespace spx {
namespace one {

// Calls f(row, (A v)[row]) for every row, on the row's owner thread.
template <int BLOCK, int ROWS, class F>
__device__ __forceinline__ void walk(int64_t n, const int32_t* __restrict__ rowptr,
                                     const int32_t* __restrict__ col,
                                     const double* __restrict__ val, const double* __restrict__ v,
                                     double* prod, F&& f) {
  for (int64_t r0 = 0; r0 < n; r0 += ROWS) {
    const int64_t r1 = r0 + ROWS < n ? r0 + ROWS : n;
    const double s = stream_rows<BLOCK, kOneDepth<true>, double, double, double, false, true>(
        rowptr, col, val, v, r0, r1, prod);
    if (threadIdx.x < r1 - r0) f(r0 + threadIdx.x, s);
  }
}

struct Csr3 {
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
};

template <int BLOCK, int ROWS>
__device__ __forceinline__ void bicg_solve(int64_t n, Csr3 A, Csr3 At,
                                           const double* __restrict__ b, double* __restrict__ x,
                                           double* __restrict__ r, double* __restrict__ rh,
                                           double* __restrict__ p, double* __restrict__ ph,
                                           double* __restrict__ q, double* __restrict__ qh,
                                           const double* __restrict__ dinv, int32_t status0,
                                           int32_t maxit, double rtol, CgScalars* st, double* prod,
                                           double* lds) {
  const int tid = threadIdx.x;
  // r = b - A x; rh = r; p = ph = D^-1 r
  double rz = 0.0, rr = 0.0, bb = 0.0;
  walk<BLOCK, ROWS>(n, A.rowptr, A.col, A.val, x, prod, [&](int64_t i, double ax) {
    const double bi = b[i];
    const double ri = bi - ax;
    const double zi = dinv[i] * ri;
    r[i] = ri;
    rh[i] = ri;
    p[i] = zi;
    ph[i] = zi;
    rz += ri * zi;
    rr += ri * ri;
    bb += bi * bi;
  });
  rz = allsum<BLOCK>(rz, lds);
  rr = allsum<BLOCK>(rr, lds);
  bb = allsum<BLOCK>(bb, lds);
  const double bnorm = sqrt(bb);
  const double thresh = rtol * bnorm;
  int32_t status = status0, iters = 0;
  double rho = rz, sigma = 0.0;
  bool done = true;
  if (status != SPX_OK) {
  } else if (sqrt(rr) <= thresh) {
  } else if (maxit <= 0) {
    status = SPX_NOT_CONVERGED;
  } else {
    done = false;
  }
  for (int32_t k = 1; !done; ++k) {
    // q = A p, qh = A^T ph; ph.q
    double dot = 0.0;
    walk<BLOCK, ROWS>(n, A.rowptr, A.col, A.val, p, prod, [&](int64_t i, double v) {
      q[i] = v;
      dot += ph[i] * v;
    });
    walk<BLOCK, ROWS>(n, At.rowptr, At.col, At.val, ph, prod, [&](int64_t i, double v) { qh[i] = v; });
    sigma = allsum<BLOCK>(dot, lds);
    if (sigma == 0.0 || !isfinite(sigma)) {
      status = SPX_BREAKDOWN;
      iters = k - 1;
      break;
    }
    const double alpha = rho / sigma;
    double rzs = 0.0, rrs = 0.0;
    for (int64_t i = tid; i < n; i += BLOCK) {
      const double xi = x[i] + alpha * p[i];
      const double ri = r[i] - alpha * q[i];
      const double rhi = rh[i] - alpha * qh[i];
      const double zi = dinv[i] * ri;
      x[i] = xi;
      r[i] = ri;
      rh[i] = rhi;
      rzs += rhi * zi;
      rrs += ri * ri;
    }
    const double rz_new = allsum<BLOCK>(rzs, lds);
    rr = allsum<BLOCK>(rrs, lds);
    iters = k;
    const bool conv = sqrt(rr) <= thresh;
    if (conv) {
      status = SPX_OK;
      break;
    }
    if (rz_new == 0.0 || !isfinite(rz_new)) {
      status = SPX_BREAKDOWN;
      break;
    }
    if (k >= maxit) {
      status = SPX_NOT_CONVERGED;
      break;
    }
    const double bt = rz_new / rho;
    rho = rz_new;
    for (int64_t i = tid; i < n; i += BLOCK) {
      p[i] = dinv[i] * r[i] + bt * p[i];
      ph[i] = dinv[i] * rh[i] + bt * ph[i];
    }
    __syncthreads();  // p and ph are gathered by every thread in the next products
  }
  if (tid == 0) {
    st->rho[0] = rho;
    st->pq = sigma;
    st->rr = rr;
    st->bb = bb;
    st->bnorm = bnorm;
    st->thresh = thresh;
    st->iters = iters;
    st->status = status;
    st->done = 1;
  }
}

struct TqVectors {
  double *w, *u, *uh, *v, *au, *t, *d, *rs;
};

// r = b - A x; w = u = rs = r; uh = D^-1 r; d = t = v = 0.  Returns r.r
// (every thread) and adds b.b into *bb when bb is given.
template <int BLOCK, int ROWS>
__device__ __forceinline__ double tq_start(int64_t n, Csr3 A, const double* __restrict__ b,
                                           const double* __restrict__ x, const TqVectors& V,
                                           const double* __restrict__ dinv, double* prod,
                                           double* lds, double* bb) {
  double rr = 0.0, bs = 0.0;
  walk<BLOCK, ROWS>(n, A.rowptr, A.col, A.val, x, prod, [&](int64_t i, double ax) {
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
    bs += bi * bi;
  });
  rr = allsum<BLOCK>(rr, lds);
  if (bb) *bb = allsum<BLOCK>(bs, lds);
  return rr;
}

// theta, tau and eta of one half-step from ||w||^2 and the previous tau.
__device__ __forceinline__ void tq_half(double ww, double tau_prev, double alpha, double& theta,
                                        double& tau, double& eta) {
  theta = sqrt(ww) / tau_prev;
  const double c = 1.0 / sqrt(1.0 + theta * theta);
  tau = tau_prev * theta * c;
  eta = c * c * alpha;
}

template <int BLOCK, int ROWS>
__device__ __forceinline__ void tfqmr_solve(int64_t n, Csr3 A, const double* __restrict__ b,
                                            double* __restrict__ x, const TqVectors& V,
                                            const double* __restrict__ dinv, int32_t status0,
                                            int32_t maxit, int32_t max_restarts, double rtol,
                                            CgScalars* st, double* prod, double* lds) {
  const int tid = threadIdx.x;
  double bb = 0.0;
  double rr = tq_start<BLOCK, ROWS>(n, A, b, x, V, dinv, prod, lds, &bb);
  const double bnorm = sqrt(bb);
  const double thresh = rtol * bnorm;
  double rho = rr, tau = sqrt(rr), theta = 0.0, eta = 0.0, beta = 0.0, sigma = 0.0;
  int32_t status = status0, iters = 0, restarts = 0;
  int64_t j0 = 0, m0 = 0;
  bool done = true;
  if (status != SPX_OK) {
  } else if (tau <= thresh) {
  } else if (maxit <= 0) {
    status = SPX_NOT_CONVERGED;
  } else {
    done = false;
  }
  for (int64_t j = 0; !done; ++j) {
    // au = A uh; v = au + beta (t + beta v); rs.v
    double sg = 0.0;
    walk<BLOCK, ROWS>(n, A.rowptr, A.col, A.val, V.uh, prod, [&](int64_t i, double a) {
      const double vi = a + beta * (V.t[i] + beta * V.v[i]);
      V.au[i] = a;
      V.v[i] = vi;
      sg += V.rs[i] * vi;
    });
    sigma = allsum<BLOCK>(sg, lds);
    if (sigma == 0.0 || !isfinite(sigma)) {
      status = SPX_BREAKDOWN;
      iters = (int32_t)(m0 + 2 * (j - j0));
      break;
    }
    const double alpha = rho / sigma;
    const double coef = theta * theta * eta / alpha;
    double ws = 0.0;
    for (int64_t i = tid; i < n; i += BLOCK) {
      const double wi = V.w[i] - alpha * V.au[i];
      const double di = V.uh[i] + coef * V.d[i];
      const double ui = V.u[i] - alpha * V.v[i];
      V.w[i] = wi;
      V.d[i] = di;
      V.u[i] = ui;
      V.uh[i] = dinv[i] * ui;
      ws += wi * wi;
    }
    double ww = allsum<BLOCK>(ws, lds);
    // half-step 2j + 1
    tq_half(ww, tau, alpha, theta, tau, eta);
    int64_t ml = 2 * (j - j0) + 1;
    iters = (int32_t)(m0 + ml);
    bool passed = sqrt((double)(ml + 1)) * tau <= thresh;
    bool verify = false;
    if (passed || iters >= maxit) {
      for (int64_t i = tid; i < n; i += BLOCK) x[i] = x[i] + eta * V.d[i];
      if (!passed) {
        status = SPX_NOT_CONVERGED;
        break;
      }
      verify = true;
    } else {
      // d = uh + coef d (x += eta d first); t = A uh; w -= alpha t
      const double coef2 = theta * theta * eta / alpha;
      double w2 = 0.0, wr = 0.0;
      walk<BLOCK, ROWS>(n, A.rowptr, A.col, A.val, V.uh, prod, [&](int64_t i, double y) {
        const double d0 = V.d[i];
        x[i] = x[i] + eta * d0;
        V.d[i] = V.uh[i] + coef2 * d0;
        V.t[i] = y;
        const double wi = V.w[i] - alpha * y;
        V.w[i] = wi;
        w2 += wi * wi;
        wr += V.rs[i] * wi;
      });
      ww = allsum<BLOCK>(w2, lds);
      const double rho_new = allsum<BLOCK>(wr, lds);
      // half-step 2j + 2
      tq_half(ww, tau, alpha, theta, tau, eta);
      ml = 2 * (j - j0) + 2;
      iters = (int32_t)(m0 + ml);
      passed = sqrt((double)(ml + 1)) * tau <= thresh;
      const bool limit = !passed && iters >= maxit;
      const bool broke = !passed && !limit && (rho_new == 0.0 || !isfinite(rho_new));
      if (passed || limit || broke) {
        for (int64_t i = tid; i < n; i += BLOCK) x[i] = x[i] + eta * V.d[i];
        if (!passed) {
          status = limit ? SPX_NOT_CONVERGED : SPX_BREAKDOWN;
          break;
        }
        verify = true;
      } else {
        beta = rho_new / rho;
        rho = rho_new;
        for (int64_t i = tid; i < n; i += BLOCK) {
          x[i] = x[i] + eta * V.d[i];
          const double ui = V.w[i] + beta * V.u[i];
          V.u[i] = ui;
          V.uh[i] = dinv[i] * ui;
        }
      }
    }
    if (verify) {
      // the cycle ended on its bound: the true residual decides
      __syncthreads();  // x is gathered by every thread
      rr = tq_start<BLOCK, ROWS>(n, A, b, x, V, dinv, prod, lds, nullptr);
      const double t = sqrt(rr);
      if (t <= thresh) {
        status = SPX_OK;
        break;
      }
      if (restarts >= max_restarts || iters >= maxit) {
        status = SPX_NOT_CONVERGED;
        break;
      }
      restarts += 1;
      rho = rr;
      tau = t;
      theta = eta = beta = 0.0;
      j0 = j + 1;
      m0 = iters;
    }
    __syncthreads();  // uh is gathered by every thread in the next product
  }
  if (tid == 0) {
    st->rho[0] = rho;
    st->tau[0] = tau;
    st->pq = sigma;
    st->rr = rr;
    st->bb = bb;
    st->bnorm = bnorm;
    st->thresh = thresh;
    st->iters = iters;
    st->restarts = restarts;
    st->status = status;
    st->done = 1;
  }
}

}  // namespace one
}  // namespace spx
