// Jacobi-CG of one system run entirely by one workgroup of BLOCK threads
// (paper Sec. 6 recurrences, the K1..K3 path's order of tests and
// statuses), shared by the single-system small solve (cg.hip) and the
// persistent batched solve (batched.hip).  The SpMV is the in-order stream
// walk over tiles of ROWS <= BLOCK rows, its products staged in `prod`
// (LDS, at least as many doubles as the largest tile has entries); the dots
// are workgroup sums.  No kernel is launched per iteration and no other
// workgroup is waited for.
#pragma once

#include <cmath>

#include "common.hpp"
#include "device.hpp"
#include "spmv_core.hpp"

namespace spx {
namespace one {

// Workgroup sum returned to every thread (every thread adds the per-wave
// sums in the same order).  lds: BLOCK / 64 doubles.
template <int BLOCK>
__device__ __forceinline__ double allsum(double v, double* lds) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < BLOCK / 64; ++i) r += lds[i];
  __syncthreads();
  return r;
}

// Solves A x = b from the guess in x with D^-1 in dinv; r, p, q are n-entry
// work vectors.  status0 / maxit: the solve's entry status (a nonzero one,
// e.g. a zero diagonal, stops it before any iteration) and iteration limit.
// Thread 0 stores the outcome in *st (done = 1).
// EAGER: the products' loads issued together (stream_rows): faster with
// many workgroups solving at once (the persistent batch), not for one
// system alone.  Members per thread and chunk: 8, or 6 in the eager form
// (2048 small systems: CG 12.4 ms at 6, 12.5 at 8, 13.1 at 4).
template <bool EAGER>
constexpr int kOneDepth = EAGER ? 6 : 8;
template <int BLOCK, int ROWS, bool EAGER = false>
__device__ __forceinline__ void cg_solve(int64_t n, const int32_t* __restrict__ rowptr,
                                         const int32_t* __restrict__ col,
                                         const double* __restrict__ val,
                                         const double* __restrict__ b, double* __restrict__ x,
                                         double* __restrict__ r, double* __restrict__ p,
                                         double* __restrict__ q, const double* __restrict__ dinv,
                                         int32_t status0, int32_t maxit, double rtol,
                                         CgScalars* st, double* prod, double* lds) {
  static_assert(ROWS <= BLOCK, "one thread per row of a tile");
  const int tid = threadIdx.x;
  // r = b - A x; p = D^-1 r
  double rz = 0.0, rr = 0.0, bb = 0.0;
  for (int64_t r0 = 0; r0 < n; r0 += ROWS) {
    const int64_t r1 = r0 + ROWS < n ? r0 + ROWS : n;
    const double ax = stream_rows<BLOCK, kOneDepth<EAGER>, double, double, double, false, EAGER>(
        rowptr, col, val, x, r0, r1, prod);
    if (tid < r1 - r0) {
      const int64_t row = r0 + tid;
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
  rz = allsum<BLOCK>(rz, lds);
  rr = allsum<BLOCK>(rr, lds);
  bb = allsum<BLOCK>(bb, lds);
  const double bnorm = sqrt(bb);
  const double thresh = rtol * bnorm;
  int32_t status = status0, iters = 0;
  double rho = rz, pq = 0.0;
  bool done = true;
  if (status != SPX_OK) {
  } else if (sqrt(rr) <= thresh) {
  } else if (maxit <= 0) {
    status = SPX_NOT_CONVERGED;
  } else {
    done = false;
  }
  for (int32_t k = 1; !done; ++k) {
    // q = A p; p.q
    double pqs = 0.0;
    for (int64_t r0 = 0; r0 < n; r0 += ROWS) {
      const int64_t r1 = r0 + ROWS < n ? r0 + ROWS : n;
      const double s = stream_rows<BLOCK, kOneDepth<EAGER>, double, double, double, false, EAGER>(
          rowptr, col, val, p, r0, r1, prod);
      if (tid < r1 - r0) {
        q[r0 + tid] = s;
        pqs += p[r0 + tid] * s;
      }
    }
    pq = allsum<BLOCK>(pqs, lds);
    if (!(pq > 0.0) || !isfinite(pq)) {
      status = SPX_BREAKDOWN;
      iters = k - 1;
      break;
    }
    const double alpha = rho / pq;
    double rzs = 0.0, rrs = 0.0;
    for (int64_t i = tid; i < n; i += BLOCK) {
      const double xi = x[i] + alpha * p[i];
      const double ri = r[i] - alpha * q[i];
      const double zi = dinv[i] * ri;
      x[i] = xi;
      r[i] = ri;
      rzs += ri * zi;
      rrs += ri * ri;
    }
    rz = allsum<BLOCK>(rzs, lds);
    rr = allsum<BLOCK>(rrs, lds);
    iters = k;
    if (sqrt(rr) <= thresh) {
      status = SPX_OK;
      break;
    }
    if (k >= maxit) {
      status = SPX_NOT_CONVERGED;
      break;
    }
    const double beta = rz / rho;
    rho = rz;
    for (int64_t i = tid; i < n; i += BLOCK) p[i] = dinv[i] * r[i] + beta * p[i];
    __syncthreads();  // p is gathered by every thread in the next product
  }
  if (tid == 0) {
    st->rho[0] = rho;
    st->pq = pq;
    st->rr = rr;
    st->bb = bb;
    st->bnorm = bnorm;
    st->thresh = thresh;
    st->iters = iters;
    st->status = status;
    st->done = 1;
  }
}

}  // namespace one
}  // namespace spx
