/*
 * CPU oracle for COO assembly, CSR products and Jacobi-preconditioned CG.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously
 * correct statement of what the GPU path computes.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or constant with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math),
 * so every floating-point operation below is evaluated exactly as written,
 * in the written order.
 *
 * Threads.  The row loops of the products, the element-wise vector updates
 * of the solvers and the 4096-element blocks of the dot products may run on
 * several OpenMP threads (oracle_set_threads).  Each output element and each
 * block sum is still formed by one thread in the written order, and block
 * sums are added in block order by one thread, so every result is bitwise
 * the same for any thread count.  The COO assembly and the other solvers
 * stay sequential.
 *
 * Status codes (same meaning as the GPU library's, defined independently):
 *   0 ok, -1 invalid argument, -2 index out of range, -4 zero diagonal,
 *   -5 not converged, -6 breakdown.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_INVALID (-1)
#define OR_RANGE (-2)
#define OR_ZERO_DIAG (-4)
#define OR_NOT_CONVERGED (-5)
#define OR_BREAKDOWN (-6)

/* Loops over n independent elements go parallel from this length on. */
#define PAR_MIN 32768
#define PAR_FOR _Pragma("omp parallel for schedule(static) if (n >= PAR_MIN)")

void oracle_set_threads(int nthreads) { omp_set_num_threads(nthreads > 0 ? nthreads : 1); }
int oracle_get_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------
 * COO -> CSR (paper Sec. 5, "Portable matrix assembly on GPUs").
 *
 * Definition: A is the sum of the contributions v[k] to entry
 * (i[k], j[k]); a triplet with a negative row or column index is ignored.
 * The stored pattern is the set of distinct (i, j) among the kept
 * triplets (it comes from the indices alone, so an entry whose
 * contributions cancel to 0.0 is still stored), rows ascending and columns
 * ascending within a row.  Each entry is the sum of its contributions in
 * increasing k, starting from +0.0.
 *
 * Helper maps: perm = the kept k sorted by (i, j) with ties in increasing
 * k; jmap[t] .. jmap[t+1]-1 is the run of perm that feeds stored entry t.
 * ---------------------------------------------------------------------- */

typedef struct {
  int32_t i, j;
  int64_t k;
} coo_key;

static int cmp_key(const void* pa, const void* pb) {
  const coo_key* a = (const coo_key*)pa;
  const coo_key* b = (const coo_key*)pb;
  if (a->i != b->i) return a->i < b->i ? -1 : 1;
  if (a->j != b->j) return a->j < b->j ? -1 : 1;
  if (a->k != b->k) return a->k < b->k ? -1 : 1;
  return 0;
}

/* rowptr[n+1], col[ncoo], jmap[ncoo+1], perm[ncoo] are caller-allocated
 * with room for the worst case (every kept triplet distinct).
 *
 * The sort is two stable counting sorts of the kept k: by column, then by
 * row.  The second pass keeps the column order of equal rows and the first
 * keeps the increasing k of equal (i, j), so perm ends ordered by (i, j)
 * with ties in increasing k. */
int oracle_coo_pattern(int64_t n, int64_t ncoo, const int32_t* i, const int32_t* j,
                       int32_t* rowptr, int32_t* col, int64_t* jmap, int32_t* perm,
                       int64_t* nnz_out, int64_t* nvalid_out) {
  if (n <= 0 || ncoo < 0) return OR_INVALID;
  int64_t nvalid = 0;
  for (int64_t k = 0; k < ncoo; k++) {
    if (i[k] < 0 || j[k] < 0) continue;
    if (i[k] >= n || j[k] >= n) return OR_RANGE;
    nvalid++;
  }
  int64_t* start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int32_t* by_col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nvalid > 0 ? nvalid : 1));
  if (!start || !by_col) {
    free(start);
    free(by_col);
    return OR_INVALID;
  }
  /* pass 1: kept k in increasing k, placed by column */
  for (int64_t c = 0; c <= n; c++) start[c] = 0;
  for (int64_t k = 0; k < ncoo; k++)
    if (i[k] >= 0 && j[k] >= 0) start[j[k] + 1]++;
  for (int64_t c = 0; c < n; c++) start[c + 1] += start[c];
  for (int64_t k = 0; k < ncoo; k++)
    if (i[k] >= 0 && j[k] >= 0) by_col[start[j[k]]++] = (int32_t)k;
  /* pass 2: that sequence, placed by row */
  for (int64_t r = 0; r <= n; r++) start[r] = 0;
  for (int64_t q = 0; q < nvalid; q++) start[i[by_col[q]] + 1]++;
  for (int64_t r = 0; r < n; r++) start[r + 1] += start[r];
  for (int64_t q = 0; q < nvalid; q++) perm[start[i[by_col[q]]]++] = by_col[q];
  free(by_col);
  free(start);

  int64_t nnz = 0;
  for (int64_t r = 0; r <= n; r++) rowptr[r] = 0;
  for (int64_t q = 0; q < nvalid; q++) {
    const int64_t k = perm[q];
    int first = (q == 0) || i[k] != i[perm[q - 1]] || j[k] != j[perm[q - 1]];
    if (first) {
      jmap[nnz] = q;
      col[nnz] = j[k];
      rowptr[i[k] + 1] += 1; /* count entries per row */
      nnz++;
    }
  }
  jmap[nnz] = nvalid;
  for (int64_t r = 0; r < n; r++) rowptr[r + 1] += rowptr[r];
  *nnz_out = nnz;
  *nvalid_out = nvalid;
  return OR_OK;
}

/* mode 0 = INSERT (a[t] = sum), 1 = ADD (a[t] = a[t] + sum). */
void oracle_coo_values(int64_t nnz, const int64_t* jmap, const int32_t* perm, const double* v,
                       int mode, double* val) {
  for (int64_t t = 0; t < nnz; t++) {
    double s = 0.0;
    for (int64_t q = jmap[t]; q < jmap[t + 1]; q++) s += v[perm[q]];
    if (mode == 1)
      val[t] = val[t] + s;
    else
      val[t] = s;
  }
}

/* kslot[k] = stored entry that triplet k feeds, or -1 when k is ignored. */
void oracle_coo_slots(int64_t ncoo, int64_t nnz, const int64_t* jmap, const int32_t* perm,
                      int32_t* kslot) {
  for (int64_t k = 0; k < ncoo; k++) kslot[k] = -1;
  for (int64_t t = 0; t < nnz; t++)
    for (int64_t q = jmap[t]; q < jmap[t + 1]; q++) kslot[perm[q]] = (int32_t)t;
}

/* Entries of the selected rows only, straight from the triplets: for each
 * selected row r (rows[s], strictly increasing), the distinct columns in
 * ascending order and their in-order sums.  Used to check very large
 * assemblies on a sample of rows.  out_ptr[nrows+1], out_col/out_val sized
 * by the caller (max_out).  Returns the number written or a status < 0. */
int64_t oracle_coo_rows(int64_t n, int64_t ncoo, const int32_t* i, const int32_t* j,
                        const double* v, int64_t nrows, const int32_t* rows,
                        int64_t* out_ptr, int32_t* out_col, double* out_val, int64_t max_out) {
  int32_t* slot = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!slot) return OR_INVALID;
  for (int64_t r = 0; r < n; r++) slot[r] = -1;
  for (int64_t s = 0; s < nrows; s++) slot[rows[s]] = (int32_t)s;
  int64_t cnt = 0;
  for (int64_t k = 0; k < ncoo; k++)
    if (i[k] >= 0 && j[k] >= 0 && slot[i[k]] >= 0) cnt++;
  coo_key* keys = (coo_key*)malloc(sizeof(coo_key) * (size_t)(cnt > 0 ? cnt : 1));
  int64_t m = 0;
  for (int64_t k = 0; k < ncoo; k++)
    if (i[k] >= 0 && j[k] >= 0 && slot[i[k]] >= 0) {
      keys[m].i = i[k];
      keys[m].j = j[k];
      keys[m].k = k;
      m++;
    }
  qsort(keys, (size_t)cnt, sizeof(coo_key), cmp_key);
  int64_t w = 0, q = 0;
  for (int64_t s = 0; s < nrows; s++) {
    out_ptr[s] = w;
    while (q < cnt && keys[q].i == rows[s]) {
      int32_t c = keys[q].j;
      double acc = 0.0;
      while (q < cnt && keys[q].i == rows[s] && keys[q].j == c) {
        acc += v[keys[q].k];
        q++;
      }
      if (w >= max_out) {
        free(keys);
        free(slot);
        return OR_INVALID;
      }
      out_col[w] = c;
      out_val[w] = acc;
      w++;
    }
  }
  out_ptr[nrows] = w;
  free(keys);
  free(slot);
  return w;
}

/* COO vector assembly (paper Sec. 5, VecSetValuesCOO): x[i] = (x[i] +) the
 * in-order sum from +0.0 of v[k] over kept k with i[k] = i, for every i that
 * some kept triplet names; other entries unchanged.  Returns -2 if an index
 * is >= n (x untouched). */
int oracle_vec_coo(int64_t n, int64_t ncoo, const int32_t* i, const double* v, int mode,
                   double* x) {
  for (int64_t k = 0; k < ncoo; k++)
    if (i[k] >= n) return OR_RANGE;
  double* s = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  char* seen = (char*)calloc((size_t)(n > 0 ? n : 1), 1);
  for (int64_t r = 0; r < n; r++) s[r] = 0.0;
  for (int64_t k = 0; k < ncoo; k++) {
    if (i[k] < 0) continue;
    s[i[k]] = s[i[k]] + v[k];
    seen[i[k]] = 1;
  }
  for (int64_t r = 0; r < n; r++)
    if (seen[r]) x[r] = mode == 1 ? x[r] + s[r] : s[r];
  free(s);
  free(seen);
  return OR_OK;
}

/* ------------------------------------------------------------------------
 * CSR products (MatMult / MatMultTranspose, paper Sec. 6).
 * ---------------------------------------------------------------------- */

void oracle_spmv(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                 const double* x, double* y) {
  PAR_FOR
  for (int64_t r = 0; r < n; r++) {
    double s = 0.0;
    for (int64_t t = rowptr[r]; t < rowptr[r + 1]; t++) s += val[t] * x[col[t]];
    y[r] = s;
  }
}

void oracle_spmv_transpose(int64_t n, const int32_t* rowptr, const int32_t* col,
                           const double* val, const double* x, double* y) {
  for (int64_t c = 0; c < n; c++) y[c] = 0.0;
  for (int64_t r = 0; r < n; r++)
    for (int64_t t = rowptr[r]; t < rowptr[r + 1]; t++) y[col[t]] += val[t] * x[r];
}

/* Y = A X for a row-major block: X[c*ldx + s], Y[r*ldy + s], s < nrhs. */
void oracle_spmm(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                 int64_t nrhs, const double* X, int64_t ldx, double* Y, int64_t ldy) {
  for (int64_t r = 0; r < n; r++)
    for (int64_t s = 0; s < nrhs; s++) {
      double acc = 0.0;
      for (int64_t t = rowptr[r]; t < rowptr[r + 1]; t++) acc += val[t] * X[(int64_t)col[t] * ldx + s];
      Y[r * ldy + s] = acc;
    }
}

/* ------------------------------------------------------------------------
 * Jacobi-preconditioned CG (Hestenes-Stiefel form), paper Sec. 6: the
 * solver is PETSc's CG, built from MatMult, dot products, AXPY updates,
 * scalar divisions and a residual-norm convergence test.
 *
 *   r = b - A x;  z = D^-1 r;  p = z;  rho = r.z
 *   repeat:  q = A p;  pq = p.q  (pq <= 0 or not finite: breakdown)
 *            alpha = rho / pq;  x += alpha p;  r -= alpha q
 *            stop when ||r|| <= rtol ||b||
 *            z = D^-1 r;  rho' = r.z;  beta = rho' / rho;  p = z + beta p
 *
 * Dot products add fixed 4096-element blocks, each summed in order, then
 * the block sums in order, so a parallel evaluation could reproduce them.
 * ---------------------------------------------------------------------- */

#define DOT_BLOCK 4096

static double dot64(int64_t n, const double* a, const double* b) {
  const int64_t nb = (n + DOT_BLOCK - 1) / DOT_BLOCK;
  double* part = (double*)malloc(sizeof(double) * (size_t)(nb > 0 ? nb : 1));
#pragma omp parallel for schedule(static) if (nb >= 8)
  for (int64_t blk = 0; blk < nb; blk++) {
    int64_t s = blk * DOT_BLOCK, e = s + DOT_BLOCK < n ? s + DOT_BLOCK : n;
    double sum = 0.0;
    for (int64_t i = s; i < e; i++) sum += a[i] * b[i];
    part[blk] = sum;
  }
  double total = 0.0;
  for (int64_t blk = 0; blk < nb; blk++) total += part[blk];
  free(part);
  return total;
}

/* fp32 vectors, products and sums in fp64 */
static double dot32(int64_t n, const float* a, const float* b) {
  const int64_t nb = (n + DOT_BLOCK - 1) / DOT_BLOCK;
  double* part = (double*)malloc(sizeof(double) * (size_t)(nb > 0 ? nb : 1));
#pragma omp parallel for schedule(static) if (nb >= 8)
  for (int64_t blk = 0; blk < nb; blk++) {
    int64_t s = blk * DOT_BLOCK, e = s + DOT_BLOCK < n ? s + DOT_BLOCK : n;
    double sum = 0.0;
    for (int64_t i = s; i < e; i++) sum += (double)a[i] * (double)b[i];
    part[blk] = sum;
  }
  double total = 0.0;
  for (int64_t blk = 0; blk < nb; blk++) total += part[blk];
  free(part);
  return total;
}

static int diag_inverse(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                        double* dinv) {
  for (int64_t r = 0; r < n; r++) {
    double d = 0.0;
    for (int64_t t = rowptr[r]; t < rowptr[r + 1]; t++)
      if (col[t] == r) d = val[t];
    if (d == 0.0) return OR_ZERO_DIAG;
    dinv[r] = 1.0 / d;
  }
  return OR_OK;
}

/* x: initial guess in, solution out.  iters: iterations performed.
 * relres: true ||b - A x|| / ||b|| of the returned x (0 when b = 0). */
int oracle_pcg(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
               const double* b, double* x, double rtol, int64_t maxit, int64_t* iters,
               double* relres) {
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* z = (double*)malloc(sizeof(double) * (size_t)n);
  double* p = (double*)malloc(sizeof(double) * (size_t)n);
  double* q = (double*)malloc(sizeof(double) * (size_t)n);
  double* dinv = (double*)malloc(sizeof(double) * (size_t)n);
  int status = diag_inverse(n, rowptr, col, val, dinv);
  int64_t k = 0;
  double bnorm = sqrt(dot64(n, b, b));
  if (status == OR_OK) {
    oracle_spmv(n, rowptr, col, val, x, q);
    PAR_FOR
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
    double rnorm = sqrt(dot64(n, r, r));
    if (!(rnorm <= rtol * bnorm)) {
      PAR_FOR
      for (int64_t i = 0; i < n; i++) z[i] = dinv[i] * r[i];
      PAR_FOR
      for (int64_t i = 0; i < n; i++) p[i] = z[i];
      double rho = dot64(n, r, z);
      status = OR_NOT_CONVERGED;
      while (k < maxit) {
        oracle_spmv(n, rowptr, col, val, p, q);
        double pq = dot64(n, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) {
          status = OR_BREAKDOWN;
          break;
        }
        double alpha = rho / pq;
        PAR_FOR
        for (int64_t i = 0; i < n; i++) x[i] = x[i] + alpha * p[i];
        PAR_FOR
        for (int64_t i = 0; i < n; i++) r[i] = r[i] - alpha * q[i];
        k++;
        rnorm = sqrt(dot64(n, r, r));
        if (rnorm <= rtol * bnorm) {
          status = OR_OK;
          break;
        }
        PAR_FOR
        for (int64_t i = 0; i < n; i++) z[i] = dinv[i] * r[i];
        double rho_new = dot64(n, r, z);
        double beta = rho_new / rho;
        PAR_FOR
        for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        rho = rho_new;
      }
    }
  }
  oracle_spmv(n, rowptr, col, val, x, q);
  PAR_FOR
  for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
  *relres = bnorm > 0.0 ? sqrt(dot64(n, r, r)) / bnorm : sqrt(dot64(n, r, r));
  *iters = k;
  free(r);
  free(z);
  free(p);
  free(q);
  free(dinv);
  return status;
}

/* ------------------------------------------------------------------------
 * Single-reduction Jacobi-PCG (Chronopoulos-Gear form): the same Krylov
 * iterates in exact arithmetic, with w = A u carried so that the dots
 * (r,u), (r,r) and (w,u) of one iteration can be reduced together (the
 * paper's Sec. 6 asynchronous-solver direction: fewer synchronisation
 * points per iteration).
 *   r = b - A x; u = D^-1 r; w = A u; gamma = r.u; delta = w.u
 *   p = u; s = w; alpha = gamma / delta
 *   repeat (k = 1, 2, ...):
 *     x += alpha p; r -= alpha s; u = D^-1 r
 *     stop when ||r|| <= rtol ||b||
 *     gamma' = r.u; beta = gamma' / gamma; w = A u; delta = w.u
 *     p = u + beta p; s = w + beta s
 *     alpha = gamma' / (delta - beta gamma' / alpha); gamma = gamma'
 * A denominator <= 0 or not finite is a breakdown.
 * ---------------------------------------------------------------------- */
int oracle_pcg_single_reduction(int64_t n, const int32_t* rowptr, const int32_t* col,
                                const double* val, const double* b, double* x, double rtol,
                                int64_t maxit, int64_t* iters, double* relres) {
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* u = (double*)malloc(sizeof(double) * (size_t)n);
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  double* p = (double*)malloc(sizeof(double) * (size_t)n);
  double* s = (double*)malloc(sizeof(double) * (size_t)n);
  double* dinv = (double*)malloc(sizeof(double) * (size_t)n);
  int status = diag_inverse(n, rowptr, col, val, dinv);
  int64_t k = 0;
  double bnorm = sqrt(dot64(n, b, b));
  if (status == OR_OK) {
    oracle_spmv(n, rowptr, col, val, x, w);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - w[i];
    double rnorm = sqrt(dot64(n, r, r));
    if (!(rnorm <= rtol * bnorm)) {
      for (int64_t i = 0; i < n; i++) u[i] = dinv[i] * r[i];
      oracle_spmv(n, rowptr, col, val, u, w);
      double gamma = dot64(n, r, u);
      double delta = dot64(n, w, u);
      for (int64_t i = 0; i < n; i++) p[i] = u[i];
      for (int64_t i = 0; i < n; i++) s[i] = w[i];
      double alpha = gamma / delta;
      status = OR_NOT_CONVERGED;
      if (!(delta > 0.0) || !isfinite(delta)) {
        status = OR_BREAKDOWN;
      } else {
        while (k < maxit) {
          for (int64_t i = 0; i < n; i++) x[i] = x[i] + alpha * p[i];
          for (int64_t i = 0; i < n; i++) r[i] = r[i] - alpha * s[i];
          for (int64_t i = 0; i < n; i++) u[i] = dinv[i] * r[i];
          k++;
          rnorm = sqrt(dot64(n, r, r));
          if (rnorm <= rtol * bnorm) {
            status = OR_OK;
            break;
          }
          if (k >= maxit) break;
          double gamma_new = dot64(n, r, u);
          double beta = gamma_new / gamma;
          oracle_spmv(n, rowptr, col, val, u, w);
          delta = dot64(n, w, u);
          for (int64_t i = 0; i < n; i++) p[i] = u[i] + beta * p[i];
          for (int64_t i = 0; i < n; i++) s[i] = w[i] + beta * s[i];
          double den = delta - beta * gamma_new / alpha;
          if (!(den > 0.0) || !isfinite(den)) {
            status = OR_BREAKDOWN;
            break;
          }
          alpha = gamma_new / den;
          gamma = gamma_new;
        }
      }
    }
  }
  oracle_spmv(n, rowptr, col, val, x, w);
  for (int64_t i = 0; i < n; i++) r[i] = b[i] - w[i];
  *relres = bnorm > 0.0 ? sqrt(dot64(n, r, r)) / bnorm : sqrt(dot64(n, r, r));
  *iters = k;
  free(r);
  free(u);
  free(w);
  free(p);
  free(s);
  free(dinv);
  return status;
}

/* ------------------------------------------------------------------------
 * Pipelined Jacobi-PCG (Ghysels and Vanroose, 2014, preconditioned form):
 * the same Krylov iterates as CG in exact arithmetic, rearranged so that
 * the dots of an iteration need not finish before its next product starts
 * (the paper's Sec. 6 aim of hiding the synchronisation of the reductions).
 * With M = D:
 *   r = b - A x; u = D^-1 r; w = A u
 *   for i = 0, 1, ...:
 *     gamma = r.u; delta = w.u; ||r||    (one reduction)
 *     stop when ||r|| <= rtol ||b||      (iters = i)
 *     m = D^-1 w; nv = A m
 *     i = 0: beta = 0, alpha = gamma / delta
 *     else:  beta = gamma / gamma_prev,
 *            alpha = gamma / (delta - beta gamma / alpha_prev)
 *     z = nv + beta z; q = m + beta q; s = w + beta s; p = u + beta p
 *       (at i = 0: z = nv, q = m, s = w, p = u)
 *     x += alpha p; r -= alpha s; u -= alpha q; w -= alpha z
 * An alpha denominator <= 0 or not finite is a breakdown; i = maxit before
 * the test passes is "not converged".
 * ---------------------------------------------------------------------- */
int oracle_pcg_pipelined(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                         const double* b, double* x, double rtol, int64_t maxit, int64_t* iters,
                         double* relres) {
  double* buf = (double*)malloc(sizeof(double) * (size_t)n * 11);
  double *r = buf, *u = buf + n, *w = buf + 2 * n, *m = buf + 3 * n, *nv = buf + 4 * n;
  double *z = buf + 5 * n, *q = buf + 6 * n, *s = buf + 7 * n, *p = buf + 8 * n;
  double *dinv = buf + 9 * n, *t = buf + 10 * n;
  int status = diag_inverse(n, rowptr, col, val, dinv);
  int64_t i = 0;
  double bnorm = sqrt(dot64(n, b, b));
  if (status == OR_OK) {
    oracle_spmv(n, rowptr, col, val, x, t);
    for (int64_t e = 0; e < n; e++) r[e] = b[e] - t[e];
    for (int64_t e = 0; e < n; e++) u[e] = dinv[e] * r[e];
    oracle_spmv(n, rowptr, col, val, u, w);
    double gamma_prev = 0.0, alpha_prev = 0.0;
    status = OR_NOT_CONVERGED;
    for (;;) {
      double gamma = dot64(n, r, u);
      double delta = dot64(n, w, u);
      double rnorm = sqrt(dot64(n, r, r));
      if (rnorm <= rtol * bnorm) {
        status = OR_OK;
        break;
      }
      if (i >= maxit) break;
      for (int64_t e = 0; e < n; e++) m[e] = dinv[e] * w[e];
      oracle_spmv(n, rowptr, col, val, m, nv);
      double beta = 0.0, den = delta;
      if (i > 0) {
        beta = gamma / gamma_prev;
        den = delta - beta * gamma / alpha_prev;
      }
      if (!(den > 0.0) || !isfinite(den)) {
        status = OR_BREAKDOWN;
        break;
      }
      double alpha = gamma / den;
      if (i == 0) {
        for (int64_t e = 0; e < n; e++) z[e] = nv[e];
        for (int64_t e = 0; e < n; e++) q[e] = m[e];
        for (int64_t e = 0; e < n; e++) s[e] = w[e];
        for (int64_t e = 0; e < n; e++) p[e] = u[e];
      } else {
        for (int64_t e = 0; e < n; e++) z[e] = nv[e] + beta * z[e];
        for (int64_t e = 0; e < n; e++) q[e] = m[e] + beta * q[e];
        for (int64_t e = 0; e < n; e++) s[e] = w[e] + beta * s[e];
        for (int64_t e = 0; e < n; e++) p[e] = u[e] + beta * p[e];
      }
      for (int64_t e = 0; e < n; e++) x[e] = x[e] + alpha * p[e];
      for (int64_t e = 0; e < n; e++) r[e] = r[e] - alpha * s[e];
      for (int64_t e = 0; e < n; e++) u[e] = u[e] - alpha * q[e];
      for (int64_t e = 0; e < n; e++) w[e] = w[e] - alpha * z[e];
      gamma_prev = gamma;
      alpha_prev = alpha;
      i++;
    }
  }
  oracle_spmv(n, rowptr, col, val, x, t);
  for (int64_t e = 0; e < n; e++) r[e] = b[e] - t[e];
  *relres = bnorm > 0.0 ? sqrt(dot64(n, r, r)) / bnorm : sqrt(dot64(n, r, r));
  *iters = i;
  free(buf);
  return status;
}

/* ------------------------------------------------------------------------
 * Jacobi-preconditioned BiCG (paper Sec. 7 names BiCG with diagonal
 * preconditioning as one of the two batched Krylov methods).  Textbook
 * preconditioned biconjugate gradients with M = D = diag(A) and the shadow
 * residual started at the residual:
 *
 *   r = b - A x;  rh = r;  z = D^-1 r;  zh = D^-1 rh;  p = z;  ph = zh
 *   rho = z.rh
 *   repeat:  q = A p;  qh = A^T ph;  sigma = ph.q  (0 or not finite: breakdown)
 *            alpha = rho / sigma;  x += alpha p;  r -= alpha q;  rh -= alpha qh
 *            stop when ||r|| <= rtol ||b||
 *            z = D^-1 r;  zh = D^-1 rh;  rho' = z.rh  (0 or not finite: breakdown)
 *            beta = rho' / rho;  p = z + beta p;  ph = zh + beta ph
 *
 * On a symmetric matrix rh stays equal to r and every quantity equals the
 * CG one above, value for value.
 * ---------------------------------------------------------------------- */
int oracle_bicg(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                const double* b, double* x, double rtol, int64_t maxit, int64_t* iters,
                double* relres) {
  const size_t bytes = sizeof(double) * (size_t)n;
  double* r = (double*)malloc(bytes);
  double* rh = (double*)malloc(bytes);
  double* z = (double*)malloc(bytes);
  double* zh = (double*)malloc(bytes);
  double* p = (double*)malloc(bytes);
  double* ph = (double*)malloc(bytes);
  double* q = (double*)malloc(bytes);
  double* qh = (double*)malloc(bytes);
  double* dinv = (double*)malloc(bytes);
  int status = diag_inverse(n, rowptr, col, val, dinv);
  int64_t k = 0;
  double bnorm = sqrt(dot64(n, b, b));
  if (status == OR_OK) {
    oracle_spmv(n, rowptr, col, val, x, q);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
    for (int64_t i = 0; i < n; i++) rh[i] = r[i];
    if (!(sqrt(dot64(n, r, r)) <= rtol * bnorm)) {
      for (int64_t i = 0; i < n; i++) z[i] = dinv[i] * r[i];
      for (int64_t i = 0; i < n; i++) zh[i] = dinv[i] * rh[i];
      for (int64_t i = 0; i < n; i++) p[i] = z[i];
      for (int64_t i = 0; i < n; i++) ph[i] = zh[i];
      double rho = dot64(n, z, rh);
      status = OR_NOT_CONVERGED;
      while (k < maxit) {
        oracle_spmv(n, rowptr, col, val, p, q);
        oracle_spmv_transpose(n, rowptr, col, val, ph, qh);
        double sigma = dot64(n, ph, q);
        if (sigma == 0.0 || !isfinite(sigma)) {
          status = OR_BREAKDOWN;
          break;
        }
        double alpha = rho / sigma;
        for (int64_t i = 0; i < n; i++) x[i] = x[i] + alpha * p[i];
        for (int64_t i = 0; i < n; i++) r[i] = r[i] - alpha * q[i];
        for (int64_t i = 0; i < n; i++) rh[i] = rh[i] - alpha * qh[i];
        k++;
        if (sqrt(dot64(n, r, r)) <= rtol * bnorm) {
          status = OR_OK;
          break;
        }
        for (int64_t i = 0; i < n; i++) z[i] = dinv[i] * r[i];
        for (int64_t i = 0; i < n; i++) zh[i] = dinv[i] * rh[i];
        double rho_new = dot64(n, z, rh);
        if (rho_new == 0.0 || !isfinite(rho_new)) {
          status = OR_BREAKDOWN;
          break;
        }
        double beta = rho_new / rho;
        for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        for (int64_t i = 0; i < n; i++) ph[i] = zh[i] + beta * ph[i];
        rho = rho_new;
      }
    }
  }
  oracle_spmv(n, rowptr, col, val, x, q);
  for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
  *relres = bnorm > 0.0 ? sqrt(dot64(n, r, r)) / bnorm : sqrt(dot64(n, r, r));
  *iters = k;
  free(r);
  free(rh);
  free(z);
  free(zh);
  free(p);
  free(ph);
  free(q);
  free(qh);
  free(dinv);
  return status;
}

/* ------------------------------------------------------------------------
 * Jacobi-preconditioned TFQMR (paper Sec. 6 and Sec. 7: the transpose-free
 * quasi-minimal residual method of Freund, 1993, with diagonal
 * preconditioning), applied from the right: the method runs on A D^-1,
 * whose residual is the true residual b - A x, and its search directions
 * are mapped back by D^-1 before they update x.
 *
 * With Ap = A D^-1, shadow vector rs = r0, half-steps m = 0, 1, 2, ...
 *   w = u = r0;  au = Ap u;  v = au;  d = 0;  tau = ||r0||;
 *   theta = eta = 0;  rho = rs.r0
 *   each iteration: sigma = rs.v (0 or not finite: breakdown);
 *     alpha = rho / sigma, shared by its two half-steps.  Half-step h:
 *       h = 0: y = au (= Ap u);   h = 1: u = u - alpha v, y = Ap u
 *       w = w - alpha y
 *       d = D^-1 u + (theta^2 eta / alpha) d          (x-space direction)
 *       theta = ||w|| / tau;  c = 1 / sqrt(1 + theta^2)
 *       tau = tau theta c;  eta = c^2 alpha;  x = x + eta d
 *       m = m + 1; the cycle ends when sqrt(m + 1) tau <= rtol ||b||, the
 *       bound ||b - A x_m|| <= sqrt(m + 1) tau_m of the method (m counted
 *       within the cycle)
 *     then rho' = rs.w (0 or not finite: breakdown);  beta = rho' / rho;
 *     u_new = w + beta u;  au = Ap u_new;  v = au + beta (y + beta v)
 * (w is the residual of the unsmoothed iterate, which advances by alpha
 * times u in each half-step; v is A D^-1 applied to the combined search
 * direction, which only the u update uses.)
 * The bound holds in exact arithmetic only: the unsmoothed residuals can
 * grow by many orders of magnitude before they fall, and rounding then
 * caps the accuracy of x well above the bound.  So when a cycle ends on the
 * bound, the true residual of x decides: at most rtol ||b|| ends the
 * solve, otherwise a new cycle starts from x with r0 = b - A x (at most
 * TFQMR_MAX_RESTARTS restarts, then "not converged").  Half-steps are
 * counted over all cycles.
 * iters counts half-steps (one product with A each); bound returns
 * sqrt(m + 1) tau of the last cycle at exit.
 * ---------------------------------------------------------------------- */
#define TFQMR_MAX_RESTARTS 8

int oracle_tfqmr(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                 const double* b, double* x, double rtol, int64_t maxit, int64_t* iters,
                 double* relres, double* bound) {
  const size_t bytes = sizeof(double) * (size_t)n;
  double* r = (double*)malloc(bytes);
  double* rs = (double*)malloc(bytes);
  double* w = (double*)malloc(bytes);
  double* u = (double*)malloc(bytes);
  double* uh = (double*)malloc(bytes);
  double* v = (double*)malloc(bytes);
  double* au = (double*)malloc(bytes);
  double* y = (double*)malloc(bytes);
  double* d = (double*)malloc(bytes);
  double* dinv = (double*)malloc(bytes);
  int status = diag_inverse(n, rowptr, col, val, dinv);
  int64_t m = 0;  /* half-steps over all cycles */
  int64_t ml = 0; /* half-steps of the current cycle */
  double bnorm = sqrt(dot64(n, b, b));
  double tau = 0.0;
  if (status == OR_OK) {
    oracle_spmv(n, rowptr, col, val, x, y);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - y[i];
    tau = sqrt(dot64(n, r, r));
    int restarts = 0;
    while (!(tau <= rtol * bnorm)) {
      /* a cycle from the residual r of the current x */
      ml = 0;
      for (int64_t i = 0; i < n; i++) {
        rs[i] = r[i];
        w[i] = r[i];
        u[i] = r[i];
        d[i] = 0.0;
      }
      for (int64_t i = 0; i < n; i++) uh[i] = dinv[i] * u[i];
      oracle_spmv(n, rowptr, col, val, uh, au);
      for (int64_t i = 0; i < n; i++) v[i] = au[i];
      double theta = 0.0, eta = 0.0;
      double rho = dot64(n, rs, r);
      status = OR_NOT_CONVERGED;
      int finished = 0, passed = 0;
      while (!finished && m < maxit) {
        double sigma = dot64(n, rs, v);
        if (sigma == 0.0 || !isfinite(sigma)) {
          status = OR_BREAKDOWN;
          break;
        }
        double alpha = rho / sigma;
        for (int h = 0; h < 2 && !finished; h++) {
          if (h == 0) {
            for (int64_t i = 0; i < n; i++) y[i] = au[i];
          } else {
            for (int64_t i = 0; i < n; i++) u[i] = u[i] - alpha * v[i];
            for (int64_t i = 0; i < n; i++) uh[i] = dinv[i] * u[i];
            oracle_spmv(n, rowptr, col, val, uh, y);
          }
          for (int64_t i = 0; i < n; i++) w[i] = w[i] - alpha * y[i];
          double coef = theta * theta * eta / alpha;
          for (int64_t i = 0; i < n; i++) d[i] = uh[i] + coef * d[i];
          theta = sqrt(dot64(n, w, w)) / tau;
          double c = 1.0 / sqrt(1.0 + theta * theta);
          tau = tau * theta * c;
          eta = c * c * alpha;
          for (int64_t i = 0; i < n; i++) x[i] = x[i] + eta * d[i];
          m++;
          ml++;
          if (sqrt((double)(ml + 1)) * tau <= rtol * bnorm) {
            passed = 1;
            finished = 1;
          } else if (m >= maxit) {
            finished = 1;
          }
        }
        if (finished) break;
        double rho_new = dot64(n, rs, w);
        if (rho_new == 0.0 || !isfinite(rho_new)) {
          status = OR_BREAKDOWN;
          break;
        }
        double beta = rho_new / rho;
        rho = rho_new;
        /* y holds Ap u of the second half-step */
        for (int64_t i = 0; i < n; i++) u[i] = w[i] + beta * u[i];
        for (int64_t i = 0; i < n; i++) uh[i] = dinv[i] * u[i];
        oracle_spmv(n, rowptr, col, val, uh, au);
        for (int64_t i = 0; i < n; i++) v[i] = au[i] + beta * (y[i] + beta * v[i]);
      }
      if (!passed) break; /* iteration limit or breakdown */
      /* the bound passed: check the true residual of x */
      oracle_spmv(n, rowptr, col, val, x, y);
      for (int64_t i = 0; i < n; i++) r[i] = b[i] - y[i];
      double rn = sqrt(dot64(n, r, r));
      if (rn <= rtol * bnorm) {
        status = OR_OK;
        break;
      }
      if (restarts == TFQMR_MAX_RESTARTS || m >= maxit) {
        status = OR_NOT_CONVERGED;
        break;
      }
      restarts++;
      tau = rn;
    }
  }
  *bound = sqrt((double)(ml + 1)) * tau;
  oracle_spmv(n, rowptr, col, val, x, y);
  for (int64_t i = 0; i < n; i++) r[i] = b[i] - y[i];
  *relres = bnorm > 0.0 ? sqrt(dot64(n, r, r)) / bnorm : sqrt(dot64(n, r, r));
  *iters = m;
  free(r);
  free(rs);
  free(w);
  free(u);
  free(uh);
  free(v);
  free(au);
  free(y);
  free(d);
  free(dinv);
  return status;
}

/* ------------------------------------------------------------------------
 * Mixed-precision iterative refinement (paper Sec. 2, multiprecision plan:
 * device data in a precision other than the solver's).  Outer loop in
 * fp64: r = b - A x in fp64, stop when ||r|| <= rtol_outer ||b||; inner
 * Jacobi-CG on fl32(A) d = fl32(r) from d = 0 with fp32 values, vectors
 * and SpMV, dot products formed and summed in fp64, stopping when
 * ||r_inner|| <= rtol_inner ||fl32(r)||; then x += d in fp64.
 * With early_exit = 1 the inner stop is instead
 * ||r_inner|| <= max(rtol_inner ||fl32(r)||, rtol_outer ||b|| / 2): the
 * second term ends the last refinement step once the outer target is in
 * reach (a reading of the plan, which fixes no inner tolerance).
 * ---------------------------------------------------------------------- */

static void spmv32(int64_t n, const int32_t* rowptr, const int32_t* col, const float* val,
                   const float* x, float* y) {
  PAR_FOR
  for (int64_t r = 0; r < n; r++) {
    float s = 0.0f;
    for (int64_t t = rowptr[r]; t < rowptr[r + 1]; t++) s += val[t] * x[col[t]];
    y[r] = s;
  }
}

int oracle_pcg_mixed(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                     const double* b, double* x, double rtol_outer, double rtol_inner,
                     int64_t maxit_outer, int64_t maxit_inner, int early_exit,
                     int64_t* outer_steps, int64_t* inner_total, double* relres) {
  int64_t nnz = rowptr[n];
  float* val32 = (float*)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
  float* dinv32 = (float*)malloc(sizeof(float) * (size_t)n);
  double* dinv = (double*)malloc(sizeof(double) * (size_t)n);
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* t64 = (double*)malloc(sizeof(double) * (size_t)n);
  float* ri = (float*)malloc(sizeof(float) * (size_t)n);
  float* d = (float*)malloc(sizeof(float) * (size_t)n);
  float* z = (float*)malloc(sizeof(float) * (size_t)n);
  float* p = (float*)malloc(sizeof(float) * (size_t)n);
  float* q = (float*)malloc(sizeof(float) * (size_t)n);
  int64_t outer = 0, inner = 0;
  int status = diag_inverse(n, rowptr, col, val, dinv);
  double bnorm = sqrt(dot64(n, b, b));
  if (status == OR_OK) {
#pragma omp parallel for schedule(static) if (nnz >= PAR_MIN)
    for (int64_t t = 0; t < nnz; t++) val32[t] = (float)val[t];
    PAR_FOR
    for (int64_t i = 0; i < n; i++) dinv32[i] = (float)dinv[i];
    status = OR_NOT_CONVERGED;
    for (;;) {
      oracle_spmv(n, rowptr, col, val, x, t64);
      PAR_FOR
      for (int64_t i = 0; i < n; i++) r[i] = b[i] - t64[i];
      double rn = sqrt(dot64(n, r, r));
      if (rn <= rtol_outer * bnorm) {
        status = OR_OK;
        break;
      }
      if (outer >= maxit_outer) break;
      outer++;
      /* inner fp32 Jacobi-CG from d = 0 */
      PAR_FOR
      for (int64_t i = 0; i < n; i++) ri[i] = (float)r[i];
      PAR_FOR
      for (int64_t i = 0; i < n; i++) d[i] = 0.0f;
      double r0 = sqrt(dot32(n, ri, ri));
      double stop_at = rtol_inner * r0;
      if (early_exit && stop_at < 0.5 * rtol_outer * bnorm) stop_at = 0.5 * rtol_outer * bnorm;
      PAR_FOR
      for (int64_t i = 0; i < n; i++) z[i] = dinv32[i] * ri[i];
      PAR_FOR
      for (int64_t i = 0; i < n; i++) p[i] = z[i];
      double rho = dot32(n, ri, z);
      int64_t it = 0;
      int bad = 0;
      while (it < maxit_inner) {
        spmv32(n, rowptr, col, val32, p, q);
        double pq = dot32(n, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) {
          bad = 1;
          break;
        }
        float a32 = (float)(rho / pq);
        PAR_FOR
        for (int64_t i = 0; i < n; i++) d[i] = d[i] + a32 * p[i];
        PAR_FOR
        for (int64_t i = 0; i < n; i++) ri[i] = ri[i] - a32 * q[i];
        it++;
        double rr = sqrt(dot32(n, ri, ri));
        if (rr <= stop_at) break;
        PAR_FOR
        for (int64_t i = 0; i < n; i++) z[i] = dinv32[i] * ri[i];
        double rho_new = dot32(n, ri, z);
        float b32 = (float)(rho_new / rho);
        PAR_FOR
        for (int64_t i = 0; i < n; i++) p[i] = z[i] + b32 * p[i];
        rho = rho_new;
      }
      inner += it;
      PAR_FOR
      for (int64_t i = 0; i < n; i++) x[i] = x[i] + (double)d[i];
      if (bad) {
        status = OR_BREAKDOWN;
        break;
      }
    }
  }
  oracle_spmv(n, rowptr, col, val, x, t64);
  PAR_FOR
  for (int64_t i = 0; i < n; i++) r[i] = b[i] - t64[i];
  *relres = bnorm > 0.0 ? sqrt(dot64(n, r, r)) / bnorm : sqrt(dot64(n, r, r));
  *outer_steps = outer;
  *inner_total = inner;
  free(val32);
  free(dinv32);
  free(dinv);
  free(r);
  free(t64);
  free(ri);
  free(d);
  free(z);
  free(p);
  free(q);
  return status;
}

/* ------------------------------------------------------------------------
 * Reverse mode through u = A^-1 b with A assembled from COO values v.
 * With adjoint lambda = A^-T (dL/du):  dL/dA_rc = -lambda_r u_c on the
 * stored pattern, and by the chain rule through the assembly sum,
 * dL/dv[k] = -lambda_{i[k]} u_{j[k]} for a kept triplet, 0 otherwise.
 * ---------------------------------------------------------------------- */

void oracle_sddmm(int64_t n, const int32_t* rowptr, const int32_t* col, const double* lam,
                  const double* u, double* G) {
  for (int64_t r = 0; r < n; r++)
    for (int64_t t = rowptr[r]; t < rowptr[r + 1]; t++) G[t] = -lam[r] * u[col[t]];
}

void oracle_coo_grad(int64_t ncoo, const int32_t* i, const int32_t* j, const double* lam,
                     const double* u, double* grad_v) {
  for (int64_t k = 0; k < ncoo; k++) {
    if (i[k] < 0 || j[k] < 0)
      grad_v[k] = 0.0;
    else
      grad_v[k] = -lam[i[k]] * u[j[k]];
  }
}

/* grad_e[e] = sum over the element's block of grad_v[k] * dv[k] */
void oracle_block_reduce(int64_t nblocks, int64_t block, const double* grad_v, const double* dv,
                         double* grad_e) {
  for (int64_t e = 0; e < nblocks; e++) {
    double s = 0.0;
    for (int64_t k = e * block; k < (e + 1) * block; k++) s += grad_v[k] * dv[k];
    grad_e[e] = s;
  }
}

/* ------------------------------------------------------------------------
 * Limited-memory BFGS, product p = H_k g (paper Sec. 8, dense
 * reformulations).  S = [s_0 .. s_{m-1}], Y = [y_0 .. y_{m-1}] hold the
 * m most recent pairs, oldest first, column-major (column j at j*n); the
 * base operator is the diagonal h0 (it may change from call to call).
 *
 * oracle_lbfgs_recursive: the two-loop recursion.
 *   q = g;  for j = m-1 .. 0:  alpha_j = s_j.q / d_j;  q -= alpha_j y_j
 *   p = h0 q;  for j = 0 .. m-1:  beta_j = y_j.p / d_j;  p += (alpha_j - beta_j) s_j
 * with d_j = s_j.y_j.  (The paper's printed listing adds a multiple of y_j
 * in the second loop; only s_j yields H_k g, which its dense formula below
 * states, so s_j is taken.)
 *
 * oracle_lbfgs_dense: the paper's intermediate dense formula
 *   H_k g = [I, -S R^-T] [I 0; Y^T I] diag(H0, D) [I Y; 0 I] [I; -R^-1 S^T] g
 * with R = triu(S^T Y), D = diag(S^T Y), evaluated right to left:
 *   c = -R^-1 (S^T g);  a = h0 (g + Y c);  f = Y^T a + D c;
 *   e = R^-T f;  p = a - S e.
 * Dot products are plain in-order sums.
 * ---------------------------------------------------------------------- */
static double dot_plain(int64_t n, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

void oracle_lbfgs_recursive(int64_t n, int64_t m, const double* S, const double* Y,
                            const double* g, const double* h0, double* p) {
  double* q = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double* alpha = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  for (int64_t i = 0; i < n; i++) q[i] = g[i];
  for (int64_t j = m - 1; j >= 0; j--) {
    const double* s = S + j * n;
    const double* y = Y + j * n;
    alpha[j] = dot_plain(n, s, q) / dot_plain(n, s, y);
    for (int64_t i = 0; i < n; i++) q[i] = q[i] - alpha[j] * y[i];
  }
  for (int64_t i = 0; i < n; i++) p[i] = h0[i] * q[i];
  for (int64_t j = 0; j < m; j++) {
    const double* s = S + j * n;
    const double* y = Y + j * n;
    double beta = dot_plain(n, y, p) / dot_plain(n, s, y);
    for (int64_t i = 0; i < n; i++) p[i] = p[i] + (alpha[j] - beta) * s[i];
  }
  free(q);
  free(alpha);
}

void oracle_lbfgs_dense(int64_t n, int64_t m, const double* S, const double* Y,
                        const double* g, const double* h0, double* p) {
  const size_t mm = (size_t)(m > 0 ? m : 1);
  double* M = (double*)malloc(sizeof(double) * mm * mm); /* M[a*m+b] = s_a.y_b */
  double* c = (double*)malloc(sizeof(double) * mm);
  double* f = (double*)malloc(sizeof(double) * mm);
  double* e = (double*)malloc(sizeof(double) * mm);
  double* a = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int64_t x = 0; x < m; x++)
    for (int64_t y = 0; y < m; y++) M[x * m + y] = dot_plain(n, S + x * n, Y + y * n);
  /* c = -R^-1 (S^T g): back substitution, R upper triangular */
  for (int64_t x = m - 1; x >= 0; x--) {
    double t = -dot_plain(n, S + x * n, g);
    for (int64_t y = x + 1; y < m; y++) t -= M[x * m + y] * c[y];
    c[x] = t / M[x * m + x];
  }
  /* a = h0 (g + Y c) */
  for (int64_t i = 0; i < n; i++) {
    double t = g[i];
    for (int64_t y = 0; y < m; y++) t += Y[y * n + i] * c[y];
    a[i] = h0[i] * t;
  }
  /* f = Y^T a + D c;  e = R^-T f: forward substitution, R^T lower */
  for (int64_t x = 0; x < m; x++) f[x] = dot_plain(n, Y + x * n, a) + M[x * m + x] * c[x];
  for (int64_t x = 0; x < m; x++) {
    double t = f[x];
    for (int64_t y = 0; y < x; y++) t -= M[y * m + x] * e[y];
    e[x] = t / M[x * m + x];
  }
  /* p = a - S e */
  for (int64_t i = 0; i < n; i++) {
    double t = a[i];
    for (int64_t x = 0; x < m; x++) t -= S[x * n + i] * e[x];
    p[i] = t;
  }
  free(M);
  free(c);
  free(f);
  free(e);
  free(a);
}
