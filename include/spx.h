/*
 * spx — sparse COO assembly, CSR products and Jacobi-preconditioned CG for
 * AMD Instinct MI355X (gfx950).  C ABI.
 *
 * Conventions for every entry point
 *   - Return value: SPX_OK (0) on success, a negative status otherwise.  No
 *     C++ exception crosses this boundary.  spx_last_error() returns a
 *     human-readable message for the last failure on the calling thread.
 *   - Array arguments are DEVICE pointers (memory of the GPU that was current
 *     when the handle was created), contiguous, owned by the caller, unless
 *     stated otherwise.  Scalar outputs (iters_out, relres_out, ...) are
 *     HOST pointers and may be NULL when not wanted.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued on it in order; inputs must stay valid until the
 *     stream has passed the call.  Calls marked "asynchronous" return before
 *     the GPU has finished; the others synchronise `stream` as documented.
 *   - Indices are int32, values float64 unless the name says otherwise.
 *   - Handles are not thread-safe: one handle must not be used from two
 *     threads or on two streams concurrently.
 */
#ifndef SPX_H
#define SPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spx_matrix* spx_handle;
typedef struct spx_batch* spx_batch_handle;
typedef struct spx_vec_coo* spx_vec_handle;
typedef struct spx_lbfgs* spx_lbfgs_handle;
typedef struct spx_split* spx_split_handle;

enum spx_status {
  SPX_OK = 0,
  SPX_INVALID_ARG = -1,        /* null pointer, n <= 0, ncoo < 0, bad mode ... */
  SPX_INDEX_OUT_OF_RANGE = -2, /* a COO index >= n (found on the device)      */
  SPX_HIP_ERROR = -3,          /* a HIP runtime call failed                   */
  SPX_ZERO_DIAGONAL = -4,      /* Jacobi preconditioner met a zero/absent a_ii */
  SPX_NOT_CONVERGED = -5,      /* iteration limit reached; x holds the last iterate */
  SPX_BREAKDOWN = -6,          /* p.Ap <= 0 or not finite (matrix not SPD)     */
  SPX_NOT_IMPLEMENTED = -7,
  SPX_OUT_OF_MEMORY = -8
};

enum spx_insert_mode { SPX_INSERT_VALUES = 0, SPX_ADD_VALUES = 1 };

/* ---------------------------------------------------------------------------
 * COO assembly — paper Sec. 5 ("Portable matrix assembly on GPUs"): the
 * matrix is the sum of the contributions v[k] to entry (i[k], j[k]); a split
 * into a symbolic stage (pattern and helper maps, once) and numeric stages
 * (values, many times); negative indices mark ignored triplets.
 * ------------------------------------------------------------------------- */

/* Symbolic stage, on the device.  Drops triplets with i[k] < 0 or j[k] < 0,
 * sorts the rest stably by (row, column), and builds the CSR pattern (rows
 * ascending, columns ascending in a row, an entry for every distinct kept
 * (i, j) even if its values later cancel) plus the helper maps that let
 * spx_set_values_coo sum duplicates without atomics:
 *   perm[q]  = original triplet index k, q < nvalid, ordered by (i, j, k);
 *   jmap[t]  = first q feeding stored entry t; jmap[nnz] = nvalid.
 * n: matrix order (1 <= n < 2^31).  ncoo: triplet count (0 <= ncoo < 2^31).
 * i, j: device int32[ncoo]; they are not referenced after the call returns
 * and may be freed (paper Sec. 5 allows this).  On success *out receives a
 * new handle owning all pattern, value and workspace memory.  Errors:
 * SPX_INVALID_ARG, SPX_INDEX_OUT_OF_RANGE (some kept index >= n),
 * SPX_OUT_OF_MEMORY, SPX_HIP_ERROR; *out is then NULL.
 * Synchronises `stream` (the host must learn nnz to size the pattern). */
int spx_coo_preallocate(int64_t n, int64_t ncoo, const int32_t* i, const int32_t* j, void* stream,
                        spx_handle* out);

/* Numeric stage.  v: device float64[ncoo] in the same order as i/j.  For
 * every stored entry t, s = +0.0 + v[perm[jmap[t]]] + ... in increasing k
 * (one thread per entry, no atomics, bitwise reproducible); mode
 * SPX_INSERT_VALUES stores s, SPX_ADD_VALUES adds s to the current value.
 * v[k] of ignored triplets is never read.  Asynchronous. */
int spx_set_values_coo(spx_handle h, const double* v, int mode, void* stream);

/* Releases everything the handle owns (synchronises the device). NULL ok. */
int spx_destroy(spx_handle h);

/* COO vector assembly — paper Sec. 5 (VecSetPreallocationCOO(x, n, i) and
 * VecSetValuesCOO(x, v, mode), the vector counterpart of the two stages
 * above).  The pattern is the set of distinct kept indices (negative i[k]
 * ignored, i[k] >= n is SPX_INDEX_OUT_OF_RANGE); i: device int32[ncoo], not
 * referenced after the call.  Synchronises `stream`. */
int spx_vec_coo_preallocate(int64_t n, int64_t ncoo, const int32_t* i, void* stream,
                            spx_vec_handle* out);

/* For every index i of the pattern, s = +0.0 + v[k] + ... over the kept k
 * with i[k] = i in increasing k; SPX_INSERT_VALUES stores x[i] = s,
 * SPX_ADD_VALUES stores x[i] = x[i] + s.  Entries of x outside the pattern
 * are left unchanged.  v: device float64[ncoo]; x: device float64[n].
 * Asynchronous. */
int spx_vec_set_values_coo(spx_vec_handle h, const double* v, int mode, double* x, void* stream);

/* HOST outputs: length, distinct indices, kept triplets, triplets. */
int spx_vec_coo_get_info(spx_vec_handle h, int64_t* n, int64_t* nunique, int64_t* nvalid,
                         int64_t* ncoo);
int spx_vec_coo_destroy(spx_vec_handle h);

/* ---------------------------------------------------------------------------
 * One rank's rows as a diagonal and an off-diagonal block — paper Sec. 5
 * (parallel matrices are distributed by rows, each process storing its
 * diagonal block, intra-process coupling, and its off-diagonal block,
 * inter-process coupling, as two sequential CSR matrices; the numeric stage
 * fills both from the one v[]).  The single-GPU half of that assembly: the
 * rank owns rows and columns [row_lo, row_hi) of an n_global x n_global
 * matrix.  A kept triplet with row in the range goes to the diagonal block
 * when its column is in the range too, else to the off-diagonal block; one
 * with its row outside the range belongs to another rank (PETSc sends it;
 * here it is only counted, as nremote, and not assembled).  Negative
 * indices are ignored; an index >= n_global is SPX_INDEX_OUT_OF_RANGE.
 *   diagonal block: (row_hi - row_lo) square, local row and column numbers;
 *   off-diagonal block: compressed both ways.  Its rows are the local rows
 *     with at least one off-diagonal entry (orows[], ascending local row
 *     numbers) and its columns the distinct off-diagonal global columns
 *     (garray[], ascending: the ghost entries of x).  It is stored as a
 *     square spx matrix of order max(nrows_offdiag, nghost, 1) whose rows
 *     from nrows_offdiag on are empty.
 * Each block is assembled exactly as spx_coo_preallocate would assemble the
 * stream with every triplet of the other block and of other ranks given
 * index -1, so its values are bitwise those sums and its jmap/perm index
 * the caller's v directly.  i, j: device int32[ncoo], not referenced after
 * the call.  Synchronises `stream`. */
int spx_split_preallocate(int64_t n_global, int64_t row_lo, int64_t row_hi, int64_t ncoo,
                          const int32_t* i, const int32_t* j, void* stream,
                          spx_split_handle* out);
/* Numeric stage of both blocks from v (device float64[ncoo], the order of
 * i/j), INSERT or ADD as spx_set_values_coo.  Asynchronous. */
int spx_split_set_values_coo(spx_split_handle h, const double* v, int mode, void* stream);
/* y = A_d x_local + A_o x_ghost: the diagonal block's product (as
 * spx_matmult), then each off-diagonal row's products added in column order
 * from +0.0 and that sum added to y at its local row.  x_local, y: device
 * float64[row_hi - row_lo]; x_ghost: device float64[nghost], x_ghost[c] the
 * value of global entry garray[c].  Asynchronous. */
int spx_split_matmult(spx_split_handle h, const double* x_local, const double* x_ghost, double* y,
                      void* stream);
/* x_ghost[c] = x_global[garray[c]]: on one GPU this stands in for the halo
 * exchange that brings the ghost entries from their owners.  x_global:
 * device float64[n_global].  Asynchronous. */
int spx_split_gather_ghosts(spx_split_handle h, const double* x_global, double* x_ghost,
                            void* stream);
/* HOST outputs: local rows, ghost columns, off-diagonal rows, triplets of
 * other ranks' rows. */
int spx_split_get_info(spx_split_handle h, int64_t* rows, int64_t* nghost, int64_t* nrows_offdiag,
                       int64_t* nremote);
/* The two blocks as borrowed matrix handles (owned by h: valid until
 * spx_split_destroy, never passed to spx_destroy), for products, solves and
 * introspection of one block. */
int spx_split_blocks(spx_split_handle h, spx_handle* diag, spx_handle* offdiag);
/* Copies garray (device int32[nghost]) and orows (device int32[nrows_offdiag]);
 * either may be NULL.  Asynchronous. */
int spx_split_get_maps(spx_split_handle h, int32_t* garray, int32_t* orows, void* stream);
int spx_split_destroy(spx_split_handle h);

/* ---------------------------------------------------------------------------
 * Products — paper Sec. 6 (MatMult inside CG).
 * ------------------------------------------------------------------------- */

/* y = A x.  x, y: device float64[n], must not overlap.  Asynchronous. */
int spx_matmult(spx_handle h, const double* x, double* y, void* stream);

/* y = A^T x through an explicit transpose (built on first use, refreshed
 * after each spx_set_values_coo; its entries are bitwise those of A).
 * Asynchronous (the first call allocates). */
int spx_matmult_transpose(spx_handle h, const double* x, double* y, void* stream);

/* Y = A X for nrhs right-hand sides stored row-major: X[c*ldx + s],
 * Y[r*ldy + s], s < nrhs (ldx, ldy >= nrhs).  Asynchronous. */
int spx_spmm(spx_handle h, int64_t nrhs, const double* X, int64_t ldx, double* Y, int64_t ldy,
             void* stream);

/* Bandwidth references for reporting the kernels against what this device
 * sustains (beside the nominal peak): y = x, and partial sums of x.  The
 * whole grid (2048 workgroups) sweeps the array in lockstep with one
 * 16-byte non-temporal access per lane.  x, y: device float64[n], 16-byte
 * aligned; partials: device float64[2048] (workgroup b's sum in
 * partials[b]).  Asynchronous. */
int spx_stream_copy(const double* x, double* y, int64_t n, void* stream);
int spx_stream_sum(const double* x, int64_t n, double* partials, void* stream);

/* ---------------------------------------------------------------------------
 * Jacobi-preconditioned CG — paper Sec. 6 (CG / CGAsync): scalars stay in
 * device memory, the host only enqueues kernels and polls a device
 * convergence flag every `check_every` iterations.
 *   r = b - A x; z = D^-1 r; p = z; rho = r.z
 *   repeat: q = A p; alpha = rho / p.q; x += alpha p; r -= alpha q;
 *           stop when ||r||_2 <= rtol ||b||_2;
 *           z = D^-1 r; beta = r.z / rho; p = z + beta p
 * The stopping test uses the recursively updated residual every iteration,
 * so the iteration count is exact whatever check_every is.
 * b: device float64[n]; x: device float64[n], initial guess in, solution out.
 * maxit >= 0; check_every >= 1.  iters_out: iterations done; relres_out:
 * true ||b - A x|| / ||b|| recomputed at exit (||b - A x|| when b = 0).
 * Errors: SPX_ZERO_DIAGONAL, SPX_BREAKDOWN, SPX_NOT_CONVERGED (x valid).
 * Synchronises `stream` at every poll and at exit. */
int spx_cg_solve(spx_handle h, const double* b, double* x, double rtol, int64_t maxit,
                 int32_t check_every, void* stream, int64_t* iters_out, double* relres_out);

/* ---------------------------------------------------------------------------
 * CG without allocation — for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same kernels, arguments, results and errors as spx_cg_solve
 * (bitwise the same x and iteration count), but the solver workspace (the
 * vectors r, p, q, u, the inverse diagonal, the workgroup partials and the
 * device scalars) lives in one static device array of the library, about
 * 80 MiB, which every GPU that runs the library holds until the process
 * ends; the host polls with plain stream synchronisations instead of events
 * and no HIP graph is captured (SPX_OPT_GRAPH and SPX_OPT_PROFILE have no
 * effect).  The call allocates nothing, provided the handle itself is
 * complete: its matrix, values and window index exist once
 * spx_set_values_coo has run.
 * Limits: n <= SPX_NOALLOC_MAX_ROWS, and at most 4096 workgroups per solver
 * kernel (the automatic launch shape uses at most 2048); beyond either the
 * call returns SPX_INVALID_ARG and launches nothing.  The current device
 * must be the handle's.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other host threads, or other streams before the first call returns)
 * race and give wrong results.  The array keeps the last call's contents;
 * each call initialises everything it reads. */
#define SPX_NOALLOC_MAX_ROWS 2097152
int spx_cg_solve_noalloc(spx_handle h, const double* b, double* x, double rtol, int64_t maxit,
                         int32_t check_every, void* stream, int64_t* iters_out,
                         double* relres_out);

/* The same solver applied to A^T (adjoint solves). */
int spx_cg_solve_transpose(spx_handle h, const double* b, double* x, double rtol, int64_t maxit,
                           int32_t check_every, void* stream, int64_t* iters_out,
                           double* relres_out);

/* ---------------------------------------------------------------------------
 * Mixed precision — paper Sec. 2 (multiprecision plan: device data in a
 * lower precision than the solver's).  Iterative refinement: outer fp64
 * residual r = b - A x and norm; inner Jacobi-CG on fl32(A) d = fl32(r) from
 * d = 0 with fp32 matrix, vectors and SpMV but fp64 dot products, stopping
 * at ||r_in|| <= rtol_inner ||fl32(r)|| (with SPX_OPT_IR_EARLY_EXIT at
 * ||r_in|| <= max(rtol_inner ||fl32(r)||, rtol_outer ||b|| / 2), which ends
 * the last step once the outer target is in reach); x += d in fp64; stop
 * when ||b - A x|| <= rtol_outer ||b||.
 * x: device float64[n], in/out (usually 0).
 * outer_out: refinement steps; inner_out: total inner iterations.
 * Synchronises `stream`. */
int spx_cg_solve_mixed(spx_handle h, const double* b, double* x, double rtol_outer,
                       double rtol_inner, int64_t maxit_outer, int64_t maxit_inner,
                       int32_t check_every, void* stream, int64_t* outer_out, int64_t* inner_out,
                       double* relres_out);

/* ---------------------------------------------------------------------------
 * Batched solves — paper Sec. 7: many independent small systems solved by one
 * batched Jacobi-preconditioned Krylov solver instead of one stacked
 * ("ensemble") system.
 * ------------------------------------------------------------------------- */

/* Groups nsys assembled handles (each with values set) into one batch.  The
 * batch references the handles' matrices (they must outlive it) and owns
 * the per-system descriptors and workspace.  Right-hand sides and solutions
 * are packed back to back: system s occupies [off_s, off_s + n_s) with
 * off_s = n_0 + ... + n_{s-1}.  Synchronises `stream`. */
int spx_batch_create(int32_t nsys, const spx_handle* hs, void* stream, spx_batch_handle* out);
int spx_batch_destroy(spx_batch_handle b);
int spx_batch_total_rows(spx_batch_handle b, int64_t* total);

/* Launch shape of the batched solvers (all fields may be 0 for automatic).
 *   blocks: workgroups shared by the systems (0: 8 per compute unit;
 *     raised to nsys if smaller).
 *   rows_per_tile: 0 lets the library choose the row walk: the window walk
 *     (256-row tiles reading x from LDS, see SPX_OPT_SPMV_VARIANT) when
 *     every system (for BiCG also every transpose) has a window index, else
 *     the stream walk with the largest tile that fits; 32, 64, 128 or 256
 *     ask for the stream walk with that many rows per workgroup tile.
 *   weight_exponent: a running system's share of the workgroups is
 *     proportional to nnz_s^weight_exponent, at least one (<= 0 means 1).
 *   check_every: iterations between host polls, at which the workgroups are
 *     re-split among the systems still running (0 means 20).
 *   persistent: 1 asks for ONE launch for the whole solve, in which each
 *     workgroup (256 threads, 1024 when a system exceeds 1024 rows) takes
 *     the next system from a queue, largest first, and runs the whole
 *     method on it alone (the fields above are then unused, and a system's
 *     largest 256-row tile, for BiCG also its transpose's, must fit 64 KB of
 *     LDS, else SPX_INVALID_ARG);
 *     -1 asks for the launch-per-phase solve above; 0 lets the library
 *     choose (persistent for at least 256 systems of at most 8192 rows
 *     each). */
typedef struct spx_batch_tuning {
  int32_t blocks;
  int32_t rows_per_tile;
  double weight_exponent;
  int32_t check_every;
  int32_t persistent;
} spx_batch_tuning;

/* Solves every system of the batch with Jacobi-CG to its own
 * ||r_s|| <= rtol ||b_s|| (the single-system algorithm above, system by
 * system).  Two launch forms (tuning->persistent): either all systems
 * advance together and each CG phase is one launch for the whole batch
 * (the workgroups form one team per running system; converged systems drop
 * out and their workgroups go to the others at the next poll), or ONE
 * launch solves the batch with each workgroup taking whole systems from a
 * queue, largest first (no host poll).  The dots are summed in different
 * orders, so the two forms' iterates agree to rounding, not bitwise.
 * b, x: packed device float64[total]; x is the initial guess
 * and receives the solutions.  tuning: may be NULL.  iters_out /
 * relres_out: HOST int64[nsys] / float64[nsys]: iterations and true
 * ||b_s - A_s x_s|| / ||b_s||.  Returns SPX_NOT_CONVERGED if a system hit
 * maxit, SPX_BREAKDOWN / SPX_ZERO_DIAGONAL if a system failed (the others
 * are still solved).  Synchronises `stream`. */
int spx_batch_cg(spx_batch_handle b, const double* bvec, double* x, double rtol, int64_t maxit,
                 const spx_batch_tuning* tuning, void* stream, int64_t* iters_out,
                 double* relres_out);

/* Batched Jacobi-preconditioned BiCG (paper Sec. 7, the batched BiCG with
 * diagonal preconditioning) for non-symmetric systems, with the arguments,
 * outputs, stopping test and statuses of spx_batch_cg.  Per system:
 *   r = b - A x; rh = r; z = D^-1 r; p = z; ph = D^-1 rh; rho = z.rh
 *   repeat: q = A p; qh = A^T ph; sigma = ph.q; alpha = rho / sigma;
 *           x += alpha p; r -= alpha q; rh -= alpha qh;
 *           stop when ||r|| <= rtol ||b||;
 *           rho' = (D^-1 r).rh; beta = rho' / rho;
 *           p = D^-1 r + beta p; ph = D^-1 rh + beta ph
 * sigma or rho' equal to 0 or not finite is SPX_BREAKDOWN.  The first call
 * builds each matrix's explicit transpose (kept by the handle).  On a
 * symmetric system the iterates are those of spx_batch_cg, bit for bit.
 * Synchronises `stream`. */
int spx_batch_bicg(spx_batch_handle b, const double* bvec, double* x, double rtol, int64_t maxit,
                   const spx_batch_tuning* tuning, void* stream, int64_t* iters_out,
                   double* relres_out);

/* Batched TFQMR (paper Secs. 6 and 7: Freund's transpose-free QMR with
 * diagonal preconditioning) for non-symmetric systems, preconditioned from
 * the right so that its residual is the true one.  Per system, with
 * Ap = A D^-1, rs = r0 = b - A x, half-steps m = 1, 2, ...:
 *   w = u = r0; au = Ap u; v = au; d = 0; tau = ||r0||; theta = eta = 0;
 *   rho = rs.r0;  per iteration: alpha = rho / rs.v, then two half-steps
 *   (y = au, then u -= alpha v and y = Ap u):
 *     w -= alpha y; d = D^-1 u + (theta^2 eta / alpha) d;
 *     theta = ||w|| / tau; c = (1 + theta^2)^-1/2; tau = tau theta c;
 *     eta = c^2 alpha; x += eta d; stop when sqrt(m + 1) tau <= rtol ||b||
 *   then rho' = rs.w, beta = rho' / rho, u = w + beta u, au = Ap u,
 *   v = au + beta (y + beta v).
 * sqrt(m + 1) tau bounds ||b - A x||, so the test certifies the true
 * residual (up to rounding).  maxit and iters_out count half-steps (one
 * product with A each); check_every counts iterations of two half-steps.
 * rs.v or rho' equal to 0 or not finite is SPX_BREAKDOWN.  Arguments,
 * outputs and statuses otherwise as spx_batch_cg.  Synchronises `stream`. */
int spx_batch_tfqmr(spx_batch_handle b, const double* bvec, double* x, double rtol, int64_t maxit,
                    const spx_batch_tuning* tuning, void* stream, int64_t* iters_out,
                    double* relres_out);

/* ---------------------------------------------------------------------------
 * Limited-memory BFGS — paper Sec. 8 (dense reformulations of algorithms):
 * the product p = H_k g with the inverse-Hessian approximation built from
 * the m most recent pairs (s_j, y_j), in the intermediate dense form
 *   H_k g = [I, -S R^-T] [I 0; Y^T I] diag(H0, D) [I Y; 0 I] [I; -R^-1 S^T] g
 * with S = [s_oldest .. s_newest], Y likewise, R = triu(S^T Y),
 * D = diag(S^T Y) and a diagonal base operator H0 = diag(h0) that may change
 * from call to call (variable metric).  This equals the two-loop recursion
 * and the m successive BFGS updates of H0.
 * ------------------------------------------------------------------------- */

/* History of m pairs (1 <= m <= 64) of vectors of length n.  The handle owns
 * S and Y (n x m each, column-major), the m x m products s_a.y_b and the
 * workspace (about 2 n m + n doubles of device memory). */
int spx_lbfgs_create(int64_t n, int32_t m, void* stream, spx_lbfgs_handle* out);
int spx_lbfgs_destroy(spx_lbfgs_handle h);
/* Forgets every pair (the next apply returns h0 g). */
int spx_lbfgs_reset(spx_lbfgs_handle h);
/* HOST outputs: length, history size, pairs held. */
int spx_lbfgs_get_info(spx_lbfgs_handle h, int64_t* n, int32_t* m, int32_t* count);

/* Appends the pair (s, y), dropping the oldest when m are held, and updates
 * the products s_a.y_b of the new row and column (one pass over S and Y).
 * s, y: device float64[n], copied.  The caller keeps to the curvature
 * condition s.y > 0 (not checked; a non-positive s_j.y_j makes later
 * products meaningless).  Asynchronous. */
int spx_lbfgs_update(spx_lbfgs_handle h, const double* s, const double* y, void* stream);

/* p = H_k g.  g: device float64[n]; h0: device float64[n] (the diagonal of
 * H0) or NULL for H0 = I; p: device float64[n], must not alias g.  Three
 * passes over the rows (S^T g; a = h0 (g + Y c) with Y^T a; p = a - S e)
 * with the two m x m triangular solves between them.  Asynchronous. */
int spx_lbfgs_apply(spx_lbfgs_handle h, const double* g, const double* h0, double* p,
                    void* stream);

/* spx_lbfgs_update(s, y) followed by spx_lbfgs_apply(g, h0, p), the step of
 * an optimiser that takes its next direction right after storing the pair,
 * with S^T g taken in the update's pass over S: one pass over S fewer (of
 * three) for the same result, bit for bit.  When g, h0 and p would make
 * the apply walk rows one at a time while the update walks them two at a
 * time (even n, a pointer off a 16-byte boundary), the two run unfused.
 * Same arguments, ownership and errors as the two calls.  Asynchronous. */
int spx_lbfgs_update_apply(spx_lbfgs_handle h, const double* s, const double* y,
                           const double* g, const double* h0, double* p, void* stream);

/* ---------------------------------------------------------------------------
 * Differentiation of u = A(v)^-1 b through the COO assembly (reverse mode).
 * ------------------------------------------------------------------------- */

/* G[t] = -lam[row t] * u[col t] for every stored entry t (the gradient of a
 * loss with respect to the assembled entries, given the adjoint lam).
 * lam, u: device float64[n]; G: device float64[nnz].  Asynchronous. */
int spx_sddmm(spx_handle h, const double* lam, const double* u, double* G, void* stream);

/* Backward of the COO assembly: grad_v[k] = G[t(k)] where t(k) is the
 * stored entry that triplet k feeds, 0.0 for ignored triplets.
 * G: device float64[nnz]; grad_v: device float64[ncoo].  Asynchronous (the
 * first call builds the triplet -> entry map). */
int spx_coo_gather(spx_handle h, const double* G, double* grad_v, void* stream);

/* Fused backward for element-contiguous COO streams (paper Sec. 5,
 * finite-element usage: each element's triplets are stored contiguously at
 * offset e*block): grad_e[e] = sum_{k in [e*block, (e+1)*block)}
 * G[t(k)] * w[k] (ignored triplets contribute 0), summed in increasing k.
 * w: device float64[ncoo] (dv[k]/dtheta_e); grad_e: device
 * float64[ncoo/block]; ncoo must be a multiple of block.  Asynchronous. */
int spx_coo_gather_blocks(spx_handle h, const double* G, const double* w, int64_t block,
                          double* grad_e, void* stream);

/* ---------------------------------------------------------------------------
 * Introspection (tests and tools).
 * ------------------------------------------------------------------------- */

/* HOST outputs: order, stored entries, kept triplets, triplets. */
int spx_get_info(spx_handle h, int64_t* n, int64_t* nnz, int64_t* nvalid, int64_t* ncoo);

/* Copies the CSR arrays of A (transpose = 0) or of the explicit A^T (1)
 * into caller DEVICE buffers rowptr[n+1], col[nnz], val[nnz]; any may be
 * NULL.  Asynchronous. */
int spx_get_csr(spx_handle h, int32_t transpose, int32_t* rowptr, int32_t* col, double* val,
                void* stream);

/* Window index of A (transpose = 0) or of the explicit A^T (1, built on
 * first use), which the window walk of the products reads.  HOST stats[4] =
 * {1 if the pattern has an index else 0, largest window in blocks of 64
 * x entries, total blocks over all tiles, entries of tiles that read x
 * directly}.  When it exists, non-NULL DEVICE buffers receive
 * ptr[ceil(n/256) + 1] (tile k's blocks are blk[ptr[k] .. ptr[k+1])),
 * blk[stats[2]] (ascending block numbers) and lcol[nnz] (entry t's window
 * position: slot of its block * 64 + col % 64; unset in tiles without a
 * window).  The copies are asynchronous on `stream`. */
int spx_get_window(spx_handle h, int32_t transpose, int64_t* stats, int32_t* ptr, int32_t* blk,
                   uint16_t* lcol, void* stream);

/* Copies the helper maps into caller DEVICE buffers jmap[nnz+1],
 * perm[nvalid] (either may be NULL).  Asynchronous. */
int spx_get_coo_maps(spx_handle h, int32_t* jmap, int32_t* perm, void* stream);

/* Device-memory hook: every device allocation the library makes (patterns,
 * values, maps, transposes, solver and batch workspaces) calls
 * alloc(bytes, ctx), which returns device memory of at least `bytes` bytes
 * (any alignment of 256 bytes or more) or NULL on failure; the block is later
 * returned with free(ptr, ctx) of the hook that made it, so the hook may be
 * changed at any time.  Both NULL restores hipMalloc/hipFree (the default).
 * Process-wide.  Lets a caller route the library's memory through its own
 * pool (the Python layer offers PyTorch's caching allocator). */
typedef void* (*spx_alloc_fn)(size_t bytes, void* ctx);
typedef void (*spx_free_fn)(void* ptr, void* ctx);
int spx_set_allocator(spx_alloc_fn alloc, spx_free_fn free, void* ctx);

/* Tuning knobs (per handle; defaults chosen from the pattern).
 *   SPX_OPT_SPMV_LANES: lanes per row of the "vector" row walk (0 = auto,
 *     else a power of two <= 64).
 *   SPX_OPT_XCD_REMAP: 1 gives each of the 8 XCDs a contiguous range of
 *     rows, 0 keeps plain workgroup order, -1 (default) picks per walk:
 *     plain order for the window walk (its x entries are staged from
 *     LDS windows) and the XCD order for the gather walks (the x entries
 *     a region gathers then stay in one XCD's L2).  Reading the option
 *     returns the order the product with A uses.
 *   SPX_OPT_PROFILE: 1 brackets every solver-iteration kernel with HIP
 *     events on the solver's stream and accumulates their durations (read
 *     with spx_get_profile).
 *   SPX_OPT_SPMV_VARIANT: 0 auto, 1 vector (L lanes per row), 2 stream
 *     (rows of a workgroup streamed through LDS), 3 DMA (the stream walk
 *     with columns and values moved into LDS by direct 16-byte loads, two
 *     staging buffers in the solver kernels), 4 window (tiles of 256 rows
 *     read the x entries they need from LDS, staged once per tile, and
 *     16-bit window columns instead of the 32-bit ones; results bitwise
 *     those of the stream walk; only for patterns with a window index, see
 *     spx_get_window, else as 0).  Auto takes the window walk when the
 *     pattern has an index and enough 256-row tiles per compute unit
 *     (smaller systems fill the chip better with the stream walk's smaller
 *     tiles): for MatMult and MatMultTranspose 2.5, for the solvers 12 (7
 *     when rows average at most 16 entries); and when rows average at most
 *     64 entries in every tile and
 *     none of SPX_OPT_ROWS_PER_BLOCK, SPX_OPT_QUAD_LOADS, SPX_OPT_PIPELINE
 *     is set.  Reading the option returns the variant MatMult resolves to.
 *   SPX_OPT_ROWS_PER_BLOCK: stream variant rows per workgroup (0 auto, else
 *     32, 64, 128 or 256).
 *   SPX_OPT_NONTEMPORAL: 1 (default) loads matrix values/columns
 *     non-temporally, 0 with the default cache policy.
 *   SPX_OPT_SOLVER_BLOCKS: workgroups of the solver's SpMV kernels (0 auto).
 *   SPX_OPT_QUAD_LOADS: 1 streams values/columns with 16-byte loads in the
 *     stream variant, 0 (default) with element loads.
 *   SPX_OPT_VECTOR_BLOCKS: workgroups of the solver's vector kernels (0
 *     auto).
 *   SPX_OPT_PIPELINE: 1 lets the solver's SpMV kernels load the next tile
 *     while reducing the current one (stream variant; default 0, measured
 *     slower on gfx950); reading it returns the register depth in use.
 *   SPX_OPT_ROWS_PER_BLOCK_F32: rows per workgroup of the fp32 copy used by
 *     the mixed-precision inner solve (0 auto: twice the fp64 tile).
 *   SPX_OPT_CG_VARIANT: form of the fp64 CG recurrences used by
 *     spx_cg_solve and spx_cg_solve_transpose.  -1 (default): form 1 for
 *     matrices of at most 2,000,000 entries (where its saved launch and
 *     reduction point per iteration pay) unless SPX_OPT_GRAPH is on, form 0
 *     otherwise; systems small enough for the one-workgroup solve still
 *     take it; reading the option returns the form a solve with A takes.
 *     0: the textbook (Hestenes-Stiefel) form, three kernels and two
 *     reduction points per iteration.  1: the Chronopoulos-Gear single-reduction form of the same
 *     method (Sec. 6 names fewer synchronisation points as the aim of the
 *     asynchronous CG): with u = D^-1 r, w = A u, s = A p kept as a vector,
 *       gamma = r.u, delta = w.u, beta = gamma_k / gamma_{k-1},
 *       alpha_k = gamma_k / (delta_k - beta_k gamma_k / alpha_{k-1}),
 *     two kernels and ONE reduction point per iteration; its iterates equal
 *     those of form 0 in exact arithmetic and differ by rounding.
 *     2: the pipelined form of Ghysels and Vanroose (preconditioned, M = D):
 *     the dots of an iteration are reduced by the next update kernel, so
 *     the product nv = A m in between never waits for a reduction (the
 *     overlap that hides an all-reduce across GPUs); two kernels per
 *     iteration, nine work vectors, about 20 vector reads and writes per
 *     row per iteration against 11 for form 0.  Same iterates in exact
 *     arithmetic.  Never chosen automatically; spx_cg_solve_noalloc refuses
 *     it (its scratch holds four vectors).
 *   SPX_OPT_GRAPH: 1 replays each full poll chunk of the textbook CG
 *     (spx_cg_solve, spx_cg_solve_transpose and the fp32 inner solve of
 *     spx_cg_solve_mixed) as one HIP graph, captured once on a private
 *     stream and kept while the operator, vectors and launch shape stay the
 *     same; the kernels then take the iteration number from the device.
 *     Same arithmetic as 0 (bitwise equal results); it only saves launch
 *     overhead, which matters for small systems.  Ignored while
 *     SPX_OPT_PROFILE is on and for the single-reduction form.  Default 0.
 *   SPX_OPT_SMALL_SOLVE: the fp64 textbook CG (spx_cg_solve and its
 *     transpose) of a small system as ONE workgroup that runs every
 *     iteration, so no kernel is launched per iteration.  0: never.
 *     1 (default): for systems of at most 2048 rows when no launch-shape
 *     option, profiling, graph replay or the single-reduction form is set.
 *     2: whenever a 256-row tile fits in 64 KB of LDS.  Same recurrences,
 *     tests and statuses; the dots are summed in another order.
 *   SPX_OPT_IR_EARLY_EXIT: inner stopping rule of spx_cg_solve_mixed.
 *     0 (default): each inner solve runs to rtol_inner relative to its
 *     right-hand side.  1: it also stops once its residual is at most
 *     rtol_outer ||b|| / 2, so the last refinement step does no more inner
 *     iterations than the outer target needs (a reading of the Sec. 2 plan,
 *     which names no inner tolerance).
 *   SPX_OPT_SPMM_TILE_ROWS: rows per tile of the staged 16-column product
 *     of spx_spmm (16, 32 or 64; 0 = default 32): each tile's distinct rows
 *     of X are staged in LDS, so the height trades the rows of X staged per
 *     matrix row against the workgroups that fit per CU (32-row tiles run
 *     pipelined: two LDS buffers per workgroup, the next tile's rows of X
 *     loading while the current tile's products are formed).  The tiles'
 *     index is rebuilt on the next product after a change.  Results are the
 *     same bits at every height. */
enum spx_option {
  SPX_OPT_SPMV_LANES = 1,
  SPX_OPT_XCD_REMAP = 2,
  SPX_OPT_PROFILE = 3,
  SPX_OPT_SPMV_VARIANT = 4,
  SPX_OPT_ROWS_PER_BLOCK = 5,
  SPX_OPT_NONTEMPORAL = 6,
  SPX_OPT_SOLVER_BLOCKS = 7,
  SPX_OPT_QUAD_LOADS = 8,
  SPX_OPT_VECTOR_BLOCKS = 9,
  SPX_OPT_PIPELINE = 10,
  SPX_OPT_ROWS_PER_BLOCK_F32 = 11,
  SPX_OPT_CG_VARIANT = 12,
  SPX_OPT_GRAPH = 13,
  SPX_OPT_SMALL_SOLVE = 14,
  SPX_OPT_IR_EARLY_EXIT = 15,
  SPX_OPT_SPMM_TILE_ROWS = 16
};
int spx_set_option(spx_handle h, int32_t option, int64_t value);
int spx_get_option(spx_handle h, int32_t option, int64_t* value);

/* Accumulated event-timed durations (HOST outputs, milliseconds and launch
 * count) of the solver kernels that did work since the last reset, by kind:
 * 0 fp64 SpMV+dot (q = A p), 1 fp64 update (x, r, dots), 2 fp64 p update,
 * 3..5 the same kernels of the fp32 inner solve. */
int spx_get_profile(spx_handle h, int32_t kind, double* total_ms, int64_t* launches);
int spx_reset_profile(spx_handle h);

/* Thread-local message of the last failure ("" if none). */
const char* spx_last_error(void);

/* Library version string. */
const char* spx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPX_H */
