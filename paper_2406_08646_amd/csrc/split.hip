// One rank's share of a row-distributed matrix (paper Sec. 5): the rows
// [lo, hi) of an n_global x n_global matrix, stored as two sequential CSR
// matrices, the diagonal block (columns in [lo, hi), intra-process
// coupling) and the off-diagonal block (every other column, inter-process
// coupling), both assembled from the one COO stream the caller passes.
//
// Each block is an ordinary spx matrix built from the full stream with
// remapped indices: a triplet that belongs to the other block, to another
// rank's rows (PETSc would route it to a send buffer) or that is ignored
// gets index -1, which the symbolic stage drops (Sec. 5's rule for negative
// indices).  So every block's jmap/perm point straight into the caller's
// v, and the numeric stage of a block is spx_set_values_coo on the full v.
// The off-diagonal block is compressed in both directions: its rows are
// the local rows that have an off-diagonal entry (`orows`, ascending) and
// its columns the distinct off-diagonal global columns (`garray`,
// ascending: the ghost entries of x a halo exchange brings in).
//
// The product y = A_d x_local + A_o x_ghost runs the diagonal block's
// product, then one kernel adds each compressed row's sum (entries in
// column order from +0.0) to y at its local row.
#include <algorithm>
#include <new>
#include <string>

#include "common.hpp"

struct spx_split {
  int device = 0;
  int64_t n_global = 0, lo = 0, hi = 0, ncoo = 0;
  int64_t nremote = 0;  // kept triplets in other ranks' rows (not assembled here)
  int64_t nghost = 0, nrows_o = 0;
  spx_handle D = nullptr;  // (hi - lo) x (hi - lo)
  spx_handle O = nullptr;  // max(nrows_o, nghost, 1) square; rows >= nrows_o empty
  int32_t* garray = nullptr;  // [nghost]
  int32_t* orows = nullptr;   // [nrows_o]
};

namespace spx {
namespace {

constexpr int kSplitBlock = 256;

// Classifies every triplet: indices for the diagonal block (local row and
// column, else -1), flags for the rows and ghost columns of the
// off-diagonal block, and counts of remote triplets and of indices >= n.
__global__ __launch_bounds__(kSplitBlock) void k_split_mark(
    const int32_t* __restrict__ i, const int32_t* __restrict__ j, int64_t ncoo, int64_t n,
    int64_t lo, int64_t hi, int32_t* __restrict__ id, int32_t* __restrict__ jd,
    uint32_t* __restrict__ rowflag, uint32_t* __restrict__ colflag,
    unsigned long long* __restrict__ counts) {
  const int64_t k = (int64_t)blockIdx.x * kSplitBlock + threadIdx.x;
  unsigned remote = 0, bad = 0;
  if (k < ncoo) {
    const int64_t r = i[k], c = j[k];
    int32_t a = -1, b = -1;
    if (r >= 0 && c >= 0) {
      if (r >= n || c >= n) {
        bad = 1;
      } else if (r < lo || r >= hi) {
        remote = 1;
      } else if (c >= lo && c < hi) {
        a = (int32_t)(r - lo);
        b = (int32_t)(c - lo);
      } else {
        rowflag[r - lo] = 1u;  // every writer stores the same value
        colflag[c] = 1u;
      }
    }
    id[k] = a;
    jd[k] = b;
  }
  const unsigned long long nr = __ballot(remote), nb = __ballot(bad);
  if ((threadIdx.x & 63) == 0) {
    if (nr) atomicAdd(&counts[0], (unsigned long long)__popcll(nr));
    if (nb) atomicAdd(&counts[1], (unsigned long long)__popcll(nb));
  }
}

// Indices of the off-diagonal block: the rank of the local row among the
// flagged rows and of the global column among the flagged columns.
__global__ __launch_bounds__(kSplitBlock) void k_split_offdiag(
    const int32_t* __restrict__ i, const int32_t* __restrict__ j, int64_t ncoo, int64_t n,
    int64_t lo, int64_t hi, const uint32_t* __restrict__ rowrank,
    const uint32_t* __restrict__ colrank, int32_t* __restrict__ io, int32_t* __restrict__ jo) {
  const int64_t k = (int64_t)blockIdx.x * kSplitBlock + threadIdx.x;
  if (k >= ncoo) return;
  const int64_t r = i[k], c = j[k];
  const bool off = r >= lo && r < hi && c >= 0 && c < n && (c < lo || c >= hi);
  io[k] = off ? (int32_t)rowrank[r - lo] : -1;
  jo[k] = off ? (int32_t)colrank[c] : -1;
}

// out[rank[t]] = t for every flagged t (the ascending list of flagged t).
__global__ __launch_bounds__(kSplitBlock) void k_flag_list(const uint32_t* __restrict__ flag,
                                                           const uint32_t* __restrict__ rank,
                                                           int64_t count, int64_t offset,
                                                           int32_t* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * kSplitBlock + threadIdx.x;
  if (t < count && flag[t]) out[rank[t]] = (int32_t)(t + offset);
}

__global__ __launch_bounds__(kSplitBlock) void k_fill_u32(uint32_t* p, int64_t count) {
  const int64_t t = (int64_t)blockIdx.x * kSplitBlock + threadIdx.x;
  if (t < count) p[t] = 0u;
}

// y[orows[r]] += sum over row r of the off-diagonal block of a_rc x_ghost[c],
// the products added in column order from +0.0; one thread per row.
__global__ __launch_bounds__(kSplitBlock) void k_split_offdiag_add(
    int64_t nrows, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const int32_t* __restrict__ orows,
    const double* __restrict__ xg, double* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * kSplitBlock + threadIdx.x;
  if (r >= nrows) return;
  double s = 0.0;
  for (int32_t t = rowptr[r]; t < rowptr[r + 1]; ++t) s += val[t] * xg[col[t]];
  const int32_t dst = orows[r];
  y[dst] = y[dst] + s;
}

__global__ __launch_bounds__(kSplitBlock) void k_split_gather(int64_t nghost,
                                                              const int32_t* __restrict__ garray,
                                                              const double* __restrict__ x,
                                                              double* __restrict__ xg) {
  const int64_t c = (int64_t)blockIdx.x * kSplitBlock + threadIdx.x;
  if (c < nghost) xg[c] = x[garray[c]];
}

inline unsigned grid_of(int64_t count) {
  return (unsigned)std::max<int64_t>(1, ceil_div(count, kSplitBlock));
}

// Device buffers of the symbolic stage, freed on every exit path.
struct SplitTemps {
  int32_t *id = nullptr, *jd = nullptr;
  uint32_t *rowflag = nullptr, *colflag = nullptr, *rowrank = nullptr, *colrank = nullptr;
  uint32_t *scan_scratch = nullptr, *totals = nullptr;
  unsigned long long* counts = nullptr;
  ~SplitTemps() {
    dfree(id);
    dfree(jd);
    dfree(rowflag);
    dfree(colflag);
    dfree(rowrank);
    dfree(colrank);
    dfree(scan_scratch);
    dfree(totals);
    dfree(counts);
  }
};

int split_build(spx_split* S, const int32_t* i, const int32_t* j, hipStream_t s) {
  const int64_t n = S->n_global, lo = S->lo, hi = S->hi, m = hi - lo, ncoo = S->ncoo;
  SplitTemps T;
  const size_t nk = (size_t)std::max<int64_t>(ncoo, 1);
  SPX_TRY(dalloc_n(&T.id, nk));
  SPX_TRY(dalloc_n(&T.jd, nk));
  SPX_TRY(dalloc_n(&T.rowflag, (size_t)m));
  SPX_TRY(dalloc_n(&T.colflag, (size_t)n));
  SPX_TRY(dalloc_n(&T.rowrank, (size_t)m));
  SPX_TRY(dalloc_n(&T.colrank, (size_t)n));
  SPX_TRY(dalloc_n(&T.scan_scratch, (size_t)scan_scratch_elems(std::max(m, n))));
  SPX_TRY(dalloc_n(&T.totals, 2));
  SPX_TRY(dalloc_n(&T.counts, 2));
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_of(m)), dim3(kSplitBlock), 0, s, T.rowflag, m);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_of(n)), dim3(kSplitBlock), 0, s, T.colflag, n);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kSplitBlock), 0, s,
                     reinterpret_cast<uint32_t*>(T.counts), (int64_t)4);
  if (ncoo > 0)
    hipLaunchKernelGGL(k_split_mark, dim3(grid_of(ncoo)), dim3(kSplitBlock), 0, s, i, j, ncoo, n,
                       lo, hi, T.id, T.jd, T.rowflag, T.colflag, T.counts);
  SPX_TRY(exclusive_scan_u32(T.rowflag, T.rowrank, m, T.totals, T.scan_scratch, s));
  SPX_TRY(exclusive_scan_u32(T.colflag, T.colrank, n, T.totals + 1, T.scan_scratch, s));
  uint32_t tot[2] = {0, 0};
  unsigned long long cnt[2] = {0, 0};
  SPX_CHECK_HIP(hipMemcpyAsync(tot, T.totals, sizeof(tot), hipMemcpyDeviceToHost, s));
  SPX_CHECK_HIP(hipMemcpyAsync(cnt, T.counts, sizeof(cnt), hipMemcpyDeviceToHost, s));
  SPX_CHECK_HIP(hipStreamSynchronize(s));
  if (cnt[1] > 0)
    return set_error(SPX_INDEX_OUT_OF_RANGE,
                     "split_preallocate: %llu triplets have an index >= n_global = %lld", cnt[1],
                     (long long)n);
  S->nremote = (int64_t)cnt[0];
  S->nrows_o = tot[0];
  S->nghost = tot[1];
  SPX_TRY(dalloc_n(&S->orows, (size_t)std::max<int64_t>(S->nrows_o, 1)));
  SPX_TRY(dalloc_n(&S->garray, (size_t)std::max<int64_t>(S->nghost, 1)));
  hipLaunchKernelGGL(k_flag_list, dim3(grid_of(m)), dim3(kSplitBlock), 0, s, T.rowflag, T.rowrank,
                     m, (int64_t)0, S->orows);
  hipLaunchKernelGGL(k_flag_list, dim3(grid_of(n)), dim3(kSplitBlock), 0, s, T.colflag, T.colrank,
                     n, (int64_t)0, S->garray);
  SPX_CHECK_HIP(hipGetLastError());
  // the diagonal block from the stream with its own indices
  SPX_TRY(spx_coo_preallocate(m, ncoo, T.id, T.jd, s, &S->D));
  // the off-diagonal block, reusing the index buffers
  if (ncoo > 0)
    hipLaunchKernelGGL(k_split_offdiag, dim3(grid_of(ncoo)), dim3(kSplitBlock), 0, s, i, j, ncoo,
                       n, lo, hi, T.rowrank, T.colrank, T.id, T.jd);
  SPX_CHECK_HIP(hipGetLastError());
  const int64_t no = std::max<int64_t>({S->nrows_o, S->nghost, (int64_t)1});
  SPX_TRY(spx_coo_preallocate(no, ncoo, T.id, T.jd, s, &S->O));
  SPX_CHECK_HIP(hipStreamSynchronize(s));  // before the temporaries go
  return SPX_OK;
}

}  // namespace
}  // namespace spx

using namespace spx;

extern "C" int spx_split_destroy(spx_split_handle S) {
  clear_error();
  if (!S) return SPX_OK;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != S->device) (void)hipSetDevice(S->device);
  (void)spx_destroy(S->D);
  (void)spx_destroy(S->O);
  dfree(S->garray);
  dfree(S->orows);
  if (cur != S->device) (void)hipSetDevice(cur);
  delete S;
  return SPX_OK;
}

extern "C" int spx_split_preallocate(int64_t n_global, int64_t row_lo, int64_t row_hi,
                                     int64_t ncoo, const int32_t* i, const int32_t* j,
                                     void* stream, spx_split_handle* out) {
  clear_error();
  if (!out) return set_error(SPX_INVALID_ARG, "split_preallocate: out is NULL");
  *out = nullptr;
  if (n_global <= 0 || n_global > INT32_MAX - 1)
    return set_error(SPX_INVALID_ARG, "split_preallocate: n_global = %lld out of [1, 2^31-2]",
                     (long long)n_global);
  if (row_lo < 0 || row_hi <= row_lo || row_hi > n_global)
    return set_error(SPX_INVALID_ARG,
                     "split_preallocate: rows [%lld, %lld) not a nonempty range of [0, %lld)",
                     (long long)row_lo, (long long)row_hi, (long long)n_global);
  if (ncoo < 0 || ncoo > INT32_MAX - 1)
    return set_error(SPX_INVALID_ARG, "split_preallocate: ncoo = %lld out of [0, 2^31-2]",
                     (long long)ncoo);
  if (ncoo > 0 && (!i || !j)) return set_error(SPX_INVALID_ARG, "split_preallocate: i or j is NULL");
  spx_split* S = new (std::nothrow) spx_split();
  if (!S) return set_error(SPX_OUT_OF_MEMORY, "split_preallocate: host allocation failed");
  S->n_global = n_global;
  S->lo = row_lo;
  S->hi = row_hi;
  S->ncoo = ncoo;
  const hipError_t e = hipGetDevice(&S->device);
  int st = e == hipSuccess ? SPX_OK
                           : set_error(SPX_HIP_ERROR, "split_preallocate: %s", hipGetErrorString(e));
  if (st == SPX_OK) st = split_build(S, i, j, static_cast<hipStream_t>(stream));
  if (st != SPX_OK) {
    const std::string msg = spx_last_error();
    (void)spx_split_destroy(S);
    return set_error(st, "%s", msg.c_str());
  }
  *out = S;
  return SPX_OK;
}

extern "C" int spx_split_set_values_coo(spx_split_handle S, const double* v, int mode,
                                        void* stream) {
  clear_error();
  if (!S) return set_error(SPX_INVALID_ARG, "split_set_values_coo: NULL handle");
  SPX_TRY(spx_set_values_coo(S->D, v, mode, stream));
  return spx_set_values_coo(S->O, v, mode, stream);
}

extern "C" int spx_split_matmult(spx_split_handle S, const double* x_local, const double* x_ghost,
                                 double* y, void* stream) {
  clear_error();
  if (!S || !x_local || !y || (S->nghost > 0 && !x_ghost))
    return set_error(SPX_INVALID_ARG, "split_matmult: NULL argument");
  SPX_TRY(spx_matmult(S->D, x_local, y, stream));
  if (S->nrows_o > 0) {
    const Csr& O = S->O->A;
    hipLaunchKernelGGL(k_split_offdiag_add, dim3(grid_of(S->nrows_o)), dim3(kSplitBlock), 0,
                       static_cast<hipStream_t>(stream), S->nrows_o, O.rowptr, O.col, O.val,
                       S->orows, x_ghost, y);
    SPX_CHECK_HIP(hipGetLastError());
  }
  return SPX_OK;
}

extern "C" int spx_split_gather_ghosts(spx_split_handle S, const double* x_global,
                                       double* x_ghost, void* stream) {
  clear_error();
  if (!S || (S->nghost > 0 && (!x_global || !x_ghost)))
    return set_error(SPX_INVALID_ARG, "split_gather_ghosts: NULL argument");
  if (S->nghost > 0) {
    hipLaunchKernelGGL(k_split_gather, dim3(grid_of(S->nghost)), dim3(kSplitBlock), 0,
                       static_cast<hipStream_t>(stream), S->nghost, S->garray, x_global, x_ghost);
    SPX_CHECK_HIP(hipGetLastError());
  }
  return SPX_OK;
}

extern "C" int spx_split_get_info(spx_split_handle S, int64_t* rows, int64_t* nghost,
                                  int64_t* nrows_offdiag, int64_t* nremote) {
  clear_error();
  if (!S) return set_error(SPX_INVALID_ARG, "split_get_info: NULL handle");
  if (rows) *rows = S->hi - S->lo;
  if (nghost) *nghost = S->nghost;
  if (nrows_offdiag) *nrows_offdiag = S->nrows_o;
  if (nremote) *nremote = S->nremote;
  return SPX_OK;
}

extern "C" int spx_split_blocks(spx_split_handle S, spx_handle* diag, spx_handle* offdiag) {
  clear_error();
  if (!S) return set_error(SPX_INVALID_ARG, "split_blocks: NULL handle");
  if (diag) *diag = S->D;
  if (offdiag) *offdiag = S->O;
  return SPX_OK;
}

extern "C" int spx_split_get_maps(spx_split_handle S, int32_t* garray, int32_t* orows,
                                  void* stream) {
  clear_error();
  if (!S) return set_error(SPX_INVALID_ARG, "split_get_maps: NULL handle");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (garray && S->nghost)
    SPX_CHECK_HIP(hipMemcpyAsync(garray, S->garray, sizeof(int32_t) * (size_t)S->nghost,
                                 hipMemcpyDeviceToDevice, s));
  if (orows && S->nrows_o)
    SPX_CHECK_HIP(hipMemcpyAsync(orows, S->orows, sizeof(int32_t) * (size_t)S->nrows_o,
                                 hipMemcpyDeviceToDevice, s));
  return SPX_OK;
}
