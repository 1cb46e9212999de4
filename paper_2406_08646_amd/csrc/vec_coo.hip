// COO vector assembly (paper Sec. 5: VecSetPreallocationCOO(x, n, i) and
// VecSetValuesCOO(x, v, mode), the vector counterpart of the matrix API).
//
// The pattern of a COO vector is the set of distinct kept indices; it is the
// diagonal of an n x n COO matrix with j = i, so the symbolic stage reuses
// the matrix path (device sort, run heads, jmap/perm) and the numeric stage
// reuses its in-order segmented sums, followed by one scatter of the sums
// into the caller's vector.  Duplicates are therefore summed in increasing
// k from +0.0, bitwise as for matrices.
#include <new>

#include "common.hpp"

struct spx_vec_coo {
  spx_handle m = nullptr;
};

namespace spx {
namespace {

__global__ void k_vec_scatter(const int32_t* __restrict__ idx, const double* __restrict__ sums,
                              int64_t count, int mode, double* __restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int32_t i = idx[t];
  x[i] = mode ? x[i] + sums[t] : sums[t];
}

}  // namespace
}  // namespace spx

using namespace spx;

extern "C" int spx_vec_coo_preallocate(int64_t n, int64_t ncoo, const int32_t* i, void* stream,
                                       spx_vec_handle* out) {
  clear_error();
  if (!out) return set_error(SPX_INVALID_ARG, "vec_coo_preallocate: out is NULL");
  *out = nullptr;
  spx_vec_coo* h = new (std::nothrow) spx_vec_coo();
  if (!h) return set_error(SPX_OUT_OF_MEMORY, "vec_coo_preallocate: host allocation failed");
  const int st = spx_coo_preallocate(n, ncoo, i, i, stream, &h->m);
  if (st != SPX_OK) {
    delete h;
    return st;
  }
  *out = h;
  return SPX_OK;
}

extern "C" int spx_vec_set_values_coo(spx_vec_handle h, const double* v, int mode, double* x,
                                      void* stream) {
  clear_error();
  if (!h || !h->m) return set_error(SPX_INVALID_ARG, "vec_set_values_coo: NULL handle");
  if (!x) return set_error(SPX_INVALID_ARG, "vec_set_values_coo: x is NULL");
  if (mode != SPX_INSERT_VALUES && mode != SPX_ADD_VALUES)
    return set_error(SPX_INVALID_ARG, "vec_set_values_coo: mode %d is not INSERT(0) or ADD(1)",
                     mode);
  if (h->m->nvalid > 0 && !v) return set_error(SPX_INVALID_ARG, "vec_set_values_coo: v is NULL");
  const int64_t cnt = h->m->A.nnz;
  if (cnt == h->m->n) {
    // every index is present: entry k of the pattern is x[k], so the sums
    // go straight into x (no scatter)
    return set_values_into(h->m, v, mode, x, static_cast<hipStream_t>(stream));
  }
  SPX_TRY(spx_set_values_coo(h->m, v, SPX_INSERT_VALUES, stream));
  if (cnt > 0)
    hipLaunchKernelGGL(k_vec_scatter, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), h->m->A.col, h->m->A.val, cnt, mode, x);
  SPX_CHECK_HIP(hipGetLastError());
  return SPX_OK;
}

extern "C" int spx_vec_coo_get_info(spx_vec_handle h, int64_t* n, int64_t* nunique,
                                    int64_t* nvalid, int64_t* ncoo) {
  clear_error();
  if (!h || !h->m) return set_error(SPX_INVALID_ARG, "vec_coo_get_info: NULL handle");
  return spx_get_info(h->m, n, nunique, nvalid, ncoo);
}

extern "C" int spx_vec_coo_destroy(spx_vec_handle h) {
  clear_error();
  if (!h) return SPX_OK;
  const int st = spx_destroy(h->m);
  delete h;
  return st;
}
