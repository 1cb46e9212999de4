// Batched Jacobi-CG over many independent systems (paper Sec. 7).
#include "common.hpp"

using namespace spx;

extern "C" int spx_batch_create(int32_t nsys, const spx_handle* hs, void* stream,
                                spx_batch_handle* out) {
  (void)nsys; (void)hs; (void)stream;
  if (out) *out = nullptr;
  return set_error(SPX_NOT_IMPLEMENTED, "batch_create: not implemented yet");
}

extern "C" int spx_batch_destroy(spx_batch_handle b) {
  (void)b;
  return SPX_OK;
}

extern "C" int spx_batch_total_rows(spx_batch_handle b, int64_t* total) {
  (void)b; (void)total;
  return set_error(SPX_NOT_IMPLEMENTED, "batch_total_rows: not implemented yet");
}

extern "C" int spx_batch_cg(spx_batch_handle b, const double* bvec, double* x, double rtol,
                            int64_t maxit, double team_weight_exponent, int32_t lanes,
                            void* stream, int64_t* iters_out, double* relres_out) {
  (void)b; (void)bvec; (void)x; (void)rtol; (void)maxit; (void)team_weight_exponent; (void)lanes;
  (void)stream; (void)iters_out; (void)relres_out;
  return set_error(SPX_NOT_IMPLEMENTED, "batch_cg: not implemented yet");
}
