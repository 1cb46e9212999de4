// Handle lifetime, error reporting, allocation and options of the C ABI.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <unordered_map>

#include "common.hpp"

namespace spx {

namespace {
thread_local char g_last_error[1024] = "";
}

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_last_error[0] = '\0'; }

// The allocator hook: every device allocation goes through the hook that is
// installed when it is made, and is returned through the same hook (a
// block's owner is recorded), so the hook may change at any time.
namespace {
struct Allocator {
  spx_alloc_fn alloc = nullptr;
  spx_free_fn free = nullptr;
  void* ctx = nullptr;
};
std::mutex g_alloc_mu;
Allocator g_alloc;                                  // current hook (alloc null: hipMalloc)
std::unordered_map<void*, Allocator> g_hook_blocks;  // blocks that came from a hook
}  // namespace

int dalloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  Allocator a;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    a = g_alloc;
  }
  if (a.alloc) {
    void* q = a.alloc(bytes, a.ctx);
    if (!q)
      return set_error(SPX_OUT_OF_MEMORY, "device allocation of %zu bytes failed (allocator hook)",
                       bytes);
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_hook_blocks[q] = a;
    *p = q;
    return SPX_OK;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return set_error(SPX_OUT_OF_MEMORY, "device allocation of %zu bytes failed: %s", bytes,
                     hipGetErrorString(e));
  }
  return SPX_OK;
}

void dfree(void* p) {
  if (!p) return;
  Allocator owner;
  bool hooked = false;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    auto it = g_hook_blocks.find(p);
    if (it != g_hook_blocks.end()) {
      owner = it->second;
      hooked = true;
      g_hook_blocks.erase(it);
    }
  }
  if (hooked) {
    if (owner.free) owner.free(p, owner.ctx);
  } else {
    (void)hipFree(p);
  }
}

int cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev < 0 || dev >= 64) dev = 0;
  if (!cached[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cached[dev] = cus;
  }
  return cached[dev];
}

static void free_csr(Csr& M) {
  dfree(M.rowptr);
  dfree(M.col);
  dfree(M.val);
  dfree(M.val32);
  dfree(M.dpos);
  dfree(M.win.lcol);
  dfree(M.win.ptr);
  dfree(M.win.blk);
  dfree(M.rs.col);
  dfree(M.rs.lidx);
  M = Csr();
}

}  // namespace spx

using namespace spx;

extern "C" int spx_destroy(spx_handle h) {
  clear_error();
  if (!h) return SPX_OK;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != h->device) (void)hipSetDevice(h->device);
  free_csr(h->A);
  free_csr(h->At);
  dfree(h->jmap);
  dfree(h->perm);
  dfree(h->tmap);
  dfree(h->kslot);
  dfree(h->dinv);
  dfree(h->dinv32);
  dfree(h->work);
  dfree(h->work32);
  dfree(h->scal);
  dfree(h->partials);
  if (h->scal_host) (void)hipHostFree(h->scal_host);
  for (hipEvent_t& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  for (int64_t k = 0; k < h->prof_ev_n; ++k) (void)hipEventDestroy(h->prof_ev[k]);
  delete[] h->prof_ev;
  for (auto& gc : h->graph)
    if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (cur != h->device) (void)hipSetDevice(cur);
  delete h;
  return SPX_OK;
}

extern "C" int spx_set_allocator(spx_alloc_fn alloc, spx_free_fn free, void* ctx) {
  clear_error();
  if ((alloc == nullptr) != (free == nullptr))
    return set_error(SPX_INVALID_ARG, "set_allocator: give both functions or neither");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc.alloc = alloc;
  g_alloc.free = free;
  g_alloc.ctx = ctx;
  return SPX_OK;
}

extern "C" int spx_set_option(spx_handle h, int32_t option, int64_t value) {
  clear_error();
  if (!h) return set_error(SPX_INVALID_ARG, "set_option: NULL handle");
  switch (option) {
    case SPX_OPT_SPMV_LANES:
      if (value != 0 && (value < 1 || value > 64 || (value & (value - 1))))
        return set_error(SPX_INVALID_ARG, "set_option: lanes %lld is not 0 or a power of two <= 64",
                         (long long)value);
      h->lanes_opt = (int)value;
      return SPX_OK;
    case SPX_OPT_XCD_REMAP:
      h->xcd_remap = value < 0 ? -1 : value ? 1 : 0;
      return SPX_OK;
    case SPX_OPT_PROFILE:
      h->profile = value ? 1 : 0;
      return SPX_OK;
    case SPX_OPT_SPMV_VARIANT:
      if (value < 0 || value > 4)
        return set_error(SPX_INVALID_ARG, "set_option: variant %lld not in 0..4", (long long)value);
      h->variant_opt = (int)value;
      return SPX_OK;
    case SPX_OPT_ROWS_PER_BLOCK:
      if (value != 0 && value != 32 && value != 64 && value != 128 && value != 256)
        return set_error(SPX_INVALID_ARG, "set_option: rows per block %lld not 0/32/64/128/256",
                         (long long)value);
      h->rows_opt = (int)value;
      return SPX_OK;
    case SPX_OPT_NONTEMPORAL:
      h->nt_opt = value ? 1 : 0;
      return SPX_OK;
    case SPX_OPT_SOLVER_BLOCKS:
    case SPX_OPT_VECTOR_BLOCKS:
      if (value < 0 || value > (1 << 20))
        return set_error(SPX_INVALID_ARG, "set_option: block count %lld out of range",
                         (long long)value);
      (option == SPX_OPT_SOLVER_BLOCKS ? h->fused_opt : h->vec_blocks_opt) = (int)value;
      return SPX_OK;
    case SPX_OPT_QUAD_LOADS:
      h->vec_opt = value ? 1 : 0;
      return SPX_OK;
    case SPX_OPT_PIPELINE:
      h->pipe_opt = value ? 1 : 0;
      return SPX_OK;
    case SPX_OPT_ROWS_PER_BLOCK_F32:
      if (value != 0 && value != 32 && value != 64 && value != 128 && value != 256)
        return set_error(SPX_INVALID_ARG, "set_option: rows per block %lld not 0/32/64/128/256",
                         (long long)value);
      h->rows32_opt = (int)value;
      return SPX_OK;
    case SPX_OPT_GRAPH:
      h->graph_opt = value ? 1 : 0;
      return SPX_OK;
    case SPX_OPT_SMALL_SOLVE:
      if (value < 0 || value > 2)
        return set_error(SPX_INVALID_ARG, "set_option: small-solve mode %lld not in 0..2",
                         (long long)value);
      h->small_opt = (int)value;
      return SPX_OK;
    case SPX_OPT_CG_VARIANT:
      if (value < -1 || value > 2)
        return set_error(SPX_INVALID_ARG, "set_option: CG variant %lld not in -1..2",
                         (long long)value);
      h->cg_variant = (int)value;
      return SPX_OK;
    case SPX_OPT_IR_EARLY_EXIT:
      h->ir_early_exit = value ? 1 : 0;
      return SPX_OK;
    case SPX_OPT_SPMM_TILE_ROWS:
      if (value != 0 && value != 16 && value != 32 && value != 64)
        return set_error(SPX_INVALID_ARG, "set_option: SpMM tile height must be 0, 16, 32 or 64");
      h->spmm_rows_opt = (int)value;
      return SPX_OK;
    default:
      return set_error(SPX_INVALID_ARG, "set_option: unknown option %d", option);
  }
}

extern "C" int spx_get_option(spx_handle h, int32_t option, int64_t* value) {
  clear_error();
  if (!h || !value) return set_error(SPX_INVALID_ARG, "get_option: NULL argument");
  switch (option) {
    case SPX_OPT_SPMV_LANES:
      *value = matmult_shape(h, h->A).lanes;
      return SPX_OK;
    case SPX_OPT_XCD_REMAP:
      *value = remap_for(h, matmult_shape(h, h->A));
      return SPX_OK;
    case SPX_OPT_PROFILE:
      *value = h->profile;
      return SPX_OK;
    case SPX_OPT_SPMV_VARIANT:
      *value = matmult_shape(h, h->A).variant;
      return SPX_OK;
    case SPX_OPT_ROWS_PER_BLOCK:
      *value = matmult_shape(h, h->A).rows;
      return SPX_OK;
    case SPX_OPT_NONTEMPORAL:
      *value = h->nt_opt;
      return SPX_OK;
    case SPX_OPT_SOLVER_BLOCKS:
      *value = fused_blocks(h);
      return SPX_OK;
    case SPX_OPT_VECTOR_BLOCKS:
      *value = vector_blocks(h);
      return SPX_OK;
    case SPX_OPT_QUAD_LOADS:
      *value = h->vec_opt;
      return SPX_OK;
    case SPX_OPT_PIPELINE:
      *value = solver_shape(h, h->A).pipe;
      return SPX_OK;
    case SPX_OPT_ROWS_PER_BLOCK_F32:
      *value = spmv_shape32(h, h->A).rows;
      return SPX_OK;
    case SPX_OPT_CG_VARIANT:
      *value = cg_form(h, h->A);
      return SPX_OK;
    case SPX_OPT_GRAPH:
      *value = h->graph_opt;
      return SPX_OK;
    case SPX_OPT_SMALL_SOLVE:
      *value = h->small_opt;
      return SPX_OK;
    case SPX_OPT_IR_EARLY_EXIT:
      *value = h->ir_early_exit;
      return SPX_OK;
    case SPX_OPT_SPMM_TILE_ROWS:
      *value = h->spmm_rows_opt ? h->spmm_rows_opt : 32;
      return SPX_OK;
    default:
      return set_error(SPX_INVALID_ARG, "get_option: unknown option %d", option);
  }
}

extern "C" int spx_get_profile(spx_handle h, int32_t kind, double* total_ms, int64_t* launches) {
  clear_error();
  if (!h || kind < 0 || kind >= 6) return set_error(SPX_INVALID_ARG, "get_profile: bad argument");
  if (total_ms) *total_ms = h->prof_ms[kind];
  if (launches) *launches = h->prof_cnt[kind];
  return SPX_OK;
}

extern "C" int spx_reset_profile(spx_handle h) {
  clear_error();
  if (!h) return set_error(SPX_INVALID_ARG, "reset_profile: NULL handle");
  for (int k = 0; k < 6; ++k) {
    h->prof_ms[k] = 0.0;
    h->prof_cnt[k] = 0;
  }
  return SPX_OK;
}

extern "C" const char* spx_last_error(void) { return g_last_error; }

extern "C" const char* spx_version(void) { return "spx 0.1 gfx950"; }
