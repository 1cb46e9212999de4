// Internal declarations shared by the spx translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "spx.h"

namespace spx {

// ----------------------------------------------------------------- errors
int set_error(int code, const char* fmt, ...);
void clear_error();

#define SPX_CHECK_HIP(call)                                                               \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return ::spx::set_error(SPX_HIP_ERROR, "%s: %s (%s:%d)", #call, hipGetErrorString(e_), \
                              __FILE__, __LINE__);                                        \
  } while (0)

#define SPX_TRY(expr)       \
  do {                      \
    int s_ = (expr);        \
    if (s_ != SPX_OK) return s_; \
  } while (0)

// ------------------------------------------------------------- allocation
// Device memory through the installed allocator hook (hipMalloc when none);
// every failure is reported as
// SPX_OUT_OF_MEMORY with the requested size.
int dalloc(void** p, size_t bytes);
void dfree(void* p);

// Every array gets 64 bytes of tail padding, so vector loads that round a
// range up to a whole 16-byte quad stay inside the allocation.
template <typename T>
inline int dalloc_n(T** p, size_t count) {
  return dalloc(reinterpret_cast<void**>(p), count * sizeof(T) + 64);
}

// ----------------------------------------------------- launch geometry
// Compute units of the current device (cached per device).
int cu_count();
constexpr int kWave = 64;
constexpr int kXcds = 8;

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ----------------------------------------------------------------- sort
// Stable LSD radix sort of (key, value) pairs by the low `bits` bits of the
// key (1 <= bits <= 64).  Sorted output is returned in (*keys_out,
// *vals_out), which point either at the input buffers or at the alternates.
// All buffers hold `count` elements; scratch is allocated internally.
int radix_sort_pairs_u64(uint64_t* keys, uint64_t* keys_alt, uint32_t* vals, uint32_t* vals_alt,
                         int64_t count, int bits, hipStream_t s, uint64_t** keys_out,
                         uint32_t** vals_out);
// first_keys (optional): the first pass reads its keys there (keys is still
// overwritten); iota_vals: the values are the item indices 0 .. count-1.
int radix_sort_pairs_u32(uint32_t* keys, uint32_t* keys_alt, uint32_t* vals, uint32_t* vals_alt,
                         int64_t count, int bits, hipStream_t s, uint32_t** keys_out,
                         uint32_t** vals_out, const uint32_t* first_keys = nullptr,
                         bool iota_vals = false);

// Exclusive scan of uint32 counts; out may alias in.  If total != nullptr
// the sum is written there (device).  scratch: scan_scratch_elems(count).
int64_t scan_scratch_elems(int64_t count);
int exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t count, uint32_t* total,
                       uint32_t* scratch, hipStream_t s);

// -------------------------------------------------------------- matrix
// How products walk a matrix (chosen once per pattern, see spmv.hip).
enum SpmvVariant {
  kVariantAuto = 0,
  kVariantVector = 1,
  kVariantStream = 2,
  kVariantDma = 3,
  kVariantWindow = 4
};

// x window of a tile of kWinRows consecutive rows: the blocks of kWinBlock
// consecutive x entries that the tile's columns fall in, ascending.  The
// window walk stages them in LDS, and lcol[t] = slot * kWinBlock +
// col[t] % kWinBlock is entry t's position in its tile's window.  A tile
// with entries whose columns span more than kWinSpan blocks, or fall in
// more than kWinMaxBlocks of them, gets an empty window and reads x
// directly.
constexpr int kWinRows = 256;
constexpr int kWinBlock = 64;
constexpr int kWinMaxBlocks = 64;
constexpr int kWinSpan = 8192;
struct Window {
  uint16_t* lcol = nullptr;  // [nnz]
  int32_t* ptr = nullptr;    // [tiles + 1]: tile k's blocks are blk[ptr[k] .. ptr[k+1])
  int32_t* blk = nullptr;    // block numbers (x entries blk * kWinBlock ...)
  int64_t max_blocks = 0;    // largest window of any tile
  int64_t total_blocks = 0;
  int64_t gather_entries = 0;  // entries of tiles without a window
};

// Rows of X a tile of `rows` consecutive rows of the matrix touches, for
// the 16-column product (spmm.hip): tile b's list holds its number of
// distinct columns, then those columns ascending, at a fixed stride; lidx
// holds each entry's position in its tile's list.  A tile with more entries
// or distinct columns than its kernel stages has the count -1 and is
// gathered directly.
struct RowSet {
  int32_t* col = nullptr;    // [tiles * stride] count, then the columns
  uint16_t* lidx = nullptr;  // [nnz] entry t's position in its tile's list
  int rows = 0;              // tile height the lists were built for
  bool built = false;
};

// What the kernels of the window walk receive.
struct WinView {
  const uint16_t* lcol;
  const int32_t* ptr;
  const int32_t* blk;
};

struct Csr {
  int64_t n = 0, nnz = 0;
  int32_t* rowptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
  float* val32 = nullptr;
  int32_t* dpos = nullptr;  // position of the diagonal entry of each row, -1 if absent
  int64_t max_row = 0;
  // largest number of entries in a block of 32/64/128/256 consecutive rows
  int64_t tile_nnz[4] = {0, 0, 0, 0};
  Window win;  // empty (lcol == nullptr) when the pattern does not profit from one
  RowSet rs;   // built on the first 16-column product
};

inline WinView win_view(const Csr& A) { return WinView{A.win.lcol, A.win.ptr, A.win.blk}; }

// Resolved launch shape of a product on one matrix.
struct SpmvShape {
  int variant;   // kVariantVector, kVariantStream, kVariantDma or kVariantWindow
  int lanes;     // vector: lanes per row
  int rows;      // stream: rows per workgroup
  size_t lds;    // stream: LDS bytes per workgroup (for 8-byte products)
  int nt;        // non-temporal matrix loads
  int vec;       // stream: 16-byte quad loads
  int pipe;      // stream, persistent kernels: next tile's loads issued early
  int64_t tile;  // stream / DMA: most entries in one tile of `rows` rows
                 // window: x entries of the largest window (LDS slots)
};

// Device-resident solver scalars of one CG run.  rho[k & 1] holds r_k . z_k,
// so the kernels of iteration k read rho[(k - 1) & 1] while one thread
// writes rho[k & 1].
struct CgScalars {
  double rho[2];
  double alpha_s[2];  // single-reduction variant: alpha_k in slot k & 1
  double alpha, beta, pq;
  double rr, bb, bnorm, thresh;
  double r0norm, rr_true, spare;
  double tau[2], theta, eta;  // TFQMR quasi-residual recurrences
  int32_t iters, done, status, maxit;
  // Launch position at which the solve stopped (INT32_MAX while running).
  // A kernel that must finish its own work after the stopping test compares
  // it with its own position instead of reading `done`, which another
  // workgroup of the same launch may already have set.
  int32_t stop_pos;
  // TFQMR cycles: verify = 1 once a cycle ended on its residual bound and
  // the true residual is still to be checked; the current cycle started at
  // iteration j0 after m0 half-steps; restarts done so far.
  int32_t verify, restarts, j0, m0;
  // iteration number of the running CG iteration, written by its update
  // kernel when the launches take it from the device (graph replay)
  int32_t kcur;
};

}  // namespace spx

struct spx_matrix {
  int device = 0;
  int64_t n = 0, ncoo = 0, nvalid = 0;
  int colbits = 0;
  spx::Csr A;   // the matrix
  spx::Csr At;  // explicit transpose (built lazily)
  int32_t* jmap = nullptr;  // [nnz+1]
  int32_t* perm = nullptr;  // [nvalid] (buffer holds ncoo)
  int32_t* tmap = nullptr;  // A^T entry -> A entry
  int32_t* kslot = nullptr; // triplet -> entry (lazy)
  bool has_t = false, valT_fresh = false, val32_fresh = false, valT32_fresh = false;
  bool dinv_fresh = false;
  double* dinv = nullptr;
  float* dinv32 = nullptr;
  // solver workspace (lazy): r, z/p, q vectors and scalars
  double* work = nullptr;
  size_t work_elems = 0;
  float* work32 = nullptr;
  spx::CgScalars* scal = nullptr;  // device [2]
  spx::CgScalars* scal_host = nullptr;  // pinned [2]
  hipEvent_t ev[2] = {nullptr, nullptr};
  double* partials = nullptr;  // device reduction partials
  int64_t partial_cap = 0;
  int lanes_opt = 0;  // 0 = auto
  int xcd_remap = -1;  // block order: 1 XCD-aware, 0 plain, -1 by walk (remap_for)
  int variant_opt = 0;   // SpmvVariant
  int rows_opt = 0;      // stream rows per workgroup, 0 = auto
  int nt_opt = 1;        // non-temporal matrix loads
  int vec_opt = 0;       // quad loads in the stream walk
  int pipe_opt = 0;      // pipelined tiles in the persistent solver kernels
  int rows32_opt = 0;    // rows per tile of the fp32 operator, 0 = auto
  int cg_variant = -1;   // 0 Hestenes-Stiefel (3 kernels), 1 single reduction (2), -1 by size (cg_form)
  int fused_opt = 0;     // workgroups of the solver SpMV kernels, 0 = auto
  int vec_blocks_opt = 0;  // workgroups of the solver vector kernels, 0 = auto
  // optional per-kernel timing of solver iterations (HIP events)
  int profile = 0;
  double prof_ms[6] = {0, 0, 0, 0, 0, 0};
  int64_t prof_cnt[6] = {0, 0, 0, 0, 0, 0};
  hipEvent_t* prof_ev = nullptr;
  int64_t prof_ev_n = 0;
  // replay of one poll chunk of CG iterations as a HIP graph (fp64, fp32)
  int graph_opt = 0;
  int small_opt = 1;  // one-workgroup solve: 0 never, 1 small systems, 2 whenever it fits
  int ir_early_exit = 0;  // refinement: 1 also ends an inner solve at rtol_outer ||b|| / 2
  int spmm_rows_opt = 0;  // tile height of the staged 16-column product, 0 = 32
  hipStream_t cap_stream = nullptr;
  struct GraphCache {
    hipGraphExec_t exec = nullptr;
    uintptr_t key[16] = {};
  } graph[2];
};

namespace spx {
// Block order of a product walk: the option's value when set, otherwise
// plain workgroup order for the window walk (the resident workgroups then
// sweep one contiguous stretch of the matrix; x comes from the staged
// windows) and the XCD-aware order for the other walks (the x entries a
// region gathers stay in its XCD's L2).
inline int remap_for(const spx_matrix* h, const SpmvShape& sh) {
  if (h->xcd_remap >= 0) return h->xcd_remap;
  return sh.variant == kVariantWindow ? 0 : 1;
}

// assembly.hip
int ensure_transpose(spx_matrix* h, hipStream_t s);
int ensure_kslot(spx_matrix* h, hipStream_t s);
int ensure_val32(spx_matrix* h, hipStream_t s);
// spmv.hip
int pick_lanes(const Csr& A, int opt);
int compute_tiles(Csr& A, hipStream_t s);
// window.hip
int build_window(Csr& A, hipStream_t s);
// assembly.hip: the numeric stage of h's pattern into out (nnz entries) in
// mode (SPX_INSERT_VALUES or SPX_ADD_VALUES); h's own values are untouched
int set_values_into(spx_handle h, const double* v, int mode, double* out, hipStream_t s);
// cg.hip: the CG form (0 textbook, 1 single reduction) a solve on M takes
int cg_form(const spx_matrix* h, const Csr& M);
SpmvShape spmv_shape(const spx_matrix* h, const Csr& A);
// MatMult's shape: the window walk from fewer tiles than the solvers'
SpmvShape matmult_shape(const spx_matrix* h, const Csr& A);
// allow_window = false: the shape the options give without the window walk;
// matmult: MatMult's threshold for the window walk
SpmvShape spmv_shape_for(const spx_matrix* h, const Csr& A, bool allow_window,
                         bool matmult = false);
SpmvShape spmv_shape32(const spx_matrix* h, const Csr& A);
SpmvShape solver_shape(const spx_matrix* h, const Csr& A);
int launch_spmv(const Csr& A, const SpmvShape& sh, const double* x, double* y, int remap,
                hipStream_t s);
int launch_spmm(const Csr& A, int64_t nrhs, const double* X, int64_t ldx, double* Y, int64_t ldy,
                hipStream_t s);
// spmm.hip: the row-set index of A (once) and the 16-column product that
// stages each tile's rows of X in LDS (X and Y contiguous, 16-byte aligned)
int build_rowset(Csr& A, int rows, hipStream_t s);
int launch_spmm_rowset(const Csr& A, const double* X, double* Y, hipStream_t s);
// cg.hip
int fused_blocks(const spx_matrix* h);
int vector_blocks(const spx_matrix* h);
}  // namespace spx
