// common.h -- internal declarations of libmxs (not part of the C ABI).
//
// Device-side conventions for gfx950:
//  * wave64 everywhere; reductions inside a wave use xor-butterflies, whose
//    result is bitwise identical in every lane (each step adds the same two
//    operands in both partner lanes), so every reduction is deterministic.
//  * cross-block reductions never use floating-point atomics or
//    device-scope fences: blocks write partial sums to fixed slots and the
//    next kernel (or a one-block finishing kernel) adds them in slot order.
//  * work-groups are dispatched round-robin over the 8 XCDs; kernels that
//    stream rows remap blockIdx so that each XCD (and its private L2) works
//    on one contiguous eighth of the rows and of the x-vector window they
//    gather from.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mxs.h"

namespace mxs {

constexpr int kWave = 64;
constexpr int kNumXcd = 8;

// ---------------------------------------------------------------------------
// host-side objects
// ---------------------------------------------------------------------------
struct Allocator {
  mxs_allocator cb{};
  bool custom = false;
  void* stream = nullptr;
  void* alloc(size_t bytes) const;
  void release(void* p) const;
};

struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace mxs

struct mxs_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  mxs::Allocator alloc;
  std::string last_error;
  int num_cus = 256;
  // grow-only scratch for solvers and format conversion
  mxs::Workspace ws;
  // grow-only scratch of the chunked products (continuation partials)
  mxs::Workspace spmv_ws;
  // pinned host mirror of small device state blocks
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  // cache-flush buffer
  void* flush = nullptr;
  size_t flush_bytes = 0;
  // solver status polling: two copies of the device state in flight, each
  // marked by an event (created with the ctx)
  hipEvent_t poll_ev[2] = {nullptr, nullptr};
};

namespace mxs {

// CSR: rows partitioned into blocks of at most block_nnz entries (a row
// longer than that is a block on its own); one wave per block.
// CSR: either the "stream" kernel over row blocks (lanes == 0) or the
// "vector" kernel with `lanes` lanes per row and `rpg` rows per lane group.
struct CsrPart {
  int32_t* rowptr = nullptr;
  int32_t* col = nullptr;
  void* val = nullptr;
  float* scale = nullptr;  // F16_ROWSCALED only
  int32_t* blocks = nullptr;  // first row of each block (nblocks + 1)
  int32_t* bnnz = nullptr;    // first entry of each block (nblocks + 1)
  int64_t nblocks = 0;
  int block_nnz = 512;
  int lanes = 0;  // 0: stream kernel; 1: thread per row; >1: lanes per row
  int rpg = 4;
  int wpb = 4;    // stream kernel: independent waves per work-group (1 or 4)
  bool rows_lds = false;  // rows-from-LDS kernel (blocks of <= 64/rl_lanes rows, block_nnz entries)
  int rl_lanes = 1;       // rows-from-LDS kernel: lanes per row (1, 2 or 4)
  int rl_step = 8;        // rows-from-LDS kernel: a lane's entries per step (8 or 16)
  bool products = false;  // products-through-LDS kernel (the same blocks)
  // merge-path kernel: equal chunks of block_nnz entries; crow[c] is the row
  // of entry c * block_nnz (crow[nchunks]: the row of the last entry)
  bool merge = false;
  int32_t* crow = nullptr;
  int64_t nchunks = 0;
  int32_t* empty_rows = nullptr;
  int64_t nempty = 0;
  // merge path over column panels (panels > 1): the entries again, panel by
  // panel; stacked row r (a row's entries in one panel, empty ones left out)
  // holds entries srowptr[r] .. srowptr[r+1]-1 of scol/sval and belongs to
  // panel srid[r] / n, row srid[r] % n; pmask[i] has bit p set when row i
  // has entries in panel p.  crow/nchunks then describe the stacked rows.
  int panels = 1;
  int32_t* srowptr = nullptr;
  int32_t* srid = nullptr;
  int32_t* scol = nullptr;
  void* sval = nullptr;
  uint8_t* pmask = nullptr;
  int64_t nsrows = 0;
  // FP64 / FP32 values: the output slot srid[r] of every entry's stacked
  // row (srow, like COO's row array), with srow, scol and sval padded with
  // zeros to whole 1024-entry chunks, so the product runs the COO chunks
  // over the panel copy (row-scaled FP16 keeps the merge kernel)
  int32_t* srow = nullptr;
};

// COO: equal chunks of block_nnz entries, one wave per chunk.  Rows cut by
// a chunk boundary are completed by a fix-up pass from per-chunk
// continuation partials; rows with no entry are listed in empty_rows.  The
// partials live in scratch memory of the product's context (or of the
// caller), never in the matrix, so a matrix is read-only during a product
// and two contexts may use it at once.
struct CooPart {
  int32_t* row = nullptr;
  int32_t* col = nullptr;
  void* val = nullptr;
  int64_t nnz = 0;
  int64_t nchunks = 0;
  int block_nnz = 512;
  int32_t* empty_rows = nullptr;
  int64_t nempty = 0;
  int wpb = 4;  // independent waves per work-group (1 or 4)
  int kernel = MXS_COO_LDS;  // MXS_COO_LDS or MXS_COO_RUNS
  // column panels (COO format only, panels > 1): the entries ordered by
  // panel, then row, then column, with row[k] = p * n + i for an entry of
  // row i in panel p; the chunks write the P * n panel partials (product
  // scratch) and a last pass adds each row's partials in panel order,
  // reading those whose bit is set in pmask[i]
  int panels = 1;
  uint8_t* pmask = nullptr;
};

// ELL: column-major padded slots; `waves` waves per 64 rows split the
// columns round-robin.
struct EllPart {
  int32_t* col = nullptr;
  void* val = nullptr;
  int64_t K = 0;
  int64_t stride = 0;
  int waves = 1;
};

}  // namespace mxs

struct mxs_matrix {
  int device = 0;
  mxs::Allocator alloc;
  int64_t n = 0, ncols = 0, nnz = 0;
  mxs_format fmt = MXS_CSR;
  mxs_dtype dt = MXS_F64;
  mxs::CsrPart csr;
  mxs::CooPart coo;
  mxs::EllPart ell;
  std::vector<void*> owned;
  int64_t bytes = 0;
  // host copy of the row pointers (analysis data kept for conversions)
  std::vector<int32_t> h_rowptr;
};

// Jacobi: 1/a_ii per row; block Jacobi: inverted diagonal blocks,
// column-major bs x bs slots.  FP64 and the same values rounded to FP32.
struct mxs_precond {
  int device = 0;
  mxs::Allocator alloc;
  int32_t kind = 0;
  int64_t n = 0;
  int32_t bs = 1;
  int64_t nb = 0;
  int64_t count = 0;  // stored values
  double* m64 = nullptr;
  float* m32 = nullptr;
};

// A directed graph stored by in-links with its transition matrix
// T[j,i] = 1/d_i (d_i = out-degree of i) as an F64 CSR matrix, and the
// nodes without out-links.
struct mxs_graph {
  int device = 0;
  mxs::Allocator alloc;
  int64_t n = 0, nnz = 0;
  mxs_matrix* T = nullptr;
  uint8_t* dangling = nullptr;
  int64_t ndangling = 0;
};

namespace mxs {

mxs_status fail(mxs_ctx* ctx, mxs_status s, const char* fmt, ...);
void* mat_alloc(mxs_matrix* A, size_t bytes);
bool ws_reserve(mxs_ctx* ctx, size_t bytes);
bool pinned_reserve(mxs_ctx* ctx, size_t bytes);

inline size_t value_bytes(mxs_dtype dt) {
  return dt == MXS_C128 ? 16 : (dt == MXS_F64 || dt == MXS_C64) ? 8 : dt == MXS_F32 ? 4 : 2;
}

// launchers shared between translation units (all enqueue on ctx->stream)
// skip (nullable, device): when *skip != 0 every kernel of the product
// returns at once (solvers queue iterations past convergence this way)
mxs_status launch_spmv(mxs_ctx* ctx, const mxs_matrix* A, const void* alpha, const void* x,
                       const void* beta, void* y, const int32_t* skip);
// Device scratch one product of A needs (continuation partials of the
// merge-path CSR and COO chunks; 0 for the other kernels), and the same
// product with that scratch supplied by the caller (at least
// spmv_scratch_bytes(A) bytes, 256-byte aligned, not in use by any other
// product until this one completes on ctx->stream).
size_t spmv_scratch_bytes(const mxs_matrix* A);
// y = A x (square A) and, in the same launches, work-group partial sums of
// w[i] * y[i] in dpart (w = x when NULL: CG's p.q with x = p), and with
// nv = 2 also of y[i]^2, interleaved (dpart[b * nv + v]): returns how many
// work-group partials (<= kDotPartials) were written, or 0 when A's kernel
// has no such form (then nothing was enqueued and the caller forms the dots
// itself).  The merge path forms x.y only; w != x or nv = 2 need the
// rows-from-LDS kernel.
constexpr int kDotPartials = 4096;
int launch_spmv_dot(mxs_ctx* ctx, const mxs_matrix* A, const void* x, void* y,
                    const int32_t* skip, double* dpart, const void* w = nullptr, int nv = 1);
// The allocation-free product's fixed device scratch (one copy per GPU, held
// until the process ends): its size, its per-device address lookup (run once
// per device by mxs_ctx_create with that device current) and that address.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
mxs_status noalloc_scratch_init(mxs_ctx* ctx);
void* noalloc_scratch(int device);
mxs_status launch_spmv_scratch(mxs_ctx* ctx, const mxs_matrix* A, const void* alpha,
                               const void* x, const void* beta, void* y, const int32_t* skip,
                               void* scratch);
// After the values of a CSR matrix changed in place: copies them into the
// column-panel copy of the merge path (no-op for other kernels).  Enqueued.
mxs_status refresh_panel_values(mxs_ctx* ctx, mxs_matrix* A);
int64_t csr_partition(const int32_t* rowptr, int64_t n, int block_nnz,
                      std::vector<int32_t>& blocks, int64_t max_rows = -1);
// Small systems (n <= 8192, rows of <= 64 entries): CG by the batched
// engine's one-work-group kernel on one slot; solves A d = rhs from d = 0
// to ||rhs - A d|| <= tol ||rhs|| (true residual checked, up to three
// replacements); scratch of small_cg_scratch(n) device bytes.
struct SmallCgResult {
  int64_t iters = 0, replacements = 0;
  double res2 = 0.0;   // last squared residual norm (true one when converged)
  double base = 0.0;   // the norm the threshold is relative to
  mxs_status status = MXS_OK;
};
bool small_cg_fits(int64_t n, int64_t max_row);
size_t small_cg_scratch(int64_t n);
constexpr size_t kSmallCgPinned = 768;  // pinned staging bytes small_cg needs
// FP64 CG on one small CSR system in one work-group, from x0 = x (updated in
// place): r0 = b - A x0, the threshold max(rel_tol * base, abs_tol) with
// base = ||r0|| (base_r0) or ||b||, every iteration and the true-residual
// check run in the kernel; b = 0 gives x = 0.
mxs_status small_cg(mxs_ctx* ctx, const mxs_matrix* A, const double* b, double* x,
                    double rel_tol, double abs_tol, bool base_r0, int64_t max_iters,
                    void* scratch, void* pinned, SmallCgResult* res);

// Small systems (n <= 4096, at most 20 / ceil(n / 1024) entries a row) by
// pipelined CG in one work-group, same contract as small_cg; scratch of
// small_pipecg_scratch(n) device bytes.
bool small_pipecg_fits(int64_t n, int64_t max_row);
size_t small_pipecg_scratch(int64_t n);
mxs_status small_pipecg(mxs_ctx* ctx, const mxs_matrix* A, const double* rhs, double* out,
                        double tol, int64_t max_iters, void* scratch, SmallCgResult* res);

// validated F64 (or C128) CSR matrix from host or device arrays (flags as
// in mxs_matrix_create_csr); val == NULL gives zero values
mxs_status create_csr(mxs_ctx* ctx, int64_t nrows, int64_t ncols, int64_t nnz,
                      const int32_t* rowptr, const int32_t* col, const double* val, int flags,
                      mxs_matrix** out, mxs_dtype dt = MXS_F64);

}  // namespace mxs

#define MXS_HIP_TRY(ctx, expr)                                                      \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return mxs::fail((ctx), MXS_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
namespace mxs {

// Logical block for hardware block `bid` of `nblk`: XCD k (= bid % 8) gets
// the k-th contiguous eighth of the logical range.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblk) {
  const int64_t per = nblk / kNumXcd, rem = nblk % kNumXcd;
  const int64_t xcd = bid % kNumXcd, idx = bid / kNumXcd;
  return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// A double moved across lanes by a DPP pattern (both 32-bit halves alike).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
}

__device__ __forceinline__ double lane_value(double v, int lane) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
}

// Sum over the wave, the same value in every lane.  Within each row of 16
// lanes, DPP moves add the neighbour (lane ^ 1), the other pair of the quad
// (lane ^ 2), the mirrored quad of the half and the mirrored half of the row;
// the two operands of each add are the same two values in either lane, so
// every lane of a row ends with the same row sum.  The four row sums are then
// read from lanes 15, 31, 47 and 63 and added in row order.  DPP moves cost a
// few cycles where the cross-lane shuffles of a butterfly go through the LDS
// crossbar; the batched kernels take two such sums per CG iteration, and every
// solver kernel takes them at its start (finishing the previous kernel's
// partials) and at its end.  All lanes of the wave must be active.
__device__ __forceinline__ double wave_total(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return ((lane_value(v, 15) + lane_value(v, 31)) + lane_value(v, 47)) + lane_value(v, 63);
}

// Sum over a work-group of BS threads; every thread gets the result.  Wave
// partials are added in wave order by all lanes (deterministic).
template <typename T, int BS>
__device__ __forceinline__ T block_sum(T v, T* lds /* BS/64 entries */) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = v;
  __syncthreads();
  T s = lds[0];
#pragma unroll
  for (int i = 1; i < BS / kWave; ++i) s += lds[i];
  __syncthreads();
  return s;
}

__device__ __forceinline__ double to_acc(double v) { return v; }
__device__ __forceinline__ float to_acc(float v) { return v; }
__device__ __forceinline__ float to_acc(_Float16 v) { return (float)v; }

// Complex values as (re, im) pairs; the CSR kernels are instantiated with
// it as value and vector type.
template <typename R>
struct cplx {
  R re, im;
  cplx() = default;
  __host__ __device__ constexpr cplx(R r) : re(r), im(0) {}
  __host__ __device__ constexpr cplx(R r, R i) : re(r), im(i) {}
};
template <typename R>
__device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename R>
__device__ __forceinline__ cplx<R> operator*(cplx<R> a, cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cplx<R>& operator+=(cplx<R>& a, cplx<R> b) {
  a = a + b;
  return a;
}
template <typename R>
__device__ __forceinline__ cplx<R>& operator*=(cplx<R>& a, cplx<R> b) {
  a = a * b;
  return a;
}
template <typename R>
__device__ __forceinline__ bool operator==(cplx<R> a, cplx<R> b) {
  return a.re == b.re && a.im == b.im;
}
template <typename R>
__device__ __forceinline__ cplx<R> to_acc(cplx<R> v) {
  return v;
}

// Lane exchanges of complex values, part by part.  The built-in overloads
// are brought into this namespace so that these do not hide them; templates
// reach these through argument-dependent lookup.
using ::__shfl;
using ::__shfl_up;
using ::__shfl_xor;
template <typename R>
__device__ __forceinline__ cplx<R> __shfl(cplx<R> v, int src, int width) {
  return {::__shfl(v.re, src, width), ::__shfl(v.im, src, width)};
}
template <typename R>
__device__ __forceinline__ cplx<R> __shfl_up(cplx<R> v, unsigned int d, int width) {
  return {::__shfl_up(v.re, d, width), ::__shfl_up(v.im, d, width)};
}
template <typename R>
__device__ __forceinline__ cplx<R> __shfl_xor(cplx<R> v, int m, int width) {
  return {::__shfl_xor(v.re, m, width), ::__shfl_xor(v.im, m, width)};
}

}  // namespace mxs
