// batch.hip -- batched persistent CG and the continuous-batching engine.
//
// Many independent SPD systems are solved by one kernel per size class:
// work-group i owns slot i, keeps the search direction p in LDS (the
// gathers of its SpMV never leave the CU) and x, r, p, q in registers for
// the rows it owns, and runs up to K CG iterations per launch (the CG of
// Saad 2003, ch. 6, with the true-residual check and up to three residual
// replacements).  The state is written back to HBM at the end of a launch,
// so launches can be repeated until every slot has finished.  A system's
// arithmetic depends only on its own data and on the threads-per-system of
// its size class (a function of n), never on the other slots, so a result
// is bitwise the same alone and in any mix.
//
// The host engine owns a device arena of `budget_bytes` managed first-fit,
// a slot table in device memory, a FIFO of submitted requests, and one
// hipGraph per step (one kernel per class + the status read-back).  Each
// mxs_batch_step retires finished slots, admits waiting requests whose
// footprint fits the arena and whose class has a free slot, uploads them,
// and launches the graph.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace mxs {
namespace {

enum : int32_t {
  SLOT_NEW = 0,
  SLOT_RUN = 1,
  SLOT_CONVERGED = 2,
  SLOT_BREAKDOWN = 3,
  SLOT_NONFINITE = 4,
  SLOT_MAXIT = 5,
  SLOT_NOTCONV = 6
};

struct SlotDesc {
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  const double* b;
  double* x;
  double* r;
  double* p;
  double tol;
  double rho, thr, res2;
  int32_t n, nnz;
  int32_t max_iters;
  int32_t active;
  int32_t iters, status, repl, pad;
};

template <int BS>
__device__ __forceinline__ double bsum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int i = 1; i < BS / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

template <int BS>
__device__ __forceinline__ int bmax(int v, int* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  int s = red[0];
#pragma unroll
  for (int i = 1; i < BS / 64; ++i) s = max(s, red[i]);
  __syncthreads();
  return s;
}

// q = A v for the thread's rows (rows tid + k*BS).  The loop over the
// entry index is outermost so that the loads of all RPT rows are in flight
// together; row pointers come from LDS.
template <int BS, int RPT>
__device__ __forceinline__ void rows_times(const int32_t* __restrict__ rpl,
                                           const int32_t* __restrict__ col,
                                           const double* __restrict__ val,
                                           const double* __restrict__ vec, int n, int maxlen,
                                           double (&q)[RPT]) {
  const int tid = threadIdx.x;
  int32_t rs[RPT], re[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int i = tid + k * BS;
    rs[k] = i < n ? rpl[i] : 0;
    re[k] = i < n ? rpl[i + 1] : 0;
    q[k] = 0.0;
  }
  for (int j = 0; j < maxlen; ++j) {
    int32_t c[RPT];
    double v[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      c[k] = 0;
      v[k] = 0.0;
      if (rs[k] + j < re[k]) {
        c[k] = col[rs[k] + j];
        v[k] = val[rs[k] + j];
      }
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k)
      if (rs[k] + j < re[k]) q[k] += v[k] * vec[c[k]];
  }
}

// One work-group per slot.  BS threads, RPT rows per thread (rows
// tid + k*BS).  LDS holds the slot's row pointers and, when USE_LDS, the
// gather vector (p, or x during the true-residual check); otherwise the
// slot's p array in HBM serves as the gather vector.  x, r and q of the
// thread's rows live in registers for the whole launch.
template <int BS, int RPT, bool USE_LDS>
__global__ __launch_bounds__(BS) void k_batch_cg(SlotDesc* __restrict__ slots, int base, int K,
                                                 int vec_cap) {
  extern __shared__ double dyn[];
  __shared__ double red[BS / 64];
  __shared__ int ired[BS / 64];
  SlotDesc* S = slots + base + blockIdx.x;
  if (!S->active || S->status >= SLOT_CONVERGED) return;
  const int n = S->n;
  const int32_t* __restrict__ rp = S->rowptr;
  const int32_t* __restrict__ col = S->col;
  const double* __restrict__ val = S->val;
  const double* __restrict__ b = S->b;
  double* __restrict__ pg = S->p;
  double* __restrict__ vec = USE_LDS ? dyn : pg;
  int32_t* rpl = (int32_t*)(dyn + (USE_LDS ? vec_cap : 0));
  const int tid = threadIdx.x;
  int mylen = 0;
  for (int i = tid; i <= n; i += BS) rpl[i] = rp[i];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int i = tid + k * BS;
    if (i < n) mylen = max(mylen, rpl[i + 1] - rpl[i]);
  }
  const int maxlen = bmax<BS>(mylen, ired);
  double x[RPT], r[RPT], q[RPT];
  double rho, thr;
  int status = SLOT_RUN;
  int it = S->iters, repl = S->repl;
  if (S->status == SLOT_NEW) {
    // x0 = 0: r = b, p = r, thr = tol * ||b||
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      x[k] = 0.0;
      r[k] = i < n ? b[i] : 0.0;
      if (i < n) vec[i] = r[k];
      acc += r[k] * r[k];
    }
    rho = bsum<BS>(acc, red);
    thr = S->tol * sqrt(rho);
    if (!isfinite(rho)) status = SLOT_NONFINITE;
    if (rho == 0.0) status = SLOT_CONVERGED;  // b = 0: x = 0
  } else {
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      x[k] = i < n ? S->x[i] : 0.0;
      r[k] = i < n ? S->r[i] : 0.0;
      if (USE_LDS && i < n) vec[i] = pg[i];
    }
    rho = S->rho;
    thr = S->thr;
  }
  __syncthreads();
  double rr = rho;
  for (int s = 0; s < K && status == SLOT_RUN; ++s) {
    rows_times<BS, RPT>(rpl, col, val, vec, n, maxlen, q);
    double pq = 0.0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      if (i < n) pq += vec[i] * q[k];
    }
    pq = bsum<BS>(pq, red);
    if (!(pq > 0.0)) {
      status = isfinite(pq) ? SLOT_BREAKDOWN : SLOT_NONFINITE;
      break;
    }
    const double alpha = rho / pq;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      if (i < n) x[k] += alpha * vec[i];
      r[k] -= alpha * q[k];
      acc += r[k] * r[k];
    }
    rr = bsum<BS>(acc, red);
    ++it;
    if (!isfinite(rr)) {
      status = SLOT_NONFINITE;
      break;
    }
    if (sqrt(rr) <= thr) {
      // true residual r_t = b - A x, with x staged in the gather vector
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * BS;
        if (i < n) vec[i] = x[k];
      }
      __syncthreads();
      rows_times<BS, RPT>(rpl, col, val, vec, n, maxlen, q);
      double tt = 0.0;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * BS;
        q[k] = i < n ? b[i] - q[k] : 0.0;
        tt += q[k] * q[k];
      }
      tt = bsum<BS>(tt, red);
      if (sqrt(tt) <= thr) {
        status = SLOT_CONVERGED;
        rr = tt;
        break;
      }
      if (repl >= 3) {
        status = SLOT_NOTCONV;
        rr = tt;
        break;
      }
      // replacement: r = b - A x, restart p = r
      ++repl;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * BS;
        r[k] = q[k];
        if (i < n) vec[i] = q[k];
      }
      rho = tt;
      rr = tt;
      __syncthreads();
      continue;
    }
    if (it >= S->max_iters) {
      status = SLOT_MAXIT;
      break;
    }
    const double beta = rr / rho;
    rho = rr;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      if (i < n) vec[i] = r[k] + beta * vec[i];
    }
    __syncthreads();
  }
  // write the state back (p persists in HBM between launches)
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int i = tid + k * BS;
    if (i < n) {
      S->x[i] = x[k];
      S->r[i] = r[k];
      if (USE_LDS) pg[i] = vec[i];
    }
  }
  if (tid == 0) {
    S->rho = rho;
    S->thr = thr;
    S->res2 = rr;
    S->iters = it;
    S->repl = repl;
    S->status = status;
  }
}

// ---------------------------------------------------------------------------
// host engine
// ---------------------------------------------------------------------------
constexpr int kMaxClasses = 8;
constexpr size_t kAlign = 256;

size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Request {
  uint64_t ticket;
  int64_t n, nnz;
  std::vector<int32_t> rowptr, col;
  std::vector<double> val, b;
  double tol;
  int64_t max_iters;
  size_t bytes;
  int cls;
};

struct Result {
  std::vector<double> x;
  mxs_solve_info info;
  bool done = false;
};

struct ClassCfg {
  int max_n;
  int block;  // threads per system
  int rpt;
  int slots;
  int base;   // first slot index
  bool lds;
};

struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(char* p, size_t s) {
    base = p;
    size = s;
    free_.clear();
    free_[0] = s;
    used = 0;
  }
  // first fit
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t noff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        used += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Slot {
  bool busy = false;
  uint64_t ticket = 0;
  size_t off = 0, bytes = 0;
  int64_t n = 0;
  double* x_dev = nullptr;
};

}  // namespace
}  // namespace mxs

struct mxs_batch {
  mxs_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  mxs::Arena arena;
  void* arena_mem = nullptr;
  mxs::SlotDesc* d_slots = nullptr;
  mxs::SlotDesc* h_slots = nullptr;    // pinned: uploads
  mxs::SlotDesc* h_status = nullptr;   // pinned: read-back of every step
  int nslots = 0;
  int K = 16;
  int nclasses = 0;
  mxs::ClassCfg cls[mxs::kMaxClasses];
  std::vector<mxs::Slot> slots;
  std::deque<mxs::Request> pending;
  std::unordered_map<uint64_t, mxs::Result> results;
  uint64_t next_ticket = 1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t branch[mxs::kMaxClasses] = {};  // capture-time fork streams
  hipEvent_t fork = nullptr, join[mxs::kMaxClasses] = {};
  char* up_stage = nullptr;    // pinned: request data on its way to the arena
  size_t up_bytes = 0;
  char* down_stage = nullptr;  // pinned: solutions on their way back
  size_t down_bytes = 0;
  bool launched = false;  // a step's graph is in flight / its status is fresh
  int64_t completed = 0;
  std::vector<uint64_t> newly_done;  // tickets retired since the last mxs_batch_completed
  uint64_t starve_ticket = 0;
  int64_t starve_steps = 0;
};

namespace mxs {
namespace {

size_t footprint(int64_t n, int64_t nnz) {
  return up((n + 1) * 4) + up(nnz * 4) + up(nnz * 8) + 4 * up(n * 8);
}

using BatchKernel = void (*)(SlotDesc*, int, int, int);

// (block, rows per thread) -> kernel; rows per thread in {1, 2, 4, 6, 8, 10, 12, 16}
constexpr int kRpt[] = {1, 2, 4, 6, 8, 10, 12, 16};

template <bool L>
BatchKernel pick(int block, int rpt) {
#define MXS_BK(B)                                          \
  if (block == B) {                                        \
    if (rpt <= 1) return k_batch_cg<B, 1, L>;              \
    if (rpt <= 2) return k_batch_cg<B, 2, L>;              \
    if (rpt <= 4) return k_batch_cg<B, 4, L>;              \
    if (rpt <= 6) return k_batch_cg<B, 6, L>;              \
    if (rpt <= 8) return k_batch_cg<B, 8, L>;              \
    if (rpt <= 10) return k_batch_cg<B, 10, L>;            \
    if (rpt <= 12) return k_batch_cg<B, 12, L>;            \
    return k_batch_cg<B, 16, L>;                           \
  }
  MXS_BK(128)
  MXS_BK(256)
  MXS_BK(512)
  MXS_BK(1024)
#undef MXS_BK
  return nullptr;
}

int rpt_for(int max_n, int block) {
  const int need = (max_n + block - 1) / block;
  for (int r : kRpt)
    if (r >= need) return r;
  return need;  // > 16: rejected by the caller
}

// LDS bytes of a class: row pointers, plus the gather vector when it fits
size_t class_lds(const ClassCfg& C) {
  return (C.lds ? (size_t)C.max_n * sizeof(double) : 0) + (size_t)(C.max_n + 1) * 4;
}

mxs_status build_graph(mxs_batch* B) {
  mxs_ctx* ctx = B->ctx;
  if (B->exec) {
    (void)hipGraphExecDestroy(B->exec);
    (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
  }
  // the class kernels are independent: each runs on its own branch of the
  // graph (fork from the main stream, join back before the status copy)
  MXS_HIP_TRY(ctx, hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
  (void)hipEventRecord(B->fork, B->stream);
  for (int c = 0; c < B->nclasses; ++c) {
    const ClassCfg& C = B->cls[c];
    if (C.slots == 0) continue;
    (void)hipStreamWaitEvent(B->branch[c], B->fork, 0);
    BatchKernel k = C.lds ? pick<true>(C.block, C.rpt) : pick<false>(C.block, C.rpt);
    hipLaunchKernelGGL(k, dim3(C.slots), dim3(C.block), class_lds(C), B->branch[c], B->d_slots,
                       C.base, B->K, C.max_n);
    (void)hipEventRecord(B->join[c], B->branch[c]);
    (void)hipStreamWaitEvent(B->stream, B->join[c], 0);
  }
  (void)hipMemcpyAsync(B->h_status, B->d_slots, sizeof(SlotDesc) * B->nslots,
                       hipMemcpyDeviceToHost, B->stream);
  hipError_t e = hipStreamEndCapture(B->stream, &B->graph);
  if (e != hipSuccess) return fail(ctx, MXS_HIP, "graph capture failed: %s", hipGetErrorString(e));
  MXS_HIP_TRY(ctx, hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
  return MXS_OK;
}

int class_of(const mxs_batch* B, int64_t n) {
  for (int c = 0; c < B->nclasses; ++c)
    if (n <= B->cls[c].max_n) return c;
  return -1;
}

bool validate_csr(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* col) {
  if (rp[0] != 0 || rp[n] != nnz) return false;
  for (int64_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return false;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      if (col[k] < 0 || col[k] >= n) return false;
      if (k > rp[i] && col[k] <= col[k - 1]) return false;
    }
  }
  return true;
}

}  // namespace
}  // namespace mxs

using namespace mxs;

extern "C" {

mxs_status mxs_batch_create(mxs_ctx* ctx, const mxs_batch_opts* opts, mxs_batch** out) {
  if (!ctx || !opts || !out || opts->budget_bytes < 4096 || opts->max_slots < 1)
    return MXS_INVALID_ARG;
  MXS_HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipDeviceProp_t prop;
  MXS_HIP_TRY(ctx, hipGetDeviceProperties(&prop, ctx->device));
  mxs_batch* B = new (std::nothrow) mxs_batch();
  if (!B) return MXS_OOM;
  B->ctx = ctx;
  B->K = opts->iters_per_step > 0 ? opts->iters_per_step : 16;
  // size classes
  int nc = opts->nclasses;
  int max_n[kMaxClasses], block[kMaxClasses], nsl[kMaxClasses];
  if (nc <= 0) {
    const int dn[4] = {1024, 2304, 4096, 10240}, db[4] = {256, 256, 512, 1024};
    nc = 4;
    for (int c = 0; c < nc; ++c) {
      max_n[c] = dn[c];
      block[c] = db[c];
      nsl[c] = 0;
    }
  } else {
    if (nc > kMaxClasses) {
      delete B;
      return fail(ctx, MXS_INVALID_ARG, "at most %d size classes", kMaxClasses);
    }
    for (int c = 0; c < nc; ++c) {
      max_n[c] = opts->class_max_n[c];
      block[c] = opts->class_block[c] > 0 ? opts->class_block[c] : 256;
      nsl[c] = opts->class_slots[c];
      if (max_n[c] <= 0 || (c > 0 && max_n[c] <= max_n[c - 1])) {
        delete B;
        return fail(ctx, MXS_INVALID_ARG, "class_max_n must be positive and increasing");
      }
    }
  }
  int assigned = 0, unassigned = 0, last_unassigned = -1;
  for (int c = 0; c < nc; ++c) {
    if (nsl[c] > 0) {
      assigned += nsl[c];
    } else {
      unassigned++;
      last_unassigned = c;
    }
  }
  int rest = opts->max_slots - assigned;
  if (rest < 0 || (unassigned && rest < unassigned)) {
    delete B;
    return fail(ctx, MXS_INVALID_ARG, "class_slots exceed max_slots");
  }
  int base = 0;
  for (int c = 0; c < nc; ++c) {
    ClassCfg& C = B->cls[c];
    C.max_n = max_n[c];
    C.block = block[c];
    if (C.block != 128 && C.block != 256 && C.block != 512 && C.block != 1024) {
      delete B;
      return fail(ctx, MXS_INVALID_ARG, "class_block must be 128, 256, 512 or 1024");
    }
    C.rpt = rpt_for(C.max_n, C.block);
    if (C.rpt > 16) {
      delete B;
      return fail(ctx, MXS_UNSUPPORTED, "class max n %d needs more than 16 rows per thread", C.max_n);
    }
    // classes without an explicit slot count share the rest evenly
    C.slots = nsl[c] > 0 ? nsl[c]
                         : rest / unassigned + (c == last_unassigned ? rest % unassigned : 0);
    C.base = base;
    // the gather vector lives in LDS when it fits beside the row pointers
    const size_t limit = (size_t)prop.sharedMemPerBlock - 1024;
    C.lds = true;
    if (class_lds(C) > limit) C.lds = false;
    if (class_lds(C) > limit) {
      delete B;
      return fail(ctx, MXS_UNSUPPORTED, "class max n %d: row pointers exceed the LDS", C.max_n);
    }
    for (int attempt = 0; attempt < 2; ++attempt) {
      const size_t lds = class_lds(C);
      if (lds <= 65536) break;
      BatchKernel k = C.lds ? pick<true>(C.block, C.rpt) : pick<false>(C.block, C.rpt);
      if (hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds) == hipSuccess)
        break;
      (void)hipGetLastError();
      C.lds = false;  // fall back to the gather vector in HBM
    }
    base += C.slots;
  }
  B->nclasses = nc;
  B->nslots = base;
  B->slots.resize(B->nslots);
  mxs_status st = MXS_OK;
  do {
    bool ok = hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&B->fork, hipEventDisableTiming) == hipSuccess;
    for (int c = 0; ok && c < nc; ++c)
      ok = hipStreamCreateWithFlags(&B->branch[c], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&B->join[c], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      st = fail(ctx, MXS_HIP, "stream or event creation failed");
      break;
    }
    B->up_bytes = std::min<size_t>(opts->budget_bytes, (size_t)256 << 20);
    B->down_bytes = (size_t)32 << 20;
    if (hipHostMalloc((void**)&B->up_stage, B->up_bytes, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&B->down_stage, B->down_bytes, hipHostMallocDefault) !=
            hipSuccess) {
      st = fail(ctx, MXS_OOM, "pinned staging buffers");
      break;
    }
    B->arena_mem = ctx->alloc.alloc(opts->budget_bytes);
    if (!B->arena_mem) {
      st = fail(ctx, MXS_OOM, "cannot allocate the %zu-byte batch arena", opts->budget_bytes);
      break;
    }
    B->arena.init((char*)B->arena_mem, opts->budget_bytes / kAlign * kAlign);
    B->d_slots = (SlotDesc*)ctx->alloc.alloc(sizeof(SlotDesc) * B->nslots);
    if (!B->d_slots || hipHostMalloc((void**)&B->h_slots, sizeof(SlotDesc) * B->nslots,
                                     hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&B->h_status, sizeof(SlotDesc) * B->nslots,
                      hipHostMallocDefault) != hipSuccess) {
      st = fail(ctx, MXS_OOM, "slot tables");
      break;
    }
    std::memset(B->h_slots, 0, sizeof(SlotDesc) * B->nslots);
    std::memset(B->h_status, 0, sizeof(SlotDesc) * B->nslots);
    if (hipMemcpyAsync(B->d_slots, B->h_slots, sizeof(SlotDesc) * B->nslots,
                       hipMemcpyHostToDevice, B->stream) != hipSuccess ||
        hipStreamSynchronize(B->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "slot table upload failed");
      break;
    }
    st = build_graph(B);
  } while (0);
  if (st) {
    mxs_batch_destroy(B);
    return st;
  }
  *out = B;
  return MXS_OK;
}

mxs_status mxs_batch_destroy(mxs_batch* B) {
  if (!B) return MXS_OK;
  if (B->stream) (void)hipStreamSynchronize(B->stream);
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->ctx) {
    B->ctx->alloc.release(B->arena_mem);
    B->ctx->alloc.release(B->d_slots);
  }
  if (B->h_slots) (void)hipHostFree(B->h_slots);
  if (B->h_status) (void)hipHostFree(B->h_status);
  if (B->up_stage) (void)hipHostFree(B->up_stage);
  if (B->down_stage) (void)hipHostFree(B->down_stage);
  for (int c = 0; c < mxs::kMaxClasses; ++c) {
    if (B->branch[c]) (void)hipStreamDestroy(B->branch[c]);
    if (B->join[c]) (void)hipEventDestroy(B->join[c]);
  }
  if (B->fork) (void)hipEventDestroy(B->fork);
  if (B->stream) (void)hipStreamDestroy(B->stream);
  delete B;
  return MXS_OK;
}

mxs_status mxs_batch_submit(mxs_batch* B, int64_t n, int64_t nnz, const int32_t* rowptr,
                            const int32_t* col, const double* val, const double* b,
                            double rel_tol, int64_t max_iters, uint64_t* ticket) {
  if (!B || !ticket || n < 1 || nnz < 0 || !rowptr || !b || (nnz && (!col || !val)))
    return MXS_INVALID_ARG;
  mxs_ctx* ctx = B->ctx;
  if (n > INT32_MAX || nnz > INT32_MAX) return fail(ctx, MXS_UNSUPPORTED, "sizes beyond int32");
  const int c = class_of(B, n);
  if (c < 0)
    return fail(ctx, MXS_UNSUPPORTED, "n = %lld exceeds the largest size class",
                (long long)n);
  const size_t bytes = footprint(n, nnz);
  if (bytes > B->arena.size)
    return fail(ctx, MXS_BUDGET, "request needs %zu bytes, budget is %zu", bytes, B->arena.size);
  if (!validate_csr(n, nnz, rowptr, col))
    return fail(ctx, MXS_INVALID_MATRIX, "submitted CSR failed validation");
  Request R;
  R.ticket = B->next_ticket++;
  R.n = n;
  R.nnz = nnz;
  R.rowptr.assign(rowptr, rowptr + n + 1);
  R.col.assign(col, col + nnz);
  R.val.assign(val, val + nnz);
  R.b.assign(b, b + n);
  R.tol = rel_tol;
  R.max_iters = max_iters > 0 ? max_iters : 20000;
  R.bytes = bytes;
  R.cls = c;
  B->pending.push_back(std::move(R));
  *ticket = B->pending.back().ticket;
  return MXS_OK;
}

mxs_status mxs_batch_step(mxs_batch* B, mxs_batch_stats* stats) {
  if (!B) return MXS_INVALID_ARG;
  mxs_ctx* ctx = B->ctx;
  MXS_HIP_TRY(ctx, hipSetDevice(ctx->device));
  // 1. retire slots the last step finished (h_status is that step's copy)
  std::vector<int> retired;
  std::vector<size_t> stage_off;
  if (B->launched) {
    size_t down = 0;
    for (int i = 0; i < B->nslots; ++i) {
      Slot& s = B->slots[i];
      if (!s.busy) continue;
      const SlotDesc& d = B->h_status[i];
      if (d.status < SLOT_CONVERGED) continue;
      const size_t xb = up(s.n * sizeof(double));
      if (down + xb > B->down_bytes) break;  // the rest retires next step
      Result& R = B->results[s.ticket];
      MXS_HIP_TRY(ctx, hipMemcpyAsync(B->down_stage + down, s.x_dev, s.n * sizeof(double),
                                      hipMemcpyDeviceToHost, B->stream));
      stage_off.push_back(down);
      down += xb;
      std::memset(&R.info, 0, sizeof(R.info));
      R.info.iters = d.iters;
      R.info.replacements = d.repl;
      const double nb = d.tol > 0 ? d.thr / d.tol : 0.0;
      R.info.relres_recurrence = nb > 0 ? sqrt(d.res2) / nb : 0.0;
      R.info.relres_true = d.status == SLOT_CONVERGED || d.status == SLOT_NOTCONV
                               ? (nb > 0 ? sqrt(d.res2) / nb : 0.0)
                               : -1.0;
      R.info.status = d.status == SLOT_CONVERGED   ? MXS_OK
                      : d.status == SLOT_BREAKDOWN ? MXS_BREAKDOWN
                      : d.status == SLOT_NONFINITE ? MXS_NONFINITE
                                                   : MXS_NOT_CONVERGED;
      retired.push_back(i);
    }
    MXS_HIP_TRY(ctx, hipStreamSynchronize(B->stream));
    for (size_t q = 0; q < retired.size(); ++q) {
      const int i = retired[q];
      Slot& s = B->slots[i];
      Result& R = B->results[s.ticket];
      const double* xs = (const double*)(B->down_stage + stage_off[q]);
      R.x.assign(xs, xs + s.n);
      R.done = true;
      B->newly_done.push_back(s.ticket);
      B->arena.release(s.off, s.bytes);
      s.busy = false;
      std::memset(&B->h_slots[i], 0, sizeof(SlotDesc));
      MXS_HIP_TRY(ctx, hipMemcpyAsync(&B->d_slots[i], &B->h_slots[i], sizeof(SlotDesc),
                                      hipMemcpyHostToDevice, B->stream));
      B->completed++;
    }
  }
  // 2. admit in FIFO order, first fit: a request that does not fit (no free
  // slot in its class, or no arena gap) is passed over by later ones,
  // unless it has been the oldest waiting request for more than 64 steps;
  // then nothing behind it is admitted until it fits (starvation guard)
  auto find_free = [&](int c) {
    const ClassCfg& C = B->cls[c];
    for (int i = C.base; i < C.base + C.slots; ++i)
      if (!B->slots[i].busy) return i;
    return -1;
  };
  std::vector<Request> uploading;
  size_t staged = 0;
  size_t idx = 0;
  while (idx < B->pending.size()) {
    Request& R = B->pending[idx];
    const bool via_stage = R.bytes <= B->up_bytes;
    if (via_stage && staged + R.bytes > B->up_bytes) break;  // stage full: next step
    const int si = find_free(R.cls);
    size_t off = 0;
    if (si < 0 || !B->arena.alloc(R.bytes, &off)) {
      if (idx == 0) {
        if (R.ticket == B->starve_ticket) {
          B->starve_steps++;
        } else {
          B->starve_ticket = R.ticket;
          B->starve_steps = 1;
        }
        if (B->starve_steps > 64) break;
      }
      ++idx;
      continue;
    }
    char* p = B->arena.base + off;
    const int64_t n = R.n, nnz = R.nnz;
    int32_t* d_rp = (int32_t*)p;
    int32_t* d_col = (int32_t*)(p + up((n + 1) * 4));
    double* d_val = (double*)(p + up((n + 1) * 4) + up(nnz * 4));
    double* d_b = (double*)((char*)d_val + up(nnz * 8));
    double* d_x = (double*)((char*)d_b + up(n * 8));
    double* d_r = (double*)((char*)d_x + up(n * 8));
    double* d_p = (double*)((char*)d_r + up(n * 8));
    // the matrix and b are packed in the pinned stage in their arena layout
    // and travel in one copy
    const size_t in_bytes = (size_t)((char*)d_x - p);
    if (via_stage) {
      char* sp = B->up_stage + staged;
      std::memcpy(sp, R.rowptr.data(), (n + 1) * 4);
      std::memcpy(sp + ((char*)d_col - p), R.col.data(), nnz * 4);
      std::memcpy(sp + ((char*)d_val - p), R.val.data(), nnz * 8);
      std::memcpy(sp + ((char*)d_b - p), R.b.data(), n * 8);
      MXS_HIP_TRY(ctx, hipMemcpyAsync(p, sp, in_bytes, hipMemcpyHostToDevice, B->stream));
      staged += up(in_bytes);
    } else {  // larger than the stage: copy from the request's own buffers
      MXS_HIP_TRY(ctx, hipMemcpyAsync(d_rp, R.rowptr.data(), (n + 1) * 4,
                                      hipMemcpyHostToDevice, B->stream));
      if (nnz) {
        MXS_HIP_TRY(ctx, hipMemcpyAsync(d_col, R.col.data(), nnz * 4, hipMemcpyHostToDevice,
                                        B->stream));
        MXS_HIP_TRY(ctx, hipMemcpyAsync(d_val, R.val.data(), nnz * 8, hipMemcpyHostToDevice,
                                        B->stream));
      }
      MXS_HIP_TRY(ctx, hipMemcpyAsync(d_b, R.b.data(), n * 8, hipMemcpyHostToDevice,
                                      B->stream));
    }
    SlotDesc& d = B->h_slots[si];
    std::memset(&d, 0, sizeof(d));
    d.rowptr = d_rp;
    d.col = d_col;
    d.val = d_val;
    d.b = d_b;
    d.x = d_x;
    d.r = d_r;
    d.p = d_p;
    d.tol = R.tol;
    d.n = (int32_t)n;
    d.nnz = (int32_t)nnz;
    d.max_iters = (int32_t)std::min<int64_t>(R.max_iters, INT32_MAX);
    d.active = 1;
    d.status = SLOT_NEW;
    MXS_HIP_TRY(ctx, hipMemcpyAsync(&B->d_slots[si], &d, sizeof(SlotDesc), hipMemcpyHostToDevice,
                                    B->stream));
    Slot& s = B->slots[si];
    s.busy = true;
    s.ticket = R.ticket;
    s.off = off;
    s.bytes = R.bytes;
    s.n = n;
    s.x_dev = d_x;
    // the host copies in R must stay alive until the uploads completed:
    // keep them until the synchronisation below
    uploading.push_back(std::move(R));
    B->pending.erase(B->pending.begin() + idx);
  }
  if (!uploading.empty()) {
    MXS_HIP_TRY(ctx, hipStreamSynchronize(B->stream));
    uploading.clear();
  }
  // 3. run K iterations of every active slot and read the statuses back
  int active = 0;
  for (const Slot& s : B->slots) active += s.busy ? 1 : 0;
  if (active > 0) {
    MXS_HIP_TRY(ctx, hipGraphLaunch(B->exec, B->stream));
    MXS_HIP_TRY(ctx, hipStreamSynchronize(B->stream));
    B->launched = true;
  } else {
    B->launched = false;
  }
  if (stats) {
    stats->active = active;
    stats->pending = (int32_t)B->pending.size();
    stats->completed = B->completed;
    stats->arena_used = (int64_t)B->arena.used;
    stats->arena_size = (int64_t)B->arena.size;
    stats->slots = B->nslots;
  }
  return MXS_OK;
}

mxs_status mxs_batch_poll(mxs_batch* B, uint64_t ticket, double* x_host, mxs_solve_info* info) {
  if (!B) return MXS_INVALID_ARG;
  auto it = B->results.find(ticket);
  if (it == B->results.end() || !it->second.done) {
    if (ticket == 0 || ticket >= B->next_ticket) return MXS_INVALID_ARG;
    return MXS_PENDING;
  }
  if (x_host) std::memcpy(x_host, it->second.x.data(), it->second.x.size() * sizeof(double));
  if (info) *info = it->second.info;
  const mxs_status st = it->second.info.status;
  B->results.erase(it);
  return st;
}

mxs_status mxs_batch_completed(mxs_batch* B, uint64_t* tickets, int64_t cap, int64_t* count) {
  if (!B || !count || (cap > 0 && !tickets)) return MXS_INVALID_ARG;
  const int64_t k = std::min<int64_t>(cap, (int64_t)B->newly_done.size());
  for (int64_t i = 0; i < k; ++i) tickets[i] = B->newly_done[i];
  B->newly_done.erase(B->newly_done.begin(), B->newly_done.begin() + k);
  *count = k;
  return MXS_OK;
}

mxs_status mxs_batch_config(const mxs_batch* B, int32_t cls, int32_t* max_n, int32_t* block,
                            int32_t* rows_per_thread, int32_t* slots, int32_t* uses_lds) {
  if (!B || cls < 0 || cls >= B->nclasses) return MXS_INVALID_ARG;
  const ClassCfg& C = B->cls[cls];
  if (max_n) *max_n = C.max_n;
  if (block) *block = C.block;
  if (rows_per_thread) *rows_per_thread = C.rpt;
  if (slots) *slots = C.slots;
  if (uses_lds) *uses_lds = C.lds ? 1 : 0;
  return MXS_OK;
}

}  // extern "C"
