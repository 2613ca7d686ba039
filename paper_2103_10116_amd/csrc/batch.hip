// batch.hip -- batched persistent CG and the continuous-batching engine.
//
// Many independent SPD systems are solved by one kernel per size class:
// work-group i owns slot i, keeps the slot's row pointers and the search
// direction p in LDS (the gathers of its SpMV never leave the CU) and x, r
// and q of the rows it owns in registers, and runs up to K CG iterations per
// launch (the CG of Saad 2003, ch. 6, with the true-residual check and up to
// three residual replacements).  The state is written back to HBM at the end
// of a launch, so launches repeat until every slot has finished.  A system's
// arithmetic depends only on its own data and on the threads-per-system of
// its size class (a function of n), never on the other slots, so a result
// is bitwise the same alone and in any mix.
//
// Host/device traffic per step is three transfers whatever the number of
// requests: the host-written descriptor table goes up in one copy, the
// kernel-written state table comes back in one copy, and a newly admitted
// slot's work-group pulls the request's packed inputs (CSR arrays and b,
// packed once at submit into pinned host memory in the slot's arena
// layout) into the arena on its first launch.  A finished slot's
// work-group writes x straight into the slot's pinned host output.
//
// The host engine owns a device arena of `budget_bytes` managed first-fit,
// the slot tables, a FIFO of submitted requests and one hipGraph per step
// (one kernel per class, on parallel branches, then the state read-back).
// Each mxs_batch_step admits waiting requests whose footprint fits the
// arena and whose class has a free slot, launches the graph, waits for it,
// and retires the slots that finished.
#include <sched.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
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

// written by the host, uploaded before every launch
struct SlotDesc {
  int32_t* rowptr;     // arena: rowptr | col | val | b | x | r | p
  int32_t* col;
  double* val;
  double* b;
  double* x;
  double* r;
  double* p;
  const uint4* src;    // pinned host: rowptr | col | val | b in the same layout
  double* xout;        // pinned host: x of a finished system
  double tol;
  int32_t n, nnz;
  int32_t max_iters;
  int32_t active;
  uint32_t gen;        // admission number; the state's gen differs until the first launch
  int32_t in_words;    // 16-byte words from src to rowptr
  float* v32;          // arena, refinement mode: the values rounded to FP32
  int32_t mode;        // 0: FP64 CG; 1: FP32-storage CG inside FP64 refinement
  float inner_tol;     // refinement mode: inner relative tolerance
  // a single solve (FP64 CG): x holds x0, the first launch forms
  // r0 = b - A x0 and stops at max(tol * base, abs_tol), base = ||r0|| when
  // base_r0, else ||b||; b = 0 gives x = 0.  Otherwise x0 = 0 and the
  // threshold is tol * ||b||.
  int32_t x0_given, base_r0;
  double abs_tol;
};

// written by the kernel, read back after every launch
struct SlotState {
  double rho, thr, res2;
  int32_t iters, status, repl;
  uint32_t gen;
  // refinement mode: inner threshold, norm of the residual being refined,
  // inner iterations of the current inner solve, phase, outer steps
  double ithr, rn;
  int32_t inner, phase, outer, pad;
  double base;  // FP64 CG: the norm the threshold is relative to
};

enum : int32_t { PH_OUTER = 0, PH_INNER = 1 };
constexpr int kIrOuterMax = 50;
constexpr int kIrInnerMax = 20000;

template <int BS>
__device__ __forceinline__ double bsum(double v, double* red) {
  v = wave_total(v);
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int i = 1; i < BS / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

// bsum with one barrier: the caller alternates two `red` buffers between
// consecutive calls, so a call's writes cannot meet the previous call's
// reads (a barrier of the call in between orders them).  The barrier also
// orders every read of shared memory before it against writes after it.
template <int BS>
__device__ __forceinline__ double bsum1(double v, double* red) {
  v = wave_total(v);
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int i = 1; i < BS / 64; ++i) s += red[i];
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
// entry index is outermost so that the loads of a group of LG rows are in
// flight together (LG = RPT up to 8 rows, else half of them, to stay within
// the 128 registers of a 1024-thread work-group); the row bounds are
// re-read from LDS rather than held in registers.
template <int BS, int RPT, typename V = double>
__device__ __forceinline__ void rows_times(const int32_t* __restrict__ rpl,
                                           const int32_t* __restrict__ col,
                                           const V* __restrict__ val,
                                           const V* __restrict__ vec, int n, int maxlen,
                                           V (&q)[RPT]) {
  constexpr int LG = RPT <= 8 ? RPT : (RPT + 1) / 2;
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < RPT; ++k) q[k] = V(0);
  for (int j = 0; j < maxlen; ++j) {
#pragma unroll
    for (int g = 0; g < RPT; g += LG) {
      int32_t c[LG];
      V v[LG];
      bool h[LG];
      // every load of the group issued together: a slot past its row's end
      // (or past n) reads entry 0 of the system, whose product is dropped
#pragma unroll
      for (int u = 0; u < LG; ++u) {
        const int i = tid + (g + u) * BS;
        const bool in = g + u < RPT && i < n;
        const int32_t e = in ? rpl[i] + j : 0;
        h[u] = in && e < rpl[i + 1];
        const int32_t es = h[u] ? e : 0;
        c[u] = col[es];
        v[u] = val[es];
      }
#pragma unroll
      for (int u = 0; u < LG; ++u) {
        const V gv = vec[c[u]];
        if (h[u]) q[g + u] += v[u] * gv;
      }
    }
  }
}

// Refinement mode (a slot's share of the mixed-precision scheme of the
// single-system solver): outer steps r = b - A x with the FP64 values and
// x += ||r|| d, inner CG in FP32 on the FP32-rounded values for
// A d = r / ||r|| to inner_tol, reductions accumulated in FP64 and rounded
// once to FP32.  An outer step and an inner iteration each take one of the
// launch's K units.  x lives in registers (FP64), the inner r and d in
// registers (FP32); the gather vector (x for an outer step, the inner p
// otherwise) is the same LDS region read as FP64 or FP32.
template <int BS, int RPT, bool USE_LDS>
__device__ __forceinline__ void ir_body(const SlotDesc& D, SlotState* S, int K, bool fresh,
                                        const int32_t* rpl, int maxlen, double* dyn,
                                        double* red) {
  const int n = D.n;
  const int tid = threadIdx.x;
  const int32_t* __restrict__ col = D.col;
  const double* __restrict__ val = D.val;
  const float* __restrict__ v32 = D.v32;
  const double* __restrict__ b = D.b;
  double* __restrict__ vec64 = USE_LDS ? dyn : D.x;
  float* __restrict__ vec32 = USE_LDS ? (float*)dyn : (float*)D.p;
  float* __restrict__ rin_g = (float*)D.r;
  float* __restrict__ d_g = (float*)D.r + n;
  double x[RPT];
  float d[RPT], rin[RPT], q[RPT];
  double thr, rn, res2;
  float rho, ithr;
  int status = SLOT_RUN, phase, inner, outer, tot;
  if (fresh) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      x[k] = 0.0;
      d[k] = 0.0f;
      rin[k] = 0.0f;
      const double bi = i < n ? b[i] : 0.0;
      acc += bi * bi;
    }
    res2 = bsum<BS>(acc, red);
    thr = D.tol * sqrt(res2);
    rn = 0.0;
    rho = 0.0f;
    ithr = 0.0f;
    phase = PH_OUTER;
    inner = outer = tot = 0;
    if (!isfinite(res2)) status = SLOT_NONFINITE;
    if (res2 == 0.0) status = SLOT_CONVERGED;  // b = 0: x = 0
  } else {
    thr = S->thr;
    rn = S->rn;
    res2 = S->res2;
    rho = (float)S->rho;
    ithr = (float)S->ithr;
    phase = S->phase;
    inner = S->inner;
    outer = S->outer;
    tot = S->iters;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      x[k] = i < n ? D.x[i] : 0.0;
      d[k] = i < n && phase == PH_INNER ? d_g[i] : 0.0f;
      rin[k] = i < n && phase == PH_INNER ? rin_g[i] : 0.0f;
      if (USE_LDS && i < n && phase == PH_INNER) vec32[i] = ((const float*)D.p)[i];
    }
  }
  __syncthreads();
  for (int u = 0; u < K && status == SLOT_RUN; ++u) {
    if (phase == PH_OUTER) {
      // r = b - A x in FP64, x staged in the gather vector
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * BS;
        if (i < n) vec64[i] = x[k];
      }
      __syncthreads();
      double r64[RPT];
      rows_times<BS, RPT, double>(rpl, col, val, vec64, n, maxlen, r64);
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * BS;
        r64[k] = i < n ? b[i] - r64[k] : 0.0;
        acc += r64[k] * r64[k];
      }
      res2 = bsum<BS>(acc, red);  // its barriers end every read of vec64
      if (!isfinite(res2)) {
        status = SLOT_NONFINITE;
        break;
      }
      const double nr = sqrt(res2);
      if (nr <= thr) {
        status = SLOT_CONVERGED;
        break;
      }
      if (outer >= kIrOuterMax || tot >= D.max_iters) {
        status = SLOT_NOTCONV;
        break;
      }
      // inner solve of A d = r / ||r|| from d = 0: its r and p start as f
      rn = nr;
      double f2 = 0.0;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * BS;
        rin[k] = i < n ? (float)(r64[k] / nr) : 0.0f;
        d[k] = 0.0f;
        if (i < n) vec32[i] = rin[k];
        f2 += (double)rin[k] * (double)rin[k];
      }
      rho = (float)bsum<BS>(f2, red);
      ithr = D.inner_tol * sqrtf(rho);
      inner = 0;
      phase = PH_INNER;
      if (!(sqrtf(rho) > ithr)) {  // nothing to solve: the correction is zero
        outer++;
        phase = PH_OUTER;
      }
      continue;
    }
    // one inner FP32 CG iteration
    rows_times<BS, RPT, float>(rpl, col, v32, vec32, n, maxlen, q);
    double pq_acc = 0.0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      if (i < n) pq_acc += (double)vec32[i] * (double)q[k];
    }
    const float pq = (float)bsum<BS>(pq_acc, red);
    bool finish = false;
    if (!(pq > 0.0f)) {
      finish = true;  // breakdown: the correction so far is still usable
    } else {
      const float alpha = rho / pq;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * BS;
        if (i < n) d[k] = d[k] + alpha * vec32[i];
        rin[k] = rin[k] - alpha * q[k];
        acc += (double)rin[k] * (double)rin[k];
      }
      const float rho_new = (float)bsum<BS>(acc, red);
      ++inner;
      ++tot;
      if (!isfinite(rho_new)) {
        status = SLOT_NONFINITE;
        break;
      }
      if (sqrtf(rho_new) <= ithr || inner >= kIrInnerMax || tot >= D.max_iters) {
        finish = true;
      } else {
        const float beta = rho_new / rho;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int i = tid + k * BS;
          if (i < n) vec32[i] = rin[k] + beta * vec32[i];
        }
        rho = rho_new;
        __syncthreads();
      }
    }
    if (finish) {
#pragma unroll
      for (int k = 0; k < RPT; ++k) x[k] = x[k] + rn * (double)d[k];
      outer++;
      phase = PH_OUTER;
    }
  }
  if (status >= SLOT_CONVERGED) {
    double* __restrict__ xo = D.xout;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      if (i < n) xo[i] = x[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      if (i < n) {
        D.x[i] = x[k];
        if (phase == PH_INNER) {
          rin_g[i] = rin[k];
          d_g[i] = d[k];
          if (USE_LDS) ((float*)D.p)[i] = vec32[i];
        }
      }
    }
  }
  if (tid == 0) {
    S->rho = rho;
    S->thr = thr;
    S->res2 = res2;
    S->iters = tot;
    S->repl = 0;
    S->status = status;
    S->ithr = ithr;
    S->rn = rn;
    S->inner = inner;
    S->phase = phase;
    S->outer = outer;
    S->gen = D.gen;
  }
}

// One work-group per slot.  BS threads, RPT rows per thread (rows
// tid + k*BS).  LDS holds the slot's row pointers and, when USE_LDS, the
// gather vector (p, or x during the true-residual check); otherwise the
// slot's p array in HBM serves as the gather vector.  x, r and q of the
// thread's rows live in registers for the whole launch.
// The FP64 CG of one slot for K iterations (the kernel's mode 0), with the
// product q = A v supplied by `spmv`: streamed from the slot's arrays, or
// from registers for systems small enough to hold there.
template <int BS, int RPT, bool USE_LDS, typename F>
__device__ __forceinline__ void cg_body(const SlotDesc& D, SlotState* S, int K, bool fresh,
                                        double* __restrict__ vec, double* __restrict__ pg,
                                        double* red, F&& spmv) {
  const int n = D.n;
  const int tid = threadIdx.x;
  const double* __restrict__ b = D.b;
  // x stays in the slot's HBM vector instead of registers when a thread
  // owns 10 or more rows (1024-thread classes run at 128 registers a lane)
  constexpr bool XG = RPT >= 10;
  double* __restrict__ xg = D.x;
  // p of the thread's own rows is also kept in registers (pr), so that only
  // the product's gathers read the gather vector
  double x[XG ? 1 : RPT], r[RPT], q[RPT], pr[RPT];
  double rho, thr;
  int status = SLOT_RUN;
  int it = 0, repl = 0;
  double base = 0.0;
  if (fresh && D.x0_given) {
    // r0 = b - A x0 (x0 staged in the gather vector), ||b|| and ||r0||
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      const double xi = i < n ? D.x[i] : 0.0;
      if constexpr (!XG) x[k] = xi;
      if (i < n) vec[i] = xi;
    }
    __syncthreads();
    spmv(vec, q);
    double bb = 0.0, acc = 0.0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      const double bi = i < n ? b[i] : 0.0;
      r[k] = i < n ? bi - q[k] : 0.0;
      bb += bi * bi;
      acc += r[k] * r[k];
    }
    const double nb2 = bsum<BS>(bb, red);  // its barriers end every read of vec
    rho = bsum<BS>(acc, red);
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      pr[k] = r[k];
      if (i < n) vec[i] = r[k];
    }
    base = D.base_r0 ? sqrt(rho) : sqrt(nb2);
    thr = fmax(D.tol * base, D.abs_tol);
    if (!isfinite(nb2) || !isfinite(rho)) {
      status = SLOT_NONFINITE;
    } else if (nb2 == 0.0) {
      // b = 0: the solution is x = 0
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * BS;
        if constexpr (XG) {
          if (i < n) xg[i] = 0.0;
        } else {
          x[k] = 0.0;
        }
      }
      rho = 0.0;
      status = SLOT_CONVERGED;
    } else if (sqrt(rho) <= thr) {
      status = SLOT_CONVERGED;  // x0 is the answer; rho is its true residual
    }
  } else if (fresh) {
    // x0 = 0: r = b, p = r, thr = tol * ||b||
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      if constexpr (XG) {
        if (i < n) xg[i] = 0.0;
      } else {
        x[k] = 0.0;
      }
      r[k] = i < n ? b[i] : 0.0;
      pr[k] = r[k];
      if (i < n) vec[i] = r[k];
      acc += r[k] * r[k];
    }
    rho = bsum<BS>(acc, red);
    base = sqrt(rho);
    thr = D.tol * base;
    if (!isfinite(rho)) status = SLOT_NONFINITE;
    if (rho == 0.0) status = SLOT_CONVERGED;  // b = 0: x = 0
  } else {
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      if constexpr (!XG) x[k] = i < n ? D.x[i] : 0.0;
      r[k] = i < n ? D.r[i] : 0.0;
      pr[k] = i < n ? pg[i] : 0.0;
      if (USE_LDS && i < n) vec[i] = pr[k];
    }
    rho = S->rho;
    thr = S->thr;
    it = S->iters;
    repl = S->repl;
    base = S->base;
  }
  __syncthreads();
  double rr = rho;
  for (int s = 0; s < K && status == SLOT_RUN; ++s) {
    spmv(vec, q);
    double pq = 0.0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      pq += pr[k] * q[k];
    }
    pq = bsum1<BS>(pq, red + BS / 64);
    if (!(pq > 0.0)) {
      status = isfinite(pq) ? SLOT_BREAKDOWN : SLOT_NONFINITE;
      break;
    }
    const double alpha = rho / pq;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      if constexpr (XG) {
        if (i < n) xg[i] += alpha * pr[k];
      } else {
        x[k] += alpha * pr[k];
      }
      r[k] -= alpha * q[k];
      acc += r[k] * r[k];
    }
    rr = bsum1<BS>(acc, red + 2 * (BS / 64));
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
        if (i < n) vec[i] = XG ? xg[i] : x[XG ? 0 : k];
      }
      __syncthreads();
      spmv(vec, q);
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
        pr[k] = q[k];
        if (i < n) vec[i] = q[k];
      }
      rho = tt;
      rr = tt;
      __syncthreads();
      continue;
    }
    if (it >= D.max_iters) {
      status = SLOT_MAXIT;
      break;
    }
    const double beta = rr / rho;
    rho = rr;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      pr[k] = r[k] + beta * pr[k];
      if (i < n) vec[i] = pr[k];
    }
    __syncthreads();
  }
  if (status >= SLOT_CONVERGED) {
    // finished: x goes straight to the slot's pinned host output
    double* __restrict__ xo = D.xout;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      if (i < n) xo[i] = XG ? xg[i] : x[XG ? 0 : k];
    }
  } else {
    // p persists in HBM between launches
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      if (i < n) {
        if constexpr (!XG) D.x[i] = x[k];
        D.r[i] = r[k];
        if (USE_LDS) pg[i] = pr[k];
      }
    }
  }
  if (tid == 0) {
    S->rho = rho;
    S->thr = thr;
    S->res2 = rr;
    S->iters = it;
    S->repl = repl;
    S->status = status;
    S->base = base;
    S->gen = D.gen;
  }
}

template <int BS, int RPT, bool USE_LDS, int MODE>
__global__ __launch_bounds__(BS) void k_batch_cg(const SlotDesc* __restrict__ desc,
                                                 SlotState* __restrict__ state, int base, int K,
                                                 int vec_cap) {
  extern __shared__ double dyn[];
  // three reduction buffers: bsum's, and the two that the CG loop's
  // one-barrier reductions alternate
  __shared__ double red[3 * (BS / 64)];
  __shared__ int ired[BS / 64];
  const SlotDesc& D = desc[base + blockIdx.x];
  SlotState* S = state + base + blockIdx.x;
  if (!D.active || D.mode != MODE) return;
  const bool fresh = S->gen != D.gen;
  if (!fresh && S->status >= SLOT_CONVERGED) return;
  const int n = D.n;
  const int tid = threadIdx.x;
  if (fresh) {
    // first launch: pull the packed inputs from pinned host memory
    const uint4* __restrict__ src = D.src;
    uint4* __restrict__ dst = (uint4*)D.rowptr;
    const int words = D.in_words;
    int w0 = tid;
    for (; w0 + 3 * BS < words; w0 += 4 * BS) {  // four 16-byte loads in flight
      const uint4 v0 = src[w0], v1 = src[w0 + BS], v2 = src[w0 + 2 * BS], v3 = src[w0 + 3 * BS];
      dst[w0] = v0;
      dst[w0 + BS] = v1;
      dst[w0 + 2 * BS] = v2;
      dst[w0 + 3 * BS] = v3;
    }
    for (; w0 < words; w0 += BS) dst[w0] = src[w0];
    __threadfence_block();
    __syncthreads();
    if (MODE == 1) {
      // refinement mode: the FP32 copy of the values, rounded to nearest
      const double* __restrict__ v = D.val;
      float* __restrict__ w = D.v32;
      for (int k = tid; k < D.nnz; k += BS) w[k] = (float)v[k];
      __threadfence_block();
      __syncthreads();
    }
  }
  const int32_t* __restrict__ rp = D.rowptr;
  const int32_t* __restrict__ col = D.col;
  const double* __restrict__ val = D.val;
  const double* __restrict__ b = D.b;
  double* __restrict__ pg = D.p;
  double* __restrict__ vec = USE_LDS ? dyn : pg;
  int32_t* rpl = (int32_t*)(dyn + (USE_LDS ? vec_cap : 0));
  int mylen = 0;
  for (int i = tid; i <= n; i += BS) rpl[i] = rp[i];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int i = tid + k * BS;
    if (i < n) mylen = max(mylen, rpl[i + 1] - rpl[i]);
  }
  const int maxlen = bmax<BS>(mylen, ired);
  if (MODE == 1) {
    ir_body<BS, RPT, USE_LDS>(D, S, K, fresh, rpl, maxlen, dyn, red);
    return;
  }
  // matrices small enough for registers (at most 24 entries a thread, 20 at
  // 1024 threads, whose lanes have 128 registers; a row's entries at most
  // that / RPT) are loaded once per launch and every product of the launch
  // reads them there; the rest stream theirs
  constexpr int ML = USE_LDS && RPT <= 4 ? (BS == 1024 ? 20 : 24) / RPT : 0;
  if constexpr (ML > 0) {
    if (maxlen <= ML) {
      int32_t cr[RPT * ML];
      double vr[RPT * ML];
      uint32_t hm = 0;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * BS;
        const int32_t a = i < n ? rpl[i] : 0, e = i < n ? rpl[i + 1] : 0;
#pragma unroll
        for (int j = 0; j < ML; ++j) {
          const bool h = a + j < e;
          const int32_t es = h ? a + j : 0;
          cr[k * ML + j] = col[es];
          vr[k * ML + j] = val[es];
          hm |= (h ? 1u : 0u) << (k * ML + j);
        }
      }
      auto spmv_reg = [&](const double* __restrict__ v, double (&q)[RPT]) {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < ML; ++j) {
            const double g = v[cr[k * ML + j]];
            if ((hm >> (k * ML + j)) & 1u) acc += vr[k * ML + j] * g;
          }
          q[k] = acc;
        }
      };
      cg_body<BS, RPT, USE_LDS>(D, S, K, fresh, vec, pg, red, spmv_reg);
      return;
    }
  }
  auto spmv_mem = [&](const double* __restrict__ v, double (&q)[RPT]) {
    rows_times<BS, RPT>(rpl, col, val, v, n, maxlen, q);
  };
  cg_body<BS, RPT, USE_LDS>(D, S, K, fresh, vec, pg, red, spmv_mem);
}

// ---------------------------------------------------------------------------
// host engine
// ---------------------------------------------------------------------------
constexpr int kMaxClasses = 8;
constexpr size_t kAlign = 256;

size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// arena layout of one system: rowptr | col | val | b | x | r | p, plus the
// FP32 values in refinement mode (there r holds the inner r and d, p the
// inner p, all FP32)
struct Layout {
  size_t col, val, b, x, r, p, v32, total;
};

Layout layout(int64_t n, int64_t nnz, int mode) {
  Layout L;
  L.col = up((n + 1) * 4);
  L.val = L.col + up(nnz * 4);
  L.b = L.val + up(nnz * 8);
  L.x = L.b + up(n * 8);
  L.r = L.x + up(n * 8);
  L.p = L.r + up(n * 8);
  L.v32 = L.p + up(n * 8);
  // (at least one FP32 value: the SpMV's loads of a system without entries
  // read entry 0, which must lie inside the system's piece)
  L.total = L.v32 + (mode == 1 ? up(std::max<int64_t>(nnz, 1) * 4) : 0);
  return L;
}

// first-fit allocator over [0, size)
struct Arena {
  size_t size = 0, used = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(size_t s) {
    size = s;
    free_.clear();
    if (s) free_[0] = s;
    used = 0;
  }
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

struct Request {
  uint64_t ticket;
  int64_t n, nnz;
  double tol;
  int64_t max_iters;
  size_t bytes;       // arena footprint
  size_t in_bytes;    // packed inputs (rowptr | col | val | b)
  int cls;
  int mode;
  float inner_tol;
  bool packed = false;   // inputs packed in the pinned input pool at in_off
  size_t in_off = 0;
  // copies of the inputs while the pinned pool had no room at submit
  std::vector<int32_t> rowptr, col;
  std::vector<double> val, b;
};

struct Result {
  std::unique_ptr<double[]> x;  // n doubles, filled at retirement
  int64_t n = 0;
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

struct Slot {
  bool busy = false;
  bool holds_input = false;  // its packed inputs are still in the pinned pool
  uint64_t ticket = 0;
  size_t off = 0, bytes = 0;
  size_t in_off = 0, in_bytes = 0;
  int64_t n = 0;
};

}  // namespace
}  // namespace mxs

struct mxs_batch {
  mxs_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  mxs::Arena arena;                    // device memory
  char* arena_mem = nullptr;
  mxs::Arena inpool;                   // pinned host memory for packed inputs
  char* in_mem = nullptr;              // host address
  char* in_dev = nullptr;              // the same memory as the device sees it
  double* xout_mem = nullptr;          // pinned: per-slot output regions (host address)
  double* xout_dev = nullptr;
  std::vector<size_t> xout_off;        // per slot, in doubles
  mxs::SlotDesc* d_desc = nullptr;
  mxs::SlotDesc* h_desc = nullptr;     // pinned
  mxs::SlotState* d_state = nullptr;
  mxs::SlotState* h_state = nullptr;   // pinned: read back by every step
  bool desc_dirty = true;
  bool in_flight = false;  // a launched step not yet finished
  int flight_active = 0;   // resident systems of the launched step
  uint32_t gen = 0;
  int nslots = 0;
  int K = 16;
  int nclasses = 0;
  mxs::ClassCfg cls[mxs::kMaxClasses];
  std::vector<mxs::Slot> slots;
  // free slots of each class, the lowest index on top
  std::vector<int> free_slots[mxs::kMaxClasses];
  std::deque<mxs::Request> pending;
  std::unordered_map<uint64_t, mxs::Result> results;
  uint64_t next_ticket = 1;
  hipGraph_t graph[4] = {};       // by mask of resident modes
  hipGraphExec_t exec[4] = {};
  hipStream_t branch[mxs::kMaxClasses] = {};  // capture-time fork streams
  hipEvent_t fork = nullptr, join[mxs::kMaxClasses] = {};
  int64_t completed = 0;
  std::vector<uint64_t> newly_done;  // tickets retired since the last mxs_batch_completed
  uint64_t starve_ticket = 0;
  int64_t starve_steps = 0;
  // guards the queue, the pools, the slots and the results, so that one
  // thread may submit while another steps; held neither while inputs are
  // validated and packed nor while a step is waited for
  std::mutex mu;
};

namespace mxs {
namespace {

using BatchKernel = void (*)(const SlotDesc*, SlotState*, int, int, int);

// (block, rows per thread) -> kernel; rows per thread in {1, 2, 4, 6, 8, 10, 12, 16}
constexpr int kRpt[] = {1, 2, 4, 6, 8, 10, 12, 16};

template <bool L, int M>
BatchKernel pick_m(int block, int rpt) {
#define MXS_BK(B)                                          \
  if (block == B) {                                        \
    if (rpt <= 1) return k_batch_cg<B, 1, L, M>;           \
    if (rpt <= 2) return k_batch_cg<B, 2, L, M>;           \
    if (rpt <= 4) return k_batch_cg<B, 4, L, M>;           \
    if (rpt <= 6) return k_batch_cg<B, 6, L, M>;           \
    if (rpt <= 8) return k_batch_cg<B, 8, L, M>;           \
    if (rpt <= 10) return k_batch_cg<B, 10, L, M>;         \
    if (rpt <= 12) return k_batch_cg<B, 12, L, M>;         \
    return k_batch_cg<B, 16, L, M>;                        \
  }
  MXS_BK(128)
  MXS_BK(256)
  MXS_BK(512)
  MXS_BK(1024)
#undef MXS_BK
  return nullptr;
}

BatchKernel pick(bool lds, int mode, int block, int rpt) {
  if (mode == 0) return lds ? pick_m<true, 0>(block, rpt) : pick_m<false, 0>(block, rpt);
  return lds ? pick_m<true, 1>(block, rpt) : pick_m<false, 1>(block, rpt);
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

// One graph per set of resident modes (bit 0: FP64 CG, bit 1: refinement):
// the class kernels are independent, so each class runs on its own branch
// (fork from the main stream, join back before the state copy), with the
// kernel of each present mode in turn.
mxs_status build_graph(mxs_batch* B, int mask) {
  mxs_ctx* ctx = B->ctx;
  MXS_HIP_TRY(ctx, hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
  (void)hipEventRecord(B->fork, B->stream);
  for (int c = 0; c < B->nclasses; ++c) {
    const ClassCfg& C = B->cls[c];
    if (C.slots == 0) continue;
    (void)hipStreamWaitEvent(B->branch[c], B->fork, 0);
    for (int mode = 0; mode < 2; ++mode) {
      if (!(mask >> mode & 1)) continue;
      BatchKernel k = pick(C.lds, mode, C.block, C.rpt);
      hipLaunchKernelGGL(k, dim3(C.slots), dim3(C.block), class_lds(C), B->branch[c],
                         B->d_desc, B->d_state, C.base, B->K, C.max_n);
    }
    (void)hipEventRecord(B->join[c], B->branch[c]);
    (void)hipStreamWaitEvent(B->stream, B->join[c], 0);
  }
  (void)hipMemcpyAsync(B->h_state, B->d_state, sizeof(SlotState) * B->nslots,
                       hipMemcpyDeviceToHost, B->stream);
  hipError_t e = hipStreamEndCapture(B->stream, &B->graph[mask]);
  if (e != hipSuccess) return fail(ctx, MXS_HIP, "graph capture failed: %s", hipGetErrorString(e));
  MXS_HIP_TRY(ctx, hipGraphInstantiate(&B->exec[mask], B->graph[mask], nullptr, nullptr, 0));
  return MXS_OK;
}

int class_of_slot(const mxs_batch* B, int slot) {
  int c = 0;
  while (c + 1 < B->nclasses && slot >= B->cls[c + 1].base) ++c;
  return c;
}

int class_of(const mxs_batch* B, int64_t n) {
  for (int c = 0; c < B->nclasses; ++c)
    if (n <= B->cls[c].max_n) return c;
  return -1;
}

// rowptr[0] = 0, rowptr[n] = nnz, rowptr monotone, 0 <= col < n and
// columns strictly increasing within each row.  The increasing test runs
// over all entries at once (a descent col[k] <= col[k-1] is allowed only
// where a row starts), so the entry loops vectorise.
bool validate_csr(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* col) {
  if (rp[0] != 0 || rp[n] != nnz) return false;
  int bad = 0;
  for (int64_t i = 0; i < n; ++i) bad |= rp[i + 1] < rp[i];
  if (bad) return false;
  const uint32_t un = (uint32_t)n;
  int64_t descents = 0;
  for (int64_t k = 0; k < nnz; ++k) bad |= (uint32_t)col[k] >= un;
  for (int64_t k = 1; k < nnz; ++k) descents += col[k] <= col[k - 1];
  if (bad) return false;
  // descents at row starts (each start position counted once)
  int64_t allowed = 0;
  for (int64_t i = 1; i < n; ++i) {
    const int32_t s = rp[i];
    if (s > rp[i - 1] && s < nnz) allowed += col[s] <= col[s - 1];
  }
  return descents == allowed;
}

// validate_csr and pack in one pass over rowptr and col: the checks run on
// the values as they are copied (false leaves `dst` partly written)
bool validate_pack(char* dst, int64_t n, int64_t nnz, const int32_t* rp, const int32_t* col,
                   const double* val, const double* b) {
  const Layout L = layout(n, nnz, 0);
  if (rp[0] != 0 || rp[n] != nnz) return false;
  int32_t* drp = (int32_t*)dst;
  int bad = 0;
  drp[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t v = rp[i + 1];
    drp[i + 1] = v;
    bad |= v < rp[i];
  }
  if (bad) return false;
  const uint32_t un = (uint32_t)n;
  int64_t descents = 0;
  if (nnz) {
    int32_t* dc = (int32_t*)(dst + L.col);
    dc[0] = col[0];
    bad |= (uint32_t)col[0] >= un;
    for (int64_t k = 1; k < nnz; ++k) {
      const int32_t c = col[k];
      dc[k] = c;
      bad |= (uint32_t)c >= un;
      descents += c <= col[k - 1];
    }
  }
  if (bad) return false;
  int64_t allowed = 0;
  for (int64_t i = 1; i < n; ++i) {
    const int32_t st = rp[i];
    if (st > rp[i - 1] && st < nnz) allowed += col[st] <= col[st - 1];
  }
  if (descents != allowed) return false;
  if (nnz) std::memcpy(dst + L.val, val, nnz * 8);
  std::memcpy(dst + L.b, b, n * 8);
  return true;
}

// packs rowptr | col | val | b at `dst` in the arena layout
void pack(char* dst, int64_t n, int64_t nnz, const int32_t* rp, const int32_t* col,
          const double* val, const double* b) {
  const Layout L = layout(n, nnz, 0);
  std::memcpy(dst, rp, (n + 1) * 4);
  if (nnz) {
    std::memcpy(dst + L.col, col, nnz * 4);
    std::memcpy(dst + L.val, val, nnz * 8);
  }
  std::memcpy(dst + L.b, b, n * 8);
}

// Host CPUs this process may run on (its affinity mask; a container or job
// slot may allow fewer than the machine has), at least 1.
unsigned usable_cpus() {
  cpu_set_t set;
  CPU_ZERO(&set);
  if (sched_getaffinity(0, sizeof(set), &set) == 0) {
    const int c = CPU_COUNT(&set);
    if (c > 0) return (unsigned)c;
  }
  return std::max(1u, std::thread::hardware_concurrency());
}

// Runs the retirement copies (pinned output -> result buffers), split by
// bytes over up to 8 threads when they add up to more than 4 MiB.
template <typename Copy>
void copy_out(const std::vector<Copy>& c) {
  size_t total = 0;
  for (const Copy& k : c) total += (size_t)k.n * sizeof(double);
  const unsigned hw = usable_cpus();
  const size_t nt = std::min<size_t>({(size_t)std::min(hw, 8u), c.size(), total >> 22});
  if (nt <= 1) {
    for (const Copy& k : c) std::memcpy(k.dst, k.src, (size_t)k.n * sizeof(double));
    return;
  }
  // contiguous runs of copies of about total / nt bytes each
  std::vector<size_t> cut{0};
  size_t acc = 0;
  for (size_t j = 0; j < c.size(); ++j) {
    acc += (size_t)c[j].n * sizeof(double);
    if (acc * nt >= total * cut.size() && cut.size() < nt) cut.push_back(j + 1);
  }
  cut.push_back(c.size());
  std::vector<std::thread> pool;
  for (size_t t = 0; t + 1 < cut.size(); ++t)
    pool.emplace_back([&, t] {
      for (size_t j = cut[t]; j < cut[t + 1]; ++j)
        std::memcpy(c[j].dst, c[j].src, (size_t)c[j].n * sizeof(double));
    });
  for (auto& th : pool) th.join();
}

mxs_status upload_desc(mxs_batch* B) {
  if (!B->desc_dirty) return MXS_OK;
  MXS_HIP_TRY(B->ctx, hipMemcpyAsync(B->d_desc, B->h_desc, sizeof(SlotDesc) * B->nslots,
                                     hipMemcpyHostToDevice, B->stream));
  B->desc_dirty = false;
  return MXS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// one system through the batched kernel (the single-system solver's path for
// small matrices): a one-slot descriptor in device scratch, one work-group
// of 1024 threads, up to 1024 iterations per launch
// ---------------------------------------------------------------------------
constexpr int kSmallBlock = 1024;

bool small_cg_fits(int64_t n, int64_t max_row) { return n >= 1 && n <= 8192 && max_row <= 64; }

size_t small_cg_scratch(int64_t n) { return 2 * kAlign + 2 * up((size_t)n * sizeof(double)); }

mxs_status small_cg(mxs_ctx* ctx, const mxs_matrix* A, const double* b, double* x,
                    double rel_tol, double abs_tol, bool base_r0, int64_t max_iters,
                    void* scratch, void* pinned, SmallCgResult* res) {
  static_assert(sizeof(SlotDesc) <= kAlign && sizeof(SlotState) <= kAlign, "staging layout");
  const int64_t n = A->n;
  // device: desc | state | r | p; pinned: desc | zeroed state (uploaded
  // together) | the state read back after each launch
  char* base = (char*)scratch;
  SlotDesc* d_desc = (SlotDesc*)base;
  SlotState* d_state = (SlotState*)(base + kAlign);
  double* r = (double*)(base + 2 * kAlign);
  double* p = (double*)(base + 2 * kAlign + up((size_t)n * sizeof(double)));
  char* hp = (char*)pinned;
  std::memset(hp, 0, 2 * kAlign);
  SlotDesc& hd = *(SlotDesc*)hp;
  SlotState& hs = *(SlotState*)(hp + 2 * kAlign);
  hd.rowptr = A->csr.rowptr;
  hd.col = A->csr.col;
  hd.val = (double*)A->csr.val;
  hd.b = const_cast<double*>(b);
  hd.x = x;
  hd.r = r;
  hd.p = p;
  hd.xout = x;
  hd.tol = rel_tol;
  hd.abs_tol = abs_tol;
  hd.x0_given = 1;
  hd.base_r0 = base_r0 ? 1 : 0;
  hd.n = (int32_t)n;
  hd.nnz = (int32_t)A->nnz;
  hd.max_iters = (int32_t)std::min<int64_t>(max_iters, INT32_MAX);
  hd.active = 1;
  hd.gen = 1;  // the zeroed state's gen differs: the first launch starts fresh
  ClassCfg C{};
  C.max_n = (int)n;
  C.block = kSmallBlock;
  C.rpt = rpt_for(C.max_n, C.block);
  C.lds = true;
  const size_t lds = class_lds(C);
  BatchKernel k = pick(true, 0, C.block, C.rpt);
  if (lds > 65536) {
    MXS_HIP_TRY(ctx, hipFuncSetAttribute((const void*)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  }
  MXS_HIP_TRY(ctx, hipMemcpyAsync(d_desc, hp, 2 * kAlign, hipMemcpyHostToDevice, ctx->stream));
  for (;;) {
    hipLaunchKernelGGL(k, dim3(1), dim3(C.block), lds, ctx->stream, d_desc, d_state, 0, 1024,
                       C.max_n);
    MXS_HIP_TRY(ctx, hipGetLastError());
    MXS_HIP_TRY(ctx, hipMemcpyAsync(&hs, d_state, sizeof(SlotState), hipMemcpyDeviceToHost,
                                    ctx->stream));
    MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (hs.status >= SLOT_CONVERGED) break;
  }
  res->iters = hs.iters;
  res->replacements = hs.repl;
  res->res2 = hs.res2;
  res->base = hs.base;
  res->status = hs.status == SLOT_CONVERGED   ? MXS_OK
                : hs.status == SLOT_BREAKDOWN ? MXS_BREAKDOWN
                : hs.status == SLOT_NONFINITE ? MXS_NONFINITE
                                              : MXS_NOT_CONVERGED;
  return MXS_OK;
}

// ---------------------------------------------------------------------------
// one small system by pipelined CG (Ghysels & Vanroose 2014, unpreconditioned)
// in one work-group of 1024 threads: the matrix lives in registers (rows
// tid + k*1024, at most 20 entries a thread), the gather vector w in one of
// two LDS buffers (w_{i+1} goes to the other one), so an iteration needs a
// single barrier, the one that completes both the (gamma, delta) partials
// and w_i.  The true-residual check and replacement follow the CG protocol
// (at most three replacements, then restart with beta = 0).
// ---------------------------------------------------------------------------
struct PipeArgs {
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  const double* b;
  double* x;     // the iterate (x0 = 0 on the first launch)
  double* vecs;  // r | w | z | s | p, ld doubles each, kept between launches
  double tol;    // threshold on ||r|| relative to ||b||
  int32_t n, ld, max_iters;
};

struct PipeState {
  double gprev, aprev, res2, thr;  // thr: tol * ||b||, set by the first launch
  int32_t iters, status, repl, restart, started, pad;
};

constexpr int kPipeBlock = 1024;

template <int RPT>
__global__ __launch_bounds__(kPipeBlock) void k_small_pipecg(PipeArgs a, PipeState* st, int K) {
  constexpr int BS = kPipeBlock, ML = 20 / RPT;
  extern __shared__ double dyn[];  // two gather buffers, then z and s, ld doubles each
  __shared__ double red[2][2][BS / 64];
  __shared__ double red2[BS / 64];
  const int n = a.n, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // buffer 0 at dyn, buffer 1 at dyn + ld (chosen by ternaries, not an
  // indexed pointer array, which would live in scratch)
  double* const wb0 = dyn;
  double* const wb1 = dyn + a.ld;
  double* __restrict__ const zl = dyn + 2 * a.ld;  // a thread's own rows only
  double* __restrict__ const sl = dyn + 3 * a.ld;
  int32_t cr[RPT * ML];
  double vr[RPT * ML];
  uint32_t hm = 0;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int i = tid + k * BS;
    const int32_t a0 = i < n ? a.rowptr[i] : 0, e0 = i < n ? a.rowptr[i + 1] : 0;
#pragma unroll
    for (int j = 0; j < ML; ++j) {
      const bool h = a0 + j < e0;
      const int32_t es = h ? a0 + j : 0;
      cr[k * ML + j] = a.col[es] * (int32_t)sizeof(double);  // byte offset
      vr[k * ML + j] = a.val[es];
      hm |= (h ? 1u : 0u) << (k * ML + j);
    }
  }
  auto spmv = [&](const double* __restrict__ v, double (&q)[RPT]) {
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < ML; ++j) {
        const double g = *(const double*)((const char*)v + cr[k * ML + j]);
        if ((hm >> (k * ML + j)) & 1u) acc += vr[k * ML + j] * g;
      }
      q[k] = acc;
    }
  };
  double* __restrict__ R = a.vecs;
  double* __restrict__ W = R + a.ld;
  double* __restrict__ Z = W + a.ld;
  double* __restrict__ Sg = Z + a.ld;
  double* __restrict__ P = Sg + a.ld;
  // p lives in HBM (P) like x, w only in its LDS buffer, z and s in LDS:
  // the 1024-thread work-group has 128 registers a lane, and the matrix
  // takes most of them
  double r[RPT];
  const PipeState ps = *st;
  int status = SLOT_RUN, it = ps.iters, repl = ps.repl;
  bool restart = ps.restart != 0;
  double gprev = ps.gprev, aprev = ps.aprev, res2 = ps.res2, thr = ps.thr;
  bool need_thr = !ps.started;
  if (!ps.started) {
    // x0 = 0: r = b, then w = A r (r staged in the second buffer)
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      r[k] = i < n ? a.b[i] : 0.0;
      if (i < n) {
        a.x[i] = 0.0;
        P[i] = 0.0;
        zl[i] = sl[i] = 0.0;
        wb1[i] = r[k];
      }
    }
    __syncthreads();
    double w[RPT];
    spmv(wb1, w);
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      if (i < n) wb0[i] = w[k];
    }
    restart = true;
  } else {
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      r[k] = i < n ? R[i] : 0.0;
      if (i < n) {
        zl[i] = Z[i];
        sl[i] = Sg[i];
        wb0[i] = W[i];
      }
    }
  }
  // w_i lives in buffer `par` (a thread reads its own rows there); the
  // loop-top barrier completes it
  int par = 0;
  for (int step = 0; step < K; ++step) {
    double* __restrict__ other = par ? wb0 : wb1;
    double* __restrict__ cur = par ? wb1 : wb0;
    double gp = 0.0, dp = 0.0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      gp += r[k] * r[k];
      if (i < n) dp += cur[i] * r[k];
    }
    gp = wave_total(gp);
    dp = wave_total(dp);
    if (lane == 0) {
      red[par][0][wv] = gp;
      red[par][1][wv] = dp;
    }
    __syncthreads();
    double gm = red[par][0][0], dl = red[par][1][0];
#pragma unroll
    for (int q = 1; q < BS / 64; ++q) {
      gm += red[par][0][q];
      dl += red[par][1][q];
    }
    if (!isfinite(gm) || !isfinite(dl)) {
      status = SLOT_NONFINITE;
      break;
    }
    if (need_thr) {  // x0 = 0: the first gamma is ||b||^2
      thr = a.tol * sqrt(gm);
      need_thr = false;
    }
    if (sqrt(gm) <= thr) {
      // true residual t = b - A x, x staged in the other buffer (its last
      // readers, the previous product, are behind the barrier above)
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * BS;
        if (i < n) other[i] = a.x[i];
      }
      __syncthreads();
      double t[RPT];
      spmv(other, t);
      double tt = 0.0;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * BS;
        t[k] = i < n ? a.b[i] - t[k] : 0.0;
        tt += t[k] * t[k];
      }
      tt = bsum<BS>(tt, red2);  // its barriers end every read of `other`
      res2 = tt;
      if (sqrt(tt) <= thr) {
        status = SLOT_CONVERGED;
        break;
      }
      if (repl >= 3) {
        status = SLOT_NOTCONV;
        break;
      }
      // replacement: r = t, w = A r, restart (beta = 0)
      ++repl;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * BS;
        r[k] = t[k];
        if (i < n) {
          zl[i] = sl[i] = 0.0;
          other[i] = r[k];
        }
      }
      __syncthreads();
      double w[RPT];
      spmv(other, w);
      // nobody reads w_i's buffer before the next loop-top barrier
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * BS;
        if (i < n) cur[i] = w[k];
      }
      restart = true;
      continue;
    }
    double q[RPT];
    spmv(cur, q);
    double beta, den;
    if (restart) {
      beta = 0.0;
      den = dl;
    } else {
      beta = gm / gprev;
      den = dl - beta * gm / aprev;
    }
    if (!(den > 0.0)) {
      status = isfinite(den) ? SLOT_BREAKDOWN : SLOT_NONFINITE;
      break;
    }
    const double alpha = gm / den;
    restart = false;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      if (i < n) {
        const double wk = cur[i];
        const double zk = q[k] + beta * zl[i];
        const double sk = wk + beta * sl[i];
        const double pk = r[k] + beta * P[i];
        zl[i] = zk;
        sl[i] = sk;
        P[i] = pk;
        a.x[i] += alpha * pk;
        r[k] -= alpha * sk;
        // w_{i+1}: its buffer's last readers are behind the barrier
        other[i] = wk - alpha * zk;
      }
    }
    gprev = gm;
    aprev = alpha;
    par ^= 1;
    res2 = gm;
    if (++it >= a.max_iters) {
      status = SLOT_MAXIT;
      break;
    }
  }
  if (status == SLOT_RUN) {
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int i = tid + k * BS;
      if (i < n) {
        R[i] = r[k];
        W[i] = (par ? wb1 : wb0)[i];
        Z[i] = zl[i];
        Sg[i] = sl[i];
      }
    }
  }
  if (tid == 0) {
    PipeState o;
    o.gprev = gprev;
    o.aprev = aprev;
    o.res2 = res2;
    o.thr = thr;
    o.iters = it;
    o.status = status;
    o.repl = repl;
    o.restart = restart ? 1 : 0;
    o.started = 1;
    o.pad = 0;
    *st = o;
  }
}

bool small_pipecg_fits(int64_t n, int64_t max_row) {
  if (n < 1 || n > 4 * kPipeBlock) return false;
  const int64_t rpt = (n + kPipeBlock - 1) / kPipeBlock;
  const int64_t r = rpt <= 1 ? 1 : rpt <= 2 ? 2 : 4;
  return max_row <= 20 / r;
}

size_t small_pipecg_scratch(int64_t n) {
  return kAlign + 5 * up((size_t)n * sizeof(double));
}

mxs_status small_pipecg(mxs_ctx* ctx, const mxs_matrix* A, const double* rhs, double* out,
                        double tol, int64_t max_iters, void* scratch, SmallCgResult* res) {
  const int64_t n = A->n;
  const size_t ld = up((size_t)n * sizeof(double)) / sizeof(double);
  PipeState* d_st = (PipeState*)scratch;
  PipeArgs a;
  a.rowptr = A->csr.rowptr;
  a.col = A->csr.col;
  a.val = (const double*)A->csr.val;
  a.b = rhs;
  a.x = out;
  a.vecs = (double*)((char*)scratch + kAlign);
  a.tol = tol;
  a.n = (int32_t)n;
  a.ld = (int32_t)ld;
  a.max_iters = (int32_t)std::min<int64_t>(max_iters, INT32_MAX);
  const int64_t rpt = (n + kPipeBlock - 1) / kPipeBlock;
  void (*k)(PipeArgs, PipeState*, int) =
      rpt <= 1 ? k_small_pipecg<1> : rpt <= 2 ? k_small_pipecg<2> : k_small_pipecg<4>;
  const size_t lds = 4 * ld * sizeof(double);
  if (lds > 65536)
    MXS_HIP_TRY(ctx, hipFuncSetAttribute((const void*)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  MXS_HIP_TRY(ctx, hipMemsetAsync(d_st, 0, sizeof(PipeState), ctx->stream));
  PipeState hs;
  std::memset(&hs, 0, sizeof(hs));
  for (;;) {
    hipLaunchKernelGGL(k, dim3(1), dim3(kPipeBlock), lds, ctx->stream, a, d_st, 1024);
    MXS_HIP_TRY(ctx, hipGetLastError());
    MXS_HIP_TRY(ctx, hipMemcpyAsync(&hs, d_st, sizeof(hs), hipMemcpyDeviceToHost, ctx->stream));
    MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (hs.status != 0 && hs.status != SLOT_RUN) break;
  }
  res->iters = hs.iters;
  res->replacements = hs.repl;
  res->res2 = hs.res2;
  res->status = hs.status == SLOT_CONVERGED   ? MXS_OK
                : hs.status == SLOT_BREAKDOWN ? MXS_BREAKDOWN
                : hs.status == SLOT_NONFINITE ? MXS_NONFINITE
                                              : MXS_NOT_CONVERGED;
  return MXS_OK;
}

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
    // (n <= 8192 and n <= 10240 are separate 1024-thread classes: 8 rows a
    // thread fit the registers, 10 do not; with fewer than 5 slots the two
    // are one class)
    const int dn[5] = {1024, 2304, 4096, 8192, 10240}, db[5] = {256, 256, 512, 1024, 1024};
    nc = 0;
    for (int c = 0; c < 5; ++c) {
      if (c == 3 && opts->max_slots < 5) continue;
      max_n[nc] = dn[c];
      block[nc] = db[c];
      nsl[nc] = 0;
      ++nc;
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
  size_t xout_total = 0;
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
      bool ok = true;
      for (int mode = 0; mode < 2; ++mode)
        ok = ok && hipFuncSetAttribute((const void*)pick(C.lds, mode, C.block, C.rpt),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds) == hipSuccess;
      if (ok) break;
      (void)hipGetLastError();
      C.lds = false;  // fall back to the gather vector in HBM
    }
    for (int i = 0; i < C.slots; ++i) {
      B->xout_off.push_back(xout_total);
      xout_total += up((size_t)C.max_n * sizeof(double)) / sizeof(double);
    }
    base += C.slots;
  }
  B->nclasses = nc;
  B->nslots = base;
  B->slots.resize(B->nslots);
  for (int c = 0; c < nc; ++c)
    for (int i = B->cls[c].base + B->cls[c].slots - 1; i >= B->cls[c].base; --i)
      B->free_slots[c].push_back(i);
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
    // pinned host memory that kernels read (packed inputs) and write
    // (finished iterates); the device addresses come from the runtime
    const size_t in_size = up(opts->staging_bytes
                                  ? opts->staging_bytes
                                  : std::min<size_t>(opts->budget_bytes, (size_t)1 << 30));
    // coherent: kernels see what the host packed, the host sees what
    // kernels wrote, with no cache maintenance in between
    const unsigned fl = hipHostMallocMapped | hipHostMallocCoherent;
    if (hipHostMalloc((void**)&B->in_mem, in_size, fl) != hipSuccess ||
        hipHostMalloc((void**)&B->xout_mem, xout_total * sizeof(double), fl) != hipSuccess) {
      st = fail(ctx, MXS_OOM, "pinned input / output pools");
      break;
    }
    if (hipHostGetDevicePointer((void**)&B->in_dev, B->in_mem, 0) != hipSuccess ||
        hipHostGetDevicePointer((void**)&B->xout_dev, B->xout_mem, 0) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "device view of pinned host memory");
      break;
    }
    B->inpool.init(in_size);
    // touch every page of the pools now, on up to 16 threads: the first
    // write to a page of pinned memory costs several times a later one, and
    // would otherwise land on the submissions of a running service
    {
      const unsigned hw = usable_cpus();
      const size_t nt = std::max<size_t>(1, std::min<size_t>({(size_t)std::min(hw, 16u),
                                                              in_size >> 24}));
      const size_t per = (in_size / nt + 4095) / 4096 * 4096;
      std::vector<std::thread> pool;
      for (size_t t = 0; t < nt; ++t)
        pool.emplace_back([&, t] {
          const size_t a = std::min(in_size, t * per), e = std::min(in_size, a + per);
          if (e > a) std::memset(B->in_mem + a, 0, e - a);
        });
      for (auto& th : pool) th.join();
      std::memset(B->xout_mem, 0, xout_total * sizeof(double));
    }
    B->arena_mem = (char*)ctx->alloc.alloc(opts->budget_bytes);
    if (!B->arena_mem) {
      st = fail(ctx, MXS_OOM, "cannot allocate the %zu-byte batch arena", opts->budget_bytes);
      break;
    }
    B->arena.init(opts->budget_bytes / kAlign * kAlign);
    B->d_desc = (SlotDesc*)ctx->alloc.alloc(sizeof(SlotDesc) * B->nslots);
    B->d_state = (SlotState*)ctx->alloc.alloc(sizeof(SlotState) * B->nslots);
    if (!B->d_desc || !B->d_state ||
        hipHostMalloc((void**)&B->h_desc, sizeof(SlotDesc) * B->nslots, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void**)&B->h_state, sizeof(SlotState) * B->nslots,
                      hipHostMallocDefault) != hipSuccess) {
      st = fail(ctx, MXS_OOM, "slot tables");
      break;
    }
    std::memset(B->h_desc, 0, sizeof(SlotDesc) * B->nslots);
    std::memset(B->h_state, 0, sizeof(SlotState) * B->nslots);
    if (hipMemcpyAsync(B->d_desc, B->h_desc, sizeof(SlotDesc) * B->nslots,
                       hipMemcpyHostToDevice, B->stream) != hipSuccess ||
        hipMemcpyAsync(B->d_state, B->h_state, sizeof(SlotState) * B->nslots,
                       hipMemcpyHostToDevice, B->stream) != hipSuccess ||
        hipStreamSynchronize(B->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "slot table upload failed");
      break;
    }
    B->desc_dirty = false;
    for (int mask = 1; mask < 4 && !st; ++mask) st = build_graph(B, mask);
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
  for (int m = 0; m < 4; ++m) {
    if (B->exec[m]) (void)hipGraphExecDestroy(B->exec[m]);
    if (B->graph[m]) (void)hipGraphDestroy(B->graph[m]);
  }
  if (B->ctx) {
    B->ctx->alloc.release(B->arena_mem);
    B->ctx->alloc.release(B->d_desc);
    B->ctx->alloc.release(B->d_state);
  }
  if (B->h_desc) (void)hipHostFree(B->h_desc);
  if (B->h_state) (void)hipHostFree(B->h_state);
  if (B->in_mem) (void)hipHostFree(B->in_mem);
  if (B->xout_mem) (void)hipHostFree(B->xout_mem);
  for (int c = 0; c < mxs::kMaxClasses; ++c) {
    if (B->branch[c]) (void)hipStreamDestroy(B->branch[c]);
    if (B->join[c]) (void)hipEventDestroy(B->join[c]);
  }
  if (B->fork) (void)hipEventDestroy(B->fork);
  if (B->stream) (void)hipStreamDestroy(B->stream);
  delete B;
  return MXS_OK;
}

mxs_status mxs_batch_submit_many(mxs_batch* B, int64_t count, const mxs_batch_request* reqs,
                                 uint64_t* tickets, mxs_status* statuses) {
  if (!B || count < 0 || (count && (!reqs || !tickets || !statuses))) return MXS_INVALID_ARG;
  mxs_ctx* ctx = B->ctx;
  // 1. sizes, class and budget, and a place in the pinned pool (in order)
  std::vector<Request> R((size_t)count);
  std::unique_lock<std::mutex> lock(B->mu);
  for (int64_t i = 0; i < count; ++i) {
    const mxs_batch_request& q = reqs[i];
    tickets[i] = 0;
    statuses[i] = MXS_OK;
    if (q.n < 1 || q.nnz < 0 || !q.rowptr || !q.b || (q.nnz && (!q.col || !q.val))) {
      statuses[i] = MXS_INVALID_ARG;
      continue;
    }
    if (q.n > INT32_MAX || q.nnz > INT32_MAX) {
      statuses[i] = fail(ctx, MXS_UNSUPPORTED, "sizes beyond int32");
      continue;
    }
    if (q.mode != 0 && q.mode != 1) {
      statuses[i] = fail(ctx, MXS_INVALID_ARG, "unknown batch mode %d", (int)q.mode);
      continue;
    }
    if (q.mode == 1 && !(q.inner_rel_tol >= 0.0 && q.inner_rel_tol < 1.0)) {
      statuses[i] = fail(ctx, MXS_INVALID_ARG, "inner tolerance must be in [0, 1)");
      continue;
    }
    const int c = class_of(B, q.n);
    if (c < 0) {
      statuses[i] = fail(ctx, MXS_UNSUPPORTED, "n = %lld exceeds the largest size class",
                         (long long)q.n);
      continue;
    }
    const Layout L = layout(q.n, q.nnz, q.mode);
    if (L.total > B->arena.size) {
      statuses[i] = fail(ctx, MXS_BUDGET, "request needs %zu bytes, budget is %zu", L.total,
                         B->arena.size);
      continue;
    }
    if (L.x > B->inpool.size) {
      statuses[i] = fail(ctx, MXS_BUDGET, "request inputs need %zu bytes of staging, have %zu",
                         L.x, B->inpool.size);
      continue;
    }
    Request& r = R[i];
    r.n = q.n;
    r.nnz = q.nnz;
    r.tol = q.rel_tol;
    r.max_iters = q.max_iters > 0 ? q.max_iters : 20000;
    r.bytes = L.total;
    r.in_bytes = L.x;
    r.cls = c;
    r.mode = q.mode;
    r.inner_tol = q.inner_rel_tol > 0.0 ? (float)q.inner_rel_tol : 1e-4f;
    // pack into pinned memory when there is room; otherwise keep a copy and
    // pack at admission
    r.packed = B->inpool.alloc(r.in_bytes, &r.in_off);
  }
  lock.unlock();
  // 2. validate and pack / copy, on worker threads for large submissions
  // (each request's pool region is its own until it is queued)
  std::vector<char> valid((size_t)count, 0);
  auto work = [&](int64_t i) {
    if (statuses[i] != MXS_OK) return;
    const mxs_batch_request& q = reqs[i];
    Request& r = R[i];
    if (r.packed) {
      valid[i] = validate_pack(B->in_mem + r.in_off, q.n, q.nnz, q.rowptr, q.col, q.val, q.b);
      return;
    }
    if (!validate_csr(q.n, q.nnz, q.rowptr, q.col)) return;
    valid[i] = 1;
    {
      r.rowptr.assign(q.rowptr, q.rowptr + q.n + 1);
      r.col.assign(q.col, q.col + q.nnz);
      r.val.assign(q.val, q.val + q.nnz);
      r.b.assign(q.b, q.b + q.n);
    }
  };
  int64_t bytes_total = 0;
  for (int64_t i = 0; i < count; ++i)
    if (statuses[i] == MXS_OK) bytes_total += (int64_t)R[i].in_bytes;
  const unsigned hw = usable_cpus();
  const int64_t nthreads =
      std::min<int64_t>({(int64_t)std::min(hw, 16u), count, bytes_total >> 20});
  if (nthreads <= 1) {
    for (int64_t i = 0; i < count; ++i) work(i);
  } else {
    std::atomic<int64_t> next{0};
    auto loop = [&]() {
      for (int64_t i; (i = next.fetch_add(1, std::memory_order_relaxed)) < count;) work(i);
    };
    std::vector<std::thread> pool;
    for (int64_t t = 1; t < nthreads; ++t) pool.emplace_back(loop);
    loop();
    for (auto& t : pool) t.join();
  }
  // 3. queue the valid ones in order
  lock.lock();
  for (int64_t i = 0; i < count; ++i) {
    if (statuses[i] != MXS_OK) continue;
    Request& r = R[i];
    if (!valid[i]) {
      if (r.packed) B->inpool.release(r.in_off, r.in_bytes);
      statuses[i] = fail(ctx, MXS_INVALID_MATRIX, "submitted CSR failed validation");
      continue;
    }
    r.ticket = B->next_ticket++;
    tickets[i] = r.ticket;
    B->pending.push_back(std::move(r));
  }
  return MXS_OK;
}

mxs_status mxs_batch_submit(mxs_batch* B, int64_t n, int64_t nnz, const int32_t* rowptr,
                            const int32_t* col, const double* val, const double* b,
                            double rel_tol, int64_t max_iters, uint64_t* ticket) {
  if (!B || !ticket) return MXS_INVALID_ARG;
  mxs_batch_request q = {n, nnz, rowptr, col, val, b, rel_tol, max_iters, 0, 0, 0.0};
  mxs_status st = MXS_OK;
  const mxs_status call = mxs_batch_submit_many(B, 1, &q, ticket, &st);
  return call ? call : st;
}

mxs_status mxs_batch_step_launch(mxs_batch* B) {
  if (!B) return MXS_INVALID_ARG;
  mxs_ctx* ctx = B->ctx;
  std::lock_guard<std::mutex> lock(B->mu);
  if (B->in_flight) return fail(ctx, MXS_INVALID_ARG, "batch step launched twice without finish");
  MXS_HIP_TRY(ctx, hipSetDevice(ctx->device));
  // 1. admit in FIFO order, first fit: a request that does not fit (no free
  // slot in its class, or no arena gap) is passed over by later ones,
  // unless it has been the oldest waiting request for more than 64 steps;
  // then nothing behind it is admitted until it fits (starvation guard).
  // One pass over the queue: admitted requests leave it, the others are
  // moved down in order; a request whose class has no free slot costs one
  // test.
  size_t keep = 0;
  bool blocked = false;
  for (size_t idx = 0; idx < B->pending.size(); ++idx) {
    Request& R = B->pending[idx];
    bool fits = false;
    size_t off = 0;
    std::vector<int>& fs = B->free_slots[R.cls];
    if (!blocked && !fs.empty() && B->arena.alloc(R.bytes, &off)) {
      fits = true;
      if (!R.packed) {
        if (B->inpool.alloc(R.in_bytes, &R.in_off)) {
          pack(B->in_mem + R.in_off, R.n, R.nnz, R.rowptr.data(), R.col.data(), R.val.data(),
               R.b.data());
          R.packed = true;
          std::vector<int32_t>().swap(R.rowptr);
          std::vector<int32_t>().swap(R.col);
          std::vector<double>().swap(R.val);
          std::vector<double>().swap(R.b);
        } else {
          B->arena.release(off, R.bytes);
          fits = false;
        }
      }
    }
    if (!fits) {
      if (keep == 0 && !blocked) {  // the oldest request still waiting
        if (R.ticket == B->starve_ticket) {
          B->starve_steps++;
        } else {
          B->starve_ticket = R.ticket;
          B->starve_steps = 1;
        }
        if (B->starve_steps > 64) blocked = true;
      }
      if (keep != idx) B->pending[keep] = std::move(R);
      ++keep;
      continue;
    }
    const int si = fs.back();
    fs.pop_back();
    char* p = (char*)B->arena_mem + off;
    const Layout L = layout(R.n, R.nnz, R.mode);
    SlotDesc& d = B->h_desc[si];
    std::memset(&d, 0, sizeof(d));
    d.rowptr = (int32_t*)p;
    d.col = (int32_t*)(p + L.col);
    d.val = (double*)(p + L.val);
    d.b = (double*)(p + L.b);
    d.x = (double*)(p + L.x);
    d.r = (double*)(p + L.r);
    d.p = (double*)(p + L.p);
    d.src = (const uint4*)(B->in_dev + R.in_off);
    d.xout = B->xout_dev + B->xout_off[si];
    d.tol = R.tol;
    d.n = (int32_t)R.n;
    d.nnz = (int32_t)R.nnz;
    d.max_iters = (int32_t)std::min<int64_t>(R.max_iters, INT32_MAX);
    d.active = 1;
    if (++B->gen == 0) ++B->gen;  // 0 marks a state no launch has written
    d.gen = B->gen;
    d.in_words = (int32_t)(R.in_bytes / 16);
    d.v32 = (float*)(p + L.v32);
    d.mode = R.mode;
    d.inner_tol = R.inner_tol;
    B->desc_dirty = true;
    Slot& s = B->slots[si];
    s.busy = true;
    s.holds_input = true;
    s.ticket = R.ticket;
    s.off = off;
    s.bytes = R.bytes;
    s.in_off = R.in_off;
    s.in_bytes = R.in_bytes;
    s.n = R.n;
  }
  B->pending.resize(keep);
  // 2. run K iterations of every resident system, read the states back
  int active = 0, mask = 0;
  for (int i = 0; i < B->nslots; ++i) {
    if (!B->slots[i].busy) continue;
    active++;
    mask |= 1 << B->h_desc[i].mode;
  }
  if (active > 0) {
    mxs_status st = upload_desc(B);
    if (st) return st;
    MXS_HIP_TRY(ctx, hipGraphLaunch(B->exec[mask], B->stream));
  }
  B->in_flight = true;
  B->flight_active = active;
  return MXS_OK;
}

mxs_status mxs_batch_step_finish(mxs_batch* B, mxs_batch_stats* stats) {
  if (!B) return MXS_INVALID_ARG;
  mxs_ctx* ctx = B->ctx;
  std::unique_lock<std::mutex> lock(B->mu);
  if (!B->in_flight) return fail(ctx, MXS_INVALID_ARG, "no batch step in flight");
  int active = B->flight_active;
  lock.unlock();
  // wait without the lock, so that submissions proceed meanwhile
  MXS_HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (active > 0) MXS_HIP_TRY(ctx, hipStreamSynchronize(B->stream));
  lock.lock();
  B->in_flight = false;
  // 3. every resident slot has copied its inputs by now; retire the
  // finished ones (their x is already in the pinned output, and is copied
  // out below, on several threads when there is much of it)
  struct Copy {
    double* dst;
    const double* src;
    int64_t n;
  };
  std::vector<Copy> copies;
  for (int i = 0; i < B->nslots && active > 0; ++i) {
    Slot& s = B->slots[i];
    if (!s.busy) continue;
    if (s.holds_input) {
      B->inpool.release(s.in_off, s.in_bytes);
      s.holds_input = false;
    }
    const SlotState& d = B->h_state[i];
    if (d.gen != B->h_desc[i].gen || d.status < SLOT_CONVERGED) continue;
    Result& R = B->results[s.ticket];
    R.x.reset(new double[(size_t)s.n]);
    R.n = s.n;
    copies.push_back({R.x.get(), B->xout_mem + B->xout_off[i], s.n});
    std::memset(&R.info, 0, sizeof(R.info));
    R.info.iters = d.iters;  // refinement mode: inner iterations in total
    R.info.replacements = d.repl;
    R.info.restarts = B->h_desc[i].mode == 1 ? d.outer : 0;  // refinement: outer steps
    const double tol = B->h_desc[i].tol;
    const double nb = tol > 0 ? d.thr / tol : 0.0;
    R.info.relres_recurrence = nb > 0 ? sqrt(d.res2) / nb : 0.0;
    R.info.relres_true = d.status == SLOT_CONVERGED || d.status == SLOT_NOTCONV
                             ? (nb > 0 ? sqrt(d.res2) / nb : 0.0)
                             : -1.0;
    R.info.status = d.status == SLOT_CONVERGED   ? MXS_OK
                    : d.status == SLOT_BREAKDOWN ? MXS_BREAKDOWN
                    : d.status == SLOT_NONFINITE ? MXS_NONFINITE
                                                 : MXS_NOT_CONVERGED;
    R.done = true;
    B->newly_done.push_back(s.ticket);
    B->arena.release(s.off, s.bytes);
    s.busy = false;
    B->free_slots[class_of_slot(B, i)].push_back(i);
    B->h_desc[i].active = 0;
    B->desc_dirty = true;
    B->completed++;
    active--;
  }
  copy_out(copies);
  if (stats) {
    int resident = 0;
    for (const Slot& s : B->slots) resident += s.busy ? 1 : 0;
    stats->active = resident;
    stats->pending = (int32_t)B->pending.size();
    stats->completed = B->completed;
    stats->arena_used = (int64_t)B->arena.used;
    stats->arena_size = (int64_t)B->arena.size;
    stats->slots = B->nslots;
  }
  return MXS_OK;
}

mxs_status mxs_batch_step(mxs_batch* B, mxs_batch_stats* stats) {
  const mxs_status st = mxs_batch_step_launch(B);
  if (st) return st;
  return mxs_batch_step_finish(B, stats);
}

mxs_status mxs_batch_poll(mxs_batch* B, uint64_t ticket, double* x_host, mxs_solve_info* info) {
  if (!B) return MXS_INVALID_ARG;
  std::lock_guard<std::mutex> lock(B->mu);
  auto it = B->results.find(ticket);
  if (it == B->results.end() || !it->second.done) {
    if (ticket == 0 || ticket >= B->next_ticket) return MXS_INVALID_ARG;
    return MXS_PENDING;
  }
  if (x_host) std::memcpy(x_host, it->second.x.get(), (size_t)it->second.n * sizeof(double));
  if (info) *info = it->second.info;
  const mxs_status st = it->second.info.status;
  B->results.erase(it);
  return st;
}

mxs_status mxs_batch_poll_many(mxs_batch* B, int64_t count, const uint64_t* tickets,
                               double* x_host, const int64_t* x_off, mxs_solve_info* infos,
                               mxs_status* statuses) {
  if (!B || count < 0 || (count && (!tickets || !statuses)) || (x_host && !x_off))
    return MXS_INVALID_ARG;
  std::lock_guard<std::mutex> lock(B->mu);
  struct Copy {
    double* dst;
    const double* src;
    int64_t n;
  };
  std::vector<Copy> copies;
  std::vector<std::unique_ptr<double[]>> hold;  // freed once the copies are done
  for (int64_t i = 0; i < count; ++i) {
    const uint64_t t = tickets[i];
    auto it = B->results.find(t);
    if (it == B->results.end() || !it->second.done) {
      statuses[i] = (t == 0 || t >= B->next_ticket) ? MXS_INVALID_ARG : MXS_PENDING;
      continue;
    }
    if (x_host) copies.push_back({x_host + x_off[i], it->second.x.get(), it->second.n});
    if (infos) infos[i] = it->second.info;
    statuses[i] = it->second.info.status;
    hold.push_back(std::move(it->second.x));
    B->results.erase(it);
  }
  copy_out(copies);
  return MXS_OK;
}

mxs_status mxs_batch_completed(mxs_batch* B, uint64_t* tickets, int64_t cap, int64_t* count) {
  if (!B || !count || (cap > 0 && !tickets)) return MXS_INVALID_ARG;
  std::lock_guard<std::mutex> lock(B->mu);
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
