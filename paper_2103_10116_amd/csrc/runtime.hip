// runtime.hip -- contexts, allocation, error strings, HBM probe and cache
// flush of libmxs.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "common.h"

namespace mxs {

void* Allocator::alloc(size_t bytes) const {
  if (bytes == 0) bytes = 1;
  if (custom) {
    // the kernels load 16-byte words from every array: a block that is not
    // 16-byte aligned is handed back and counts as a failed allocation
    void* p = cb.alloc(bytes, stream, cb.user);
    if (p && ((uintptr_t)p & 15) != 0) {
      cb.free(p, stream, cb.user);
      return nullptr;
    }
    return p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void Allocator::release(void* p) const {
  if (!p) return;
  if (custom)
    cb.free(p, stream, cb.user);
  else
    (void)hipFree(p);
}

mxs_status fail(mxs_ctx* ctx, mxs_status s, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->last_error = buf;
  }
  return s;
}

bool ws_reserve(mxs_ctx* ctx, size_t bytes) {
  if (ctx->ws.bytes >= bytes) return true;
  // the stream may still use the old buffer
  if (ctx->ws.ptr) {
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return false;
    ctx->alloc.release(ctx->ws.ptr);
  }
  size_t want = bytes + bytes / 4;
  ctx->ws.ptr = ctx->alloc.alloc(want);
  ctx->ws.bytes = ctx->ws.ptr ? want : 0;
  return ctx->ws.ptr != nullptr;
}

bool pinned_reserve(mxs_ctx* ctx, size_t bytes) {
  if (ctx->pinned_bytes >= bytes) return true;
  if (ctx->pinned) {
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return false;
    (void)hipHostFree(ctx->pinned);
  }
  ctx->pinned = nullptr;
  ctx->pinned_bytes = 0;
  if (hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    ctx->pinned = nullptr;
    return false;
  }
  ctx->pinned_bytes = bytes;
  return true;
}

// ---------------------------------------------------------------------------
// HBM probe kernels: 16-byte accesses, grid-stride, 256 threads
// ---------------------------------------------------------------------------
// Each thread moves four 16-byte elements per iteration, all loads issued
// before any use, so a wave keeps 4 KB in flight.
constexpr int kProbeUnroll = 2;

__global__ __launch_bounds__(256) void k_probe_read(const double2* __restrict__ a, int64_t n2,
                                                    double* __restrict__ sink) {
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (kProbeUnroll - 1) * stride < n2; i += kProbeUnroll * stride) {
    double2 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = a[i + u * stride];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) s += v[u].x + v[u].y;
  }
  for (; i < n2; i += stride) s += a[i].x + a[i].y;
  s = wave_sum(s);
  // keeps the loads alive; never true for the fill values used here
  if (s == 1.2345e300) sink[0] = s;
}

// one 16-byte element per thread, no loop: the grid covers the array.  NT:
// a non-temporal load, as the products use for matrices larger than the
// Infinity Cache (the faster of the two read shapes sets the read figure)
template <bool NT>
__global__ __launch_bounds__(256) void k_probe_read1(const double2* __restrict__ a, int64_t n2,
                                                     double* __restrict__ sink) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < n2) {
    if constexpr (NT) {
      const d2 v = __builtin_nontemporal_load(reinterpret_cast<const d2*>(a) + i);
      s = v.x + v.y;
    } else {
      s = a[i].x + a[i].y;
    }
  }
  s = wave_sum(s);
  if (s == 1.2345e300) sink[0] = s;
}

// Random indices in [0, nx): the finaliser of MurmurHash3 (a published
// 64-bit mixing function) applied to the entry number.
__global__ __launch_bounds__(256) void k_fill_random_index(int32_t* __restrict__ idx,
                                                           int64_t count, int64_t nx) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride) {
    uint64_t h = (uint64_t)k + 0x9E3779B97F4A7C15ull;
    h ^= h >> 33;
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
    h *= 0xc4ceb9fe1a85ec53ull;
    h ^= h >> 33;
    idx[k] = (int32_t)(h % (uint64_t)nx);
  }
}

// count loads x[idx[k]]: each thread takes eight indices per step (index
// loads coalesced across the block), all eight gathers in flight together
template <typename T>
__global__ __launch_bounds__(256) void k_probe_gather(const int32_t* __restrict__ idx,
                                                      const T* __restrict__ x, int64_t count,
                                                      double* __restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * 256 * 8;
  T acc = 0;
  for (int64_t base = (int64_t)blockIdx.x * 256 * 8 + threadIdx.x; base < count;
       base += stride) {
    int32_t c[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) c[t] = base + t * 256 < count ? idx[base + t * 256] : 0;
    T g[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) g[t] = x[c[t]];
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (base + t * 256 < count) acc += g[t];
  }
  if (acc == T(1.2345e30)) sink[0] = (double)acc;
}

__global__ __launch_bounds__(256) void k_probe_copy1(const double2* __restrict__ a,
                                                     double2* __restrict__ b, int64_t n2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n2) b[i] = a[i];
}

__global__ __launch_bounds__(256) void k_probe_copy(const double2* __restrict__ a,
                                                    double2* __restrict__ b, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (kProbeUnroll - 1) * stride < n2; i += kProbeUnroll * stride) {
    double2 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = a[i + u * stride];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) b[i + u * stride] = v[u];
  }
  for (; i < n2; i += stride) b[i] = a[i];
}

__global__ __launch_bounds__(256) void k_probe_triad(double2* __restrict__ a,
                                                     const double2* __restrict__ b,
                                                     const double2* __restrict__ c, double s,
                                                     int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (kProbeUnroll - 1) * stride < n2; i += kProbeUnroll * stride) {
    double2 bv[kProbeUnroll], cv[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) {
      bv[u] = b[i + u * stride];
      cv[u] = c[i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) {
      double2 r;
      r.x = bv[u].x + s * cv[u].x;
      r.y = bv[u].y + s * cv[u].y;
      a[i + u * stride] = r;
    }
  }
  for (; i < n2; i += stride) {
    double2 r;
    r.x = b[i].x + s * c[i].x;
    r.y = b[i].y + s * c[i].y;
    a[i] = r;
  }
}

__global__ __launch_bounds__(256) void k_fill(double2* __restrict__ a, int64_t n2, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) {
    double2 r;
    r.x = v;
    r.y = v + 1.0;
    a[i] = r;
  }
}

// a cache-evicting pass that only reads: the caches end up holding clean
// lines of the buffer, so the next kernel's misses evict them without
// write-backs (a writing pass would leave up to the Infinity Cache's size
// of dirty lines for the timed kernel to write back)
__global__ __launch_bounds__(256) void k_flush(double2* __restrict__ a, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) {
    const double2 r = a[i];
    s += r.x + r.y;
  }
  if (s == 1.2345e300) a[0].x = s;  // never true: keeps the reads
}

}  // namespace mxs

using namespace mxs;

extern "C" {

const char* mxs_version(void) { return "mxs 0.1.0 (gfx950)"; }

const char* mxs_status_string(mxs_status s) {
  switch (s) {
    case MXS_OK: return "MXS_OK";
    case MXS_INVALID_ARG: return "MXS_INVALID_ARG";
    case MXS_INVALID_MATRIX: return "MXS_INVALID_MATRIX";
    case MXS_UNSUPPORTED: return "MXS_UNSUPPORTED";
    case MXS_OOM: return "MXS_OOM";
    case MXS_HIP: return "MXS_HIP";
    case MXS_NOT_CONVERGED: return "MXS_NOT_CONVERGED";
    case MXS_BREAKDOWN: return "MXS_BREAKDOWN";
    case MXS_NONFINITE: return "MXS_NONFINITE";
    case MXS_BUDGET: return "MXS_BUDGET";
    case MXS_PENDING: return "MXS_PENDING";
    default: return "MXS_UNKNOWN";
  }
}

const char* mxs_last_error(const mxs_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

mxs_status mxs_ctx_create(int device, void* hip_stream, const mxs_allocator* alloc,
                          mxs_ctx** out) {
  if (!out) return MXS_INVALID_ARG;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return MXS_INVALID_ARG;
  }
  if (alloc && (!alloc->alloc || !alloc->free)) return MXS_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return MXS_HIP;
  mxs_ctx* ctx = new (std::nothrow) mxs_ctx();
  if (!ctx) return MXS_OOM;
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  if (alloc) {
    ctx->alloc.cb = *alloc;
    ctx->alloc.custom = true;
  }
  ctx->alloc.stream = hip_stream;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cus = prop.multiProcessorCount;
  if (!pinned_reserve(ctx, 4096)) {
    delete ctx;
    return MXS_OOM;
  }
  mxs_status st = noalloc_scratch_init(ctx);
  for (int i = 0; i < 2 && !st; ++i)
    if (hipEventCreateWithFlags(&ctx->poll_ev[i], hipEventDisableTiming) != hipSuccess)
      st = fail(ctx, MXS_HIP, "event creation failed");
  if (st) {
    for (hipEvent_t e : ctx->poll_ev)
      if (e) (void)hipEventDestroy(e);
    (void)hipHostFree(ctx->pinned);
    delete ctx;
    return st;
  }
  *out = ctx;
  return MXS_OK;
}

mxs_status mxs_ctx_destroy(mxs_ctx* ctx) {
  if (!ctx) return MXS_OK;
  (void)hipStreamSynchronize(ctx->stream);
  ctx->alloc.release(ctx->ws.ptr);
  ctx->alloc.release(ctx->spmv_ws.ptr);
  ctx->alloc.release(ctx->flush);
  for (hipEvent_t e : ctx->poll_ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
  return MXS_OK;
}

mxs_status mxs_ctx_set_stream(mxs_ctx* ctx, void* hip_stream) {
  if (!ctx) return MXS_INVALID_ARG;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->alloc.stream = hip_stream;
  return MXS_OK;
}

mxs_status mxs_ctx_synchronize(mxs_ctx* ctx) {
  if (!ctx) return MXS_INVALID_ARG;
  MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MXS_OK;
}

mxs_status mxs_hbm_probe(mxs_ctx* ctx, size_t bytes, int reps, mxs_bw_result* out) {
  if (!ctx || !out || bytes < (1u << 20) || reps < 1) return MXS_INVALID_ARG;
  MXS_HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int64_t n2 = (int64_t)(bytes / 16);
  const size_t nb = (size_t)n2 * 16;
  double2 *a = (double2*)ctx->alloc.alloc(nb), *b = (double2*)ctx->alloc.alloc(nb),
          *c = (double2*)ctx->alloc.alloc(nb);
  double* sink = (double*)ctx->alloc.alloc(64);
  mxs_status st = MXS_OK;
  if (!a || !b || !c || !sink) {
    st = fail(ctx, MXS_OOM, "hbm_probe: cannot allocate 3 x %zu bytes", nb);
  } else {
    const int grid = ctx->num_cus * 16;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    k_fill<<<grid, 256, 0, ctx->stream>>>(a, n2, 1.0);
    k_fill<<<grid, 256, 0, ctx->stream>>>(b, n2, 2.0);
    k_fill<<<grid, 256, 0, ctx->stream>>>(c, n2, 3.0);
    // each kernel in two launch shapes (a grid-stride loop over 16 blocks
    // per CU, and one element per thread); the faster one counts
    const unsigned one_shot = (unsigned)((n2 + 255) / 256);
    float best[3] = {1e30f, 1e30f, 1e30f};
    for (int r = 0; r < reps + 1; ++r) {
      for (int kk = 0; kk < 6; ++kk) {
        (void)hipEventRecord(e0, ctx->stream);
        if (kk == 0) k_probe_read<<<grid, 256, 0, ctx->stream>>>(a, n2, sink);
        if (kk == 1) k_probe_read1<false><<<one_shot, 256, 0, ctx->stream>>>(a, n2, sink);
        if (kk == 5) k_probe_read1<true><<<one_shot, 256, 0, ctx->stream>>>(a, n2, sink);
        if (kk == 2) k_probe_copy<<<grid, 256, 0, ctx->stream>>>(a, b, n2);
        if (kk == 3) k_probe_copy1<<<one_shot, 256, 0, ctx->stream>>>(a, b, n2);
        if (kk == 4) k_probe_triad<<<grid, 256, 0, ctx->stream>>>(a, b, c, 0.5, n2);
        (void)hipEventRecord(e1, ctx->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const int slot = kk < 2 || kk == 5 ? 0 : kk < 4 ? 1 : 2;
        if (r > 0 && ms < best[slot]) best[slot] = ms;  // first round is warm-up
      }
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) st = fail(ctx, MXS_HIP, "hbm_probe: %s", hipGetErrorString(err));
    const double gb = (double)nb / 1e9;
    out->read_gbs = gb / (best[0] * 1e-3);
    out->copy_gbs = 2.0 * gb / (best[1] * 1e-3);
    out->triad_gbs = 3.0 * gb / (best[2] * 1e-3);
    out->best_gbs = out->read_gbs;
    if (out->copy_gbs > out->best_gbs) out->best_gbs = out->copy_gbs;
    if (out->triad_gbs > out->best_gbs) out->best_gbs = out->triad_gbs;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  (void)hipStreamSynchronize(ctx->stream);
  ctx->alloc.release(a);
  ctx->alloc.release(b);
  ctx->alloc.release(c);
  ctx->alloc.release(sink);
  return st;
}

mxs_status mxs_gather_probe(mxs_ctx* ctx, int64_t nx, int64_t count, int value_bytes, int reps,
                            double* gathers_per_s) {
  if (!ctx || !gathers_per_s || nx < 1 || nx > INT32_MAX || count < 1 || reps < 1 ||
      (value_bytes != 4 && value_bytes != 8))
    return MXS_INVALID_ARG;
  MXS_HIP_TRY(ctx, hipSetDevice(ctx->device));
  void* x = ctx->alloc.alloc((size_t)nx * value_bytes + 16);
  int32_t* idx = (int32_t*)ctx->alloc.alloc((size_t)count * 4 + 16);
  double* sink = (double*)ctx->alloc.alloc(64);
  mxs_status st = MXS_OK;
  if (!x || !idx || !sink) {
    st = fail(ctx, MXS_OOM, "gather_probe: cannot allocate %lld values and %lld indices",
              (long long)nx, (long long)count);
  } else {
    const int grid = ctx->num_cus * 16;
    const int64_t n2 = (int64_t)((size_t)nx * value_bytes / 16);
    if (n2 > 0) k_fill<<<grid, 256, 0, ctx->stream>>>((double2*)x, n2, 1.0);
    k_fill_random_index<<<grid, 256, 0, ctx->stream>>>(idx, count, nx);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 1e30f;
    for (int r = 0; r < reps + 1; ++r) {  // first run is warm-up
      (void)hipEventRecord(e0, ctx->stream);
      if (value_bytes == 8)
        k_probe_gather<double><<<grid, 256, 0, ctx->stream>>>(idx, (const double*)x, count, sink);
      else
        k_probe_gather<float><<<grid, 256, 0, ctx->stream>>>(idx, (const float*)x, count, sink);
      (void)hipEventRecord(e1, ctx->stream);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (r > 0 && ms < best) best = ms;
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) st = fail(ctx, MXS_HIP, "gather_probe: %s", hipGetErrorString(err));
    *gathers_per_s = (double)count / (best * 1e-3);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  (void)hipStreamSynchronize(ctx->stream);
  ctx->alloc.release(x);
  ctx->alloc.release(idx);
  ctx->alloc.release(sink);
  return st;
}

mxs_status mxs_flush_cache(mxs_ctx* ctx, size_t bytes) {
  if (!ctx) return MXS_INVALID_ARG;
  if (bytes < 4096) bytes = 4096;
  if (ctx->flush_bytes < bytes) {
    if (ctx->flush) {
      MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      ctx->alloc.release(ctx->flush);
    }
    ctx->flush = ctx->alloc.alloc(bytes);
    ctx->flush_bytes = ctx->flush ? bytes : 0;
    if (!ctx->flush) return fail(ctx, MXS_OOM, "flush_cache: cannot allocate %zu bytes", bytes);
    k_fill<<<ctx->num_cus * 16, 256, 0, ctx->stream>>>((double2*)ctx->flush,
                                                       (int64_t)(bytes / 16), 0.0);
  }
  k_flush<<<ctx->num_cus * 16, 256, 0, ctx->stream>>>((double2*)ctx->flush,
                                                      (int64_t)(bytes / 16));
  MXS_HIP_TRY(ctx, hipGetLastError());
  return MXS_OK;
}

}  // extern "C"
