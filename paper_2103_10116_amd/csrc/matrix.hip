// matrix.hip -- CSR ingest (validation on the GPU), format conversions and
// value casts on the GPU, export and bookkeeping.
//
// The O(n) analysis of the row pointers (row-length maximum and histogram,
// the SpMV work partition, empty-row lists, overflow offsets of the hybrid
// format) runs on the host from one copy of rowptr, as an analysis phase;
// every O(nnz) pass -- validation of the column indices, the layout
// transforms and the value casts -- runs on the GPU.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "common.h"

namespace mxs {

void* mat_alloc(mxs_matrix* A, size_t bytes) {
  void* p = A->alloc.alloc(bytes);
  if (p) {
    A->owned.push_back(p);
    A->bytes += (int64_t)bytes;
  }
  return p;
}

// Greedy row-block partition: consecutive rows are packed while the block
// holds at most `C` entries and `C` rows; a row longer than C is a block of
// its own.  Returns the block count; blocks[b]..blocks[b+1] are the rows.
int64_t csr_partition(const int32_t* rp, int64_t n, int C, std::vector<int32_t>& blocks,
                      int64_t max_rows) {
  if (max_rows < 0) max_rows = C;
  blocks.clear();
  blocks.push_back(0);
  int64_t cur_nnz = 0, cur_rows = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t L = (int64_t)rp[i + 1] - rp[i];
    if (L > C) {
      if (cur_rows) blocks.push_back((int32_t)i);
      blocks.push_back((int32_t)(i + 1));
      cur_nnz = cur_rows = 0;
      continue;
    }
    if (cur_rows && (cur_nnz + L > C || cur_rows + 1 > max_rows)) {
      blocks.push_back((int32_t)i);
      cur_nnz = cur_rows = 0;
    }
    cur_nnz += L;
    cur_rows += 1;
  }
  if (cur_rows) blocks.push_back((int32_t)n);
  return (int64_t)blocks.size() - 1;
}

namespace {

constexpr int kErrRowptr = 1, kErrCol = 2, kErrRange = 4, kErrNonfinite = 8, kErrOrder = 16;

int grid_for(mxs_ctx* ctx, int64_t work, int bs) {
  int64_t g = (work + bs - 1) / bs;
  const int64_t cap = (int64_t)ctx->num_cus * 32;
  if (g > cap) g = cap;
  return (int)(g < 1 ? 1 : g);
}

// ---- validation ------------------------------------------------------------
__global__ void k_check_rowptr(int64_t n, int64_t nnz, const int32_t* __restrict__ rp,
                               int* __restrict__ err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride) {
    const int32_t v = rp[i];
    bool bad = v < 0 || (int64_t)v > nnz;
    if (i == 0) bad |= v != 0;
    if (i == n) bad |= (int64_t)v != nnz;
    if (i < n) bad |= rp[i + 1] < v;
    if (bad) atomicOr(err, kErrRowptr);
  }
}

// one thread per row; only launched once the row pointers passed.  A column
// outside [0, ncols) sets kErrCol; a row whose columns do not ascend
// strictly sets kErrOrder and, when `disorder` is given, its flag there.
__global__ void k_check_cols(int64_t n, int64_t ncols, const int32_t* __restrict__ rp,
                             const int32_t* __restrict__ col, int* __restrict__ err,
                             uint8_t* __restrict__ disorder) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    int64_t prev = -1;
    bool unordered = false;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int64_t c = col[k];
      if (c < 0 || c >= ncols) {
        atomicOr(err, kErrCol);
        break;
      }
      unordered |= c <= prev;
      prev = c;
    }
    if (unordered) atomicOr(err, kErrOrder);
    if (disorder) disorder[i] = unordered ? 1 : 0;
  }
}

// ---- ingest of unordered rows: sort by column, sum repeats -----------------
// A row's entries are ordered by the 64-bit key (column << 32 | position in
// the row): a total order, so the sort is stable by construction and equal
// columns keep their input order.  Bitonic sort over the next power of two
// (padding keys ~0 sort last); `nt` threads of one work-group, a barrier
// after every compare-exchange step.
__device__ void bitonic_sort(uint64_t* s, int64_t P2, int tid, int nt) {
  for (int64_t k = 2; k <= P2; k <<= 1) {
    for (int64_t j = k >> 1; j > 0; j >>= 1) {
      for (int64_t t = tid; t < P2 / 2; t += nt) {
        const int64_t lo = 2 * j * (t / j) + (t % j), hi = lo + j;
        const bool up = (lo & k) == 0;
        const uint64_t a = s[lo], b = s[hi];
        if ((a > b) == up) {
          s[lo] = b;
          s[hi] = a;
        }
      }
      __syncthreads();
    }
  }
}

// distinct columns among a row's L sorted keys, summed over the work-group
__device__ int32_t count_heads(const uint64_t* s, int64_t L, int tid, int nt, int32_t* red) {
  int32_t h = 0;
  for (int64_t t = tid; t < L; t += nt) h += (t == 0 || (s[t] >> 32) != (s[t - 1] >> 32));
  h = wave_sum(h);
  if ((tid & 63) == 0) red[tid >> 6] = h;
  __syncthreads();
  int32_t tot = 0;
  for (int w = 0; w < nt / 64; ++w) tot += red[w];
  return tot;
}

constexpr int kSortLds = 2048;  // rows up to this length are sorted in LDS

// one work-group of 256 threads per listed row (2 <= length <= kSortLds):
// sort in LDS, write the sorted keys over the row's slots, count its columns
__global__ __launch_bounds__(256) void k_sort_rows_lds(const int32_t* __restrict__ rows,
                                                       const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col,
                                                       uint64_t* __restrict__ keys,
                                                       int32_t* __restrict__ cnt) {
  __shared__ uint64_t s[kSortLds];
  __shared__ int32_t red[4];
  const int32_t i = rows[blockIdx.x];
  const int32_t b = rp[i];
  const int64_t L = rp[i + 1] - b;
  int64_t P2 = 1;
  while (P2 < L) P2 <<= 1;
  for (int64_t t = threadIdx.x; t < P2; t += 256)
    s[t] = t < L ? ((uint64_t)(uint32_t)col[b + t] << 32) | (uint64_t)t : ~0ull;
  __syncthreads();
  bitonic_sort(s, P2, threadIdx.x, 256);
  for (int64_t t = threadIdx.x; t < L; t += 256) keys[b + t] = s[t];
  const int32_t h = count_heads(s, L, threadIdx.x, 256, red);
  if (threadIdx.x == 0) cnt[i] = h;
}

// one longer row by one work-group of 1024 threads in global memory
// (tmp holds P2 keys; a work-group's barrier orders its global accesses)
__global__ __launch_bounds__(1024) void k_sort_row_global(int32_t i, const int32_t* __restrict__ rp,
                                                          const int32_t* __restrict__ col,
                                                          uint64_t* __restrict__ tmp, int64_t P2,
                                                          uint64_t* __restrict__ keys,
                                                          int32_t* __restrict__ cnt) {
  __shared__ int32_t red[16];
  const int32_t b = rp[i];
  const int64_t L = rp[i + 1] - b;
  for (int64_t t = threadIdx.x; t < P2; t += 1024)
    tmp[t] = t < L ? ((uint64_t)(uint32_t)col[b + t] << 32) | (uint64_t)t : ~0ull;
  __syncthreads();
  bitonic_sort(tmp, P2, threadIdx.x, 1024);
  for (int64_t t = threadIdx.x; t < L; t += 1024) keys[b + t] = tmp[t];
  const int32_t h = count_heads(tmp, L, threadIdx.x, 1024, red);
  if (threadIdx.x == 0) cnt[i] = h;
}

// New CSR arrays: one wave per row.  Rows in order are copied; a sorted row
// keeps one entry per distinct column, whose value is the sum of that
// column's values in input order (sorted keys of equal column hold
// ascending input positions), added left to right by the lane that holds
// the column's first key.  vpe = doubles per value (2: complex, parts
// summed separately).
__global__ __launch_bounds__(256) void k_compact_rows(int64_t n, const int32_t* __restrict__ rp,
                                                      const int32_t* __restrict__ nrp,
                                                      const uint8_t* __restrict__ disorder,
                                                      const int32_t* __restrict__ col,
                                                      const double* __restrict__ val, int vpe,
                                                      const uint64_t* __restrict__ keys,
                                                      int32_t* __restrict__ ocol,
                                                      double* __restrict__ oval) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += nw) {
    const int64_t b = rp[i], L = rp[i + 1] - b, ob = nrp[i];
    if (!disorder[i]) {
      for (int64_t t = lane; t < L; t += 64) {
        ocol[ob + t] = col[b + t];
        for (int q = 0; q < vpe; ++q) oval[(ob + t) * vpe + q] = val[(b + t) * vpe + q];
      }
      continue;
    }
    int64_t base = 0;
    for (int64_t t0 = 0; t0 < L; t0 += 64) {
      const int64_t t = t0 + lane;
      bool head = false;
      uint64_t k = 0;
      if (t < L) {
        k = keys[b + t];
        head = t == 0 || (keys[b + t - 1] >> 32) != (k >> 32);
      }
      const uint64_t mask = __ballot(head);
      const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
      if (head) {
        const int64_t pos = ob + base + __popcll(mask & below);
        const uint32_t c = (uint32_t)(k >> 32);
        double s0 = val[(b + (int64_t)(uint32_t)k) * vpe];
        double s1 = vpe == 2 ? val[(b + (int64_t)(uint32_t)k) * vpe + 1] : 0.0;
        for (int64_t u = t + 1; u < L; ++u) {
          const uint64_t k2 = keys[b + u];
          if ((uint32_t)(k2 >> 32) != c) break;
          const int64_t src = (b + (int64_t)(uint32_t)k2) * vpe;
          s0 = s0 + val[src];
          if (vpe == 2) s1 = s1 + val[src + 1];
        }
        ocol[pos] = (int32_t)c;
        oval[pos * vpe] = s0;
        if (vpe == 2) oval[pos * vpe + 1] = s1;
      }
      base += __popcll(mask);
    }
  }
}

// ---- value casts -----------------------------------------------------------
template <typename V>
__device__ __forceinline__ V cast_val(double v, int* err);

template <>
__device__ __forceinline__ double cast_val<double>(double v, int*) {
  return v;
}

template <>
__device__ __forceinline__ float cast_val<float>(double v, int* err) {
  const float f = (float)v;  // v_cvt_f32_f64: round to nearest even
  if (isfinite(v) && !isfinite(f)) atomicOr(err, kErrRange);
  return f;
}

template <typename V>
__global__ void k_cast(int64_t count, const double* __restrict__ in, V* __restrict__ out,
                       int* __restrict__ err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride)
    out[k] = cast_val<V>(in[k], err);
}

// binary16 code of a double, rounded to nearest even, by integer arithmetic
// on the IEEE fields (1 sign, 5 exponent bits biased by 15, 10 fraction
// bits; subnormals are multiples of 2^-24)
__device__ __forceinline__ uint16_t f64_to_f16_bits(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint16_t sign = (uint16_t)((b >> 48) & 0x8000u);
  const int ex = (int)((b >> 52) & 0x7ff);
  const uint64_t frac = b & 0xFFFFFFFFFFFFFull;
  if (ex == 0x7ff) return (uint16_t)(sign | (frac ? 0x7e00u : 0x7c00u));
  if (ex == 0) return sign;  // double subnormal or zero: far below half's range
  int e = ex - 1023;
  const uint64_t m = frac | (1ull << 52);  // 53-bit significand
  if (e > 15) return (uint16_t)(sign | 0x7c00u);
  int shift = (e >= -14) ? 42 : 42 + (-14 - e);  // bits dropped below the half ulp
  if (shift > 53) return sign;                   // below 2^-25: rounds to 0
  uint64_t q = m >> shift;
  const uint64_t rem = m & ((1ull << shift) - 1);
  const uint64_t half = 1ull << (shift - 1);
  if (rem > half || (rem == half && (q & 1))) q += 1;
  if (e >= -14) {
    if (q == 2048) {
      q = 1024;
      e += 1;
      if (e > 15) return (uint16_t)(sign | 0x7c00u);
    }
    return (uint16_t)(sign | (uint16_t)(((e + 15) << 10) | (int)(q - 1024)));
  }
  return (uint16_t)(sign | (uint16_t)q);  // subnormal, or 1024 = smallest normal
}

// one thread per row: power-of-two scale 2^ceil(log2 max|a|) and codes
__global__ void k_rowscale_f16(int64_t n, const int32_t* __restrict__ rp,
                               const double* __restrict__ val, uint16_t* __restrict__ h,
                               float* __restrict__ scale, int* __restrict__ err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int32_t a = rp[i], e = rp[i + 1];
    double m = 0.0;
    for (int32_t k = a; k < e; ++k) {
      const double v = val[k];
      if (!isfinite(v)) atomicOr(err, kErrNonfinite);
      m = fmax(m, fabs(v));
    }
    int E = 0;
    if (m > 0.0) {
      const uint64_t bits = (uint64_t)__double_as_longlong(m);
      const int ex = (int)((bits >> 52) & 0x7ff);
      const bool pow2 = (bits & 0xFFFFFFFFFFFFFull) == 0;
      E = ex - 1023 + (pow2 ? 0 : 1);
      if (ex == 0 || E > 127 || E < -126) {
        atomicOr(err, kErrRange);
        E = 0;
      }
    }
    scale[i] = ldexpf(1.0f, E);
    for (int32_t k = a; k < e; ++k) h[k] = f64_to_f16_bits(ldexp(val[k], -E));
  }
}

// ---- layout transforms -----------------------------------------------------
__global__ void k_coo_rows(int64_t n, const int32_t* __restrict__ rp, int32_t* __restrict__ row) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) row[k] = (int32_t)i;
}

template <typename V>
__global__ void k_fill_ell(int64_t n, int64_t K, int64_t ldk, const int32_t* __restrict__ rp,
                           const int32_t* __restrict__ col, const double* __restrict__ val,
                           int32_t* __restrict__ ecol, V* __restrict__ eval,
                           int* __restrict__ err) {
  const int64_t total = K * ldk;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < total; s += stride) {
    const int64_t j = s / ldk, i = s - j * ldk;
    int32_t c = -1;
    V v = (V)0;  // padding: column -1, value +0
    if (i < n) {
      const int32_t a = rp[i];
      if (j < (int64_t)(rp[i + 1] - a)) {
        c = col[a + j];
        v = cast_val<V>(val[a + j], err);
      }
    }
    ecol[s] = c;
    eval[s] = v;
  }
}

// hybrid overflow: entries K.. of each row, to offsets off[i]
template <typename V>
__global__ void k_fill_hyb_coo(int64_t n, int64_t K, const int32_t* __restrict__ rp,
                               const int32_t* __restrict__ col, const double* __restrict__ val,
                               const int64_t* __restrict__ off, int32_t* __restrict__ crow,
                               int32_t* __restrict__ ccol, V* __restrict__ cval,
                               int* __restrict__ err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    int64_t d = off[i];
    for (int64_t k = (int64_t)rp[i] + K; k < (int64_t)rp[i + 1]; ++k, ++d) {
      crow[d] = (int32_t)i;
      ccol[d] = col[k];
      cval[d] = cast_val<V>(val[k], err);
    }
  }
}

// ---- column panels of the merge path ---------------------------------------
// Entries of row i per column slice [p*W, (p+1)*W): a row's columns ascend,
// so each slice boundary is found by binary search.
__global__ void k_panel_counts(int64_t n, int P, int64_t W, const int32_t* __restrict__ rp,
                               const int32_t* __restrict__ col, int32_t* __restrict__ cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int32_t e = rp[i + 1];
    int32_t prev = rp[i];
    for (int p = 0; p < P; ++p) {
      int32_t lo = prev, hi = e;
      if (p < P - 1) {
        const int64_t lim = (int64_t)(p + 1) * W;
        while (lo < hi) {
          const int32_t mid = lo + (hi - lo) / 2;
          if ((int64_t)col[mid] < lim) lo = mid + 1;
          else hi = mid;
        }
      } else {
        lo = e;
      }
      cnt[(int64_t)p * n + i] = lo - prev;
      prev = lo;
    }
  }
}

// Copies each row's entries of slice p to its stacked row (dst[p*n + i]);
// E is the raw value word (8, 4 or 2 bytes), copied bit for bit.
template <typename E>
__global__ void k_panel_scatter(int64_t n, int P, const int32_t* __restrict__ rp,
                                const int32_t* __restrict__ cnt, const int32_t* __restrict__ dst,
                                const int32_t* __restrict__ col, const E* __restrict__ val,
                                int32_t* __restrict__ scol, E* __restrict__ sval) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    int32_t k = rp[i];
    for (int p = 0; p < P; ++p) {
      const int32_t c = cnt[(int64_t)p * n + i];
      const int32_t d = dst[(int64_t)p * n + i];
      for (int32_t t = 0; t < c; ++t) {
        scol[d + t] = col[k + t];
        sval[d + t] = val[k + t];
      }
      k += c;
    }
  }
}

// Row index of every entry of the panel-ordered COO arrays: entries
// srowptr[r] .. srowptr[r+1]-1 belong to stacked row r, output index srid[r].
__global__ void k_coo_stacked_rows(int64_t m, const int32_t* __restrict__ srowptr,
                                   const int32_t* __restrict__ srid,
                                   int32_t* __restrict__ row) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += stride) {
    const int32_t v = srid[r];
    for (int32_t k = srowptr[r]; k < srowptr[r + 1]; ++k) row[k] = v;
  }
}

// Copies the current values into the panel copy again, one thread per
// stacked row r (row i = srid[r] % n of panel p = srid[r] / n): the slice's
// first entry in row i is found by binary search, as at set-up.
template <typename E>
__global__ void k_panel_refresh(int64_t m, int64_t n, int64_t W,
                                const int32_t* __restrict__ srowptr,
                                const int32_t* __restrict__ srid, const int32_t* __restrict__ rp,
                                const int32_t* __restrict__ col, const E* __restrict__ val,
                                E* __restrict__ sval) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += stride) {
    const int64_t f = srid[r], p = f / n, i = f - p * n;
    int32_t lo = rp[i], hi = rp[i + 1];
    const int64_t lim = p * W;
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo) / 2;
      if ((int64_t)col[mid] < lim) lo = mid + 1;
      else hi = mid;
    }
    for (int32_t d = srowptr[r], e = srowptr[r + 1]; d < e; ++d, ++lo) sval[d] = val[lo];
  }
}

// ---- helpers ---------------------------------------------------------------
mxs_status read_err(mxs_ctx* ctx, int* d_err, int* out) {
  MXS_HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, d_err, sizeof(int), hipMemcpyDeviceToHost,
                                  ctx->stream));
  MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  *out = *(int*)ctx->pinned;
  return MXS_OK;
}

mxs_matrix* new_matrix(mxs_ctx* ctx) {
  mxs_matrix* A = new (std::nothrow) mxs_matrix();
  if (A) {
    A->device = ctx->device;
    A->alloc = ctx->alloc;
  }
  return A;
}

void free_matrix(mxs_matrix* A) {
  if (!A) return;
  (void)hipSetDevice(A->device);
  for (void* p : A->owned) A->alloc.release(p);
  delete A;
}

// the SpMV kernels are instantiated for 256, 512 and 1024 entries per wave
int clamp_block_nnz(int v) {
  if (v <= 0) return 512;
  if (v <= 256) return 256;
  if (v <= 512) return 512;
  return 1024;
}

// Uploads a host array into matrix-owned device memory.
template <typename T>
T* upload(mxs_ctx* ctx, mxs_matrix* A, const std::vector<T>& h) {
  T* d = (T*)mat_alloc(A, h.size() * sizeof(T) + 16);
  if (d && !h.empty())
    if (hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, ctx->stream) !=
        hipSuccess)
      return nullptr;
  return d;
}

// Merge-path partition: equal chunks of C entries, the row of each chunk's
// first entry (and of the last entry overall), continuation scratch and the
// list of empty rows.  A chunk's rows must fit its LDS table of C + 2 row
// pointers, which long runs of empty rows can break.
int merge_chunk(const mxs_convert_opts* opts) {
  return opts && opts->block_nnz > 0
             ? (opts->block_nnz <= 256 ? 256 : opts->block_nnz <= 512 ? 512 : 1024)
             : 512;
}

// The row of each chunk's first entry (crow[nchunks]: the row of the last
// entry); false when some chunk's rows outgrow its table of C + 2 pointers.
bool merge_rows(const std::vector<int32_t>& rp, int64_t nnz, int C, std::vector<int32_t>& crow,
                int64_t* bad_chunk) {
  const int64_t nchunks = (nnz + C - 1) / C;
  crow.assign((size_t)nchunks + 1, 0);
  int64_t r = 0;
  for (int64_t c = 0; c < nchunks; ++c) {
    while (rp[r + 1] <= c * C) ++r;
    crow[c] = (int32_t)r;
  }
  if (nnz > 0) {
    while (rp[r + 1] <= nnz - 1) ++r;
    crow[nchunks] = (int32_t)r;
  }
  for (int64_t c = 0; c < nchunks; ++c)
    if (crow[c + 1] - crow[c] + 1 > C + 1) {
      *bad_chunk = c;
      return false;
    }
  return true;
}

// Column panels for the merge path: the caller's choice, else (auto) panels
// when x (ncols values of the compute type) exceeds 4 MiB, P the smallest
// power of two that cuts it into slices of at most 2 MiB.  Random gathers
// from x run near the L2's request rate only while each XCD's slice of x
// stays in its 4 MB L2 (gathers from an 8 MiB x: 107e9/s; 4 MiB: 196e9/s;
// 2 MiB: 226e9/s).  Measured on the 2^20 power-law matrices (cold / warm):
// FP64 s = 1.79 197 / 197 us without panels, 145 / 136 with 4; random SPD
// 133 / 133 vs 138 / 107; FP32 (x of 4 MiB) gains nothing (s = 2.0 57 / 53
// vs 63 / 55 with 2).  Stacked rows are indexed by p*n + i in int32.
int merge_panels(const mxs_matrix* A, const mxs_convert_opts* opts) {
  const int req = opts ? opts->col_panels : 0;
  if (req == 1) return 1;
  const int64_t xb = A->ncols * (A->dt == MXS_F64 ? 8 : 4);
  int P = 1;
  if (req > 1) {
    P = req <= 2 ? 2 : req <= 4 ? 4 : 8;
  } else if (xb > (int64_t(4) << 20)) {
    while (P < 8 && (xb + P - 1) / P > (int64_t(2) << 20)) P <<= 1;
  }
  if (P > 1 && ((int64_t)P * A->n > INT32_MAX || A->ncols < P)) P = 1;
  return P;
}

// Stacked rows of the column panels (see CsrPart) and their chunk table.
mxs_status build_panels(mxs_ctx* ctx, mxs_matrix* A, int P, int C) {
  CsrPart& S = A->csr;
  const int64_t n = A->n, nnz = A->nnz;
  const int64_t W = (A->ncols + P - 1) / P;
  const size_t vb = value_bytes(A->dt);
  std::vector<int32_t> cnt((size_t)P * n), dst((size_t)P * n, -1), srp, srid, crow;
  std::vector<uint8_t> mask((size_t)n, 0);
  int32_t* d_cnt = (int32_t*)ctx->alloc.alloc((size_t)P * n * 4 + 4);
  int32_t* d_dst = (int32_t*)ctx->alloc.alloc((size_t)P * n * 4 + 4);
  mxs_status st = MXS_OK;
  do {
    if (!d_cnt || !d_dst) {
      st = fail(ctx, MXS_OOM, "column panels: counts");
      break;
    }
    k_panel_counts<<<grid_for(ctx, n, 256), 256, 0, ctx->stream>>>(n, P, W, S.rowptr, S.col,
                                                                     d_cnt);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(cnt.data(), d_cnt, (size_t)P * n * 4, hipMemcpyDeviceToHost,
                       ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "column panels: counting failed");
      break;
    }
    int64_t pos = 0;
    for (int p = 0; p < P; ++p)
      for (int64_t i = 0; i < n; ++i) {
        const int32_t c = cnt[(size_t)p * n + i];
        if (c == 0) continue;
        srid.push_back((int32_t)((int64_t)p * n + i));
        srp.push_back((int32_t)pos);
        dst[(size_t)p * n + i] = (int32_t)pos;
        mask[(size_t)i] |= (uint8_t)(1u << p);
        pos += c;
      }
    srp.push_back((int32_t)pos);
    int64_t bad = 0;
    if (pos != nnz || !merge_rows(srp, nnz, C, crow, &bad)) {
      st = fail(ctx, MXS_HIP, "column panels: inconsistent counts");
      break;
    }
    S.srowptr = upload(ctx, A, srp);
    S.srid = upload(ctx, A, srid);
    S.pmask = upload(ctx, A, mask);
    S.crow = upload(ctx, A, crow);
    // padded to whole 1024-entry chunks (zeros) for the COO chunks
    const size_t npad = (size_t)((nnz + 1023) / 1024 * 1024);
    S.scol = (int32_t*)mat_alloc(A, npad * 4 + 4);
    S.sval = mat_alloc(A, npad * vb + 16);
    if (vb != 2) S.srow = (int32_t*)mat_alloc(A, npad * 4 + 4);
    if (!S.srowptr || !S.srid || !S.pmask || !S.crow || !S.scol || !S.sval ||
        (vb != 2 && !S.srow)) {
      st = fail(ctx, MXS_OOM, "column panels");
      break;
    }
    if (hipMemsetAsync(S.scol, 0, npad * 4 + 4, ctx->stream) != hipSuccess ||
        hipMemsetAsync(S.sval, 0, npad * vb + 16, ctx->stream) != hipSuccess ||
        (S.srow && hipMemsetAsync(S.srow, 0, npad * 4 + 4, ctx->stream) != hipSuccess)) {
      st = fail(ctx, MXS_HIP, "column panels: clearing failed");
      break;
    }
    if (hipMemcpyAsync(d_dst, dst.data(), (size_t)P * n * 4, hipMemcpyHostToDevice,
                       ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "copy failed");
      break;
    }
    const int g = grid_for(ctx, n, 256);
    if (vb == 8)
      k_panel_scatter<uint64_t><<<g, 256, 0, ctx->stream>>>(
          n, P, S.rowptr, d_cnt, d_dst, S.col, (const uint64_t*)S.val, S.scol, (uint64_t*)S.sval);
    else if (vb == 4)
      k_panel_scatter<uint32_t><<<g, 256, 0, ctx->stream>>>(
          n, P, S.rowptr, d_cnt, d_dst, S.col, (const uint32_t*)S.val, S.scol, (uint32_t*)S.sval);
    else
      k_panel_scatter<uint16_t><<<g, 256, 0, ctx->stream>>>(
          n, P, S.rowptr, d_cnt, d_dst, S.col, (const uint16_t*)S.val, S.scol, (uint16_t*)S.sval);
    if (S.srow && !srid.empty())
      k_coo_stacked_rows<<<grid_for(ctx, (int64_t)srid.size(), 256), 256, 0, ctx->stream>>>(
          (int64_t)srid.size(), S.srowptr, S.srid, S.srow);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "column panels: scatter failed");
      break;
    }
    S.panels = P;
    S.nsrows = (int64_t)srid.size();
    S.merge = true;
    S.block_nnz = C;
    S.nchunks = (nnz + C - 1) / C;
    S.nblocks = S.nchunks;
    S.nempty = 0;  // the pass that adds the panels' partials writes every row
  } while (0);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->alloc.release(d_cnt);
  ctx->alloc.release(d_dst);
  return st;
}

}  // namespace

mxs_status refresh_panel_values(mxs_ctx* ctx, mxs_matrix* A) {
  const CsrPart& S = A->csr;
  if (A->fmt != MXS_CSR || !S.merge || S.panels <= 1 || S.nsrows == 0) return MXS_OK;
  const int64_t W = (A->ncols + S.panels - 1) / S.panels;
  const int g = grid_for(ctx, S.nsrows, 256);
  const size_t vb = value_bytes(A->dt);
  if (vb == 8)
    k_panel_refresh<uint64_t><<<g, 256, 0, ctx->stream>>>(S.nsrows, A->n, W, S.srowptr, S.srid,
                                                          S.rowptr, S.col,
                                                          (const uint64_t*)S.val,
                                                          (uint64_t*)S.sval);
  else if (vb == 4)
    k_panel_refresh<uint32_t><<<g, 256, 0, ctx->stream>>>(S.nsrows, A->n, W, S.srowptr, S.srid,
                                                          S.rowptr, S.col,
                                                          (const uint32_t*)S.val,
                                                          (uint32_t*)S.sval);
  else
    k_panel_refresh<uint16_t><<<g, 256, 0, ctx->stream>>>(S.nsrows, A->n, W, S.srowptr, S.srid,
                                                          S.rowptr, S.col,
                                                          (const uint16_t*)S.val,
                                                          (uint16_t*)S.sval);
  MXS_HIP_TRY(ctx, hipGetLastError());
  return MXS_OK;
}

namespace {

mxs_status build_csr_merge(mxs_ctx* ctx, mxs_matrix* A, const mxs_convert_opts* opts) {
  if (A->dt != MXS_F64 && A->dt != MXS_F32 && A->dt != MXS_F16_ROWSCALED)
    return fail(ctx, MXS_UNSUPPORTED,
                "the merge-path CSR kernel takes FP64, FP32 or row-scaled FP16 values");
  const std::vector<int32_t>& rp = A->h_rowptr;
  const int64_t n = A->n, nnz = A->nnz;
  const int C = merge_chunk(opts);
  // one wave per work-group unless asked (power law, cold: FP32 s = 2.0
  // 56.5 vs 58.0 us, s = 1.79 119.1 vs 119.5 us)
  A->csr.wpb = (opts && opts->waves_per_group > 1) ? 4 : 1;
  const int panels = merge_panels(A, opts);
  if (panels > 1 && nnz > 0) return build_panels(ctx, A, panels, C);
  std::vector<int32_t> crow, empty;
  int64_t bad = 0;
  if (!merge_rows(rp, nnz, C, crow, &bad))
    return fail(ctx, MXS_UNSUPPORTED,
                "merge-path CSR: chunk %lld spans %d rows (empty rows), more than %d",
                (long long)bad, crow[bad + 1] - crow[bad] + 1, C + 1);
  CsrPart& P = A->csr;
  P.merge = true;
  P.block_nnz = C;
  P.nchunks = (nnz + C - 1) / C;
  P.nblocks = P.nchunks;
  for (int64_t i = 0; i < n; ++i)
    if (rp[i + 1] == rp[i]) empty.push_back((int32_t)i);
  P.nempty = (int64_t)empty.size();
  P.crow = upload(ctx, A, crow);
  P.empty_rows = upload(ctx, A, empty);
  if (!P.crow || !P.empty_rows) return fail(ctx, MXS_OOM, "merge-path CSR set-up");
  // the host vectors are freed on return: the copies must finish first
  MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MXS_OK;
}

// Chooses the CSR kernel from the row lengths (or the caller's options) and
// builds the row-block partition the stream kernel needs.
mxs_status build_csr_partition(mxs_ctx* ctx, mxs_matrix* A, int block_nnz,
                               const mxs_convert_opts* opts = nullptr) {
  const std::vector<int32_t>& rp = A->h_rowptr;
  int64_t maxL = 0;
  for (int64_t i = 0; i < A->n; ++i) maxL = std::max<int64_t>(maxL, rp[i + 1] - rp[i]);
  const double mean = A->n ? (double)A->nnz / (double)A->n : 0.0;
  int G = 4;
  while (G < 64 && G < mean) G <<= 1;
  const int kind = opts ? opts->csr_kernel : MXS_CSR_AUTO;
  if (opts && opts->lanes_per_row > 0) {
    G = 1;
    while (G < 64 && G < opts->lanes_per_row) G <<= 1;
    if (G == 2) G = 4;
  }
  // AUTO: the row-block stream kernel when some row is longer than 64
  // entries (power-law rows); otherwise one of the two LDS kernels over
  // blocks of <= 64 rows.  Measured on the 128^3 stencils: rows from LDS for
  // 4- and 2-byte values (27-point FP32 98 vs 117 us for products, FP16 83
  // vs 132 us, 7-point FP32 27 vs 34 us) and for FP64 rows of at most 8
  // entries (7-point 36.8 vs 39.1 us); products otherwise (27-point FP64 146
  // vs 150 us, complex values), whose LDS holds one value per entry instead
  // of a value and an index.
  int kind_eff = kind;
  if (kind == MXS_CSR_AUTO) {
    const bool narrow = A->dt == MXS_F32 || A->dt == MXS_F16_ROWSCALED;
    kind_eff = maxL > 64                             ? MXS_CSR_STREAM
               : (narrow || (A->dt == MXS_F64 && maxL <= 8)) ? MXS_CSR_ROWS_LDS
                                                             : MXS_CSR_PRODUCTS;
    // rows over 64 entries (power law): the merge path for FP64/FP32 values
    // when every chunk's rows fit its table (cold, 2^20 rows: s = 2.0 FP32
    // 56.5 vs 65.6 us for the row-block stream kernel, FP64 84.8 vs 90.8;
    // s = 1.79 FP32 119.1 vs 134.5, FP64 198.3 vs 201.5)
    // (with column panels the stacked rows are never empty, so every chunk
    // fits its table)
    std::vector<int32_t> crow;
    int64_t bad = 0;
    if (maxL > 64 && (A->dt == MXS_F64 || A->dt == MXS_F32 || A->dt == MXS_F16_ROWSCALED) &&
        (merge_panels(A, opts) > 1 || merge_rows(rp, A->nnz, merge_chunk(opts), crow, &bad)))
      kind_eff = MXS_CSR_MERGE;
  }
  if (kind_eff == MXS_CSR_MERGE) return build_csr_merge(ctx, A, opts);
  bool vec = kind_eff == MXS_CSR_VECTOR;
  A->csr.lanes = vec ? G : 0;
  A->csr.wpb = (opts && opts->waves_per_group == 1) ? 1 : 4;
  if (kind_eff == MXS_CSR_PRODUCTS)
    A->csr.wpb = (opts && opts->waves_per_group > 0)
                     ? (opts->waves_per_group == 1 ? 1 : opts->waves_per_group == 2 ? 2 : 4)
                     : 2;
  int rpg = (opts && opts->rows_per_group > 0) ? opts->rows_per_group : (G >= 8 ? 8 : 4);
  A->csr.rpg = rpg <= 2 ? 2 : rpg <= 4 ? 4 : 8;
  if (A->csr.rpg > G) A->csr.rpg = G;
  std::vector<int32_t> blocks, bnnz;
  A->csr.rows_lds = kind_eff == MXS_CSR_ROWS_LDS;
  A->csr.products = kind_eff == MXS_CSR_PRODUCTS;
  A->csr.rl_lanes = 1;
  int max_rows = -1;
  if (A->csr.rows_lds || A->csr.products) {
    // LDS-kernel blocks: at most 64 rows; entry budget 64 * (longest row)
    // rounded up to 512 or 1024 (2048 only on request: its LDS footprint
    // halves the waves per CU); rows longer than it get a wave of their own
    const int64_t want = 64 * std::max<int64_t>(maxL, 1);
    block_nnz = A->csr.products || want <= 512 ? 512 : 1024;
    if (opts && opts->block_nnz > 0) block_nnz = opts->block_nnz <= 512 ? 512
                                                : opts->block_nnz <= 1024 ? 1024 : 2048;
    max_rows = 64;
    if (A->csr.rows_lds) {
      // lanes per row: the fewest that fill the wave when 64/G rows of the
      // longest length fit the entry budget (or the caller's 1, 2 or 4)
      int g = 1;
      if (opts && opts->lanes_per_row > 0)
        g = opts->lanes_per_row >= 4 ? 4 : opts->lanes_per_row >= 2 ? 2 : 1;
      else
        while (g < 4 && (64 / g) * std::max<int64_t>(maxL, 1) > block_nnz) g <<= 1;
      A->csr.rl_lanes = g;
      // a lane's share of the longest row in one step when it exceeds 8
      A->csr.rl_step = (std::max<int64_t>(maxL, 1) + g - 1) / g > 8 ? 16 : 8;
      max_rows = 64 / g;
    }
  } else if (kind == MXS_CSR_AUTO && !(opts && opts->block_nnz > 0)) {
    block_nnz = 1024;
  }
  A->csr.block_nnz = block_nnz;
  A->csr.nblocks = csr_partition(rp.data(), A->n, block_nnz, blocks, max_rows);
  bnnz.resize(blocks.size());
  for (size_t b = 0; b < blocks.size(); ++b) bnnz[b] = rp[blocks[b]];
  A->csr.blocks = upload(ctx, A, blocks);
  A->csr.bnnz = upload(ctx, A, bnnz);
  if (!A->csr.blocks || !A->csr.bnnz)
    return fail(ctx, MXS_OOM, "cannot upload the row-block partition");
  // the host vectors are freed on return: the copies must finish first
  MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MXS_OK;
}

// maxlen (the most entries a row has in the part) and vb (value bytes)
// choose the AUTO kernel
mxs_status setup_coo_part(mxs_ctx* ctx, mxs_matrix* A, mxs::CooPart& P, int64_t nnz,
                          int64_t maxlen, size_t vb, int block_nnz,
                          const std::vector<int32_t>& empty, const mxs_convert_opts* opts) {
  const int wpb = opts ? opts->waves_per_group : 0;
  const int kind = opts ? opts->coo_kernel : MXS_COO_AUTO;
  P.wpb = wpb == 1 ? 1 : 4;
  // Runs wholly in registers win only for 4-byte values on short rows
  // (7-point stencil FP32: 37.1 vs 39.0 us; FP64: 48.5 vs 46.6).  With longer
  // rows a lane's run holds one row's entries at scattered offsets, whose
  // gathers touch more cache lines than the LDS kernel's coalesced ones
  // (27-point FP64 194 vs 187 us; power law s = 2.0, cold, 91 vs 89 us).
  P.kernel = kind == MXS_COO_LDS || kind == MXS_COO_RUNS ? kind
             : (vb <= 4 && maxlen <= 16)                 ? MXS_COO_RUNS
                                                         : MXS_COO_LDS;
  P.nnz = nnz;
  P.block_nnz = block_nnz;
  P.nchunks = (nnz + block_nnz - 1) / block_nnz;
  P.nempty = (int64_t)empty.size();
  P.empty_rows = upload(ctx, A, empty);
  if (!P.empty_rows) return fail(ctx, MXS_OOM, "coo setup");
  MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MXS_OK;
}

template <typename V>
mxs_status cast_into(mxs_ctx* ctx, int64_t count, const double* in, void* out, int* d_err) {
  if (count == 0) return MXS_OK;
  if (sizeof(V) == sizeof(double)) {
    MXS_HIP_TRY(ctx, hipMemcpyAsync(out, in, count * sizeof(double), hipMemcpyDeviceToDevice,
                                    ctx->stream));
    return MXS_OK;
  }
  k_cast<V><<<grid_for(ctx, count, 256), 256, 0, ctx->stream>>>(count, in, (V*)out, d_err);
  MXS_HIP_TRY(ctx, hipGetLastError());
  return MXS_OK;
}

// COO arrays of nnz entries, allocated to a whole number of the largest
// chunk (1024 entries) with the padding zeroed (row 0, column 0, value 0), so
// a kernel may load every chunk in full; padded entries are never summed.
mxs_status alloc_coo_arrays(mxs_ctx* ctx, mxs_matrix* A, mxs::CooPart& P, int64_t nnz,
                            size_t vb) {
  const int64_t cap = (nnz + 1023) / 1024 * 1024;
  const int64_t slots = cap > 0 ? cap : 1;
  P.row = (int32_t*)mat_alloc(A, (size_t)slots * 4);
  P.col = (int32_t*)mat_alloc(A, (size_t)slots * 4);
  P.val = mat_alloc(A, (size_t)slots * vb);
  if (!P.row || !P.col || !P.val) return fail(ctx, MXS_OOM, "coo arrays");
  const int64_t pad = slots - nnz;
  MXS_HIP_TRY(ctx, hipMemsetAsync(P.row + nnz, 0, (size_t)pad * 4, ctx->stream));
  MXS_HIP_TRY(ctx, hipMemsetAsync(P.col + nnz, 0, (size_t)pad * 4, ctx->stream));
  MXS_HIP_TRY(ctx, hipMemsetAsync((char*)P.val + (size_t)nnz * vb, 0, (size_t)pad * vb,
                                  ctx->stream));
  return MXS_OK;
}

// COO arrays in panel order (see CooPart) from the FP64 CSR source S: the
// entries counted per row and panel, placed by the merge path's scatter
// (FP64 values, cast afterwards), and each given its stacked output index.
template <typename V>
mxs_status build_coo_panels(mxs_ctx* ctx, const mxs_matrix* S, mxs_matrix* A, int P,
                            int* d_err) {
  CooPart& C = A->coo;
  const int64_t n = S->n, nnz = S->nnz;
  const int64_t W = (S->ncols + P - 1) / P;
  std::vector<int32_t> cnt((size_t)P * n), dst((size_t)P * n, -1), srp, srid;
  std::vector<uint8_t> mask((size_t)n, 0);
  int32_t* d_cnt = (int32_t*)ctx->alloc.alloc((size_t)P * n * 4 + 4);
  int32_t* d_dst = (int32_t*)ctx->alloc.alloc((size_t)P * n * 4 + 4);
  int32_t* d_srp = nullptr;
  int32_t* d_srid = nullptr;
  double* v64 = sizeof(V) == 8 ? (double*)C.val : (double*)ctx->alloc.alloc((size_t)nnz * 8 + 8);
  mxs_status st = MXS_OK;
  do {
    if (!d_cnt || !d_dst || !v64) {
      st = fail(ctx, MXS_OOM, "COO column panels: counts");
      break;
    }
    k_panel_counts<<<grid_for(ctx, n, 256), 256, 0, ctx->stream>>>(n, P, W, S->csr.rowptr,
                                                                     S->csr.col, d_cnt);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(cnt.data(), d_cnt, (size_t)P * n * 4, hipMemcpyDeviceToHost,
                       ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "COO column panels: counting failed");
      break;
    }
    int64_t pos = 0;
    for (int p = 0; p < P; ++p)
      for (int64_t i = 0; i < n; ++i) {
        const int32_t c = cnt[(size_t)p * n + i];
        if (c == 0) continue;
        srid.push_back((int32_t)((int64_t)p * n + i));
        srp.push_back((int32_t)pos);
        dst[(size_t)p * n + i] = (int32_t)pos;
        mask[(size_t)i] |= (uint8_t)(1u << p);
        pos += c;
      }
    srp.push_back((int32_t)pos);
    if (pos != nnz) {
      st = fail(ctx, MXS_HIP, "COO column panels: inconsistent counts");
      break;
    }
    C.pmask = upload(ctx, A, mask);
    d_srp = (int32_t*)ctx->alloc.alloc(srp.size() * 4 + 4);
    d_srid = (int32_t*)ctx->alloc.alloc(srid.size() * 4 + 4);
    if (!C.pmask || !d_srp || !d_srid) {
      st = fail(ctx, MXS_OOM, "COO column panels");
      break;
    }
    if (hipMemcpyAsync(d_dst, dst.data(), (size_t)P * n * 4, hipMemcpyHostToDevice,
                       ctx->stream) != hipSuccess ||
        hipMemcpyAsync(d_srp, srp.data(), srp.size() * 4, hipMemcpyHostToDevice, ctx->stream) !=
            hipSuccess ||
        (!srid.empty() && hipMemcpyAsync(d_srid, srid.data(), srid.size() * 4,
                                         hipMemcpyHostToDevice, ctx->stream) != hipSuccess)) {
      st = fail(ctx, MXS_HIP, "copy failed");
      break;
    }
    const int g = grid_for(ctx, n, 256);
    k_panel_scatter<uint64_t><<<g, 256, 0, ctx->stream>>>(
        n, P, S->csr.rowptr, d_cnt, d_dst, S->csr.col, (const uint64_t*)S->csr.val, C.col,
        (uint64_t*)v64);
    k_coo_stacked_rows<<<grid_for(ctx, (int64_t)srid.size(), 256), 256, 0, ctx->stream>>>(
        (int64_t)srid.size(), d_srp, d_srid, C.row);
    if (hipGetLastError() != hipSuccess) {
      st = fail(ctx, MXS_HIP, "COO column panels: scatter failed");
      break;
    }
    if (sizeof(V) != 8) {
      st = cast_into<V>(ctx, nnz, v64, C.val, d_err);
      if (st) break;
    }
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "COO column panels: set-up failed");
      break;
    }
    C.panels = P;
  } while (0);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->alloc.release(d_cnt);
  ctx->alloc.release(d_dst);
  ctx->alloc.release(d_srp);
  ctx->alloc.release(d_srid);
  if (sizeof(V) != 8) ctx->alloc.release(v64);
  return st;
}

// The hybrid format's COO part in panel order (see CooPart): its entries,
// already in A->coo in row order with their values cast, are counted per row
// and panel over the part's own row pointers `off`, moved bit for bit into
// panel order, and each given its stacked output index.
template <typename V>
mxs_status hyb_coo_panels(mxs_ctx* ctx, mxs_matrix* A, int P, const std::vector<int64_t>& off) {
  using E = std::conditional_t<sizeof(V) == 8, uint64_t, uint32_t>;
  static_assert(sizeof(V) == sizeof(E), "FP64 or FP32 values");
  CooPart& C = A->coo;
  const int64_t n = A->n, cnnz = off[(size_t)n];
  const int64_t W = (A->ncols + P - 1) / P;
  std::vector<int32_t> rp32((size_t)n + 1), cnt((size_t)P * n), dst((size_t)P * n, -1), srp, srid;
  for (int64_t i = 0; i <= n; ++i) rp32[(size_t)i] = (int32_t)off[(size_t)i];
  std::vector<uint8_t> mask((size_t)n, 0);
  int32_t* d_rp = (int32_t*)ctx->alloc.alloc(((size_t)n + 1) * 4);
  int32_t* d_cnt = (int32_t*)ctx->alloc.alloc((size_t)P * n * 4 + 4);
  int32_t* d_dst = (int32_t*)ctx->alloc.alloc((size_t)P * n * 4 + 4);
  int32_t* d_col = (int32_t*)ctx->alloc.alloc((size_t)cnnz * 4 + 4);
  E* d_val = (E*)ctx->alloc.alloc((size_t)cnnz * sizeof(E) + 8);
  int32_t* d_srp = nullptr;
  int32_t* d_srid = nullptr;
  mxs_status st = MXS_OK;
  do {
    if (!d_rp || !d_cnt || !d_dst || !d_col || !d_val) {
      st = fail(ctx, MXS_OOM, "hybrid column panels: work arrays");
      break;
    }
    if (hipMemcpyAsync(d_rp, rp32.data(), ((size_t)n + 1) * 4, hipMemcpyHostToDevice,
                       ctx->stream) != hipSuccess ||
        hipMemcpyAsync(d_col, C.col, (size_t)cnnz * 4, hipMemcpyDeviceToDevice, ctx->stream) !=
            hipSuccess ||
        hipMemcpyAsync(d_val, C.val, (size_t)cnnz * sizeof(E), hipMemcpyDeviceToDevice,
                       ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "copy failed");
      break;
    }
    k_panel_counts<<<grid_for(ctx, n, 256), 256, 0, ctx->stream>>>(n, P, W, d_rp, d_col, d_cnt);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(cnt.data(), d_cnt, (size_t)P * n * 4, hipMemcpyDeviceToHost,
                       ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "hybrid column panels: counting failed");
      break;
    }
    int64_t pos = 0;
    for (int p = 0; p < P; ++p)
      for (int64_t i = 0; i < n; ++i) {
        const int32_t c = cnt[(size_t)p * n + i];
        if (c == 0) continue;
        srid.push_back((int32_t)((int64_t)p * n + i));
        srp.push_back((int32_t)pos);
        dst[(size_t)p * n + i] = (int32_t)pos;
        mask[(size_t)i] |= (uint8_t)(1u << p);
        pos += c;
      }
    srp.push_back((int32_t)pos);
    if (pos != cnnz) {
      st = fail(ctx, MXS_HIP, "hybrid column panels: inconsistent counts");
      break;
    }
    C.pmask = upload(ctx, A, mask);
    d_srp = (int32_t*)ctx->alloc.alloc(srp.size() * 4 + 4);
    d_srid = (int32_t*)ctx->alloc.alloc(srid.size() * 4 + 4);
    if (!C.pmask || !d_srp || !d_srid) {
      st = fail(ctx, MXS_OOM, "hybrid column panels");
      break;
    }
    if (hipMemcpyAsync(d_dst, dst.data(), (size_t)P * n * 4, hipMemcpyHostToDevice,
                       ctx->stream) != hipSuccess ||
        hipMemcpyAsync(d_srp, srp.data(), srp.size() * 4, hipMemcpyHostToDevice, ctx->stream) !=
            hipSuccess ||
        (!srid.empty() && hipMemcpyAsync(d_srid, srid.data(), srid.size() * 4,
                                         hipMemcpyHostToDevice, ctx->stream) != hipSuccess)) {
      st = fail(ctx, MXS_HIP, "copy failed");
      break;
    }
    k_panel_scatter<E><<<grid_for(ctx, n, 256), 256, 0, ctx->stream>>>(
        n, P, d_rp, d_cnt, d_dst, d_col, d_val, C.col, (E*)C.val);
    if (!srid.empty())
      k_coo_stacked_rows<<<grid_for(ctx, (int64_t)srid.size(), 256), 256, 0, ctx->stream>>>(
          (int64_t)srid.size(), d_srp, d_srid, C.row);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "hybrid column panels: scatter failed");
      break;
    }
    C.panels = P;
  } while (0);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->alloc.release(d_rp);
  ctx->alloc.release(d_cnt);
  ctx->alloc.release(d_dst);
  ctx->alloc.release(d_col);
  ctx->alloc.release(d_val);
  ctx->alloc.release(d_srp);
  ctx->alloc.release(d_srid);
  return st;
}

template <typename V>
mxs_status convert_typed(mxs_ctx* ctx, const mxs_matrix* S, mxs_matrix* A, mxs_format fmt,
                         const mxs_convert_opts* opts, int* d_err) {
  const int64_t n = S->n, nnz = S->nnz;
  const int bnnz = clamp_block_nnz(opts ? opts->block_nnz : 0);
  const int32_t* rp = S->csr.rowptr;
  const size_t vb = sizeof(V);
  const std::vector<int32_t>& hrp = S->h_rowptr;
  int64_t Kmax = 0;
  for (int64_t i = 0; i < n; ++i) Kmax = std::max<int64_t>(Kmax, hrp[i + 1] - hrp[i]);
  const int64_t stride = (n + 63) / 64 * 64;

  if (fmt == MXS_CSR) {
    A->csr.rowptr = (int32_t*)mat_alloc(A, (n + 1) * 4);
    A->csr.col = (int32_t*)mat_alloc(A, nnz * 4 + 4);
    A->csr.val = mat_alloc(A, nnz * vb + 8);
    if (!A->csr.rowptr || !A->csr.col || !A->csr.val) return fail(ctx, MXS_OOM, "csr arrays");
    MXS_HIP_TRY(ctx, hipMemcpyAsync(A->csr.rowptr, rp, (n + 1) * 4, hipMemcpyDeviceToDevice,
                                    ctx->stream));
    if (nnz)
      MXS_HIP_TRY(ctx, hipMemcpyAsync(A->csr.col, S->csr.col, nnz * 4, hipMemcpyDeviceToDevice,
                                      ctx->stream));
    mxs_status st = cast_into<V>(ctx, nnz, (const double*)S->csr.val, A->csr.val, d_err);
    if (st) return st;
    A->h_rowptr = hrp;
    return build_csr_partition(ctx, A, bnnz, opts);
  }

  if (fmt == MXS_COO) {
    if (mxs_status st = alloc_coo_arrays(ctx, A, A->coo, nnz, vb)) return st;
    // column panels: asked for, or (auto) for rows longer than 64 entries
    // (power-law patterns, whose gathers range over all of x) when x is
    // large enough for the merge path's rule
    const int req = opts ? opts->col_panels : 0;
    const int P = (req > 1 || (req == 0 && Kmax > 64)) ? merge_panels(A, opts) : 1;
    if (P > 1 && nnz > 0) {
      mxs_status st = build_coo_panels<V>(ctx, S, A, P, d_err);
      if (st) return st;
      return setup_coo_part(ctx, A, A->coo, nnz, Kmax, vb, bnnz, std::vector<int32_t>(), opts);
    }
    k_coo_rows<<<grid_for(ctx, n, 256), 256, 0, ctx->stream>>>(n, rp, A->coo.row);
    MXS_HIP_TRY(ctx, hipGetLastError());
    if (nnz)
      MXS_HIP_TRY(ctx, hipMemcpyAsync(A->coo.col, S->csr.col, nnz * 4, hipMemcpyDeviceToDevice,
                                      ctx->stream));
    mxs_status st = cast_into<V>(ctx, nnz, (const double*)S->csr.val, A->coo.val, d_err);
    if (st) return st;
    std::vector<int32_t> empty;
    for (int64_t i = 0; i < n; ++i)
      if (hrp[i + 1] == hrp[i]) empty.push_back((int32_t)i);
    // arrays larger than the 256 MB Infinity Cache are streamed with
    // non-temporal loads; there the default chunk is 256 entries, whose
    // kernel keeps 8 waves a SIMD (27-point 128^3: FP64 179 vs 182 us,
    // FP32 143 vs 152 us at 512)
    const bool big = (double)nnz * (8 + vb) > 256.0 * (1 << 20);
    const int cb = (opts && opts->block_nnz > 0) || !big ? bnnz : 256;
    return setup_coo_part(ctx, A, A->coo, nnz, Kmax, vb, cb, empty, opts);
  }

  // ELL and HYB
  int64_t K;
  if (fmt == MXS_ELL) {
    K = Kmax;
    if (opts && opts->ell_width > 0) {
      if (opts->ell_width < Kmax)
        return fail(ctx, MXS_INVALID_ARG, "ell_width %lld < longest row %lld",
                    (long long)opts->ell_width, (long long)Kmax);
      K = opts->ell_width;
    }
  } else if (opts && opts->ell_width > 0) {
    K = std::min<int64_t>(opts->ell_width, Kmax);
  } else {
    // byte model: one more column costs stride*(V+4) bytes and saves
    // #{L_i >= K}*(V+8) COO bytes
    std::vector<int64_t> ge((size_t)Kmax + 2, 0);
    for (int64_t i = 0; i < n; ++i) ge[hrp[i + 1] - hrp[i]] += 1;
    for (int64_t k = Kmax - 1; k >= 0; --k) ge[k] += ge[k + 1];
    K = 0;
    for (int64_t k = 1; k <= Kmax; ++k) {
      if ((double)ge[k] * (double)(vb + 8) > (double)stride * (double)(vb + 4))
        K = k;
      else
        break;
    }
  }
  const double ell_bytes = (double)K * (double)stride * (double)(vb + 4);
  if (opts && opts->max_ell_bytes > 0 && ell_bytes > (double)opts->max_ell_bytes)
    return fail(ctx, MXS_UNSUPPORTED, "ELL part needs %.0f bytes > max_ell_bytes", ell_bytes);
  A->ell.K = K;
  A->ell.stride = stride;
  int waves = 1;  // chains of at most ~256 slots per lane-accumulator group
  while (waves < 16 && (K + waves - 1) / waves > 256) waves <<= 1;
  A->ell.waves = waves;
  if (K > 0) {
    A->ell.col = (int32_t*)mat_alloc(A, (size_t)(K * stride) * 4);
    A->ell.val = mat_alloc(A, (size_t)(K * stride) * vb);
    if (!A->ell.col || !A->ell.val) return fail(ctx, MXS_OOM, "ELL arrays (%.0f bytes)", ell_bytes);
    k_fill_ell<V><<<grid_for(ctx, K * stride, 256), 256, 0, ctx->stream>>>(
        n, K, stride, rp, S->csr.col, (const double*)S->csr.val, A->ell.col, (V*)A->ell.val,
        d_err);
    MXS_HIP_TRY(ctx, hipGetLastError());
  }
  if (fmt == MXS_ELL) return MXS_OK;

  std::vector<int64_t> off((size_t)n + 1, 0);
  std::vector<int32_t> empty;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t L = hrp[i + 1] - hrp[i];
    off[i + 1] = off[i] + std::max<int64_t>(L - K, 0);
    if (L == 0) empty.push_back((int32_t)i);
  }
  const int64_t cnnz = off[n];
  if (mxs_status st = alloc_coo_arrays(ctx, A, A->coo, cnnz, vb)) return st;
  int64_t* d_off = upload(ctx, A, off);
  if (!d_off) return fail(ctx, MXS_OOM, "hyb coo");
  if (cnnz) {
    k_fill_hyb_coo<V><<<grid_for(ctx, n, 256), 256, 0, ctx->stream>>>(
        n, K, rp, S->csr.col, (const double*)S->csr.val, d_off, A->coo.row, A->coo.col,
        (V*)A->coo.val, d_err);
    MXS_HIP_TRY(ctx, hipGetLastError());
  }
  // column panels for the COO part, by the COO format's rule (rows longer
  // than 64 entries and an x above 4 MiB, or asked for); the pass that adds
  // the panel partials writes every row
  const int req = opts ? opts->col_panels : 0;
  const int P = (cnnz > 0 && (req > 1 || (req == 0 && Kmax > 64))) ? merge_panels(A, opts) : 1;
  if (P > 1) {
    if (mxs_status st = hyb_coo_panels<V>(ctx, A, P, off)) return st;
    return setup_coo_part(ctx, A, A->coo, cnnz, std::max<int64_t>(Kmax - K, 0), vb, bnnz,
                          std::vector<int32_t>(), opts);
  }
  return setup_coo_part(ctx, A, A->coo, cnnz, std::max<int64_t>(Kmax - K, 0), vb, bnnz,
                        empty, opts);
}

}  // namespace
}  // namespace mxs

using namespace mxs;

extern "C" {

mxs_status mxs_matrix_create_csr(mxs_ctx* ctx, int64_t nrows, int64_t ncols, int64_t nnz,
                                 const int32_t* rowptr, const int32_t* col, const double* val,
                                 int flags, mxs_matrix** out) {
  if (!ctx || !out) return MXS_INVALID_ARG;
  if (nnz > 0 && !val) return fail(ctx, MXS_INVALID_ARG, "NULL array");
  return mxs::create_csr(ctx, nrows, ncols, nnz, rowptr, col, val, flags, out);
}

mxs_status mxs_matrix_create_csr_complex(mxs_ctx* ctx, int64_t nrows, int64_t ncols, int64_t nnz,
                                         const int32_t* rowptr, const int32_t* col,
                                         const double* val, int flags, mxs_matrix** out) {
  if (!ctx || !out) return MXS_INVALID_ARG;
  if (nnz > 0 && !val) return fail(ctx, MXS_INVALID_ARG, "NULL array");
  return mxs::create_csr(ctx, nrows, ncols, nnz, rowptr, col, val, flags, out, MXS_C128);
}

}  // extern "C"

namespace mxs {
namespace {

void mat_release(mxs_matrix* A, void* p, size_t bytes) {
  auto it = std::find(A->owned.begin(), A->owned.end(), p);
  if (it != A->owned.end()) {
    A->owned.erase(it);
    A->bytes -= (int64_t)bytes;
  }
  A->alloc.release(p);
}

// Rows flagged in `disorder` (device, one byte per row) are ordered by
// column and their repeated columns summed in input order; the matrix's
// rowptr/col/val are replaced by the result (A->nnz updated).
mxs_status sort_and_sum(mxs_ctx* ctx, mxs_matrix* A, const uint8_t* disorder, int vpe) {
  const int64_t n = A->n, nnz = A->nnz;
  std::vector<int32_t> rp((size_t)n + 1);
  std::vector<uint8_t> dis((size_t)n);
  MXS_HIP_TRY(ctx, hipMemcpyAsync(rp.data(), A->csr.rowptr, (n + 1) * 4, hipMemcpyDeviceToHost,
                                  ctx->stream));
  MXS_HIP_TRY(ctx, hipMemcpyAsync(dis.data(), disorder, n, hipMemcpyDeviceToHost, ctx->stream));
  MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  std::vector<int32_t> shortrows, longrows;
  int64_t maxp2 = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!dis[i]) continue;
    const int64_t L = (int64_t)rp[i + 1] - rp[i];
    if (L <= kSortLds) {
      shortrows.push_back((int32_t)i);
    } else {
      longrows.push_back((int32_t)i);
      int64_t p2 = 1;
      while (p2 < L) p2 <<= 1;
      maxp2 = std::max(maxp2, p2);
    }
  }
  const Allocator& al = ctx->alloc;
  uint64_t* keys = (uint64_t*)al.alloc((size_t)nnz * 8 + 8);
  int32_t* cnt = (int32_t*)al.alloc((size_t)n * 4 + 4);
  int32_t* d_short = (int32_t*)al.alloc(shortrows.size() * 4 + 4);
  int32_t* nrp_d = (int32_t*)al.alloc((size_t)(n + 1) * 4);
  uint64_t* tmp = maxp2 ? (uint64_t*)al.alloc((size_t)maxp2 * 8) : nullptr;
  int32_t *ocol = nullptr;
  double* oval = nullptr;
  mxs_status st = MXS_OK;
  std::vector<int32_t> hcnt((size_t)n), nrp((size_t)n + 1);
  do {
    if (!keys || !cnt || !d_short || !nrp_d || (maxp2 && !tmp)) {
      st = fail(ctx, MXS_OOM, "sorting the rows: scratch for %lld entries", (long long)nnz);
      break;
    }
    if (!shortrows.empty()) {
      if (hipMemcpyAsync(d_short, shortrows.data(), shortrows.size() * 4, hipMemcpyHostToDevice,
                         ctx->stream) != hipSuccess) {
        st = fail(ctx, MXS_HIP, "copy failed");
        break;
      }
      k_sort_rows_lds<<<(unsigned)shortrows.size(), 256, 0, ctx->stream>>>(
          d_short, A->csr.rowptr, A->csr.col, keys, cnt);
    }
    for (int32_t i : longrows) {
      int64_t p2 = 1;
      while (p2 < (int64_t)rp[i + 1] - rp[i]) p2 <<= 1;
      k_sort_row_global<<<1, 1024, 0, ctx->stream>>>(i, A->csr.rowptr, A->csr.col, tmp, p2, keys,
                                                   cnt);
    }
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(hcnt.data(), cnt, n * 4, hipMemcpyDeviceToHost, ctx->stream) !=
            hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "sorting the rows failed");
      break;
    }
    nrp[0] = 0;
    for (int64_t i = 0; i < n; ++i)
      nrp[i + 1] = nrp[i] + (dis[i] ? hcnt[i] : rp[i + 1] - rp[i]);
    const int64_t nn = nrp[n];
    ocol = (int32_t*)mat_alloc(A, (size_t)nn * 4 + 4);
    oval = (double*)mat_alloc(A, (size_t)nn * 8 * vpe + 16);
    if (!ocol || !oval) {
      st = fail(ctx, MXS_OOM, "summed CSR arrays (%lld entries)", (long long)nn);
      break;
    }
    if (hipMemcpyAsync(nrp_d, nrp.data(), (n + 1) * 4, hipMemcpyHostToDevice, ctx->stream) !=
        hipSuccess) {
      st = fail(ctx, MXS_HIP, "copy failed");
      break;
    }
    if (n > 0)
      k_compact_rows<<<grid_for(ctx, (n + 3) / 4, 1), 256, 0, ctx->stream>>>(
          n, A->csr.rowptr, nrp_d, disorder, A->csr.col, (const double*)A->csr.val, vpe, keys,
          ocol, oval);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(A->csr.rowptr, nrp_d, (n + 1) * 4, hipMemcpyDeviceToDevice,
                       ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "compacting the rows failed");
      break;
    }
    mat_release(A, A->csr.col, (size_t)nnz * 4 + 4);
    mat_release(A, A->csr.val, (size_t)nnz * 8 * vpe + 16);
    A->csr.col = ocol;
    A->csr.val = oval;
    A->nnz = nn;
  } while (0);
  (void)hipStreamSynchronize(ctx->stream);
  al.release(keys);
  al.release(cnt);
  al.release(d_short);
  al.release(nrp_d);
  al.release(tmp);
  return st;
}

}  // namespace
}  // namespace mxs

// validated CSR from host or device arrays; val == NULL gives zero values
mxs_status mxs::create_csr(mxs_ctx* ctx, int64_t nrows, int64_t ncols, int64_t nnz,
                           const int32_t* rowptr, const int32_t* col, const double* val,
                           int flags, mxs_matrix** out, mxs_dtype dt) {
  const size_t vb = dt == MXS_C128 ? 16 : 8;
  if (!ctx || !out) return MXS_INVALID_ARG;
  if (nrows < 0 || ncols < 0 || nnz < 0)
    return fail(ctx, MXS_INVALID_ARG, "negative size");
  if (nrows > INT32_MAX - 1 || ncols > INT32_MAX || nnz > INT32_MAX)
    return fail(ctx, MXS_UNSUPPORTED, "sizes beyond int32 indices");
  if (!rowptr || (nnz > 0 && !col))
    return fail(ctx, MXS_INVALID_ARG, "NULL array");
  const bool sort_sum = (flags & MXS_SORT_AND_SUM) != 0;
  const int where = flags & ~MXS_SORT_AND_SUM;
  if (where != MXS_HOST_PTRS && where != MXS_DEVICE_PTRS)
    return fail(ctx, MXS_INVALID_ARG, "unknown flags %d", flags);
  MXS_HIP_TRY(ctx, hipSetDevice(ctx->device));
  mxs_matrix* A = new_matrix(ctx);
  if (!A) return MXS_OOM;
  A->n = nrows;
  A->ncols = ncols;
  A->nnz = nnz;
  A->fmt = MXS_CSR;
  A->dt = dt;
  mxs_status st = MXS_OK;
  do {
    A->csr.rowptr = (int32_t*)mat_alloc(A, (nrows + 1) * 4);
    A->csr.col = (int32_t*)mat_alloc(A, nnz * 4 + 4);
    A->csr.val = mat_alloc(A, nnz * vb + 16);
    if (!A->csr.rowptr || !A->csr.col || !A->csr.val || !ws_reserve(ctx, 256)) {
      st = fail(ctx, MXS_OOM, "cannot allocate CSR arrays (%lld entries)", (long long)nnz);
      break;
    }
    const hipMemcpyKind kind =
        where == MXS_HOST_PTRS ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (hipMemcpyAsync(A->csr.rowptr, rowptr, (nrows + 1) * 4, kind, ctx->stream) ||
        (nnz && hipMemcpyAsync(A->csr.col, col, nnz * 4, kind, ctx->stream)) ||
        (nnz && val && hipMemcpyAsync(A->csr.val, val, nnz * vb, kind, ctx->stream)) ||
        (nnz && !val && hipMemsetAsync(A->csr.val, 0, nnz * vb, ctx->stream))) {
      st = fail(ctx, MXS_HIP, "copying the CSR arrays failed");
      break;
    }
    int* d_err = (int*)ctx->ws.ptr;
    if (hipMemsetAsync(d_err, 0, sizeof(int), ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "memset failed");
      break;
    }
    k_check_rowptr<<<grid_for(ctx, nrows + 1, 256), 256, 0, ctx->stream>>>(nrows, nnz,
                                                                           A->csr.rowptr, d_err);
    int err = 0;
    if ((st = read_err(ctx, d_err, &err))) break;
    if (err) {
      st = fail(ctx, MXS_INVALID_MATRIX,
                "row pointers must start at 0, never decrease and end at nnz");
      break;
    }
    if (nrows > 0) {
      uint8_t* disorder = sort_sum ? (uint8_t*)ctx->alloc.alloc((size_t)nrows) : nullptr;
      if (sort_sum && !disorder) {
        st = fail(ctx, MXS_OOM, "row flags");
        break;
      }
      k_check_cols<<<grid_for(ctx, nrows, 256), 256, 0, ctx->stream>>>(
          nrows, ncols, A->csr.rowptr, A->csr.col, d_err, disorder);
      if ((st = read_err(ctx, d_err, &err))) {
        ctx->alloc.release(disorder);
        break;
      }
      if (err & kErrCol) {
        st = fail(ctx, MXS_INVALID_MATRIX, "column indices must lie in [0, ncols)");
      } else if ((err & kErrOrder) && !sort_sum) {
        st = fail(ctx, MXS_INVALID_MATRIX,
                  "column indices must ascend strictly in each row (or pass MXS_SORT_AND_SUM)");
      } else if (err & kErrOrder) {
        st = sort_and_sum(ctx, A, disorder, dt == MXS_C128 ? 2 : 1);
      }
      (void)hipStreamSynchronize(ctx->stream);
      ctx->alloc.release(disorder);
      if (st) break;
    }
    A->h_rowptr.resize((size_t)nrows + 1);
    if (hipMemcpyAsync(A->h_rowptr.data(), A->csr.rowptr, (nrows + 1) * 4,
                       hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "reading back the row pointers failed");
      break;
    }
    st = build_csr_partition(ctx, A, 512);
  } while (0);
  if (st) {
    (void)hipStreamSynchronize(ctx->stream);
    free_matrix(A);
    return st;
  }
  *out = A;
  return MXS_OK;
}

namespace mxs {
namespace {

// complex CSR to complex CSR: the same pattern, values copied (C128) or
// each part rounded to FP32 (C64), a partition for the new options
mxs_status convert_complex(mxs_ctx* ctx, const mxs_matrix* src, mxs_dtype dt,
                           const mxs_convert_opts* opts, mxs_matrix** out) {
  MXS_HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (!ws_reserve(ctx, 256)) return fail(ctx, MXS_OOM, "workspace");
  mxs_matrix* A = new_matrix(ctx);
  if (!A) return MXS_OOM;
  const int64_t n = src->n, nnz = src->nnz;
  A->n = n;
  A->ncols = src->ncols;
  A->nnz = nnz;
  A->fmt = MXS_CSR;
  A->dt = dt;
  int* d_err = (int*)ctx->ws.ptr;
  mxs_status st = MXS_OK;
  do {
    A->csr.rowptr = (int32_t*)mat_alloc(A, (n + 1) * 4);
    A->csr.col = (int32_t*)mat_alloc(A, nnz * 4 + 4);
    A->csr.val = mat_alloc(A, nnz * value_bytes(dt) + 16);
    if (!A->csr.rowptr || !A->csr.col || !A->csr.val) {
      st = fail(ctx, MXS_OOM, "complex csr arrays");
      break;
    }
    if (hipMemsetAsync(d_err, 0, sizeof(int), ctx->stream) != hipSuccess ||
        hipMemcpyAsync(A->csr.rowptr, src->csr.rowptr, (n + 1) * 4, hipMemcpyDeviceToDevice,
                       ctx->stream) != hipSuccess ||
        (nnz && hipMemcpyAsync(A->csr.col, src->csr.col, nnz * 4, hipMemcpyDeviceToDevice,
                               ctx->stream) != hipSuccess)) {
      st = fail(ctx, MXS_HIP, "copy failed");
      break;
    }
    // (re, im) pairs are 2 nnz doubles: the elementwise casts apply as is
    st = dt == MXS_C128
             ? cast_into<double>(ctx, 2 * nnz, (const double*)src->csr.val, A->csr.val, d_err)
             : cast_into<float>(ctx, 2 * nnz, (const double*)src->csr.val, A->csr.val, d_err);
    if (st) break;
    int err = 0;
    if ((st = read_err(ctx, d_err, &err))) break;
    if (err & kErrRange) {
      st = fail(ctx, MXS_UNSUPPORTED, "a value exceeds the FP32 range");
      break;
    }
    A->h_rowptr = src->h_rowptr;
    st = build_csr_partition(ctx, A, clamp_block_nnz(opts ? opts->block_nnz : 0), opts);
  } while (0);
  if (st) {
    (void)hipStreamSynchronize(ctx->stream);
    free_matrix(A);
    return st;
  }
  *out = A;
  return MXS_OK;
}

}  // namespace
}  // namespace mxs

extern "C" {

mxs_status mxs_matrix_convert(mxs_ctx* ctx, const mxs_matrix* src, mxs_format fmt,
                              mxs_dtype dt, const mxs_convert_opts* opts, mxs_matrix** out) {
  if (!ctx || !src || !out) return MXS_INVALID_ARG;
  if (fmt < MXS_CSR || fmt > MXS_HYB || dt < MXS_F64 || dt > MXS_C64)
    return fail(ctx, MXS_INVALID_ARG, "unknown format or dtype");
  if (opts && (opts->coo_kernel < MXS_COO_AUTO || opts->coo_kernel > MXS_COO_RUNS))
    return fail(ctx, MXS_INVALID_ARG, "unknown coo_kernel");
  if (src->fmt == MXS_CSR && src->dt == MXS_C128) {
    if (fmt != MXS_CSR || (dt != MXS_C128 && dt != MXS_C64))
      return fail(ctx, MXS_UNSUPPORTED, "complex values convert to complex CSR only");
    return convert_complex(ctx, src, dt, opts, out);
  }
  if (src->fmt != MXS_CSR || src->dt != MXS_F64)
    return fail(ctx, MXS_UNSUPPORTED, "conversion source must be an F64 or C128 CSR matrix");
  if (dt > MXS_F16_ROWSCALED)
    return fail(ctx, MXS_UNSUPPORTED, "real values convert to real types only");
  if (dt == MXS_F16_ROWSCALED && fmt != MXS_CSR)
    return fail(ctx, MXS_UNSUPPORTED, "F16_ROWSCALED is offered for CSR only");
  MXS_HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (!ws_reserve(ctx, 256)) return fail(ctx, MXS_OOM, "workspace");
  mxs_matrix* A = new_matrix(ctx);
  if (!A) return MXS_OOM;
  A->n = src->n;
  A->ncols = src->ncols;
  A->nnz = src->nnz;
  A->fmt = fmt;
  A->dt = dt;
  int* d_err = (int*)ctx->ws.ptr;
  mxs_status st = MXS_OK;
  do {
    if (hipMemsetAsync(d_err, 0, sizeof(int), ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "memset failed");
      break;
    }
    if (dt == MXS_F64) {
      st = convert_typed<double>(ctx, src, A, fmt, opts, d_err);
    } else if (dt == MXS_F32) {
      st = convert_typed<float>(ctx, src, A, fmt, opts, d_err);
    } else {
      const int64_t n = src->n, nnz = src->nnz;
      A->csr.rowptr = (int32_t*)mat_alloc(A, (n + 1) * 4);
      A->csr.col = (int32_t*)mat_alloc(A, nnz * 4 + 4);
      A->csr.val = mat_alloc(A, nnz * 2 + 8);
      A->csr.scale = (float*)mat_alloc(A, n * 4 + 4);
      if (!A->csr.rowptr || !A->csr.col || !A->csr.val || !A->csr.scale) {
        st = fail(ctx, MXS_OOM, "f16 arrays");
        break;
      }
      if (hipMemcpyAsync(A->csr.rowptr, src->csr.rowptr, (n + 1) * 4, hipMemcpyDeviceToDevice,
                         ctx->stream) ||
          (nnz && hipMemcpyAsync(A->csr.col, src->csr.col, nnz * 4, hipMemcpyDeviceToDevice,
                                 ctx->stream))) {
        st = fail(ctx, MXS_HIP, "copy failed");
        break;
      }
      if (n > 0)
        k_rowscale_f16<<<grid_for(ctx, n, 256), 256, 0, ctx->stream>>>(
            n, src->csr.rowptr, (const double*)src->csr.val, (uint16_t*)A->csr.val, A->csr.scale,
            d_err);
      A->h_rowptr = src->h_rowptr;
      st = build_csr_partition(ctx, A, clamp_block_nnz(opts ? opts->block_nnz : 0), opts);
    }
    if (st) break;
    int err = 0;
    if ((st = read_err(ctx, d_err, &err))) break;
    if (err & kErrNonfinite) {
      st = fail(ctx, MXS_UNSUPPORTED, "non-finite value cannot be stored with a row scale");
      break;
    }
    if (err & kErrRange) {
      st = fail(ctx, MXS_UNSUPPORTED, "value outside the range of the target type");
      break;
    }
  } while (0);
  if (st) {
    (void)hipStreamSynchronize(ctx->stream);
    free_matrix(A);
    return st;
  }
  *out = A;
  return MXS_OK;
}

mxs_status mxs_matrix_info(const mxs_matrix* A, mxs_matrix_desc* out) {
  if (!A || !out) return MXS_INVALID_ARG;
  std::memset(out, 0, sizeof(*out));
  out->nrows = A->n;
  out->ncols = A->ncols;
  out->nnz = A->nnz;
  out->format = A->fmt;
  out->dtype = A->dt;
  out->ell_width = A->ell.K;
  out->ell_stride = A->ell.stride;
  out->coo_nnz = (A->fmt == MXS_COO || A->fmt == MXS_HYB) ? A->coo.nnz : 0;
  out->blocks = A->fmt == MXS_CSR ? A->csr.nblocks
                : (A->fmt == MXS_COO || A->fmt == MXS_HYB) ? A->coo.nchunks
                                                           : (A->ell.stride / 64);
  out->block_nnz = A->fmt == MXS_CSR ? A->csr.block_nnz : A->coo.block_nnz;
  out->lanes_per_row = A->fmt != MXS_CSR ? 0 : A->csr.rows_lds ? A->csr.rl_lanes : A->csr.lanes;
  out->rows_per_group = A->fmt == MXS_CSR ? A->csr.rpg : 0;
  out->waves_per_group = A->fmt == MXS_CSR ? A->csr.wpb : A->coo.wpb;
  out->csr_kernel = A->fmt != MXS_CSR  ? 0
                    : A->csr.merge    ? MXS_CSR_MERGE
                    : A->csr.products ? MXS_CSR_PRODUCTS
                    : A->csr.rows_lds ? MXS_CSR_ROWS_LDS
                    : A->csr.lanes >= 1 ? MXS_CSR_VECTOR
                                       : MXS_CSR_STREAM;
  out->coo_kernel = A->fmt == MXS_COO || (A->fmt == MXS_HYB && A->coo.nnz > 0) ? A->coo.kernel : 0;
  out->col_panels = A->fmt == MXS_CSR && A->csr.merge           ? A->csr.panels
                    : A->fmt == MXS_COO || A->fmt == MXS_HYB     ? A->coo.panels
                                                                 : 0;
  out->bytes = A->bytes;
  return MXS_OK;
}

mxs_status mxs_matrix_export(mxs_ctx* ctx, const mxs_matrix* A, mxs_array which, void* dst,
                             size_t bytes) {
  if (!ctx || !A || !dst) return MXS_INVALID_ARG;
  const size_t vb = value_bytes(A->dt);
  const void* src = nullptr;
  size_t size = 0;
  const bool csr = A->fmt == MXS_CSR, coo = A->fmt == MXS_COO, hyb = A->fmt == MXS_HYB,
             ell = A->fmt == MXS_ELL;
  switch (which) {
    case MXS_ARR_ROWPTR:
      if (csr) src = A->csr.rowptr, size = (A->n + 1) * 4;
      break;
    case MXS_ARR_COL:
      if (csr) src = A->csr.col, size = A->nnz * 4;
      if (coo) src = A->coo.col, size = A->nnz * 4;
      break;
    case MXS_ARR_VAL:
      if (csr) src = A->csr.val, size = A->nnz * vb;
      if (coo) src = A->coo.val, size = A->nnz * vb;
      break;
    case MXS_ARR_ROW:
      if (coo) src = A->coo.row, size = A->nnz * 4;
      break;
    case MXS_ARR_ELL_COL:
      if (ell || hyb) src = A->ell.col, size = A->ell.K * A->ell.stride * 4;
      break;
    case MXS_ARR_ELL_VAL:
      if (ell || hyb) src = A->ell.val, size = A->ell.K * A->ell.stride * vb;
      break;
    case MXS_ARR_COO_ROW:
      if (hyb) src = A->coo.row, size = A->coo.nnz * 4;
      break;
    case MXS_ARR_COO_COL:
      if (hyb) src = A->coo.col, size = A->coo.nnz * 4;
      break;
    case MXS_ARR_COO_VAL:
      if (hyb) src = A->coo.val, size = A->coo.nnz * vb;
      break;
    case MXS_ARR_SCALE:
      if (csr && A->dt == MXS_F16_ROWSCALED) src = A->csr.scale, size = A->n * 4;
      break;
  }
  if (!src && size == 0 && which != MXS_ARR_ELL_COL && which != MXS_ARR_ELL_VAL &&
      which != MXS_ARR_COO_ROW && which != MXS_ARR_COO_COL && which != MXS_ARR_COO_VAL)
    return fail(ctx, MXS_INVALID_ARG, "matrix has no such array");
  if (bytes != size)
    return fail(ctx, MXS_INVALID_ARG, "export buffer is %zu bytes, array is %zu", bytes, size);
  if (size) {
    MXS_HIP_TRY(ctx, hipMemcpyAsync(dst, src, size, hipMemcpyDeviceToHost, ctx->stream));
    MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  }
  return MXS_OK;
}

mxs_status mxs_matrix_destroy(mxs_matrix* A) {
  free_matrix(A);
  return MXS_OK;
}

}  // extern "C"
