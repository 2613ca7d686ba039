// spmv.hip -- y = alpha*A*x + beta*y for CSR, COO, ELL and hybrid ELL+COO
// storage on gfx950 (paper, section "Central Sparse Linear Algebra
// Functionality"; the byte-per-entry model of its "SpMV Performance
// Analysis" subsection makes every variant HBM-bound, so none uses MFMA).
//
// CSR  -- five kernels.  Stream: one wave per row block (<= 64*NPL
//         entries, whole rows); the wave streams the block's values and
//         column indices with fully coalesced loads, gathers x, and stages
//         the products and the block's row pointers in LDS.  Each lane then
//         owns NPL consecutive products, sums the row segments it holds, and
//         a segmented inclusive scan across the 64 lanes joins the segments
//         of rows that straddle lanes; a row longer than the block budget
//         gets a wave of its own with four independent accumulators per lane.
//         Merge path: the same lane runs over equal chunks of entries
//         whatever the rows, each entry's row found from the chunk's row
//         pointers in LDS, cut rows fixed up as for COO.  Rows-from-LDS and
//         products-through-LDS: blocks of at most 64 rows for short-row
//         matrices.  Vector: G lanes per row, on request.
// COO  -- same lane-run/segmented-scan scheme over fixed chunks of 64*NPL
//         entries.  A row cut by a chunk boundary is written by the chunk
//         where it starts; later chunks store their part as a continuation
//         partial that a small fix-up pass adds in chunk order.  No
//         floating-point atomics, so the result is deterministic.
// ELL  -- thread per row over the column-major slots; W waves per 64 rows
//         take the columns round-robin (each lane keeps four accumulators),
//         and a wave stops at the first slot group where all its rows are
//         padding (padding is always at the end of a row).
// HYB  -- ELL kernel for the regular part, then the COO kernel in
//         accumulate mode for the overflow.
//
// Per-lane sequential chains are at most NPL (+ the scan depth of 6) for
// CSR/COO blocks and at most a quarter of a row's entries per wave for long
// rows and ELL; the FP64 error stays far below 1e-13 * sum|a_ij||x_j|.
#include <type_traits>

#include <algorithm>
#include <mutex>

#include "common.h"

namespace mxs {
namespace {

// LDS index with one pad slot every 32 elements: a lane reading NPL
// consecutive products then hits spread-out banks.
__device__ __forceinline__ int pad(int k) { return k + (k >> 5); }

template <typename T>
__device__ __forceinline__ T combine(T alpha, T s, T beta, const T* __restrict__ y, int64_t i) {
  return beta == T(0) ? alpha * s : alpha * s + beta * y[i];
}

// Matrix values staged in registers as raw bits: a 2-byte value takes a
// whole register, so that a predicated load never has to merge into a
// register that an earlier load still fills (which would make each load wait
// for the one before it).
template <typename V>
struct Raw {
  using type = V;
  static __device__ __forceinline__ V load(const V* p, int64_t i) { return p[i]; }
  static __device__ __forceinline__ V value(V r) { return r; }
  static __device__ __forceinline__ void store(V* d, int i, V r) { d[i] = r; }
};
template <>
struct Raw<_Float16> {
  using type = uint32_t;
  static __device__ __forceinline__ uint32_t load(const _Float16* p, int64_t i) {
    return reinterpret_cast<const uint16_t*>(p)[i];
  }
  static __device__ __forceinline__ _Float16 value(uint32_t r) {
    return __builtin_bit_cast(_Float16, (uint16_t)r);
  }
  static __device__ __forceinline__ void store(_Float16* d, int i, uint32_t r) {
    reinterpret_cast<uint16_t*>(d)[i] = (uint16_t)r;
  }
};

// One element of a streamed matrix array.  NT: a non-temporal load, for
// matrices whose streamed arrays exceed the 256 MB Infinity Cache: on the
// 27-point 128^3 matrix (906 MB of COO arrays) a bare stream of row, col and
// val with its x gathers takes 10% less time than with ordinary loads, and
// the y stores written among the reads cost 22 instead of 28 us; the
// products themselves run 3-11% faster.  Matrices that fit the cache keep
// ordinary loads, which leave their lines there for the next product (a
// solver's).
template <bool NT, typename E>
__device__ __forceinline__ E ld_stream(const E* p) {
  if constexpr (!NT) {
    return *p;
  } else if constexpr (std::is_same_v<E, cplx<double>> || std::is_same_v<E, cplx<float>>) {
    // both parts in one load (entries are 2 x 8 or 2 x 4 bytes and every
    // device allocation is 16-byte aligned, so each entry is aligned to its size)
    using R = decltype(p->re);
    typedef R r2 __attribute__((ext_vector_type(2)));
    const r2 v = __builtin_nontemporal_load(reinterpret_cast<const r2*>(p));
    return E(v.x, v.y);
  } else {
    return __builtin_nontemporal_load(p);
  }
}

// Streamed bytes above which a product reads its matrix non-temporally.
constexpr double kStreamNtBytes = 256.0 * (1 << 20);

// Value types whose streamed loads may be non-temporal (FP16 bit patterns
// keep ordinary loads).
template <typename V>
constexpr bool kNtValue = std::is_same_v<V, double> || std::is_same_v<V, float> ||
                          std::is_same_v<V, cplx<double>> || std::is_same_v<V, cplx<float>>;

// ---------------------------------------------------------------------------
// CSR
// ---------------------------------------------------------------------------
// Synchronises the lanes of one wave (LDS written by some lanes is then
// visible to the others); the waves of a work-group stay independent.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename V, typename T, int NPL, bool SCALED, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_csr(int64_t nblocks,
                                                  const int32_t* __restrict__ blocks,
                                                  const int32_t* __restrict__ bnnz,
                                                  const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ col,
                                                  const V* __restrict__ val,
                                                  const float* __restrict__ scale,
                                                  const T* __restrict__ x, T* __restrict__ y,
                                                  T alpha, T beta,
                                                  const int32_t* __restrict__ skip) {
  constexpr int C = 64 * NPL;
  __shared__ T prod_all[WPB][C + C / 32];
  __shared__ int32_t rp_all[WPB][C + 1];
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63;
  // wave-uniform (scalar block-bound loads)
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  T* prod = prod_all[wv];
  int32_t* rp = rp_all[wv];
  const int64_t b = xcd_remap(blockIdx.x, gridDim.x) * WPB + wv;
  if (b >= nblocks) return;
  const int32_t r0 = blocks[b], r1 = blocks[b + 1];
  const int32_t s = bnnz[b], e = bnnz[b + 1];  // = rowptr[r0], rowptr[r1]
  const int nr = r1 - r0, len = e - s;

  auto emit = [&](int r, T sum) {
    const int64_t i = (int64_t)r0 + r;
    if (SCALED) sum *= (T)scale[i];
    y[i] = combine(alpha, sum, beta, y, i);
  };

  if (len > C) {  // a single long row
    T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int32_t k = s + lane;
    for (; k + 192 < e; k += 256) {
      const int32_t c0 = col[k], c1 = col[k + 64], c2 = col[k + 128], c3 = col[k + 192];
      const T v0 = to_acc(val[k]), v1 = to_acc(val[k + 64]), v2 = to_acc(val[k + 128]),
              v3 = to_acc(val[k + 192]);
      a0 += v0 * x[c0];
      a1 += v1 * x[c1];
      a2 += v2 * x[c2];
      a3 += v3 * x[c3];
    }
    for (; k < e; k += 64) a0 += to_acc(val[k]) * x[col[k]];
    const T acc = wave_sum((a0 + a1) + (a2 + a3));
    if (lane == 0) emit(0, acc);
    return;
  }

  {
    int32_t c[NPL];
    typename Raw<V>::type v[NPL];
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int k = t * 64 + lane;
      c[t] = 0;  // (v[t] of an unused slot is never read)
      if (k < len) {
        c[t] = col[s + k];
        v[t] = Raw<V>::load(val, s + k);
      }
    }
    // gathers issued for every slot (column 0 where the block has ended,
    // so all of them are in flight together); the product of an unused
    // slot is discarded, never stored
    T g[NPL];
#pragma unroll
    for (int t = 0; t < NPL; ++t) g[t] = x[c[t]];
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int k = t * 64 + lane;
      if (k < len) prod[pad(k)] = to_acc(Raw<V>::value(v[t])) * g[t];
    }
  }
  for (int i = lane; i <= nr; i += 64) rp[i] = rowptr[r0 + i] - s;
  wave_sync();

  for (int i = lane; i < nr; i += 64)
    if (rp[i] == rp[i + 1]) emit(i, T(0));  // empty rows

  const int k0 = lane * NPL;
  const bool active = k0 < len;
  const int k1 = min(k0 + NPL, len);
  T v = 0, hsum = 0, tsum = 0;
  int f = 1, hrow = 0, trow = 0;
  bool multi = false, hstart = false, tend = false;
  if (active) {
    int lo = 0, hi = nr;  // row holding entry k0: rp[lo] <= k0 < rp[lo+1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (rp[mid] <= k0)
        lo = mid;
      else
        hi = mid;
    }
    hrow = lo;
    hstart = rp[lo] == k0;
    int r = lo, rend = rp[lo + 1];
    T sum = 0;
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int k = k0 + t;
      if (k < k1) {
        if (k == rend) {
          if (!multi) {
            hsum = sum;
            multi = true;
          } else {
            emit(r, sum);  // a row that starts and ends in this lane
          }
          do {
            ++r;
            rend = rp[r + 1];
          } while (rend <= k);
          sum = 0;
        }
        sum += prod[pad(k)];
      }
    }
    trow = r;
    tsum = sum;
    tend = rend == k1;
    if (!multi) hsum = sum;
    v = multi ? tsum : hsum;
    f = (multi || hstart) ? 1 : 0;
  }
  // inclusive segmented scan over lanes: a set flag starts a new row
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T ov = __shfl_up(v, d, 64);
    const int of = __shfl_up(f, d, 64);
    if (lane >= d) {
      if (!f) v = ov + v;
      f |= of;
    }
  }
  const T before = __shfl_up(v, 1, 64);
  if (active) {
    if (multi) {
      emit(hrow, hstart ? hsum : before + hsum);
      if (tend) emit(trow, tsum);
    } else if (tend) {
      emit(hrow, v);
    }
  }
}

// ---------------------------------------------------------------------------
// CSR, vector variant for regular row lengths: G lanes per row, each group
// of G lanes owns RPG consecutive rows and issues the loads of all of them
// before using any (one entry per lane per row, a tail loop for rows longer
// than G).  No LDS; the butterfly over the G lanes leaves every row sum in
// every lane of the group, and lane r of the group stores row r.
// ---------------------------------------------------------------------------
template <typename V, typename T, int G, int RPG, bool SCALED>
__global__ __launch_bounds__(256) void k_csr_vec(int64_t n, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col,
                                                 const V* __restrict__ val,
                                                 const float* __restrict__ scale,
                                                 const T* __restrict__ x, T* __restrict__ y,
                                                 T alpha, T beta,
                                                 const int32_t* __restrict__ skip) {
  static_assert(RPG <= G, "lane r of a group stores row r");
  if (skip && *skip) return;
  constexpr int GROUPS = 256 / G;
  const int li = threadIdx.x % G;
  const int64_t base =
      (xcd_remap(blockIdx.x, gridDim.x) * GROUPS + threadIdx.x / G) * (int64_t)RPG;
  if (base >= n) return;
  int32_t rp[RPG + 1];
#pragma unroll
  for (int r = 0; r <= RPG; ++r) rp[r] = rowptr[min<int64_t>(base + r, n)];
  int32_t c[RPG];
  T v[RPG];
#pragma unroll
  for (int r = 0; r < RPG; ++r) {
    const int32_t k = rp[r] + li;
    c[r] = 0;
    v[r] = 0;
    if (k < rp[r + 1]) {
      c[r] = col[k];
      v[r] = to_acc(val[k]);
    }
  }
  T sum[RPG];
#pragma unroll
  for (int r = 0; r < RPG; ++r) {
    sum[r] = T(0);
    if (rp[r] + li < rp[r + 1]) sum[r] = v[r] * x[c[r]];
  }
#pragma unroll
  for (int r = 0; r < RPG; ++r)
    for (int32_t k = rp[r] + li + G; k < rp[r + 1]; k += G) sum[r] += to_acc(val[k]) * x[col[k]];
#pragma unroll
  for (int r = 0; r < RPG; ++r) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) sum[r] += __shfl_xor(sum[r], o, 64);
  }
  T mine = sum[0];
#pragma unroll
  for (int r = 1; r < RPG; ++r)
    if (li == r) mine = sum[r];
  const int64_t i = base + li;
  if (li < RPG && i < n) {
    if (SCALED) mine *= (T)scale[i];
    y[i] = combine(alpha, mine, beta, y, i);
  }
}

// ---------------------------------------------------------------------------
// CSR, rows from LDS: a wave owns a block of at most 64/G rows and CMAX
// entries.  All of the block's column indices and values are loaded at once
// (fully coalesced, CMAX/64 of each per lane in flight together) and copied
// into LDS; then G neighbouring lanes walk each row out of LDS (lane h of a
// row takes its entries h, h+G, h+2G, ...), so the x gathers of one step
// come from neighbouring rows (contiguous on banded and stencil matrices, as
// in ELL) while HBM sees only contiguous reads.  G > 1 keeps every lane busy
// when a block holds fewer than 64 rows.  A row longer than CMAX is a block
// of its own and takes the whole wave, reading straight from global memory.
// (Staging the next block while walking the current one was measured
// slower: the extra registers cost more occupancy than the overlap gains.)
// ---------------------------------------------------------------------------
// One row block (b) of the rows-from-LDS kernel, by one wave; vl/cl are the
// wave's LDS tables.  With DOT the lanes that write a row i also return
// x[i] * y[i] (the product's own inner product p.q when x = p and y = q = A p),
// else 0.
template <typename V, typename T, int CMAX, bool SCALED, int G, int ST, bool DOT,
          bool NT = false>
__device__ __forceinline__ double rl_block(int64_t b, const int32_t* __restrict__ blocks,
                                           const int32_t* __restrict__ bnnz,
                                           const int32_t* __restrict__ rowptr,
                                           const int32_t* __restrict__ col,
                                           const V* __restrict__ val,
                                           const float* __restrict__ scale,
                                           const T* __restrict__ x, T* __restrict__ y, T alpha,
                                           T beta, V* vl, int32_t* cl,
                                           const T* __restrict__ wdot = nullptr,
                                           double* d1 = nullptr) {
  constexpr int U = CMAX / 64;  // entries per lane of a full block
  const int lane = threadIdx.x & 63;
  const int32_t r0 = blocks[b], r1 = blocks[b + 1];
  const int32_t s = bnnz[b], e = bnnz[b + 1];
  const int nr = r1 - r0, len = e - s;
  if (len > CMAX) {  // a single long row
    T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int32_t k = s + lane;
    for (; k + 192 < e; k += 256) {
      const int32_t c0 = col[k], c1 = col[k + 64], c2 = col[k + 128], c3 = col[k + 192];
      const T v0 = to_acc(val[k]), v1 = to_acc(val[k + 64]), v2 = to_acc(val[k + 128]),
              v3 = to_acc(val[k + 192]);
      a0 += v0 * x[c0];
      a1 += v1 * x[c1];
      a2 += v2 * x[c2];
      a3 += v3 * x[c3];
    }
    for (; k < e; k += 64) a0 += to_acc(val[k]) * x[col[k]];
    T acc = wave_sum((a0 + a1) + (a2 + a3));
    if (lane == 0) {
      if (SCALED) acc *= (T)scale[r0];
      const T out = combine(alpha, acc, beta, y, r0);
      y[r0] = out;
      if constexpr (DOT) return (double)x[r0] * (double)out;
    }
    return 0.0;
  }
  // bounds of the lane's row (an empty range at len for lanes past the
  // block): loaded unconditionally so that their wait can be deferred
  const int rl = lane / G, h = lane % G;
  const int32_t ra = rowptr[r0 + (rl < nr ? rl : nr)] - s;
  const int32_t rb = rowptr[r0 + (rl < nr ? rl + 1 : nr)] - s;
  {
    int32_t c[U];
    typename Raw<V>::type v[U];
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const int k = t * 64 + lane;
      if (k < len) {
        if constexpr (NT) {
          c[t] = ld_stream<true>(col + s + k);
          v[t] = ld_stream<true>(val + s + k);
        } else {
          c[t] = col[s + k];
          v[t] = Raw<V>::load(val, s + k);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const int k = t * 64 + lane;
      if (k < len) {
        cl[k] = c[t];
        Raw<V>::store(vl, k, v[t]);
      }
    }
  }
  wave_sync();
  // ST (8 or 16) of the lane's entries per step, their gathers in flight
  // together; slots past the row's end read the row's first entry and add
  // nothing
  T acc[4] = {T(0), T(0), T(0), T(0)};
  for (int32_t k = ra + h; k < rb; k += ST * G) {
    int32_t cc[ST];
    T vv[ST];
#pragma unroll
    for (int t = 0; t < ST; ++t) {
      const int32_t kk = k + t * G < rb ? k + t * G : ra;
      cc[t] = cl[kk];
      vv[t] = to_acc(vl[kk]);
    }
    T g[ST];
#pragma unroll
    for (int t = 0; t < ST; ++t) g[t] = x[cc[t]];
#pragma unroll
    for (int t = 0; t < ST; ++t)
      if (k + t * G < rb) acc[t & 3] += vv[t] * g[t];
  }
  T sum = (acc[0] + acc[1]) + (acc[2] + acc[3]);
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if (h != 0 || rl >= nr) return 0.0;
  const int64_t i = (int64_t)r0 + rl;
  if (SCALED) sum *= (T)scale[i];
  const T out = combine(alpha, sum, beta, y, i);
  y[i] = out;
  if constexpr (DOT) {
    if (d1) *d1 = (double)out * (double)out;
    return (double)wdot[i] * (double)out;
  }
  return 0.0;
}

template <typename V, typename T, int CMAX, bool SCALED, int WPB, int G, int ST, bool NT = false>
__global__ __launch_bounds__(64 * WPB) void k_csr_rl(int64_t nblocks,
                                                     const int32_t* __restrict__ blocks,
                                                     const int32_t* __restrict__ bnnz,
                                                     const int32_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ col,
                                                     const V* __restrict__ val,
                                                     const float* __restrict__ scale,
                                                     const T* __restrict__ x, T* __restrict__ y,
                                                     T alpha, T beta,
                                                     const int32_t* __restrict__ skip) {
  __shared__ V vl_all[WPB][CMAX];
  __shared__ int32_t cl_all[WPB][CMAX];
  if (skip && *skip) return;
  // wave-uniform (scalar block-bound loads)
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t b = xcd_remap(blockIdx.x, gridDim.x) * WPB + wv;
  if (b >= nblocks) return;
  rl_block<V, T, CMAX, SCALED, G, ST, false, NT>(b, blocks, bnnz, rowptr, col, val, scale, x, y,
                                                 alpha, beta, vl_all[wv], cl_all[wv]);
}

// The same product, y = A x, where each work-group of WPB waves (one row
// block each) also stores the sum of w[i] * y[i] over its rows (w = x for
// the p.q of a CG iteration, another vector for BiCGSTAB's r_hat.v) to
// part[blockIdx.x * NV] and, with NV = 2, the sum of y[i]^2 to
// part[blockIdx.x * NV + 1].  WPB is chosen so that the partials stay few
// enough for every block of the next kernel to add them.
template <typename V, typename T, int CMAX, bool SCALED, int WPB, int G, int ST, int NV>
__global__ __launch_bounds__(64 * WPB) void k_csr_rl_dot(int64_t nblocks,
                                                         const int32_t* __restrict__ blocks,
                                                         const int32_t* __restrict__ bnnz,
                                                         const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col,
                                                         const V* __restrict__ val,
                                                         const float* __restrict__ scale,
                                                         const T* __restrict__ x,
                                                         T* __restrict__ y,
                                                         const T* __restrict__ w,
                                                         double* __restrict__ part,
                                                         const int32_t* __restrict__ skip) {
  __shared__ V vl_all[WPB][CMAX];
  __shared__ int32_t cl_all[WPB][CMAX];
  __shared__ double red[NV][WPB];
  if (skip && *skip) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t b = xcd_remap(blockIdx.x, gridDim.x) * WPB + wv;
  double acc = 0.0, acc1 = 0.0;
  if (b < nblocks)
    acc = rl_block<V, T, CMAX, SCALED, G, ST, true>(b, blocks, bnnz, rowptr, col, val, scale, x,
                                                    y, T(1), T(0), vl_all[wv], cl_all[wv], w,
                                                    NV == 2 ? &acc1 : nullptr);
  acc = wave_total(acc);
  if constexpr (NV == 2) acc1 = wave_total(acc1);
  if ((threadIdx.x & 63) == 0) {
    red[0][wv] = acc;
    if constexpr (NV == 2) red[1][wv] = acc1;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double t = red[threadIdx.x][0];
#pragma unroll
    for (int q = 1; q < WPB; ++q) t += red[threadIdx.x][q];
    part[(int64_t)blockIdx.x * NV + threadIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// CSR, products through LDS: the same row blocks as above (<= 64 rows,
// <= CMAX entries), but every lane of the wave first forms products
// val[k] * x[col[k]] for a contiguous slice of the block's entries (loads
// coalesced, all gathers of a round in flight together) and stores them in
// LDS; then lane r sums row r's products in entry order with four
// interleaved accumulators.  LDS holds one value per entry (8 bytes in
// FP64) instead of a value and an index.
// ---------------------------------------------------------------------------
template <typename V, typename T, int CMAX, bool SCALED, int WPB, bool NT = false>
__global__ __launch_bounds__(64 * WPB) void k_csr_pr(int64_t nblocks,
                                                     const int32_t* __restrict__ blocks,
                                                     const int32_t* __restrict__ bnnz,
                                                     const int32_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ col,
                                                     const V* __restrict__ val,
                                                     const float* __restrict__ scale,
                                                     const T* __restrict__ x, T* __restrict__ y,
                                                     T alpha, T beta,
                                                     const int32_t* __restrict__ skip) {
  __shared__ T pl_all[WPB][CMAX];
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63;
  // wave-uniform (scalar block-bound loads)
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  T* pl = pl_all[wv];
  const int64_t b = xcd_remap(blockIdx.x, gridDim.x) * WPB + wv;
  if (b >= nblocks) return;
  const int32_t r0 = blocks[b], r1 = blocks[b + 1];
  const int32_t s = bnnz[b], e = bnnz[b + 1];
  const int nr = r1 - r0, len = e - s;
  if (len > CMAX) {  // a single long row
    T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int32_t k = s + lane;
    for (; k + 192 < e; k += 256) {
      const int32_t c0 = col[k], c1 = col[k + 64], c2 = col[k + 128], c3 = col[k + 192];
      const T v0 = to_acc(val[k]), v1 = to_acc(val[k + 64]), v2 = to_acc(val[k + 128]),
              v3 = to_acc(val[k + 192]);
      a0 += v0 * x[c0];
      a1 += v1 * x[c1];
      a2 += v2 * x[c2];
      a3 += v3 * x[c3];
    }
    for (; k < e; k += 64) a0 += to_acc(val[k]) * x[col[k]];
    T acc = wave_sum((a0 + a1) + (a2 + a3));
    if (lane == 0) {
      if (SCALED) acc *= (T)scale[r0];
      y[r0] = combine(alpha, acc, beta, y, r0);
    }
    return;
  }
  // row bounds of lane `lane` (an empty range at len for lanes past the
  // block): loaded unconditionally so that their wait can be deferred
  const int32_t ra = rowptr[r0 + (lane < nr ? lane : nr)] - s;
  const int32_t rb = rowptr[r0 + (lane < nr ? lane + 1 : nr)] - s;
  // products, U entries per lane in flight per round (sixteen for 4-byte
  // values in blocks of 1024 entries or more, else eight)
  constexpr int U = sizeof(T) == 4 && CMAX >= 1024 ? 16 : 8;
  for (int base = 0; base < len; base += U * 64) {
    int32_t c[U];
    typename Raw<V>::type v[U];
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const int k = base + t * 64 + lane;
      c[t] = 0;  // (v[t] of an unused slot is never read)
      if (k < len) {
        if constexpr (NT) {
          c[t] = ld_stream<true>(col + s + k);
          v[t] = ld_stream<true>(val + s + k);
        } else {
          c[t] = col[s + k];
          v[t] = Raw<V>::load(val, s + k);
        }
      }
    }
    // every gather in flight together (column 0 for unused slots, whose
    // products are discarded)
    T g[U];
#pragma unroll
    for (int t = 0; t < U; ++t) g[t] = x[c[t]];
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const int k = base + t * 64 + lane;
      if (k < len) pl[k] = to_acc(Raw<V>::value(v[t])) * g[t];
    }
  }
  wave_sync();
  if (lane >= nr) return;
  T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int32_t k = ra;
  for (; k + 3 < rb; k += 4) {
    s0 += pl[k];
    s1 += pl[k + 1];
    s2 += pl[k + 2];
    s3 += pl[k + 3];
  }
  for (; k < rb; ++k) s0 += pl[k];
  T sum = (s0 + s1) + (s2 + s3);
  const int64_t i = (int64_t)r0 + lane;
  if (SCALED) sum *= (T)scale[i];
  y[i] = combine(alpha, sum, beta, y, i);
}

// ---------------------------------------------------------------------------
// CSR, one thread per row: neighbouring lanes hold neighbouring rows, so on
// banded/stencil matrices the x gathers of one instruction are contiguous
// (as in ELL); the row's entries stream through the L1 over the iterations
// of the lane's loop.  Four independent accumulators per lane.
// ---------------------------------------------------------------------------
template <typename V, typename T, bool SCALED>
__global__ __launch_bounds__(256) void k_csr_row(int64_t n, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col,
                                                 const V* __restrict__ val,
                                                 const float* __restrict__ scale,
                                                 const T* __restrict__ x, T* __restrict__ y,
                                                 T alpha, T beta,
                                                 const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t i = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const int32_t a = rowptr[i], e = rowptr[i + 1];
  T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int32_t k = a;
  for (; k + 3 < e; k += 4) {
    const int32_t c0 = col[k], c1 = col[k + 1], c2 = col[k + 2], c3 = col[k + 3];
    const T v0 = to_acc(val[k]), v1 = to_acc(val[k + 1]), v2 = to_acc(val[k + 2]),
            v3 = to_acc(val[k + 3]);
    s0 += v0 * x[c0];
    s1 += v1 * x[c1];
    s2 += v2 * x[c2];
    s3 += v3 * x[c3];
  }
  for (; k < e; ++k) s0 += to_acc(val[k]) * x[col[k]];
  T sum = (s0 + s1) + (s2 + s3);
  if (SCALED) sum *= (T)scale[i];
  y[i] = combine(alpha, sum, beta, y, i);
}

// ---------------------------------------------------------------------------
// COO
// ---------------------------------------------------------------------------
// Loads the NPL consecutive elements p[0..NPL) into out: 16-byte loads when
// the run is a whole number of them (p is then 16-byte aligned: every device
// allocation is, and runs start at multiples of NPL elements), else one load
// each.
// NT: non-temporal loads (see ld_stream).
template <int NPL, bool NT = false, typename E>
__device__ __forceinline__ void load_run(const E* __restrict__ p, E (&out)[NPL]) {
  if constexpr ((NPL * sizeof(E)) % 16 == 0) {
    constexpr int NW = (int)(NPL * sizeof(E) / 16);
    typedef uint32_t w4 __attribute__((ext_vector_type(4)));
    w4 w[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      if constexpr (NT)
        w[j] = __builtin_nontemporal_load(reinterpret_cast<const w4*>(p) + j);
      else
        w[j] = reinterpret_cast<const w4*>(p)[j];
    }
    __builtin_memcpy(out, w, sizeof(out));
  } else {
#pragma unroll
    for (int t = 0; t < NPL; ++t) out[t] = p[t];
  }
}


// COO, one wave per chunk of 64*NPL entries, each lane's run held in
// registers: lane l loads entries l*NPL .. l*NPL+NPL-1 of the chunk itself
// (16-byte loads of row, col and val; the arrays are padded to whole chunks,
// so no load is masked), forms the products and sums the rows inside its
// run.  A segmented scan over the lanes (a lane's value is the sum of its
// last row; the flag says that row starts in the lane) joins rows across
// lanes; neighbouring lanes' rows come by shuffles.  A row that continues
// from the previous chunk leaves its partial in cont_row/cont_val for the
// fix-up pass, so no floating-point atomics are used and the result does not
// depend on scheduling.  k_coo adds in the same order (there the products
// are rounded before they are added; here they may be fused into the adds).
template <typename V, typename T, int NPL, bool ACCUM, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_coo_runs(int64_t nnz, int64_t nchunks,
                                                      const int32_t* __restrict__ row,
                                                      const int32_t* __restrict__ col,
                                                      const V* __restrict__ val,
                                                      const T* __restrict__ x, T* __restrict__ y,
                                                      T alpha, T beta,
                                                      int32_t* __restrict__ cont_row,
                                                      T* __restrict__ cont_val,
                                                      const int32_t* __restrict__ skip) {
  constexpr int C = 64 * NPL;
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ch = xcd_remap(blockIdx.x, gridDim.x) * WPB + wv;
  if (ch >= nchunks) return;
  const int64_t s = ch * C;
  const int len = (int)((nnz - s) < C ? (nnz - s) : C);
  const int k0 = lane * NPL;
  const int m = len - k0 < 0 ? 0 : (len - k0 < NPL ? len - k0 : NPL);  // entries of this lane
  const int32_t e0 = s > 0 ? row[s - 1] : -1;  // row just before the chunk
  // the arrays are padded to whole chunks with zeros, so every lane loads a
  // full run; entries past len are never summed (their column 0 is gathered)
  int32_t r[NPL], c[NPL];
  V v[NPL];
  load_run<NPL>(row + s + k0, r);
  load_run<NPL>(col + s + k0, c);
  load_run<NPL>(val + s + k0, v);
  T prod[NPL];
#pragma unroll
  for (int t = 0; t < NPL; ++t) prod[t] = x[c[t]];
#pragma unroll
  for (int t = 0; t < NPL; ++t) prod[t] = to_acc(v[t]) * prod[t];

  const int32_t first = __shfl(r[0], 0, 64);
  const int32_t prev_last = __shfl_up(r[NPL - 1], 1, 64);
  const int32_t next_first = __shfl_down(r[0], 1, 64);
  const bool first_continues = e0 == first;

  auto emit = [&](int32_t rr, T sum) {
    if (first_continues && rr == first) {
      cont_row[ch] = rr;
      cont_val[ch] = sum;
    } else if (ACCUM) {
      y[rr] = alpha * sum + y[rr];
    } else {
      y[rr] = combine(alpha, sum, beta, y, rr);
    }
  };
  if (lane == 0 && !first_continues) cont_row[ch] = -1;

  const bool active = m > 0;
  T vs = 0, hsum = 0, tsum = 0;
  int f = 1;
  int32_t hrow = 0, trow = 0;
  bool multi = false, hstart = false, tend = false;
  if (active) {
    hrow = r[0];
    hstart = (lane == 0 ? e0 : prev_last) != hrow;
    int32_t cur = hrow;
    T sum = 0;
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      if (t < m) {
        if (r[t] != cur) {
          if (!multi) {
            hsum = sum;
            multi = true;
          } else {
            emit(cur, sum);
          }
          cur = r[t];
          sum = 0;
        }
        sum += prod[t];
      }
    }
    trow = cur;
    tsum = sum;
    tend = (k0 + m == len) || next_first != cur;
    if (!multi) hsum = sum;
    vs = multi ? tsum : hsum;
    f = (multi || hstart) ? 1 : 0;
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T ov = __shfl_up(vs, d, 64);
    const int of = __shfl_up(f, d, 64);
    if (lane >= d) {
      if (!f) vs = ov + vs;
      f |= of;
    }
  }
  const T up = __shfl_up(vs, 1, 64);
  const T before = lane > 0 ? up : T(0);
  if (active) {
    if (multi) {
      emit(hrow, hstart ? hsum : before + hsum);
      if (tend) emit(trow, tsum);
    } else if (tend) {
      emit(hrow, vs);
    }
  }
}

// COO, products staged in LDS: a chunk's col and val are loaded coalesced
// (slot t of lane l is entry t*64 + l), so neighbouring lanes gather
// neighbouring entries' x; the products go to LDS and lane l reads back the
// run l*NPL .. l*NPL+NPL-1, whose row indices it loads itself.  The run is
// summed and rows are joined across lanes as in k_coo_runs.
template <typename V, typename T, int NPL, bool ACCUM, int WPB, bool NT = false>
__global__ __launch_bounds__(64 * WPB) void k_coo(int64_t nnz, int64_t nchunks,
                                                      const int32_t* __restrict__ row,
                                                      const int32_t* __restrict__ col,
                                                      const V* __restrict__ val,
                                                      const T* __restrict__ x, T* __restrict__ y,
                                                      T alpha, T beta,
                                                      int32_t* __restrict__ cont_row,
                                                      T* __restrict__ cont_val,
                                                      const int32_t* __restrict__ skip) {
  constexpr int C = 64 * NPL;
  if (skip && *skip) return;
  __shared__ T prod_all[WPB][C + C / 32];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  T* prod = prod_all[wv];
  const int64_t ch = xcd_remap(blockIdx.x, gridDim.x) * WPB + wv;
  if (ch >= nchunks) return;
  const int64_t s = ch * C;
  const int len = (int)((nnz - s) < C ? (nnz - s) : C);
  const int k0 = lane * NPL;
  const int m = len - k0 < 0 ? 0 : (len - k0 < NPL ? len - k0 : NPL);
  const int32_t e0 = s > 0 ? row[s - 1] : -1;
  int32_t r[NPL];
  {
    // padded arrays: every slot of the chunk is loadable; slots past len
    // gather x[0] and are never summed
    int32_t c[NPL];
    V v[NPL];
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      c[t] = ld_stream<NT>(col + s + t * 64 + lane);
      v[t] = ld_stream<NT>(val + s + t * 64 + lane);
    }
    load_run<NPL, NT>(row + s + k0, r);
    T g[NPL];
#pragma unroll
    for (int t = 0; t < NPL; ++t) g[t] = x[c[t]];
#pragma unroll
    for (int t = 0; t < NPL; ++t) prod[pad(t * 64 + lane)] = to_acc(v[t]) * g[t];
  }
  wave_sync();
  const int32_t first = __shfl(r[0], 0, 64);
  const int32_t prev_last = __shfl_up(r[NPL - 1], 1, 64);
  const int32_t next_first = __shfl_down(r[0], 1, 64);
  const bool first_continues = e0 == first;

  auto emit = [&](int32_t rr, T sum) {
    if (first_continues && rr == first) {
      cont_row[ch] = rr;
      cont_val[ch] = sum;
    } else if (ACCUM) {
      y[rr] = alpha * sum + y[rr];
    } else {
      y[rr] = combine(alpha, sum, beta, y, rr);
    }
  };
  if (lane == 0 && !first_continues) cont_row[ch] = -1;

  // the lane's products, all read before the first is used
  T pv[NPL];
#pragma unroll
  for (int t = 0; t < NPL; ++t) pv[t] = prod[pad(k0 + t)];
  const bool active = m > 0;
  T vs = 0, hsum = 0, tsum = 0;
  int f = 1;
  int32_t hrow = 0, trow = 0;
  bool multi = false, hstart = false, tend = false;
  if (active) {
    hrow = r[0];
    hstart = (lane == 0 ? e0 : prev_last) != hrow;
    int32_t cur = hrow;
    T sum = 0;
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      if (t < m) {
        if (r[t] != cur) {
          if (!multi) {
            hsum = sum;
            multi = true;
          } else {
            emit(cur, sum);
          }
          cur = r[t];
          sum = 0;
        }
        sum += pv[t];
      }
    }
    trow = cur;
    tsum = sum;
    tend = (k0 + m == len) || next_first != cur;
    if (!multi) hsum = sum;
    vs = multi ? tsum : hsum;
    f = (multi || hstart) ? 1 : 0;
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T ov = __shfl_up(vs, d, 64);
    const int of = __shfl_up(f, d, 64);
    if (lane >= d) {
      if (!f) vs = ov + vs;
      f |= of;
    }
  }
  const T up = __shfl_up(vs, 1, 64);
  const T before = lane > 0 ? up : T(0);
  if (active) {
    if (multi) {
      emit(hrow, hstart ? hsum : before + hsum);
      if (tend) emit(trow, tsum);
    } else if (tend) {
      emit(hrow, vs);
    }
  }
}

// CSR by the merge path: chunk `ch` holds entries s .. s+len-1 (equal
// chunks of C = 64 * NPL entries whatever the rows).  Its col and val are
// loaded coalesced (slot t of lane l is entry t*64 + l; slots past the
// matrix's last entry re-read it, their products are never summed), the
// products go to LDS, and the row pointers of rows crow[ch] .. crow[ch+1]
// (at most C + 2 values, checked at set-up) go to a second LDS table, where
// each lane finds the row of the first entry of its run
// (l*NPL .. l*NPL+NPL-1) by binary search and steps through the rest.  The
// runs are then summed and joined across lanes exactly as in k_coo, and rows
// cut by chunk edges are completed by k_coo_fix.  Against COO it reads no
// row index per entry; against the row-block stream kernel every wave gets
// the same number of entries whatever the row lengths.
//
// PANEL: the matrix is the stack of column panels (rows are a row's entries
// of one column slice; rid gives each stacked row's slot p*n + i): a row's
// sum is stored as is (no alpha, beta, scale) to y[rid[row]], the panel
// partials that k_panel_add joins.
//
// dchunk (not with PANEL; alpha = 1, beta = 0): each chunk also stores the
// sum of x[row] * s over the partial sums s it emits, cut rows' pieces
// included, so the chunks' values add up to x.y (CG's p.q) once k_coo_fix
// has completed the cut rows: x_r (s_1 + s_2) = x_r s_1 + x_r s_2.
template <typename V, typename T, int NPL, int WPB, bool SCALED, bool PANEL>
__global__ __launch_bounds__(64 * WPB) void k_csr_merge(int64_t nnz, int64_t nchunks,
                                                       const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ crow,
                                                       const int32_t* __restrict__ col,
                                                       const V* __restrict__ val,
                                                       const float* __restrict__ scale,
                                                       const int32_t* __restrict__ rid,
                                                       const T* __restrict__ x, T* __restrict__ y,
                                                       T alpha, T beta,
                                                       int32_t* __restrict__ cont_row,
                                                       T* __restrict__ cont_val,
                                                       const int32_t* __restrict__ skip,
                                                       double* __restrict__ dchunk) {
  constexpr int C = 64 * NPL;
  if (skip && *skip) return;
  __shared__ T prod_all[WPB][C + C / 32];
  __shared__ int32_t rl_all[WPB][C + 2];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  T* prod = prod_all[wv];
  int32_t* rl = rl_all[wv];
  const int64_t ch = xcd_remap(blockIdx.x, gridDim.x) * WPB + wv;
  if (ch >= nchunks) return;
  const int64_t s = ch * C;
  const int len = (int)((nnz - s) < C ? (nnz - s) : C);
  const int32_t r0 = crow[ch], r1 = crow[ch + 1];
  const int span = r1 - r0 + 2;  // row pointers r0 .. r1 + 1 (<= C + 2)
  for (int j = lane; j < span; j += 64) rl[j] = rowptr[r0 + j];
  {
    int32_t c[NPL];
    typename Raw<V>::type v[NPL];  // 2-byte values staged one per register
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int k = t * 64 + lane;
      const int64_t kk = s + (k < len ? k : len - 1);
      c[t] = col[kk];
      v[t] = Raw<V>::load(val, kk);
    }
    T g[NPL];
#pragma unroll
    for (int t = 0; t < NPL; ++t) g[t] = x[c[t]];
#pragma unroll
    for (int t = 0; t < NPL; ++t)
      prod[pad(t * 64 + lane)] = to_acc(Raw<V>::value(v[t])) * g[t];
  }
  wave_sync();
  const int k0 = lane * NPL;
  const int m = len - k0 < 0 ? 0 : (len - k0 < NPL ? len - k0 : NPL);  // entries of this lane
  T pv[NPL];
#pragma unroll
  for (int t = 0; t < NPL; ++t) pv[t] = prod[pad(k0 + t)];
  // rows of the run: the last table index j with rl[j] <= entry (rl[0] <= s,
  // and rl[span - 1] lies past the chunk's last entry, so j stays in range)
  int32_t r[NPL];
  {
    const int32_t kg = (int32_t)s + (m > 0 ? k0 : 0);
    int lo = 0, hi = span - 2;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rl[mid] <= kg) lo = mid;
      else hi = mid - 1;
    }
    int j = lo;
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      if (t < m)
        while (rl[j + 1] <= kg + t) ++j;
      r[t] = r0 + j;
    }
  }
  const int32_t first = r0;
  const int32_t prev_last = __shfl_up(r[NPL - 1], 1, 64);
  const int32_t next_first = __shfl_down(r[0], 1, 64);
  const bool first_continues = rl[0] < s;  // row r0 began in an earlier chunk

  // a row's partial sums are scaled (FP16 values with per-row scales) before
  // they are stored or joined by the fix-up pass
  double dacc = 0.0;
  auto emit = [&](int32_t rr, T sum) {
    if (SCALED) sum *= (T)scale[rr];
    if (!PANEL && dchunk) dacc += (double)x[rr] * (double)sum;
    if (first_continues && rr == first) {
      cont_row[ch] = rr;
      cont_val[ch] = sum;
    } else if (PANEL) {
      y[rid[rr]] = sum;
    } else {
      y[rr] = combine(alpha, sum, beta, y, rr);
    }
  };
  if (lane == 0 && !first_continues) cont_row[ch] = -1;

  const bool active = m > 0;
  T vs = 0, hsum = 0, tsum = 0;
  int f = 1;
  int32_t hrow = 0, trow = 0;
  bool multi = false, hstart = false, tend = false;
  if (active) {
    hrow = r[0];
    hstart = lane == 0 ? !first_continues : prev_last != hrow;
    int32_t cur = hrow;
    T sum = 0;
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      if (t < m) {
        if (r[t] != cur) {
          if (!multi) {
            hsum = sum;
            multi = true;
          } else {
            emit(cur, sum);
          }
          cur = r[t];
          sum = 0;
        }
        sum += pv[t];
      }
    }
    trow = cur;
    tsum = sum;
    tend = (k0 + m == len) || next_first != cur;
    if (!multi) hsum = sum;
    vs = multi ? tsum : hsum;
    f = (multi || hstart) ? 1 : 0;
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T ov = __shfl_up(vs, d, 64);
    const int of = __shfl_up(f, d, 64);
    if (lane >= d) {
      if (!f) vs = ov + vs;
      f |= of;
    }
  }
  const T up = __shfl_up(vs, 1, 64);
  const T before = lane > 0 ? up : T(0);
  if (active) {
    if (multi) {
      emit(hrow, hstart ? hsum : before + hsum);
      if (tend) emit(trow, tsum);
    } else if (tend) {
      emit(hrow, vs);
    }
  }
  if (!PANEL && dchunk) {
    const double t = wave_total(dacc);
    if (lane == 0) dchunk[ch] = t;
  }
}

// Adds the continuation partials of rows that straddle chunks, in chunk
// order, to the value their first chunk wrote (at y[rid[r]] when rid is
// given: the stacked rows of column panels).  With dpart (256 threads a
// work-group) each work-group also stores the sum of its chunks' dchunk
// values, in chunk order, to dpart[blockIdx.x].
template <typename T>
__global__ __launch_bounds__(256) void k_coo_fix(int64_t nchunks,
                                                 const int32_t* __restrict__ cont_row,
                                                 const T* __restrict__ cont_val,
                                                 T* __restrict__ y, T alpha,
                                                 const int32_t* __restrict__ skip,
                                                 const int32_t* __restrict__ rid,
                                                 const double* __restrict__ dchunk = nullptr,
                                                 double* __restrict__ dpart = nullptr) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool on = c < nchunks && !(skip && *skip);
  if (on) {
    const int32_t r = cont_row[c];
    if (r >= 0 && !(c > 0 && cont_row[c - 1] == r)) {
      T sum = cont_val[c];
      for (int64_t d = c + 1; d < nchunks && cont_row[d] == r; ++d) sum += cont_val[d];
      const int64_t i = rid ? rid[r] : r;
      y[i] = y[i] + alpha * sum;
    }
  }
  if (dpart) {
    __shared__ double red[4];
    const double t = wave_total(on ? dchunk[c] : 0.0);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) dpart[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
  }
}

// Column panels: y_i = alpha * s_i * (sum of row i's panel partials, in
// panel order) + beta * y_i, over every row (a row with no entries gets 0).
// With DOT (x = p, y = q = A p of a CG iteration) each work-group also
// stores the sum of x[i] * y[i] over its rows to dpart[blockIdx.x].
template <typename T, bool SCALED, bool DOT>
__global__ __launch_bounds__(256) void k_panel_add(int64_t n, int P,
                                                   const uint8_t* __restrict__ mask,
                                                   const T* __restrict__ part,
                                                   const float* __restrict__ scale,
                                                   T* __restrict__ y, T alpha, T beta,
                                                   const int32_t* __restrict__ skip,
                                                   const T* __restrict__ x,
                                                   double* __restrict__ dpart) {
  if (skip && *skip) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double dot = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const unsigned m = mask[i];
    T v[8];
#pragma unroll
    for (int p = 0; p < 8; ++p)
      if (p < P) v[p] = (m >> p) & 1u ? part[(int64_t)p * n + i] : T(0);
    T s = 0;
#pragma unroll
    for (int p = 0; p < 8; ++p)
      if (p < P) s += v[p];
    if (SCALED) s *= (T)scale[i];
    const T out = combine(alpha, s, beta, y, i);
    y[i] = out;
    if constexpr (DOT) dot += (double)x[i] * (double)out;
  }
  if constexpr (DOT) {
    __shared__ double red[4];
    dot = wave_total(dot);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dot;
    __syncthreads();
    if (threadIdx.x == 0) dpart[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
  }
}

template <typename T>
__global__ void k_empty_rows(int64_t count, const int32_t* __restrict__ rows,
                             T* __restrict__ y, T beta, const int32_t* __restrict__ skip) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count || (skip && *skip)) return;
  const int32_t r = rows[k];
  y[r] = beta == T(0) ? T(0) : beta * y[r];
}

// ---------------------------------------------------------------------------
// ELL
// ---------------------------------------------------------------------------
template <typename V, typename T, int W, bool NT = false>
__global__ __launch_bounds__(64 * W) void k_ell(int64_t n, int64_t K, int64_t ld,
                                                const int32_t* __restrict__ ecol,
                                                const V* __restrict__ eval,
                                                const T* __restrict__ x, T* __restrict__ y,
                                                T alpha, T beta,
                                                const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t g = xcd_remap(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = g * 64 + lane;  // < ld: the grid covers ld / 64 groups
  // Four slots per round, in one of two forms chosen by measurement on the
  // 27-point 128^3 matrix.  With FP64 values the per-slot form (each slot's
  // value load and gather under its own test) runs at 136 us against 140 us
  // for the batched form; with FP32 values the batched form (index and
  // value loads of all four slots together, slots past K re-reading slot j
  // so every load is unconditional, then the four gathers, padding reading
  // x[0] with its product discarded by a select) runs at 93 us against
  // 101 us.  In both, padding never multiplies x.
  T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (int64_t j = w; j < K; j += 4 * W) {
    if constexpr (sizeof(V) == 8) {
      const int64_t o0 = j * ld + i;
      const int32_t c0 = ld_stream<NT>(ecol + o0);
      const int32_t c1 = (j + W < K) ? ld_stream<NT>(ecol + o0 + W * ld) : -1;
      const int32_t c2 = (j + 2 * W < K) ? ld_stream<NT>(ecol + o0 + 2 * W * ld) : -1;
      const int32_t c3 = (j + 3 * W < K) ? ld_stream<NT>(ecol + o0 + 3 * W * ld) : -1;
      if (c0 >= 0) a0 += to_acc(ld_stream<NT>(eval + o0)) * x[c0];
      if (c1 >= 0) a1 += to_acc(ld_stream<NT>(eval + o0 + W * ld)) * x[c1];
      if (c2 >= 0) a2 += to_acc(ld_stream<NT>(eval + o0 + 2 * W * ld)) * x[c2];
      if (c3 >= 0) a3 += to_acc(ld_stream<NT>(eval + o0 + 3 * W * ld)) * x[c3];
      if (!__any(c3 >= 0)) break;  // every later slot of these rows is padding
    } else {
      int32_t c[4];
      V v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t jj = j + u * W;
        const int64_t o = (jj < K ? jj : j) * ld + i;
        c[u] = ld_stream<NT>(ecol + o);
        v[u] = ld_stream<NT>(eval + o);
      }
#pragma unroll
      for (int u = 1; u < 4; ++u)
        if (j + u * W >= K) c[u] = -1;
      T g[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) g[u] = x[c[u] >= 0 ? c[u] : 0];
      a0 += c[0] >= 0 ? to_acc(v[0]) * g[0] : T(0);
      a1 += c[1] >= 0 ? to_acc(v[1]) * g[1] : T(0);
      a2 += c[2] >= 0 ? to_acc(v[2]) * g[2] : T(0);
      a3 += c[3] >= 0 ? to_acc(v[3]) * g[3] : T(0);
      if (!__any(c[3] >= 0)) break;  // every later slot of these rows is padding
    }
  }
  T acc = (a0 + a1) + (a2 + a3);
  if (W > 1) {
    __shared__ T red[W][64];
    red[w][lane] = acc;
    __syncthreads();
    if (w != 0) return;
    acc = red[0][lane];
#pragma unroll
    for (int q = 1; q < W; ++q) acc += red[q][lane];
  }
  if (i < n) y[i] = combine(alpha, acc, beta, y, i);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename V, typename T, int G, bool SCALED>
void launch_csr_vec(mxs_ctx* ctx, const mxs_matrix* A, T alpha, const T* x, T beta, T* y,
                    const int32_t* skip) {
  const CsrPart& P = A->csr;
  const V* val = (const V*)P.val;
  const int rows_per_wg = (256 / G) * P.rpg;
  const dim3 grid((unsigned)((A->n + rows_per_wg - 1) / rows_per_wg));
  if (P.rpg == 8)
    k_csr_vec<V, T, G, (G >= 8 ? 8 : G), SCALED><<<grid, 256, 0, ctx->stream>>>(
        A->n, P.rowptr, P.col, val, P.scale, x, y, alpha, beta, skip);
  else if (P.rpg == 2)
    k_csr_vec<V, T, G, 2, SCALED><<<grid, 256, 0, ctx->stream>>>(
        A->n, P.rowptr, P.col, val, P.scale, x, y, alpha, beta, skip);
  else
    k_csr_vec<V, T, G, 4, SCALED><<<grid, 256, 0, ctx->stream>>>(
        A->n, P.rowptr, P.col, val, P.scale, x, y, alpha, beta, skip);
}

template <typename V, typename T, bool SCALED, int WPB>
void launch_csr_stream(mxs_ctx* ctx, const CsrPart& P, T alpha, const T* x, T beta, T* y,
                       const int32_t* skip) {
  const V* val = (const V*)P.val;
  const dim3 grid((unsigned)((P.nblocks + WPB - 1) / WPB));
  switch (P.block_nnz) {
    case 256:
      k_csr<V, T, 4, SCALED, WPB><<<grid, 64 * WPB, 0, ctx->stream>>>(
          P.nblocks, P.blocks, P.bnnz, P.rowptr, P.col, val, P.scale, x, y, alpha, beta, skip);
      break;
    case 1024:
      k_csr<V, T, 16, SCALED, WPB><<<grid, 64 * WPB, 0, ctx->stream>>>(
          P.nblocks, P.blocks, P.bnnz, P.rowptr, P.col, val, P.scale, x, y, alpha, beta, skip);
      break;
    default:
      k_csr<V, T, 8, SCALED, WPB><<<grid, 64 * WPB, 0, ctx->stream>>>(
          P.nblocks, P.blocks, P.bnnz, P.rowptr, P.col, val, P.scale, x, y, alpha, beta, skip);
  }
}

template <typename V, typename T, bool SCALED, int CMAX, int G>
void launch_csr_rl_g(mxs_ctx* ctx, const CsrPart& P, T alpha, const T* x, T beta, T* y,
                     const int32_t* skip, bool nt) {
  constexpr int WPB = 2;
  const dim3 grid((unsigned)((P.nblocks + WPB - 1) / WPB));
  if constexpr (CMAX == 1024 && kNtValue<V>) {
    if (nt) {
      if (P.rl_step == 16)
        k_csr_rl<V, T, CMAX, SCALED, WPB, G, 16, true><<<grid, 64 * WPB, 0, ctx->stream>>>(
            P.nblocks, P.blocks, P.bnnz, P.rowptr, P.col, (const V*)P.val, P.scale, x, y, alpha,
            beta, skip);
      else
        k_csr_rl<V, T, CMAX, SCALED, WPB, G, 8, true><<<grid, 64 * WPB, 0, ctx->stream>>>(
            P.nblocks, P.blocks, P.bnnz, P.rowptr, P.col, (const V*)P.val, P.scale, x, y, alpha,
            beta, skip);
      return;
    }
  }
  if (P.rl_step == 16)
    k_csr_rl<V, T, CMAX, SCALED, WPB, G, 16><<<grid, 64 * WPB, 0, ctx->stream>>>(
        P.nblocks, P.blocks, P.bnnz, P.rowptr, P.col, (const V*)P.val, P.scale, x, y, alpha,
        beta, skip);
  else
    k_csr_rl<V, T, CMAX, SCALED, WPB, G, 8><<<grid, 64 * WPB, 0, ctx->stream>>>(
        P.nblocks, P.blocks, P.bnnz, P.rowptr, P.col, (const V*)P.val, P.scale, x, y, alpha,
        beta, skip);
}

template <typename V, typename T, bool SCALED, int CMAX>
void launch_csr_rl(mxs_ctx* ctx, const CsrPart& P, T alpha, const T* x, T beta, T* y,
                   const int32_t* skip, bool nt) {
  if (P.rl_lanes == 4)
    launch_csr_rl_g<V, T, SCALED, CMAX, 4>(ctx, P, alpha, x, beta, y, skip, nt);
  else if (P.rl_lanes == 2)
    launch_csr_rl_g<V, T, SCALED, CMAX, 2>(ctx, P, alpha, x, beta, y, skip, nt);
  else
    launch_csr_rl_g<V, T, SCALED, CMAX, 1>(ctx, P, alpha, x, beta, y, skip, nt);
}

template <typename V, typename T, bool SCALED, int CMAX, int G, int ST, int WPB>
int launch_csr_rl_dot_w(mxs_ctx* ctx, const CsrPart& P, const T* x, T* y, const int32_t* skip,
                        double* dpart, const T* w, int nv) {
  const int g = (int)((P.nblocks + WPB - 1) / WPB);
  if (nv == 2)
    k_csr_rl_dot<V, T, CMAX, SCALED, WPB, G, ST, 2><<<g, 64 * WPB, 0, ctx->stream>>>(
        P.nblocks, P.blocks, P.bnnz, P.rowptr, P.col, (const V*)P.val, P.scale, x, y, w, dpart,
        skip);
  else
    k_csr_rl_dot<V, T, CMAX, SCALED, WPB, G, ST, 1><<<g, 64 * WPB, 0, ctx->stream>>>(
        P.nblocks, P.blocks, P.bnnz, P.rowptr, P.col, (const V*)P.val, P.scale, x, y, w, dpart,
        skip);
  return g;
}

// the fewest waves per work-group (2, 4 or 8) that keep the partials within
// kDotPartials; 0 (no launch) when even 8 do not
template <typename V, typename T, bool SCALED, int CMAX, int G, int ST>
int launch_csr_rl_dot_g(mxs_ctx* ctx, const CsrPart& P, const T* x, T* y, const int32_t* skip,
                        double* dpart, const T* w, int nv) {
  // LDS of a work-group: WPB tables of CMAX values and column indices
  constexpr size_t per_wave = (size_t)CMAX * (sizeof(V) + sizeof(int32_t));
  if (P.nblocks <= 2 * (int64_t)kDotPartials)
    return launch_csr_rl_dot_w<V, T, SCALED, CMAX, G, ST, 2>(ctx, P, x, y, skip, dpart, w, nv);
  if constexpr (4 * per_wave <= 98304) {
    if (P.nblocks <= 4 * (int64_t)kDotPartials)
      return launch_csr_rl_dot_w<V, T, SCALED, CMAX, G, ST, 4>(ctx, P, x, y, skip, dpart, w, nv);
  }
  if constexpr (8 * per_wave <= 98304) {
    if (P.nblocks <= 8 * (int64_t)kDotPartials)
      return launch_csr_rl_dot_w<V, T, SCALED, CMAX, G, ST, 8>(ctx, P, x, y, skip, dpart, w, nv);
  }
  return 0;
}

template <typename V, typename T, bool SCALED, int CMAX>
int launch_csr_rl_dot(mxs_ctx* ctx, const CsrPart& P, const T* x, T* y, const int32_t* skip,
                      double* dpart, const T* w, int nv) {
#define MXS_RL_DOT(GG)                                                               \
  return P.rl_step == 16                                                             \
             ? launch_csr_rl_dot_g<V, T, SCALED, CMAX, GG, 16>(ctx, P, x, y, skip, dpart, w, nv) \
             : launch_csr_rl_dot_g<V, T, SCALED, CMAX, GG, 8>(ctx, P, x, y, skip, dpart, w, nv);
  if (P.rl_lanes == 4) MXS_RL_DOT(4)
  if (P.rl_lanes == 2) MXS_RL_DOT(2)
  MXS_RL_DOT(1)
#undef MXS_RL_DOT
}

template <typename V, typename T, bool SCALED, int CMAX, int WPB>
void launch_csr_pr_w(mxs_ctx* ctx, const CsrPart& P, T alpha, const T* x, T beta, T* y,
                     const int32_t* skip, bool nt) {
  const dim3 grid((unsigned)((P.nblocks + WPB - 1) / WPB));
  if constexpr (CMAX == 512 && kNtValue<V>) {
    if (nt) {
      k_csr_pr<V, T, CMAX, SCALED, WPB, true><<<grid, 64 * WPB, 0, ctx->stream>>>(
          P.nblocks, P.blocks, P.bnnz, P.rowptr, P.col, (const V*)P.val, P.scale, x, y, alpha,
          beta, skip);
      return;
    }
  }
  k_csr_pr<V, T, CMAX, SCALED, WPB><<<grid, 64 * WPB, 0, ctx->stream>>>(
      P.nblocks, P.blocks, P.bnnz, P.rowptr, P.col, (const V*)P.val, P.scale, x, y, alpha, beta,
      skip);
}

template <typename V, typename T, bool SCALED, int CMAX>
void launch_csr_pr(mxs_ctx* ctx, const CsrPart& P, T alpha, const T* x, T beta, T* y,
                   const int32_t* skip, bool nt) {
  if (P.wpb == 1)
    launch_csr_pr_w<V, T, SCALED, CMAX, 1>(ctx, P, alpha, x, beta, y, skip, nt);
  else if (P.wpb == 2)
    launch_csr_pr_w<V, T, SCALED, CMAX, 2>(ctx, P, alpha, x, beta, y, skip, nt);
  else
    launch_csr_pr_w<V, T, SCALED, CMAX, 4>(ctx, P, alpha, x, beta, y, skip, nt);
}

// continuation partials of a chunked product: the row each chunk's first
// run ends in (or -1) and that run's partial sum, one per chunk
struct Cont {
  int32_t* row;
  void* val;
};

Cont cont_of(void* scratch, int64_t nchunks) {
  const size_t rb = ((size_t)(nchunks + 1) * sizeof(int32_t) + 255) & ~(size_t)255;
  return Cont{(int32_t*)scratch, (char*)scratch + rb};
}

template <typename V, typename T, int NPL, int WPB, bool SCALED, bool PANEL>
void launch_csr_merge_w(mxs_ctx* ctx, const CsrPart& P, int64_t nnz, T alpha, const T* x,
                        T beta, T* y, const int32_t* skip, Cont c, double* dchunk) {
  const dim3 grid((unsigned)((P.nchunks + WPB - 1) / WPB));
  if constexpr (PANEL)
    k_csr_merge<V, T, NPL, WPB, false, true><<<grid, 64 * WPB, 0, ctx->stream>>>(
        nnz, P.nchunks, P.srowptr, P.crow, P.scol, (const V*)P.sval, nullptr, P.srid, x, y,
        T(1), T(0), c.row, (T*)c.val, skip, nullptr);
  else
    k_csr_merge<V, T, NPL, WPB, SCALED, false><<<grid, 64 * WPB, 0, ctx->stream>>>(
        nnz, P.nchunks, P.rowptr, P.crow, P.col, (const V*)P.val, P.scale, nullptr, x, y,
        alpha, beta, c.row, (T*)c.val, skip, dchunk);
}

template <typename V, typename T, int NPL, bool SCALED, bool PANEL>
void launch_csr_merge_n(mxs_ctx* ctx, const CsrPart& P, int64_t nnz, T alpha, const T* x,
                        T beta, T* y, const int32_t* skip, Cont c, double* dchunk) {
  if (P.wpb == 1)
    launch_csr_merge_w<V, T, NPL, 1, SCALED, PANEL>(ctx, P, nnz, alpha, x, beta, y, skip, c,
                                                     dchunk);
  else
    launch_csr_merge_w<V, T, NPL, 4, SCALED, PANEL>(ctx, P, nnz, alpha, x, beta, y, skip, c,
                                                     dchunk);
}

template <typename V, typename T, bool SCALED, bool PANEL>
void launch_csr_merge_c(mxs_ctx* ctx, const CsrPart& P, int64_t nnz, T alpha, const T* x,
                        T beta, T* y, const int32_t* skip, Cont c, double* dchunk = nullptr) {
  switch (P.block_nnz) {
    case 256: launch_csr_merge_n<V, T, 4, SCALED, PANEL>(ctx, P, nnz, alpha, x, beta, y, skip, c, dchunk); break;
    case 512: launch_csr_merge_n<V, T, 8, SCALED, PANEL>(ctx, P, nnz, alpha, x, beta, y, skip, c, dchunk); break;
    default: launch_csr_merge_n<V, T, 16, SCALED, PANEL>(ctx, P, nnz, alpha, x, beta, y, skip, c, dchunk);
  }
}

// bytes of the continuation partials of `nchunks` chunks (row indices
// rounded to 256 bytes, then one partial of up to 8 bytes each, rounded)
size_t cont_bytes(int64_t nchunks) {
  const size_t rb = ((size_t)(nchunks + 1) * sizeof(int32_t) + 255) & ~(size_t)255;
  return rb + (((size_t)(nchunks + 1) * sizeof(double) + 255) & ~(size_t)255);
}

template <typename V, typename T, bool ACCUM, int WPB>
void launch_coo_chunks(mxs_ctx* ctx, const CooPart& P, T alpha, const T* x, T beta, T* y,
                       const int32_t* skip, Cont c);

// merge-path CSR: empty rows, the chunks, then the fix-up of cut rows; with
// column panels: the stacked chunks into the panel partials (scratch after
// the continuation partials), their fix-up, then the pass that adds them.
// With FP64 or FP32 values the panel copy also holds each entry's output
// slot (srow), and a plain product runs its chunks as COO chunks: on the
// power-law and random SPD matrices 76 vs 89 us (s = 2.0), 142 vs 145
// (s = 1.79) and 122 vs 137 (random SPD), cold, FP64: no row-pointer table,
// search or slot lookup per chunk.
// With dpart (CG's q = A p, alpha = 1, beta = 0) the partials of p.q go to
// dpart and their count to *ndpart: from the panel-adding pass, or without
// panels from the fix-up pass over the chunks' own sums (scratch after the
// continuation partials), one per 256 chunks.
template <typename V, typename T, bool SCALED>
void launch_csr_merge(mxs_ctx* ctx, const mxs_matrix* A, T alpha, const T* x, T beta, T* y,
                      const int32_t* skip, void* scratch, double* dpart = nullptr,
                      int* ndpart = nullptr) {
  const CsrPart& P = A->csr;
  if (P.panels > 1) {
    if (P.nchunks == 0) return;
    const Cont c = cont_of(scratch, P.nchunks);
    T* part = (T*)((char*)scratch + cont_bytes(P.nchunks));
    // plain products take the COO chunks; CG's product with its p.q keeps
    // the merge kernel, whose smaller footprint (no row index per entry)
    // shares the Infinity Cache better with the solver's vectors: random
    // SPD 121.8 vs 128.0 us per CG iteration, same box
    bool as_coo = false;
    if constexpr (!SCALED) as_coo = P.srow != nullptr && dpart == nullptr;
    if (as_coo) {
      CooPart Q;
      Q.row = P.srow;
      Q.col = P.scol;
      Q.val = P.sval;
      Q.nnz = A->nnz;
      Q.nchunks = P.nchunks;
      Q.block_nnz = P.block_nnz;
      Q.wpb = P.wpb;
      Q.kernel = MXS_COO_LDS;
      if constexpr (!SCALED) {
        if (P.wpb == 4)
          launch_coo_chunks<V, T, false, 4>(ctx, Q, T(1), x, T(0), part, skip, c);
        else
          launch_coo_chunks<V, T, false, 1>(ctx, Q, T(1), x, T(0), part, skip, c);
      }
      if (P.nchunks > 1)
        k_coo_fix<T><<<(unsigned)((P.nchunks + 255) / 256), 256, 0, ctx->stream>>>(
            P.nchunks, c.row, (T*)c.val, part, T(1), skip, nullptr);
    } else {
      launch_csr_merge_c<V, T, false, true>(ctx, P, A->nnz, alpha, x, beta, part, skip, c);
      if (P.nchunks > 1)
        k_coo_fix<T><<<(unsigned)((P.nchunks + 255) / 256), 256, 0, ctx->stream>>>(
            P.nchunks, c.row, (T*)c.val, part, T(1), skip, P.srid);
    }
    const unsigned g = (unsigned)std::min<int64_t>((A->n + 255) / 256, (int64_t)ctx->num_cus * 16);
    if (dpart) {
      const unsigned gd = std::min<unsigned>(g, kDotPartials);
      k_panel_add<T, SCALED, true><<<gd, 256, 0, ctx->stream>>>(
          A->n, P.panels, P.pmask, part, P.scale, y, alpha, beta, skip, x, dpart);
      *ndpart = (int)gd;
    } else {
      k_panel_add<T, SCALED, false><<<g, 256, 0, ctx->stream>>>(
          A->n, P.panels, P.pmask, part, P.scale, y, alpha, beta, skip, nullptr, nullptr);
    }
    return;
  }
  if (P.nempty > 0)
    k_empty_rows<T><<<(unsigned)((P.nempty + 255) / 256), 256, 0, ctx->stream>>>(
        P.nempty, P.empty_rows, y, beta, skip);
  if (P.nchunks == 0) return;
  const Cont c = cont_of(scratch, P.nchunks);
  const unsigned gf = (unsigned)((P.nchunks + 255) / 256);
  if (dpart) {
    double* dchunk = (double*)((char*)scratch + cont_bytes(P.nchunks));
    launch_csr_merge_c<V, T, SCALED, false>(ctx, P, A->nnz, alpha, x, beta, y, skip, c,
                                            dchunk);
    k_coo_fix<T><<<gf, 256, 0, ctx->stream>>>(P.nchunks, c.row, (T*)c.val, y, alpha, skip,
                                              nullptr, dchunk, dpart);
    *ndpart = (int)gf;
    return;
  }
  launch_csr_merge_c<V, T, SCALED, false>(ctx, P, A->nnz, alpha, x, beta, y, skip, c);
  if (P.nchunks > 1)
    k_coo_fix<T><<<gf, 256, 0, ctx->stream>>>(P.nchunks, c.row, (T*)c.val, y, alpha, skip,
                                              nullptr);
}

template <typename V, typename T, bool SCALED>
void launch_csr(mxs_ctx* ctx, const mxs_matrix* A, T alpha, const T* x, T beta, T* y,
                const int32_t* skip, void* scratch) {
  const CsrPart& P = A->csr;
  if (P.merge) {
    // set-up admits FP64, FP32 and row-scaled FP16 values
    if constexpr (std::is_same_v<V, double> || std::is_same_v<V, float> ||
                  std::is_same_v<V, _Float16>)
      launch_csr_merge<V, T, SCALED>(ctx, A, alpha, x, beta, y, skip, scratch);
    return;
  }
  // col and val of a matrix larger than the Infinity Cache are streamed
  // non-temporally
  const bool nt = (double)A->nnz * (4 + sizeof(V)) > kStreamNtBytes;
  if (P.products) {
    if (P.nblocks == 0) return;
    if (P.block_nnz <= 512)
      launch_csr_pr<V, T, SCALED, 512>(ctx, P, alpha, x, beta, y, skip, nt);
    else if (P.block_nnz <= 1024)
      launch_csr_pr<V, T, SCALED, 1024>(ctx, P, alpha, x, beta, y, skip, nt);
    else
      launch_csr_pr<V, T, SCALED, 2048>(ctx, P, alpha, x, beta, y, skip, nt);
    return;
  }
  if (P.rows_lds) {
    if (P.nblocks == 0) return;
    if (P.block_nnz <= 512)
      launch_csr_rl<V, T, SCALED, 512>(ctx, P, alpha, x, beta, y, skip, nt);
    else if (P.block_nnz <= 1024)
      launch_csr_rl<V, T, SCALED, 1024>(ctx, P, alpha, x, beta, y, skip, nt);
    else
      launch_csr_rl<V, T, SCALED, 2048>(ctx, P, alpha, x, beta, y, skip, nt);
    return;
  }
  if (P.lanes == 1) {
    const dim3 grid((unsigned)((A->n + 255) / 256));
    k_csr_row<V, T, SCALED><<<grid, 256, 0, ctx->stream>>>(A->n, P.rowptr, P.col,
                                                          (const V*)P.val, P.scale, x, y,
                                                          alpha, beta, skip);
    return;
  }
  if (P.lanes > 1) {
    switch (P.lanes) {
      case 4: launch_csr_vec<V, T, 4, SCALED>(ctx, A, alpha, x, beta, y, skip); break;
      case 8: launch_csr_vec<V, T, 8, SCALED>(ctx, A, alpha, x, beta, y, skip); break;
      case 16: launch_csr_vec<V, T, 16, SCALED>(ctx, A, alpha, x, beta, y, skip); break;
      case 32: launch_csr_vec<V, T, 32, SCALED>(ctx, A, alpha, x, beta, y, skip); break;
      default: launch_csr_vec<V, T, 64, SCALED>(ctx, A, alpha, x, beta, y, skip); break;
    }
    return;
  }
  if (P.nblocks == 0) return;
  if (P.wpb == 4)
    launch_csr_stream<V, T, SCALED, 4>(ctx, P, alpha, x, beta, y, skip);
  else
    launch_csr_stream<V, T, SCALED, 1>(ctx, P, alpha, x, beta, y, skip);
}

template <typename V, typename T, bool ACCUM, int WPB>
void launch_coo_chunks(mxs_ctx* ctx, const CooPart& P, T alpha, const T* x, T beta, T* y,
                       const int32_t* skip, Cont c) {
  const V* val = (const V*)P.val;
  const dim3 grid((unsigned)((P.nchunks + WPB - 1) / WPB));
  T* cv = (T*)c.val;
  if (P.kernel == MXS_COO_RUNS) {
    switch (P.block_nnz) {
      case 256:
        k_coo_runs<V, T, 4, ACCUM, WPB><<<grid, 64 * WPB, 0, ctx->stream>>>(
            P.nnz, P.nchunks, P.row, P.col, val, x, y, alpha, beta, c.row, cv, skip);
        break;
      case 1024:
        k_coo_runs<V, T, 16, ACCUM, WPB><<<grid, 64 * WPB, 0, ctx->stream>>>(
            P.nnz, P.nchunks, P.row, P.col, val, x, y, alpha, beta, c.row, cv, skip);
        break;
      default:
        k_coo_runs<V, T, 8, ACCUM, WPB><<<grid, 64 * WPB, 0, ctx->stream>>>(
            P.nnz, P.nchunks, P.row, P.col, val, x, y, alpha, beta, c.row, cv, skip);
    }
    return;
  }
  if (P.block_nnz <= 512 && (double)P.nnz * (8 + sizeof(V)) > kStreamNtBytes) {
    if (P.block_nnz == 256)
      k_coo<V, T, 4, ACCUM, WPB, true><<<grid, 64 * WPB, 0, ctx->stream>>>(
          P.nnz, P.nchunks, P.row, P.col, val, x, y, alpha, beta, c.row, cv, skip);
    else
      k_coo<V, T, 8, ACCUM, WPB, true><<<grid, 64 * WPB, 0, ctx->stream>>>(
          P.nnz, P.nchunks, P.row, P.col, val, x, y, alpha, beta, c.row, cv, skip);
    return;
  }
  switch (P.block_nnz) {
    case 256:
      k_coo<V, T, 4, ACCUM, WPB><<<grid, 64 * WPB, 0, ctx->stream>>>(
          P.nnz, P.nchunks, P.row, P.col, val, x, y, alpha, beta, c.row, cv, skip);
      break;
    case 1024:
      k_coo<V, T, 16, ACCUM, WPB><<<grid, 64 * WPB, 0, ctx->stream>>>(
          P.nnz, P.nchunks, P.row, P.col, val, x, y, alpha, beta, c.row, cv, skip);
      break;
    default:
      k_coo<V, T, 8, ACCUM, WPB><<<grid, 64 * WPB, 0, ctx->stream>>>(
          P.nnz, P.nchunks, P.row, P.col, val, x, y, alpha, beta, c.row, cv, skip);
  }
}

template <typename V, typename T, bool ACCUM>
void launch_coo(mxs_ctx* ctx, const CooPart& P, int64_t n, T alpha, const T* x, T beta, T* y,
                const int32_t* skip, void* scratch) {
  if (P.panels > 1) {
    // column panels: the chunks write the panel partials (scratch after the
    // continuation partials) with alpha = 1, beta = 0, the cut rows are
    // completed there, and the last pass forms y = alpha sum + beta y
    if (P.nchunks == 0) return;
    const Cont c = cont_of(scratch, P.nchunks);
    T* part = (T*)((char*)scratch + cont_bytes(P.nchunks));
    if (P.wpb == 4)
      launch_coo_chunks<V, T, false, 4>(ctx, P, T(1), x, T(0), part, skip, c);
    else
      launch_coo_chunks<V, T, false, 1>(ctx, P, T(1), x, T(0), part, skip, c);
    if (P.nchunks > 1)
      k_coo_fix<T><<<(unsigned)((P.nchunks + 255) / 256), 256, 0, ctx->stream>>>(
          P.nchunks, c.row, (T*)c.val, part, T(1), skip, nullptr);
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, (int64_t)ctx->num_cus * 16);
    k_panel_add<T, false, false><<<g, 256, 0, ctx->stream>>>(
        n, P.panels, P.pmask, part, nullptr, y, alpha, ACCUM ? T(1) : beta, skip, nullptr,
        nullptr);
    return;
  }
  if (!ACCUM && P.nempty > 0)
    k_empty_rows<T><<<(unsigned)((P.nempty + 255) / 256), 256, 0, ctx->stream>>>(
        P.nempty, P.empty_rows, y, beta, skip);
  if (P.nchunks == 0) return;
  const Cont c = cont_of(scratch, P.nchunks);
  if (P.wpb == 4)
    launch_coo_chunks<V, T, ACCUM, 4>(ctx, P, alpha, x, beta, y, skip, c);
  else
    launch_coo_chunks<V, T, ACCUM, 1>(ctx, P, alpha, x, beta, y, skip, c);
  if (P.nchunks > 1)
    k_coo_fix<T><<<(unsigned)((P.nchunks + 255) / 256), 256, 0, ctx->stream>>>(
        P.nchunks, c.row, (T*)c.val, y, alpha, skip, nullptr);
}

template <typename V, typename T>
void launch_ell(mxs_ctx* ctx, const mxs_matrix* A, T alpha, const T* x, T beta, T* y,
                const int32_t* skip) {
  const EllPart& P = A->ell;
  if (P.stride == 0) return;
  const dim3 grid((unsigned)(P.stride / 64));
  const V* val = (const V*)P.val;
  switch (P.waves) {
#define MXS_ELL_CASE(WW)                                                                   \
  case WW:                                                                                 \
    k_ell<V, T, WW><<<grid, 64 * WW, 0, ctx->stream>>>(A->n, P.K, P.stride, P.col, val, x, y, \
                                                        alpha, beta, skip);                \
    break;
    MXS_ELL_CASE(2)
    MXS_ELL_CASE(4)
    MXS_ELL_CASE(8)
    MXS_ELL_CASE(16)
#undef MXS_ELL_CASE
    default:
      if ((double)P.K * P.stride * (4 + sizeof(V)) > kStreamNtBytes)
        k_ell<V, T, 1, true><<<grid, 64, 0, ctx->stream>>>(A->n, P.K, P.stride, P.col, val, x, y,
                                                           alpha, beta, skip);
      else
        k_ell<V, T, 1><<<grid, 64, 0, ctx->stream>>>(A->n, P.K, P.stride, P.col, val, x, y,
                                                     alpha, beta, skip);
  }
}

template <typename V, typename T, bool SCALED>
void launch_typed(mxs_ctx* ctx, const mxs_matrix* A, T alpha, const T* x, T beta, T* y,
                  const int32_t* skip, void* scratch) {
  switch (A->fmt) {
    case MXS_CSR:
      launch_csr<V, T, SCALED>(ctx, A, alpha, x, beta, y, skip, scratch);
      break;
    case MXS_COO:
      launch_coo<V, T, false>(ctx, A->coo, A->n, alpha, x, beta, y, skip, scratch);
      break;
    case MXS_ELL:
      launch_ell<V, T>(ctx, A, alpha, x, beta, y, skip);
      break;
    case MXS_HYB:
      if (A->ell.K == 0) {
        launch_coo<V, T, false>(ctx, A->coo, A->n, alpha, x, beta, y, skip, scratch);
      } else {
        launch_ell<V, T>(ctx, A, alpha, x, beta, y, skip);
        launch_coo<V, T, true>(ctx, A->coo, A->n, alpha, x, beta, y, skip, scratch);
      }
      break;
  }
}

}  // namespace

size_t spmv_scratch_bytes(const mxs_matrix* A) {
  int64_t chunks = 0;
  if (A->fmt == MXS_CSR && A->csr.merge) chunks = A->csr.nchunks;
  if (A->fmt == MXS_COO || A->fmt == MXS_HYB) chunks = A->coo.nchunks;
  if (chunks == 0) return 0;
  size_t b = cont_bytes(chunks);
  // column panels: one partial of up to 8 bytes per row and panel
  if (A->fmt == MXS_CSR && A->csr.merge && A->csr.panels > 1)
    b += (size_t)A->csr.panels * (size_t)A->n * sizeof(double);
  if ((A->fmt == MXS_COO || A->fmt == MXS_HYB) && A->coo.panels > 1)
    b += (size_t)A->coo.panels * (size_t)A->n * sizeof(double);
  return b;
}

mxs_status launch_spmv_scratch(mxs_ctx* ctx, const mxs_matrix* A, const void* alpha,
                               const void* x, const void* beta, void* y, const int32_t* skip,
                               void* scratch) {
  if (A->n == 0) return MXS_OK;
  if (A->dt == MXS_F64) {
    launch_typed<double, double, false>(ctx, A, *(const double*)alpha, (const double*)x,
                                        *(const double*)beta, (double*)y, skip, scratch);
  } else if (A->dt == MXS_F32) {
    launch_typed<float, float, false>(ctx, A, *(const float*)alpha, (const float*)x,
                                      *(const float*)beta, (float*)y, skip, scratch);
  } else if (A->dt == MXS_C128) {
    using Z = cplx<double>;
    if (A->fmt != MXS_CSR) return fail(ctx, MXS_UNSUPPORTED, "complex values are CSR only");
    launch_csr<Z, Z, false>(ctx, A, *(const Z*)alpha, (const Z*)x, *(const Z*)beta, (Z*)y, skip,
                            scratch);
  } else if (A->dt == MXS_C64) {
    using Z = cplx<float>;
    if (A->fmt != MXS_CSR) return fail(ctx, MXS_UNSUPPORTED, "complex values are CSR only");
    launch_csr<Z, Z, false>(ctx, A, *(const Z*)alpha, (const Z*)x, *(const Z*)beta, (Z*)y, skip,
                            scratch);
  } else {
    launch_typed<_Float16, float, true>(ctx, A, *(const float*)alpha, (const float*)x,
                                        *(const float*)beta, (float*)y, skip, scratch);
  }
  MXS_HIP_TRY(ctx, hipGetLastError());
  return MXS_OK;
}

// ---------------------------------------------------------------------------
// scratch of the allocation-free product: a fixed array in each GPU's copy of
// the code object.  Host code never passes the array's name to a kernel: the
// name is only a host-side stand-in, so the device address of each GPU's
// copy is looked up once (with that GPU current) and kept per device.
// ---------------------------------------------------------------------------
namespace {
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

mxs_status noalloc_scratch_init(mxs_ctx* ctx) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return fail(ctx, MXS_UNSUPPORTED, "device %d beyond the scratch table", ctx->device);
  if (g_scratch_ptr[ctx->device]) return MXS_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(ctx, MXS_HIP, "looking up the product scratch on device %d: %s", ctx->device,
                hipGetErrorString(e));
  }
  g_scratch_ptr[ctx->device] = p;
  return MXS_OK;
}

void* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

// y = A x together with work-group partial sums of x[i] * y[i] (CG's p.q),
// for the kernels that write each row's result once from one lane: the
// rows-from-LDS CSR kernel and the column-panel merge path (whose last pass
// forms the rows).  Returns the number of partials written to dpart (at most
// kDotPartials), or 0 when A's kernel has no such form (nothing enqueued).
template <typename V, typename T, bool SCALED>
int launch_dot_typed(mxs_ctx* ctx, const mxs_matrix* A, const T* x, T* y, const int32_t* skip,
                     double* dpart, void* scratch, const T* w, int nv) {
  const CsrPart& P = A->csr;
  if (P.rows_lds && P.nblocks > 0) {
    const T* wd = w ? w : x;
    if (P.block_nnz <= 512)
      return launch_csr_rl_dot<V, T, SCALED, 512>(ctx, P, x, y, skip, dpart, wd, nv);
    if (P.block_nnz <= 1024)
      return launch_csr_rl_dot<V, T, SCALED, 1024>(ctx, P, x, y, skip, dpart, wd, nv);
    return launch_csr_rl_dot<V, T, SCALED, 2048>(ctx, P, x, y, skip, dpart, wd, nv);
  }
  // the merge path forms x.y only
  if ((w && w != x) || nv != 1) return 0;
  if (P.merge && P.nchunks > 0 && (P.panels > 1 || (P.nchunks + 255) / 256 <= kDotPartials)) {
    if constexpr (std::is_same_v<V, double> || std::is_same_v<V, float> ||
                  std::is_same_v<V, _Float16>) {
      int nd = 0;
      launch_csr_merge<V, T, SCALED>(ctx, A, T(1), x, T(0), y, skip, scratch, dpart, &nd);
      return nd;
    }
  }
  return 0;
}

int launch_spmv_dot(mxs_ctx* ctx, const mxs_matrix* A, const void* x, void* y,
                    const int32_t* skip, double* dpart, const void* w, int nv) {
  if (A->fmt != MXS_CSR || A->n == 0 || A->n != A->ncols || nv < 1 || nv > 2) return 0;
  const CsrPart& P = A->csr;
  if (!(P.rows_lds && P.nblocks > 0) && !(P.merge && P.nchunks > 0)) return 0;
  if (!(P.rows_lds && P.nblocks > 0) && ((w && w != x) || nv != 1)) return 0;
  // the merge path without panels also keeps one dot partial per chunk
  const size_t need = spmv_scratch_bytes(A) +
                      (P.merge && P.panels <= 1 ? (size_t)P.nchunks * sizeof(double) : 0);
  if (need > ctx->spmv_ws.bytes) {
    if (ctx->spmv_ws.ptr) {
      if (hipStreamSynchronize(ctx->stream) != hipSuccess) return 0;
      ctx->alloc.release(ctx->spmv_ws.ptr);
    }
    const size_t want = need + need / 4;
    ctx->spmv_ws.ptr = ctx->alloc.alloc(want);
    ctx->spmv_ws.bytes = ctx->spmv_ws.ptr ? want : 0;
    if (!ctx->spmv_ws.ptr) return 0;
  }
  void* sc = ctx->spmv_ws.ptr;
  int g = 0;
  if (A->dt == MXS_F64)
    g = launch_dot_typed<double, double, false>(ctx, A, (const double*)x, (double*)y, skip, dpart,
                                                sc, (const double*)w, nv);
  else if (A->dt == MXS_F32)
    g = launch_dot_typed<float, float, false>(ctx, A, (const float*)x, (float*)y, skip, dpart, sc,
                                              (const float*)w, nv);
  else if (A->dt == MXS_F16_ROWSCALED)
    g = launch_dot_typed<_Float16, float, true>(ctx, A, (const float*)x, (float*)y, skip, dpart,
                                                sc, (const float*)w, nv);
  return g;
}

// The context's own scratch, grown (after the stream has drained) when a
// product needs more than it holds.
mxs_status launch_spmv(mxs_ctx* ctx, const mxs_matrix* A, const void* alpha, const void* x,
                       const void* beta, void* y, const int32_t* skip) {
  const size_t need = spmv_scratch_bytes(A);
  if (need > ctx->spmv_ws.bytes) {
    if (ctx->spmv_ws.ptr) {
      MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      ctx->alloc.release(ctx->spmv_ws.ptr);
    }
    const size_t want = need + need / 4;
    ctx->spmv_ws.ptr = ctx->alloc.alloc(want);
    ctx->spmv_ws.bytes = ctx->spmv_ws.ptr ? want : 0;
    if (!ctx->spmv_ws.ptr) return fail(ctx, MXS_OOM, "product scratch (%zu bytes)", want);
  }
  return launch_spmv_scratch(ctx, A, alpha, x, beta, y, skip, ctx->spmv_ws.ptr);
}

}  // namespace mxs

extern "C" mxs_status mxs_spmv(mxs_ctx* ctx, const void* alpha, const mxs_matrix* A,
                               const void* x, const void* beta, void* y) {
  if (!ctx || !A || !alpha || !beta) return MXS_INVALID_ARG;
  if (A->n > 0 && !y) return mxs::fail(ctx, MXS_INVALID_ARG, "y is NULL");
  if (A->nnz > 0 && !x) return mxs::fail(ctx, MXS_INVALID_ARG, "x is NULL");
  return mxs::launch_spmv(ctx, A, alpha, x, beta, y, nullptr);
}

extern "C" mxs_status mxs_spmv_noalloc(mxs_ctx* ctx, const void* alpha, const mxs_matrix* A,
                                       const void* x, const void* beta, void* y) {
  if (!ctx || !A || !alpha || !beta) return MXS_INVALID_ARG;
  if (A->n > 0 && !y) return mxs::fail(ctx, MXS_INVALID_ARG, "y is NULL");
  if (A->nnz > 0 && !x) return mxs::fail(ctx, MXS_INVALID_ARG, "x is NULL");
  if (A->device != ctx->device)
    return mxs::fail(ctx, MXS_INVALID_ARG, "matrix on device %d, ctx on device %d", A->device,
                     ctx->device);
  const size_t need = mxs::spmv_scratch_bytes(A);
  if (need > mxs::kNoAllocScratchBytes)
    return mxs::fail(ctx, MXS_UNSUPPORTED,
                     "this product needs %zu bytes of scratch; the allocation-free product "
                     "holds %zu",
                     need, mxs::kNoAllocScratchBytes);
  void* p = mxs::noalloc_scratch(ctx->device);
  if (!p) return mxs::fail(ctx, MXS_HIP, "product scratch of device %d not set up", ctx->device);
  return mxs::launch_spmv_scratch(ctx, A, alpha, x, beta, y, nullptr, p);
}
