// solvers.hip -- fused BLAS-1 reduction kernels and the Krylov solver
// drivers (CG, preconditioned CG, pipelined CG, BiCGSTAB, CGS, restarted
// GMRES), mixed-precision iterative refinement and PageRank, all on the GPU.
//
// The paper names CG, BiCGSTAB, CGS and GMRES as the solvers built on SpMV,
// and PageRank's power iteration beside them (its section "Central Sparse
// Linear Algebra Functionality"; textbook forms in Saad 2003 and Saad &
// Schultz 1986), and runs the solvers in its "Krylov Solver Performance
// Analysis" subsection.  Design for one MI355X:
//  * every scalar of the recurrences (rho, alpha, beta, omega, the Hessenberg
//    column, Givens rotations) lives in device memory: a reduction kernel's
//    blocks write partial sums and the next kernel's blocks (or a one-block
//    finishing kernel) add them in block order, so an iteration never waits
//    for the host and needs no device-scope fence;
//  * a device status word stops all queued work once the solver converged
//    or broke down: the host enqueues `check_every` iterations, then reads
//    the status once (pinned memory);
//  * reductions accumulate in FP64 (also for the FP32 inner solver of
//    iterative refinement) with a fixed order: per-thread grid-stride sums,
//    wave butterflies, wave partials in order, block partials in order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "common.h"

namespace mxs {
namespace {

constexpr int RB = 512;      // threads per reduction block
constexpr int MAXG = 512;    // reduction grid cap (partials per reduction)
constexpr int MAXM = 32;     // largest GMRES restart length

enum : int32_t {
  RUN = 0,
  ST_CONVERGED = 1,
  ST_BREAKDOWN = 2,
  ST_NONFINITE = 3,
  ST_HALF = 4,   // BiCGSTAB: ||s|| met the tolerance, x += alpha p pending
  ST_MAXIT = 5
};

// Device-resident solver state.  Within one kernel no field is written that
// another block of the same launch reads, except the terminal status `done`
// (every block reaches the same decision from the same partials, so an
// early or late read of it is equivalent).  Scalars that change every
// iteration and are read by the kernel that replaces them are kept in two
// slots indexed by the iteration's parity.
struct KState {
  double rho[2];    // CG: r.r ; BiCGSTAB: r_hat.r (both by iteration parity)
  double alpha, omega, thr, res2, dot[2], restart_rhr;
  int64_t iters, max_iters;
  int32_t done;     // one of the ST_* values; every kernel returns at once if set
  int32_t cycle;    // GMRES: 1 once the current cycle must end
  int32_t k;        // GMRES: Arnoldi steps taken in the current cycle
  int32_t m;        // GMRES restart length
  double est;       // GMRES residual estimate |g_{k}|
  double H[(MAXM + 1) * MAXM];  // column-major, leading dimension MAXM+1
  double cs[MAXM], sn[MAXM], g[MAXM + 1], y[MAXM], h2[MAXM + 1];
  // pipelined CG: gamma and alpha by iteration parity, and the iteration
  // that starts a recurrence (beta = 0, gamma and delta from dot[])
  double pg[2], palpha[2];
  int64_t restart_at;
  // CG: 0, or the iteration the x update stops at plus one (the update of
  // iteration k runs while k < halt - 1); set with the terminal status by
  // the kernel that decides it, so that the other blocks of that same
  // launch, which may already see `done`, still finish their x update
  int64_t halt;
};

int red_grid(int64_t n) {
  int64_t g = (n + RB * 4 - 1) / (RB * 4);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, MAXG));
}

// Sums NV per-thread values over the block with one barrier: every wave
// reduces its values with butterflies, lane 0 stores them to LDS, and thread
// v adds value v over the waves in wave order.  Result valid in thread v.
template <int NV>
__device__ __forceinline__ double block_sum_multi(const double (&acc)[NV], double (*lds)[NV]) {
  const int w = threadIdx.x / 64, lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double s = wave_total(acc[i]);
    if (lane == 0) lds[w][i] = s;
  }
  __syncthreads();
  double s = 0.0;
  if ((int)threadIdx.x < NV) {
    s = lds[0][threadIdx.x];
#pragma unroll
    for (int q = 1; q < RB / 64; ++q) s += lds[q][threadIdx.x];
  }
  return s;
}

// Block partial sums of NV values to part[blockIdx.x * NV + v] (plain
// stores: the consumer is a later kernel).
template <int NV>
__device__ __forceinline__ void block_partials(const double (&acc)[NV], double* __restrict__ part) {
  __shared__ double lds[RB / 64][NV];
  const double s = block_sum_multi<NV>(acc, lds);
  if ((int)threadIdx.x < NV) part[(int64_t)blockIdx.x * NV + threadIdx.x] = s;
}

// Adds the `g` block partials of NV values written by an earlier kernel, in
// block order; every thread of every calling block gets the same totals.
template <int NV>
__device__ __forceinline__ void finish(const double* __restrict__ part, int g, double (&out)[NV]) {
  __shared__ double lds[RB / 64][NV];
  __shared__ double res[NV];
  // g <= MAXG == RB: thread b holds block b's partials; all NV loads are
  // issued before any is used
  static_assert(MAXG <= RB, "one partial row per thread");
  double acc[NV];
  const bool has = (int)threadIdx.x < g;
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = has ? part[(int64_t)threadIdx.x * NV + v] : 0.0;
  const double s = block_sum_multi<NV>(acc, lds);
  if ((int)threadIdx.x < NV) res[threadIdx.x] = s;
  __syncthreads();
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v] = res[v];
}

// The same for up to 8 * RB partials (the product-with-dot kernels write one
// per work-group): thread t adds partials t, t + RB, ... in that order.
template <int NV>
__device__ __forceinline__ void finish_wide(const double* __restrict__ part, int g,
                                            double (&out)[NV]) {
  __shared__ double lds[RB / 64][NV];
  __shared__ double res[NV];
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double t[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int b = (int)threadIdx.x + j * RB;
      t[j] = b < g ? part[(int64_t)b * NV + v] : 0.0;
    }
    double a = t[0];
#pragma unroll
    for (int j = 1; j < 8; ++j) a += t[j];
    acc[v] = a;
  }
  const double s = block_sum_multi<NV>(acc, lds);
  if ((int)threadIdx.x < NV) res[threadIdx.x] = s;
  __syncthreads();
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v] = res[v];
}

// Wave sums of NV (a power of two <= 32) per-lane values by a transposing
// butterfly: at each of the first log2(NV) steps a lane keeps half of its
// values and adds its partner's copy of them (NV-1 exchanges in all instead
// of 6 NV), then plain butterflies finish.  Lane l ends with the sum of
// value (l >> (6 - log2 NV)) over the wave; the order is fixed, so the
// result is deterministic.
template <int H, int O, int NV>
__device__ __forceinline__ void transposed_steps(double (&a)[NV], int lane) {
  if constexpr (H > 1) {
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int q = 0; q < H / 2; ++q) {
      const double keep = up ? a[q + H / 2] : a[q];
      const double send = up ? a[q] : a[q + H / 2];
      a[q] = keep + __shfl_xor(send, O, 64);
    }
    transposed_steps<H / 2, O / 2, NV>(a, lane);
  } else {
#pragma unroll
    for (int o = O; o > 0; o >>= 1) a[0] += __shfl_xor(a[0], o, 64);
  }
}

template <int NV>
__device__ __forceinline__ double wave_sum_transposed(double (&a)[NV]) {
  transposed_steps<NV, 32, NV>(a, threadIdx.x & 63);
  return a[0];
}

// Block partial sums of NV values (a power of two <= 32) to
// part[blockIdx.x * MAXM + v]: transposed wave sums, then thread v adds
// value v over the waves in wave order.
template <int NV>
__device__ __forceinline__ void block_partials_m(double (&acc)[NV], double* __restrict__ part) {
  static_assert(NV <= 32 && (NV & (NV - 1)) == 0, "power of two up to 32");
  __shared__ double lds[RB / 64][NV];
  constexpr int SH = NV == 1 ? 6 : NV == 2 ? 5 : NV == 4 ? 4 : NV == 8 ? 3 : NV == 16 ? 2 : 1;
  const double s = wave_sum_transposed<NV>(acc);
  const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
  if ((lane & ((1 << SH) - 1)) == 0) lds[w][lane >> SH] = s;
  __syncthreads();
  if ((int)threadIdx.x < NV) {
    double t = lds[0][threadIdx.x];
#pragma unroll
    for (int q = 1; q < RB / 64; ++q) t += lds[q][threadIdx.x];
    part[(int64_t)blockIdx.x * MAXM + threadIdx.x] = t;
  }
}

// Totals of the first `nv` values of g block partials laid out as
// part[b * MAXM + v] (b < g <= RB), for the one-block finishing kernel.
// Loads are coalesced: thread t reads entries t, t + RB, t + 2 RB, ... of the
// flat array, all of value t % MAXM (RB is a multiple of MAXM), and adds
// them in block order; the RB / MAXM threads of one value are then added in
// thread order.  Thread v < nv gets total v in `out`.
__device__ __forceinline__ double finish_m(const double* __restrict__ part, int g) {
  static_assert(RB % MAXM == 0 && MAXM == 32, "flat layout");
  __shared__ double lds[RB / 64][MAXM];
  const int t = threadIdx.x, total = g * MAXM;
  double v[MAXM];
#pragma unroll
  for (int k = 0; k < MAXM; ++k) v[k] = t + k * RB < total ? part[t + k * RB] : 0.0;
  double a = 0.0;
#pragma unroll
  for (int k = 0; k < MAXM; ++k) a += v[k];
  // lanes l and l + 32 of a wave hold the same value
  a += __shfl_xor(a, 32, 64);
  const int lane = t & 63, w = t / 64;
  if (lane < MAXM) lds[w][lane] = a;
  __syncthreads();
  double out = 0.0;
  if (t < MAXM) {
    out = lds[0][t];
#pragma unroll
    for (int q = 1; q < RB / 64; ++q) out += lds[q][t];
  }
  return out;
}

__device__ __forceinline__ bool lead() { return blockIdx.x == 0 && threadIdx.x == 0; }

#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < (n); i += (int64_t)gridDim.x * RB)

// The values one element of a vector kernel reads.
template <typename T, int N>
struct Pack {
  T v[N];
};

// Visits the thread's grid-stride elements i = first, first + S, ... < n
// (S = gridDim.x * RB) four per round: load(i) returns the Pack element i
// reads, use(i, pack) does its arithmetic and stores.  A round issues the
// loads of all four elements before the first use, so the memory system sees
// four independent loads per vector instead of one; the uses run in index
// order, so a sum over the thread's elements adds in the same order as a
// plain grid-stride loop.
template <typename Load, typename Use>
__device__ __forceinline__ void strided4(int64_t n, Load load, Use use) {
  const int64_t S = (int64_t)gridDim.x * RB;
  int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
  for (; i + 3 * S < n; i += 4 * S) {
    const auto e0 = load(i);
    const auto e1 = load(i + S);
    const auto e2 = load(i + 2 * S);
    const auto e3 = load(i + 3 * S);
    use(i, e0);
    use(i + S, e1);
    use(i + 2 * S, e2);
    use(i + 3 * S, e3);
  }
  for (; i < n; i += S) use(i, load(i));
}

// strided4 whose first round of loads is issued before `pre` runs (a
// kernel's finishing of the previous kernel's partials, whose result the
// uses need): the reduction's latency overlaps the first loads.
template <typename Load, typename Pre, typename Use>
__device__ __forceinline__ void strided4_pre(int64_t n, Load load, Pre pre, Use use) {
  const int64_t S = (int64_t)gridDim.x * RB;
  int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
  using E = decltype(load(i));
  E e[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (i + j * S < n) e[j] = load(i + j * S);
  pre();
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (i + j * S < n) use(i + j * S, e[j]);
  i += 4 * S;
  for (; i + 3 * S < n; i += 4 * S) {
    const auto e0 = load(i);
    const auto e1 = load(i + S);
    const auto e2 = load(i + 2 * S);
    const auto e3 = load(i + 3 * S);
    use(i, e0);
    use(i + S, e1);
    use(i + 2 * S, e2);
    use(i + 3 * S, e3);
  }
  for (; i < n; i += S) use(i, load(i));
}

// ---------------------------------------------------------------------------
// generic reductions
// ---------------------------------------------------------------------------
// partials of a.b and c.d (c may be NULL)
template <typename T>
__global__ __launch_bounds__(RB) void k_dots(int64_t n, const T* __restrict__ a,
                                             const T* __restrict__ b, const T* __restrict__ c,
                                             const T* __restrict__ d, double* part) {
  double acc[2] = {0.0, 0.0};
  if (c)
    strided4(
        n, [&](int64_t i) { return Pack<T, 4>{{a[i], b[i], c[i], d[i]}}; },
        [&](int64_t, const Pack<T, 4>& e) {
          acc[0] += (double)e.v[0] * (double)e.v[1];
          acc[1] += (double)e.v[2] * (double)e.v[3];
        });
  else
    strided4(
        n, [&](int64_t i) { return Pack<T, 2>{{a[i], b[i]}}; },
        [&](int64_t, const Pack<T, 2>& e) { acc[0] += (double)e.v[0] * (double)e.v[1]; });
  block_partials<2>(acc, part);
}

__global__ __launch_bounds__(RB) void k_dots_fin(const double* part, int g, KState* st) {
  double out[2];
  finish<2>(part, g, out);
  if (threadIdx.x == 0) {
    st->dot[0] = out[0];
    st->dot[1] = out[1];
  }
}

// ---------------------------------------------------------------------------
// CG (Hestenes-Stiefel)
// ---------------------------------------------------------------------------
// partials of p.q, for products that do not form them themselves
template <typename T>
__global__ __launch_bounds__(RB) void k_cg_pq(int64_t n, const T* __restrict__ p,
                                              const T* __restrict__ q, double* __restrict__ pa,
                                              const KState* st) {
  if (st->done) return;
  double acc[1] = {0.0};
  strided4(
      n, [&](int64_t i) { return Pack<T, 2>{{p[i], q[i]}}; },
      [&](int64_t, const Pack<T, 2>& e) { acc[0] += (double)e.v[0] * (double)e.v[1]; });
  block_partials<1>(acc, pa);
}

// CG in three launches, B_csr + 64n bytes per iteration in FP64.  Iteration k
// (parity par):
//   q = A p with the product's own partials of p.q (launch_spmv_dot), or the
//   product and k_cg_pq when A's kernel has no such form;
//   k_cg_r: alpha = rho[par] / (p.q), r -= alpha q, partials of r.r (reads
//   r, q; writes r);
//   k_cg_xp: rho' = r.r, stopping test, x += alpha p, beta = rho'/rho[par],
//   p = r + beta p (reads x, r, p; writes x, p).
// The x update rides with the direction update, so it must run in every
// block even when the same launch decides that CG has converged: its blocks
// skip by `halt`, not by `done` (see KState).
template <typename T>
__global__ __launch_bounds__(RB) void k_cg_r(int64_t n, T* __restrict__ r,
                                             const T* __restrict__ q,
                                             const double* __restrict__ pa, int ga,
                                             double* __restrict__ pb, KState* st, int par,
                                             int64_t k) {
  if (st->done) return;
  double pq[1];
  bool broke = false;
  T a = 0;
  double acc[1] = {0.0};
  strided4_pre(
      n, [&](int64_t i) { return Pack<T, 2>{{r[i], q[i]}}; },
      [&]() {
        finish_wide<1>(pa, ga, pq);
        broke = !isfinite(pq[0]) || pq[0] <= 0.0;
        if (broke) {
          if (lead()) {
            st->done = isfinite(pq[0]) ? ST_BREAKDOWN : ST_NONFINITE;
            st->halt = k + 1;
          }
          return;
        }
        const double alpha = st->rho[par] / pq[0];
        if (lead()) st->alpha = alpha;
        a = (T)alpha;
      },
      [&](int64_t i, const Pack<T, 2>& e) {
        if (broke) return;
        const T ri = e.v[0] - a * e.v[1];
        r[i] = ri;
        acc[0] += (double)ri * (double)ri;
      });
  if (broke) return;
  block_partials<1>(acc, pb);
}

template <typename T>
__global__ __launch_bounds__(RB) void k_cg_xp(int64_t n, T* __restrict__ x,
                                              const T* __restrict__ r, T* __restrict__ p,
                                              const double* __restrict__ pb, int g, KState* st,
                                              int par, int64_t k) {
  const int64_t halt = st->halt;
  if (halt != 0 && k >= halt - 1) return;
  double rr[1];
  finish<1>(pb, g, rr);
  const double rn = rr[0];
  const bool bad = !isfinite(rn);
  const bool conv = !bad && sqrt(rn) <= st->thr;
  const bool maxit = k + 1 >= st->max_iters;
  const bool stop = bad || conv || maxit;
  if (lead()) {
    st->iters = k + 1;
    st->res2 = rn;
    st->rho[1 - par] = rn;
    if (bad)
      st->done = ST_NONFINITE;
    else if (conv)
      st->done = ST_CONVERGED;
    else if (maxit)
      st->done = ST_MAXIT;
    if (stop) st->halt = k + 2;
  }
  const T a = (T)st->alpha;
  if (stop) {
    strided4(
        n, [&](int64_t i) { return Pack<T, 2>{{x[i], p[i]}}; },
        [&](int64_t i, const Pack<T, 2>& e) { x[i] = e.v[0] + a * e.v[1]; });
    return;
  }
  const T beta = (T)(rn / st->rho[par]);
  strided4(
      n, [&](int64_t i) { return Pack<T, 3>{{x[i], r[i], p[i]}}; },
      [&](int64_t i, const Pack<T, 3>& e) {
        x[i] = e.v[0] + a * e.v[2];
        p[i] = e.v[1] + beta * e.v[2];
      });
}

// ---------------------------------------------------------------------------
// BiCGSTAB (r_hat = r0).  Iteration k (par = k & 1), rho[par] = previous
// r_hat.r, rho[1-par] = current one:
//   k_bi_p: (from the last update's partials) stopping test on ||r||,
//           beta = (rho'/rho)(alpha/omega), p = r + beta (p - omega v)
//   v = A p;  k_bi_rv: partials of r_hat.v
//   k_bi_s: alpha = rho' / (r_hat.v), s = r - alpha v, partials of s.s
//   t = A s;  k_bi_omega: ||s|| test (half step), partials of t.s, t.t
//   k_bi_update: omega, x += alpha p + omega s, r = s - omega t,
//                partials of r.r and r_hat.r
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RB) void k_bi_p(int64_t n, const double* __restrict__ r,
                                             double* __restrict__ p,
                                             const double* __restrict__ v,
                                             const double* __restrict__ pc, int g, KState* st,
                                             int par, int64_t k, int first) {
  if (st->done) return;
  double rr_rhr[2];
  if (first) {
    rr_rhr[0] = st->res2;
    rr_rhr[1] = st->restart_rhr;
  } else {
    finish<2>(pc, g, rr_rhr);
  }
  const double rn = rr_rhr[0], rhr = rr_rhr[1];
  const double w = st->omega, a = st->alpha;
  int32_t verdict = RUN;
  if (!isfinite(rn) || !isfinite(rhr))
    verdict = ST_NONFINITE;
  else if (sqrt(rn) <= st->thr)
    verdict = ST_CONVERGED;
  else if (k >= st->max_iters)
    verdict = ST_MAXIT;
  else if (rhr == 0.0 || w == 0.0)
    verdict = ST_BREAKDOWN;
  if (lead()) {
    st->res2 = rn;
    st->rho[1 - par] = rhr;
    if (verdict != RUN) st->done = verdict;
  }
  if (verdict != RUN) return;
  const double beta = (rhr / st->rho[par]) * (a / w);
  strided4(
      n, [&](int64_t i) { return Pack<double, 3>{{r[i], p[i], v[i]}}; },
      [&](int64_t i, const Pack<double, 3>& e) { p[i] = e.v[0] + beta * (e.v[1] - w * e.v[2]); });
}

__global__ __launch_bounds__(RB) void k_bi_rv(int64_t n, const double* __restrict__ rh,
                                              const double* __restrict__ v,
                                              double* __restrict__ pa, const KState* st) {
  if (st->done) return;
  double acc[1] = {0.0};
  strided4(
      n, [&](int64_t i) { return Pack<double, 2>{{rh[i], v[i]}}; },
      [&](int64_t, const Pack<double, 2>& e) { acc[0] += e.v[0] * e.v[1]; });
  block_partials<1>(acc, pa);
}

__global__ __launch_bounds__(RB) void k_bi_s(int64_t n, const double* __restrict__ r,
                                             const double* __restrict__ v,
                                             double* __restrict__ s,
                                             const double* __restrict__ pa, int g,
                                             double* __restrict__ pb, KState* st, int par) {
  if (st->done) return;
  double rv[1];
  finish_wide<1>(pa, g, rv);  // the product's partials when it formed r_hat.v
  if (!isfinite(rv[0]) || rv[0] == 0.0) {
    if (lead()) st->done = isfinite(rv[0]) ? ST_BREAKDOWN : ST_NONFINITE;
    return;
  }
  const double a = st->rho[1 - par] / rv[0];
  if (lead()) st->alpha = a;
  double acc[1] = {0.0};
  strided4(
      n, [&](int64_t i) { return Pack<double, 2>{{r[i], v[i]}}; },
      [&](int64_t i, const Pack<double, 2>& e) {
        const double si = e.v[0] - a * e.v[1];
        s[i] = si;
        acc[0] += si * si;
      });
  block_partials<1>(acc, pb);
}

__global__ __launch_bounds__(RB) void k_bi_omega(int64_t n, const double* __restrict__ t,
                                                 const double* __restrict__ s,
                                                 const double* __restrict__ pb, int g,
                                                 double* __restrict__ pd, KState* st, int64_t k) {
  if (st->done) return;
  double ss[1];
  finish<1>(pb, g, ss);
  if (!isfinite(ss[0])) {
    if (lead()) st->done = ST_NONFINITE;
    return;
  }
  if (sqrt(ss[0]) <= st->thr) {
    if (lead()) {
      st->res2 = ss[0];
      st->iters = k + 1;
      st->done = ST_HALF;
    }
    return;
  }
  double acc[2] = {0.0, 0.0};
  strided4(
      n, [&](int64_t i) { return Pack<double, 2>{{t[i], s[i]}}; },
      [&](int64_t, const Pack<double, 2>& e) {
        acc[0] += e.v[0] * e.v[1];
        acc[1] += e.v[0] * e.v[0];
      });
  block_partials<2>(acc, pd);
}

// pd holds the partials of (t.s, t.t): k_bi_omega's, or (half != 0) those
// the product t = A s formed itself, when this kernel first takes the
// half-step test on s.s (pb, gb partials) that k_bi_omega would have taken.
__global__ __launch_bounds__(RB) void k_bi_update(int64_t n, double* __restrict__ x,
                                                  const double* __restrict__ p,
                                                  const double* __restrict__ s,
                                                  const double* __restrict__ t,
                                                  double* __restrict__ r,
                                                  const double* __restrict__ rh,
                                                  const double* __restrict__ pd, int g,
                                                  double* __restrict__ pc, KState* st,
                                                  int64_t k, int half,
                                                  const double* __restrict__ pb, int gb) {
  if (st->done) return;
  if (half) {
    double ss[1];
    finish<1>(pb, gb, ss);
    if (!isfinite(ss[0])) {
      if (lead()) st->done = ST_NONFINITE;
      return;
    }
    if (sqrt(ss[0]) <= st->thr) {
      if (lead()) {
        st->res2 = ss[0];
        st->iters = k + 1;
        st->done = ST_HALF;
      }
      return;
    }
  }
  double tstt[2];
  finish_wide<2>(pd, g, tstt);
  if (!isfinite(tstt[0]) || !isfinite(tstt[1]) || tstt[1] == 0.0) {
    if (lead()) st->done = tstt[1] == 0.0 ? ST_BREAKDOWN : ST_NONFINITE;
    return;
  }
  const double w = tstt[0] / tstt[1];
  const double a = st->alpha;
  if (lead()) {
    st->omega = w;
    st->iters = k + 1;
  }
  double acc[2] = {0.0, 0.0};
  strided4(
      n, [&](int64_t i) { return Pack<double, 5>{{x[i], p[i], s[i], t[i], rh[i]}}; },
      [&](int64_t i, const Pack<double, 5>& e) {
        x[i] = e.v[0] + a * e.v[1] + w * e.v[2];
        const double ri = e.v[2] - w * e.v[3];
        r[i] = ri;
        acc[0] += ri * ri;
        acc[1] += e.v[4] * ri;
      });
  block_partials<2>(acc, pc);
}

// the half step x += alpha p, launched once by the host after it read
// ST_HALF (every queued kernel of later iterations returned early, so p and
// alpha are those of the converging iteration)
__global__ __launch_bounds__(RB) void k_bi_half(int64_t n, double* __restrict__ x,
                                                const double* __restrict__ p,
                                                const KState* st) {
  const double a = st->alpha;
  strided4(
      n, [&](int64_t i) { return Pack<double, 2>{{x[i], p[i]}}; },
      [&](int64_t i, const Pack<double, 2>& e) { x[i] = e.v[0] + a * e.v[1]; });
}

// ---------------------------------------------------------------------------
// GMRES(m): classical Gram-Schmidt with one reorthogonalisation pass.  The
// multi-dot partials of (j+1) values per block are finished by a one-block
// kernel that also owns the small dense work (Hessenberg column, Givens).
// ---------------------------------------------------------------------------
// The three passes over the basis are instantiated for JB = 8, 16 and 32
// vectors (the smallest that holds v_0..v_j), so that short bases do not pay
// registers, and occupancy, for 32.
// partials of V(:,0..j)^T w
template <int JB>
__global__ __launch_bounds__(RB) void k_gm_dots(int64_t n, int64_t ldv, int j,
                                                const double* __restrict__ V,
                                                const double* __restrict__ w,
                                                double* __restrict__ part, const KState* st) {
  if (st->done || st->cycle) return;
  double acc[JB];
#pragma unroll
  for (int i = 0; i < JB; ++i) acc[i] = 0.0;
  GRID_STRIDE(r, n) {
    const double wr = w[r];
    double vr[JB];
#pragma unroll
    for (int i = 0; i < JB; ++i) vr[i] = i <= j ? V[i * ldv + r] : 0.0;
#pragma unroll
    for (int i = 0; i < JB; ++i) acc[i] += vr[i] * wr;
  }
  block_partials_m<JB>(acc, part);
}

// w -= V h (first-pass coefficients); partials of V^T w on the updated rows
template <int JB>
__global__ __launch_bounds__(RB) void k_gm_orth(int64_t n, int64_t ldv, int j,
                                                const double* __restrict__ V,
                                                double* __restrict__ w,
                                                double* __restrict__ part, const KState* st) {
  if (st->done || st->cycle) return;
  __shared__ double h[JB];
  if (threadIdx.x < JB)
    h[threadIdx.x] = (int)threadIdx.x <= j ? st->H[j * (MAXM + 1) + threadIdx.x] : 0.0;
  __syncthreads();
  double acc[JB];
#pragma unroll
  for (int i = 0; i < JB; ++i) acc[i] = 0.0;
  GRID_STRIDE(r, n) {
    double vr[JB];
    double wr = w[r];
#pragma unroll
    for (int i = 0; i < JB; ++i) {
      vr[i] = i <= j ? V[i * ldv + r] : 0.0;
      wr -= h[i] * vr[i];
    }
    w[r] = wr;
#pragma unroll
    for (int i = 0; i < JB; ++i) acc[i] += vr[i] * wr;
  }
  block_partials_m<JB>(acc, part);
}

// w -= V h2; partials of w.w
template <int JB>
__global__ __launch_bounds__(RB) void k_gm_norm(int64_t n, int64_t ldv, int j,
                                                const double* __restrict__ V,
                                                double* __restrict__ w,
                                                double* __restrict__ part, const KState* st) {
  if (st->done || st->cycle) return;
  __shared__ double h[JB];
  if (threadIdx.x < JB) h[threadIdx.x] = (int)threadIdx.x <= j ? st->h2[threadIdx.x] : 0.0;
  __syncthreads();
  double acc[1] = {0.0};
  GRID_STRIDE(r, n) {
    double vr[JB];
#pragma unroll
    for (int i = 0; i < JB; ++i) vr[i] = i <= j ? V[i * ldv + r] : 0.0;
    double wr = w[r];
#pragma unroll
    for (int i = 0; i < JB; ++i) wr -= h[i] * vr[i];
    w[r] = wr;
    acc[0] += wr * wr;
  }
  block_partials<1>(acc, part);
}

// One block.  stage 1: H(:,j) = first-pass coefficients; stage 2: second
// pass h2 added to H(:,j); stage 3: h_{j+1,j} = ||w||, Givens rotations,
// residual estimate, end-of-cycle test.
__global__ __launch_bounds__(RB) void k_gm_fin(const double* __restrict__ part, int g, int j,
                                               int stage, KState* st) {
  if (st->done || st->cycle) return;
  const int L = MAXM + 1;
  double* Hj = st->H + j * L;
  if (stage < 3) {
    const double out = finish_m(part, g);
    const int i = threadIdx.x;
    if (i <= j) {
      if (stage == 1) {
        Hj[i] = out;
      } else {
        st->h2[i] = out;
        Hj[i] += out;
      }
    }
    return;
  }
  double ww[1];
  finish<1>(part, g, ww);
  // stage the column, the rotations and g in LDS with parallel loads; one
  // thread then runs the short sequential recurrence on LDS
  __shared__ double hc[MAXM + 1], c_[MAXM], s_[MAXM], gg[2];
  __shared__ int verdict;
  const int t = threadIdx.x;
  if (t <= j) hc[t] = Hj[t];
  if (t < j) {
    c_[t] = st->cs[t];
    s_[t] = st->sn[t];
  }
  if (t == 0) gg[0] = st->g[j];
  __syncthreads();
  if (t == 0) {
    const double hn = sqrt(ww[0]);
    const int64_t it = st->iters + 1;
    verdict = 0;
    if (!isfinite(hn)) {
      verdict = ST_NONFINITE;
    } else {
      hc[j + 1] = hn;
      for (int i = 0; i < j; ++i) {
        const double a = hc[i], c = hc[i + 1];
        hc[i] = c_[i] * a + s_[i] * c;
        hc[i + 1] = -s_[i] * a + c_[i] * c;
      }
      const double a = hc[j], c = hc[j + 1];
      const double d = sqrt(a * a + c * c);
      if (d == 0.0) {
        verdict = ST_BREAKDOWN;
      } else {
        c_[j] = a / d;
        s_[j] = c / d;
        hc[j] = d;
        hc[j + 1] = 0.0;
        gg[1] = -s_[j] * gg[0];
        gg[0] = c_[j] * gg[0];
        const double est = fabs(gg[1]);
        st->k = j + 1;
        st->est = est;
        st->res2 = hn;  // h_{j+1,j} for the scaling kernel
        st->cs[j] = c_[j];
        st->sn[j] = s_[j];
        st->g[j] = gg[0];
        st->g[j + 1] = gg[1];
        if (est <= st->thr || hn == 0.0 || it >= st->max_iters || j + 1 >= st->m) st->cycle = 1;
      }
    }
    st->iters = it;
    if (verdict) st->done = verdict;
  }
  __syncthreads();
  if (verdict == 0 && t <= j + 1) Hj[t] = hc[t];
}

// v_{j+1} = w / h_{j+1,j}
__global__ __launch_bounds__(RB) void k_gm_scale(int64_t n, const double* __restrict__ w,
                                                 double* __restrict__ vn, const KState* st) {
  if (st->done || st->cycle) return;
  const double inv = 1.0 / st->res2;
  strided4(
      n, [&](int64_t i) { return Pack<double, 1>{{w[i]}}; },
      [&](int64_t i, const Pack<double, 1>& e) { vn[i] = e.v[0] * inv; });
}

// back substitution R y = g: the triangle is staged in LDS by all threads,
// then solved by one (k <= 32)
__global__ __launch_bounds__(RB) void k_gm_backsolve(KState* st) {
  if (st->done) return;
  constexpr int L = MAXM + 1;
  __shared__ double R[MAXM * L], gy[MAXM];
  const int k = st->k;
  for (int e = threadIdx.x; e < k * L; e += RB) R[e] = st->H[e];
  if ((int)threadIdx.x < k) gy[threadIdx.x] = st->g[threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int i = k - 1; i >= 0; --i) {
      double s = gy[i];
      for (int l = i + 1; l < k; ++l) s -= R[l * L + i] * gy[l];
      gy[i] = s / R[i * L + i];
    }
  __syncthreads();
  if ((int)threadIdx.x < k) st->y[threadIdx.x] = gy[threadIdx.x];
}

// x += V(:, 0..k-1) y
__global__ __launch_bounds__(RB) void k_gm_xupdate(int64_t n, int64_t ldv,
                                                   const double* __restrict__ V,
                                                   double* __restrict__ x, const KState* st) {
  if (st->done) return;
  __shared__ double y[MAXM];
  const int k = st->k;
  if (threadIdx.x < MAXM) y[threadIdx.x] = (int)threadIdx.x < k ? st->y[threadIdx.x] : 0.0;
  __syncthreads();
  GRID_STRIDE(r, n) {
    double xr = x[r];
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < k) xr += y[i] * V[i * ldv + r];
    x[r] = xr;
  }
}

// v_0 = r / beta with beta = sqrt(dot[0]); the one-block kernel below
// resets the cycle state first
__global__ void k_gm_reset(KState* st) {
  const double beta = sqrt(st->dot[0]);
  for (int i = 0; i <= MAXM; ++i) st->g[i] = 0.0;
  st->g[0] = beta;
  st->k = 0;
  st->cycle = 0;
}

__global__ __launch_bounds__(RB) void k_gm_start(int64_t n, const double* __restrict__ r,
                                                 double* __restrict__ v0, const KState* st) {
  const double inv = 1.0 / st->g[0];
  strided4(
      n, [&](int64_t i) { return Pack<double, 1>{{r[i]}}; },
      [&](int64_t i, const Pack<double, 1>& e) { v0[i] = e.v[0] * inv; });
}

// ---------------------------------------------------------------------------
// iterative refinement helpers
// ---------------------------------------------------------------------------
// f = float(r / sigma)
__global__ __launch_bounds__(RB) void k_ir_scale(int64_t n, const double* __restrict__ r,
                                                 double sigma, float* __restrict__ f) {
  strided4(
      n, [&](int64_t i) { return Pack<double, 1>{{r[i]}}; },
      [&](int64_t i, const Pack<double, 1>& e) { f[i] = (float)(e.v[0] / sigma); });
}

// x += d
__global__ __launch_bounds__(RB) void k_add(int64_t n, double* __restrict__ x,
                                            const double* __restrict__ d) {
  strided4(
      n, [&](int64_t i) { return Pack<double, 2>{{x[i], d[i]}}; },
      [&](int64_t i, const Pack<double, 2>& e) { x[i] = e.v[0] + e.v[1]; });
}

// p = z + c p in float: the first direction of an inner solve that carries
// the previous solve's last direction (c rescales it to the new right-hand
// side and is the CG coefficient beta)
__global__ __launch_bounds__(RB) void k_ir_carry(int64_t n, const float* __restrict__ z,
                                                 float* __restrict__ p, float c) {
  strided4(
      n, [&](int64_t i) { return Pack<float, 2>{{z[i], p[i]}}; },
      [&](int64_t i, const Pack<float, 2>& e) { p[i] = e.v[0] + c * e.v[1]; });
}

// x += sigma * double(d)
__global__ __launch_bounds__(RB) void k_ir_update(int64_t n, double* __restrict__ x,
                                                  const float* __restrict__ d, double sigma) {
  strided4(
      n, [&](int64_t i) { return Pack<double, 2>{{x[i], (double)d[i]}}; },
      [&](int64_t i, const Pack<double, 2>& e) { x[i] = e.v[0] + sigma * e.v[1]; });
}

// ---------------------------------------------------------------------------
// Pipelined CG (Ghysels & Vanroose 2014, unpreconditioned).  Iteration k
// (par = k & 1) is two launches: q = A w, then k_pipe_update, which
// finishes the partials of gamma = r.r and delta = w.r written by the
// previous update (they do not depend on q), tests gamma, forms
// beta = gamma / gamma_prev and alpha = gamma / (delta - beta gamma /
// alpha_prev), updates z = q + beta z, s = w + beta s, p = r + beta p,
// x += alpha p, r -= alpha s, w -= alpha z, and writes the partials of the
// next gamma and delta.  Partial buffers alternate by parity.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RB) void k_pipe_update(int64_t n, double* __restrict__ x,
                                                    double* __restrict__ r,
                                                    double* __restrict__ w,
                                                    const double* __restrict__ q,
                                                    double* __restrict__ z,
                                                    double* __restrict__ s,
                                                    double* __restrict__ p,
                                                    const double* __restrict__ pin, int g,
                                                    double* __restrict__ pout, KState* st,
                                                    int64_t k) {
  if (st->done) return;
  const int par = (int)(k & 1);
  const bool fresh = k == st->restart_at;
  double gd[2];
  if (fresh) {
    gd[0] = st->dot[0];
    gd[1] = st->dot[1];
  } else {
    finish<2>(pin, g, gd);
  }
  const double gamma = gd[0], delta = gd[1];
  double beta = 0.0, den = delta;
  if (!fresh) {
    beta = gamma / st->pg[1 - par];
    den = delta - beta * gamma / st->palpha[1 - par];
  }
  int32_t verdict = RUN;
  if (!isfinite(gamma) || !isfinite(delta))
    verdict = ST_NONFINITE;
  else if (sqrt(gamma) <= st->thr)
    verdict = ST_CONVERGED;
  else if (k >= st->max_iters)
    verdict = ST_MAXIT;
  else if (!isfinite(den))
    verdict = ST_NONFINITE;
  else if (den <= 0.0)
    verdict = ST_BREAKDOWN;
  const double alpha = gamma / den;
  if (lead()) {
    st->res2 = gamma;
    st->iters = verdict == RUN ? k + 1 : k;
    if (verdict != RUN) {
      st->done = verdict;
    } else {
      st->pg[par] = gamma;
      st->palpha[par] = alpha;
    }
  }
  if (verdict != RUN) return;
  double acc[2] = {0.0, 0.0};
  // e = (q, w, r, x, z, s, p); a fresh recurrence (beta = 0) reads no z, s, p
  const auto use = [&](int64_t i, const Pack<double, 7>& e) {
    const double zi = e.v[0] + beta * e.v[4];
    const double si = e.v[1] + beta * e.v[5];
    const double pi = e.v[2] + beta * e.v[6];
    z[i] = zi;
    s[i] = si;
    p[i] = pi;
    x[i] = e.v[3] + alpha * pi;
    const double ri = e.v[2] - alpha * si;
    const double wi = e.v[1] - alpha * zi;
    r[i] = ri;
    w[i] = wi;
    acc[0] += ri * ri;
    acc[1] += wi * ri;
  };
  if (fresh)
    strided4(
        n, [&](int64_t i) { return Pack<double, 7>{{q[i], w[i], r[i], x[i], 0.0, 0.0, 0.0}}; },
        use);
  else
    strided4(
        n,
        [&](int64_t i) { return Pack<double, 7>{{q[i], w[i], r[i], x[i], z[i], s[i], p[i]}}; },
        use);
  block_partials<2>(acc, pout);
}

// ---------------------------------------------------------------------------
// CGS (Sonneveld 1989; Saad 2003, Algorithm 7.6), r_hat = r0.  Iteration k
// (par = k & 1), rho[par] = (r_hat, r):
//   v = A p;   k_cgs_sigma: partials of r_hat.v (or the product forms them)
//   k_cgs_qw:  alpha = rho[par] / (r_hat.v), q = u - alpha v, w = u + q,
//              x += alpha w
//   v = A w;   k_cgs_r: r -= alpha v, partials of (r.r, r_hat.r)
//   k_cgs_dir: stopping test on r.r, rho[1-par] = r_hat.r,
//              beta = rho[1-par] / rho[par], u = r + beta q,
//              p = u + beta (q + beta p)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RB) void k_cgs_sigma(int64_t n, const double* __restrict__ rh,
                                                  const double* __restrict__ v,
                                                  double* __restrict__ pa, const KState* st) {
  if (st->done) return;
  double acc[1] = {0.0};
  strided4(
      n, [&](int64_t i) { return Pack<double, 2>{{rh[i], v[i]}}; },
      [&](int64_t, const Pack<double, 2>& e) { acc[0] += e.v[0] * e.v[1]; });
  block_partials<1>(acc, pa);
}

__global__ __launch_bounds__(RB) void k_cgs_qw(int64_t n, const double* __restrict__ u,
                                               const double* __restrict__ v,
                                               double* __restrict__ q, double* __restrict__ w,
                                               double* __restrict__ x,
                                               const double* __restrict__ pa, int g, KState* st,
                                               int par) {
  if (st->done) return;
  double sg[1];
  finish_wide<1>(pa, g, sg);  // the product's partials when it formed r_hat.v
  if (!isfinite(sg[0]) || sg[0] == 0.0) {
    if (lead()) st->done = isfinite(sg[0]) ? ST_BREAKDOWN : ST_NONFINITE;
    return;
  }
  const double a = st->rho[par] / sg[0];
  if (lead()) st->alpha = a;
  strided4(
      n, [&](int64_t i) { return Pack<double, 3>{{u[i], v[i], x[i]}}; },
      [&](int64_t i, const Pack<double, 3>& e) {
        const double qi = e.v[0] - a * e.v[1];
        const double wi = e.v[0] + qi;
        q[i] = qi;
        w[i] = wi;
        x[i] = e.v[2] + a * wi;
      });
}

__global__ __launch_bounds__(RB) void k_cgs_r(int64_t n, double* __restrict__ r,
                                              const double* __restrict__ v,
                                              const double* __restrict__ rh,
                                              double* __restrict__ pb, const KState* st) {
  if (st->done) return;
  const double a = st->alpha;
  double acc[2] = {0.0, 0.0};
  strided4(
      n, [&](int64_t i) { return Pack<double, 3>{{r[i], v[i], rh[i]}}; },
      [&](int64_t i, const Pack<double, 3>& e) {
        const double ri = e.v[0] - a * e.v[1];
        r[i] = ri;
        acc[0] += ri * ri;
        acc[1] += e.v[2] * ri;
      });
  block_partials<2>(acc, pb);
}

__global__ __launch_bounds__(RB) void k_cgs_dir(int64_t n, const double* __restrict__ r,
                                                const double* __restrict__ q,
                                                double* __restrict__ u, double* __restrict__ p,
                                                const double* __restrict__ pb, int g, KState* st,
                                                int par, int64_t k) {
  if (st->done) return;
  double t[2];
  finish<2>(pb, g, t);
  const double rr = t[0], rhr = t[1];
  int32_t verdict = RUN;
  if (!isfinite(rr))
    verdict = ST_NONFINITE;
  else if (sqrt(rr) <= st->thr)
    verdict = ST_CONVERGED;
  else if (k + 1 >= st->max_iters)
    verdict = ST_MAXIT;
  else if (!isfinite(rhr))
    verdict = ST_NONFINITE;
  else if (rhr == 0.0)
    verdict = ST_BREAKDOWN;
  if (lead()) {
    st->iters = k + 1;
    st->res2 = rr;
    st->rho[1 - par] = rhr;
    if (verdict != RUN) st->done = verdict;
  }
  if (verdict != RUN) return;
  const double beta = rhr / st->rho[par];
  strided4(
      n, [&](int64_t i) { return Pack<double, 3>{{r[i], q[i], p[i]}}; },
      [&](int64_t i, const Pack<double, 3>& e) {
        const double ui = e.v[0] + beta * e.v[1];
        u[i] = ui;
        p[i] = ui + beta * (e.v[1] + beta * e.v[2]);
      });
}

// ---------------------------------------------------------------------------
// Preconditioned CG (Saad 2003, Algorithm 9.1), PC = 1 Jacobi (z = dinv r,
// never stored: formed where it is used), PC = 2 block Jacobi (z stored).
// Iteration k (par = k & 1), rho[par] = (r, z) of the previous step:
//   q = A p;  k_cg_pq: partials of p.q;
//   k_pcg_update: alpha = rho[par] / (p.q), x += alpha p, r -= alpha q,
//                 partials of (r.z, r.r) (Jacobi) or r.r (block);
//   [block: k_bj_apply: z = M^{-1} r, partials of r.z]
//   k_pcg_direction: stopping test on r.r, rho[1-par] = r.z,
//                    p = z + (rho[1-par] / rho[par]) p.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(RB) void k_jac_apply(int64_t n, const T* __restrict__ dinv,
                                                  const T* __restrict__ r, T* __restrict__ z) {
  strided4(
      n, [&](int64_t i) { return Pack<T, 2>{{dinv[i], r[i]}}; },
      [&](int64_t i, const Pack<T, 2>& e) { z[i] = e.v[0] * e.v[1]; });
}

// z = M^{-1} r for block Jacobi: a wave holds G = 64 / bs blocks, lane l
// row l % bs of block l / bs; the block's r values travel by shuffles.
// Grid-stride over waves (fixed order); partials of r.z when `part`.
template <typename T>
__global__ __launch_bounds__(RB) void k_bj_apply(int64_t n, int bs, const T* __restrict__ minv,
                                                 const T* __restrict__ r, T* __restrict__ z,
                                                 double* __restrict__ part, const KState* st) {
  if (st && st->done) return;
  const int lane = threadIdx.x & 63;
  const int G = 64 / bs;
  const int gi = lane / bs, i = lane - gi * bs;
  const int64_t nb = (n + bs - 1) / bs;
  const int64_t nwaves = (int64_t)gridDim.x * (RB / 64);
  double acc[1] = {0.0};
  for (int64_t wb = (int64_t)blockIdx.x * (RB / 64) + threadIdx.x / 64; wb * G < nb;
       wb += nwaves) {
    const int64_t blk = wb * G + gi;
    const bool on = gi < G && blk < nb;
    const int64_t r0 = blk * bs;
    const int m = on ? (int)((n - r0) < bs ? (n - r0) : bs) : 0;
    const bool row = i < m;
    const T ri = row ? r[r0 + i] : T(0);
    const T* __restrict__ M = minv + (on ? blk : 0) * bs * bs;
    T sum = 0;
    for (int j = 0; j < bs; ++j) {
      const T rj = __shfl(ri, gi * bs + j, 64);
      if (row && j < m) sum += M[j * bs + i] * rj;
    }
    if (row) {
      z[r0 + i] = sum;
      acc[0] += (double)ri * (double)sum;
    }
  }
  if (part) block_partials<1>(acc, part);
}

template <typename T, int PC>
__global__ __launch_bounds__(RB) void k_pcg_update(int64_t n, T* __restrict__ x,
                                                   const T* __restrict__ p, T* __restrict__ r,
                                                   const T* __restrict__ q,
                                                   const T* __restrict__ dinv,
                                                   const double* __restrict__ pa, int g,
                                                   double* __restrict__ pb, KState* st, int par) {
  if (st->done) return;
  double pq[1];
  finish<1>(pa, g, pq);
  if (!isfinite(pq[0]) || pq[0] <= 0.0) {
    if (lead()) st->done = isfinite(pq[0]) ? ST_BREAKDOWN : ST_NONFINITE;
    return;
  }
  const double alpha = st->rho[par] / pq[0];
  if (lead()) st->alpha = alpha;
  const T a = (T)alpha;
  double acc[2] = {0.0, 0.0};
  // e = (x, p, r, q, dinv); block Jacobi reads no dinv
  const auto use = [&](int64_t i, const Pack<T, 5>& e) {
    x[i] = e.v[0] + a * e.v[1];
    const T ri = e.v[2] - a * e.v[3];
    r[i] = ri;
    if (PC == 1) acc[1] += (double)ri * (double)(e.v[4] * ri);
    acc[0] += (double)ri * (double)ri;
  };
  strided4(
      n,
      [&](int64_t i) {
        return Pack<T, 5>{{x[i], p[i], r[i], q[i], PC == 1 ? dinv[i] : T(0)}};
      },
      use);
  if (PC == 1) {
    block_partials<2>(acc, pb);
  } else {
    const double rr[1] = {acc[0]};
    block_partials<1>(rr, pb);
  }
}

template <typename T, int PC>
__global__ __launch_bounds__(RB) void k_pcg_direction(int64_t n, const T* __restrict__ r,
                                                      T* __restrict__ p,
                                                      const T* __restrict__ z,
                                                      const T* __restrict__ dinv,
                                                      const double* __restrict__ pb,
                                                      const double* __restrict__ pc, int g,
                                                      KState* st, int par, int64_t k) {
  if (st->done) return;
  double rr, rz;
  if (PC == 1) {
    double t[2];
    finish<2>(pb, g, t);
    rr = t[0];
    rz = t[1];
  } else {
    double t1[1], t2[1];
    finish<1>(pb, g, t1);
    finish<1>(pc, g, t2);
    rr = t1[0];
    rz = t2[0];
  }
  const bool bad = !isfinite(rr) || !isfinite(rz);
  const bool conv = !bad && sqrt(rr) <= st->thr;
  const bool maxit = k + 1 >= st->max_iters;
  const bool brk = !(rz > 0.0);
  if (lead()) {
    st->iters = k + 1;
    st->res2 = rr;
    st->rho[1 - par] = rz;
    if (bad)
      st->done = ST_NONFINITE;
    else if (conv)
      st->done = ST_CONVERGED;
    else if (maxit)
      st->done = ST_MAXIT;
    else if (brk)
      st->done = ST_BREAKDOWN;
  }
  if (bad || conv || maxit || brk) return;
  const T beta = (T)(rz / st->rho[par]);
  if (PC == 1)
    strided4(
        n, [&](int64_t i) { return Pack<T, 3>{{dinv[i], r[i], p[i]}}; },
        [&](int64_t i, const Pack<T, 3>& e) { p[i] = e.v[0] * e.v[1] + beta * e.v[2]; });
  else
    strided4(
        n, [&](int64_t i) { return Pack<T, 2>{{z[i], p[i]}}; },
        [&](int64_t i, const Pack<T, 2>& e) { p[i] = e.v[0] + beta * e.v[1]; });
}

// ---------------------------------------------------------------------------
// PageRank by power iteration (Page, Brin, Motwani & Winograd 1998) over the
// transition matrix T (T[j,i] = 1/d_i, stored by in-links).  Iteration k:
//   z = T x (the library's SpMV, any format);
//   k_pr_update: finishes the partials written by the previous update (or
//   the set-up), the dangling mass m = sum of x over nodes without
//   out-links and the L1 change of the previous step; stops on that change;
//   x = damping (z + m/n) + (1 - damping)/n in place; partials of the new
//   dangling mass and of |x_new - x_old|.  Partial buffers alternate.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_outdeg(int64_t nnz, const int32_t* __restrict__ col,
                                                int32_t* __restrict__ d) {
  // integer counts: the result does not depend on the order of the adds
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * 256)
    atomicAdd(&d[col[k]], 1);
}

__global__ __launch_bounds__(256) void k_transition(int64_t nnz, const int32_t* __restrict__ col,
                                                    const int32_t* __restrict__ d,
                                                    double* __restrict__ val) {
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * 256)
    val[k] = 1.0 / (double)d[col[k]];
}

__global__ __launch_bounds__(256) void k_dangling(int64_t n, const int32_t* __restrict__ d,
                                                  uint8_t* __restrict__ mask) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) mask[i] = d[i] == 0 ? 1 : 0;
}

__global__ __launch_bounds__(RB) void k_pr_init(int64_t n, double* __restrict__ x,
                                                const uint8_t* __restrict__ mask,
                                                double* __restrict__ pout) {
  const double u = 1.0 / (double)n;
  double acc[2] = {0.0, 0.0};
  GRID_STRIDE(i, n) {
    x[i] = u;
    if (mask[i]) acc[0] += u;
  }
  block_partials<2>(acc, pout);
}

__global__ __launch_bounds__(RB) void k_pr_update(int64_t n, double* __restrict__ x,
                                                  const double* __restrict__ z,
                                                  const uint8_t* __restrict__ mask,
                                                  double damping, const double* __restrict__ pin,
                                                  int g, double* __restrict__ pout, KState* st,
                                                  int64_t k) {
  if (st->done) return;
  double md[2];
  finish<2>(pin, g, md);
  const double mass = md[0], change = md[1];
  int32_t verdict = RUN;
  if (k > 0 && !isfinite(change))
    verdict = ST_NONFINITE;
  else if (k > 0 && change <= st->thr)
    verdict = ST_CONVERGED;
  else if (k >= st->max_iters)
    verdict = ST_MAXIT;
  if (lead()) {
    if (k > 0) st->res2 = change;
    st->iters = verdict == RUN ? k + 1 : k;  // steps taken once this one is done
    if (verdict != RUN) st->done = verdict;
  }
  if (verdict != RUN) return;
  const double nd = (double)n;
  const double tele = (1.0 - damping) / nd;
  const double share = mass / nd;
  double acc[2] = {0.0, 0.0};
  strided4(
      n, [&](int64_t i) { return Pack<double, 3>{{z[i], x[i], mask[i] ? 1.0 : 0.0}}; },
      [&](int64_t i, const Pack<double, 3>& e) {
        const double xn = damping * (e.v[0] + share) + tele;
        acc[1] += fabs(xn - e.v[1]);
        x[i] = xn;
        if (e.v[2] != 0.0) acc[0] += xn;
      });
  block_partials<2>(acc, pout);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Work {
  KState* st;        // device
  KState* hst;       // pinned mirror
  double* pa;        // four partial buffers of MAXG * 2 doubles
  double* pb;
  double* pc;
  double* pd;
  double* pm;        // MAXG * MAXM doubles (GMRES multi-dots)
  double* pw;        // kDotPartials doubles (partials of a product with its dot)
  char* vec;         // vectors
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

mxs_status get_work(mxs_ctx* ctx, size_t vec_bytes, Work* w) {
  const size_t st_bytes = align_up(sizeof(KState), 256);
  const size_t p2 = (size_t)MAXG * 2 * sizeof(double);
  const size_t pm = (size_t)MAXG * MAXM * sizeof(double);
  const size_t pw = (size_t)kDotPartials * sizeof(double);
  const size_t total = st_bytes + 4 * p2 + pm + pw + vec_bytes + 256;
  if (!ws_reserve(ctx, total)) return fail(ctx, MXS_OOM, "solver workspace of %zu bytes", total);
  // host mirror + the two polling copies
  if (!pinned_reserve(ctx, 3 * st_bytes)) return fail(ctx, MXS_OOM, "pinned state mirror");
  char* base = (char*)ctx->ws.ptr;
  w->st = (KState*)base;
  w->pa = (double*)(base + st_bytes);
  w->pb = (double*)(base + st_bytes + p2);
  w->pc = (double*)(base + st_bytes + 2 * p2);
  w->pd = (double*)(base + st_bytes + 3 * p2);
  w->pm = (double*)(base + st_bytes + 4 * p2);
  w->pw = (double*)(base + st_bytes + 4 * p2 + pm);
  w->vec = base + st_bytes + 4 * p2 + pm + pw;
  w->hst = (KState*)ctx->pinned;
  MXS_HIP_TRY(ctx, hipMemsetAsync(w->st, 0, sizeof(KState), ctx->stream));
  return MXS_OK;
}

mxs_status push_state(mxs_ctx* ctx, Work& w) {
  MXS_HIP_TRY(ctx, hipMemcpyAsync(w.st, w.hst, sizeof(KState), hipMemcpyHostToDevice,
                                  ctx->stream));
  // the pinned buffer is reused by pull_state: the upload must finish first
  MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MXS_OK;
}

mxs_status pull_state(mxs_ctx* ctx, Work& w) {
  MXS_HIP_TRY(ctx, hipMemcpyAsync(w.hst, w.st, sizeof(KState), hipMemcpyDeviceToHost,
                                  ctx->stream));
  MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MXS_OK;
}

// enqueues a.b (and c.d) into st->dot without synchronising
template <typename T>
void enqueue_dots(mxs_ctx* ctx, Work& w, int64_t n, const T* a, const T* b, const T* c,
                  const T* d) {
  const int g = red_grid(n);
  k_dots<T><<<g, RB, 0, ctx->stream>>>(n, a, b, c, d, w.pa);
  k_dots_fin<<<1, RB, 0, ctx->stream>>>(w.pa, g, w.st);
}

// dot products of device vectors into the host mirror (synchronising)
template <typename T>
mxs_status dots(mxs_ctx* ctx, Work& w, int64_t n, const T* a, const T* b, const T* c,
                const T* d, double* out0, double* out1) {
  enqueue_dots<T>(ctx, w, n, a, b, c, d);
  MXS_HIP_TRY(ctx, hipGetLastError());
  MXS_HIP_TRY(ctx, hipMemcpyAsync(w.hst->dot, w.st->dot, 2 * sizeof(double),
                                  hipMemcpyDeviceToHost, ctx->stream));
  MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  *out0 = w.hst->dot[0];
  if (out1) *out1 = w.hst->dot[1];
  return MXS_OK;
}

// r = b - A x in FP64
mxs_status residual(mxs_ctx* ctx, const mxs_matrix* A, const double* b, const double* x,
                    double* r) {
  const int64_t n = A->n;
  MXS_HIP_TRY(ctx, hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice,
                                  ctx->stream));
  const double m1 = -1.0, one = 1.0;
  return launch_spmv(ctx, A, &m1, x, &one, r, nullptr);
}

mxs_status map_done(int32_t done) {
  switch (done) {
    case ST_BREAKDOWN: return MXS_BREAKDOWN;
    case ST_NONFINITE: return MXS_NONFINITE;
    case ST_MAXIT: return MXS_NOT_CONVERGED;
    default: return MXS_OK;
  }
}

struct Stop {
  int64_t max_iters;
  double rel_tol, abs_tol;
  int baseline, check_every, max_repl;
};

Stop read_stop(const mxs_stop* s, int64_t default_max) {
  Stop o{default_max, 1e-10, 0.0, MXS_BASELINE_RHS, 16, 3};
  if (s) {
    if (s->max_iters > 0) o.max_iters = s->max_iters;
    o.rel_tol = s->rel_tol;
    o.abs_tol = s->abs_tol;
    o.baseline = s->baseline;
    if (s->check_every > 0) o.check_every = s->check_every;
    if (s->max_replacements >= 0) o.max_repl = s->max_replacements;
  }
  return o;
}

// Runs CG iterations from the state already on the device until the
// device status is set.  Vectors of type T; the operator is A.
// The host polls the device status without leaving the GPU idle: after
// each batch of `check_every` iterations it enqueues a copy of the state
// into one of two pinned slots and an event, enqueues the next batch, and
// only then waits for the previous batch's copy.  A batch enqueued after
// the one that finished the solve returns at once in every kernel.
struct StatusPoll {
  mxs_ctx* ctx;
  Work& w;
  KState* slot[2];
  StatusPoll(mxs_ctx* c, Work& wk) : ctx(c), w(wk) {
    const size_t stb = align_up(sizeof(KState), 256);
    slot[0] = (KState*)((char*)ctx->pinned + stb);
    slot[1] = (KState*)((char*)ctx->pinned + 2 * stb);
  }
  mxs_status record(int s) {
    MXS_HIP_TRY(ctx, hipMemcpyAsync(slot[s], w.st, sizeof(KState), hipMemcpyDeviceToHost,
                                    ctx->stream));
    MXS_HIP_TRY(ctx, hipEventRecord(ctx->poll_ev[s], ctx->stream));
    return MXS_OK;
  }
  mxs_status wait(int s) {
    MXS_HIP_TRY(ctx, hipEventSynchronize(ctx->poll_ev[s]));
    return MXS_OK;
  }
};

// Enqueues batch(k0) for k0 = k, k + C, k + 2C, ... until the device status
// is set, polling it through StatusPoll; returns with the final state in
// w.hst.
template <typename Batch>
mxs_status run_polled(mxs_ctx* ctx, Work& w, int64_t k, int C, const char* what, Batch batch) {
  StatusPoll poll(ctx, w);
  mxs_status s;
  if ((s = batch(k)) || (s = poll.record(0))) return s;
  int cur = 0;
  int64_t seen = k;
  for (int64_t kq = k + C;; kq += C) {
    if ((s = batch(kq)) || (s = poll.record(1 - cur)) || (s = poll.wait(cur))) return s;
    const KState& sn = *poll.slot[cur];
    if (sn.done) return pull_state(ctx, w);
    if (sn.iters <= seen)
      return fail(ctx, MXS_HIP, "%s made no progress (device state not updated)", what);
    seen = sn.iters;
    cur = 1 - cur;
  }
}

template <typename T>
mxs_status cg_loop(mxs_ctx* ctx, const mxs_matrix* A, Work& w, T* x, T* r, T* p, T* q,
                   int check_every) {
  const int64_t n = A->n;
  const int g = red_grid(n);
  const T one = 1, zero = 0;
  return run_polled(ctx, w, w.hst->iters, check_every, "CG", [&](int64_t k0) -> mxs_status {
    for (int64_t kk = k0; kk < k0 + check_every; ++kk) {
      const int par = (int)(kk & 1);
      // q = A p and p.q: in the product's own launches when its kernel
      // offers that, else a separate reduction
      const double* pq = w.pw;
      int gq = launch_spmv_dot(ctx, A, p, q, &w.st->done, w.pw);
      if (gq == 0) {
        mxs_status s = launch_spmv(ctx, A, &one, p, &zero, q, &w.st->done);
        if (s) return s;
        k_cg_pq<T><<<g, RB, 0, ctx->stream>>>(n, p, q, w.pa, w.st);
        pq = w.pa;
        gq = g;
      }
      k_cg_r<T><<<g, RB, 0, ctx->stream>>>(n, r, q, pq, gq, w.pb, w.st, par, kk);
      k_cg_xp<T><<<g, RB, 0, ctx->stream>>>(n, x, r, p, w.pb, g, w.st, par, kk);
    }
    MXS_HIP_TRY(ctx, hipGetLastError());
    return MXS_OK;
  });
}

void fill_info(mxs_solve_info* info, const KState& h, double base, double relres_true,
               int64_t repl, int64_t restarts, mxs_status st) {
  if (!info) return;
  info->iters = h.iters;
  info->relres_recurrence = sqrt(h.res2 > 0 ? h.res2 : 0.0) / base;
  info->relres_true = relres_true;
  info->replacements = repl;
  info->restarts = restarts;
  info->status = st;
}

mxs_status zero_solution(mxs_ctx* ctx, double* x, int64_t n, mxs_solve_info* info) {
  MXS_HIP_TRY(ctx, hipMemsetAsync(x, 0, n * sizeof(double), ctx->stream));
  MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  KState z{};
  fill_info(info, z, 1.0, 0.0, 0, 0, MXS_OK);
  return MXS_OK;
}

bool small_path(const mxs_matrix* A, const Stop& stop) {
  if (A->fmt != MXS_CSR || A->dt != MXS_F64 || stop.max_repl != 3 || A->n > 8192) return false;
  int64_t maxL = 0;
  for (int64_t i = 0; i < A->n; ++i)
    maxL = std::max<int64_t>(maxL, A->h_rowptr[i + 1] - A->h_rowptr[i]);
  return small_cg_fits(A->n, maxL);
}

// CG on a small CSR system: one work-group runs the whole solve (initial
// residual, norms, iterations, true-residual check) and x is updated in
// place; the host only reads the final state.
mxs_status solve_cg_small(mxs_ctx* ctx, const mxs_matrix* A, const double* b, double* x,
                          const Stop& stop, mxs_solve_info* info) {
  const int64_t n = A->n;
  if (!ws_reserve(ctx, small_cg_scratch(n)))
    return fail(ctx, MXS_OOM, "solver workspace of %zu bytes", small_cg_scratch(n));
  if (!pinned_reserve(ctx, kSmallCgPinned)) return fail(ctx, MXS_OOM, "pinned staging");
  SmallCgResult sr;
  mxs_status s = small_cg(ctx, A, b, x, stop.rel_tol, stop.abs_tol,
                          stop.baseline == MXS_BASELINE_INITIAL, stop.max_iters, ctx->ws.ptr,
                          ctx->pinned, &sr);
  if (s) return s;
  const double base = sr.base > 0 ? sr.base : 1.0;
  KState h{};
  h.iters = sr.iters;
  h.res2 = sr.res2;
  if (sr.status == MXS_OK) {
    // res2 is the kernel's true residual of the returned x (0 when b = 0)
    fill_info(info, h, base, sqrt(sr.res2) / base, sr.replacements, 0, MXS_OK);
    return MXS_OK;
  }
  if (sr.status == MXS_NONFINITE) {
    fill_info(info, h, base, NAN, sr.replacements, 0, MXS_NONFINITE);
    return fail(ctx, MXS_NONFINITE, "non-finite value in CG (right-hand side, x0 or iterate)");
  }
  // stopped early: the true residual of the returned x for the report
  const size_t ld = align_up((size_t)n, 64);
  Work w;
  if ((s = get_work(ctx, ld * sizeof(double), &w))) return s;
  double* r = (double*)w.vec;
  double rt2;
  if ((s = residual(ctx, A, b, x, r))) return s;
  if ((s = dots<double>(ctx, w, n, r, r, (const double*)nullptr, (const double*)nullptr, &rt2,
                        nullptr)))
    return s;
  fill_info(info, h, base, sqrt(rt2) / base, sr.replacements, 0, sr.status);
  return fail(ctx, sr.status, sr.status == MXS_BREAKDOWN
                                  ? "CG breakdown: p.Ap <= 0 (matrix not SPD)"
                                  : "CG stopped after %lld iterations, relres %.3e",
              (long long)sr.iters, sqrt(rt2) / base);
}

mxs_status solve_cg(mxs_ctx* ctx, const mxs_matrix* A, const double* b, double* x,
                    const Stop& stop, mxs_solve_info* info) {
  if (small_path(A, stop)) return solve_cg_small(ctx, A, b, x, stop, info);
  const int64_t n = A->n;
  const size_t ld = align_up((size_t)n, 64);
  Work w;
  mxs_status s = get_work(ctx, 3 * ld * sizeof(double), &w);
  if (s) return s;
  double* r = (double*)w.vec;
  double* p = r + ld;
  double* q = p + ld;
  double nb2, nr2;
  if ((s = residual(ctx, A, b, x, r))) return s;
  if ((s = dots<double>(ctx, w, n, b, b, r, r, &nb2, &nr2))) return s;
  const double nb = sqrt(nb2), nr0 = sqrt(nr2);
  if (!std::isfinite(nb)) return fail(ctx, MXS_NONFINITE, "non-finite right-hand side");
  if (nb == 0.0) return zero_solution(ctx, x, n, info);
  if (!std::isfinite(nr0)) return fail(ctx, MXS_NONFINITE, "non-finite initial residual");
  const double base = stop.baseline == MXS_BASELINE_INITIAL ? (nr0 > 0 ? nr0 : 1.0) : nb;
  const double thr = std::max(stop.rel_tol * base, stop.abs_tol);
  KState& h = *w.hst;
  std::memset(&h, 0, sizeof(KState));
  h.rho[0] = nr2;
  h.res2 = nr2;
  h.thr = thr;
  h.max_iters = stop.max_iters;
  h.done = nr0 <= thr ? ST_CONVERGED : RUN;
  if ((s = push_state(ctx, w))) return s;
  MXS_HIP_TRY(ctx, hipMemcpyAsync(p, r, n * sizeof(double), hipMemcpyDeviceToDevice,
                                  ctx->stream));
  int64_t repl = 0;
  double relres_true = nr0 / base;
  for (;;) {
    if (h.done == RUN) {
      if ((s = cg_loop<double>(ctx, A, w, x, r, p, q, stop.check_every))) return s;
    }
    if (h.done == ST_BREAKDOWN || h.done == ST_NONFINITE) {
      s = map_done(h.done);
      fill_info(info, h, base, relres_true, repl, 0, s);
      return fail(ctx, s, h.done == ST_BREAKDOWN ? "CG breakdown: p.Ap <= 0 (matrix not SPD)"
                                                 : "non-finite value in CG");
    }
    // true residual check (also after max_iters)
    double rt2;
    if ((s = residual(ctx, A, b, x, r))) return s;
    if ((s = dots<double>(ctx, w, n, r, r, (const double*)nullptr, (const double*)nullptr,
                          &rt2, nullptr)))
      return s;
    relres_true = sqrt(rt2) / base;
    const int32_t why = h.done;
    if (why == ST_CONVERGED && sqrt(rt2) <= thr) {
      fill_info(info, h, base, relres_true, repl, 0, MXS_OK);
      return MXS_OK;
    }
    if (why == ST_MAXIT || repl >= stop.max_repl || h.iters >= stop.max_iters) {
      fill_info(info, h, base, relres_true, repl, 0, MXS_NOT_CONVERGED);
      return fail(ctx, MXS_NOT_CONVERGED, "CG stopped after %lld iterations, relres %.3e",
                  (long long)h.iters, relres_true);
    }
    // residual replacement: r = b - A x (already in r), restart p = r
    repl++;
    h.rho[h.iters & 1] = rt2;
    h.res2 = rt2;
    h.done = RUN;
    h.halt = 0;
    if ((s = push_state(ctx, w))) return s;
    MXS_HIP_TRY(ctx, hipMemcpyAsync(p, r, n * sizeof(double), hipMemcpyDeviceToDevice,
                                    ctx->stream));
  }
}

// z = M^{-1} r (enqueued)
template <typename T>
void apply_precond(mxs_ctx* ctx, const mxs_precond* M, const T* mv, int64_t n, const T* r,
                   T* z) {
  const int g = red_grid(n);
  if (M->kind == MXS_PRECOND_JACOBI)
    k_jac_apply<T><<<g, RB, 0, ctx->stream>>>(n, mv, r, z);
  else
    k_bj_apply<T><<<g, RB, 0, ctx->stream>>>(n, M->bs, mv, r, z, nullptr, nullptr);
}

// Preconditioned CG iterations from the state on the device until the
// device status is set; mv = M's values in the vector type.
template <typename T, int PC>
mxs_status pcg_loop(mxs_ctx* ctx, const mxs_matrix* A, const mxs_precond* M, const T* mv,
                    Work& w, T* x, T* r, T* p, T* q, T* z, int check_every) {
  const int64_t n = A->n;
  const int g = red_grid(n);
  const T one = 1, zero = 0;
  return run_polled(ctx, w, w.hst->iters, check_every, "PCG", [&](int64_t k0) -> mxs_status {
    for (int64_t k = k0; k < k0 + check_every; ++k) {
      const int par = (int)(k & 1);
      mxs_status s = launch_spmv(ctx, A, &one, p, &zero, q, &w.st->done);
      if (s) return s;
      k_cg_pq<T><<<g, RB, 0, ctx->stream>>>(n, p, q, w.pa, w.st);
      k_pcg_update<T, PC><<<g, RB, 0, ctx->stream>>>(n, x, p, r, q, mv, w.pa, g, w.pb, w.st,
                                                     par);
      if (PC == 2)
        k_bj_apply<T><<<g, RB, 0, ctx->stream>>>(n, M->bs, mv, r, z, w.pc, w.st);
      k_pcg_direction<T, PC><<<g, RB, 0, ctx->stream>>>(n, r, p, z, mv, w.pb, w.pc, g, w.st,
                                                        par, k);
    }
    MXS_HIP_TRY(ctx, hipGetLastError());
    return MXS_OK;
  });
}

template <typename T>
mxs_status pcg_run(mxs_ctx* ctx, const mxs_matrix* A, const mxs_precond* M, const T* mv,
                   Work& w, T* x, T* r, T* p, T* q, T* z, int check_every) {
  return M->kind == MXS_PRECOND_JACOBI
             ? pcg_loop<T, 1>(ctx, A, M, mv, w, x, r, p, q, z, check_every)
             : pcg_loop<T, 2>(ctx, A, M, mv, w, x, r, p, q, z, check_every);
}

mxs_status solve_pcg(mxs_ctx* ctx, const mxs_matrix* A, const mxs_precond* M, const double* b,
                     double* x, const Stop& stop, mxs_solve_info* info) {
  const int64_t n = A->n;
  const size_t ld = align_up((size_t)n, 64);
  Work w;
  mxs_status s = get_work(ctx, 4 * ld * sizeof(double), &w);
  if (s) return s;
  double* r = (double*)w.vec;
  double* p = r + ld;
  double* q = p + ld;
  double* z = q + ld;
  double nb2, nr2, rz;
  if ((s = residual(ctx, A, b, x, r))) return s;
  if ((s = dots<double>(ctx, w, n, b, b, r, r, &nb2, &nr2))) return s;
  const double nb = sqrt(nb2), nr0 = sqrt(nr2);
  if (!std::isfinite(nb)) return fail(ctx, MXS_NONFINITE, "non-finite right-hand side");
  if (nb == 0.0) return zero_solution(ctx, x, n, info);
  if (!std::isfinite(nr0)) return fail(ctx, MXS_NONFINITE, "non-finite initial residual");
  const double base = stop.baseline == MXS_BASELINE_INITIAL ? (nr0 > 0 ? nr0 : 1.0) : nb;
  const double thr = std::max(stop.rel_tol * base, stop.abs_tol);
  KState& h = *w.hst;
  // z = M^{-1} r, rho = r.z, p = z
  auto restart = [&](double rr) -> mxs_status {
    apply_precond<double>(ctx, M, M->m64, n, r, z);
    mxs_status e = dots<double>(ctx, w, n, r, z, (const double*)nullptr, (const double*)nullptr,
                                &rz, nullptr);
    if (e) return e;
    h.rho[h.iters & 1] = rz;
    h.res2 = rr;
    h.done = sqrt(rr) <= thr ? ST_CONVERGED
             : !std::isfinite(rz) ? ST_NONFINITE
             : rz > 0.0 ? RUN : ST_BREAKDOWN;
    if ((e = push_state(ctx, w))) return e;
    MXS_HIP_TRY(ctx, hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice,
                                    ctx->stream));
    return MXS_OK;
  };
  std::memset(&h, 0, sizeof(KState));
  h.thr = thr;
  h.max_iters = stop.max_iters;
  if ((s = restart(nr2))) return s;
  int64_t repl = 0;
  double relres_true = nr0 / base;
  for (;;) {
    if (h.done == RUN) {
      if ((s = pcg_run<double>(ctx, A, M, M->m64, w, x, r, p, q, z, stop.check_every)))
        return s;
    }
    if (h.done == ST_BREAKDOWN || h.done == ST_NONFINITE) {
      s = map_done(h.done);
      fill_info(info, h, base, relres_true, repl, 0, s);
      return fail(ctx, s, h.done == ST_BREAKDOWN
                              ? "PCG breakdown: p.Ap <= 0 or r.z <= 0 (A or M not SPD)"
                              : "non-finite value in PCG");
    }
    double rt2;
    if ((s = residual(ctx, A, b, x, r))) return s;
    if ((s = dots<double>(ctx, w, n, r, r, (const double*)nullptr, (const double*)nullptr,
                          &rt2, nullptr)))
      return s;
    relres_true = sqrt(rt2) / base;
    const int32_t why = h.done;
    if (why == ST_CONVERGED && sqrt(rt2) <= thr) {
      fill_info(info, h, base, relres_true, repl, 0, MXS_OK);
      return MXS_OK;
    }
    if (why == ST_MAXIT || repl >= stop.max_repl || h.iters >= stop.max_iters) {
      fill_info(info, h, base, relres_true, repl, 0, MXS_NOT_CONVERGED);
      return fail(ctx, MXS_NOT_CONVERGED, "PCG stopped after %lld iterations, relres %.3e",
                  (long long)h.iters, relres_true);
    }
    // residual replacement: r = b - A x (already in r), restart p = z
    repl++;
    if ((s = restart(rt2))) return s;
  }
}

mxs_status solve_bicgstab(mxs_ctx* ctx, const mxs_matrix* A, const double* b, double* x,
                          const Stop& stop, mxs_solve_info* info) {
  const int64_t n = A->n;
  const size_t ld = align_up((size_t)n, 64);
  Work w;
  mxs_status s = get_work(ctx, 6 * ld * sizeof(double), &w);
  if (s) return s;
  double* r = (double*)w.vec;
  double* rh = r + ld;
  double* p = rh + ld;
  double* v = p + ld;
  double* sv = v + ld;
  double* t = sv + ld;
  double nb2, nr2;
  if ((s = residual(ctx, A, b, x, r))) return s;
  if ((s = dots<double>(ctx, w, n, b, b, r, r, &nb2, &nr2))) return s;
  const double nb = sqrt(nb2), nr0 = sqrt(nr2);
  if (!std::isfinite(nb)) return fail(ctx, MXS_NONFINITE, "non-finite right-hand side");
  if (nb == 0.0) return zero_solution(ctx, x, n, info);
  if (!std::isfinite(nr0)) return fail(ctx, MXS_NONFINITE, "non-finite initial residual");
  const double base = stop.baseline == MXS_BASELINE_INITIAL ? (nr0 > 0 ? nr0 : 1.0) : nb;
  const double thr = std::max(stop.rel_tol * base, stop.abs_tol);
  const int g = red_grid(n);
  const double one = 1.0, zero = 0.0;
  KState& h = *w.hst;
  std::memset(&h, 0, sizeof(KState));
  int64_t repl = 0;
  double relres_true = nr0 / base;
  int32_t done = nr0 <= thr ? ST_CONVERGED : RUN;
  int64_t iters = 0;
  double rr = nr2;
  for (;;) {
    if (done == RUN) {
      // (re)start: r_hat = r, p = v = 0, rho = alpha = omega = 1
      MXS_HIP_TRY(ctx, hipMemcpyAsync(rh, r, n * sizeof(double), hipMemcpyDeviceToDevice,
                                      ctx->stream));
      MXS_HIP_TRY(ctx, hipMemsetAsync(p, 0, n * sizeof(double), ctx->stream));
      MXS_HIP_TRY(ctx, hipMemsetAsync(v, 0, n * sizeof(double), ctx->stream));
      std::memset(&h, 0, sizeof(KState));
      h.rho[iters & 1] = 1.0;
      h.alpha = 1.0;
      h.omega = 1.0;
      h.restart_rhr = rr;  // r_hat . r = r . r
      h.res2 = rr;
      h.thr = thr;
      h.iters = iters;
      h.max_iters = stop.max_iters;
      if ((s = push_state(ctx, w))) return s;
    }
    bool first = true;
    while (done == RUN) {
      s = run_polled(ctx, w, iters, stop.check_every, "BiCGSTAB", [&](int64_t k0) -> mxs_status {
        for (int64_t k = k0; k < k0 + stop.check_every; ++k) {
          const int par = (int)(k & 1);
          k_bi_p<<<g, RB, 0, ctx->stream>>>(n, r, p, v, w.pc, g, w.st, par, k, first ? 1 : 0);
          first = false;
          mxs_status e;
          // v = A p with r_hat.v formed by the product when its kernel can
          // (rows from LDS), else a separate reduction
          const double* pv = w.pw;
          int gv = launch_spmv_dot(ctx, A, p, v, &w.st->done, w.pw, rh, 1);
          if (gv == 0) {
            if ((e = launch_spmv(ctx, A, &one, p, &zero, v, &w.st->done))) return e;
            k_bi_rv<<<g, RB, 0, ctx->stream>>>(n, rh, v, w.pa, w.st);
            pv = w.pa;
            gv = g;
          }
          k_bi_s<<<g, RB, 0, ctx->stream>>>(n, r, v, sv, pv, gv, w.pb, w.st, par);
          // t = A s with t.s and t.t formed by the product (the half-step
          // test then moves into k_bi_update), else k_bi_omega forms them
          int gt = launch_spmv_dot(ctx, A, sv, t, &w.st->done, w.pm, nullptr, 2);
          if (gt == 0) {
            if ((e = launch_spmv(ctx, A, &one, sv, &zero, t, &w.st->done))) return e;
            k_bi_omega<<<g, RB, 0, ctx->stream>>>(n, t, sv, w.pb, g, w.pd, w.st, k);
            k_bi_update<<<g, RB, 0, ctx->stream>>>(n, x, p, sv, t, r, rh, w.pd, g, w.pc, w.st,
                                                   k, 0, w.pb, g);
          } else {
            k_bi_update<<<g, RB, 0, ctx->stream>>>(n, x, p, sv, t, r, rh, w.pm, gt, w.pc, w.st,
                                                   k, 1, w.pb, g);
          }
        }
        MXS_HIP_TRY(ctx, hipGetLastError());
        return MXS_OK;
      });
      if (s) return s;
      done = h.done;
      iters = h.iters;
      if (done == ST_HALF) {
        k_bi_half<<<g, RB, 0, ctx->stream>>>(n, x, p, w.st);
        MXS_HIP_TRY(ctx, hipGetLastError());
        done = ST_CONVERGED;
      }
    }
    if (done == ST_BREAKDOWN || done == ST_NONFINITE) {
      s = map_done(done);
      fill_info(info, h, base, relres_true, repl, 0, s);
      return fail(ctx, s, done == ST_BREAKDOWN ? "BiCGSTAB breakdown" : "non-finite value in BiCGSTAB");
    }
    double rt2;
    if ((s = residual(ctx, A, b, x, r))) return s;
    if ((s = dots<double>(ctx, w, n, r, r, (const double*)nullptr, (const double*)nullptr,
                          &rt2, nullptr)))
      return s;
    relres_true = sqrt(rt2) / base;
    h.iters = iters;
    if (done == ST_CONVERGED && sqrt(rt2) <= thr) {
      fill_info(info, h, base, relres_true, repl, 0, MXS_OK);
      return MXS_OK;
    }
    if (done == ST_MAXIT || repl >= stop.max_repl || iters >= stop.max_iters) {
      fill_info(info, h, base, relres_true, repl, 0, MXS_NOT_CONVERGED);
      return fail(ctx, MXS_NOT_CONVERGED, "BiCGSTAB stopped after %lld iterations, relres %.3e",
                  (long long)iters, relres_true);
    }
    repl++;
    rr = rt2;
    done = RUN;
  }
}

// small systems for the one-work-group pipelined CG (see small_pipecg)
bool small_pipe_path(const mxs_matrix* A, const Stop& stop) {
  if (A->fmt != MXS_CSR || A->dt != MXS_F64 || stop.max_repl != 3 || A->n > 4096) return false;
  int64_t maxL = 0;
  for (int64_t i = 0; i < A->n; ++i)
    maxL = std::max<int64_t>(maxL, A->h_rowptr[i + 1] - A->h_rowptr[i]);
  return small_pipecg_fits(A->n, maxL);
}

mxs_status solve_pipecg(mxs_ctx* ctx, const mxs_matrix* A, const double* b, double* x,
                        const Stop& stop, mxs_solve_info* info) {
  const int64_t n = A->n;
  const size_t ld = align_up((size_t)n, 64);
  const bool small = small_pipe_path(A, stop);
  Work w;
  mxs_status s = get_work(
      ctx, 6 * ld * sizeof(double) + (small ? ld * sizeof(double) + small_pipecg_scratch(n) : 0),
      &w);
  if (s) return s;
  double* r = (double*)w.vec;
  double* wv = r + ld;
  double* q = wv + ld;
  double* z = q + ld;
  double* sv = z + ld;
  double* p = sv + ld;
  double nb2, nr2;
  if ((s = residual(ctx, A, b, x, r))) return s;
  if ((s = dots<double>(ctx, w, n, b, b, r, r, &nb2, &nr2))) return s;
  const double nb = sqrt(nb2), nr0 = sqrt(nr2);
  if (!std::isfinite(nb)) return fail(ctx, MXS_NONFINITE, "non-finite right-hand side");
  if (nb == 0.0) return zero_solution(ctx, x, n, info);
  if (!std::isfinite(nr0)) return fail(ctx, MXS_NONFINITE, "non-finite initial residual");
  const double base = stop.baseline == MXS_BASELINE_INITIAL ? (nr0 > 0 ? nr0 : 1.0) : nb;
  const double thr = std::max(stop.rel_tol * base, stop.abs_tol);
  const int g = red_grid(n);
  const double one = 1.0, zero = 0.0;
  KState& h = *w.hst;
  if (small && nr0 > thr) {
    // one work-group runs every iteration: A d = r0 from d = 0, then x += d
    double* d = p + ld;
    SmallCgResult sr;
    if ((s = small_pipecg(ctx, A, r, d, thr / nr0, stop.max_iters, d + ld, &sr))) return s;
    k_add<<<red_grid(n), RB, 0, ctx->stream>>>(n, x, d);
    MXS_HIP_TRY(ctx, hipGetLastError());
    double rt2;
    if ((s = residual(ctx, A, b, x, r))) return s;
    if ((s = dots<double>(ctx, w, n, r, r, (const double*)nullptr, (const double*)nullptr,
                          &rt2, nullptr)))
      return s;
    std::memset(&h, 0, sizeof(KState));
    h.iters = sr.iters;
    h.res2 = sr.res2;
    mxs_status st = sr.status;
    if (st == MXS_OK && !(sqrt(rt2) <= thr)) st = MXS_NOT_CONVERGED;
    fill_info(info, h, base, sqrt(rt2) / base, sr.replacements, 0, st);
    if (st == MXS_OK) return MXS_OK;
    return fail(ctx, st, st == MXS_BREAKDOWN   ? "pipelined CG breakdown: p.Ap <= 0"
                         : st == MXS_NONFINITE ? "non-finite value in pipelined CG"
                                               : "pipelined CG stopped after %lld iterations, relres %.3e",
                (long long)sr.iters, sqrt(rt2) / base);
  }
  std::memset(&h, 0, sizeof(KState));
  h.thr = thr;
  h.max_iters = stop.max_iters;
  h.res2 = nr2;
  // (re)start: w = A r, gamma = r.r and delta = w.r into dot[]
  auto restart = [&]() -> mxs_status {
    mxs_status e = launch_spmv(ctx, A, &one, r, &zero, wv, nullptr);
    if (e) return e;
    double gm, dl;
    if ((e = dots<double>(ctx, w, n, r, r, wv, r, &gm, &dl))) return e;
    h.dot[0] = gm;
    h.dot[1] = dl;
    h.restart_at = h.iters;
    h.done = RUN;
    return push_state(ctx, w);
  };
  int64_t repl = 0;
  double relres_true = nr0 / base;
  if (nr0 <= thr) {
    h.done = ST_CONVERGED;
  } else if ((s = restart())) {
    return s;
  }
  for (;;) {
    if (h.done == RUN) {
      s = run_polled(ctx, w, h.iters, stop.check_every, "pipelined CG",
                     [&](int64_t k0) -> mxs_status {
                       for (int64_t k = k0; k < k0 + stop.check_every; ++k) {
                         double* pin = (k & 1) ? w.pb : w.pa;
                         double* pout = (k & 1) ? w.pa : w.pb;
                         mxs_status e = launch_spmv(ctx, A, &one, wv, &zero, q, &w.st->done);
                         if (e) return e;
                         k_pipe_update<<<g, RB, 0, ctx->stream>>>(n, x, r, wv, q, z, sv, p, pin,
                                                                  g, pout, w.st, k);
                       }
                       MXS_HIP_TRY(ctx, hipGetLastError());
                       return MXS_OK;
                     });
      if (s) return s;
    }
    if (h.done == ST_BREAKDOWN || h.done == ST_NONFINITE) {
      s = map_done(h.done);
      fill_info(info, h, base, relres_true, repl, 0, s);
      return fail(ctx, s, h.done == ST_BREAKDOWN ? "pipelined CG breakdown: p.Ap <= 0"
                                                 : "non-finite value in pipelined CG");
    }
    double rt2;
    if ((s = residual(ctx, A, b, x, r))) return s;
    if ((s = dots<double>(ctx, w, n, r, r, (const double*)nullptr, (const double*)nullptr,
                          &rt2, nullptr)))
      return s;
    relres_true = sqrt(rt2) / base;
    if (h.done == ST_CONVERGED && sqrt(rt2) <= thr) {
      fill_info(info, h, base, relres_true, repl, 0, MXS_OK);
      return MXS_OK;
    }
    if (h.done == ST_MAXIT || repl >= stop.max_repl || h.iters >= stop.max_iters) {
      fill_info(info, h, base, relres_true, repl, 0, MXS_NOT_CONVERGED);
      return fail(ctx, MXS_NOT_CONVERGED,
                  "pipelined CG stopped after %lld iterations, relres %.3e",
                  (long long)h.iters, relres_true);
    }
    // residual replacement: r = b - A x (already in r), restart the recurrences
    repl++;
    h.res2 = rt2;
    if ((s = restart())) return s;
  }
}

mxs_status solve_cgs(mxs_ctx* ctx, const mxs_matrix* A, const double* b, double* x,
                     const Stop& stop, mxs_solve_info* info) {
  const int64_t n = A->n;
  const size_t ld = align_up((size_t)n, 64);
  Work w;
  mxs_status s = get_work(ctx, 7 * ld * sizeof(double), &w);
  if (s) return s;
  double* r = (double*)w.vec;
  double* rh = r + ld;
  double* p = rh + ld;
  double* u = p + ld;
  double* q = u + ld;
  double* v = q + ld;
  double* wv = v + ld;
  double nb2, nr2;
  if ((s = residual(ctx, A, b, x, r))) return s;
  if ((s = dots<double>(ctx, w, n, b, b, r, r, &nb2, &nr2))) return s;
  const double nb = sqrt(nb2), nr0 = sqrt(nr2);
  if (!std::isfinite(nb)) return fail(ctx, MXS_NONFINITE, "non-finite right-hand side");
  if (nb == 0.0) return zero_solution(ctx, x, n, info);
  if (!std::isfinite(nr0)) return fail(ctx, MXS_NONFINITE, "non-finite initial residual");
  const double base = stop.baseline == MXS_BASELINE_INITIAL ? (nr0 > 0 ? nr0 : 1.0) : nb;
  const double thr = std::max(stop.rel_tol * base, stop.abs_tol);
  const int g = red_grid(n);
  const double one = 1.0, zero = 0.0;
  KState& h = *w.hst;
  std::memset(&h, 0, sizeof(KState));
  int64_t repl = 0;
  double relres_true = nr0 / base;
  int32_t done = nr0 <= thr ? ST_CONVERGED : RUN;
  int64_t iters = 0;
  double rr = nr2;
  for (;;) {
    if (done == RUN) {
      // (re)start: r_hat = u = p = r, rho = r_hat . r = r . r
      for (double* dst : {rh, u, p})
        MXS_HIP_TRY(ctx, hipMemcpyAsync(dst, r, n * sizeof(double), hipMemcpyDeviceToDevice,
                                        ctx->stream));
      std::memset(&h, 0, sizeof(KState));
      h.rho[iters & 1] = rr;
      h.res2 = rr;
      h.thr = thr;
      h.iters = iters;
      h.max_iters = stop.max_iters;
      if ((s = push_state(ctx, w))) return s;
    }
    if (done == RUN) {
      s = run_polled(ctx, w, iters, stop.check_every, "CGS", [&](int64_t k0) -> mxs_status {
        for (int64_t k = k0; k < k0 + stop.check_every; ++k) {
          const int par = (int)(k & 1);
          mxs_status e;
          // v = A p with r_hat.v formed by the product when its kernel can
          const double* ps = w.pw;
          int gs = launch_spmv_dot(ctx, A, p, v, &w.st->done, w.pw, rh, 1);
          if (gs == 0) {
            if ((e = launch_spmv(ctx, A, &one, p, &zero, v, &w.st->done))) return e;
            k_cgs_sigma<<<g, RB, 0, ctx->stream>>>(n, rh, v, w.pa, w.st);
            ps = w.pa;
            gs = g;
          }
          k_cgs_qw<<<g, RB, 0, ctx->stream>>>(n, u, v, q, wv, x, ps, gs, w.st, par);
          if ((e = launch_spmv(ctx, A, &one, wv, &zero, v, &w.st->done))) return e;
          k_cgs_r<<<g, RB, 0, ctx->stream>>>(n, r, v, rh, w.pb, w.st);
          k_cgs_dir<<<g, RB, 0, ctx->stream>>>(n, r, q, u, p, w.pb, g, w.st, par, k);
        }
        MXS_HIP_TRY(ctx, hipGetLastError());
        return MXS_OK;
      });
      if (s) return s;
      done = h.done;
      iters = h.iters;
    }
    if (done == ST_BREAKDOWN || done == ST_NONFINITE) {
      s = map_done(done);
      fill_info(info, h, base, relres_true, repl, 0, s);
      return fail(ctx, s, done == ST_BREAKDOWN ? "CGS breakdown" : "non-finite value in CGS");
    }
    double rt2;
    if ((s = residual(ctx, A, b, x, r))) return s;
    if ((s = dots<double>(ctx, w, n, r, r, (const double*)nullptr, (const double*)nullptr,
                          &rt2, nullptr)))
      return s;
    relres_true = sqrt(rt2) / base;
    h.iters = iters;
    if (done == ST_CONVERGED && sqrt(rt2) <= thr) {
      fill_info(info, h, base, relres_true, repl, 0, MXS_OK);
      return MXS_OK;
    }
    if (done == ST_MAXIT || repl >= stop.max_repl || iters >= stop.max_iters) {
      fill_info(info, h, base, relres_true, repl, 0, MXS_NOT_CONVERGED);
      return fail(ctx, MXS_NOT_CONVERGED, "CGS stopped after %lld iterations, relres %.3e",
                  (long long)iters, relres_true);
    }
    repl++;
    rr = rt2;
    done = RUN;
  }
}

// the three Gram-Schmidt passes of step j and their finishing kernels
template <int JB>
void gm_passes_jb(mxs_ctx* ctx, int g, int64_t n, size_t ld, int j, const double* V,
                  double* wv, const Work& w) {
  k_gm_dots<JB><<<g, RB, 0, ctx->stream>>>(n, ld, j, V, wv, w.pm, w.st);
  k_gm_fin<<<1, RB, 0, ctx->stream>>>(w.pm, g, j, 1, w.st);
  k_gm_orth<JB><<<g, RB, 0, ctx->stream>>>(n, ld, j, V, wv, w.pm, w.st);
  k_gm_fin<<<1, RB, 0, ctx->stream>>>(w.pm, g, j, 2, w.st);
  k_gm_norm<JB><<<g, RB, 0, ctx->stream>>>(n, ld, j, V, wv, w.pa, w.st);
  k_gm_fin<<<1, RB, 0, ctx->stream>>>(w.pa, g, j, 3, w.st);
}

void gm_passes(mxs_ctx* ctx, int g, int64_t n, size_t ld, int j, const double* V, double* wv,
               const Work& w) {
  static_assert(MAXM == 32, "buckets of 8, 16 and 32 basis vectors");
  if (j < 8)
    gm_passes_jb<8>(ctx, g, n, ld, j, V, wv, w);
  else if (j < 16)
    gm_passes_jb<16>(ctx, g, n, ld, j, V, wv, w);
  else
    gm_passes_jb<32>(ctx, g, n, ld, j, V, wv, w);
}

mxs_status solve_gmres(mxs_ctx* ctx, const mxs_matrix* A, const double* b, double* x,
                       const Stop& stop, int m, mxs_solve_info* info) {
  if (m < 1 || m > MAXM)
    return fail(ctx, MXS_UNSUPPORTED, "GMRES restart length must be in [1, %d]", MAXM);
  const int64_t n = A->n;
  const size_t ld = align_up((size_t)n, 64);
  Work w;
  mxs_status s = get_work(ctx, (size_t)(m + 3) * ld * sizeof(double), &w);
  if (s) return s;
  double* V = (double*)w.vec;  // m+1 basis vectors
  double* wv = V + (size_t)(m + 1) * ld;
  double* r = wv + ld;
  double nb2, nr2;
  if ((s = residual(ctx, A, b, x, r))) return s;
  if ((s = dots<double>(ctx, w, n, b, b, r, r, &nb2, &nr2))) return s;
  const double nb = sqrt(nb2), nr0 = sqrt(nr2);
  if (!std::isfinite(nb)) return fail(ctx, MXS_NONFINITE, "non-finite right-hand side");
  if (nb == 0.0) return zero_solution(ctx, x, n, info);
  if (!std::isfinite(nr0)) return fail(ctx, MXS_NONFINITE, "non-finite initial residual");
  const double base = stop.baseline == MXS_BASELINE_INITIAL ? (nr0 > 0 ? nr0 : 1.0) : nb;
  const double thr = std::max(stop.rel_tol * base, stop.abs_tol);
  const int g = red_grid(n);
  const double one = 1.0, zero = 0.0;
  KState& h = *w.hst;
  std::memset(&h, 0, sizeof(KState));
  h.thr = thr;
  h.max_iters = stop.max_iters;
  h.m = m;
  h.dot[0] = nr2;
  if ((s = push_state(ctx, w))) return s;
  double beta = nr0;
  int64_t restarts = 0;
  double est = nr0;
  while (beta > thr) {
    if (h.iters >= stop.max_iters) {
      fill_info(info, h, base, beta / base, 0, restarts, MXS_NOT_CONVERGED);
      if (info) info->relres_recurrence = est / base;
      return fail(ctx, MXS_NOT_CONVERGED, "GMRES stopped after %lld steps, relres %.3e",
                  (long long)h.iters, beta / base);
    }
    const int64_t before = h.iters;
    k_gm_reset<<<1, 1, 0, ctx->stream>>>(w.st);
    k_gm_start<<<g, RB, 0, ctx->stream>>>(n, r, V, w.st);
    for (int j = 0; j < m; ++j) {
      double* vj = V + (size_t)j * ld;
      if ((s = launch_spmv(ctx, A, &one, vj, &zero, wv, &w.st->cycle))) return s;
      gm_passes(ctx, g, n, ld, j, V, wv, w);
      k_gm_scale<<<g, RB, 0, ctx->stream>>>(n, wv, V + (size_t)(j + 1) * ld, w.st);
    }
    k_gm_backsolve<<<1, RB, 0, ctx->stream>>>(w.st);
    k_gm_xupdate<<<g, RB, 0, ctx->stream>>>(n, ld, V, x, w.st);
    MXS_HIP_TRY(ctx, hipGetLastError());
    if ((s = residual(ctx, A, b, x, r))) return s;
    enqueue_dots<double>(ctx, w, n, r, r, nullptr, nullptr);
    if ((s = pull_state(ctx, w))) return s;
    if (h.done == ST_BREAKDOWN || h.done == ST_NONFINITE) {
      s = map_done(h.done);
      fill_info(info, h, base, beta / base, 0, restarts, s);
      return fail(ctx, s, "GMRES %s", h.done == ST_BREAKDOWN ? "breakdown" : "non-finite value");
    }
    if (h.iters <= before)
      return fail(ctx, MXS_HIP, "GMRES made no progress (device state not updated)");
    est = h.est;
    beta = sqrt(h.dot[0]);
    if (!std::isfinite(beta)) return fail(ctx, MXS_NONFINITE, "non-finite GMRES residual");
    if (beta <= thr) break;
    restarts++;
  }
  fill_info(info, h, base, beta / base, 0, restarts, MXS_OK);
  if (info) info->relres_recurrence = est / base;
  return MXS_OK;
}

}  // namespace

// exported for the iterative refinement driver below
mxs_status solve_dispatch(mxs_ctx* ctx, mxs_solver kind, const mxs_matrix* A, const double* b,
                          double* x, const mxs_stop* stop, const mxs_solver_opts* opts,
                          mxs_solve_info* info) {
  if (opts && opts->precond && kind != MXS_CG)
    return fail(ctx, MXS_UNSUPPORTED, "preconditioning is implemented for CG only");
  switch (kind) {
    case MXS_CG:
      if (opts && opts->precond) {
        const mxs_precond* M = opts->precond;
        if (M->n != A->n) return fail(ctx, MXS_INVALID_ARG, "preconditioner size differs");
        return solve_pcg(ctx, A, M, b, x, read_stop(stop, 20000), info);
      }
      return solve_cg(ctx, A, b, x, read_stop(stop, 20000), info);
    case MXS_BICGSTAB:
      return solve_bicgstab(ctx, A, b, x, read_stop(stop, 10000), info);
    case MXS_CGS:
      return solve_cgs(ctx, A, b, x, read_stop(stop, 10000), info);
    case MXS_PIPECG:
      return solve_pipecg(ctx, A, b, x, read_stop(stop, 20000), info);
    case MXS_GMRES:
      return solve_gmres(ctx, A, b, x, read_stop(stop, 20000),
                         opts && opts->restart > 0 ? opts->restart : 30, info);
  }
  return fail(ctx, MXS_INVALID_ARG, "unknown solver %d", (int)kind);
}

mxs_status solve_ir_impl(mxs_ctx* ctx, const mxs_matrix* A64, const mxs_matrix* Al,
                         const double* b, double* x, const mxs_stop* outer, double inner_tol,
                         int64_t inner_max, int variant, const mxs_precond* M,
                         mxs_ir_info* info) {
  const int64_t n = A64->n;
  const size_t ld = align_up((size_t)n, 64);
  Work w;
  mxs_status s = get_work(ctx, ld * sizeof(double) + 5 * ld * sizeof(float), &w);
  if (s) return s;
  double* r = (double*)w.vec;
  float* d = (float*)(r + ld);
  float* rf = d + ld;
  float* pf = rf + ld;
  float* qf = pf + ld;
  float* zf = qf + ld;
  const Stop st = read_stop(outer, 50);
  const int64_t outer_max = st.max_iters;
  const double tol = st.rel_tol;
  if (inner_max <= 0) inner_max = 20000;
  double nb2;
  if ((s = dots<double>(ctx, w, n, b, b, nullptr, nullptr, &nb2, nullptr))) return s;
  const double nb = sqrt(nb2);
  mxs_ir_info out{};
  if (!std::isfinite(nb)) return fail(ctx, MXS_NONFINITE, "non-finite right-hand side");
  if (nb == 0.0) {
    MXS_HIP_TRY(ctx, hipMemsetAsync(x, 0, n * sizeof(double), ctx->stream));
    MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (info) *info = out;
    return MXS_OK;
  }
  const int g = red_grid(n);
  KState& h = *w.hst;
  mxs_status result = MXS_OK;
  const bool last_step = (variant & MXS_IR_LAST_STEP) != 0;
  const bool carry = (variant & MXS_IR_CARRY_DIRECTION) != 0;
  // what the carried direction needs from the previous inner solve: its
  // residual norm sigma, its last rho = r_k.z_k, the reduction its
  // recurrence residual claimed, and whether it took a step without
  // breaking down (pf then still holds its last direction p_k)
  double nr_prev = 0.0, rho_prev = 0.0, claimed = 0.0;
  bool usable = false;
  for (;;) {
    double nr2;
    if ((s = residual(ctx, A64, b, x, r))) return s;
    if ((s = dots<double>(ctx, w, n, r, r, nullptr, nullptr, &nr2, nullptr))) return s;
    const double nr = sqrt(nr2), relres = nr / nb;
    out.relres_true = relres;
    if (!std::isfinite(nr)) {
      result = fail(ctx, MXS_NONFINITE, "non-finite residual in refinement");
      break;
    }
    if (relres <= tol) break;
    if (out.outer_iters >= outer_max) {
      result = fail(ctx, MXS_NOT_CONVERGED, "refinement stopped after %lld outer steps",
                    (long long)out.outer_iters);
      break;
    }
    double itol = inner_tol;
    if (last_step && relres * inner_tol <= tol) itol = std::max(itol, 0.1 * tol / relres);
    // inner FP32 CG from d = 0 on A_low d = f, f = r / ||r||
    k_ir_scale<<<g, RB, 0, ctx->stream>>>(n, r, nr, rf);
    MXS_HIP_TRY(ctx, hipMemsetAsync(d, 0, n * sizeof(float), ctx->stream));
    double f2, rz;
    // z = M^{-1} f (z = f without a preconditioner), rho = f.z
    const float* z0 = rf;
    if (M) {
      apply_precond<float>(ctx, M, M->m32, n, rf, zf);
      if ((s = dots<float>(ctx, w, n, rf, rf, rf, zf, &f2, &rz))) return s;
      z0 = zf;
    } else {
      if ((s = dots<float>(ctx, w, n, rf, rf, nullptr, nullptr, &f2, nullptr))) return s;
      rz = f2;
    }
    // Carried direction: the previous solve's quantities, normalised by
    // nr_prev, grow by sc = nr_prev / nr against f (p_k -> sc p_k,
    // rho_k -> sc^2 rho_k), so the CG direction is z + beta sc p_k with
    // beta = rz / (sc^2 rho_k), i.e. z + cc p_k.  It is carried only while
    // the FP64 residual followed the recurrence the direction was built for:
    // a true reduction nr / nr_prev more than twice the recurrence's own
    // means A_low is too far from A64 for its directions to serve this step.
    const float cc = carry && usable ? (float)(rz / ((nr_prev / nr) * rho_prev)) : 0.0f;
    if (carry && usable && nr <= 2.0 * claimed * nr_prev && std::isfinite(cc)) {
      k_ir_carry<<<g, RB, 0, ctx->stream>>>(n, z0, pf, cc);
    } else {
      MXS_HIP_TRY(ctx, hipMemcpyAsync(pf, z0, n * sizeof(float), hipMemcpyDeviceToDevice,
                                      ctx->stream));
    }
    std::memset(&h, 0, sizeof(KState));
    h.rho[0] = rz;
    h.res2 = f2;
    h.thr = itol * sqrt(f2);
    h.max_iters = inner_max;
    h.done = f2 == 0.0 ? ST_CONVERGED : rz > 0.0 ? RUN : ST_BREAKDOWN;
    if ((s = push_state(ctx, w))) return s;
    if (h.done == RUN) {
      if (M)
        s = pcg_run<float>(ctx, Al, M, M->m32, w, d, rf, pf, qf, zf, st.check_every);
      else
        s = cg_loop<float>(ctx, Al, w, d, rf, pf, qf, st.check_every);
      if (s) return s;
    }
    out.inner_iters_total += h.iters;
    // the inner kernels leave p_k in pf and rho_k in rho[k & 1] when the
    // tolerance or the step cap stops iteration k
    usable = h.iters > 0 && (h.done == ST_CONVERGED || h.done == ST_MAXIT) &&
             h.rho[(h.iters - 1) & 1] > 0.0;
    rho_prev = usable ? h.rho[(h.iters - 1) & 1] : 0.0;
    claimed = f2 > 0.0 ? sqrt(h.res2 / f2) : 0.0;
    nr_prev = nr;
    if (h.done == ST_NONFINITE) {
      result = fail(ctx, MXS_NONFINITE, "non-finite value in the inner solve");
      break;
    }
    // a breakdown or max_iters in the inner solve still yields a usable
    // correction; the FP64 residual decides
    k_ir_update<<<g, RB, 0, ctx->stream>>>(n, x, d, nr);
    MXS_HIP_TRY(ctx, hipGetLastError());
    out.outer_iters++;
  }
  out.status = result;
  if (info) *info = out;
  return result;
}

}  // namespace mxs

using namespace mxs;

extern "C" {

mxs_status mxs_solve(mxs_ctx* ctx, mxs_solver kind, const mxs_matrix* A, const double* b,
                     double* x, const mxs_stop* stop, const mxs_solver_opts* opts,
                     mxs_solve_info* info) {
  if (!ctx || !A) return MXS_INVALID_ARG;
  if (A->dt != MXS_F64)
    return fail(ctx, MXS_UNSUPPORTED, "mxs_solve needs an F64 matrix (use mxs_solve_ir)");
  if (A->n != A->ncols) return fail(ctx, MXS_INVALID_ARG, "matrix is not square");
  if (A->n > 0 && (!b || !x)) return fail(ctx, MXS_INVALID_ARG, "NULL vector");
  if (info) std::memset(info, 0, sizeof(*info));
  if (A->n == 0) return MXS_OK;
  MXS_HIP_TRY(ctx, hipSetDevice(ctx->device));
  return solve_dispatch(ctx, kind, A, b, x, stop, opts, info);
}

mxs_status mxs_solve_ir(mxs_ctx* ctx, const mxs_matrix* A64, const mxs_matrix* A_low,
                        const double* b, double* x, const mxs_stop* outer,
                        double inner_rel_tol, int64_t inner_max, int32_t variant,
                        const mxs_precond* inner_precond, mxs_ir_info* info) {
  if (!ctx || !A64 || !A_low) return MXS_INVALID_ARG;
  if (A64->dt != MXS_F64 || (A_low->dt != MXS_F32 && A_low->dt != MXS_F16_ROWSCALED))
    return fail(ctx, MXS_UNSUPPORTED, "need an F64 matrix and an F32 or F16_ROWSCALED copy");
  if (A64->n != A64->ncols || A_low->n != A64->n || A_low->ncols != A64->ncols)
    return fail(ctx, MXS_INVALID_ARG, "matrix shapes differ or are not square");
  if (A64->n > 0 && (!b || !x)) return fail(ctx, MXS_INVALID_ARG, "NULL vector");
  if (info) std::memset(info, 0, sizeof(*info));
  if (A64->n == 0) return MXS_OK;
  if (!(inner_rel_tol > 0.0 && inner_rel_tol < 1.0))
    return fail(ctx, MXS_INVALID_ARG, "inner tolerance must be in (0, 1)");
  MXS_HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (inner_precond && inner_precond->n != A64->n)
    return fail(ctx, MXS_INVALID_ARG, "preconditioner size differs");
  return solve_ir_impl(ctx, A64, A_low, b, x, outer, inner_rel_tol, inner_max,
                       variant, inner_precond, info);
}

mxs_status mxs_graph_create(mxs_ctx* ctx, int64_t n, int64_t nnz, const int32_t* rowptr,
                            const int32_t* col, int32_t flags, mxs_graph** out) {
  if (!ctx || !out) return MXS_INVALID_ARG;
  if (flags != MXS_HOST_PTRS && flags != MXS_DEVICE_PTRS)
    return fail(ctx, MXS_INVALID_ARG, "unknown flags %d", flags);
  MXS_HIP_TRY(ctx, hipSetDevice(ctx->device));
  mxs_graph* G = new (std::nothrow) mxs_graph();
  if (!G) return MXS_OOM;
  G->device = ctx->device;
  G->alloc = ctx->alloc;
  G->n = n;
  G->nnz = nnz;
  // the pattern is validated by the CSR constructor (rows ascending,
  // sources in range, sorted and distinct) before any index is used
  mxs_status st = create_csr(ctx, n, n, nnz, rowptr, col, nullptr, flags, &G->T);
  if (st) {
    delete G;
    return st;
  }
  int32_t* d = (int32_t*)G->alloc.alloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  G->dangling = (uint8_t*)G->alloc.alloc((size_t)(n > 0 ? n : 1));
  std::vector<int32_t> hd((size_t)n);
  do {
    if (!d || !G->dangling) {
      st = fail(ctx, MXS_OOM, "graph set-up");
      break;
    }
    if (n == 0) break;
    if (hipMemsetAsync(d, 0, n * sizeof(int32_t), ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "memset failed");
      break;
    }
    const unsigned ge = (unsigned)std::min<int64_t>((nnz + 255) / 256 + 1, 65536);
    k_outdeg<<<ge, 256, 0, ctx->stream>>>(nnz, G->T->csr.col, d);
    k_transition<<<ge, 256, 0, ctx->stream>>>(nnz, G->T->csr.col, d, (double*)G->T->csr.val);
    if ((st = refresh_panel_values(ctx, G->T))) break;
    k_dangling<<<(unsigned)((n + 255) / 256), 256, 0, ctx->stream>>>(n, d, G->dangling);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(hd.data(), d, n * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream) !=
            hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "graph set-up kernels failed");
      break;
    }
    for (int32_t v : hd) G->ndangling += v == 0;
  } while (0);
  G->alloc.release(d);
  if (st) {
    mxs_graph_destroy(G);
    return st;
  }
  *out = G;
  return MXS_OK;
}

mxs_status mxs_graph_destroy(mxs_graph* G) {
  if (!G) return MXS_OK;
  (void)hipSetDevice(G->device);
  if (G->T) mxs_matrix_destroy(G->T);
  G->alloc.release(G->dangling);
  delete G;
  return MXS_OK;
}

const mxs_matrix* mxs_graph_transition(const mxs_graph* G) { return G ? G->T : nullptr; }

mxs_status mxs_pagerank(mxs_ctx* ctx, const mxs_graph* G, const mxs_matrix* op, double damping,
                        double tol, int64_t max_iters, double* x, mxs_pagerank_info* info) {
  if (!ctx || !G || (G->n > 0 && !x)) return MXS_INVALID_ARG;
  if (info) std::memset(info, 0, sizeof(*info));
  if (!(damping >= 0.0 && damping < 1.0))
    return fail(ctx, MXS_INVALID_ARG, "damping must lie in [0, 1)");
  if (!(tol >= 0.0)) return fail(ctx, MXS_INVALID_ARG, "negative tolerance");
  const mxs_matrix* T = op ? op : G->T;
  if (T->n != G->n || T->ncols != G->n || T->dt != MXS_F64)
    return fail(ctx, MXS_INVALID_ARG, "the operator must be the graph's F64 transition matrix");
  const int64_t n = G->n;
  if (n == 0) return MXS_OK;
  MXS_HIP_TRY(ctx, hipSetDevice(ctx->device));
  Work w;
  mxs_status s = get_work(ctx, align_up((size_t)n, 64) * sizeof(double), &w);
  if (s) return s;
  double* z = (double*)w.vec;
  const int g = red_grid(n);
  KState& h = *w.hst;
  std::memset(&h, 0, sizeof(KState));
  h.thr = tol;
  h.max_iters = max_iters > 0 ? max_iters : 1000;
  if ((s = push_state(ctx, w))) return s;
  k_pr_init<<<g, RB, 0, ctx->stream>>>(n, x, G->dangling, w.pa);
  const double one = 1.0, zero = 0.0;
  int64_t k = 0;
  const int check_every = 16;
  while (h.done == RUN) {
    const int64_t before = k;
    for (int it = 0; it < check_every; ++it, ++k) {
      double* pin = (k & 1) ? w.pb : w.pa;
      double* pout = (k & 1) ? w.pa : w.pb;
      if ((s = launch_spmv(ctx, T, &one, x, &zero, z, &w.st->done))) return s;
      k_pr_update<<<g, RB, 0, ctx->stream>>>(n, x, z, G->dangling, damping, pin, g, pout, w.st,
                                             k);
    }
    MXS_HIP_TRY(ctx, hipGetLastError());
    if ((s = pull_state(ctx, w))) return s;
    if (h.done == RUN && h.iters <= before)
      return fail(ctx, MXS_HIP, "PageRank made no progress (device state not updated)");
    k = h.iters;
  }
  const mxs_status res = h.done == ST_CONVERGED ? MXS_OK
                         : h.done == ST_MAXIT   ? MXS_NOT_CONVERGED
                                                : MXS_NONFINITE;
  if (info) {
    info->iters = h.iters;
    info->delta = h.res2;
    info->status = res;
  }
  if (res == MXS_NOT_CONVERGED)
    return fail(ctx, res, "PageRank stopped after %lld iterations, L1 change %.3e",
                (long long)h.iters, h.res2);
  if (res == MXS_NONFINITE) return fail(ctx, res, "non-finite value in PageRank");
  return MXS_OK;
}

}  // extern "C"
