// precond.hip -- Jacobi and block-Jacobi preconditioners (set-up and the
// C entry points); their application lives with the solvers.
//
// Jacobi: M = diag(A), stored as 1/a_ii (FP64, and rounded to FP32 for the
// FP32 inner solves of iterative refinement).  Block Jacobi: M = the dense
// diagonal blocks A[I,I] over consecutive row ranges of `bs` rows (the last
// one ragged), stored inverted, column-major in bs x bs slots.  Both follow
// the stationary preconditioners of Saad 2003, ch. 10; Ginkgo's block
// Jacobi, which the paper lists among the library's preconditioners, finds
// block boundaries from the sparsity pattern instead (not done here).
#include <cmath>
#include <cstring>
#include <new>

#include "common.h"

namespace mxs {
namespace {

constexpr int kMaxBs = 32;

// thread per row; the columns of a row are sorted, so the diagonal entry
// is found by binary search
__global__ __launch_bounds__(256) void k_jacobi_setup(int64_t n, const int32_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col,
                                                      const double* __restrict__ val,
                                                      double* __restrict__ m64,
                                                      float* __restrict__ m32,
                                                      int32_t* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t lo = rp[i], hi = rp[i + 1];
  double d = 0.0;
  while (lo < hi) {
    const int32_t mid = lo + (hi - lo) / 2;
    const int32_t c = col[mid];
    if (c == i) {
      d = val[mid];
      break;
    }
    if (c < i)
      lo = mid + 1;
    else
      hi = mid;
  }
  if (d == 0.0 || !isfinite(d)) *bad = 1;
  const double inv = 1.0 / d;
  m64[i] = inv;
  m32[i] = (float)inv;
}

// One wave per diagonal block: the block and an identity are assembled in
// LDS as [A_II | I] and reduced by Gauss-Jordan elimination with partial
// pivoting (largest magnitude, first on ties); lane t owns column t of the
// augmented matrix.  The inverse is written column-major, zero-padded.
__global__ __launch_bounds__(64) void k_bj_setup(int64_t n, int bs, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col,
                                                 const double* __restrict__ val,
                                                 double* __restrict__ m64,
                                                 float* __restrict__ m32,
                                                 int32_t* __restrict__ bad) {
  __shared__ double aug[kMaxBs][2 * kMaxBs + 1];
  __shared__ double fcol[kMaxBs];
  __shared__ int piv_s;
  const int lane = threadIdx.x;
  const int64_t blk = blockIdx.x;
  const int64_t r0 = blk * bs;
  const int m = (int)((n - r0) < bs ? (n - r0) : bs);
  for (int t = lane; t < kMaxBs * (2 * kMaxBs + 1); t += 64) (&aug[0][0])[t] = 0.0;
  __syncthreads();
  if (lane < m) aug[lane][m + lane] = 1.0;
  for (int i = 0; i < m; ++i)
    for (int32_t k = rp[r0 + i] + lane; k < rp[r0 + i + 1]; k += 64) {
      const int64_t c = (int64_t)col[k] - r0;
      if (c >= 0 && c < m) aug[i][c] = val[k];
    }
  __syncthreads();
  bool singular = false;
  for (int c = 0; c < m; ++c) {
    if (lane == 0) {
      int p = c;
      for (int i = c + 1; i < m; ++i)
        if (fabs(aug[i][c]) > fabs(aug[p][c])) p = i;
      piv_s = p;
    }
    __syncthreads();
    const int p = piv_s;
    const double pv = aug[p][c];  // the same value in every lane
    if (pv == 0.0 || !isfinite(pv)) {
      singular = true;
      break;
    }
    if (p != c && lane < 2 * m) {
      const double t = aug[c][lane];
      aug[c][lane] = aug[p][lane];
      aug[p][lane] = t;
    }
    __syncthreads();
    if (lane < 2 * m) aug[c][lane] /= pv;
    if (lane < m) fcol[lane] = aug[lane][c];
    __syncthreads();
    if (lane < 2 * m) {
      const double pr = aug[c][lane];
      for (int r = 0; r < m; ++r)
        if (r != c) aug[r][lane] -= fcol[r] * pr;
    }
    __syncthreads();
  }
  if (singular) {
    if (lane == 0) *bad = 1;
    return;
  }
  double* M = m64 + blk * bs * bs;
  float* M32 = m32 + blk * bs * bs;
  for (int t = lane; t < bs * bs; t += 64) {
    const int j = t / bs, i = t - j * bs;
    const double v = (i < m && j < m) ? aug[i][m + j] : 0.0;
    if (!isfinite(v)) *bad = 1;
    M[t] = v;
    M32[t] = (float)v;
  }
}

}  // namespace
}  // namespace mxs

using namespace mxs;

extern "C" {

mxs_status mxs_precond_create(mxs_ctx* ctx, const mxs_matrix* A, int32_t kind,
                              int32_t block_size, mxs_precond** out) {
  if (!ctx || !A || !out) return MXS_INVALID_ARG;
  if (A->fmt != MXS_CSR || A->dt != MXS_F64)
    return fail(ctx, MXS_UNSUPPORTED, "a preconditioner is built from an F64 CSR matrix");
  if (A->n != A->ncols) return fail(ctx, MXS_INVALID_ARG, "matrix is not square");
  int bs = 1;
  if (kind == MXS_PRECOND_BLOCK_JACOBI) {
    if (block_size < 1 || block_size > kMaxBs)
      return fail(ctx, MXS_INVALID_ARG, "block size must be in [1, %d]", kMaxBs);
    bs = block_size;
  } else if (kind != MXS_PRECOND_JACOBI) {
    return fail(ctx, MXS_INVALID_ARG, "unknown preconditioner %d", (int)kind);
  }
  MXS_HIP_TRY(ctx, hipSetDevice(ctx->device));
  mxs_precond* M = new (std::nothrow) mxs_precond();
  if (!M) return MXS_OOM;
  M->device = ctx->device;
  M->alloc = ctx->alloc;
  M->kind = kind;
  M->n = A->n;
  M->bs = bs;
  M->nb = (A->n + bs - 1) / bs;
  const int64_t count = kind == MXS_PRECOND_JACOBI ? A->n : M->nb * bs * bs;
  M->count = count;
  M->m64 = (double*)M->alloc.alloc((size_t)(count > 0 ? count : 1) * sizeof(double));
  M->m32 = (float*)M->alloc.alloc((size_t)(count > 0 ? count : 1) * sizeof(float));
  int32_t* d_bad = (int32_t*)M->alloc.alloc(sizeof(int32_t));
  if (!M->m64 || !M->m32 || !d_bad) {
    M->alloc.release(d_bad);
    mxs_precond_destroy(M);
    return fail(ctx, MXS_OOM, "preconditioner storage");
  }
  mxs_status st = MXS_OK;
  int32_t bad = 0;
  do {
    if (hipMemsetAsync(d_bad, 0, sizeof(int32_t), ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "memset failed");
      break;
    }
    if (A->n > 0) {
      if (kind == MXS_PRECOND_JACOBI)
        k_jacobi_setup<<<(unsigned)((A->n + 255) / 256), 256, 0, ctx->stream>>>(
            A->n, A->csr.rowptr, A->csr.col, (const double*)A->csr.val, M->m64, M->m32, d_bad);
      else
        k_bj_setup<<<(unsigned)M->nb, 64, 0, ctx->stream>>>(
            A->n, bs, A->csr.rowptr, A->csr.col, (const double*)A->csr.val, M->m64, M->m32,
            d_bad);
    }
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream) !=
            hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
      st = fail(ctx, MXS_HIP, "preconditioner set-up failed");
      break;
    }
    if (bad)
      st = fail(ctx, MXS_BREAKDOWN,
                kind == MXS_PRECOND_JACOBI ? "zero, missing or non-finite diagonal entry"
                                           : "singular or non-finite diagonal block");
  } while (0);
  M->alloc.release(d_bad);
  if (st) {
    mxs_precond_destroy(M);
    return st;
  }
  *out = M;
  return MXS_OK;
}

mxs_status mxs_precond_destroy(mxs_precond* M) {
  if (!M) return MXS_OK;
  (void)hipSetDevice(M->device);
  M->alloc.release(M->m64);
  M->alloc.release(M->m32);
  delete M;
  return MXS_OK;
}

mxs_status mxs_precond_export(mxs_ctx* ctx, const mxs_precond* M, double* host, size_t bytes) {
  if (!ctx || !M || !host) return MXS_INVALID_ARG;
  if (bytes < (size_t)M->count * sizeof(double))
    return fail(ctx, MXS_INVALID_ARG, "export buffer of %zu bytes, need %zu", bytes,
                (size_t)M->count * sizeof(double));
  MXS_HIP_TRY(ctx, hipSetDevice(ctx->device));
  MXS_HIP_TRY(ctx, hipMemcpyAsync(host, M->m64, (size_t)M->count * sizeof(double),
                                  hipMemcpyDeviceToHost, ctx->stream));
  MXS_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MXS_OK;
}

}  // extern "C"
