/*
 * oracle.c -- CPU oracle (TEST INFRASTRUCTURE ONLY; see oracle.h).
 *
 * What it computes, and where each definition comes from:
 *
 *  - CSR and COO storage and the sparse matrix-vector product y = A x are
 *    the ones the paper uses in its section "Central Sparse Linear Algebra
 *    Functionality": COO keeps (row, column, value) for every stored entry,
 *    CSR replaces the row indices of a row-sorted COO matrix by pointers to
 *    the first entry of each row.  The product and its scaled form
 *    y = alpha*A*x + beta*y follow the BLAS convention that beta == 0 does
 *    not read y.
 *  - ELL is only named by the paper (its preamble defines the macro); the
 *    padded column-major layout used here is the standard one of Williams et
 *    al., the SpMV survey the paper cites.  Hybrid ELL+COO is not in the paper
 *    at all; its split width follows the byte-count model of the paper's
 *    "SpMV Performance Analysis" subsection (value + index bytes per ELL slot
 *    against value + two index bytes per COO entry).
 *  - CG, BiCGSTAB and GMRES are the Krylov solvers of the same section; the
 *    paper gives no algorithm text and refers to Saad's book (2nd ed., 2003)
 *    and to Saad & Schultz (1986) for GMRES.  The textbook forms are written
 *    out below in that notation.
 *  - Row sums are accumulated with the compensated dot product of Ogita,
 *    Rump & Oishi ("Accurate sum and dot product", 2005) and rounded once,
 *    so the oracle's own error is about one unit in the last place and the
 *    per-entry tolerance of a GPU comparison measures the GPU alone.
 *  - Mixed-precision iterative refinement is not in the paper; it is the
 *    classical scheme (residual and update in FP64, correction solved in
 *    FP32) with the inner solver being the CG below run in float.  Its
 *    carried-direction form keeps the inner CG's search direction from one
 *    refinement step to the next: the FP64 residual then replaces the FP32
 *    recurrence residual inside one continuing CG, the residual replacement
 *    of van der Vorst & Ye (SIAM J. Sci. Comput. 22, 2000) used with a
 *    low-precision iteration as in the "reliable updates" of Clark et al.
 *    (Comput. Phys. Commun. 181, 2010).
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Timing builds only (-fopenmp, the host baseline): row loops and vector
 * updates split over threads give the same results as the single thread
 * (each entry is computed alone); the solvers' inner products are summed in
 * a different order there.  The parity build has no OpenMP and these are
 * empty. */
#ifdef _OPENMP
#define ORC_PAR_FOR _Pragma("omp parallel for schedule(static)")
#define ORC_PAR_SUM_S _Pragma("omp parallel for schedule(static) reduction(+:s)")
#else
#define ORC_PAR_FOR
#define ORC_PAR_SUM_S
#endif

/* ------------------------------------------------------------------------ */
/* compensated accumulation (Ogita-Rump-Oishi Dot2)                         */
/* ------------------------------------------------------------------------ */
typedef struct {
  double s;     /* running sum                              */
  double c;     /* accumulated rounding errors              */
  double naive; /* plain sum, used when a term is not finite */
} acc_t;

static void acc_init(acc_t* a, double start) {
  a->s = start;
  a->c = 0.0;
  a->naive = start;
}

static void acc_add(acc_t* a, double u, double v) {
  double h = u * v;
  double r = fma(u, v, -h); /* exact error of the product */
  double s = a->s + h;
  double z = s - a->s;
  double q = (a->s - (s - z)) + (h - z); /* exact error of the sum */
  a->s = s;
  a->c = a->c + (q + r);
  a->naive = a->naive + h;
}

static double acc_result(const acc_t* a) {
  double res = a->s + a->c;
  if (!isfinite(a->naive) || !isfinite(res)) return a->naive;
  return res;
}

static double scale_out(double alpha, double s, double beta, double yold) {
  if (beta == 0.0) return alpha * s;
  return alpha * s + beta * yold;
}

/* ------------------------------------------------------------------------ */
/* ingest                                                                   */
/* ------------------------------------------------------------------------ */
int orc_csr_validate(int64_t n, int64_t ncols, int64_t nnz,
                     const int32_t* rowptr, const int32_t* col) {
  if (n < 0 || ncols < 0 || nnz < 0) return ORC_INVALID_ARG;
  if (n > INT32_MAX || ncols > INT32_MAX || nnz > INT32_MAX)
    return ORC_UNSUPPORTED;
  if (rowptr[0] != 0 || (int64_t)rowptr[n] != nnz) return ORC_INVALID_MATRIX;
  for (int64_t i = 0; i < n; ++i) {
    if (rowptr[i + 1] < rowptr[i]) return ORC_INVALID_MATRIX;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      if (col[k] < 0 || (int64_t)col[k] >= ncols) return ORC_INVALID_MATRIX;
      if (k > rowptr[i] && col[k] <= col[k - 1]) return ORC_INVALID_MATRIX;
    }
  }
  return ORC_OK;
}

/* Ingest of a row-grouped coordinate list whose columns may be unordered or
 * repeated within a row (paper, "Central Sparse Linear Algebra
 * Functionality": CSR is the row-sorted coordinate list compressed by row
 * pointers; an entry listed twice stands for the sum of its values).  Each
 * row's entries are ordered by column with ties kept in input order (a
 * sort whose key is the pair (column, position in the row), so it is
 * stable by construction), and each run of equal columns becomes one entry
 * whose value is the run's values added left to right, i.e. in input
 * order: ((v0 + v1) + v2) + ...  A run that sums to zero stays as an
 * explicit zero.  Row pointers and column range are checked as in
 * orc_csr_validate (order and repeats are what this routine repairs).
 * vpe = doubles per value (1 real, 2 complex as (re, im), parts summed
 * separately).  Outputs: rowptr_out[n+1], col_out / val_out with room for
 * nnz entries; *nnz_out = entries kept. */
typedef struct {
  int32_t col;
  int64_t pos;
} orc_key;

static int orc_key_cmp(const void* a, const void* b) {
  const orc_key* x = (const orc_key*)a;
  const orc_key* y = (const orc_key*)b;
  if (x->col != y->col) return x->col < y->col ? -1 : 1;
  return x->pos < y->pos ? -1 : (x->pos > y->pos ? 1 : 0);
}

int orc_csr_sort_and_sum(int64_t n, int64_t ncols, int64_t nnz,
                         const int32_t* rowptr, const int32_t* col,
                         const double* val, int vpe, int32_t* rowptr_out,
                         int32_t* col_out, double* val_out, int64_t* nnz_out) {
  if (n < 0 || ncols < 0 || nnz < 0 || (vpe != 1 && vpe != 2)) return ORC_INVALID_ARG;
  if (n > INT32_MAX || ncols > INT32_MAX || nnz > INT32_MAX) return ORC_UNSUPPORTED;
  if (rowptr[0] != 0 || (int64_t)rowptr[n] != nnz) return ORC_INVALID_MATRIX;
  for (int64_t i = 0; i < n; ++i) {
    if (rowptr[i + 1] < rowptr[i]) return ORC_INVALID_MATRIX;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
      if (col[k] < 0 || (int64_t)col[k] >= ncols) return ORC_INVALID_MATRIX;
  }
  int64_t maxlen = 0;
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] - rowptr[i] > maxlen) maxlen = rowptr[i + 1] - rowptr[i];
  orc_key* keys = (orc_key*)malloc((size_t)(maxlen > 0 ? maxlen : 1) * sizeof(orc_key));
  if (!keys) return ORC_INVALID_ARG;
  int64_t out = 0;
  rowptr_out[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t s = rowptr[i], L = rowptr[i + 1] - rowptr[i];
    for (int64_t t = 0; t < L; ++t) {
      keys[t].col = col[s + t];
      keys[t].pos = t;
    }
    qsort(keys, (size_t)L, sizeof(orc_key), orc_key_cmp);
    int64_t t = 0;
    while (t < L) {
      const int32_t c = keys[t].col;
      for (int q = 0; q < vpe; ++q) {
        double sum = val[(s + keys[t].pos) * vpe + q];
        for (int64_t u = t + 1; u < L && keys[u].col == c; ++u)
          sum = sum + val[(s + keys[u].pos) * vpe + q];
        val_out[out * vpe + q] = sum;
      }
      col_out[out] = c;
      ++out;
      while (t < L && keys[t].col == c) ++t;
    }
    rowptr_out[i + 1] = (int32_t)out;
  }
  free(keys);
  *nnz_out = out;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* conversions                                                              */
/* ------------------------------------------------------------------------ */
void orc_csr_to_coo(int64_t n, const int32_t* rowptr, int32_t* row_out) {
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) row_out[k] = (int32_t)i;
}

void orc_coo_to_csr(int64_t n, int64_t nnz, const int32_t* row,
                    int32_t* rowptr_out) {
  for (int64_t i = 0; i <= n; ++i) rowptr_out[i] = 0;
  for (int64_t k = 0; k < nnz; ++k) rowptr_out[row[k] + 1] += 1;
  for (int64_t i = 0; i < n; ++i) rowptr_out[i + 1] += rowptr_out[i];
}

int64_t orc_ell_width(int64_t n, const int32_t* rowptr) {
  int64_t K = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t L = rowptr[i + 1] - rowptr[i];
    if (L > K) K = L;
  }
  return K;
}

int64_t orc_ell_stride(int64_t n) { return (n + 63) / 64 * 64; }

void orc_csr_to_ell(int64_t n, const int32_t* rowptr, const int32_t* col,
                    const double* val, int64_t K, int64_t stride,
                    int32_t* ecol, double* eval) {
  for (int64_t j = 0; j < K; ++j)
    for (int64_t i = 0; i < stride; ++i) {
      int64_t slot = j * stride + i;
      int64_t L = (i < n) ? (int64_t)(rowptr[i + 1] - rowptr[i]) : 0;
      if (j < L) {
        ecol[slot] = col[rowptr[i] + j];
        eval[slot] = val[rowptr[i] + j];
      } else {
        ecol[slot] = -1;
        eval[slot] = 0.0;
      }
    }
}

/* Width of the ELL part of a hybrid matrix.  One more ELL column costs
 * stride slots of (value + 4) bytes; it removes #{rows with length >= K}
 * entries of (value + 8) bytes from the COO part.  K_h is the largest K for
 * which every column up to K pays for itself.                              */
int64_t orc_hyb_width(int64_t n, const int32_t* rowptr, int value_bytes) {
  int64_t stride = orc_ell_stride(n);
  int64_t Kmax = orc_ell_width(n, rowptr);
  int64_t* count = (int64_t*)calloc((size_t)Kmax + 2, sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i) count[rowptr[i + 1] - rowptr[i]] += 1;
  /* count_ge[K] = #{L_i >= K}, computed from the top down in place */
  for (int64_t K = Kmax - 1; K >= 0; --K) count[K] += count[K + 1];
  int64_t Kh = 0;
  for (int64_t K = 1; K <= Kmax; ++K) {
    double coo_bytes_saved = (double)count[K] * (double)(value_bytes + 8);
    double ell_bytes_added = (double)stride * (double)(value_bytes + 4);
    if (coo_bytes_saved > ell_bytes_added)
      Kh = K;
    else
      break;
  }
  free(count);
  return Kh;
}

int64_t orc_csr_to_hyb(int64_t n, const int32_t* rowptr, const int32_t* col,
                       const double* val, int64_t K, int64_t stride,
                       int32_t* ecol, double* eval, int32_t* crow,
                       int32_t* ccol, double* cval) {
  int64_t c = 0;
  for (int64_t j = 0; j < K; ++j)
    for (int64_t i = 0; i < stride; ++i) {
      int64_t slot = j * stride + i;
      int64_t L = (i < n) ? (int64_t)(rowptr[i + 1] - rowptr[i]) : 0;
      if (j < L) {
        ecol[slot] = col[rowptr[i] + j];
        eval[slot] = val[rowptr[i] + j];
      } else {
        ecol[slot] = -1;
        eval[slot] = 0.0;
      }
    }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = rowptr[i] + K; k < rowptr[i + 1]; ++k) {
      crow[c] = (int32_t)i;
      ccol[c] = col[k];
      cval[c] = val[k];
      ++c;
    }
  return c;
}

int orc_cast_f32(int64_t count, const double* in, float* out) {
  for (int64_t k = 0; k < count; ++k) {
    float f = (float)in[k]; /* IEEE round to nearest, ties to even */
    if (isfinite(in[k]) && !isfinite(f)) return ORC_UNSUPPORTED;
    out[k] = f;
  }
  return ORC_OK;
}

/* IEEE 754 binary16 from its definition: 1 sign bit, 5 exponent bits with
 * bias 15, 10 fraction bits; normal numbers (1024+f)*2^(e-25), subnormals
 * f*2^-24.  Rounding is to nearest, ties to even.                          */
uint16_t orc_f64_to_f16(double v) {
  uint16_t sign = signbit(v) ? 0x8000u : 0u;
  if (isnan(v)) return (uint16_t)(sign | 0x7e00u);
  double a = fabs(v);
  if (isinf(a)) return (uint16_t)(sign | 0x7c00u);
  if (a == 0.0) return sign;
  int e2;
  frexp(a, &e2); /* a = f * 2^e2 with f in [0.5, 1) */
  int E = e2 - 1;  /* floor(log2 a) */
  if (E < -14) E = -14; /* subnormal range: spacing 2^-24 */
  double q = ldexp(a, 10 - E); /* a / spacing, exact */
  double fl = floor(q);
  double frac = q - fl;
  uint64_t m = (uint64_t)fl;
  if (frac > 0.5 || (frac == 0.5 && (m & 1u))) m += 1;
  if (m >= 2048) {
    m >>= 1;
    E += 1;
  }
  if (E > 15) return (uint16_t)(sign | 0x7c00u);
  if (m < 1024) return (uint16_t)(sign | (uint16_t)m);
  return (uint16_t)(sign | (uint16_t)(((E + 15) << 10) | (int)(m - 1024)));
}

double orc_f16_to_f64(uint16_t h) {
  int s = h >> 15;
  int e = (h >> 10) & 31;
  int f = h & 1023;
  double v;
  if (e == 0)
    v = ldexp((double)f, -24);
  else if (e == 31)
    v = f ? NAN : INFINITY;
  else
    v = ldexp((double)(1024 + f), e - 25);
  return s ? -v : v;
}

/* Per-row power-of-two scale s_i = 2^ceil(log2 max|a_ij|) (1 for an empty or
 * all-zero row), stored as FP32; h = binary16(a / s_i).                     */
int orc_rowscale_f16(int64_t n, const int32_t* rowptr, const double* val,
                     uint16_t* h, float* scale) {
  for (int64_t i = 0; i < n; ++i) {
    double m = 0.0;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      if (!isfinite(val[k])) return ORC_UNSUPPORTED;
      if (fabs(val[k]) > m) m = fabs(val[k]);
    }
    double s = 1.0;
    if (m > 0.0) {
      int e2;
      double f = frexp(m, &e2); /* m = f * 2^e2 */
      int E = (f == 0.5) ? e2 - 1 : e2;
      if (E > 127 || E < -126) return ORC_UNSUPPORTED;
      s = ldexp(1.0, E);
    }
    scale[i] = (float)s;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
      h[k] = orc_f64_to_f16(val[k] / s);
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* SpMV                                                                     */
/* ------------------------------------------------------------------------ */
void orc_spmv_csr(int64_t n, const int32_t* rowptr, const int32_t* col,
                  const double* val, const double* x, double alpha,
                  double beta, double* y, int mode) {
  ORC_PAR_FOR
  for (int64_t i = 0; i < n; ++i) {
    double s;
    if (mode == 1) {
      s = 0.0;
      for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
        s = s + val[k] * x[col[k]];
    } else {
      acc_t a;
      acc_init(&a, 0.0);
      for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
        acc_add(&a, val[k], x[col[k]]);
      s = acc_result(&a);
    }
    y[i] = scale_out(alpha, s, beta, beta == 0.0 ? 0.0 : y[i]);
  }
}

void orc_spmv_csr_z(int64_t n, const int32_t* rowptr, const int32_t* col,
                    const double* val, const double* x, const double* alpha,
                    const double* beta, double* y) {
  const int beta0 = beta[0] == 0.0 && beta[1] == 0.0;
  for (int64_t i = 0; i < n; ++i) {
    acc_t re, im;
    acc_init(&re, 0.0);
    acc_init(&im, 0.0);
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      const double ar = val[2 * k], ai = val[2 * k + 1];
      const double xr = x[2 * col[k]], xi = x[2 * col[k] + 1];
      acc_add(&re, ar, xr);
      acc_add(&re, -ai, xi);
      acc_add(&im, ar, xi);
      acc_add(&im, ai, xr);
    }
    const double sr = acc_result(&re), si = acc_result(&im);
    double yr = alpha[0] * sr - alpha[1] * si;
    double yi = alpha[0] * si + alpha[1] * sr;
    if (!beta0) {
      const double br = beta[0], bi = beta[1];
      const double or_ = y[2 * i], oi = y[2 * i + 1];
      yr = yr + (br * or_ - bi * oi);
      yi = yi + (br * oi + bi * or_);
    }
    y[2 * i] = yr;
    y[2 * i + 1] = yi;
  }
}

void orc_absrow_z(int64_t n, const int32_t* rowptr, const int32_t* col,
                  const double* val, const double* x, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
      s = s + hypot(val[2 * k], val[2 * k + 1]) *
                  hypot(x[2 * col[k]], x[2 * col[k] + 1]);
    out[i] = s;
  }
}

void orc_spmv_coo(int64_t n, int64_t nnz, const int32_t* row,
                  const int32_t* col, const double* val, const double* x,
                  double alpha, double beta, double* y) {
  acc_t* a = (acc_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(acc_t));
  for (int64_t i = 0; i < n; ++i) acc_init(&a[i], 0.0);
  for (int64_t k = 0; k < nnz; ++k) acc_add(&a[row[k]], val[k], x[col[k]]);
  for (int64_t i = 0; i < n; ++i)
    y[i] = scale_out(alpha, acc_result(&a[i]), beta, beta == 0.0 ? 0.0 : y[i]);
  free(a);
}

void orc_spmv_ell(int64_t n, int64_t K, int64_t stride, const int32_t* ecol,
                  const double* eval, const double* x, double alpha,
                  double beta, double* y) {
  for (int64_t i = 0; i < n; ++i) {
    acc_t a;
    acc_init(&a, 0.0);
    for (int64_t j = 0; j < K; ++j) {
      int32_t c = ecol[j * stride + i];
      if (c < 0) continue; /* padding slot */
      acc_add(&a, eval[j * stride + i], x[c]);
    }
    y[i] = scale_out(alpha, acc_result(&a), beta, beta == 0.0 ? 0.0 : y[i]);
  }
}

void orc_spmv_hyb(int64_t n, int64_t K, int64_t stride, const int32_t* ecol,
                  const double* eval, int64_t cnnz, const int32_t* crow,
                  const int32_t* ccol, const double* cval, const double* x,
                  double alpha, double beta, double* y) {
  acc_t* a = (acc_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(acc_t));
  for (int64_t i = 0; i < n; ++i) {
    acc_init(&a[i], 0.0);
    for (int64_t j = 0; j < K; ++j) {
      int32_t c = ecol[j * stride + i];
      if (c < 0) continue;
      acc_add(&a[i], eval[j * stride + i], x[c]);
    }
  }
  for (int64_t k = 0; k < cnnz; ++k) acc_add(&a[crow[k]], cval[k], x[ccol[k]]);
  for (int64_t i = 0; i < n; ++i)
    y[i] = scale_out(alpha, acc_result(&a[i]), beta, beta == 0.0 ? 0.0 : y[i]);
  free(a);
}

void orc_spmv_csr_f16(int64_t n, const int32_t* rowptr, const int32_t* col,
                      const uint16_t* h, const float* scale, const double* x,
                      double alpha, double beta, double* y) {
  for (int64_t i = 0; i < n; ++i) {
    acc_t a;
    acc_init(&a, 0.0);
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
      acc_add(&a, orc_f16_to_f64(h[k]), x[col[k]]);
    double s = (double)scale[i] * acc_result(&a);
    y[i] = scale_out(alpha, s, beta, beta == 0.0 ? 0.0 : y[i]);
  }
}

void orc_absrow(int64_t n, const int32_t* rowptr, const int32_t* col,
                const double* val, const double* x, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
      s = s + fabs(val[k]) * fabs(x[col[k]]);
    out[i] = s;
  }
}

/* ------------------------------------------------------------------------ */
/* dense reference routines                                                 */
/* ------------------------------------------------------------------------ */
void orc_dense_matvec(int64_t n, int64_t m, const double* A, const double* x,
                      double* y) {
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t j = 0; j < m; ++j) s = s + A[i * m + j] * x[j];
    y[i] = s;
  }
}

/* Gaussian elimination with partial pivoting on a copy of row-major A. */
int orc_dense_lu_solve(int64_t n, const double* A, const double* b,
                       double* x) {
  double* M = (double*)malloc((size_t)(n * n > 0 ? n * n : 1) * sizeof(double));
  double* r = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  memcpy(M, A, (size_t)(n * n) * sizeof(double));
  memcpy(r, b, (size_t)n * sizeof(double));
  int status = ORC_OK;
  for (int64_t k = 0; k < n; ++k) {
    int64_t p = k;
    for (int64_t i = k + 1; i < n; ++i)
      if (fabs(M[i * n + k]) > fabs(M[p * n + k])) p = i;
    if (M[p * n + k] == 0.0) {
      status = ORC_BREAKDOWN;
      break;
    }
    if (p != k) {
      for (int64_t j = 0; j < n; ++j) {
        double t = M[k * n + j];
        M[k * n + j] = M[p * n + j];
        M[p * n + j] = t;
      }
      double t = r[k];
      r[k] = r[p];
      r[p] = t;
    }
    for (int64_t i = k + 1; i < n; ++i) {
      double l = M[i * n + k] / M[k * n + k];
      M[i * n + k] = 0.0;
      for (int64_t j = k + 1; j < n; ++j) M[i * n + j] -= l * M[k * n + j];
      r[i] -= l * r[k];
    }
  }
  if (status == ORC_OK)
    for (int64_t i = n - 1; i >= 0; --i) {
      double s = r[i];
      for (int64_t j = i + 1; j < n; ++j) s -= M[i * n + j] * x[j];
      x[i] = s / M[i * n + i];
    }
  free(M);
  free(r);
  return status;
}

/* ------------------------------------------------------------------------ */
/* vector helpers for the solvers (plain ascending loops)                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t n;
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
} csr_t;

static void matvec(const csr_t* A, const double* x, double* y) {
  orc_spmv_csr(A->n, A->rowptr, A->col, A->val, x, 1.0, 0.0, y, 0);
}

/* r = b - A x, each entry accumulated accurately and rounded once */
static void residual(const csr_t* A, const double* b, const double* x,
                     double* r) {
  ORC_PAR_FOR
  for (int64_t i = 0; i < A->n; ++i) {
    acc_t a;
    acc_init(&a, b[i]);
    for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
      acc_add(&a, -A->val[k], x[A->col[k]]);
    r[i] = acc_result(&a);
  }
}

static double dot(int64_t n, const double* a, const double* b) {
  double s = 0.0;
  ORC_PAR_SUM_S
  for (int64_t i = 0; i < n; ++i) s = s + a[i] * b[i];
  return s;
}

static double nrm2(int64_t n, const double* a) { return sqrt(dot(n, a, a)); }

static double* vec(int64_t n) {
  return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
}

static double threshold(const orc_stop* st, double nb, double nr0) {
  double base = st->baseline == 1 ? nr0 : nb;
  double t = st->rel_tol * base;
  return t > st->abs_tol ? t : st->abs_tol;
}

static double baseline_norm(const orc_stop* st, double nb, double nr0) {
  double base = st->baseline == 1 ? nr0 : nb;
  return base > 0.0 ? base : 1.0;
}

/* ------------------------------------------------------------------------ */
/* CG (Hestenes-Stiefel, unpreconditioned; Saad 2003, ch. 6)                */
/* ------------------------------------------------------------------------ */
int orc_cg(int64_t n, const int32_t* rowptr, const int32_t* col,
           const double* val, const double* b, double* x,
           const orc_stop* stop, orc_info* info, double* hist,
           int64_t hist_cap) {
  csr_t A = {n, rowptr, col, val};
  memset(info, 0, sizeof(*info));
  double nb = nrm2(n, b);
  if (!isfinite(nb)) return ORC_NONFINITE;
  if (nb == 0.0) {
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    return ORC_OK;
  }
  double *r = vec(n), *p = vec(n), *q = vec(n);
  residual(&A, b, x, r);
  double rho = dot(n, r, r);
  double nr0 = sqrt(rho);
  double thr = threshold(stop, nb, nr0);
  double base = baseline_norm(stop, nb, nr0);
  int status = ORC_OK;
  memcpy(p, r, (size_t)n * sizeof(double));
  int64_t it = 0, repl = 0;
  int check = sqrt(rho) <= thr;
  for (;;) {
    if (check) {
      /* stopping test on the recurrence residual passed: verify the true
       * residual b - A x, replacing r and restarting p if it disagrees */
      residual(&A, b, x, r);
      double nt = nrm2(n, r);
      info->relres_true = nt / base;
      if (nt <= thr) break;
      if (repl >= stop->max_replacements) {
        status = ORC_NOT_CONVERGED;
        break;
      }
      repl++;
      rho = nt * nt;
      memcpy(p, r, (size_t)n * sizeof(double));
      check = 0;
    }
    if (it >= stop->max_iters) {
      residual(&A, b, x, q);
      info->relres_true = nrm2(n, q) / base;
      status = ORC_NOT_CONVERGED;
      break;
    }
    matvec(&A, p, q);
    double pq = dot(n, p, q);
    if (!isfinite(pq)) {
      status = ORC_NONFINITE;
      break;
    }
    if (pq <= 0.0) {
      status = ORC_BREAKDOWN;
      break;
    }
    double alpha = rho / pq;
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
    double rho_new = dot(n, r, r);
    ++it;
    info->relres_recurrence = sqrt(rho_new) / base;
    double beta = rho_new / rho;
    if (hist && 2 * it <= hist_cap) {
      hist[2 * (it - 1)] = alpha;
      hist[2 * (it - 1) + 1] = beta;
    }
    if (sqrt(rho_new) <= thr) {
      check = 1;
      continue;
    }
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
    rho = rho_new;
  }
  info->iters = it;
  info->replacements = repl;
  free(r);
  free(p);
  free(q);
  return status;
}

/* ------------------------------------------------------------------------ */
/* PageRank by power iteration (Page, Brin, Motwani & Winograd 1998)        */
/* ------------------------------------------------------------------------ */
int orc_pagerank(int64_t n, const int32_t* rowptr, const int32_t* col,
                 double damping, double tol, int64_t max_iters, double* x,
                 int64_t* iters, double* delta) {
  *iters = 0;
  *delta = 0.0;
  if (n <= 0) return ORC_OK;
  int64_t* d = (int64_t*)calloc((size_t)n, sizeof(int64_t));
  double* xn = vec(n);
  for (int64_t k = 0; k < rowptr[n]; ++k) d[col[k]]++;
  ORC_PAR_FOR
  for (int64_t i = 0; i < n; ++i) x[i] = 1.0 / (double)n;
  int status = ORC_NOT_CONVERGED;
  for (int64_t it = 0; it < max_iters; ++it) {
    double dangling = 0.0;
    for (int64_t i = 0; i < n; ++i)
      if (d[i] == 0) dangling = dangling + x[i];
    double ch = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      double s = 0.0;
      for (int64_t k = rowptr[j]; k < rowptr[j + 1]; ++k)
        s = s + x[col[k]] / (double)d[col[k]];
      xn[j] = damping * (s + dangling / (double)n) + (1.0 - damping) / (double)n;
      ch = ch + fabs(xn[j] - x[j]);
    }
    memcpy(x, xn, (size_t)n * sizeof(double));
    *iters = it + 1;
    *delta = ch;
    if (!isfinite(ch)) {
      status = ORC_NONFINITE;
      break;
    }
    if (ch <= tol) {
      status = ORC_OK;
      break;
    }
  }
  free(d);
  free(xn);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Jacobi and block-Jacobi preconditioners, preconditioned CG               */
/* (Saad 2003, ch. 10 and Algorithm 9.1)                                     */
/* ------------------------------------------------------------------------ */
int orc_jacobi(int64_t n, const int32_t* rowptr, const int32_t* col,
               const double* val, double* dinv) {
  for (int64_t i = 0; i < n; ++i) {
    double d = 0.0;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
      if (col[k] == i) d = val[k];
    if (d == 0.0 || !isfinite(d)) return ORC_BREAKDOWN;
    dinv[i] = 1.0 / d;
  }
  return ORC_OK;
}

int orc_block_jacobi(int64_t n, const int32_t* rowptr, const int32_t* col,
                     const double* val, int64_t bs, double* binv) {
  if (bs < 1) return ORC_INVALID_ARG;
  int64_t nb = (n + bs - 1) / bs;
  double* B = (double*)malloc((size_t)(bs * bs) * sizeof(double));
  double* e = (double*)malloc((size_t)bs * sizeof(double));
  double* y = (double*)malloc((size_t)bs * sizeof(double));
  int status = ORC_OK;
  for (int64_t k = 0; k < nb && status == ORC_OK; ++k) {
    int64_t r0 = k * bs, m = (n - r0) < bs ? (n - r0) : bs;
    /* the dense block A[I,I], row-major m x m */
    for (int64_t t = 0; t < m * m; ++t) B[t] = 0.0;
    for (int64_t i = 0; i < m; ++i)
      for (int64_t q = rowptr[r0 + i]; q < rowptr[r0 + i + 1]; ++q)
        if (col[q] >= r0 && col[q] < r0 + m) B[i * m + (col[q] - r0)] = val[q];
    double* slot = binv + k * bs * bs;
    for (int64_t t = 0; t < bs * bs; ++t) slot[t] = 0.0;
    for (int64_t j = 0; j < m; ++j) {
      for (int64_t i = 0; i < m; ++i) e[i] = i == j ? 1.0 : 0.0;
      if (orc_dense_lu_solve(m, B, e, y) != ORC_OK) {
        status = ORC_BREAKDOWN;
        break;
      }
      for (int64_t i = 0; i < m; ++i) {
        if (!isfinite(y[i])) status = ORC_BREAKDOWN;
        slot[j * bs + i] = y[i];
      }
    }
  }
  free(B);
  free(e);
  free(y);
  return status;
}

void orc_prec_apply(int64_t n, int kind, int64_t bs, const double* minv,
                    const double* r, double* z) {
  if (kind == 1) {
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) z[i] = minv[i] * r[i];
    return;
  }
  for (int64_t r0 = 0; r0 < n; r0 += bs) {
    int64_t m = (n - r0) < bs ? (n - r0) : bs;
    const double* slot = minv + (r0 / bs) * bs * bs;
    for (int64_t i = 0; i < m; ++i) {
      double s = 0.0;
      for (int64_t j = 0; j < m; ++j) s = s + slot[j * bs + i] * r[r0 + j];
      z[r0 + i] = s;
    }
  }
}

int orc_pcg(int64_t n, const int32_t* rowptr, const int32_t* col,
            const double* val, int kind, int64_t bs, const double* minv,
            const double* b, double* x, const orc_stop* stop, orc_info* info) {
  csr_t A = {n, rowptr, col, val};
  memset(info, 0, sizeof(*info));
  if (kind != 1 && kind != 2) return ORC_INVALID_ARG;
  double nb = nrm2(n, b);
  if (!isfinite(nb)) return ORC_NONFINITE;
  if (nb == 0.0) {
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    return ORC_OK;
  }
  double *r = vec(n), *z = vec(n), *p = vec(n), *q = vec(n);
  residual(&A, b, x, r);
  orc_prec_apply(n, kind, bs, minv, r, z);
  double rho = dot(n, r, z);
  double nr0 = nrm2(n, r);
  double thr = threshold(stop, nb, nr0);
  double base = baseline_norm(stop, nb, nr0);
  int status = ORC_OK;
  memcpy(p, z, (size_t)n * sizeof(double));
  int64_t it = 0, repl = 0;
  int check = nr0 <= thr;
  for (;;) {
    if (check) {
      residual(&A, b, x, r);
      double nt = nrm2(n, r);
      info->relres_true = nt / base;
      if (nt <= thr) break;
      if (repl >= stop->max_replacements) {
        status = ORC_NOT_CONVERGED;
        break;
      }
      repl++;
      orc_prec_apply(n, kind, bs, minv, r, z);
      rho = dot(n, r, z);
      memcpy(p, z, (size_t)n * sizeof(double));
      check = 0;
    }
    if (it >= stop->max_iters) {
      residual(&A, b, x, q);
      info->relres_true = nrm2(n, q) / base;
      status = ORC_NOT_CONVERGED;
      break;
    }
    if (!(rho > 0.0)) {  /* (r, M^{-1} r) > 0 for SPD M and r != 0 */
      status = isfinite(rho) ? ORC_BREAKDOWN : ORC_NONFINITE;
      break;
    }
    matvec(&A, p, q);
    double pq = dot(n, p, q);
    if (!isfinite(pq)) {
      status = ORC_NONFINITE;
      break;
    }
    if (pq <= 0.0) {
      status = ORC_BREAKDOWN;
      break;
    }
    double alpha = rho / pq;
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
    orc_prec_apply(n, kind, bs, minv, r, z);
    double rho_new = dot(n, r, z);
    double rr = dot(n, r, r);
    ++it;
    info->relres_recurrence = sqrt(rr) / base;
    if (sqrt(rr) <= thr) {
      check = 1;
      continue;
    }
    double beta = rho_new / rho;
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    rho = rho_new;
  }
  info->iters = it;
  info->replacements = repl;
  free(r);
  free(z);
  free(p);
  free(q);
  return status;
}

/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* Pipelined CG (Ghysels & Vanroose 2014), unpreconditioned                  */
/* ------------------------------------------------------------------------ */
int orc_pipecg(int64_t n, const int32_t* rowptr, const int32_t* col,
               const double* val, const double* b, double* x,
               const orc_stop* stop, orc_info* info) {
  csr_t A = {n, rowptr, col, val};
  memset(info, 0, sizeof(*info));
  double nb = nrm2(n, b);
  if (!isfinite(nb)) return ORC_NONFINITE;
  if (nb == 0.0) {
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    return ORC_OK;
  }
  double *r = vec(n), *w = vec(n), *q = vec(n), *z = vec(n), *s = vec(n),
         *p = vec(n);
  residual(&A, b, x, r);
  double nr0 = nrm2(n, r);
  double thr = threshold(stop, nb, nr0);
  double base = baseline_norm(stop, nb, nr0);
  int status = ORC_OK;
  int64_t it = 0, repl = 0;
  int fresh = 1;               /* next step starts a recurrence (beta = 0) */
  double gamma_old = 0.0, alpha_old = 0.0;
  matvec(&A, r, w);
  for (;;) {
    double gamma = dot(n, r, r);
    double delta = dot(n, w, r);
    info->relres_recurrence = sqrt(gamma) / base;
    if (!isfinite(gamma) || !isfinite(delta)) {
      status = ORC_NONFINITE;
      break;
    }
    if (sqrt(gamma) <= thr) {
      /* verify b - A x; on disagreement replace r and restart */
      residual(&A, b, x, r);
      double nt = nrm2(n, r);
      info->relres_true = nt / base;
      if (nt <= thr) break;
      if (repl >= stop->max_replacements) {
        status = ORC_NOT_CONVERGED;
        break;
      }
      repl++;
      matvec(&A, r, w);
      fresh = 1;
      continue;
    }
    if (it >= stop->max_iters) {
      residual(&A, b, x, q);
      info->relres_true = nrm2(n, q) / base;
      status = ORC_NOT_CONVERGED;
      break;
    }
    matvec(&A, w, q);
    double beta, alpha, den;
    if (fresh) {
      beta = 0.0;
      den = delta;
    } else {
      beta = gamma / gamma_old;
      den = delta - beta * gamma / alpha_old;
    }
    if (!isfinite(den)) {
      status = ORC_NONFINITE;
      break;
    }
    if (den <= 0.0) { /* (p, A p) > 0 for SPD A */
      status = ORC_BREAKDOWN;
      break;
    }
    alpha = gamma / den;
    if (fresh) {
      for (int64_t i = 0; i < n; ++i) {
        z[i] = q[i];
        s[i] = w[i];
        p[i] = r[i];
      }
    } else {
      for (int64_t i = 0; i < n; ++i) {
        z[i] = q[i] + beta * z[i];
        s[i] = w[i] + beta * s[i];
        p[i] = r[i] + beta * p[i];
      }
    }
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * s[i];
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) w[i] = w[i] - alpha * z[i];
    gamma_old = gamma;
    alpha_old = alpha;
    fresh = 0;
    ++it;
  }
  info->iters = it;
  info->replacements = repl;
  free(r);
  free(w);
  free(q);
  free(z);
  free(s);
  free(p);
  return status;
}

/* ------------------------------------------------------------------------ */
/* CGS (Sonneveld 1989; Saad 2003, Algorithm 7.6), r_hat = r_0              */
/* ------------------------------------------------------------------------ */
int orc_cgs(int64_t n, const int32_t* rowptr, const int32_t* col,
            const double* val, const double* b, double* x,
            const orc_stop* stop, orc_info* info) {
  csr_t A = {n, rowptr, col, val};
  memset(info, 0, sizeof(*info));
  double nb = nrm2(n, b);
  if (!isfinite(nb)) return ORC_NONFINITE;
  if (nb == 0.0) {
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    return ORC_OK;
  }
  double *r = vec(n), *rh = vec(n), *p = vec(n), *u = vec(n), *q = vec(n),
         *v = vec(n), *w = vec(n);
  residual(&A, b, x, r);
  double nr0 = nrm2(n, r);
  double thr = threshold(stop, nb, nr0);
  double base = baseline_norm(stop, nb, nr0);
  int status = ORC_OK;
  int64_t it = 0, repl = 0;
  int restart = 1;
  int check = nr0 <= thr;
  double rho = 0.0;
  for (;;) {
    if (check) {
      residual(&A, b, x, r);
      double nt = nrm2(n, r);
      info->relres_true = nt / base;
      if (nt <= thr) break;
      if (repl >= stop->max_replacements) {
        status = ORC_NOT_CONVERGED;
        break;
      }
      repl++;
      restart = 1;
      check = 0;
    }
    if (restart) {
      memcpy(rh, r, (size_t)n * sizeof(double));
      memcpy(u, r, (size_t)n * sizeof(double));
      memcpy(p, r, (size_t)n * sizeof(double));
      rho = dot(n, rh, r);
      restart = 0;
    }
    if (it >= stop->max_iters) {
      residual(&A, b, x, w);
      info->relres_true = nrm2(n, w) / base;
      status = ORC_NOT_CONVERGED;
      break;
    }
    if (!isfinite(rho)) {
      status = ORC_NONFINITE;
      break;
    }
    if (rho == 0.0) {
      status = ORC_BREAKDOWN;
      break;
    }
    matvec(&A, p, v);
    double sigma = dot(n, rh, v);
    if (!isfinite(sigma)) {
      status = ORC_NONFINITE;
      break;
    }
    if (sigma == 0.0) {
      status = ORC_BREAKDOWN;
      break;
    }
    double alpha = rho / sigma;
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) q[i] = u[i] - alpha * v[i];
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) w[i] = u[i] + q[i];
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * w[i];
    matvec(&A, w, v); /* v = A (u + q) */
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * v[i];
    ++it;
    double nr = nrm2(n, r);
    info->relres_recurrence = nr / base;
    if (!isfinite(nr)) {
      status = ORC_NONFINITE;
      break;
    }
    if (nr <= thr) {
      check = 1;
      continue;
    }
    double rho_new = dot(n, rh, r);
    double beta = rho_new / rho;
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) u[i] = r[i] + beta * q[i];
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) p[i] = u[i] + beta * (q[i] + beta * p[i]);
    rho = rho_new;
  }
  info->iters = it;
  info->replacements = repl;
  free(r);
  free(rh);
  free(p);
  free(u);
  free(q);
  free(v);
  free(w);
  return status;
}

/* ------------------------------------------------------------------------ */
/* BiCGSTAB (van der Vorst 1992; Saad 2003, ch. 7), r_hat = r_0             */
/* ------------------------------------------------------------------------ */
int orc_bicgstab(int64_t n, const int32_t* rowptr, const int32_t* col,
                 const double* val, const double* b, double* x,
                 const orc_stop* stop, orc_info* info) {
  csr_t A = {n, rowptr, col, val};
  memset(info, 0, sizeof(*info));
  double nb = nrm2(n, b);
  if (!isfinite(nb)) return ORC_NONFINITE;
  if (nb == 0.0) {
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    return ORC_OK;
  }
  double *r = vec(n), *rh = vec(n), *p = vec(n), *v = vec(n), *s = vec(n),
         *t = vec(n);
  residual(&A, b, x, r);
  double nr0 = nrm2(n, r);
  double thr = threshold(stop, nb, nr0);
  double base = baseline_norm(stop, nb, nr0);
  int status = ORC_OK;
  int64_t it = 0, repl = 0;
  int restart = 1;
  int check = nr0 <= thr;
  double rho = 1.0, alpha = 1.0, omega = 1.0;
  for (;;) {
    if (check) {
      residual(&A, b, x, r);
      double nt = nrm2(n, r);
      info->relres_true = nt / base;
      if (nt <= thr) break;
      if (repl >= stop->max_replacements) {
        status = ORC_NOT_CONVERGED;
        break;
      }
      repl++;
      restart = 1;
      check = 0;
    }
    if (restart) {
      memcpy(rh, r, (size_t)n * sizeof(double));
      ORC_PAR_FOR
      for (int64_t i = 0; i < n; ++i) p[i] = v[i] = 0.0;
      rho = alpha = omega = 1.0;
      restart = 0;
    }
    if (it >= stop->max_iters) {
      residual(&A, b, x, t);
      info->relres_true = nrm2(n, t) / base;
      status = ORC_NOT_CONVERGED;
      break;
    }
    double rho1 = dot(n, rh, r);
    if (!isfinite(rho1)) {
      status = ORC_NONFINITE;
      break;
    }
    if (rho1 == 0.0 || omega == 0.0) {
      status = ORC_BREAKDOWN;
      break;
    }
    double beta = (rho1 / rho) * (alpha / omega);
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
    matvec(&A, p, v);
    double rv = dot(n, rh, v);
    if (!isfinite(rv)) {
      status = ORC_NONFINITE;
      break;
    }
    if (rv == 0.0) {
      status = ORC_BREAKDOWN;
      break;
    }
    alpha = rho1 / rv;
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
    ++it;
    double ns = nrm2(n, s);
    info->relres_recurrence = ns / base;
    if (ns <= thr) {
      /* half step: the first update already meets the tolerance */
      ORC_PAR_FOR
      for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
      check = 1;
      continue;
    }
    matvec(&A, s, t);
    double tt = dot(n, t, t);
    if (!isfinite(tt)) {
      status = ORC_NONFINITE;
      break;
    }
    if (tt == 0.0) {
      status = ORC_BREAKDOWN;
      break;
    }
    omega = dot(n, t, s) / tt;
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i] + omega * s[i];
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
    double nr = nrm2(n, r);
    info->relres_recurrence = nr / base;
    rho = rho1;
    if (nr <= thr) check = 1;
  }
  info->iters = it;
  info->replacements = repl;
  free(r);
  free(rh);
  free(p);
  free(v);
  free(s);
  free(t);
  return status;
}

/* ------------------------------------------------------------------------ */
/* GMRES(m) (Saad & Schultz 1986), modified Gram-Schmidt Arnoldi, Givens    */
/* rotations on the Hessenberg matrix, restart after m steps                */
/* ------------------------------------------------------------------------ */
int orc_gmres(int64_t n, const int32_t* rowptr, const int32_t* col,
              const double* val, const double* b, double* x, int64_t m,
              const orc_stop* stop, orc_info* info, double* hist,
              int64_t hist_cap) {
  csr_t A = {n, rowptr, col, val};
  memset(info, 0, sizeof(*info));
  if (m < 1) return ORC_INVALID_ARG;
  double nb = nrm2(n, b);
  if (!isfinite(nb)) return ORC_NONFINITE;
  if (nb == 0.0) {
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    return ORC_OK;
  }
  double* V = vec((m + 1) * n);
  double* H = vec((m + 1) * m); /* H[i*m + j] = h_{i,j}, 0-based */
  double *cs = vec(m), *sn = vec(m), *g = vec(m + 1), *y = vec(m);
  double *w = vec(n), *r = vec(n);
  residual(&A, b, x, r);
  double beta = nrm2(n, r);
  double thr = threshold(stop, nb, beta);
  double base = baseline_norm(stop, nb, beta);
  info->relres_true = beta / base;
  int status = ORC_OK;
  int64_t it = 0, nhist = 0;
  while (beta > thr) {
    if (it >= stop->max_iters) {
      status = ORC_NOT_CONVERGED;
      break;
    }
    for (int64_t i = 0; i < n; ++i) V[i] = r[i] / beta;
    for (int64_t i = 0; i <= m; ++i) g[i] = 0.0;
    g[0] = beta;
    int64_t k = 0;
    for (int64_t j = 0; j < m && it < stop->max_iters; ++j) {
      double* vj = V + j * n;
      matvec(&A, vj, w);
      ++it;
      for (int64_t i = 0; i <= j; ++i) {
        double* vi = V + i * n;
        double h = dot(n, w, vi);
        H[i * m + j] = h;
        for (int64_t l = 0; l < n; ++l) w[l] = w[l] - h * vi[l];
      }
      double hnext = nrm2(n, w);
      if (!isfinite(hnext)) {
        status = ORC_NONFINITE;
        break;
      }
      H[(j + 1) * m + j] = hnext;
      for (int64_t i = 0; i < j; ++i) {
        double a = H[i * m + j], c = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a + sn[i] * c;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
      }
      double a = H[j * m + j], c = H[(j + 1) * m + j];
      double d = sqrt(a * a + c * c);
      if (d == 0.0) {
        status = ORC_BREAKDOWN;
        break;
      }
      cs[j] = a / d;
      sn[j] = c / d;
      H[j * m + j] = d;
      H[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      k = j + 1;
      double est = fabs(g[j + 1]);
      info->relres_recurrence = est / base;
      if (hist && nhist < hist_cap) hist[nhist++] = est;
      if (est <= thr || hnext == 0.0) break; /* converged or happy breakdown */
      double* vn = V + (j + 1) * n;
      for (int64_t l = 0; l < n; ++l) vn[l] = w[l] / hnext;
    }
    if (status != ORC_OK) break;
    /* back substitution R y = g, then x += V_k y */
    for (int64_t i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int64_t l = i + 1; l < k; ++l) s = s - H[i * m + l] * y[l];
      y[i] = s / H[i * m + i];
    }
    for (int64_t i = 0; i < k; ++i) {
      double* vi = V + i * n;
      for (int64_t l = 0; l < n; ++l) x[l] = x[l] + y[i] * vi[l];
    }
    residual(&A, b, x, r);
    beta = nrm2(n, r);
    info->relres_true = beta / base;
    if (beta <= thr) break;
    info->restarts++;
  }
  info->iters = it;
  free(V);
  free(H);
  free(cs);
  free(sn);
  free(g);
  free(y);
  free(w);
  free(r);
  return status;
}

/* ------------------------------------------------------------------------ */
/* mixed-precision iterative refinement                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t n;
  const int32_t* rowptr;
  const int32_t* col;
  int kind;
  const float* v32;
  const uint16_t* h16;
  const float* scale;
} lowmat_t;

/* FP32 operator: y_i = sum_j a_ij x_j in float, ascending order; for the
 * FP16 storage y_i = s_i * sum_j float(h_ij) x_j.                         */
static void low_matvec(const lowmat_t* L, const float* x, float* y) {
  ORC_PAR_FOR
  for (int64_t i = 0; i < L->n; ++i) {
    float s = 0.0f;
    for (int64_t k = L->rowptr[i]; k < L->rowptr[i + 1]; ++k) {
      float a = L->kind == 0 ? L->v32[k] : (float)orc_f16_to_f64(L->h16[k]);
      s = s + a * x[L->col[k]];
    }
    y[i] = L->kind == 0 ? s : L->scale[i] * s;
  }
}

/* reductions accumulate in double and round once to float */
static float fdot(int64_t n, const float* a, const float* b) {
  double s = 0.0;
  ORC_PAR_SUM_S
  for (int64_t i = 0; i < n; ++i) s = s + (double)a[i] * (double)b[i];
  return (float)s;
}

/* z = M^{-1} r in float (kind 0: z = r) */
static void low_prec_apply(int64_t n, int kind, int64_t bs, const float* minv,
                           const float* r, float* z) {
  if (kind == 0) {
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) z[i] = r[i];
  } else if (kind == 1) {
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) z[i] = minv[i] * r[i];
  } else {
    for (int64_t r0 = 0; r0 < n; r0 += bs) {
      int64_t m = (n - r0) < bs ? (n - r0) : bs;
      const float* slot = minv + (r0 / bs) * bs * bs;
      for (int64_t i = 0; i < m; ++i) {
        float s = 0.0f;
        for (int64_t j = 0; j < m; ++j) s = s + slot[j * bs + i] * r[r0 + j];
        z[r0 + i] = s;
      }
    }
  }
}

/* inner FP32 (preconditioned) CG from d = 0 on A_low d = f, to
 * ||r|| <= tol * ||f||; without a preconditioner z = r and this is plain CG */
/* Inner CG in float on L d = f from d = 0 (Hestenes-Stiefel, as cg()
 * above, with z = M^{-1} r).  p is the caller's direction vector.  When
 * carry > 0 the first direction is not z but z + (rho / (carry * *rho_io)) p:
 * p and *rho_io hold the last direction p_k and rho_k = r_k.z_k of the
 * previous inner solve, and carry is the factor s by which that solve's
 * normalised quantities grow when they are expressed relative to the new
 * right-hand side (p_k becomes s p_k, rho_k becomes s^2 rho_k), so the
 * first direction is the CG direction z + beta (s p_k) with
 * beta = rho / (s^2 rho_k).  On return p and *rho_io hold this solve's
 * last direction and its rho, *usable says whether they may be carried
 * (at least one step, and no breakdown), and *reduction is the recurrence
 * residual's final norm over its initial one.                             */
static int64_t low_cg(const lowmat_t* L, const float* f, float* d, float tol,
                      int64_t maxit, int pc_kind, int64_t bs,
                      const float* minv, float* p, double carry, double* rho_io,
                      int* usable, double* reduction) {
  int64_t n = L->n;
  float* r = (float*)malloc((size_t)(n > 0 ? n : 1) * sizeof(float));
  float* z = (float*)malloc((size_t)(n > 0 ? n : 1) * sizeof(float));
  float* q = (float*)malloc((size_t)(n > 0 ? n : 1) * sizeof(float));
  for (int64_t i = 0; i < n; ++i) {
    d[i] = 0.0f;
    r[i] = f[i];
  }
  low_prec_apply(n, pc_kind, bs, minv, r, z);
  float rho = fdot(n, r, z);
  float rr = fdot(n, r, r);
  float c = carry > 0.0 ? (float)((double)rho / (carry * *rho_io)) : 0.0f;
  if (carry > 0.0 && isfinite(c)) {
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) p[i] = z[i] + c * p[i];
  } else {
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) p[i] = z[i];
  }
  float thr = tol * sqrtf(rr);
  const float rr0 = rr;
  int64_t it = 0;
  int broke = 0;
  while (sqrtf(rr) > thr && it < maxit) {
    low_matvec(L, p, q);
    float pq = fdot(n, p, q);
    if (!(pq > 0.0f)) {
      broke = 1;
      break;
    }
    float alpha = rho / pq;
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) d[i] = d[i] + alpha * p[i];
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
    low_prec_apply(n, pc_kind, bs, minv, r, z);
    float rho_new = fdot(n, r, z);
    rr = fdot(n, r, r);
    ++it;
    /* the last direction stays p_k with rho_k whether the tolerance or the
     * step cap ends the solve */
    if (sqrtf(rr) <= thr || it >= maxit) break;
    float beta = rho_new / rho;
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    rho = rho_new;
  }
  *rho_io = rho;
  *usable = it > 0 && !broke && rho > 0.0f;
  *reduction = sqrt((double)rr / (double)rr0);
  free(r);
  free(z);
  free(q);
  return it;
}

int orc_ir(int64_t n, const int32_t* rowptr, const int32_t* col,
           const double* val64, int low_kind, const float* val32,
           const uint16_t* h16, const float* scale, const double* b,
           double* x, double outer_tol, int64_t outer_max, double inner_tol,
           int64_t inner_max, int last_step_variant, orc_ir_info* info) {
  return orc_ir_pc(n, rowptr, col, val64, low_kind, val32, h16, scale, b, x,
                   outer_tol, outer_max, inner_tol, inner_max,
                   last_step_variant, 0, 1, NULL, info);
}

int orc_ir_pc(int64_t n, const int32_t* rowptr, const int32_t* col,
              const double* val64, int low_kind, const float* val32,
              const uint16_t* h16, const float* scale, const double* b,
              double* x, double outer_tol, int64_t outer_max,
              double inner_tol, int64_t inner_max, int last_step_variant,
              int pc_kind, int64_t bs, const float* minv32,
              orc_ir_info* info) {
  csr_t A = {n, rowptr, col, val64};
  lowmat_t L = {n, rowptr, col, low_kind, val32, h16, scale};
  memset(info, 0, sizeof(*info));
  double nb = nrm2(n, b);
  if (!isfinite(nb)) return ORC_NONFINITE;
  if (nb == 0.0) {
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    return ORC_OK;
  }
  double* r = vec(n);
  float* f = (float*)malloc((size_t)(n > 0 ? n : 1) * sizeof(float));
  float* d = (float*)malloc((size_t)(n > 0 ? n : 1) * sizeof(float));
  float* p = (float*)malloc((size_t)(n > 0 ? n : 1) * sizeof(float));
  int status = ORC_OK;
  /* the previous step's residual norm, its inner rho, the reduction its
   * recurrence residual claimed and whether its last direction may be
   * carried (ORC_IR_CARRY) */
  double sigma_prev = 0.0, rho_prev = 0.0, claimed = 0.0;
  int usable = 0;
  for (;;) {
    residual(&A, b, x, r); /* FP64 residual with the FP64 matrix */
    double nr = nrm2(n, r);
    double relres = nr / nb;
    info->relres_true = relres;
    if (!isfinite(nr)) {
      status = ORC_NONFINITE;
      break;
    }
    if (relres <= outer_tol) break;
    if (info->outer_iters >= outer_max) {
      status = ORC_NOT_CONVERGED;
      break;
    }
    double sigma = nr;
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) f[i] = (float)(r[i] / sigma);
    double tol = inner_tol;
    if ((last_step_variant & ORC_IR_LAST_STEP) && relres * inner_tol <= outer_tol) {
      double t2 = 0.1 * outer_tol / relres;
      if (t2 > tol) tol = t2;
    }
    /* carried direction: the previous normalised quantities grow by
     * sigma_prev / sigma relative to the new right-hand side r / sigma.  It
     * is carried only while the FP64 residual followed the recurrence the
     * direction was built for: a true reduction sigma / sigma_prev more
     * than twice the recurrence's own means the low-precision operator is
     * too far from A for its directions to serve the next step. */
    double carry = ((last_step_variant & ORC_IR_CARRY) && usable &&
                    sigma <= 2.0 * claimed * sigma_prev) ? sigma_prev / sigma : 0.0;
    info->inner_iters_total += low_cg(&L, f, d, (float)tol, inner_max, pc_kind, bs,
                                      minv32, p, carry, &rho_prev, &usable, &claimed);
    sigma_prev = sigma;
    ORC_PAR_FOR
    for (int64_t i = 0; i < n; ++i) x[i] = x[i] + sigma * (double)d[i];
    info->outer_iters++;
  }
  free(r);
  free(f);
  free(d);
  free(p);
  return status;
}
