/*
 * oracle.h -- CPU oracle for the sparse matrix-vector product and the Krylov
 * solvers of Tsai, Cojean & Anzt, "Porting a sparse linear algebra math
 * library to Intel GPUs" (arXiv 2103.10116).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously
 * correct FP64 definition that the GPU library is checked against.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no source, header or helper with the GPU library and the
 * GPU library never calls it.
 *
 * Conventions: n = rows, ncols = columns, int32 CSR indices, int64 sizes.
 * Every routine is single-threaded and built with -ffp-contract=off, so the
 * only fused multiply-adds are the explicit fma() calls of the exact
 * two-product in the accurate dot product.
 */
#ifndef MXS_ORACLE_H
#define MXS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_INVALID_ARG = 1,
  ORC_INVALID_MATRIX = 2,
  ORC_UNSUPPORTED = 3,
  ORC_NOT_CONVERGED = 6,
  ORC_BREAKDOWN = 7,
  ORC_NONFINITE = 8
};

/* ---- CSR ingest ------------------------------------------------------- */
int orc_csr_validate(int64_t n, int64_t ncols, int64_t nnz,
                     const int32_t* rowptr, const int32_t* col);
/* Rows ordered by column (ties in input order), repeated columns summed in
 * input order; vpe = doubles per value (1 real, 2 complex). */
int orc_csr_sort_and_sum(int64_t n, int64_t ncols, int64_t nnz,
                         const int32_t* rowptr, const int32_t* col,
                         const double* val, int vpe, int32_t* rowptr_out,
                         int32_t* col_out, double* val_out, int64_t* nnz_out);

/* ---- format conversions ----------------------------------------------- */
void orc_csr_to_coo(int64_t n, const int32_t* rowptr, int32_t* row_out);
void orc_coo_to_csr(int64_t n, int64_t nnz, const int32_t* row,
                    int32_t* rowptr_out);
int64_t orc_ell_width(int64_t n, const int32_t* rowptr);
int64_t orc_ell_stride(int64_t n);
void orc_csr_to_ell(int64_t n, const int32_t* rowptr, const int32_t* col,
                    const double* val, int64_t K, int64_t stride,
                    int32_t* ecol, double* eval);
int64_t orc_hyb_width(int64_t n, const int32_t* rowptr, int value_bytes);
int64_t orc_csr_to_hyb(int64_t n, const int32_t* rowptr, const int32_t* col,
                       const double* val, int64_t K, int64_t stride,
                       int32_t* ecol, double* eval, int32_t* crow,
                       int32_t* ccol, double* cval);
int orc_cast_f32(int64_t count, const double* in, float* out);
uint16_t orc_f64_to_f16(double v);
double orc_f16_to_f64(uint16_t h);
int orc_rowscale_f16(int64_t n, const int32_t* rowptr, const double* val,
                     uint16_t* h, float* scale);

/* ---- SpMV: y = alpha*A*x + beta*y; beta == 0 never reads y -------------
 * mode 0: accurate row sums (compensated dot product, rounded once)
 * mode 1: naive ascending-order sums (for the dense cross-check)          */
void orc_spmv_csr(int64_t n, const int32_t* rowptr, const int32_t* col,
                  const double* val, const double* x, double alpha,
                  double beta, double* y, int mode);
void orc_spmv_coo(int64_t n, int64_t nnz, const int32_t* row,
                  const int32_t* col, const double* val, const double* x,
                  double alpha, double beta, double* y);
void orc_spmv_ell(int64_t n, int64_t K, int64_t stride, const int32_t* ecol,
                  const double* eval, const double* x, double alpha,
                  double beta, double* y);
void orc_spmv_hyb(int64_t n, int64_t K, int64_t stride, const int32_t* ecol,
                  const double* eval, int64_t cnnz, const int32_t* crow,
                  const int32_t* ccol, const double* cval, const double* x,
                  double alpha, double beta, double* y);
void orc_spmv_csr_f16(int64_t n, const int32_t* rowptr, const int32_t* col,
                      const uint16_t* h, const float* scale, const double* x,
                      double alpha, double beta, double* y);
/* Complex CSR product (the library's complex value types, named in the
 * paper's experiment-setup footnote): val, x, y, alpha, beta hold (re, im)
 * pairs.  Each row's real and imaginary sums are accumulated with the
 * compensated dot product (real part: re*re and -im*im terms; imaginary
 * part: re*im and im*re terms) and rounded once; then
 * y = alpha s + beta y in complex arithmetic (beta == 0 never reads y).
 * absrow_z gives sum_j |a_ij| |x_j| with complex moduli. */
void orc_spmv_csr_z(int64_t n, const int32_t* rowptr, const int32_t* col,
                    const double* val, const double* x, const double* alpha,
                    const double* beta, double* y);
void orc_absrow_z(int64_t n, const int32_t* rowptr, const int32_t* col,
                  const double* val, const double* x, double* out);
/* sum_j |a_ij| |x_j| per row (the scale of the per-entry error bound) */
void orc_absrow(int64_t n, const int32_t* rowptr, const int32_t* col,
                const double* val, const double* x, double* out);

/* ---- dense reference routines ---------------------------------------- */
void orc_dense_matvec(int64_t n, int64_t m, const double* A, const double* x,
                      double* y);
int orc_dense_lu_solve(int64_t n, const double* A, const double* b,
                       double* x);

/* ---- Krylov solvers --------------------------------------------------- */
typedef struct {
  int64_t max_iters;
  double rel_tol;
  double abs_tol;
  int32_t baseline;     /* 0: relative to ||b||, 1: relative to ||r0|| */
  int32_t max_replacements;
} orc_stop;

typedef struct {
  int64_t iters;
  double relres_recurrence;
  double relres_true;
  int64_t replacements;
  int64_t restarts;
} orc_info;

/* hist (nullable, capacity hist_cap doubles): CG writes (alpha_k, beta_k)
 * pairs, GMRES writes the residual estimate |g_{j+1}| after every step.  */
int orc_cg(int64_t n, const int32_t* rowptr, const int32_t* col,
           const double* val, const double* b, double* x,
           const orc_stop* stop, orc_info* info, double* hist,
           int64_t hist_cap);
int orc_bicgstab(int64_t n, const int32_t* rowptr, const int32_t* col,
                 const double* val, const double* b, double* x,
                 const orc_stop* stop, orc_info* info);
/* Pipelined CG (Ghysels & Vanroose 2014, unpreconditioned): the same
 * iterates as CG in exact arithmetic, with the two inner products of an
 * iteration, gamma = (r, r) and delta = (w, r) for w = A r, computed
 * together and independent of that iteration's product q = A w.  The
 * stopping test is on sqrt(gamma); the true-residual check and
 * replacements of orc_cg apply (a replacement restarts with w = A r and
 * beta = 0). */
int orc_pipecg(int64_t n, const int32_t* rowptr, const int32_t* col,
               const double* val, const double* b, double* x,
               const orc_stop* stop, orc_info* info);

/* CGS (Sonneveld 1989; Saad 2003, Algorithm 7.6), r_hat = r_0; the
 * stopping rule and replacements of orc_bicgstab (a replacement restarts
 * with r_hat = u = p = r). */
int orc_cgs(int64_t n, const int32_t* rowptr, const int32_t* col,
            const double* val, const double* b, double* x,
            const orc_stop* stop, orc_info* info);
int orc_gmres(int64_t n, const int32_t* rowptr, const int32_t* col,
              const double* val, const double* b, double* x, int64_t m,
              const orc_stop* stop, orc_info* info, double* hist,
              int64_t hist_cap);

/* ---- preconditioners (Saad 2003, ch. 10) -----------------------------
 * kind 1, Jacobi: M = diag(A), minv holds dinv_i = 1 / a_ii.
 * kind 2, block Jacobi: M = the diagonal blocks A[I,I] over consecutive row
 * ranges I = [k bs, min((k+1) bs, n)); minv holds their inverses, block k
 * column-major in a bs x bs slot (entry (i, j) at k bs^2 + j bs + i, zero
 * beyond the block's size).  Column j of an inverse solves A[I,I] y = e_j
 * with orc_dense_lu_solve.  Both return ORC_BREAKDOWN when a diagonal entry
 * is zero or missing, or a block is singular. */
int orc_jacobi(int64_t n, const int32_t* rowptr, const int32_t* col,
               const double* val, double* dinv);
int orc_block_jacobi(int64_t n, const int32_t* rowptr, const int32_t* col,
                     const double* val, int64_t bs, double* binv);
/* z = M^{-1} r */
void orc_prec_apply(int64_t n, int kind, int64_t bs, const double* minv,
                    const double* r, double* z);
/* Preconditioned CG (Saad 2003, Algorithm 9.1): rho = (r, z), z = M^{-1} r,
 * p = z + beta p; the stopping test is on ||r|| with the true-residual check
 * and residual replacement of orc_cg (a replacement restarts p = z). */
int orc_pcg(int64_t n, const int32_t* rowptr, const int32_t* col,
            const double* val, int kind, int64_t bs, const double* minv,
            const double* b, double* x, const orc_stop* stop, orc_info* info);

/* ---- PageRank (Page, Brin, Motwani & Winograd 1998) --------------------
 * The graph is given by its in-links: row j of (rowptr, col) lists the
 * sources i of the edges i -> j (sorted, no repeats), every edge of weight
 * one.  With d_i the out-degree of i (its occurrences in col) and D the
 * nodes without out-links, the power iteration from x_0 = 1/n is
 *   x_{k+1,j} = damping * (sum_{i -> j} x_{k,i} / d_i + sum_{i in D} x_{k,i} / n)
 *               + (1 - damping) / n
 * until ||x_{k+1} - x_k||_1 <= tol (then x = x_{k+1}, *iters = k + 1) or
 * max_iters steps (ORC_NOT_CONVERGED).  *delta = the last L1 change. */
int orc_pagerank(int64_t n, const int32_t* rowptr, const int32_t* col,
                 double damping, double tol, int64_t max_iters, double* x,
                 int64_t* iters, double* delta);

/* Mixed-precision iterative refinement: FP64 residual and update, inner CG
 * in FP32 on a low-precision copy of A.  low_kind 0: FP32 values (val32);
 * low_kind 1: FP16 values with a per-row power-of-two scale (h16, scale).
 * last_step_variant holds flags: ORC_IR_LAST_STEP loosens the inner
 * tolerance of the last step to max(inner_tol, 0.1*tol/relres) once
 * relres*inner_tol <= tol; ORC_IR_CARRY starts each inner CG after the
 * first from the previous one's last direction, rescaled to the new
 * right-hand side (z + rho/(s rho_k) p_k with s = the previous residual
 * norm over the new one), instead of from z, whenever the previous inner
 * solve took a step, did not break down, and the FP64 residual fell to at
 * most twice the fraction its recurrence residual claimed. */
#define ORC_IR_LAST_STEP 1
#define ORC_IR_CARRY 2
typedef struct {
  int64_t outer_iters;
  int64_t inner_iters_total;
  double relres_true;
} orc_ir_info;
int orc_ir(int64_t n, const int32_t* rowptr, const int32_t* col,
           const double* val64, int low_kind, const float* val32,
           const uint16_t* h16, const float* scale, const double* b,
           double* x, double outer_tol, int64_t outer_max, double inner_tol,
           int64_t inner_max, int last_step_variant, orc_ir_info* info);
/* The same with a preconditioned inner CG (pc_kind 0: none, 1 / 2 as
 * above), minv32 = the preconditioner rounded to FP32. */
int orc_ir_pc(int64_t n, const int32_t* rowptr, const int32_t* col,
              const double* val64, int low_kind, const float* val32,
              const uint16_t* h16, const float* scale, const double* b,
              double* x, double outer_tol, int64_t outer_max,
              double inner_tol, int64_t inner_max, int last_step_variant,
              int pc_kind, int64_t bs, const float* minv32,
              orc_ir_info* info);

#ifdef __cplusplus
}
#endif
#endif
