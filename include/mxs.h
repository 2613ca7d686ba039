/*
 * mxs.h -- C ABI of libmxs, an MI355X (gfx950) implementation of the sparse
 * matrix-vector product and the Krylov solvers studied in Tsai, Cojean &
 * Anzt, "Porting a sparse linear algebra math library to Intel GPUs"
 * (arXiv 2103.10116), section "Central Sparse Linear Algebra Functionality".
 *
 * General rules
 * -------------
 *  - Every function returns an mxs_status; MXS_OK (0) is success.  Output
 *    parameters are written only on success (solver info blocks are also
 *    written when the status is MXS_NOT_CONVERGED or MXS_BREAKDOWN).
 *  - No C++ exception crosses this boundary.  mxs_last_error(ctx) returns a
 *    human-readable detail string for the last failing call on that ctx.
 *  - Indices are int32 (n, ncols and nnz must be <= INT32_MAX, otherwise
 *    MXS_UNSUPPORTED); sizes in the signatures are int64.
 *  - "Device pointer" means memory on the ctx's GPU (e.g. a torch tensor's
 *    data_ptr()).  The library never frees memory it did not allocate.
 *  - All GPU work is enqueued on the ctx's HIP stream.  mxs_spmv returns
 *    without synchronising; calls that must report a result to the host
 *    (matrix creation/conversion, solvers, probes) synchronise that stream.
 *  - A ctx must not be used by two host threads at the same time.  A
 *    matrix is read-only during a product or a solve: the chunked products
 *    (merge-path CSR, COO, the COO part of hybrid) keep their per-chunk
 *    continuation partials in scratch memory of the ctx, so one matrix may
 *    be used by several ctxs on different streams at once.
 */
#ifndef MXS_H
#define MXS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mxs_status;
#define MXS_OK 0
#define MXS_INVALID_ARG 1      /* bad argument (NULL handle, size < 0, ...)   */
#define MXS_INVALID_MATRIX 2   /* CSR failed validation (see mxs_matrix_create_csr) */
#define MXS_UNSUPPORTED 3      /* size beyond int32, value outside FP32 range, format/dtype combination not offered */
#define MXS_OOM 4              /* device allocation failed                     */
#define MXS_HIP 5              /* a HIP runtime call failed                    */
#define MXS_NOT_CONVERGED 6    /* max_iters reached; x holds the last iterate  */
#define MXS_BREAKDOWN 7        /* solver breakdown (e.g. p.Ap <= 0 in CG)      */
#define MXS_NONFINITE 8        /* NaN/Inf met in the right-hand side or a reduction */
#define MXS_BUDGET 9           /* request exceeds the batch memory budget     */
#define MXS_PENDING 10         /* batch poll: not finished yet (not an error) */

typedef enum { MXS_CSR = 0, MXS_COO = 1, MXS_ELL = 2, MXS_HYB = 3 } mxs_format;

/* Value storage: FP64; FP32 (round to nearest even from FP64); FP16 with a
 * per-row power-of-two scale s_i = 2^ceil(log2 max_j |a_ij|) held in FP32
 * and binary16 codes of a_ij / s_i (CSR only); complex FP64 and complex
 * FP32 as (re, im) pairs (CSR only; the library's complex value types, named
 * in the paper's experiment-setup footnote). */
typedef enum {
  MXS_F64 = 0,
  MXS_F32 = 1,
  MXS_F16_ROWSCALED = 2,
  MXS_C128 = 3,
  MXS_C64 = 4
} mxs_dtype;

typedef struct mxs_ctx mxs_ctx;
typedef struct mxs_matrix mxs_matrix;

/* Optional device allocator.  alloc returns device memory of at least
 * `bytes` bytes usable on `stream`, 16-byte aligned at least (hipMalloc and
 * torch's caching allocator give 256 or more), or NULL on failure; free
 * releases it.  A block that is not 16-byte aligned is freed again at once
 * and the call that needed it fails with MXS_OOM. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, void* stream, void* user);
  void* user;
} mxs_allocator;

/* ---------------------------------------------------------------------- */
/* context                                                                 */
/* ---------------------------------------------------------------------- */

/* Creates a context on HIP device `device` that enqueues its work on
 * `hip_stream` (a hipStream_t; NULL = the device's null stream).  `alloc`
 * may be NULL, in which case hipMalloc/hipFree are used.  The stream is
 * borrowed and must outlive the context. */
mxs_status mxs_ctx_create(int device, void* hip_stream, const mxs_allocator* alloc,
                          mxs_ctx** out);
/* Releases the context's workspaces.  NULL is a no-op. */
mxs_status mxs_ctx_destroy(mxs_ctx* ctx);
/* Switches the stream later calls enqueue on. */
mxs_status mxs_ctx_set_stream(mxs_ctx* ctx, void* hip_stream);
/* Waits for all work enqueued on the ctx stream. */
mxs_status mxs_ctx_synchronize(mxs_ctx* ctx);

/* ---------------------------------------------------------------------- */
/* matrices                                                                */
/* ---------------------------------------------------------------------- */
#define MXS_HOST_PTRS 0   /* rowptr/col/val are host memory (copied in)   */
#define MXS_DEVICE_PTRS 1 /* rowptr/col/val are device memory (copied)    */
#define MXS_SORT_AND_SUM 2 /* OR-ed with one of the above: see below        */

/* Ingest a CSR matrix (paper, section "Central Sparse Linear Algebra
 * Functionality": row pointers to the first entry of each row of a
 * row-sorted coordinate list).  Layout: rowptr[nrows+1] int32,
 * col[nnz] int32, val[nnz] FP64.  The arrays are validated on the GPU:
 * rowptr[0] == 0, rowptr non-decreasing, rowptr[nrows] == nnz,
 * 0 <= col < ncols, columns strictly ascending within each row (sorted, no
 * duplicates); any violation returns MXS_INVALID_MATRIX.  With
 * MXS_SORT_AND_SUM in flags, rows whose columns are unordered or repeated
 * are repaired on the GPU instead of rejected: each such row is ordered by
 * column (a stable sort: equal columns keep their input order) and every
 * run of equal columns becomes one entry whose value is the run's values
 * added left to right in input order (a run summing to zero stays as an
 * explicit zero); the matrix then has nnz' <= nnz entries
 * (mxs_matrix_info).  Row pointers and the column range are checked either
 * way.  The matrix owns device copies of the arrays (format MXS_CSR, dtype
 * MXS_F64) and the row-block partition its SpMV kernel uses.  Synchronises
 * the ctx stream. */
mxs_status mxs_matrix_create_csr(mxs_ctx* ctx, int64_t nrows, int64_t ncols, int64_t nnz,
                                 const int32_t* rowptr, const int32_t* col,
                                 const double* val, int flags, mxs_matrix** out);

/* The same for complex FP64 values: val holds 2*nnz doubles, (re, im) of
 * each entry in CSR order.  The matrix has dtype MXS_C128; mxs_matrix_convert
 * turns it into CSR MXS_C128 (other kernel options) or MXS_C64 (each part
 * rounded to nearest even; MXS_UNSUPPORTED beyond the FP32 range).  Other
 * formats are not offered for complex values.  mxs_spmv takes alpha, beta
 * as host (re, im) pairs of the compute type (double or float) and x, y as
 * device arrays of pairs.  MXS_SORT_AND_SUM sums the real and imaginary
 * parts of repeated columns separately, each in input order. */
mxs_status mxs_matrix_create_csr_complex(mxs_ctx* ctx, int64_t nrows, int64_t ncols, int64_t nnz,
                                         const int32_t* rowptr, const int32_t* col,
                                         const double* val, int flags, mxs_matrix** out);

typedef struct {
  int64_t ell_width;      /* ELL: 0 = max row length; HYB: 0 = byte-model width, else forced K */
  int64_t max_ell_bytes;  /* 0 = no limit; ELL/HYB larger than this -> MXS_UNSUPPORTED */
  int32_t block_nnz;      /* CSR/COO: entries per work unit (256, 512 or 1024; others are rounded up); 0 = 512
                             (COO without column panels whose arrays exceed 256 MiB: 256) */
  int32_t csr_kernel;     /* CSR: MXS_CSR_AUTO, MXS_CSR_STREAM (row blocks), MXS_CSR_VECTOR (lanes per row), MXS_CSR_ROWS_LDS, MXS_CSR_PRODUCTS */
  int32_t lanes_per_row;  /* CSR vector kernel: 1 (thread per row), 4, 8, 16, 32 or 64; 0 = from the mean row length.
                             CSR rows-from-LDS kernel: 1, 2 or 4 lanes per row; 0 = the fewest that fill a wave */
  int32_t rows_per_group; /* CSR vector kernel: 2, 4 or 8 rows per lane group; 0 = default */
  int32_t waves_per_group;/* CSR stream / COO: independent waves per work-group, 1 or 4 (0 = 4) */
  int32_t coo_kernel;     /* COO and the COO part of HYB: MXS_COO_AUTO, MXS_COO_LDS, MXS_COO_RUNS */
  int32_t col_panels;     /* merge-path CSR, COO and the COO part of HYB: column panels (0 = auto,
                             1 = none, 2, 4 or 8; see below) */
} mxs_convert_opts;

#define MXS_CSR_AUTO 0   /* MERGE if a row exceeds 64 entries (real values whose chunks fit, else
                            STREAM); else ROWS_LDS for F32/F16
                            values and for F64 rows of at most 8 entries, PRODUCTS otherwise */
#define MXS_CSR_STREAM 1
#define MXS_CSR_VECTOR 2
#define MXS_CSR_ROWS_LDS 3 /* blocks of <= 64/G rows staged in LDS, G = 1, 2 or 4 lanes per row */
#define MXS_CSR_PRODUCTS 4 /* blocks of <= 64 rows; products formed by all lanes, summed per row from LDS */
#define MXS_CSR_MERGE 5    /* equal chunks of block_nnz entries whatever the rows (merge path): each
                              chunk's row pointers staged in LDS give the row of every entry; rows cut
                              by chunk edges completed by a fix-up pass.  FP64, FP32 and row-scaled
                              FP16 values, and no chunk may span more than block_nnz + 1 rows (long
                              runs of empty rows): otherwise MXS_UNSUPPORTED.
                              Column panels (col_panels = P > 1): the columns are cut into P equal
                              slices and the matrix keeps, besides its CSR arrays, a copy of its
                              entries ordered panel by panel (each row's entries of one slice form a
                              row of that panel; empty ones are left out), so that each XCD's share
                              of the chunks gathers x from one slice only, which stays in the XCD's
                              L2.  Each panel writes per-row partial sums into the ctx's scratch and
                              a last pass adds a row's partials in panel order.  Auto (0): panels
                              when x is larger than 4 MiB, P the smallest power of two that cuts it
                              into slices of at most 2 MiB (at most 8), none otherwise.
                              COO and the COO part of HYB take the same panels (auto: when a row has
                              more than 64 entries and x is larger than 4 MiB): their arrays then
                              hold the entries ordered by (panel, row, column), the row index of an
                              entry of row i in panel p being p * nrows + i (so exports show that
                              order), and a last pass adds each row's panel partials. */

#define MXS_COO_AUTO 0 /* RUNS for FP32/FP16 values when no row has more than 16 entries in
                          the part, else LDS */
#define MXS_COO_LDS 1  /* a chunk's col and val loaded coalesced (entry t*64 + lane) and the products
                          staged in LDS; each lane then sums a run of consecutive entries, whose
                          row indices it loads itself */
#define MXS_COO_RUNS 2 /* each lane loads its run of consecutive entries itself (16-byte loads)
                          and keeps it in registers; neighbouring rows by shuffles, no LDS */

/* Converts `src` (an FP64 CSR matrix from mxs_matrix_create_csr) to another
 * format and value type, on the GPU.  Layouts (all int32 indices):
 *  - CSR: as ingested.
 *  - COO: row[k], col[k], val[k] in exactly the CSR order (row-major,
 *    columns ascending).
 *  - ELL: width K (max row length unless forced), stride = nrows rounded up
 *    to a multiple of 64; slot (i, j) at j*stride + i (int64 offset) holds
 *    the j-th entry of row i; padding slots hold column -1 and value +0.
 *  - HYB: ELL part of width K_h holding the first min(L_i, K_h) entries of
 *    each row, the remaining entries in a COO part in CSR order.  The
 *    default K_h is the largest K for which each ELL column saves more COO
 *    bytes than it costs: #{rows with L_i >= K} * (V+8) > stride * (V+4),
 *    V = value bytes (the byte-per-entry model of the paper's "SpMV
 *    Performance Analysis" subsection).
 *  - F32 values are round-to-nearest-even casts; a finite FP64 value beyond
 *    the FP32 range returns MXS_UNSUPPORTED.  F16_ROWSCALED is CSR only.
 * The new matrix is independent of `src`.  Synchronises the ctx stream. */
mxs_status mxs_matrix_convert(mxs_ctx* ctx, const mxs_matrix* src, mxs_format fmt,
                              mxs_dtype dt, const mxs_convert_opts* opts, mxs_matrix** out);

typedef struct {
  int64_t nrows, ncols, nnz;
  int32_t format, dtype;
  int64_t ell_width, ell_stride; /* ELL / ELL part of HYB */
  int64_t coo_nnz;               /* COO entries (HYB: overflow part) */
  int64_t blocks;                /* work units of the SpMV kernel */
  int64_t bytes;                 /* device bytes owned by the matrix */
  int32_t block_nnz;
  int32_t lanes_per_row;         /* CSR vector kernel: 1 = thread per row, else lanes per row;
                                    rows-from-LDS kernel: lanes per row; other kernels 0 */
  int32_t rows_per_group;
  int32_t waves_per_group;       /* CSR stream / COO work-group shape */
  int32_t csr_kernel;            /* CSR: the kernel in use (MXS_CSR_STREAM ... MXS_CSR_PRODUCTS) */
  int32_t coo_kernel;            /* COO / COO part of HYB: the kernel in use (MXS_COO_LDS or
                                    MXS_COO_RUNS); other formats 0 */
  int32_t col_panels;            /* merge-path CSR, COO, HYB's COO part: column panels in use
                                    (1 = none); other formats and kernels 0 */
} mxs_matrix_desc;

mxs_status mxs_matrix_info(const mxs_matrix* A, mxs_matrix_desc* out);

/* Arrays a matrix exposes to mxs_matrix_export. */
typedef enum {
  MXS_ARR_ROWPTR = 0,  /* CSR: int32[nrows+1]                        */
  MXS_ARR_COL = 1,     /* CSR/COO: int32[nnz]                        */
  MXS_ARR_VAL = 2,     /* CSR/COO: value type [nnz] (F16: uint16)   */
  MXS_ARR_ROW = 3,     /* COO: int32[nnz]                            */
  MXS_ARR_ELL_COL = 4, /* ELL/HYB: int32[K*stride]                   */
  MXS_ARR_ELL_VAL = 5, /* ELL/HYB: value type [K*stride]            */
  MXS_ARR_COO_ROW = 6, /* HYB overflow: int32[coo_nnz]               */
  MXS_ARR_COO_COL = 7,
  MXS_ARR_COO_VAL = 8,
  MXS_ARR_SCALE = 9    /* F16_ROWSCALED: float[nrows]                */
} mxs_array;

/* Copies one array of `A` to host memory `dst` of `bytes` bytes (must equal
 * the array's size, else MXS_INVALID_ARG).  Synchronises the ctx stream. */
mxs_status mxs_matrix_export(mxs_ctx* ctx, const mxs_matrix* A, mxs_array which, void* dst,
                             size_t bytes);

/* Frees the matrix's device memory.  NULL is a no-op. */
mxs_status mxs_matrix_destroy(mxs_matrix* A);

/* ---------------------------------------------------------------------- */
/* sparse matrix-vector product                                            */
/* ---------------------------------------------------------------------- */

/* y = alpha * A * x + beta * y (paper, section "Central Sparse Linear
 * Algebra Functionality"), any format.  alpha and beta point to host
 * scalars of the compute type: double for F64 matrices, float for F32 and
 * F16_ROWSCALED.  x (ncols entries) and y (nrows entries) are device
 * vectors of the compute type; they must not overlap.  beta == 0 never
 * reads y (NaN/Inf in the old y do not propagate).  Asynchronous.
 * The products of a matrix whose streamed arrays exceed 256 MiB (larger
 * than the Infinity Cache) read those arrays with non-temporal loads, so
 * they do not displace x, y and the dirty lines of y from the caches;
 * smaller matrices keep ordinary loads, which leave them cached for the
 * next product. */
mxs_status mxs_spmv(mxs_ctx* ctx, const void* alpha, const mxs_matrix* A, const void* x,
                    const void* beta, void* y);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as mxs_spmv, same arguments, same kernels and the same result bit
 * for bit, but it never allocates or frees memory.  The scratch that the
 * chunked kernels need (merge-path CSR, COO and the COO part of hybrid keep
 * one row index and one partial sum per chunk) comes from a fixed device
 * array of MXS_NOALLOC_SCRATCH_BYTES (64 MiB) in each GPU's copy of the
 * library, set up by mxs_ctx_create and held until the process ends.  A
 * product needing more scratch than that returns MXS_UNSUPPORTED before
 * anything is enqueued.  Every call on one GPU shares that GPU's array:
 * calls whose work overlaps on one GPU (two streams, two contexts, two host
 * threads) race and must be ordered by the caller; calls on one stream are
 * ordered by it.  The array keeps the last call's contents; nothing in it
 * needs to start at zero (every chunk writes its slot before it is read).
 * Asynchronous. */
#define MXS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
mxs_status mxs_spmv_noalloc(mxs_ctx* ctx, const void* alpha, const mxs_matrix* A, const void* x,
                            const void* beta, void* y);

/* ---------------------------------------------------------------------- */
/* Krylov solvers                                                          */
/* ---------------------------------------------------------------------- */
typedef enum {
  MXS_CG = 0,
  MXS_BICGSTAB = 1,
  MXS_GMRES = 2,
  MXS_CGS = 3,
  MXS_PIPECG = 4
} mxs_solver;

#define MXS_BASELINE_RHS 0      /* tolerance relative to ||b||_2          */
#define MXS_BASELINE_INITIAL 1  /* tolerance relative to ||b - A x0||_2   */

typedef struct {
  int64_t max_iters;        /* CG/BiCGSTAB iterations, GMRES inner steps */
  double rel_tol;           /* stop when ||r|| <= max(rel_tol*baseline, abs_tol) */
  double abs_tol;
  int32_t baseline;         /* MXS_BASELINE_* */
  int32_t check_every;      /* iterations between host reads of the device convergence flag (0 = default) */
  int32_t max_replacements; /* true-residual replacements before NOT_CONVERGED (default 3 if < 0) */
} mxs_stop;

/* Preconditioners (the stationary ones of Saad 2003, ch. 10; the paper
 * lists Jacobi-type preconditioning among the library's functionality):
 *  MXS_PRECOND_JACOBI: M = diag(A), stored as 1/a_ii.
 *  MXS_PRECOND_BLOCK_JACOBI: M = the dense diagonal blocks A[I,I] over
 *    consecutive ranges of block_size rows (1..32, the last range ragged),
 *    inverted at set-up by Gauss-Jordan elimination with partial pivoting.
 * Both keep FP64 values and a copy rounded to FP32 (used by the FP32 inner
 * solve of mxs_solve_ir). */
typedef struct mxs_precond mxs_precond;
#define MXS_PRECOND_JACOBI 1
#define MXS_PRECOND_BLOCK_JACOBI 2

/* Builds M from an F64 CSR matrix (else MXS_UNSUPPORTED).  MXS_BREAKDOWN if
 * a diagonal entry is zero, missing or non-finite (Jacobi) or a block is
 * singular (block Jacobi); MXS_INVALID_ARG for an unknown kind or a block
 * size outside [1, 32].  M owns its device memory and is independent of A.
 * Synchronises the ctx stream. */
mxs_status mxs_precond_create(mxs_ctx* ctx, const mxs_matrix* A, int32_t kind,
                              int32_t block_size, mxs_precond** out);
mxs_status mxs_precond_destroy(mxs_precond* M);
/* Copies the FP64 values to host memory: n values 1/a_ii (Jacobi), or
 * ceil(n/bs) column-major bs x bs inverses, entry (i, j) of block k at
 * k*bs*bs + j*bs + i, zero beyond a ragged block (block Jacobi).  `bytes`
 * must hold them all.  Synchronises the ctx stream. */
mxs_status mxs_precond_export(mxs_ctx* ctx, const mxs_precond* M, double* host, size_t bytes);

typedef struct {
  int32_t restart;              /* GMRES restart length m (0 = 30) */
  int32_t reserved;
  const mxs_precond* precond;   /* CG only (preconditioned CG); NULL = none */
} mxs_solver_opts;

typedef struct {
  int64_t iters;             /* SpMV-based iterations (BiCGSTAB: full or half steps; GMRES: inner steps) */
  double relres_recurrence;  /* last recurrence residual / baseline */
  double relres_true;        /* ||b - A x|| / baseline, recomputed in FP64 at the end */
  int64_t replacements;
  int64_t restarts;
  int32_t status;
} mxs_solve_info;

/* Solves A x = b (paper, section "Central Sparse Linear Algebra
 * Functionality"; textbook forms from Saad 2003 and, for GMRES, Saad &
 * Schultz 1986).  A: an F64 matrix in any format (else MXS_UNSUPPORTED);
 * b, x: FP64 device vectors of nrows entries, x holds x0 on entry and the
 * iterate on exit.  CG: Hestenes-Stiefel.  BiCGSTAB: r_hat = r0.  CGS
 * (Sonneveld; Saad 2003, Algorithm 7.6): r_hat = r0, two products per
 * iteration, a replacement restarts r_hat = u = p = r.  Pipelined CG
 * (Ghysels & Vanroose 2014, unpreconditioned): CG's iterates in exact
 * arithmetic, with both inner products of an iteration independent of its
 * product, so an iteration is one product and one fused update kernel; a
 * replacement restarts the recurrences.  GMRES(m):
 * classical Gram-Schmidt with reorthogonalisation, Givens rotations and
 * the triangular solve on the GPU.  The solver stops when the recurrence
 * residual meets the tolerance and then checks the true residual b - A x in
 * FP64; if that fails it replaces r by it (CG/BiCGSTAB restart from the
 * current x) up to max_replacements times.  b == 0 returns x = 0 after 0
 * iterations.  With opts->precond, CG is the preconditioned CG of Saad
 * 2003, Algorithm 9.1 (rho = r.z, z = M^{-1} r, p = z + beta p; the stopping
 * test stays on ||r||; a replacement restarts p = z; (r, z) <= 0 is a
 * breakdown); BiCGSTAB and GMRES return MXS_UNSUPPORTED with a
 * preconditioner.  Returns MXS_OK, MXS_NOT_CONVERGED, MXS_BREAKDOWN or
 * MXS_NONFINITE; `info` (nullable) is filled in all four cases.
 * Synchronises the ctx stream. */
mxs_status mxs_solve(mxs_ctx* ctx, mxs_solver kind, const mxs_matrix* A, const double* b,
                     double* x, const mxs_stop* stop, const mxs_solver_opts* opts,
                     mxs_solve_info* info);

typedef struct {
  int64_t outer_iters;
  int64_t inner_iters_total;
  double relres_true;   /* final ||b - A64 x|| / ||b|| in FP64 */
  int32_t status;
} mxs_ir_info;

/* Mixed-precision iterative refinement (not in the paper; the classical
 * scheme): r = b - A64 x in FP64 with the FP64 matrix, stop when
 * ||r||/||b|| <= outer->rel_tol, else solve A_low d = r/||r|| by CG in FP32
 * (FP32 vectors and accumulation) to inner_rel_tol and update
 * x += ||r|| d in FP64.  A64: F64 CSR; A_low: F32 or F16_ROWSCALED CSR with
 * the same pattern (any other value type of either, complex ones included,
 * returns MXS_UNSUPPORTED before any work is enqueued).  `variant` holds
 * flags:
 *   MXS_IR_LAST_STEP loosens the inner tolerance to
 *     max(inner_rel_tol, 0.1*tol/relres) once relres*inner_rel_tol <= tol;
 *   MXS_IR_CARRY_DIRECTION starts every inner CG after the first from the
 *     previous one's last direction p_k, rescaled to the new right-hand side,
 *     instead of from z = M^{-1} f: with s = (previous ||r||) / (new ||r||),
 *     p = z + (f.z / (s rho_k)) p_k, rho_k = r_k.z_k of that last step.  The
 *     FP64 residual then replaces the FP32 recurrence residual inside one
 *     continuing CG (residual replacement, van der Vorst & Ye, SIAM J. Sci.
 *     Comput. 22, 2000; with a low-precision iteration as in the "reliable
 *     updates" of Clark et al., Comput. Phys. Commun. 181, 2010), so the
 *     inner steps do not start over at every refinement step.  The step
 *     restarts instead (p = z) when the previous solve took no step or broke
 *     down, when the new ||r|| exceeds twice the previous ||r|| times the
 *     reduction the previous FP32 recurrence residual claimed (A_low too far
 *     from A64 for its directions to serve the next step), or when the
 *     coefficient is not finite in FP32.
 * inner_precond (nullable, built from A64) turns the inner solve into
 * preconditioned CG with the FP32 copy of M.  Synchronises the ctx stream. */
#define MXS_IR_LAST_STEP 1
#define MXS_IR_CARRY_DIRECTION 2
mxs_status mxs_solve_ir(mxs_ctx* ctx, const mxs_matrix* A64, const mxs_matrix* A_low,
                        const double* b, double* x, const mxs_stop* outer,
                        double inner_rel_tol, int64_t inner_max, int32_t variant,
                        const mxs_precond* inner_precond, mxs_ir_info* info);

/* ---------------------------------------------------------------------- */
/* PageRank                                                                */
/* ---------------------------------------------------------------------- */
/* PageRank by power iteration over the SpMV (Page, Brin, Motwani & Winograd
 * 1998; the paper names it beside the Krylov solvers as an SpMV-based
 * method).  A graph is given by its in-links: row j of (rowptr, col) lists
 * the sources i of the edges i -> j, sorted and distinct (validated as a
 * CSR pattern; MXS_INVALID_MATRIX otherwise); every edge has weight one.
 * mxs_graph_create counts out-degrees d_i on the GPU and stores the
 * transition matrix T[j,i] = 1/d_i as an F64 CSR matrix
 * (mxs_graph_transition; it may be converted to any format and passed as
 * `op`) and the set D of nodes without out-links.  flags: MXS_HOST_PTRS or
 * MXS_DEVICE_PTRS (repeated edges are rejected: MXS_SORT_AND_SUM is not
 * accepted here). */
typedef struct mxs_graph mxs_graph;

typedef struct {
  int64_t iters;    /* power steps taken */
  double delta;     /* ||x_k - x_{k-1}||_1 of the last step */
  int32_t status;
} mxs_pagerank_info;

mxs_status mxs_graph_create(mxs_ctx* ctx, int64_t n, int64_t nnz, const int32_t* rowptr,
                            const int32_t* col, int32_t flags, mxs_graph** out);
mxs_status mxs_graph_destroy(mxs_graph* G);
/* The transition matrix T owned by G (valid until mxs_graph_destroy). */
const mxs_matrix* mxs_graph_transition(const mxs_graph* G);

/* From x_0 = 1/n: x_{k+1} = damping (T x_k + m_k/n) + (1 - damping)/n with
 * m_k = sum of x_k over D, until ||x_{k+1} - x_k||_1 <= tol (MXS_OK) or
 * max_iters steps (0 = 1000; MXS_NOT_CONVERGED).  x: device FP64 vector of
 * n entries (output).  op: NULL for T, else T in another format.  damping
 * in [0, 1).  Every reduction is in fixed order (no floating-point
 * atomics), so the result is reproducible.  Synchronises the ctx stream. */
mxs_status mxs_pagerank(mxs_ctx* ctx, const mxs_graph* G, const mxs_matrix* op, double damping,
                        double tol, int64_t max_iters, double* x, mxs_pagerank_info* info);

/* ---------------------------------------------------------------------- */
/* batched CG and continuous batching                                      */
/* ---------------------------------------------------------------------- */
/* Not in the paper: many independent SPD systems A_i x_i = b_i solved by
 * the CG of the solvers above, one work-group per system, in a persistent
 * kernel per size class captured in one hipGraph per step.  The engine
 * holds the systems' matrices and Krylov state in a device arena of
 * budget_bytes; requests wait in a FIFO and are admitted (first fit, with a
 * starvation guard) when their class has a free slot and their footprint
 * 4(n+1) + 12 nnz + 32 n bytes (rounded to 256-byte pieces) fits the arena.
 * A system's arithmetic depends only on its own data and on its class's
 * threads-per-system (a function of n alone), so each result is bitwise
 * identical whether it ran alone or among others. */
typedef struct mxs_batch mxs_batch;

typedef struct {
  size_t budget_bytes;      /* device arena for matrices and vectors */
  int32_t max_slots;        /* systems resident at once (all classes) */
  int32_t iters_per_step;   /* CG iterations per slot per step (0 = 16) */
  int32_t nclasses;         /* 0 = defaults (n <= 1024, 2304, 4096, 8192, 10240 with 256, 256,
                               512, 1024, 1024 threads per system; below 5 slots the
                               8192 class is left out) */
  int32_t class_max_n[8];   /* increasing upper bounds of n per class */
  int32_t class_block[8];   /* threads per system: 128, 256, 512 or 1024 (autotuner output) */
  int32_t class_slots[8];   /* slots per class; 0 = an even share of the rest */
  size_t staging_bytes;     /* pinned host pool holding submitted inputs until their first
                               step; 0 = min(budget_bytes, 1 GiB).  Requests beyond it are
                               kept as ordinary host copies and packed at admission. */
} mxs_batch_opts;

typedef struct {
  int32_t active;           /* slots still holding a system after this step */
  int32_t pending;          /* submitted, not yet admitted */
  int32_t slots;
  int32_t reserved;
  int64_t completed;        /* systems retired so far */
  int64_t arena_used, arena_size;
} mxs_batch_stats;

/* Threads: submissions (mxs_batch_submit, mxs_batch_submit_many) may run on
 * one thread while another steps, polls and lists completed tickets; the
 * engine serializes its queue, pools and results internally and holds its
 * lock neither while a submission validates and packs its inputs nor while
 * a step is waited for.  Two steps, or create/destroy, must not overlap
 * other calls on the same batch. */
mxs_status mxs_batch_create(mxs_ctx* ctx, const mxs_batch_opts* opts, mxs_batch** out);
mxs_status mxs_batch_destroy(mxs_batch* batch);

/* Queues A x = b (host CSR arrays and b, copied before the call returns;
 * x0 = 0) to relative tolerance rel_tol (relative to ||b||).  MXS_BUDGET if
 * its footprint alone exceeds the arena (or its inputs the pinned staging
 * pool), MXS_UNSUPPORTED if n exceeds the
 * largest class, MXS_INVALID_MATRIX if the CSR is malformed (checked on the
 * host). */
mxs_status mxs_batch_submit(mxs_batch* batch, int64_t n, int64_t nnz, const int32_t* rowptr,
                            const int32_t* col, const double* val, const double* b,
                            double rel_tol, int64_t max_iters, uint64_t* ticket);

/* One request of mxs_batch_submit_many: the arguments of mxs_batch_submit. */
typedef struct {
  int64_t n, nnz;
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  const double* b;
  double rel_tol;
  int64_t max_iters;        /* 0 = 20000 (refinement mode: inner iterations in total) */
  int32_t mode;             /* MXS_BATCH_FP64 or MXS_BATCH_IR_FP32 */
  int32_t reserved;
  double inner_rel_tol;     /* refinement mode: inner tolerance, 0 = 1e-4 */
} mxs_batch_request;

/* Batch modes.  MXS_BATCH_FP64: CG in FP64.  MXS_BATCH_IR_FP32: the
 * mixed-precision scheme of mxs_solve_ir with an F32 copy of the values
 * (rounded to nearest by the kernel on the request's first step): FP64
 * residual r = b - A x and update x += ||r|| d, inner FP32 CG on
 * A d = r / ||r|| to inner_rel_tol (reductions accumulated in FP64),
 * at most 50 outer steps; the footprint grows by 4 nnz bytes.  Its result
 * reports inner iterations in total as `iters` and outer steps as
 * `restarts`. */
#define MXS_BATCH_FP64 0
#define MXS_BATCH_IR_FP32 1

/* Queues `count` requests as mxs_batch_submit would, validating and
 * packing them on up to 16 host threads.  tickets[i] receives request i's
 * ticket (0 if it was rejected) and statuses[i] its status (the codes of
 * mxs_batch_submit); tickets are issued in array order.  Returns
 * MXS_INVALID_ARG for bad arguments of the call itself, else MXS_OK. */
mxs_status mxs_batch_submit_many(mxs_batch* batch, int64_t count, const mxs_batch_request* reqs,
                                 uint64_t* tickets, mxs_status* statuses);

/* One step: admit waiting requests, run iters_per_step CG iterations on
 * every resident system, read their states back and retire the systems
 * that finished (their results can be polled when this returns).
 * Synchronous.  Per step the host exchanges three things with the device
 * whatever the number of requests: the slot descriptor table (up), the
 * slot state table (down) and the graph launch; a new slot's inputs are
 * pulled by its work-group from pinned host memory (packed there once at
 * submit) and a finished slot's x is written by its work-group into pinned
 * host memory. */
mxs_status mxs_batch_step(mxs_batch* batch, mxs_batch_stats* stats);

/* mxs_batch_step in two halves, so that host work overlaps the device's.
 * mxs_batch_step_launch admits waiting requests and launches the step
 * without waiting for it; mxs_batch_step_finish waits for it, retires the
 * finished systems and fills stats (nullable).  Between the two the caller
 * may submit (the packing of new inputs then overlaps the step), poll and
 * list completed tickets; a second launch before the finish, or a finish
 * without a launch, returns MXS_INVALID_ARG.  mxs_batch_destroy waits for a
 * launched step. */
mxs_status mxs_batch_step_launch(mxs_batch* batch);
mxs_status mxs_batch_step_finish(mxs_batch* batch, mxs_batch_stats* stats);

/* MXS_PENDING while the request runs or waits; otherwise copies x (n
 * doubles) to x_host (nullable), fills info (nullable), forgets the ticket
 * and returns the solve's status (MXS_OK when it converged). */
mxs_status mxs_batch_poll(mxs_batch* batch, uint64_t ticket, double* x_host,
                          mxs_solve_info* info);

/* mxs_batch_poll for `count` tickets in one call (one lock, one crossing of
 * the boundary): request i's x (n_i doubles) goes to x_host + x_off[i]
 * (offsets in doubles, the caller's layout; x_host nullable), its info to
 * infos[i] (infos nullable) and the status mxs_batch_poll would return to
 * statuses[i]; a PENDING request's x and info are left untouched and its
 * ticket is kept.  Returns MXS_INVALID_ARG for bad arguments of the call
 * itself (count < 0, NULL tickets or statuses, NULL x_off with x_host),
 * else MXS_OK; an unknown ticket gets MXS_INVALID_ARG in statuses[i]. */
mxs_status mxs_batch_poll_many(mxs_batch* batch, int64_t count, const uint64_t* tickets,
                               double* x_host, const int64_t* x_off, mxs_solve_info* infos,
                               mxs_status* statuses);

/* Moves up to `cap` tickets retired since the previous call into
 * tickets[] (oldest first); *count receives how many were written. */
mxs_status mxs_batch_completed(mxs_batch* batch, uint64_t* tickets, int64_t cap, int64_t* count);

/* The configuration of size class `cls` (for reports and the autotuner). */
mxs_status mxs_batch_config(const mxs_batch* batch, int32_t cls, int32_t* max_n, int32_t* block,
                            int32_t* rows_per_thread, int32_t* slots, int32_t* uses_lds);

/* ---------------------------------------------------------------------- */
/* measurement                                                             */
/* ---------------------------------------------------------------------- */
typedef struct {
  double read_gbs;   /* sum-reduction over one array (the faster of ordinary
                        and non-temporal loads, as the products use both) */
  double copy_gbs;   /* b = a                                  */
  double triad_gbs;  /* a = b + s*c                            */
  double best_gbs;   /* max of the three                       */
} mxs_bw_result;

/* Attainable HBM bandwidth, in the spirit of the BabelStream runs of the
 * paper's "Bandwidth Tests and Roofline Performance Model" subsection:
 * `bytes` per array (>= 1 GiB recommended, well beyond the 256 MB
 * Infinity Cache), `reps` timed repetitions per kernel (best kept).
 * Counts bytes read + written.  Synchronises the ctx stream. */
mxs_status mxs_hbm_probe(mxs_ctx* ctx, size_t bytes, int reps, mxs_bw_result* out);

/* Random-gather throughput, the ceiling of SpMV on matrices whose columns
 * are scattered over all of x (the power-law patterns): each entry's x load
 * then touches a cache line of its own, so gathers per second, not HBM
 * bytes, bound the product.  Times `count` loads x[idx[k]] from an x of `nx`
 * values of `value_bytes` (4 or 8), idx uniform over [0, nx) (a fixed hash
 * of k, streamed as int32), eight gathers per thread in flight; best of
 * `reps` runs after a warm-up run (x stays in whatever cache level holds
 * it).  Writes gathers per second.  Synchronises the ctx stream. */
mxs_status mxs_gather_probe(mxs_ctx* ctx, int64_t nx, int64_t count, int value_bytes, int reps,
                            double* gathers_per_s);

/* Reads `bytes` bytes of a ctx-owned scratch buffer (written once, when it
 * is allocated or grown) so that later reads of other data come from HBM
 * rather than from the last-level cache; the caches are left holding clean
 * lines, so the next kernel pays no write-backs for them.  Asynchronous. */
mxs_status mxs_flush_cache(mxs_ctx* ctx, size_t bytes);

const char* mxs_status_string(mxs_status s);
const char* mxs_last_error(const mxs_ctx* ctx);
const char* mxs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MXS_H */
