/*
 * gko.h -- C ABI of the MI355X (gfx950) sparse linear-algebra library.
 *
 * The operations are the ones the paper benchmarks: sparse matrix-vector
 * products in several storage formats (Sec. 6.1) and memory-bound Krylov
 * solvers built on them (Sec. 6.2).  Device memory and streams are supplied
 * by the caller (in practice PyTorch); every compute step runs in this
 * library's own HIP kernels.
 *
 * Conventions for every call:
 *  - Pointers named as device pointers must point to device memory on the
 *    context's GPU, suitably aligned for their element type.  The library
 *    never takes ownership of caller memory.
 *  - Column indices are int32.  Row offsets are int32 internally; int64 row
 *    offsets are accepted at creation when nnz < 2^31.
 *  - Work is enqueued on the context's stream.  Calls documented as
 *    asynchronous return before the GPU finishes; caller buffers must stay
 *    valid until the stream reaches the call.
 *  - No call aborts or throws.  Every call returns a gko_status; on failure
 *    gko_last_error() returns a message for the calling thread.
 *  - A context and everything created from it belong to one host thread at a
 *    time (like a BLAS handle).
 */
#ifndef GKO_MI355X_H
#define GKO_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gko_status {
    GKO_OK = 0,
    GKO_ERR_INVALID_ARG = 1,   /* bad pointer, size, option or malformed matrix */
    GKO_ERR_DIM_MISMATCH = 2,  /* operand shapes do not agree */
    GKO_ERR_UNSUPPORTED = 3,   /* valid request this library does not do (e.g. infeasible ELL) */
    GKO_ERR_ALLOC = 4,         /* device allocation failed */
    GKO_ERR_HIP = 5,           /* a HIP runtime call failed */
    GKO_ERR_NOT_CONVERGED = 6, /* iteration limit reached; x holds the last iterate */
    GKO_ERR_BREAKDOWN = 7,     /* NaN/Inf, or a zero denominator in the recurrence */
    GKO_ERR_NOT_SPD = 8        /* CG found p^T A p <= 0 */
} gko_status;

typedef enum gko_dtype { GKO_F64 = 0, GKO_F32 = 1 } gko_dtype;
typedef enum gko_itype { GKO_I32 = 0, GKO_I64 = 1 } gko_itype;

/* Storage formats of the SpMV family (Sec. 6.1 compares SpMV kernels that
 * differ in storage format and processing strategy).
 *  CSR       : row offsets, columns, values; a subwarp of w lanes per row,
 *              w in {1,...,64} picked from the mean row length.
 *  CSR_MERGE : the same arrays plus a merge-path partition; equal shares of
 *              (rows + nonzeros) per workgroup, independent of row lengths.
 *  COO       : row-major sorted (row, col, val) triplets; equal nonzero
 *              shares per wavefront, segmented reduction keyed on row.
 *  ELL       : column-major padded slots, width K = longest row, leading
 *              dimension n rounded up to 64, padding col = -1, val = +0.0.
 *  HYBRID    : ELL of width K* plus a COO tail holding the rest, where K*
 *              minimises n*K*(s+4) + (s+8)*tail(K) bytes (s = value size),
 *              ties to the smaller K.
 *  AUTO      : (gko_convert only) the context's selector model if one is set
 *              (gko_context_set_selector), else the fastest by timing of the
 *              six formats CSR, CSR_MERGE, COO, ELL, HYBRID and SELLP.
 *  SELLP     : sliced ELL with padding (Anzt, Tomov and Dongarra 2014), not
 *              sorted, stride factor 1: slices of 64 consecutive rows, slice s
 *              padded to its own longest row w_s and column-major inside the
 *              slice.  Entry j of row i = 64 s + r is slot sets[s] + 64 j + r,
 *              sets[0] = 0, sets[s+1] = sets[s] + 64 w_s; padding (and rows
 *              >= n_rows of the last slice) is col = -1, val = +0.0.  AUTO
 *              and the selector score it beside the five formats of Sec. 6.1
 *              (six classes). */
typedef enum gko_format {
    GKO_FMT_CSR = 0,
    GKO_FMT_CSR_MERGE = 1,
    GKO_FMT_COO = 2,
    GKO_FMT_ELL = 3,
    GKO_FMT_HYBRID = 4,
    GKO_FMT_AUTO = 5,
    GKO_FMT_SELLP = 6
} gko_format;

typedef struct gko_context_s *gko_context;
typedef struct gko_matrix_s *gko_matrix;

/* ---------------------------------------------------------------- context */

/* Create a context bound to hip_stream (a hipStream_t; NULL = the null
 * stream) on the current HIP device.  *out receives the handle. */
gko_status gko_context_create(void *hip_stream, gko_context *out);
gko_status gko_context_destroy(gko_context ctx);
/* Rebind the context to another stream of the same device. */
gko_status gko_context_set_stream(gko_context ctx, void *hip_stream);

/* Device allocator used for every buffer the library owns (matrix storage,
 * solver workspaces).  alloc(bytes, stream, user) returns device memory or
 * NULL; dealloc(ptr, stream, user) releases it.  Passing NULL for both
 * restores the default (hipMallocAsync / hipFreeAsync on the context
 * stream).  Must be called before matrices are created. */
typedef void *(*gko_alloc_fn)(size_t bytes, void *stream, void *user);
typedef void (*gko_dealloc_fn)(void *ptr, void *stream, void *user);
gko_status gko_context_set_allocator(gko_context ctx, gko_alloc_fn alloc,
                                     gko_dealloc_fn dealloc, void *user);

/* ---------------------------------------------------------------- matrices */

/* Create a matrix in CSR format from caller-owned device arrays, which are
 * copied: the handle owns its storage and the caller may free its arrays
 * once the call returns (the call synchronises the stream).
 *   row_ptr : n_rows + 1 offsets of type row_ptr_type, row_ptr[0] = 0,
 *             non-decreasing, row_ptr[n_rows] = nnz.
 *   col_idx : nnz int32 columns in [0, n_cols), strictly increasing per row.
 *   values  : nnz values of type dt.
 * The structure is validated on the device; a violation returns
 * GKO_ERR_INVALID_ARG and creates nothing. */
gko_status gko_matrix_create_csr(gko_context ctx, int64_t n_rows, int64_t n_cols, int64_t nnz,
                                 gko_dtype dt, const void *row_ptr, gko_itype row_ptr_type,
                                 const int32_t *col_idx, const void *values, gko_matrix *out);
gko_status gko_matrix_destroy(gko_matrix A);
/* Deep copy (same format and storage). */
gko_status gko_matrix_clone(gko_matrix A, gko_matrix *out);

typedef struct gko_matrix_desc {
    int32_t format;        /* gko_format currently stored */
    int32_t dtype;         /* gko_dtype */
    int64_t n_rows, n_cols, nnz;
    int64_t ell_width;     /* ELL / HYBRID: K (slots per row), else 0 */
    int64_t ell_ld;        /* ELL / HYBRID: leading dimension, else 0 */
    int64_t coo_nnz;       /* COO: nnz; HYBRID: tail entries; else 0 */
    int64_t stored_bytes;  /* bytes of device storage held by the handle */
    int32_t csr_kernel;    /* CSR: 0 = the row-per-thread kernel (entries staged through LDS,
                              csr_row_lanes lanes per row), else the lanes of the subwarp per
                              row reading its entries from memory; other formats: -1 */
    int32_t max_row_len;   /* longest row (-1 where not yet computed) */
    int64_t csr_long_rows; /* CSR: rows handed to the workgroup-per-row kernel, else 0 */
    int64_t sellp_slices;  /* SELLP: ceil(n_rows / sellp_slice), else 0 */
    int64_t sellp_slots;   /* SELLP: sets[sellp_slices], slots incl. padding, else 0 */
    int32_t sellp_slice;   /* SELLP: rows per slice (64), else 0 */
    int32_t csr_row_lanes; /* CSR with csr_kernel 0: lanes per row (1 for a mean row length
                              below 12, 4 below 56, else 8), else 0 */
    int64_t sellp_wide_slices; /* SELLP: slices wider than 512 slots, summed by column chunks */
} gko_matrix_desc;
gko_status gko_matrix_describe(gko_matrix A, gko_matrix_desc *out);

/* Export the logical matrix as CSR into caller device buffers (n_rows+1
 * int32 offsets, nnz columns, nnz values), whatever the stored format; the
 * stored format is not changed.  Synchronises the stream. */
gko_status gko_matrix_export_csr(gko_matrix A, int32_t *row_ptr, int32_t *col_idx, void *values);
/* Export the raw stored arrays (for layout checks).  Each pointer may be
 * NULL to skip it; the call fails with GKO_ERR_INVALID_ARG if the format
 * stores no such array.  Sizes follow gko_matrix_desc:
 *   ell_col/ell_val   : ell_width * ell_ld     (ELL, HYBRID)
 *   coo_row/coo_col/coo_val : coo_nnz          (COO; HYBRID tail) */
gko_status gko_matrix_export_storage(gko_matrix A, int32_t *ell_col, void *ell_val,
                                     int32_t *coo_row, int32_t *coo_col, void *coo_val);
/* Export the SELL-P arrays of a matrix stored as SELLP (else
 * GKO_ERR_INVALID_ARG) into caller device buffers; NULL skips an array.
 *   slice_sets   : sellp_slices + 1 int64 slot offsets
 *   slice_widths : sellp_slices int32 widths
 *   col / val    : sellp_slots columns (int32) / values (the matrix dtype)
 * Synchronises the stream. */
gko_status gko_matrix_export_sellp(gko_matrix A, int64_t *slice_sets, int32_t *slice_widths,
                                   int32_t *col, void *val);

/* ---------------------------------------------------------------- SpMV (Sec. 6.1) */

/* y <- alpha * A * x + beta * y in A's value type (alpha and beta rounded to
 * it).  x: n_cols device values, y: n_rows device values, both of A's dtype.
 * beta == 0 means y is not read.  With no entries, y <- beta y and x is not
 * read (it may be NULL when n_cols == 0).  x and y must not overlap
 * (GKO_ERR_INVALID_ARG).  Asynchronous; deterministic (bitwise repeatable). */
gko_status gko_spmv(gko_matrix A, double alpha, const void *x, double beta, void *y);

/* Convert A's storage in place to fmt; the logical matrix is unchanged.
 * Converting between any two formats is bit-exact.  ELL and SELLP are
 * refused with GKO_ERR_UNSUPPORTED (A unchanged) when their padded slots
 * would exceed 4x the CSR storage.  GKO_FMT_AUTO asks the context's selector model, or
 * without one times one SpMV in every feasible format and keeps the fastest.
 * Synchronises the stream. */
gko_status gko_convert(gko_matrix A, gko_format fmt);

/* ---------------------------------------------------------------- reductions */

/* *result (device, one double) <- sum_i x_i y_i, and <- ||x||_2 for
 * gko_norm2.  x, y: n device values of dtype dt.  Accumulates in FP64 with a
 * fixed reduction tree (bitwise repeatable).  Asynchronous. */
gko_status gko_dot(gko_context ctx, gko_dtype dt, int64_t n, const void *x, const void *y,
                   double *result);
gko_status gko_norm2(gko_context ctx, gko_dtype dt, int64_t n, const void *x, double *result);

/* ---------------------------------------------------------------- bandwidth probe */

/* STREAM-style kernels on FP64 device arrays of n elements, the achievable
 * bandwidth that the paper measures before its SpMV and solver results
 * (Sec. 6):  GKO_STREAM_COPY: c[i] = a[i];  GKO_STREAM_TRIAD: c[i] = a[i] + s * b[i]
 * (multiply and add rounded separately).  b is ignored by COPY.  c must not
 * overlap a or b.  Asynchronous.  Also serves as a transfer of known size
 * for scaling hardware byte counters. */
typedef enum gko_stream_op { GKO_STREAM_COPY = 0, GKO_STREAM_TRIAD = 1 } gko_stream_op;
gko_status gko_stream(gko_context ctx, gko_stream_op op, int64_t n, const double *a,
                      const double *b, double s, double *c);

/* Random-gather probe, the ceiling of an SpMV whose x gathers miss the L2:
 * y[i] = x[idx[i]] for i < n (x: m FP64 values, idx: n int32 indices; an
 * index outside [0, m) reads 0).  Index and output streams bypass the caches
 * (non-temporal) as an SpMV's matrix streams do.  idx and y 16-byte aligned,
 * 1 <= m < 2^28, x and y must not overlap (else GKO_ERR_INVALID_ARG).
 * Asynchronous. */
gko_status gko_gather_probe(gko_context ctx, int64_t n, const double *x, int64_t m,
                            const int32_t *idx, double *y);

/* ---------------------------------------------------------------- Krylov solvers (Sec. 6.2) */

typedef enum gko_precision { GKO_PREC_FP64 = 0, GKO_PREC_MIXED_IR = 1 } gko_precision;
typedef enum gko_precond { GKO_PRECOND_NONE = 0, GKO_PRECOND_BLOCK_JACOBI = 1 } gko_precond;

typedef struct gko_solver_opts {
    int32_t precision;   /* gko_precision; MIXED_IR = FP64 refinement around an FP32 inner PCG */
    int32_t precond;     /* gko_precond */
    int32_t block_size;  /* block-Jacobi block size: 1, 2, 4, 8 or 16 (default 8) */
    int32_t check_every; /* host convergence polls every this many iterations (default 16) */
    double inner_tol;    /* MIXED_IR: inner relative tolerance (default 1e-5) */
    int32_t max_inner;   /* MIXED_IR: inner iteration cap per outer step (default 1000) */
    int32_t max_outer;   /* MIXED_IR: outer step cap (default 20) */
    int32_t single_workgroup; /* 1 (default): FP64 unpreconditioned CG on a CSR matrix whose
                                 direction vector fits in one workgroup's LDS (n up to 8192 on
                                 gfx950), and GMRES on a CSR matrix of up to 4096 rows with a
                                 restart length of up to 64, run as one launch on one
                                 workgroup; 0: always the multi-kernel path.  Same steps and
                                 stopping tests either way. */
    int32_t krylov_dim;  /* GMRES restart length m, 1..128 (default 30) */
    int32_t graphs;      /* 1 (default): on matrices of at most 2^20 rows, the multi-kernel
                            CG, flexible CG, pipelined CG, BiCGSTAB and CGS loops capture one
                            polling interval (check_every iterations of kernel launches) into
                            a HIP graph once per solve and replay it on the context stream;
                            0: always launch kernel by kernel.  The graph holds the same
                            kernels with the same arguments, so results are identical. */
} gko_solver_opts;

typedef struct gko_solve_info {
    int32_t status;            /* gko_status of the solve */
    int32_t iterations;        /* Krylov iterations (FP64) or total inner iterations (MIXED_IR) */
    int32_t outer_iterations;  /* MIXED_IR refinement steps, GMRES cycles, else 0 */
    int32_t restarts;          /* true-residual restarts */
    double rel_residual;       /* recursive ||r|| / ||b|| at exit */
    double true_rel_residual;  /* ||b - A x|| / ||b|| recomputed at exit */
    double seconds;            /* wall time of the solve call */
    double setup_seconds;      /* part of it spent building the preconditioner */
    int32_t reorthogonalized;  /* GMRES: Arnoldi steps that took a second Gram-Schmidt round */
    int32_t pad;
} gko_solve_info;

gko_status gko_context_set_solver_opts(gko_context ctx, const gko_solver_opts *opts);
gko_status gko_context_get_solver_opts(gko_context ctx, gko_solver_opts *out);
gko_status gko_context_get_solve_info(gko_context ctx, gko_solve_info *out);

/* Solve A x = b by (preconditioned) CG, Hestenes-Stiefel form: q = A p,
 * alpha = rho / p.q, x += alpha p, r -= alpha q, z = M^-1 r, rho' = r.z,
 * p = z + (rho'/rho) p.  A square, SPD, FP64.  b, x: device FP64 arrays of
 * n_rows; x is the initial guess on entry and the solution on return.  Stops
 * when ||r||_2 <= tol ||b||_2; the true residual is then recomputed and the
 * iteration restarted from x if it misses tol (at most twice).  ||b|| = 0
 * gives x = 0.  tol > 0 and finite, maxit >= 0; with MIXED_IR precision
 * maxit caps the inner iterations summed over all refinement steps.  b and x
 * must not overlap (GKO_ERR_INVALID_ARG).  Synchronous.  Returns GKO_OK,
 * GKO_ERR_NOT_CONVERGED, GKO_ERR_NOT_SPD or GKO_ERR_BREAKDOWN. */
gko_status gko_cg_solve(gko_matrix A, const void *b, void *x, double tol, int32_t maxit);

/* gko_cg_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same CG, from the same kernels, with every work buffer (r, p, q, the
 * reduction partials and ticket, the iteration scalars) in one static device
 * array of GKO_NOALLOC_SCRATCH_BYTES that the library holds on each device
 * until the process ends.  It calls no hipMalloc, hipFree or other allocating
 * routine, and launches kernel by kernel (no HIP graph is instantiated); it
 * still copies the iteration scalars to the host and synchronizes the stream
 * to test convergence.  The caller passes A, b and x as for gko_cg_solve.
 *   Requires precision FP64 and no preconditioner (else GKO_ERR_UNSUPPORTED),
 *   and n_rows <= GKO_CG_NOALLOC_MAX_ROWS (else GKO_ERR_INVALID_ARG, nothing
 *   launched).  Small CSR systems take the single-workgroup launch as in
 *   gko_cg_solve.  Results are bitwise those of gko_cg_solve (its graph
 *   replay does not change them).
 *   Every call on a device shares that device's array, which keeps the last
 *   call's contents (each call clears what must start at zero): calls that
 *   overlap on one device, from several streams or host threads, race. */
#define GKO_NOALLOC_SCRATCH_BYTES (64u << 20)
#define GKO_CG_NOALLOC_MAX_ROWS 2752448
gko_status gko_cg_solve_noalloc(gko_matrix A, const void *b, void *x, double tol, int32_t maxit);

/* Flexible CG (Notay 2000, one previous direction kept conjugate): CG with
 * the Polak-Ribiere coefficient beta = z'.(r' - r) / (z.r), which keeps
 * consecutive directions A-conjugate also when the preconditioner is not a
 * fixed symmetric operator; with the library's fixed SPD preconditioners it
 * agrees with CG up to rounding.  The same options (precision, precond,
 * block_size, check_every), stopping test, restarts, statuses and solve info
 * as gko_cg_solve; no single-workgroup path. */
gko_status gko_fcg_solve(gko_matrix A, const void *b, void *x, double tol, int32_t maxit);

/* Pipelined (P)CG (Ghysels and Vanroose, Parallel Computing 40, 2014): CG
 * rearranged so that u = M^-1 r and w = A u are carried by recurrences and
 * each iteration needs one product and one fused vector kernel with a single
 * reduction (r.u, w.u, r.r), at the price of more vector traffic (13 vector
 * passes per iteration without a preconditioner, CG's fused path 9).  Equal
 * to CG's iterates in exact arithmetic; its recursive residual drifts
 * further from the true one, which the true-residual check and restarts
 * catch.  The same options, stopping test, statuses and solve info as
 * gko_cg_solve; no single-workgroup path. */
gko_status gko_pipecg_solve(gko_matrix A, const void *b, void *x, double tol, int32_t maxit);

/* Solve A x = b by unpreconditioned BiCGSTAB (van der Vorst), shadow
 * residual r0, same conventions as gko_cg_solve.  Breakdown (|rho|, |rhat.v|
 * or t.t below 1e-300, or omega = 0) returns GKO_ERR_BREAKDOWN. */
gko_status gko_bicgstab_solve(gko_matrix A, const void *b, void *x, double tol, int32_t maxit);

/* Solve A x = b by unpreconditioned CGS (Sonneveld 1989; Saad Alg. 7.5),
 * shadow residual rhat = r0: t = A p, alpha = rho / t.rhat, q = u - alpha t,
 * x += alpha (u + q), r -= alpha A (u + q), rho' = r.rhat,
 * u = r + (rho'/rho) q, p = u + beta (q + beta p).  A square, FP64.  Stops
 * when the recursive ||r||_2 <= tol ||b||_2; the true relative residual is
 * reported in the solve info (CGS's recursive residual can drift from it),
 * no restart.  Breakdown when |rho| or |t.rhat| falls below 1e-300.  Same
 * argument conventions as gko_cg_solve; returns GKO_OK,
 * GKO_ERR_NOT_CONVERGED or GKO_ERR_BREAKDOWN. */
gko_status gko_cgs_solve(gko_matrix A, const void *b, void *x, double tol, int32_t maxit);

/* Solve A x = b by restarted GMRES(m) (Saad and Schultz 1986), m =
 * krylov_dim of the solver options, unpreconditioned, FP64.  A cycle starts
 * from r = b - A x, builds an orthonormal Krylov basis by classical
 * Gram-Schmidt (a second round when the first leaves less than 1/sqrt(2) of
 * the vector's length), reduces the Hessenberg matrix by Givens rotations,
 * and ends after m steps, when the least-squares residual estimate reaches
 * tol ||b||_2, on an invariant subspace, or at maxit; then x += V y.  The
 * next cycle's true residual decides convergence.  Device memory: (m + 1)
 * basis vectors of n_rows doubles.  iterations counts Arnoldi steps and
 * outer_iterations the cycles; rel_residual is the last estimate.  Same
 * argument conventions as gko_cg_solve; returns GKO_OK,
 * GKO_ERR_NOT_CONVERGED or GKO_ERR_BREAKDOWN. */
gko_status gko_gmres_solve(gko_matrix A, const void *b, void *x, double tol, int32_t maxit);

/* ---------------------------------------------------------------- batched CG */

typedef struct gko_batch_s *gko_batch;

/* Create a batch of nsys independent square systems from caller device
 * arrays, which are copied (the call synchronises the stream):
 *   row_off[nsys+1] (int64): system i has rows row_off[i] .. row_off[i+1]-1
 *                            of the concatenated vectors; 1 <= m_i <= 2048.
 *   nnz_off[nsys+1] (int64): its entries are nnz_off[i] .. nnz_off[i+1]-1.
 *   row_ptr_local          : m_i + 1 local offsets per system (starting at 0),
 *                            stored back to back from index row_off[i] + i.
 *   col_idx (int32)        : local column indices in [0, m_i).
 *   values                 : FP64 or FP32 (dt).
 * Systems are queued largest first (by rows, then nonzeros) for the solve.  A malformed
 * system returns GKO_ERR_INVALID_ARG. */
gko_status gko_batch_create_csr(gko_context ctx, int64_t nsys, const int64_t *row_off,
                                const int64_t *nnz_off, const int32_t *row_ptr_local,
                                const int32_t *col_idx, const void *values, gko_dtype dt,
                                gko_batch *out);
gko_status gko_batch_destroy(gko_batch B);

/* Solve every system by CG from x = 0 in ONE persistent kernel launch: each
 * workgroup takes systems from an atomic queue and iterates one system at a
 * time with its vectors in LDS, so no host round trip happens until all are
 * done.  FP64 batches run FP64 CG; FP32 batches run FP32 CG iterations inside
 * FP64 iterative refinement (residual, norms and update in FP64).
 *   b, x            : FP64 device arrays of row_off[nsys] entries (x is output);
 *                     they must not overlap (GKO_ERR_INVALID_ARG).
 *   tol             : per-system stop ||b_i - A_i x_i||_2 <= tol ||b_i||_2.
 *   maxit           : iteration cap per system (inner iterations for FP32).
 *   iters_out       : device int32[nsys], iterations used.
 *   relres_out      : device double[nsys], true relative residual at exit.
 * Synchronous.  Returns GKO_OK if every system converged, else the worst of
 * GKO_ERR_NOT_CONVERGED, GKO_ERR_BREAKDOWN, GKO_ERR_NOT_SPD (inspect the
 * per-system outputs). */
gko_status gko_batch_cg_solve(gko_batch B, const double *b, double *x, double tol, int32_t maxit,
                              int32_t *iters_out, double *relres_out);

/* Workgroup size used by gko_batch_cg_solve: 64, 128, 256 or 512 threads.
 * A new batch starts from the autotune cache's choice (size and LDS mode)
 * for its device architecture and shape (dtype, nsys, total rows, nnz,
 * largest system) when the cache holds one, else from 64 (largest system
 * <= 256 rows) or 128 threads with the direction-only LDS mode where it fits. */
gko_status gko_batch_set_block(gko_batch B, int32_t block);
gko_status gko_batch_get_block(gko_batch B, int32_t *block);

/* What the persistent kernel keeps in LDS, and how many systems a workgroup
 * solves at a time.  ALL: x, r, p and q of the current system (rows that do
 * not fit the register cache are read from memory each iteration).
 * DIRECTION: every system's rows (up to 5 entries, up to min(4, 1024 /
 * block) rows per thread) and its x, r and q stay in registers and only the
 * direction p goes through LDS (m doubles per workgroup instead of 4m):
 * FP64 batches whose every system fits the register cache at the workgroup
 * size.  WAVE_SYSTEMS: systems of at most 256 rows are solved one per
 * wavefront with their rows in registers (block / 64 of them per workgroup
 * at a time, each wavefront taking its own systems from the queue, sums
 * within the wavefront and no workgroup barrier); larger systems take the
 * whole workgroup.  FP64 batches use it with the DIRECTION layout (where
 * DIRECTION fits), FP32 batches with the ALL layout (where every row has at
 * most 5 entries).  set_lds_mode fails with GKO_ERR_UNSUPPORTED where the
 * mode does not fit; a later set_block to a size where it does not fit
 * falls back to ALL.  get_lds_mode returns the mode in effect. */
typedef enum gko_batch_lds {
    GKO_BATCH_LDS_ALL = 0,
    GKO_BATCH_LDS_DIRECTION = 1,
    GKO_BATCH_WAVE_SYSTEMS = 2
} gko_batch_lds;
gko_status gko_batch_set_lds_mode(gko_batch B, int32_t mode);
gko_status gko_batch_get_lds_mode(gko_batch B, int32_t *mode);

/* The launch gko_batch_cg_solve makes at the current workgroup size: how
 * many workgroups are resident on the device at once (the persistent grid,
 * capped by nsys at launch) and the dynamic LDS each takes (the iteration
 * vectors of the largest system).  Host outputs. */
gko_status gko_batch_launch_info(gko_batch B, int32_t *resident_workgroups,
                                 int64_t *lds_bytes_per_workgroup);

/* Time one full batched solve for each workgroup size (64, 128, 256, 512)
 * and mode of gko_batch_lds on the given right-hand sides and keep the
 * fastest pair for this batch.  times_ms[12] (host) receives the timings,
 * entry 3 j + mode for size j of that list (infinity where the mode does not
 * fit); *block_out
 * (host) the chosen size (gko_batch_get_lds_mode gives the mode).
 * x, iters and relres are scratch outputs as in gko_batch_cg_solve.
 * The choice is also stored in the on-disk autotune cache, a text file of
 * "key = block mode" lines: the file named by the environment variable
 * GKO_AUTOTUNE_CACHE (set but empty: no cache), else
 * $XDG_CACHE_HOME/gko_mi355x/autotune, else ~/.cache/gko_mi355x/autotune;
 * a file that cannot be written is skipped without an error. */
gko_status gko_batch_autotune(gko_batch B, const double *b, double *x, double tol, int32_t maxit,
                              int32_t *iters_out, double *relres_out, int32_t *block_out,
                              float *times_ms);

/* ---------------------------------------------------------------- format selector */

/* 32 structural features of A, in this order (FP32, host array):
 *  0 log10 n     1 log10 nnz     2 mean row length   3 std of row lengths
 *  4 cv          5 min length    6 max length        7/8/9 p50/p90/p99 length
 * 10 max/mean   11 frac empty rows   12 frac rows of length <= 4
 * 13 ELL padding n*max/nnz   14 HYB width / mean   15 HYB tail / nnz
 * 16 Gini of row lengths     17 entropy of the row-length distribution
 * 18 share of nnz in the longest ceil(n/100) rows
 * 19 log10 CSR working set (12 nnz + 4(n+1) + 8 n_cols + 8 n bytes)
 * 20 SELL-P padding: slots of the 64-row slices / nnz (1 when nnz = 0)
 * 21 n_cols / n   22 mean |i-j| / n_cols   23 max |i-j| / n_cols   24 frac i == j
 * 25 frac |i-j| <= 1   26 frac |i-j| <= 64   27 log10(1 + mean in-row column gap)
 * 28 frac of in-row gaps equal to 1   29 64-byte x segments touched per entry
 * 30 frac of entries whose transpose is stored (square only)
 * 31 log10(1 + mean column span of nonempty rows)
 * Percentile p: smallest L with #rows(len <= L) >= ceil(p n).  Synchronous. */
gko_status gko_matrix_features(gko_matrix A, float *features);

/* The SpMV formats the autotuner times and the selector scores, in this
 * order: CSR, CSR_MERGE, COO, ELL, HYBRID, SELLP. */
#define GKO_SELECTOR_CLASSES 6

/* Exhaustive autotune: time one SpMV of a clone of A in every format of the
 * GKO_SELECTOR_CLASSES list (mean of 5 after 2 warm-ups; infinity when a
 * format is infeasible).  A is not changed.  *best (host) receives the
 * fastest, times_ms[GKO_SELECTOR_CLASSES] (host, may be NULL) the timings. */
gko_status gko_autotune_format(gko_matrix A, gko_format *best, float *times_ms);

/* The selector network: an MLP 32 -> 64 -> 64 -> 6 (ReLU, ReLU, linear) on
 * z-scored features, FP32.  Output f predicts ln(t_f / t_best) for the six
 * formats in the order above; the selected format is the argmin among the
 * feasible ones (ELL and SELLP within the 4x storage limit).  Parameters
 * (6662 floats): W1[64][32], b1[64], W2[64][64], b2[64], W3[6][64], b3[6],
 * row-major (out x in). */
typedef struct gko_mlp_s *gko_mlp;

/* Create from initial parameters (host array of 6662 floats); normalisation
 * starts as mean 0, std 1; Adam state at zero. */
gko_status gko_mlp_create(gko_context ctx, const float *params, gko_mlp *out);
gko_status gko_mlp_destroy(gko_mlp M);
/* Copy parameters (6662) and normalisation (mean[32] then std[32]) to host;
 * either pointer may be NULL. */
gko_status gko_mlp_get_params(gko_mlp M, float *params, float *norm);
/* Per-feature mean and std (floored at 1e-6) of n samples X (device, n x 32). */
gko_status gko_mlp_fit_normalization(gko_mlp M, int64_t n, const float *X);
/* out (device, n x 6) <- network(X) for n samples X (device, n x 32). */
gko_status gko_mlp_forward(gko_mlp M, int64_t n, const float *X, float *out);
/* Masked mean squared loss L = sum mask (out - Y)^2 / sum mask over n samples
 * (X: n x 32, Y and mask: n x 6, device) and its gradient.  grad: device
 * float[6662], loss: device double.  The backward pass uses relu'(0) = 0. */
gko_status gko_mlp_loss_grad(gko_mlp M, int64_t n, const float *X, const float *Y,
                             const float *mask, float *grad, double *loss);
/* steps full-batch Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning
 * rate lr) on the GPU; the Adam state persists across calls.  loss_history
 * (device float[steps], may be NULL) receives the loss before each step. */
gko_status gko_mlp_train(gko_mlp M, int64_t n, const float *X, const float *Y, const float *mask,
                         int32_t steps, float lr, float *loss_history);
/* Save / load parameters and normalisation (binary: magic "GKOMLP1", version,
 * parameter count, arch string, norm[64], params[6662]; little endian).
 * Loading refuses a file whose parameter count differs. */
gko_status gko_mlp_save(gko_mlp M, const char *path);
gko_status gko_mlp_load(gko_context ctx, const char *path, gko_mlp *out);

/* Predicted-fastest feasible format of A; scores[6] (host, may be NULL)
 * receive the network outputs.  A is not changed. */
gko_status gko_select_format(gko_matrix A, gko_mlp model, gko_format *out, float *scores);
/* Model used by gko_convert(A, GKO_FMT_AUTO) on this context (NULL: time all
 * formats instead).  The context does not own the model. */
gko_status gko_context_set_selector(gko_context ctx, gko_mlp model);

/* ---------------------------------------------------------------- errors */

/* Message of the last failing call on this thread ("" if none). */
const char *gko_last_error(void);
const char *gko_status_string(gko_status s);

#ifdef __cplusplus
}
#endif

#endif /* GKO_MI355X_H */
