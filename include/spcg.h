/*
 * spcg.h -- C ABI of the MI355X (gfx950) CSR SpMV / conjugate-gradient library.
 *
 * The operations follow the data-parallel kernels of Weinberg, "Data-parallel
 * programming with Intel Array Building Blocks" (arXiv 1211.1581):
 *   - CSR storage in three arrays and the row-wise product y = A x (Sec. 3.2);
 *   - the conjugate-gradient solver for SPD systems (Sec. 3.4, Fig. 6 and the
 *     loop that follows it: one SpMV, two inner products, three vector updates
 *     per pass).
 * Beyond the paper: Jacobi, learned (M^-1 = G G^T, the network that predicts
 * G) and FSAI preconditioning, an FP32-inner / FP64-outer mixed-precision
 * solver, and the single-reduction (Chronopoulos-Gear) form of the loop.
 *
 * Conventions for every call:
 *   - Pointers prefixed d_ are device pointers (HBM of the current device),
 *     h_ are host pointers.  The caller owns all of them; the library never
 *     frees caller memory and never calls hipMalloc on a solve path (the
 *     matrix handle allocates its analysis arrays once, in spcg_csr_create).
 *   - Indices are int32, CSR column indices are 0-based, rows ascend.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls
 *     marked "asynchronous" only enqueue work on it.
 *   - Return value: an SPCG_* status code.  No exception crosses the ABI.
 *   - A handle may be used from one stream at a time.
 */
#ifndef SPCG_H
#define SPCG_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------------------- status codes */
#define SPCG_OK 0
#define SPCG_NOT_CONVERGED 1 /* x valid, maxit reached */
#define SPCG_FELL_BACK 2     /* learned form missed its budget or broke down; Jacobi-PCG finished */
#define SPCG_INVALID_ARG (-1)
#define SPCG_INVALID_CSR (-2)
#define SPCG_HIP_ERROR (-3)
#define SPCG_NOT_SPD (-4)     /* p.Ap <= 0, r.z <= 0 or a non-positive diagonal */
#define SPCG_NON_FINITE (-5)  /* NaN/Inf in the input or in a residual */
#define SPCG_TOO_LARGE (-6)   /* the solve needs more than the static scratch area (cg_solve_static) */

/* value types */
#define SPCG_F64 0
#define SPCG_F32 1

/* preconditioners and precisions of cg_solve */
#define SPCG_PRECOND_NONE 0
#define SPCG_PRECOND_JACOBI 1
#define SPCG_PRECOND_LEARNED 2
#define SPCG_PREC_F64 0
#define SPCG_PREC_MIXED 1
/* CG variants of cg_solve */
#define SPCG_CG_STANDARD 0          /* the loop of Sec. 3.4: two reductions per pass */
#define SPCG_CG_SINGLE_REDUCTION 1  /* Chronopoulos-Gear: one joint reduction per pass */

/* Largest row count, column count and nnz of a matrix handle. */
#define SPCG_MAX_INDEX 2147418111

typedef struct spcg_csr *spcg_csr_t;

/* Human-readable name of a status code (static string). */
const char *spcg_status_str(int status);

/* Text of the last HIP error seen by the library on this thread ("" if none). */
const char *spcg_last_error(void);

/*
 * Create a matrix handle (Sec. 3.2: values, column of each value, position of
 * each row's first value; here with n_rows + 1 entries so the last row's end
 * is explicit).
 *   0 <= n_rows, n_cols, nnz <= SPCG_MAX_INDEX (2^31 - 2^16 - 1), else
 *   SPCG_INVALID_ARG: the kernels index with 32-bit integers and step up to a
 *   few thousand entries past a position, so the top 2^16 values are kept free
 *   d_row_ptr int32[n_rows+1], d_col int32[nnz], d_vals (F64: double[nnz],
 *   F32: float[nnz]); all borrowed: they must stay alive and unchanged until
 *   spcg_csr_destroy.  Columns need not be sorted; duplicates are summed.
 *   The products read d_col and d_vals as vectors of up to 16 bytes starting at
 *   any element (the unaligned access mode, ROCm's default, serves them), never
 *   past nnz; the arrays need only their element alignment.
 * The structure is validated on the device (row_ptr[0] = 0, non-decreasing,
 * row_ptr[n] = nnz, 0 <= col < n_cols) -> SPCG_INVALID_CSR.  Then the row
 * analysis runs: a partition of the rows into blocks of bounded work (and the
 * value offset of each block), and a second one into blocks of a larger bound
 * for the products in FP32 (spcg_csr_wide_blocks).  Synchronous: returns after `stream` has
 * finished the analysis.  The handle owns its analysis arrays (device memory).
 */
int spcg_csr_create(spcg_csr_t *out, int32_t n_rows, int32_t n_cols, int64_t nnz,
                    const int32_t *d_row_ptr, const int32_t *d_col, const void *d_vals,
                    int32_t dtype, hipStream_t stream);

/* Release a handle's analysis arrays (synchronises the device first). */
int spcg_csr_destroy(spcg_csr_t A);

/*
 * Load policy of the matrix streams, process-wide.  The MI355X holds a 256 MB
 * memory-side cache in front of HBM.  A product, or a CG pass loop, whose
 * matrices stream at most `bytes` per product or pass (col + vals + row_ptr;
 * in the learned form A, G and G^T together, else G and G^T alone) reads them
 * with cache-allocating loads, so repeated products find them in that cache;
 * larger ones are read with non-temporal loads, which leave it to the rest,
 * except that the product of a plain, Jacobi or mixed-precision cg_solve
 * still reads a share of such a matrix's row blocks with cache-allocating
 * loads: (bytes - the bytes of p, r and D^-1) / matrix bytes, in sixteenths,
 * spread over the whole matrix (at 160^3, 5/16 of the 358 MB FP64 matrix).
 * bytes >= 0 sets the limit (0: always non-temporal) and returns the previous
 * one; bytes < 0 only returns the current one.  Default 192 MiB.  The policy
 * changes speed only: results are bitwise identical either way.  Takes effect
 * for calls made after it returns.
 */
int64_t spcg_keep_bytes(int64_t bytes);

/* Analysis summary: row blocks, blocks ending in a long row, longest row. */
int spcg_csr_info(spcg_csr_t A, int64_t *n_blocks, int64_t *n_long_rows, int64_t *max_row_len);

/*
 * Row blocks of the second partition that a handle keeps for its products in
 * FP32 (Sec. 3.2's per-row sums over blocks of at most 2048 merge items, rows
 * plus entries, instead of 1536: an FP32 block carries more entries through
 * the same chain of dependent loads, and its LDS still leaves room for 8
 * workgroups per CU).  spmv_csr on an F32 handle (unless runs are on), the
 * inner product of a mixed-precision cg_solve and the FP32 products of
 * spcg_mpnn_loss_grad use it; every other kernel uses the partition of
 * spcg_csr_info.  *n_wide_blocks = 0 for empty matrices.
 */
int spcg_csr_wide_blocks(spcg_csr_t A, int64_t *n_wide_blocks);

/*
 * Row-length binning of y = A x (Sec. 3.2's per-row reduction with a lane
 * group per row sized by the row's length), process-wide policy.  Bin b < 7
 * holds the rows of at most 4 * 2^b entries (rows of 0..4, 5..8, ..., 129..256
 * entries), reduced by groups of 2^b lanes (one lane per row up to a whole
 * wavefront per row); bin 7 holds longer rows, one wavefront per row.  The
 * analysis lists each bin's rows (12 bytes per row, owned by the handle).
 *   SPCG_BINNING_OFF (default): spmv_csr uses the row-block kernel (rows
 *     partitioned into blocks of bounded work, staged through LDS, with a
 *     lane count per block from its mean row length), which measured faster
 *     on the irregular lognormal matrix (103 against 130 us in FP64);
 *   SPCG_BINNING_ON: spcg_csr_create builds the bins and spmv_csr uses them
 *     (rows of at most 4 entries everywhere keep the short-row kernel).
 * The policy at spcg_csr_create decides whether a handle has bins; the policy
 * at spmv_csr whether they are used.  mode < 0 only returns the current
 * policy; otherwise sets it and returns the previous one (SPCG_INVALID_ARG
 * for an unknown mode).  The CG solver's products keep the row-block kernel.
 * Both kernels sum each row in a fixed order that depends only on the matrix
 * (the two orders differ, within rounding).
 */
#define SPCG_NUM_BINS 8
#define SPCG_BINNING_OFF 0
#define SPCG_BINNING_ON 1
int spcg_row_binning(int mode);

/* Rows per bin of a handle built with bins (else SPCG_INVALID_ARG);
 * counts: int64_t[SPCG_NUM_BINS]. */
int spcg_csr_bin_counts(spcg_csr_t A, int64_t *counts);

/*
 * Run-compressed column indices of y = A x, process-wide policy: the index
 * side of the paper's contiguous-section SpMV (Sec. 3.2, the second mapped
 * kernel, which reads x over sections of consecutive columns as one piece).
 * At spcg_csr_create the library cuts the entries each row block stages into
 * chunks of 64 and, per chunk, keeps a 64-bit mask of run starts (an entry
 * whose column is not its predecessor's plus one), the chunk's first start and
 * the start columns (8 + 4 bytes per chunk and 4 per start, owned by the
 * handle); spmv_csr then derives each column from its run start, so inside a
 * run no index is read.  The products and their order are unchanged: results
 * are bitwise equal to the plain kernel's.  Entries of a row longer than the
 * row block's slab keep reading the column array.
 *   SPCG_RUNS_OFF (default): plain columns.  Measured cold on this chip the
 *     run layout is slower although it reads fewer bytes (128^3 7-point, 6 %
 *     fewer: 54.5 against 43.5 us; 2^20 rows of bandwidth 63, 30 % fewer:
 *     185 against 161 us): finding a column costs one more dependent load
 *     (mask and start, then the start column) before the gather of x, and the
 *     product is bound by that chain, not by bytes;
 *   SPCG_RUNS_ON: spcg_csr_create builds the runs and spmv_csr uses them.
 * The policy at spcg_csr_create decides whether a handle has runs; the policy
 * at spmv_csr whether they are used.  mode < 0 only returns the current
 * policy.  Binning (SPCG_BINNING_ON) takes precedence in spmv_csr; the CG
 * solver's products read the plain columns.
 */
#define SPCG_RUNS_OFF 0
#define SPCG_RUNS_ON 1
int spcg_run_columns(int mode);

/* Chunks and run starts of a handle built with runs (else SPCG_INVALID_ARG). */
int spcg_csr_run_info(spcg_csr_t A, int64_t *n_chunks, int64_t *n_starts);

/*
 * Column panels for y = A x, process-wide policy: x staged in LDS, for
 * matrices whose columns scatter over an x much larger than a CU's LDS (each
 * gather of such a matrix is otherwise its own vector-L1 miss).  At
 * spcg_csr_create the library cuts every row into pieces of at most 32
 * entries taken with a stride (piece j of a row of np pieces holds its entries
 * j, j + np, ...), the rows into one range of balanced work per 4 CUs and the
 * columns into panels of 64 KB of doubles or 112 KB of floats (8192 or 28672
 * elements).  A piece's entries in one panel form a segment; the segments of
 * each (range, panel) block are packed into 1024 lanes of equal height, and
 * the library keeps its own copy of the values in that order with one 32-bit
 * word per entry (the column in the panel, the piece's index in its range, a
 * padding flag and a segment-end flag): (value size + 4) bytes per entry plus
 * the padding, and a partial-product buffer of 4 x n_rows values, owned by the
 * handle.  spmv_csr then runs 4 workgroups of 1024 threads per range, one per
 * group of panels holding a quarter of the range's entries; each thread sums
 * its lane's segments serially into LDS accumulators of the pieces, each row
 * adds its pieces into its group's partial vector, and a second kernel adds
 * the four parts in order.  The order of every addition is fixed by the
 * matrix (results repeat bitwise; they differ from the row-block kernel's
 * within rounding).  Products of one handle share its partial buffer, so they
 * are serialized: a product issued on another stream than the handle's last
 * one waits for that one to finish (hipStreamWaitEvent; host calls on one
 * handle take a lock).  Built only for rows with strictly increasing columns,
 * n_cols >= 4, at most 1024 panels, at most 10240 pieces per range and a
 * padded copy of at most 2 nnz + 2^24 entries (blocks too sparse to fill their
 * lanes are not worth it); otherwise the handle has no panels and the other
 * kernels run.  Used only when x is 16-byte aligned.
 * The copy must be rebuilt (a new handle) if the values change.
 *   SPCG_PANELS_OFF: no panels;
 *   SPCG_PANELS_ON: spcg_csr_create builds them (within the limits above) and
 *     spmv_csr uses them;
 *   SPCG_PANELS_AUTO (default): spcg_csr_create builds them only while the
 *     row-binning and run policies are off, for matrices whose rows gather
 *     from across a wide x: at least 65536 rows, at least 16 entries per row
 *     on average, and a median span (last column - first column) of 4096
 *     sampled rows above a quarter of n_cols; spmv_csr uses the panels a
 *     handle has.  Banded, stencil and other local-column matrices keep the
 *     row-block kernel (their x comes from the caches), so does every matrix
 *     of short rows.
 * The policy at spcg_csr_create decides whether a handle has panels; the
 * policy at spmv_csr whether they are used (under ON and AUTO).  mode < 0 only
 * returns the current policy.  Panels take precedence over bins and runs; the
 * CG solver's products keep the row-block kernel.
 */
#define SPCG_PANELS_OFF 0
#define SPCG_PANELS_ON 1
#define SPCG_PANELS_AUTO 2
int spcg_column_panels(int mode);

/* Row ranges, column panels and entries of the panel copy (padding included)
 * of a handle built with panels (else SPCG_INVALID_ARG); null pointers are
 * skipped. */
int spcg_csr_panel_info(spcg_csr_t A, int64_t *n_ranges, int64_t *n_panels, int64_t *n_entries);

/*
 * y = A x (Sec. 3.2): y_i = sum over the entries k of row i of vals[k] * x[col[k]],
 * for all n_rows rows, overwriting y (an empty row gives 0).  x: n_cols
 * elements, y: n_rows elements, both of the handle's dtype; FP32 matrices
 * accumulate in FP32.  x and y must not overlap.  Asynchronous.  The sum
 * order inside a row is fixed by the analysis, so repeated calls give
 * bitwise-identical y.
 */
int spmv_csr(spcg_csr_t A, const void *d_x, void *d_y, hipStream_t stream);

/*
 * Deterministic inner product *d_out = sum_i a_i b_i (FP64), the reduction
 * the CG loop uses (Sec. 3.4: two reductions per pass).  Fixed-order blocked
 * summation; d_work: spcg_dot_workspace_bytes(n) bytes.  Asynchronous.
 */
size_t spcg_dot_workspace_bytes(int64_t n);
int spcg_dot(int64_t n, const double *d_a, const double *d_b, double *d_out, void *d_work,
             hipStream_t stream);

typedef struct {
    double tol;          /* stop when ||r_k||_2 <= tol ||b||_2 (default 1e-10) */
    int32_t maxit;       /* cap on passes (products A p), >= 0 */
    int32_t precond;     /* SPCG_PRECOND_* */
    int32_t precision;   /* SPCG_PREC_F64 or SPCG_PREC_MIXED (Jacobi inner) */
    int32_t check_every; /* passes enqueued between host checks of the device flag; 0 = adaptive */
    double delta;        /* mixed: FP64 residual replacement when ||r32|| < delta * ||r at last replacement|| */
    spcg_csr_t G;        /* learned: lower-triangular factor (pattern of tril(A)), F32 values */
    spcg_csr_t GT;       /* learned: its transpose (pattern of triu(A)), F32 values */
    int32_t budget;      /* learned: passes allowed before the Jacobi fallback */
    int32_t small_path;  /* 1 = allow the single-workgroup solver for small n, 0 = never */
    int32_t timing;      /* N > 0: bracket the SpMV launch of every N-th pass of the loop with
                            HIP events on `stream` and report their summed duration and count
                            (events are created on the handle the first time; each bracketed
                            launch costs a few microseconds more, so N > 1 samples) */
    int32_t variant;     /* SPCG_CG_STANDARD, or SPCG_CG_SINGLE_REDUCTION (FP64 with NONE or
                            JACOBI only): u = M^-1 r, w = A u and s = A p by recurrence, so
                            r.u, w.u and r.r come from one reduction per pass (Chronopoulos
                            and Gear); the same iterates in exact arithmetic */
} spcg_cg_opts;

typedef struct {
    int32_t iters;          /* passes of the (first) solver: products A p */
    int32_t iters_fallback; /* passes of the Jacobi fallback (learned form); iters + iters_fallback
                               <= maxit */
    int32_t n_updates;      /* mixed: FP64 residual replacements */
    int32_t n_restarts;     /* true-residual restarts */
    double true_relres;     /* ||b - A x||_2 / ||b||_2 recomputed in FP64 at exit */
    double spmv_ms;         /* timing > 0: summed duration of the timed SpMV launches */
    int32_t spmv_calls;     /* timing > 0: number of SpMV launches that ran and were timed */
    int32_t reserved;
} spcg_cg_result;

/* Fill opts with defaults: tol 1e-10, maxit 20000, Jacobi, FP64, adaptive checks, delta 0.1,
 * standard variant. */
void spcg_cg_default_opts(spcg_cg_opts *opts);

/* Bytes of device workspace cg_solve needs for A and opts (256-byte aligned pointer).  Besides the
 * vectors and partial sums it holds the solver's own copies: for precision MIXED the FP32 values of A
 * and 2-byte column offsets; for precond LEARNED with factors of at most 8 entries per row, G and G^T
 * as padded column-major planes (8 bytes per slot).  So the size depends on opts->precision,
 * opts->precond and the factor handles. */
size_t spcg_cg_workspace_bytes(spcg_csr_t A, const spcg_cg_opts *opts);

/*
 * Solve A x = b for SPD A by preconditioned conjugate gradients (Sec. 3.4):
 *   r0 = b - A x0, z = M^-1 r, p = z;  per pass: q = A p, alpha = (r.z)/(p.q),
 *   x += alpha p, r -= alpha q, z = M^-1 r, beta = (r'.z')/(r.z), p = z + beta p;
 *   stop when ||r|| <= tol ||b|| or after maxit passes.  On exit the residual
 *   is recomputed in FP64; a gap above tol restarts from it (within maxit).
 * A: F64 handle.  d_b double[n], d_x double[n] (in: x0, out: x).
 * d_work: spcg_cg_workspace_bytes(A, opts) bytes, 256-byte aligned.
 * h_hist: NULL or host double[maxit + 1] receiving ||r_k|| / ||b|| for
 *   k = 0..iters + iters_fallback (FP32 estimates between replacements for the
 *   mixed form; after a learned-form fallback, entry iters is the residual the
 *   Jacobi phase starts from and its passes follow).
 * res: filled on every return that is not INVALID_ARG.
 * ||b|| = 0 gives x = 0 and zero passes.  Synchronous (returns after the
 * final check); the loop itself keeps its scalars on the device and the host
 * reads one status word every check_every passes.
 * Mixed precision: FP32 values, vectors and reductions inside, FP64 only for
 * r = b - A x, x += d and the final check.  Learned: M^-1 = G G^T for at most
 * `budget` passes, then Jacobi-PCG from the current x (from x0 after a
 * breakdown) and status SPCG_FELL_BACK; maxit bounds the passes of both
 * phases together.
 */
int cg_solve(spcg_csr_t A, const double *d_b, double *d_x, const spcg_cg_opts *opts,
             void *d_work, size_t work_bytes, spcg_cg_result *res, double *h_hist,
             hipStream_t stream);

/*
 * cg_solve without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, semantics and results as cg_solve
 * (bitwise: the same kernels run), except that the workspace is the library's
 * static device scratch area of SPCG_STATIC_WORK_BYTES (96 MiB: the 128^3
 * 7-point Jacobi-PCG workspace, 67.5 MB, fits; every device the library runs
 * on holds one such area until the process ends).  The call allocates nothing:
 * no hipMalloc, no hipFree, no event (opts->timing must be 0, else
 * SPCG_INVALID_ARG).  A solve whose spcg_cg_workspace_bytes exceeds the area
 * returns SPCG_TOO_LARGE (spcg_last_error gives both sizes) before any work.
 * The current device must be the handle's (else SPCG_INVALID_ARG).  All calls
 * on one device share that device's area: calls that overlap on one device
 * (two host threads, or two streams whose work interleaves) race and give
 * wrong results; the area keeps the last call's contents, and every solve
 * initialises what it reads.  Synchronous, like cg_solve.
 */
#define SPCG_STATIC_WORK_BYTES ((size_t)96 << 20)
int cg_solve_static(spcg_csr_t A, const double *d_b, double *d_x, const spcg_cg_opts *opts,
                    spcg_cg_result *res, double *h_hist, hipStream_t stream);

/* ------------------------------ factorized sparse approximate inverse (FSAI) */

/*
 * Values of the classical factorized sparse approximate inverse (Kolotilina
 * and Yeremin) on a given lower pattern: a non-learned factor G for
 * M^-1 = G G^T (cg_solve with SPCG_PRECOND_LEARNED and opts.G / opts.GT).
 * Column i of G has the row set J_i = {j >= i : G_ji in the pattern}, sorted,
 * J_i[0] = i; the library solves the dense SPD system A[J_i, J_i] y = e_1 and
 * sets G[J_i, i] = y / sqrt(y_1), so (G^T A G)_ii = 1; with the full lower
 * pattern G G^T = A^-1 exactly.
 * A: square F64 handle (entries of A[J_i, J_i] are read from the rows in J_i;
 * duplicates are summed).  G, GT: F32 handles of the same order, GT the
 * transpose of G with the diagonal first in every row (sorted columns do
 * that), at most SPCG_FSAI_MAX_SET entries per row of GT; both value arrays
 * are overwritten, so they must be writable device memory.
 * Errors: SPCG_INVALID_ARG for types, sizes or patterns that break these
 * rules, SPCG_NOT_SPD if a local system is not positive definite,
 * SPCG_NON_FINITE for NaN/Inf.  Synchronous.
 */
#define SPCG_FSAI_MAX_SET 8
int spcg_fsai_values(spcg_csr_t A, spcg_csr_t G, spcg_csr_t GT, hipStream_t stream);

/* ------------------------------------------- learned factor (G on tril(A)) */

/*
 * Message-passing network that predicts the factor G of M^-1 = G G^T on A's
 * own lower-triangular pattern (G_ii = a_ii^-1/2 exp(o_ii), G_ij = a_ii^-1/2 o_ij,
 * j < i): width 32, SiLU, 4 edge/node layers, BF16 matrix-core MLPs with FP32
 * accumulation.  Its weights are one FP32 vector of SPCG_MPNN_PARAMS values in
 * this order (row-major [out][in] matrices):
 *   node encoder W (32x2), b (32); edge encoder W (32x2), b (32);
 *   4 x { W1e (32x96), c1e, W2e (32x32), c2e, W1n (32x64), c1n, W2n (32x32), c2n };
 *   head w_e (32), c_e (1), w_n (32), c_n (1).
 * A zero head makes G = D^-1/2, i.e. Jacobi.
 */
#define SPCG_MPNN_PARAMS 29442
#define SPCG_MPNN_TRAIN 1

typedef struct spcg_mpnn *spcg_mpnn_t;

/*
 * Per-matrix network state for A (F64 handle, square, sorted columns, one
 * positive diagonal entry per row, structurally symmetric): edge lists,
 * reverse-edge map, the patterns of G = tril and G^T = triu, features, and
 * the factor values.  With SPCG_MPNN_TRAIN it also keeps an FP32 copy of A's
 * values for the probe loss.  A must outlive the graph.  Allocates these
 * per-matrix arrays once (like spcg_csr_create); the network calls below run
 * on a caller workspace.  Synchronous.  SPCG_INVALID_CSR for a pattern that
 * breaks the rules above, SPCG_NOT_SPD for a non-positive diagonal.
 */
int spcg_mpnn_create(spcg_mpnn_t *out, spcg_csr_t A, int32_t flags, hipStream_t stream);
int spcg_mpnn_destroy(spcg_mpnn_t g);
int spcg_mpnn_info(spcg_mpnn_t g, int64_t *n_edges, int64_t *nnz_factor);

/*
 * Bytes of device workspace (256-byte aligned) that spcg_mpnn_predict needs
 * for graphs of up to max_rows rows and max_edges off-diagonal entries: BF16
 * node and edge activations of two alternating layers, the BF16 weight copies
 * and a few scalars.  With SPCG_MPNN_TRAIN: what spcg_mpnn_loss_grad needs
 * (every layer's activations, the FP32 backward scratch, the probe products
 * and the per-workgroup partials; about 0.6 GB for a 48^3 matrix).  One
 * workspace serves many graphs used one at a time on one stream.  0 for
 * invalid sizes.
 */
size_t spcg_mpnn_workspace_bytes(int64_t max_rows, int64_t max_edges, int32_t flags);

/* Handles of G and G^T (FP32 values owned by the graph, filled by predict),
 * ready for spcg_cg_opts.G / .GT.  Valid until spcg_mpnn_destroy. */
int spcg_mpnn_factor(spcg_mpnn_t g, spcg_csr_t *G, spcg_csr_t *GT);

/* Device arrays of G (row_ptr int32[n+1], col int32[nnz_factor], values
 * float[nnz_factor], CSR order) and of G^T's values in G^T's CSR order. */
int spcg_mpnn_factor_arrays(spcg_mpnn_t g, const int32_t **d_row_ptr, const int32_t **d_col,
                            const float **d_vals, const float **d_t_vals);

/* Inference: G and G^T values from the weights d_w (float[SPCG_MPNN_PARAMS]).
 * d_work: at least spcg_mpnn_workspace_bytes(n, n_edges, 0) bytes, 256-byte
 * aligned, caller-owned (else SPCG_INVALID_ARG).  Asynchronous. */
int spcg_mpnn_predict(spcg_mpnn_t g, const float *d_w, void *d_work, size_t work_bytes,
                      hipStream_t stream);

/*
 * Probe loss L = sum_k ||G^T A G v_k - v_k||^2 / (n m) for the m probe vectors
 * d_probes (float[m][n], 1 <= m <= 64) and, if d_grad is not NULL, dL/dw into
 * d_grad (float[SPCG_MPNN_PARAMS], overwritten).  The graph needs
 * SPCG_MPNN_TRAIN; d_work at least spcg_mpnn_workspace_bytes(n, n_edges,
 * SPCG_MPNN_TRAIN) bytes, 256-byte aligned, caller-owned.  Runs the forward
 * pass too (G and G^T values are updated).  h_loss: NULL or receives L (then
 * the call synchronises `stream`).
 */
int spcg_mpnn_loss_grad(spcg_mpnn_t g, const float *d_w, const float *d_probes, int32_t m,
                        float *d_grad, double *h_loss, void *d_work, size_t work_bytes,
                        hipStream_t stream);

/* One Adam step on FP32 master weights: m, v moments in place, bias-corrected
 * with step t >= 1.  Asynchronous. */
int spcg_adam_step(float *d_w, const float *d_g, float *d_m, float *d_v, int64_t n, int32_t t,
                   float lr, float beta1, float beta2, float eps, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* SPCG_H */
