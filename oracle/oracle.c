/*
 * oracle.c -- correctness oracle for the CSR SpMV / conjugate-gradient path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no source, header,
 * table or helper with the HIP library; it is plain, slow, sequential-order
 * C on the host, written from the paper's definitions:
 *
 *   - CSR with three arrays (values, column of each value, first value of
 *     each row) and the row-wise product y_i = sum_k vals[k] * x[col[k]]
 *     (Sec. 3.2, the mapped per-row reduction, and the private-accumulator
 *     OpenMP variant of the same section);
 *   - conjugate gradients for SPD systems (Sec. 3.4, Fig. 6 and the loop
 *     that follows it), with one SpMV, two inner products and three vector
 *     updates per pass.
 *
 * Readings where the paper is garbled or silent (documented with the tests):
 *   * the row loop covers all n rows and overwrites y (the OpenMP listings
 *     stop one row early and accumulate into y; the mapped kernel zeroes its
 *     accumulator first);
 *   * CG starts from r0 = b - A x0, p0 = M^-1 r0; alpha is formed before the
 *     updates that use it and beta before the direction update (Fig. 6 prints
 *     them afterwards and sets r0 = b);
 *   * the stop test is relative, ||r_k||_2 <= tol ||b||_2, checked before each
 *     pass, with an iteration cap (Fig. 6 compares an unspecified absolute
 *     threshold with |r|^2).
 *
 * Floating point: FP64, IEEE, compiled with -ffp-contract=off; every row sum
 * runs in index order.  Inner products use fixed-order blocked summation
 * (blocks of 4096 in index order, then the block sums in order), so results
 * do not depend on the thread count.  The mixed-precision solver's inner
 * iteration uses C float arithmetic (FP32 values, vectors and accumulation),
 * the precision the mixed form prescribes.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_FELL_BACK 2
#define OR_INVALID_ARG (-1)
#define OR_INVALID_CSR (-2)
#define OR_NOT_SPD (-4)
#define OR_NON_FINITE (-5)

#define OR_PRECOND_NONE 0
#define OR_PRECOND_JACOBI 1
#define OR_PRECOND_G 2

#define DOT_BLOCK 4096

/* ------------------------------------------------------------------ CSR -- */

/* Structural check of a CSR matrix: row_ptr[0] = 0, row_ptr non-decreasing,
 * row_ptr[n] = nnz, every column in [0, n_cols).  Returns OR_OK or
 * OR_INVALID_CSR (OR_INVALID_ARG for negative sizes). */
int oracle_csr_check(int32_t n_rows, int32_t n_cols, int64_t nnz,
                     const int32_t *row_ptr, const int32_t *col) {
    if (n_rows < 0 || n_cols < 0 || nnz < 0) return OR_INVALID_ARG;
    if (row_ptr[0] != 0) return OR_INVALID_CSR;
    for (int32_t i = 0; i < n_rows; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return OR_INVALID_CSR;
    if ((int64_t)row_ptr[n_rows] != nnz) return OR_INVALID_CSR;
    for (int64_t k = 0; k < nnz; ++k)
        if (col[k] < 0 || col[k] >= n_cols) return OR_INVALID_CSR;
    return OR_OK;
}

/* y = A x, all n rows, overwrite (Sec. 3.2).  Each row is summed from zero in
 * index order; rows are independent, so threading over rows leaves every
 * bit of y unchanged. */
/* Thread count of the OpenMP row loops (host plumbing for timing runs; the
 * results do not depend on it).  n <= 0 leaves it unchanged.  Returns the
 * previous maximum. */
int oracle_set_threads(int n) {
    const int old = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return old;
}

void oracle_spmv_csr(int32_t n_rows, const int32_t *row_ptr, const int32_t *col,
                     const double *vals, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n_rows; ++i) {
        double t = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            t += vals[k] * x[col[k]];
        y[i] = t;
    }
}

/* The same row sums for FP32 values and FP32 x, accumulated in FP64.  A
 * product of two floats is exact in double, so y is the FP32 product up to
 * FP64 rounding: the yardstick for an FP32-accumulating kernel. */
void oracle_spmv_csr_f32in(int32_t n_rows, const int32_t *row_ptr, const int32_t *col,
                           const float *vals, const float *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n_rows; ++i) {
        double t = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            t += (double)vals[k] * (double)x[col[k]];
        y[i] = t;
    }
}

/* y = A^T x for a CSR A with n_rows rows and n_cols columns (scatter form). */
void oracle_spmv_csr_transpose(int32_t n_rows, int32_t n_cols, const int32_t *row_ptr,
                               const int32_t *col, const double *vals,
                               const double *x, double *y) {
    for (int32_t j = 0; j < n_cols; ++j) y[j] = 0.0;
    for (int32_t i = 0; i < n_rows; ++i)
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            y[col[k]] += vals[k] * x[i];
}

/* --------------------------------------------------------- inner products -- */

double oracle_dot(int64_t n, const double *a, const double *b) {
    int64_t nb = (n + DOT_BLOCK - 1) / DOT_BLOCK;
    double *part = (double *)malloc((size_t)(nb > 0 ? nb : 1) * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t blk = 0; blk < nb; ++blk) {
        double t = 0.0;
        int64_t e = (blk + 1) * DOT_BLOCK < n ? (blk + 1) * DOT_BLOCK : n;
        for (int64_t i = blk * DOT_BLOCK; i < e; ++i) t += a[i] * b[i];
        part[blk] = t;
    }
    double s = 0.0;
    for (int64_t blk = 0; blk < nb; ++blk) s += part[blk];
    free(part);
    return s;
}

static float dot_f32(int64_t n, const float *a, const float *b) {
    int64_t nb = (n + DOT_BLOCK - 1) / DOT_BLOCK;
    float *part = (float *)malloc((size_t)(nb > 0 ? nb : 1) * sizeof(float));
#pragma omp parallel for schedule(static)
    for (int64_t blk = 0; blk < nb; ++blk) {
        float t = 0.0f;
        int64_t e = (blk + 1) * DOT_BLOCK < n ? (blk + 1) * DOT_BLOCK : n;
        for (int64_t i = blk * DOT_BLOCK; i < e; ++i) t += a[i] * b[i];
        part[blk] = t;
    }
    float s = 0.0f;
    for (int64_t blk = 0; blk < nb; ++blk) s += part[blk];
    free(part);
    return s;
}

/* The same FP32 inner product summed as a balanced binary tree: at each level
 * the adjacent pairs (2i, 2i + 1) are added and an unpaired last element moves
 * up unchanged, until one value is left.  This is the order of a data-parallel
 * reduction (the paper's CG takes its inner products with a whole-container
 * add-reduce), and its rounding error grows with log2(n), not with the block
 * length of the sequential order above. */
static float dot_f32_tree(int64_t n, const float *a, const float *b) {
    if (n <= 0) return 0.0f;
    float *u = (float *)malloc((size_t)n * sizeof(float));
    float *v = (float *)malloc((size_t)((n + 1) / 2) * sizeof(float));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) u[i] = a[i] * b[i];
    int64_t m = n;
    while (m > 1) {
        const int64_t h = m / 2;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < h; ++i) v[i] = u[2 * i] + u[2 * i + 1];
        if (m & 1) v[h] = u[m - 1];
        m = (m + 1) / 2;
        float *t = u;
        u = v;
        v = t;
    }
    const float s = u[0];
    free(u);
    free(v);
    return s;
}

/* -------------------------------------------------------- preconditioners -- */

/* dinv_i = 1 / a_ii, the diagonal summed over duplicate entries.  A missing or
 * non-positive diagonal cannot belong to an SPD matrix: OR_NOT_SPD. */
int oracle_jacobi_dinv(int32_t n, const int32_t *row_ptr, const int32_t *col,
                       const double *vals, double *dinv) {
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col[k] == i) d += vals[k];
        if (!(d > 0.0)) return isfinite(d) ? OR_NOT_SPD : OR_NON_FINITE;
        dinv[i] = 1.0 / d;
    }
    return OR_OK;
}

typedef struct {
    int kind;                 /* OR_PRECOND_* */
    const double *dinv;       /* JACOBI */
    const int32_t *g_row_ptr; /* G: lower-triangular CSR, M^-1 = G G^T */
    const int32_t *g_col;
    const double *g_vals;
    double *tmp;              /* n scratch for G^T r */
} precond_t;

/* z = M^-1 r */
static void apply_precond(const precond_t *M, int32_t n, const double *r, double *z) {
    if (M->kind == OR_PRECOND_NONE) {
        memcpy(z, r, (size_t)n * sizeof(double));
    } else if (M->kind == OR_PRECOND_JACOBI) {
        for (int32_t i = 0; i < n; ++i) z[i] = M->dinv[i] * r[i];
    } else {
        oracle_spmv_csr_transpose(n, n, M->g_row_ptr, M->g_col, M->g_vals, r, M->tmp);
        oracle_spmv_csr(n, M->g_row_ptr, M->g_col, M->g_vals, M->tmp, z);
    }
}

static int all_finite(int64_t n, const double *v) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* ------------------------------------------------------------------- CG -- */

/*
 * Preconditioned CG (Sec. 3.4), M^-1 = I, D^-1 or G G^T.
 *
 *   r = b - A x0;  z = M^-1 r;  p = z;  rho = r.z;  hist[0] = ||r|| / ||b||
 *   while ||r|| > tol ||b||  and  k < maxit:
 *       q = A p;  sigma = p.q   (sigma <= 0: not SPD)
 *       alpha = rho / sigma;  x += alpha p;  r -= alpha q
 *       z = M^-1 r;  rho' = r.z;  beta = rho' / rho;  p = z + beta p
 *       k += 1;  hist[k] = ||r|| / ||b||
 *
 * On exit the residual b - A x is recomputed in FP64; if it misses tol while
 * the recursive one passed, the loop restarts from the true residual (at most
 * four times), within maxit.  `iters` counts passes = products A p.
 * ||b|| = 0 gives x = 0 and zero iterations.  hist must hold maxit + 1.
 */
int oracle_pcg(int32_t n, const int32_t *row_ptr, const int32_t *col, const double *vals,
               const double *b, double *x, int precond_kind, const double *dinv_in,
               const int32_t *g_row_ptr, const int32_t *g_col, const double *g_vals,
               double tol, int32_t maxit, int32_t *iters, double *hist, double *true_relres) {
    *iters = 0;
    *true_relres = 0.0;
    if (n < 0 || maxit < 0 || !(tol >= 0.0)) return OR_INVALID_ARG;
    if (!all_finite(n, b) || !all_finite(n, x)) return OR_NON_FINITE;
    double nb = sqrt(oracle_dot(n, b, b));
    if (nb == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        if (hist) hist[0] = 0.0;
        return OR_OK;
    }
    size_t bytes = (size_t)(n > 0 ? n : 1) * sizeof(double);
    double *r = malloc(bytes), *z = malloc(bytes), *p = malloc(bytes), *q = malloc(bytes);
    double *dinv = NULL, *tmp = malloc(bytes);
    precond_t M = {precond_kind, NULL, g_row_ptr, g_col, g_vals, tmp};
    int status = OR_OK;
    if (precond_kind == OR_PRECOND_JACOBI) {
        if (dinv_in) {
            M.dinv = dinv_in;
        } else {
            dinv = malloc(bytes);
            status = oracle_jacobi_dinv(n, row_ptr, col, vals, dinv);
            M.dinv = dinv;
        }
    } else if (precond_kind != OR_PRECOND_NONE && precond_kind != OR_PRECOND_G) {
        status = OR_INVALID_ARG;
    }
    int32_t k = 0;
    int restarts = 0;
    double rr = 0.0, rho = 0.0;
    if (status != OR_OK) goto done;

    /* r0 = b - A x0 */
    oracle_spmv_csr(n, row_ptr, col, vals, x, q);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    for (;;) {
        apply_precond(&M, n, r, z);
        memcpy(p, z, bytes);
        rho = oracle_dot(n, r, z);
        rr = oracle_dot(n, r, r);
        if (hist) hist[k] = sqrt(rr) / nb;
        if (!isfinite(rho) || !isfinite(rr)) { status = OR_NON_FINITE; goto done; }
        if (rr > 0.0 && !(rho > 0.0)) { status = OR_NOT_SPD; goto done; }

        while (sqrt(rr) > tol * nb && k < maxit) {
            oracle_spmv_csr(n, row_ptr, col, vals, p, q);
            double sigma = oracle_dot(n, p, q);
            if (!isfinite(sigma)) { status = OR_NON_FINITE; goto done; }
            if (!(sigma > 0.0)) { status = OR_NOT_SPD; goto done; }
            double alpha = rho / sigma;
            for (int32_t i = 0; i < n; ++i) x[i] += alpha * p[i];
            for (int32_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
            apply_precond(&M, n, r, z);
            double rho_new = oracle_dot(n, r, z);
            rr = oracle_dot(n, r, r);
            ++k;
            if (hist) hist[k] = sqrt(rr) / nb;
            if (!isfinite(rho_new) || !isfinite(rr)) { status = OR_NON_FINITE; goto done; }
            if (rr > 0.0 && !(rho_new > 0.0)) { status = OR_NOT_SPD; goto done; }
            double beta = rho_new / rho;
            for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
            rho = rho_new;
        }
        /* true residual, FP64 */
        oracle_spmv_csr(n, row_ptr, col, vals, x, q);
        for (int32_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
        double tr = sqrt(oracle_dot(n, r, r)) / nb;
        *true_relres = tr;
        if (tr <= tol) { status = OR_OK; break; }
        if (k >= maxit || restarts >= 4) { status = OR_NOT_CONVERGED; break; }
        ++restarts; /* residual gap: restart from the true residual */
    }
done:
    *iters = k;
    free(r); free(z); free(p); free(q); free(tmp); free(dinv);
    return status;
}

/*
 * Single-reduction PCG (Chronopoulos and Gear, 1989): the same Krylov iterates
 * as the loop above in exact arithmetic, with the two inner products of a
 * pass replaced by one joint reduction.  With u = M^-1 r and w = A u:
 *
 *   r = b - A x0;  u = M^-1 r;  w = A u;  gamma = r.u;  delta = w.u
 *   alpha = gamma / delta;  beta = 0;  p = s = 0
 *   while ||r|| > tol ||b||  and  k < maxit:
 *       p = u + beta p;  s = w + beta s          (s = A p by recurrence)
 *       x += alpha p;  r -= alpha s;  u = M^-1 r;  w = A u
 *       gamma' = r.u;  delta = w.u;  (and ||r||^2)      -- one reduction
 *       beta = gamma' / gamma;  alpha = gamma' / (delta - beta gamma' / alpha)
 *       k += 1;  hist[k] = ||r|| / ||b||
 *
 * A non-positive gamma (with r != 0) or denominator means A or M is not SPD.
 * Exit, true-residual restart (from u = M^-1 r, p = s = 0), ||b|| = 0 and
 * status codes as oracle_pcg.  precond_kind: NONE or JACOBI.
 */
int oracle_cg_single_reduction(int32_t n, const int32_t *row_ptr, const int32_t *col,
                               const double *vals, const double *b, double *x, int precond_kind,
                               double tol, int32_t maxit, int32_t *iters, double *hist,
                               double *true_relres) {
    *iters = 0;
    *true_relres = 0.0;
    if (n < 0 || maxit < 0 || !(tol >= 0.0)) return OR_INVALID_ARG;
    if (precond_kind != OR_PRECOND_NONE && precond_kind != OR_PRECOND_JACOBI) return OR_INVALID_ARG;
    if (!all_finite(n, b) || !all_finite(n, x)) return OR_NON_FINITE;
    double nb = sqrt(oracle_dot(n, b, b));
    if (nb == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        if (hist) hist[0] = 0.0;
        return OR_OK;
    }
    size_t bytes = (size_t)(n > 0 ? n : 1) * sizeof(double);
    double *r = malloc(bytes), *u = malloc(bytes), *w = malloc(bytes), *p = malloc(bytes);
    double *sv = malloc(bytes), *dinv = NULL;
    precond_t M = {precond_kind, NULL, NULL, NULL, NULL, NULL};
    int status = OR_OK;
    if (precond_kind == OR_PRECOND_JACOBI) {
        dinv = malloc(bytes);
        status = oracle_jacobi_dinv(n, row_ptr, col, vals, dinv);
        M.dinv = dinv;
    }
    int32_t k = 0;
    int restarts = 0;
    if (status != OR_OK) goto done;

    oracle_spmv_csr(n, row_ptr, col, vals, x, w);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - w[i];
    for (;;) {
        apply_precond(&M, n, r, u);
        oracle_spmv_csr(n, row_ptr, col, vals, u, w);
        double gamma = oracle_dot(n, r, u);
        double delta = oracle_dot(n, w, u);
        double rr = oracle_dot(n, r, r);
        if (hist) hist[k] = sqrt(rr) / nb;
        if (!isfinite(gamma) || !isfinite(delta) || !isfinite(rr)) { status = OR_NON_FINITE; goto done; }
        if (rr > 0.0 && (!(gamma > 0.0) || !(delta > 0.0))) { status = OR_NOT_SPD; goto done; }
        double alpha = rr > 0.0 ? gamma / delta : 0.0, beta = 0.0;
        for (int32_t i = 0; i < n; ++i) p[i] = sv[i] = 0.0;

        while (sqrt(rr) > tol * nb && k < maxit) {
            for (int32_t i = 0; i < n; ++i) p[i] = u[i] + beta * p[i];
            for (int32_t i = 0; i < n; ++i) sv[i] = w[i] + beta * sv[i];
            for (int32_t i = 0; i < n; ++i) x[i] += alpha * p[i];
            for (int32_t i = 0; i < n; ++i) r[i] -= alpha * sv[i];
            apply_precond(&M, n, r, u);
            oracle_spmv_csr(n, row_ptr, col, vals, u, w);
            double gamma_new = oracle_dot(n, r, u);
            delta = oracle_dot(n, w, u);
            rr = oracle_dot(n, r, r);
            ++k;
            if (hist) hist[k] = sqrt(rr) / nb;
            if (!isfinite(gamma_new) || !isfinite(delta) || !isfinite(rr)) { status = OR_NON_FINITE; goto done; }
            if (sqrt(rr) <= tol * nb) break;
            if (!(gamma_new > 0.0)) { status = OR_NOT_SPD; goto done; }
            beta = gamma_new / gamma;
            double denom = delta - beta * gamma_new / alpha;
            if (!isfinite(denom)) { status = OR_NON_FINITE; goto done; }
            if (!(denom > 0.0)) { status = OR_NOT_SPD; goto done; }
            alpha = gamma_new / denom;
            gamma = gamma_new;
        }
        /* true residual, FP64 */
        oracle_spmv_csr(n, row_ptr, col, vals, x, w);
        for (int32_t i = 0; i < n; ++i) r[i] = b[i] - w[i];
        double tr = sqrt(oracle_dot(n, r, r)) / nb;
        *true_relres = tr;
        if (tr <= tol) { status = OR_OK; break; }
        if (k >= maxit || restarts >= 4) { status = OR_NOT_CONVERGED; break; }
        ++restarts;
    }
done:
    *iters = k;
    free(r); free(u); free(w); free(p); free(sv); free(dinv);
    return status;
}

/*
 * Learned-preconditioner solve with Jacobi fallback.  Runs PCG with
 * M^-1 = G G^T for at most `budget` passes; if that does not reach tol, or
 * breaks down (not SPD / non-finite), Jacobi-PCG finishes from the current x
 * (from x0 after a breakdown) and the status is OR_FELL_BACK when it
 * converges.  iters_learned / iters_fallback count the passes of each phase,
 * whose sum maxit bounds.
 */
int oracle_pcg_learned(int32_t n, const int32_t *row_ptr, const int32_t *col,
                       const double *vals, const double *b, double *x,
                       const int32_t *g_row_ptr, const int32_t *g_col, const double *g_vals,
                       double tol, int32_t maxit, int32_t budget,
                       int32_t *iters_learned, int32_t *iters_fallback,
                       double *hist_learned, double *hist_fallback, double *true_relres) {
    *iters_fallback = 0;
    double *x0 = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    memcpy(x0, x, (size_t)n * sizeof(double));
    int32_t lim = budget < maxit ? budget : maxit;
    int st = oracle_pcg(n, row_ptr, col, vals, b, x, OR_PRECOND_G, NULL, g_row_ptr, g_col,
                        g_vals, tol, lim, iters_learned, hist_learned, true_relres);
    if (st == OR_OK || st == OR_INVALID_ARG) { free(x0); return st; }
    if (st == OR_NOT_SPD || st == OR_NON_FINITE) memcpy(x, x0, (size_t)n * sizeof(double));
    free(x0);
    int32_t rest = maxit - *iters_learned;  /* maxit bounds both phases together */
    if (rest < 0) rest = 0;
    int st2 = oracle_pcg(n, row_ptr, col, vals, b, x, OR_PRECOND_JACOBI, NULL, NULL, NULL,
                         NULL, tol, rest, iters_fallback, hist_fallback, true_relres);
    return st2 == OR_OK ? OR_FELL_BACK : st2;
}

/*
 * Mixed precision, reliable-update form: an FP32 Jacobi-PCG on A32 = fl32(A)
 * (FP32 values, vectors and accumulation) under FP64 residual replacement.
 *
 *   x64 = x0;  r64 = b - A x64;  r32 = fl32(r64);  z = dinv32 r32;  p = z;
 *   rho = r32.z;  x32 = 0;  rlast = ||r64||
 *   loop (inner FP32 passes):
 *       q = A32 p;  alpha = rho / (p.q);  x32 += alpha p;  r32 -= alpha q
 *       z = dinv32 r32;  rho' = r32.z;  beta = rho'/rho;  p = z + beta p
 *       if ||r32|| < delta rlast  or  ||r32|| <= tol ||b||  or  k = maxit:
 *           x64 += x32;  x32 = 0;  r64 = b - A x64  (FP64)
 *           r32 = fl32(r64);  z = dinv32 r32;  rho = r32.z;  rlast = ||r64||
 *           stop when ||r64|| <= tol ||b||            (p is kept)
 *
 * The FP32 inner products are summed in blocks of 4096 in index order
 * (dot_order 0) or as a balanced binary tree (dot_order 1); FP64 ones always
 * in blocks.  The FP32 recursion is sensitive to this choice: sequential
 * FP32 sums of 4096 terms carry errors up to ~4096 u32, a tree ~log2(n) u32.
 * dinv32 = fl32(1 / a_ii) with the division in FP64.  hist[k] is the FP32
 * recursive estimate ||r32|| / ||b|| (after a replacement, the FP64 value).
 * n_updates counts FP64 residual replacements (outer refinements).
 */
int oracle_cg_mixed(int32_t n, const int32_t *row_ptr, const int32_t *col, const double *vals,
                    const double *b, double *x, double tol, int32_t maxit, double delta,
                    int dot_order, int32_t *iters, int32_t *n_updates, double *hist,
                    double *true_relres) {
    *iters = 0;
    *n_updates = 0;
    *true_relres = 0.0;
    if (n < 0 || maxit < 0 || !(tol >= 0.0) || !(delta > 0.0 && delta < 1.0)) return OR_INVALID_ARG;
    if (dot_order != 0 && dot_order != 1) return OR_INVALID_ARG;
    if (!all_finite(n, b) || !all_finite(n, x)) return OR_NON_FINITE;
    double nb = sqrt(oracle_dot(n, b, b));
    if (nb == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        if (hist) hist[0] = 0.0;
        return OR_OK;
    }
    int64_t nnz = row_ptr[n];
    size_t nd = (size_t)(n > 0 ? n : 1);
    double *dinv = malloc(nd * sizeof(double)), *r64 = malloc(nd * sizeof(double));
    double *t64 = malloc(nd * sizeof(double));
    float *v32 = malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(float));
    float *dinv32 = malloc(nd * sizeof(float)), *r32 = malloc(nd * sizeof(float));
    float *z32 = malloc(nd * sizeof(float)), *p32 = malloc(nd * sizeof(float));
    float *q32 = malloc(nd * sizeof(float)), *x32 = malloc(nd * sizeof(float));
    float (*dotf)(int64_t, const float *, const float *) = dot_order ? dot_f32_tree : dot_f32;
    int32_t k = 0;
    int status = oracle_jacobi_dinv(n, row_ptr, col, vals, dinv);
    if (status != OR_OK) goto done;
    for (int64_t e = 0; e < nnz; ++e) v32[e] = (float)vals[e];
    for (int32_t i = 0; i < n; ++i) dinv32[i] = (float)dinv[i];

    /* r64 = b - A x64 */
    oracle_spmv_csr(n, row_ptr, col, vals, x, t64);
    for (int32_t i = 0; i < n; ++i) r64[i] = b[i] - t64[i];
    double rlast = sqrt(oracle_dot(n, r64, r64));
    if (hist) hist[0] = rlast / nb;
    for (int32_t i = 0; i < n; ++i) {
        r32[i] = (float)r64[i];
        z32[i] = dinv32[i] * r32[i];
        p32[i] = z32[i];
        x32[i] = 0.0f;
    }
    float rho = dotf(n, r32, z32);
    status = OR_NOT_CONVERGED;
    if (rlast <= tol * nb) { status = OR_OK; goto finish; }
    while (k < maxit) {
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            float t = 0.0f;
            for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) t += v32[e] * p32[col[e]];
            q32[i] = t;
        }
        float sigma = dotf(n, p32, q32);
        if (!isfinite(sigma)) { status = OR_NON_FINITE; goto finish; }
        if (!(sigma > 0.0f)) { status = OR_NOT_SPD; goto finish; }
        float alpha = rho / sigma;
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            x32[i] += alpha * p32[i];
            r32[i] -= alpha * q32[i];
            z32[i] = dinv32[i] * r32[i];
        }
        float rho_new = dotf(n, r32, z32);
        float rr = dotf(n, r32, r32);
        float beta = rho_new / rho;
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) p32[i] = z32[i] + beta * p32[i];
        rho = rho_new;
        ++k;
        double est = sqrt((double)rr);
        if (hist) hist[k] = est / nb;
        if (!isfinite(est) || !isfinite(rho)) { status = OR_NON_FINITE; goto finish; }
        if (est < delta * rlast || est <= tol * nb || k == maxit) {
            /* FP64 residual replacement; the direction p is kept */
            for (int32_t i = 0; i < n; ++i) { x[i] += (double)x32[i]; x32[i] = 0.0f; }
            oracle_spmv_csr(n, row_ptr, col, vals, x, t64);
            for (int32_t i = 0; i < n; ++i) r64[i] = b[i] - t64[i];
            rlast = sqrt(oracle_dot(n, r64, r64));
            ++*n_updates;
            if (hist) hist[k] = rlast / nb;
            for (int32_t i = 0; i < n; ++i) {
                r32[i] = (float)r64[i];
                z32[i] = dinv32[i] * r32[i];
            }
            rho = dotf(n, r32, z32);
            if (rlast <= tol * nb) { status = OR_OK; break; }
        }
    }
finish:
    for (int32_t i = 0; i < n; ++i) x[i] += (double)x32[i];
    oracle_spmv_csr(n, row_ptr, col, vals, x, t64);
    for (int32_t i = 0; i < n; ++i) r64[i] = b[i] - t64[i];
    *true_relres = sqrt(oracle_dot(n, r64, r64)) / nb;
    if (status == OR_OK && *true_relres > tol) status = OR_NOT_CONVERGED;
done:
    *iters = k;
    free(dinv); free(r64); free(t64); free(v32); free(dinv32); free(r32);
    free(z32); free(p32); free(q32); free(x32);
    return status;
}
