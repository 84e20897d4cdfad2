/*
 * Oracle core -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, sequential FP64 block Cholesky of a symmetric positive definite
 * matrix held as an M x M grid of dense blocks, followed by the forward and
 * backward triangular solves.  Only tests/, the smoke check and the CPU leg of
 * the benchmark may load this file; the product library never does.
 *
 * What it computes is the plain definition the paper relies on: the Cholesky
 * factor L with A = L L^T and a positive diagonal is unique, so the factor of the
 * permuted KKT matrix (paper, Sec. 3.1, Fig. 2: hat Psi = hat L hat L^T) and the
 * solution of hat L hat y = hat r, hat L^T hat x = hat y (Sec. 3.2) are fixed by
 * the matrix and the block order alone.  The order is chosen by the caller:
 * natural order gives the sequential method (the p = 1 case), the segmented
 * order of Sec. 3.1 gives the parallel method's factor.
 *
 * Algorithm: the textbook right-looking (outer product) block Cholesky.  For
 * block column j:  L_jj = chol(A_jj);  L_ij = A_ij L_jj^{-T} for every stored
 * block below it;  A_il -= L_ij L_lj^T for every pair of stored blocks i >= l > j
 * (a block that was a structural zero is created: fill-in).  Structural zero
 * blocks (never stored) are skipped: they contribute exact zeros.
 * The scalar Cholesky of a diagonal block is the column-by-column definition
 *   L[c][c] = sqrt(A[c][c] - sum_{l<c} L[c][l]^2),
 *   L[r][c] = (A[r][c] - sum_{l<c} L[r][l] L[c][l]) / L[c][c],  r > c,
 * and reads only the lower triangle of A_jj.
 *
 * No BLAS, no blocking beyond the given grid, no reordering, no fast-math.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int M;          /* number of block rows (= block columns) */
    int *sz;        /* sz[i]: rows of block row i */
    long *off;      /* scalar offset of block row i inside a stacked vector */
    long n;         /* total scalar size */
    double **blk;   /* blk[i*M + j], i >= j: row-major sz[i] x sz[j]; NULL = zero */
} ob_matrix;

ob_matrix *ob_create(int M, const int *sizes)
{
    if (M < 1) return NULL;
    ob_matrix *A = (ob_matrix *)calloc(1, sizeof(ob_matrix));
    if (!A) return NULL;
    A->M = M;
    A->sz = (int *)malloc(sizeof(int) * (size_t)M);
    A->off = (long *)malloc(sizeof(long) * (size_t)M);
    A->blk = (double **)calloc((size_t)M * (size_t)M, sizeof(double *));
    if (!A->sz || !A->off || !A->blk) { free(A->sz); free(A->off); free(A->blk); free(A); return NULL; }
    long o = 0;
    for (int i = 0; i < M; ++i) {
        A->sz[i] = sizes[i];
        A->off[i] = o;
        o += sizes[i];
    }
    A->n = o;
    return A;
}

void ob_free(ob_matrix *A)
{
    if (!A) return;
    for (long t = 0; t < (long)A->M * A->M; ++t) free(A->blk[t]);
    free(A->blk); free(A->sz); free(A->off); free(A);
}

static double *ob_slot(ob_matrix *A, int i, int j, int create)
{
    double **p = &A->blk[(long)i * A->M + j];
    if (!*p && create) *p = (double *)calloc((size_t)A->sz[i] * (size_t)A->sz[j], sizeof(double));
    return *p;
}

/* Store block (i, j), i >= j, row-major sz[i] x sz[j] (copied).  Returns 0, or -1. */
int ob_set(ob_matrix *A, int i, int j, const double *a)
{
    if (!A || i < 0 || j < 0 || i >= A->M || j > i) return -1;
    double *d = ob_slot(A, i, j, 1);
    if (!d) return -1;
    memcpy(d, a, sizeof(double) * (size_t)A->sz[i] * (size_t)A->sz[j]);
    return 0;
}

/* Copy block (i, j) into out.  Returns 1 if stored, 0 for a structural zero, -1 on error. */
int ob_get(const ob_matrix *A, int i, int j, double *out)
{
    if (!A || i < 0 || j < 0 || i >= A->M || j >= A->M) return -1;
    const double *d = A->blk[(long)i * A->M + j];
    if (!d) return 0;
    memcpy(out, d, sizeof(double) * (size_t)A->sz[i] * (size_t)A->sz[j]);
    return 1;
}

/* Scalar Cholesky of the m x m block a (lower triangle read, factor written to the
 * lower triangle, upper triangle zeroed).  Returns 0, or 1 if a pivot is not
 * positive and finite. */
static int chol_block(double *a, int m)
{
    for (int c = 0; c < m; ++c) {
        double s = a[c * m + c];
        for (int l = 0; l < c; ++l) s -= a[c * m + l] * a[c * m + l];
        if (!(s > 0.0) || !isfinite(s)) return 1;
        double d = sqrt(s);
        a[c * m + c] = d;
        for (int r = c + 1; r < m; ++r) {
            double t = a[r * m + c];
            for (int l = 0; l < c; ++l) t -= a[r * m + l] * a[c * m + l];
            a[r * m + c] = t / d;
        }
    }
    for (int r = 0; r < m; ++r)
        for (int c = r + 1; c < m; ++c) a[r * m + c] = 0.0;
    return 0;
}

/* X <- X L^{-T} for X (rows x m), L (m x m) lower: solve X L^T = B row by row. */
static void trsm_right_lt(double *x, int rows, const double *L, int m)
{
    for (int r = 0; r < rows; ++r) {
        double *xr = x + (long)r * m;
        for (int c = 0; c < m; ++c) {
            double t = xr[c];
            for (int l = 0; l < c; ++l) t -= xr[l] * L[c * m + l];
            xr[c] = t / L[c * m + c];
        }
    }
}

/* C (ri x rl) -= X (ri x k) Y(rl x k)^T */
static void gemm_sub_nt(double *C, const double *X, const double *Y, int ri, int rl, int k)
{
    for (int a = 0; a < ri; ++a)
        for (int b = 0; b < rl; ++b) {
            double s = 0.0;
            for (int t = 0; t < k; ++t) s += X[(long)a * k + t] * Y[(long)b * k + t];
            C[(long)a * rl + b] -= s;
        }
}

/* In-place block Cholesky.  Returns 0 on success, j+1 if the diagonal block of
 * block column j (0-based) is not positive definite, -1 on bad input. */
int ob_cholesky(ob_matrix *A)
{
    if (!A) return -1;
    const int M = A->M;
    for (int j = 0; j < M; ++j) {
        double *Ljj = ob_slot(A, j, j, 0);
        if (!Ljj) return j + 1;               /* a zero diagonal block is singular */
        if (chol_block(Ljj, A->sz[j])) return j + 1;
        for (int i = j + 1; i < M; ++i) {
            double *Lij = ob_slot(A, i, j, 0);
            if (Lij) trsm_right_lt(Lij, A->sz[i], Ljj, A->sz[j]);
        }
        for (int i = j + 1; i < M; ++i) {
            const double *Lij = A->blk[(long)i * M + j];
            if (!Lij) continue;
            for (int l = j + 1; l <= i; ++l) {
                const double *Llj = A->blk[(long)l * M + j];
                if (!Llj) continue;
                double *Ail = ob_slot(A, i, l, 1);
                if (!Ail) return -1;
                gemm_sub_nt(Ail, Lij, Llj, A->sz[i], A->sz[l], A->sz[j]);
            }
        }
    }
    return 0;
}

/* Solve L L^T x = b in place for a factored matrix.  x is n x nrhs row-major with
 * the rows of block row i at off[i].  Forward: x_i -= sum_{j<i} L_ij x_j, then
 * x_i = L_ii^{-1} x_i.  Backward: x_i -= sum_{l>i} L_li^T x_l, then x_i = L_ii^{-T} x_i. */
int ob_solve(const ob_matrix *A, double *x, int nrhs)
{
    if (!A || !x || nrhs < 1) return -1;
    const int M = A->M;
    for (int i = 0; i < M; ++i) {
        const int mi = A->sz[i];
        double *xi = x + A->off[i] * nrhs;
        for (int j = 0; j < i; ++j) {
            const double *L = A->blk[(long)i * M + j];
            if (!L) continue;
            const int mj = A->sz[j];
            const double *xj = x + A->off[j] * nrhs;
            for (int r = 0; r < mi; ++r)
                for (int q = 0; q < nrhs; ++q) {
                    double s = 0.0;
                    for (int c = 0; c < mj; ++c) s += L[(long)r * mj + c] * xj[(long)c * nrhs + q];
                    xi[(long)r * nrhs + q] -= s;
                }
        }
        const double *D = A->blk[(long)i * M + i];
        for (int q = 0; q < nrhs; ++q)
            for (int r = 0; r < mi; ++r) {
                double t = xi[(long)r * nrhs + q];
                for (int c = 0; c < r; ++c) t -= D[r * mi + c] * xi[(long)c * nrhs + q];
                xi[(long)r * nrhs + q] = t / D[r * mi + r];
            }
    }
    for (int i = M - 1; i >= 0; --i) {
        const int mi = A->sz[i];
        double *xi = x + A->off[i] * nrhs;
        for (int l = i + 1; l < M; ++l) {
            const double *L = A->blk[(long)l * M + i];
            if (!L) continue;
            const int ml = A->sz[l];
            const double *xl = x + A->off[l] * nrhs;
            for (int c = 0; c < mi; ++c)
                for (int q = 0; q < nrhs; ++q) {
                    double s = 0.0;
                    for (int r = 0; r < ml; ++r) s += L[(long)r * mi + c] * xl[(long)r * nrhs + q];
                    xi[(long)c * nrhs + q] -= s;
                }
        }
        const double *D = A->blk[(long)i * M + i];
        for (int q = 0; q < nrhs; ++q)
            for (int c = mi - 1; c >= 0; --c) {
                double t = xi[(long)c * nrhs + q];
                for (int r = c + 1; r < mi; ++r) t -= D[r * mi + c] * xi[(long)r * nrhs + q];
                xi[(long)c * nrhs + q] = t / D[c * mi + c];
            }
    }
    return 0;
}

long ob_size(const ob_matrix *A) { return A ? A->n : -1; }
