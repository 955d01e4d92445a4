/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the dense
 * LU (partial pivoting) and Cholesky factorizations and their solves.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or helper with the
 * HIP path.
 *
 * Conventions: column-major, element (i, j) of a matrix with leading
 * dimension ld sits at a[i + j*ld]; all indices 0-based inside, pivots are
 * reported 1-based (LAPACK interchange convention).  Arithmetic is IEEE
 * binary64; the file is compiled with -ffp-contract=off so that every
 * multiply and subtract is rounded separately, exactly as the statements are
 * written in the paper.
 *
 * OpenMP parallelism only splits independent columns of one elimination
 * step: every element is still updated by exactly one thread, in increasing
 * k order, with the same operations, so the results are bitwise independent
 * of the thread count.
 */
#include <math.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(a, ld, i, j) ((a)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

void oracle_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Host memory bandwidth probe reported beside the CPU baseline (not part of
 * the method): a STREAM-style triad c = a + s*b over n doubles per array,
 * all threads, first touch by the same static partition.  Returns the best
 * of `reps` passes in GB/s, counting 24 bytes per element (two reads, one
 * write); 0 if the arrays cannot be allocated.
 */
#include <stdlib.h>
#include <time.h>

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

double oracle_host_triad_gbs(long n, int reps)
{
    double *a = malloc((size_t)n * sizeof(double));
    double *b = malloc((size_t)n * sizeof(double));
    double *c = malloc((size_t)n * sizeof(double));
    double best = 0.0;
    if (!a || !b || !c) { free(a); free(b); free(c); return 0.0; }
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) { a[i] = 1.0; b[i] = 2.0; c[i] = 0.0; }
    for (int r = 0; r < reps; ++r) {
        const double t0 = now_s();
        #pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) c[i] = a[i] + 3.0 * b[i];
        const double t = now_s() - t0;
        const double gbs = 24.0 * (double)n / t * 1e-9;
        if (gbs > best) best = gbs;
    }
    free(a); free(b); free(c);
    return best;
}

/*
 * LU factorization with partial (row) pivoting of an m x n matrix, in place.
 *
 * Follows the two statements of the in-place LU program (Sec. 6.1 and the
 * LU program figure of Sec. 2.2):
 *   S1: A[i,k] = A[i,k] / A[k,k]                 (i > k)
 *   S2: A[i,j] = A[i,j] - A[i,k] * A[k,j]        (i, j > k)
 * preceded in every step k by the row pivoting that the paper leaves out of
 * its bound analysis (Sec. 6.1): the pivot is the first row, in current
 * order, of largest |A[i,k]| among rows i >= k (strict '>' keeps the lowest
 * index on ties), and rows k and p are exchanged across all n columns.
 *
 * A zero pivot column (all |A[i,k]| == 0, i >= k) records info = k+1 for the
 * first such k and skips the division and update of that step (LAPACK
 * getf2 semantics; the update would only subtract zero products).
 *
 * ksteps limits the number of elimination steps performed (ksteps >=
 * min(m, n) runs the full factorization).  After s steps, the leading s
 * columns hold L, the leading s rows hold U, and the trailing block holds
 * the Schur complement.  ipiv[k] is written for k < min(m, n, ksteps).
 *
 * Returns info (0 = success, k+1 = first exactly zero pivot).
 */
int oracle_dgetrf(int m, int n, double *a, int lda, int *ipiv, int ksteps)
{
    int info = 0;
    int kend = m < n ? m : n;
    if (ksteps < kend) kend = ksteps;
    for (int k = 0; k < kend; ++k) {
        int p = k;
        double best = fabs(AT(a, lda, k, k));
        for (int i = k + 1; i < m; ++i) {
            double v = fabs(AT(a, lda, i, k));
            if (v > best) { best = v; p = i; }
        }
        ipiv[k] = p + 1;
        if (AT(a, lda, p, k) == 0.0) {
            if (info == 0) info = k + 1;
            continue;
        }
        if (p != k) {
            #pragma omp parallel for schedule(static)
            for (int j = 0; j < n; ++j) {
                double t = AT(a, lda, k, j);
                AT(a, lda, k, j) = AT(a, lda, p, j);
                AT(a, lda, p, j) = t;
            }
        }
        const double akk = AT(a, lda, k, k);
        for (int i = k + 1; i < m; ++i)                           /* S1 */
            AT(a, lda, i, k) = AT(a, lda, i, k) / akk;
        #pragma omp parallel for schedule(static)
        for (int j = k + 1; j < n; ++j) {                         /* S2 */
            const double akj = AT(a, lda, k, j);
            double *colj = &AT(a, lda, 0, j);
            const double *colk = &AT(a, lda, 0, k);
            for (int i = k + 1; i < m; ++i) {
                double prod = colk[i] * akj;
                colj[i] = colj[i] - prod;
            }
        }
    }
    return info;
}

/*
 * Solve A X = B with the factors of oracle_dgetrf (n x n, nrhs columns):
 * apply the interchanges ipiv[0..n-1] to B in order, then forward
 * substitution with the unit lower L, then back substitution with U.
 */
void oracle_dgetrs(int n, int nrhs, const double *a, int lda, const int *ipiv,
                   double *b, int ldb)
{
    #pragma omp parallel for schedule(static)
    for (int c = 0; c < nrhs; ++c) {
        double *x = &AT(b, ldb, 0, c);
        for (int k = 0; k < n; ++k) {
            int p = ipiv[k] - 1;
            if (p != k) { double t = x[k]; x[k] = x[p]; x[p] = t; }
        }
        for (int j = 0; j < n; ++j) {
            const double xj = x[j];
            for (int i = j + 1; i < n; ++i) {
                double prod = AT(a, lda, i, j) * xj;
                x[i] = x[i] - prod;
            }
        }
        for (int j = n - 1; j >= 0; --j) {
            x[j] = x[j] / AT(a, lda, j, j);
            const double xj = x[j];
            for (int i = 0; i < j; ++i) {
                double prod = AT(a, lda, i, j) * xj;
                x[i] = x[i] - prod;
            }
        }
    }
}

/*
 * Cholesky factorization A = L L^T, lower triangle, in place.
 *
 * Follows the three statements of the Cholesky listing (Sec. 6.2):
 *   S1: L(k,k) = sqrt(L(k,k))
 *   S2: L(i,k) = L(i,k) / L(k,k)                 (i > k)
 *   S3: L(i,j) = L(i,j) - L(i,k) * L(j,k)        (k < j <= i)
 * Only the lower triangle (i >= j) is read or written.  Before S1, a pivot
 * that is not strictly positive (or is NaN) stops the factorization with
 * info = k+1: the leading minor of order k+1 is not positive definite.
 *
 * ksteps limits the number of outer steps (ksteps >= n: full).
 * Returns info.
 */
int oracle_dpotrf(int n, double *a, int lda, int ksteps)
{
    int kend = ksteps < n ? ksteps : n;
    for (int k = 0; k < kend; ++k) {
        const double d = AT(a, lda, k, k);
        if (!(d > 0.0)) return k + 1;
        AT(a, lda, k, k) = sqrt(d);                               /* S1 */
        const double lkk = AT(a, lda, k, k);
        for (int i = k + 1; i < n; ++i)                           /* S2 */
            AT(a, lda, i, k) = AT(a, lda, i, k) / lkk;
        #pragma omp parallel for schedule(static)
        for (int j = k + 1; j < n; ++j) {                         /* S3 */
            const double ljk = AT(a, lda, j, k);
            double *colj = &AT(a, lda, 0, j);
            const double *colk = &AT(a, lda, 0, k);
            for (int i = j; i < n; ++i) {
                double prod = colk[i] * ljk;
                colj[i] = colj[i] - prod;
            }
        }
    }
    return 0;
}

/*
 * Solve A X = B with the lower Cholesky factor: forward substitution with L,
 * then back substitution with L^T.
 */
void oracle_dpotrs(int n, int nrhs, const double *a, int lda, double *b, int ldb)
{
    #pragma omp parallel for schedule(static)
    for (int c = 0; c < nrhs; ++c) {
        double *x = &AT(b, ldb, 0, c);
        for (int j = 0; j < n; ++j) {
            x[j] = x[j] / AT(a, lda, j, j);
            const double xj = x[j];
            for (int i = j + 1; i < n; ++i) {
                double prod = AT(a, lda, i, j) * xj;
                x[i] = x[i] - prod;
            }
        }
        for (int j = n - 1; j >= 0; --j) {
            double s = x[j];
            for (int i = j + 1; i < n; ++i) {
                double prod = AT(a, lda, i, j) * x[i];
                s = s - prod;
            }
            x[j] = s / AT(a, lda, j, j);
        }
    }
}
