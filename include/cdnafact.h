/*
 * cdnafact.h -- dense LU (partial pivoting) and Cholesky factorizations,
 * solves, mixed-precision solvers with iterative refinement, and batched
 * small factorizations for AMD Instinct MI355X (gfx950).
 *
 * The method is the blocked right-looking factorization whose dominant cost
 * is the Schur-complement update of the trailing matrix (Kwasniewski et al.,
 * "On the Parallel I/O Optimality of Linear Algebra Kernels: Near-Optimal
 * Matrix Factorizations", Sec. 7: the A00 / A10 / A01 / A11 routines, and
 * Table 1).  One GPU; no collectives.
 *
 * Conventions (every entry point):
 *  - Matrices are column-major: element (i, j) is at A[i + j*lda], 0-based,
 *    with lda >= max(1, n).  Sizes are 32-bit ints; leading dimensions are
 *    32-bit ints and offsets are computed in 64 bits.
 *  - Every matrix, vector, ipiv and info pointer is a DEVICE pointer owned
 *    by the caller (hipMalloc'd or from a tensor), unless the argument is
 *    documented as "host".  The library never frees caller memory.
 *  - The library owns only a workspace inside the handle.  It grows lazily
 *    (hipMalloc) up to a cap set with cdf_set_workspace_limit(); a call that
 *    would need more returns CDF_ERR_ALLOC without launching anything.
 *  - Calls are asynchronous on the handle's stream (cdf_set_stream) unless
 *    documented otherwise.  Outputs are valid once that stream reaches the
 *    point after the call.
 *  - Return codes report API-level outcomes; numerical outcomes (singular
 *    or not positive definite input) are written to the device int *info
 *    with LAPACK meaning.  On CDF_ERR_INVALID_ARG, cdf_last_bad_arg(h) gives
 *    the 1-based position of the first bad argument (LAPACK's info = -i).
 *  - n == 0 (or nrhs == 0) is a valid no-op returning CDF_OK.
 *  - Calls that overlap on one handle must not be issued from several host
 *    threads at once; distinct handles are independent.
 */
#ifndef CDNAFACT_H
#define CDNAFACT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define CDF_API __attribute__((visibility("default")))
#else
#define CDF_API
#endif

typedef enum {
    CDF_OK = 0,
    CDF_ERR_INVALID_ARG = 1,     /* argument out of range; see cdf_last_bad_arg */
    CDF_ERR_HIP = 2,             /* a HIP runtime call failed */
    CDF_ERR_ALLOC = 3,           /* workspace allocation failed or exceeds the cap */
    CDF_ERR_NOT_CONVERGED = 4,   /* iterative refinement did not reach its target */
    CDF_ERR_UNSUPPORTED = 5,     /* valid but unimplemented option (e.g. uplo 'U') */
    CDF_ERR_TIMEOUT = 6          /* a device-side wait ran out of its time budget (see
                                    cdf_device_status); the outputs of that call are invalid */
} cdf_status_t;

/*
 * Device info value written by the LU factorizations (cdf_dgetrf and the
 * mixed LU) when a wait of the panel's grid-wide pivot exchange ran out of
 * its budget (CDF_PARAM_LEAF_WAIT_US): the factors and pivots are invalid.
 * Every workgroup still ends normally, and the remaining work of the call
 * runs to completion on identity interchanges.  Negative, so it cannot be
 * confused with LAPACK's zero-pivot info.
 */
#define CDF_INFO_TIMEOUT (-1000)

typedef struct cdf_handle_s *cdf_handle_t;

/* Create a handle bound to the current HIP device, on the null stream. */
CDF_API cdf_status_t cdf_create(cdf_handle_t *h);
/* Destroy a handle and free its workspace (synchronizes its stream). */
CDF_API cdf_status_t cdf_destroy(cdf_handle_t h);
/* Set the stream (a hipStream_t, passed as void*) that later calls enqueue on. */
CDF_API cdf_status_t cdf_set_stream(cdf_handle_t h, void *stream);
/* Cap the handle's workspace in bytes (0 = no cap). */
CDF_API cdf_status_t cdf_set_workspace_limit(cdf_handle_t h, size_t bytes);
/* Bytes currently held by the handle's workspace. */
CDF_API size_t cdf_workspace_bytes(cdf_handle_t h);
/* 1-based index of the first invalid argument of the last failed call, else 0. */
CDF_API int cdf_last_bad_arg(cdf_handle_t h);
/* Human-readable name of a status code (static storage). */
CDF_API const char *cdf_status_string(cdf_status_t s);
/*
 * Synchronizes the handle's streams, then returns CDF_ERR_TIMEOUT if a wait
 * of the LU panel's grid exchange ran out of budget in the most recent LU
 * factorization on this handle (each factorization clears the flag when it
 * starts), else CDF_OK.  CDF_ERR_HIP if a synchronization fails.
 */
CDF_API cdf_status_t cdf_device_status(cdf_handle_t h);

/* Tunable parameters (block sizes chosen per call when left at 0 = auto). */
typedef enum {
    CDF_PARAM_LU_NB = 0,         /* LU outer panel width (multiple of 32, <= 512) */
    CDF_PARAM_CHOL_NB = 1,       /* Cholesky outer block width (multiple of 32, <= 512) */
    CDF_PARAM_LU_LEAF_ROWS = 2,  /* rows per thread in the LU panel leaf (1 or 2) */
    CDF_PARAM_MIXED_NB = 3,      /* block width of the mixed-precision factorizations (multiple of 32,
                                    <= 512; look-ahead where it is a multiple of 128) */
    CDF_PARAM_VBATCH_NB = 4,     /* batched panel width: 0 = 32 where it fits in LDS, 16 = always 16 */
    CDF_PARAM_VBATCH_WG_PER_CU = 5, /* batched persistent workgroups per CU (1 or 2; 0 = 1) */
    CDF_PARAM_GEMM_WG_PER_CU = 6,   /* update-GEMM workgroups resident per CU in this handle's
                                       factorizations (3, 4 or 5; 0 = 5, all of the LDS).  Fewer
                                       leave room for the panel kernels on the second stream.
                                       Passed with each launch: handles do not affect each other. */
    CDF_PARAM_LU_U12 = 7,           /* how the LUs (FP64 and mixed) form U12 = L11^-1 A12: 0 = with
                                       L11^-1 formed beside the update, as one matrix-core GEMM (when
                                       the workspace allows); 1 = blocked substitution in place, which
                                       reproduces exactly representable factors exactly */
    CDF_PARAM_LEAF_WAIT_US = 8,     /* budget of one wait of the LU panel's grid-wide pivot exchange, in
                                       microseconds (0 = 2 s).  A workgroup that waits longer stops,
                                       sets the device error word and writes CDF_INFO_TIMEOUT */
    CDF_PARAM_TEST_EXCHANGE_FAIL = 9, /* testing only: 1 = the exchange waits for a tag no workgroup
                                       writes, so every wait of a multi-workgroup leaf runs out of its
                                       budget (exercises the timeout path); 0 = normal */
    CDF_PARAM_SPD_REFINE = 10,      /* refinement of cdf_dposv_mixed (low-precision formats): 0 = auto
                                       (classical refinement; after three corrections short of the
                                       target, or when the factorization breaks down, preconditioned
                                       CG, see cdf_dposv_mixed), 1 = classical refinement only,
                                       2 = preconditioned CG from the start */
    CDF_PARAM_PCG_MAX_ITER = 11,    /* iteration cap of that preconditioned CG (0 = 400) */
    CDF_PARAM_GEMM_TILE = 12,       /* tile of the FP64 update GEMM C -= A B: 0 or 64 = 64 x 64, 128 =
                                       128 x 128 (faster alone on large square products, slower inside
                                       the LU beside its panel kernels) */
    CDF_PARAM_LU_PIVOT = 13,        /* pivot choice of the LUs (cdf_dgetrf, cdf_dgesv, the mixed LU):
                                       0 = partial pivoting (LAPACK getrf pivots), 1 = tournament
                                       pivoting (Sec. 7.3): every 32-column leaf of a panel picks its
                                       pivots in rounds of local LUs over row blocks, a different but
                                       equally valid row order (|L| may exceed 1) */
    CDF_PARAM_TOURN_BLOCK = 14,     /* tournament: rows per first-round block, 32..256 (0 = 256); raised
                                       where a leaf has more than 512 such blocks; tournament pivoting
                                       needs n <= 131072 (512 blocks of 256 rows) */
    CDF_PARAM_TOURN_FANIN = 15,     /* tournament: candidate sets merged per node, 2..8 (0 = 8) */
    CDF_PARAM_COUNT = 16
} cdf_param_t;
CDF_API cdf_status_t cdf_set_param(cdf_handle_t h, cdf_param_t p, int value);
CDF_API int cdf_get_param(cdf_handle_t h, cdf_param_t p);

/*
 * LU factorization with partial pivoting, in place: P A = L U.
 * Sec. 7 (Algorithm 1, routines A00/A10/A01/A11) and Sec. 6.1 (statements
 * S1/S2); the pivot rule is classic partial pivoting (first row of largest
 * magnitude in the current column, lowest row index on ties), not the
 * tournament pivoting of Sec. 7.3, so the interchanges equal those of
 * unblocked Gaussian elimination with partial pivoting.
 *   n     order of A (>= 0)
 *   A     device, n x n, lda >= max(1, n); on exit unit-lower L strictly
 *         below the diagonal and U on and above it
 *   ipiv  device int[n]; on exit 1-based interchanges: row k was swapped
 *         with row ipiv[k]-1 at step k (LAPACK convention)
 *   info  device int; on exit 0, or j > 0 if U(j-1,j-1) is exactly zero for
 *         the first such j (the factorization is still completed)
 * Workspace: about 0.5 MB, plus 512 x n + 2 x 512 x 512 doubles when U12 is
 * formed through L11^-1 (CDF_PARAM_LU_U12 = 0; if the cap set by
 * cdf_set_workspace_limit refuses those, U12 is solved in place instead).
 * Runs on the handle's stream and two more streams of the handle; the call
 * returns once the work is queued, and all of it is ordered before later
 * work on the handle's stream.
 */
CDF_API cdf_status_t cdf_dgetrf(cdf_handle_t h, int n, double *A, int lda, int *ipiv, int *info);

/*
 * For callers that cannot allocate device memory (work under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the LU of
 * cdf_dgetrf, same arguments, outputs and info, allocating nothing.
 *   - Its scratch (the panel leaf's exchange area, the panels' pivots and
 *     interchange pairs; 576 KB) is a static device array, one copy per GPU,
 *     held until the process ends; its address is looked up when a handle is
 *     created on that GPU.  The handle's workspace is not used or grown.
 *   - n <= CDF_NOALLOC_MAX_N (the exchange area's 256 workgroup slots of
 *     512 rows); larger n returns CDF_ERR_INVALID_ARG (argument 2).
 *   - U12 = L11^-1 A12 is solved in place (as CDF_PARAM_LU_U12 = 1), and
 *     everything runs on the handle's stream (no look-ahead streams, no
 *     events), so the factors equal those of cdf_dgetrf with
 *     CDF_PARAM_LU_U12 = 1 bit for bit.
 *   - Every call on a GPU uses that GPU's one scratch array and leaves its
 *     last contents there (each call zeroes what must start at zero): calls
 *     that overlap in time on one GPU, from any handle or stream, race and
 *     must not be issued.
 *   - CDF_ERR_HIP if the scratch could not be located on this device.
 */
#define CDF_NOALLOC_MAX_N 131072
CDF_API cdf_status_t cdf_dgetrf_noalloc(cdf_handle_t h, int n, double *A, int lda, int *ipiv, int *info);

/*
 * Solve A X = B with the factors of cdf_dgetrf: B <- P B, then the unit
 * lower and upper triangular solves.  trans must be 'N'.
 *   A, ipiv  device, as left by cdf_dgetrf; B device n x nrhs, ldb >= n;
 *   on exit B holds X.
 * For nrhs <= 4 each triangular solve is one launch whose workgroups pass
 * solved 64-row blocks to each other through device flags (n/64 + 1 ints of
 * the handle's workspace).
 */
CDF_API cdf_status_t cdf_dgetrs(cdf_handle_t h, char trans, int n, int nrhs, const double *A, int lda,
                        const int *ipiv, double *B, int ldb);

/*
 * Cholesky factorization A = L L^T, in place, lower triangle (uplo 'L';
 * 'U' returns CDF_ERR_UNSUPPORTED).  Sec. 6.2 (Cholesky listing) and
 * Sec. 7.5 / Table 1 (potrf of A00, trsm, triangular gemm of A11).
 * Only the lower triangle is read or written.
 *   info  device int; 0, or j > 0 if the leading minor of order j is not
 *         positive definite (the factorization stops there).
 */
CDF_API cdf_status_t cdf_dpotrf(cdf_handle_t h, char uplo, int n, double *A, int lda, int *info);

/* Solve A X = B with the lower Cholesky factor (L then L^T); B is overwritten. */
CDF_API cdf_status_t cdf_dpotrs(cdf_handle_t h, char uplo, int n, int nrhs, const double *A, int lda,
                        double *B, int ldb);

/* Precision of the trailing update in the mixed-precision solvers. */
typedef enum {
    CDF_UPD_FP64 = 0,            /* binary64 update (plain FP64 factorization) */
    CDF_UPD_BF16 = 1,            /* bfloat16 operands, binary32 accumulation */
    CDF_UPD_FP16 = 2,            /* binary16 operands with per-tile 2^e scaling, binary32 accumulation */
    CDF_UPD_FP8E4M3 = 3          /* OCP E4M3FN operands with per-tile 2^e scaling, binary32 accumulation */
} cdf_update_prec_t;

/*
 * Mixed-precision solve of A X = B by LU and classical iterative
 * refinement.  A binary32 working copy W of A is factored with a binary64
 * panel (pivot search, interchanges, triangular solves) and a trailing
 * update in precision p; the refinement loop computes r = B - A X in
 * binary64 with the original A and corrects X with solves on W until the
 * HPL scaled residual ||A x - b||_inf / (eps (||A||_inf ||x||_inf +
 * ||b||_inf) n), eps = 2^-53, is <= 16 for every column.  Low-precision LU
 * with refinement is the related work the paper cites (Sec. 11).
 *   A        device n x n (not modified); B device n x nrhs (not modified)
 *   X        device n x nrhs, ldx >= n: the solution on exit
 *   max_iter maximum number of corrections (>= 0)
 *   iters    host int: corrections applied
 *   scaled_resid host double: final scaled residual (max over columns)
 *   info     device int: factorization info of W as for cdf_dgetrf
 * Returns CDF_ERR_NOT_CONVERGED when the target is not reached within
 * max_iter or the residual stagnates (X then holds the last iterate).
 * Synchronizes the handle's stream once per refinement iteration.
 */
CDF_API cdf_status_t cdf_dgesv_mixed(cdf_handle_t h, cdf_update_prec_t p, int n, int nrhs, const double *A,
                             int lda, const double *B, int ldb, double *X, int ldx, int max_iter,
                             int *iters, double *scaled_resid, int *info);

/*
 * As cdf_dgesv_mixed, for symmetric positive definite A, by lower Cholesky
 * (only the lower triangle of A is read).  When classical refinement does
 * not reach the target with the low-precision factor (CDF_PARAM_SPD_REFINE
 * = 0), the solver falls back to the method of Higham and Pranesh (2021,
 * "Exploiting lower precision arithmetic in solving symmetric positive
 * definite linear systems and least squares problems"): binary64
 * preconditioned conjugate gradients, every column on its own, with the
 * low-precision Cholesky factor as the preconditioner; if that factorization
 * broke down (a non-positive pivot), A + sigma diag(A) is factored instead
 * for sigma = u, 4u, 16u, ... (u = the format's unit roundoff; six shifts at
 * most).  The stopping test is the same HPL scaled residual <= 16 of the
 * true residual b - A x with the original A.  max_iter caps the classical
 * corrections; CDF_PARAM_PCG_MAX_ITER the CG iterations; iters reports
 * both together and cdf_mixed_report the details.  info is that of the last
 * factorization run.
 */
CDF_API cdf_status_t cdf_dposv_mixed(cdf_handle_t h, cdf_update_prec_t p, int n, int nrhs, const double *A,
                             int lda, const double *B, int ldb, double *X, int ldx, int max_iter,
                             int *iters, double *scaled_resid, int *info);

/* Refinement methods reported by cdf_mixed_report. */
#define CDF_REFINE_CLASSICAL 1
#define CDF_REFINE_PCG 2
/*
 * What the last cdf_dgesv_mixed / cdf_dposv_mixed on this handle did (host
 * outputs; any may be NULL): the refinement method that ran last, the
 * diagonal shift sigma of the factorization used, the number of
 * factorizations, classical corrections and CG iterations.
 */
CDF_API cdf_status_t cdf_mixed_report(cdf_handle_t h, int *method, double *shift, int *factorizations,
                                      int *corrections, int *pcg_iterations);

/*
 * The factorization step of cdf_dgesv_mixed on its own: W <- binary32(A),
 * then blocked LU of W with a binary64 panel (pivot search, interchanges,
 * L11^-1 A12) and the trailing update in precision p (BF16, FP16 or E4M3,
 * 128-row / 128-column scale tiles, binary32 accumulation).
 *   A device n x n (not modified); W device float n x n (ldw >= n), on exit
 *   the binary32 factors as for cdf_dgetrf; ipiv device int[n] (1-based);
 *   info device int as for cdf_dgetrf.
 */
CDF_API cdf_status_t cdf_sgetrf_mixed(cdf_handle_t h, cdf_update_prec_t p, int n, const double *A, int lda,
                                      float *W, int ldw, int *ipiv, int *info);

/*
 * The factorization step of cdf_dposv_mixed on its own: lower(W) <-
 * binary32(lower(A)), then blocked lower Cholesky of W with binary64
 * diagonal blocks and L21 solves and the trailing update in precision p.
 * The strict upper triangle of W is not written.
 */
CDF_API cdf_status_t cdf_spotrf_mixed(cdf_handle_t h, cdf_update_prec_t p, char uplo, int n, const double *A,
                                      int lda, float *W, int ldw, int *info);

/*
 * Quantize an m x n binary32 matrix tile by tile (the operand encoding of
 * the low-precision trailing update).  Tiles are tm x tn blocks anchored at
 * (0, 0).  For each tile, e = floor(log2(maxfinite / amax)) (capped at 64;
 * 0 for an all-zero tile; always 0 for BF16) and every element is encoded
 * as the format's nearest value (ties to even, E4M3 saturating) of x * 2^e.
 *   p     CDF_UPD_BF16, CDF_UPD_FP16 or CDF_UPD_FP8E4M3
 *   X     device float, ldx >= m
 *   Q     device codes (2 bytes for BF16/FP16, 1 byte for E4M3), column-major
 *         with leading dimension ldq >= m (in elements).  Rows [m, min(ldq,
 *         32*ceil(m/32))) are written as zero codes (the padding the update
 *         reads).
 *   exps  device int[ceil(m/tm) * ceil(n/tn)], tile (ti, tj) at ti + tj*ceil(m/tm)
 */
CDF_API cdf_status_t cdf_quantize(cdf_handle_t h, cdf_update_prec_t p, int m, int n, const float *X, int ldx,
                          int tm, int tn, void *Q, int ldq, int *exps);

/*
 * Low-precision Schur-complement update C <- C - dq(A) dq(B) with binary32
 * accumulation (Sec. 7, routine A11, in the update precision), where dq
 * multiplies each code's value by 2^-e of its tile.  For each T x T tile the
 * product of the codes is accumulated in binary32 from zero, then
 * C - 2^-(ea+eb) * sum is rounded once.  Operands are given K-contiguous,
 * as cdf_quantize writes them with tm = k and tn = T (T = cdf_update_tile(p)):
 *   QA    codes of A^T (k x m, leading dimension lda), 16-byte aligned;
 *         ea[i] is the exponent of rows [T*i, T*i+T) of A
 *   QB    codes of B (k x n, leading dimension ldb), 16-byte aligned; eb[j]
 *         is the exponent of columns [T*j, T*j+T) of B
 *   lda, ldb multiples of 32 and >= 32*ceil(k/32); codes of rows [k, lda) are zero
 *   C     device float m x n (ldc >= m)
 */
CDF_API cdf_status_t cdf_lowp_update(cdf_handle_t h, cdf_update_prec_t p, int m, int n, int k,
                             const void *QA, int lda, const int *ea, const void *QB, int ldb,
                             const int *eb, float *C, int ldc);
/* Tile size T of the low-precision update (rows of A / columns of B per scale). */
CDF_API int cdf_update_tile(cdf_update_prec_t p);

/*
 * FP64 Schur-complement update C <- C - A B (Sec. 7, routine A11; Table 1,
 * local gemm), the dominant step of the LU factorization.
 *   A device m x k (lda >= m), B device k x n (ldb >= k), C device m x n (ldc >= m).
 */
CDF_API cdf_status_t cdf_dgemm_update(cdf_handle_t h, int m, int n, int k, const double *A, int lda,
                              const double *B, int ldb, double *C, int ldc);

/* ---------------------------------------------------------------- batched */

typedef enum { CDF_F64 = 0, CDF_F32 = 1 } cdf_dtype_t;
typedef struct cdf_vbatch_plan_s *cdf_vbatch_plan_t;

/*
 * Plan a batch of independent small factorizations of uneven sizes, run as
 * one persistent kernel launch (problems handed out largest first from a
 * device work counter), preceded by a small kernel that gathers the
 * problems' descriptors.
 *   batch      number of problems (>= 0)
 *   n_host     host int[batch], orders 1 <= n <= 1024
 *   kind_host  host int[batch]: 0 = LU with partial pivoting, 1 = lower Cholesky
 *   dt         element type of the matrices
 * The plan holds its own device copies of the sizes and schedule.
 */
CDF_API cdf_status_t cdf_vbatch_plan_create(cdf_handle_t h, int batch, const int *n_host, const int *kind_host,
                                    cdf_dtype_t dt, cdf_vbatch_plan_t *plan);
/*
 * Run a planned batch on the handle's stream.  Runs of one plan share its
 * work counter and descriptors: runs of a plan that overlap in time race.
 *   A_array    device array of device pointers to the matrices (double* or float*)
 *   lda_array  device int[batch]
 *   ipiv_array device array of device int* (LU problems; may hold NULL for Cholesky)
 *   info_array device int[batch]: LAPACK info per problem
 * The pointer arrays are read at run time, so a plan may be replayed on new data.
 */
CDF_API cdf_status_t cdf_vbatch_run(cdf_handle_t h, cdf_vbatch_plan_t plan, void *const *A_array,
                            const int *lda_array, int *const *ipiv_array, int *info_array);
CDF_API cdf_status_t cdf_vbatch_plan_destroy(cdf_vbatch_plan_t plan);

/* ------------------------------------------------------------- I/O bound */

/*
 * Sequential (one processor) I/O lower bound in elements for fast memory of
 * m_elems elements (Sec. 6.1 and 6.2):
 *   kind 0 (LU):       (2n^3 - 6n^2 + 4n) / (3 sqrt(M)) + n(n-1)/2
 *   kind 1 (Cholesky): n^3 / (3 sqrt(M)) + n^2/2 + n
 * Returns a negative value for an invalid kind or m_elems <= 0.  Host only.
 */
CDF_API double cdf_io_lower_bound_elems(int kind, double n, double m_elems);

/*
 * General I/O lower bound of a statement of a disjoint-access affine program
 * (Sec. 3 and 4), host only.  A statement with loop nest depth l reads m
 * input accesses; access j is given by the set of distinct iteration
 * variables that index it (bit t of access_vars[j] for variable t; its
 * dimension is the number of bits) and its dominator weight (1, or 1/rho_S
 * when it reads the output of a producer statement S, Sec. 4.2).  u is the
 * number of out-degree-one input predecessors every compute vertex has
 * (Sec. 3.2; 0 = none known), nvertices the statement's compute vertices |V|,
 * array_id[j] names the array of access j (for the program bound).
 */
#define CDF_DAAP_MAX_VARS 8
#define CDF_DAAP_MAX_ACCESSES 8
typedef struct {
    int nvars;
    int naccesses;
    unsigned access_vars[CDF_DAAP_MAX_ACCESSES];
    double access_weight[CDF_DAAP_MAX_ACCESSES];
    int array_id[CDF_DAAP_MAX_ACCESSES];
    int u;
    double nvertices;
} cdf_daap_statement_t;

/*
 * rho  = min over X > M of chi(X) / (X - M), capped at 1/u (the maximum
 *        computational intensity), attained at x0 (Sec. 3.2);
 * chi  = chi(x0), the largest subcomputation whose dominator set has x0
 *        vertices; tile[t] = |D^t| there (the extents of an I/O-optimal tile);
 *        access[j] = weighted size of access j there;
 * q    = nvertices / rho, the lower bound on loads and stores.
 */
typedef struct {
    double rho, x0, chi, q;
    double tile[CDF_DAAP_MAX_VARS];
    double access[CDF_DAAP_MAX_ACCESSES];
} cdf_daap_result_t;

/*
 * chi(X) = max prod_t D_t s.t. sum_j w_j prod_{t in access j} D_t <= X,
 * D_t >= 1 (continuous relaxation, Sec. 3.2), and the maximizing D_t in
 * tile[0..nvars) (tile may be NULL).  CDF_ERR_INVALID_ARG for an invalid
 * statement (depth or access count out of range, an empty access, a
 * non-positive weight, a variable that indexes no access) or X not above the
 * sum of the weights.
 */
CDF_API cdf_status_t cdf_daap_chi(const cdf_daap_statement_t *s, double X, double *chi, double *tile);
/* The statement's bound for a fast memory of M elements (M > 0). */
CDF_API cdf_status_t cdf_daap_statement_bound(const cdf_daap_statement_t *s, double M, cdf_daap_result_t *r);
/*
 * Bound of a program of n statements (Sec. 4): the sum of their bounds minus
 * the input loads that statements sharing an array (equal array_id) can
 * share: each statement alone loads access[j] * nvertices / chi elements of
 * it in its optimal schedule, and at least the largest of these remain.
 */
CDF_API cdf_status_t cdf_daap_program_bound(int n, const cdf_daap_statement_t *s, double M, double *q);

/* ------------------------------------------------------- kernel timing */

/*
 * Kernel timing for roofline measurement (instrumentation, not part of the
 * method).  Between cdf_profile_begin and cdf_profile_end, every launch of
 * the FP64 update GEMM kernels made by this handle's factorizations (on any
 * of its streams) is bracketed by two HIP events recorded on the stream it
 * is launched on.
 *   kernel   0: C -= A B (the LU trailing update and the panels' own updates)
 *            1: A B^T, 2: A^T B, 3: A^T B^T, 4: lower-triangle A B^T (SYRK)
 *            5: the products that form U12 = L11^-1 A12 and L11^-1 itself
 *               (the LU's triangular solve done as matrix products)
 *   launches number of launches of that kernel (host)
 *   total_ms sum of their event-measured durations in ms (host)
 *   flops    sum of their algorithmic flops 2mnk (m(m+1)k for SYRK) (host)
 *   bytes    sum of their algorithmic bytes: C read and written once and each
 *            operand read once, 8(2mn + mk + kn) (8(m(m+1) + 2mk) for SYRK) (host)
 * cdf_profile_end synchronizes the recorded events and stops recording;
 * the records stay readable (one call per kernel kind) until the next
 * cdf_profile_begin.  Without a cdf_profile_begin it returns zeros.
 */
CDF_API cdf_status_t cdf_profile_begin(cdf_handle_t h);
CDF_API cdf_status_t cdf_profile_end(cdf_handle_t h, int kernel, long long *launches, double *total_ms,
                                     double *flops, double *bytes);

#ifdef __cplusplus
}
#endif
#endif /* CDNAFACT_H */
