// Internal declarations shared by the HIP sources of libcdnafact.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <type_traits>

#include "cdnafact.h"

namespace cdf {
struct ProfState;
// What the last mixed-precision solve on a handle did (cdf_mixed_report).
struct MixedReport {
    int method = 0;          // CDF_REFINE_CLASSICAL or CDF_REFINE_PCG (0: none)
    double shift = 0.0;      // sigma of the factorization used (A + sigma diag(A))
    int factorizations = 0;  // low-precision factorizations run
    int corrections = 0;     // classical corrections applied
    int pcg_iterations = 0;  // PCG iterations
};
}

struct cdf_handle_s {
    int device = 0;
    int num_cus = 256;
    hipStream_t stream = nullptr;
    void *ws = nullptr;          // lazily grown workspace
    size_t ws_bytes = 0;
    size_t ws_limit = 0;         // 0 = no cap
    unsigned leaf_epoch = 0;     // next epoch of the panel leaf's exchange tags
    int bad_arg = 0;
    hipStream_t aux = nullptr;   // second stream for look-ahead (default priority)
    hipStream_t aux2 = nullptr;  // third stream: LU interchanges on finished L columns
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int params[CDF_PARAM_COUNT] = {};
    int wall_khz = 100000;       // rate of the device's constant wall clock
    int leaf_occ[2] = {0, 0};    // resident leaf workgroups per CU (R = 1, 2); 0 = not yet queried
    int *last_err = nullptr;     // error word of the most recent LU's leaf exchange (cdf_device_status)
    cdf::ProfState *prof = nullptr;  // kernel-timing records (cdf_profile_begin / _end)
    cdf::MixedReport mixed_report;    // what the last mixed-precision solve did
};

namespace cdf {

// Compile-time loop: f(integral_constant<int, I>) for I in [B, E), so that
// register-array indices are constants before any optimization runs.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Bytes at the head of the workspace reserved for the panel leaf's exchange
// (its last 256 bytes hold the device error word of the bounded waits).
constexpr size_t kLeafWsBytes = 512 * 1024;
// Default budget of one wait of the leaf's grid exchange (microseconds).  A
// legitimate wait lasts as long as the longest kernel beside the leaf keeps
// CUs busy (tens of ms for the first trailing update at n = 65536).
constexpr long long kLeafWaitUsDefault = 2000000;

// Grows the handle's workspace to at least `bytes` (synchronizing the stream
// before a reallocation).  Returns CDF_ERR_ALLOC on failure or above the cap.
cdf_status_t ws_reserve(cdf_handle_t h, size_t bytes);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Kernel-timing records of a handle (cdf_profile_begin / _end) and the kinds
// they are filed under.
enum ProfKind { PROF_NN = 0, PROF_NT = 1, PROF_TN = 2, PROF_TT = 3, PROF_SYRK = 4, PROF_U12 = 5, PROF_KINDS = 6 };
int prof_begin(ProfState *st, hipStream_t s, int kind, double flops, double bytes);  // -1 when not timing
void prof_end(ProfState *st, hipStream_t s, int slot);
hipError_t prof_enable(ProfState **st);  // creates the records on first use
hipError_t prof_collect(ProfState *st, int kind, long long *launches, double *total_ms, double *flops,
                        double *bytes);
void prof_free(ProfState *st);

// Per-call options of the FP64 GEMM: update-GEMM workgroups resident per CU
// (3..5; 0 = 5), the calling handle's timing records (null: not timed), and
// the kind a timed launch is filed under (-1: by its shape).
struct GemmCtx {
    int wg_per_cu = 0;
    ProfState *prof = nullptr;
    int tag = -1;
    int tile = 0;  // NN update tile: 0 = by size, 64, 128
};
GemmCtx gemm_ctx(cdf_handle_t h, int tag = -1);

// C = beta*C + alpha*op(A)*op(B); op(A) is m x k, op(B) is k x n.
// ta: 0 -> A is m x k, 1 -> A is k x m (op = transpose); same for tb.
// lower: only the lower triangle (i >= j) of C is read or written (C square).
// stop: optional device flag; a nonzero value makes the launch a no-op.
// ctx: launch options (null: five workgroups per CU, not timed).
hipError_t dgemm(hipStream_t s, int ta, int tb, int m, int n, int k, double alpha,
                 const double *A, int lda, const double *B, int ldb, double beta,
                 double *C, int ldc, bool lower, const int *stop = nullptr, const GemmCtx *ctx = nullptr);

// The binary64 factorizations behind cdf_dgetrf / cdf_dpotrf on the handle's
// stream (look-ahead on its second stream); getrf_fp64 takes a device work
// area of getrf_ws_ints() ints (panel pivots and interchange pairs) besides
// the leaf's exchange area at the head of the handle's workspace, and
// optionally (lu_w, getrf_w_doubles(n) doubles, 256-byte aligned) the area
// for U12 through L11^-1 (null: U12 by blocked substitution in place).
size_t getrf_ws_ints();
size_t getrf_w_doubles(int n);
hipError_t getrf_fp64(cdf_handle_t h, int n, double *A, int lda, int *ipiv, int *info, int *ws_ints,
                      double *lu_w = nullptr);
hipError_t potrf_fp64(cdf_handle_t h, int n, double *A, int lda, int *info);
// The binary64 LU with U12 solved in place (no inverse, no U12 buffer), its
// exchange in `la`, on the handle's stream alone (no look-ahead streams, no
// events): needs only `la` and getrf_ws_ints() ints of device memory.
struct LeafArea;
hipError_t getrf_inplace_one_stream(cdf_handle_t h, const LeafArea &la, int n, double *A, int lda, int *ipiv,
                                    int *info, int *ws_ints);

// Looks up the device address of the allocation-free LU's scratch array on
// `device` (the current device), once per device; later calls return the
// first result.  Called at handle creation.
hipError_t noalloc_setup(int device);

// Creates the handle's second stream (default priority) and its two events.
hipError_t ensure_aux(cdf_handle_t h);

// Li (kb x kb, leading dimension ldi) = L^-1 for the unit lower triangle of
// L (kb x kb, leading dimension ldl), by blocked forward substitution; then
// *good = 1, unless an entry exceeds kInverseBound in magnitude: then Li is
// set to the identity and *good = 0 (the caller solves by substitution).
constexpr double kInverseBound = 16.0;
hipError_t unit_lower_inverse(hipStream_t s, int kb, const double *L, int ldl, double *Li, int ldi, int *good,
                              const GemmCtx *ctx = nullptr);

// Device area of the leaf's grid exchange (kLeafWsBytes: tags, tagged rows,
// and in its last 256 bytes the error word) and the host-side counter of the
// epochs issued on it (below 64: the area is zeroed before the next leaf).
struct LeafArea {
    void *base;
    unsigned *epoch;
};
LeafArea handle_leaf_area(cdf_handle_t h);  // the head of the handle's workspace
// LU panel leaf: factor the m x n (n <= 32) column block at A with partial
// pivoting; writes absolute 1-based pivots ipiv[0..n) (row offset `row0`
// added), first zero pivot into *info (as info_base + j + 1) if *info == 0.
// The leaf also applies its interchanges to the other columns [0, c0) and
// [c0 + n, region_cols) of the region (region_rows rows) it belongs to; A is
// region + c0 + c0 * lda.  Its grid exchange uses `la`.
hipError_t lu_leaf(cdf_handle_t h, const LeafArea &la, hipStream_t stream, int m, int n, double *A, int lda,
                   int *ipiv, int row0, int *info, int info_base, int rows_per_thread, double *region,
                   int region_rows, int region_cols, int c0);
// The area's device error word (set when a wait of the exchange ran out of
// budget) and its reset, ordered on `stream`; every factorization that runs
// leaves resets it first.
int *leaf_error_word(const LeafArea &la);
hipError_t leaf_reset_error(const LeafArea &la, hipStream_t stream);
// The leaf kernel for two rows per thread (for hipLaunchKernel / occupancy).
const void *leaf_kernel_r2();

// Recursive LU panel of columns [c0, c0+w) of the m x ncols region A (rows
// [c0, m)) on stream s; interchanges are applied to all other columns of the
// region; pivots are relative to the region's row 0; info offset by info_off.
// tourn: the leaves choose their pivots by tournament (tourn_leaf).
hipError_t lu_panel(cdf_handle_t h, const LeafArea &la, hipStream_t s, int m, int ncols, double *A, int lda,
                    int *ipiv, int *info, int c0, int w, int info_off, bool tourn = false);

// Tournament-pivoting leaf: the same contract as lu_leaf (m x w block at A,
// w <= 32, pivots ipiv[0..w) region-relative 1-based with row0 added, first
// zero pivot into *info, interchanges applied to every column of the
// region), with the pivots chosen by tournament rounds over row blocks of
// CDF_PARAM_TOURN_BLOCK rows, CDF_PARAM_TOURN_FANIN sets per round.  Its
// candidate sets and final block live in `la` from kTournOffset on (beyond
// the exchange area, before the error word).
constexpr size_t kTournOffset = 320 * 1024;
constexpr int kTournMaxSets = 512;
size_t tourn_ws_bytes();
hipError_t tourn_leaf(cdf_handle_t h, const LeafArea &la, hipStream_t s, int m, int w, double *A, int lda,
                      int *ipiv, int row0, int *info, int info_base, double *region, int region_rows,
                      int region_cols);

// Panel-wide interchanges: build (dst, src) pairs of ipiv[k1..k2) (<= 256,
// region-relative, 1-based) once into `pairs` (pairs_ints() ints), then
// apply them to any column range.
size_t pairs_ints();
hipError_t build_pairs(hipStream_t s, const int *ipiv, int k1, int k2, int nrows, int *pairs);
hipError_t apply_pairs(hipStream_t s, int c0, int c1, double *A, int lda, const int *pairs);
hipError_t apply_pairs(hipStream_t s, int c0, int c1, float *A, int lda, const int *pairs);
// ipiv_out[i] = ipiv_in[i] + off for i < count.
hipError_t offset_pivots(hipStream_t s, const int *ipiv_in, int *ipiv_out, int count, int off);
// Block column of a lower Cholesky (m x kb, its diagonal block on top),
// factored in sub-blocks of 64 columns on stream s; info offset by info_off.
hipError_t potrf_panel(cdf_handle_t h, hipStream_t s, int m, int kb, double *A, int lda, int *info, int info_off,
                       bool prio = false);

// Apply interchanges ipiv[k1..k2) (absolute, 1-based) to rows of columns
// [c0, c1) of A (nrows rows); an entry outside [k+1, nrows] is ignored.
hipError_t laswp(hipStream_t s, int c0, int c1, double *A, int lda, const int *ipiv, int k1,
                 int k2, int nrows);
// Sets *p = v on the stream (a kernel, so that graph capture stays clean).
hipError_t fill_int(hipStream_t s, int *p, int count, int v);
// Same for a binary32 matrix.
hipError_t slaswp(hipStream_t s, int c0, int c1, float *A, int lda, const int *ipiv, int k1,
                  int k2, int nrows);

// Triangular solves with a small triangle T (nb <= 512 on the left, <= 256
// on the right) applied to an nb x ncols block B (left side) or an
// nrows x nb block (right side).  Every launch is a no-op while *stop != 0.
// max_wg > 0 caps a left solve's grid (its workgroups loop over column
// blocks): a launch that is usually a no-op then costs few workgroups.
//   left, lower, no-trans, unit:      B <- T^-1 B
//   left, lower, no-trans, non-unit:  B <- T^-1 B
//   left, lower, trans, non-unit:     B <- T^-T B
//   left, upper, no-trans, non-unit:  B <- T^-1 B
//   right, lower, trans, non-unit:    B <- B T^-T
enum TrsmKind { TRSM_LLNU = 0, TRSM_LLNN = 1, TRSM_LLTN = 2, TRSM_LUNN = 3, TRSM_RLTN = 4 };
hipError_t trsm_small(hipStream_t s, TrsmKind kind, int nb, int ncols, const double *T, int ldt,
                      double *B, int ldb, const int *stop = nullptr, int max_wg = 0);
// Same with a binary32 right-hand block (arithmetic in binary64).
hipError_t trsm_small(hipStream_t s, TrsmKind kind, int nb, int ncols, const double *T, int ldt,
                      float *B, int ldb, const int *stop = nullptr, int max_wg = 0);
// B (nrows x nb, nb <= 64) <- B L^-T, L lower non-unit (the right-side solve
// of trsm_small), with the solve's waves at raised priority if prio.
hipError_t trsm_rltn_small(hipStream_t s, int nb, int nrows, const double *T, int ldt, double *B, int ldb,
                           const int *stop, bool prio);

// Full triangular solve with a large n x n factor (blocked: bs-wide diagonal
// solves + GEMM updates; bs <= 256).
hipError_t trsm_blocked(hipStream_t s, TrsmKind kind, int n, int ncols, const double *T, int ldt,
                        double *B, int ldb, int bs = 128, const GemmCtx *ctx = nullptr);
// Solve with few right-hand sides (ncols <= 4): 64-row diagonal blocks solved
// by one wave in registers, off-diagonal blocks applied GEMV-style.  With a
// device work area `sync` of trsv_sync_ints(n) ints (LLNU, LLNN, LUNN), the
// whole solve is one launch whose workgroups hand solved blocks to each
// other through flags; otherwise one launch per 64-row block.
size_t trsv_sync_ints(int n);
hipError_t trsv_blocked(hipStream_t s, TrsmKind kind, int n, int ncols, const double *T, int ldt, double *B,
                        int ldb, int *sync = nullptr);

// Solves through inverted diagonal blocks (many right-hand sides, one factor
// applied many times).  inv_lower_blocks: Tinv block q (bs x bs, leading
// dimension bs, at Tinv + q bs^2; inv_blocks_doubles(n, bs) doubles) =
// inverse of the diagonal block q of the lower non-unit triangle of T
// (bs <= 512).  symmetrize_lower: the strict upper triangle of A receives the
// transpose of its strict lower one.  trsm_inv_lower: Y <- L^-1 X
// (transposed = false) or Y <- L^-T X (transposed = true, reading L^T from
// T's upper triangle as symmetrize_lower leaves it); X is overwritten.
size_t inv_blocks_doubles(int n, int bs);
hipError_t inv_lower_blocks(hipStream_t s, int n, const double *T, int ldt, int bs, double *Tinv);
hipError_t symmetrize_lower(hipStream_t s, int n, double *A, int lda);
hipError_t trsm_inv_lower(hipStream_t s, bool transposed, int n, int nrhs, const double *T, int ldt,
                          const double *Tinv, int bs, double *X, int ldx, double *Y, int ldy);

// Cholesky of one diagonal block (n <= 128) held in LDS; stops at the first
// non-positive pivot, writing info_base + j + 1 into *info if *info == 0.
// *info != 0 on entry makes the kernel return without touching A.
// prio: the block is on the critical chain beside the low-precision update
// (blocks of at most 64 columns then run as one wave at raised priority).
hipError_t potrf_diag(hipStream_t s, int n, double *A, int lda, int *info, int info_base, bool prio = false);

// Mixed-precision helpers.
hipError_t convert_d2s(hipStream_t s, int m, int n, const double *A, int lda, float *W, int ldw,
                       bool lower_only);
hipError_t convert_s2d(hipStream_t s, int m, int n, const float *W, int ldw, double *A, int lda,
                       bool lower_only);
// transpose_out: Q[k + i*ldq] = code(X[i, k]) (K = columns of X), else
// Q[i + j*ldq] = code(X[i, j]) (K = rows of X).  K is zero-padded up to
// min(ldq, 32*ceil(K/32)).
hipError_t quantize(hipStream_t s, int fmt, int m, int n, const float *X, int ldx, int tm, int tn,
                    void *Q, int ldq, int *exps, bool transpose_out);
hipError_t lowp_update(hipStream_t s, int fmt, int m, int n, int k, const void *QA, int lda,
                       const int *ea, const void *QB, int ldb, const int *eb, float *C, int ldc,
                       bool lower, const int *stop);
int lowp_tile(int fmt);

// r = b - A x for nrhs columns, binary64 (A n x n); also writes per-column
// partial infinity norms used by the scaled residual.
hipError_t residual(hipStream_t s, int n, int nrhs, const double *A, int lda, const double *X,
                    int ldx, const double *B, int ldb, double *R, int ldr);
// out[0] = ||A||_inf (max row sum of |a_ij|), using `tmp` (n doubles).
hipError_t norm_inf_rows(hipStream_t s, int n, const double *A, int lda, double *tmp, double *out,
                         bool symmetric_lower);
// per column c: out[3c+0] = max|R|, out[3c+1] = max|X|, out[3c+2] = max|B|
hipError_t col_absmax3(hipStream_t s, int n, int nrhs, const double *R, int ldr, const double *X,
                       int ldx, const double *B, int ldb, double *out);
hipError_t axpy_cols(hipStream_t s, int n, int nrhs, const double *D, int ldd, double *X, int ldx);
hipError_t copy_cols(hipStream_t s, int n, int nrhs, const double *S, int lds, double *D, int ldd);

}  // namespace cdf

#define CDF_HIP_TRY(expr)                                   \
    do {                                                    \
        hipError_t _e = (expr);                             \
        if (_e != hipSuccess) return CDF_ERR_HIP;           \
    } while (0)

#define CDF_HIP_RET(expr)                                   \
    do {                                                    \
        hipError_t _e = (expr);                             \
        if (_e != hipSuccess) return _e;                    \
    } while (0)
