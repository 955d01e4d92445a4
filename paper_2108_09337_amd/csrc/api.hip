// C-ABI entry points of libcdnafact: argument checking, workspace, and the
// blocked right-looking drivers (Sec. 7, Algorithm 1 routines A00 / A10 /
// A01 / A11 on one GPU; Sec. 7.5 for Cholesky).
#include "internal.h"

#include <cmath>
#include <cstring>
#include <new>

namespace {

__global__ void fill_int_kernel(int *p, int count, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// Guard of L^-1: eight columns of Li (kb x kb) per workgroup; an entry
// above `bound` in magnitude (or NaN) clears *good (set to 1 beforehand).
__global__ __launch_bounds__(256) void inverse_check_kernel(int kb, const double *Li, int ldi, double bound,
                                                            int *good) {
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const int j = blockIdx.x * 8 + threadIdx.x / 32;
    int mine = 0;
    if (j < kb)
        for (int i = threadIdx.x % 32; i < kb; i += 32)
            if (!(fabs(Li[(size_t)i + (size_t)j * ldi]) <= bound)) mine = 1;
    if (mine) atomicOr(&bad, 1);
    __syncthreads();
    if (threadIdx.x == 0 && bad) atomicAnd(good, 0);
}

// Li = identity where the guard cleared *good.
__global__ void inverse_reset_kernel(int kb, double *Li, int ldi, const int *good) {
    if (*good != 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i < kb) Li[(size_t)i + (size_t)j * ldi] = i == j ? 1.0 : 0.0;
}

// X (n x n, leading dimension ld) = identity; *flag = 1
__global__ void eye_kernel(int n, double *X, int ld, int *flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i < n) X[(size_t)i + (size_t)j * ld] = i == j ? 1.0 : 0.0;
    if (i == 0 && j == 0) *flag = 1;
}

inline cdf_status_t bad(cdf_handle_t h, int pos) {
    h->bad_arg = pos;
    return CDF_ERR_INVALID_ARG;
}

inline int lu_nb(cdf_handle_t h, int n) {
    const int v = h->params[CDF_PARAM_LU_NB];
    return v > 0 ? v : (n >= 16384 ? 512 : 256);
}

inline int chol_nb(cdf_handle_t h, int n) {
    const int v = h->params[CDF_PARAM_CHOL_NB];
    return v > 0 ? v : (n >= 16384 ? 512 : 128);
}

// LU workspace: the leaf's exchange area, the current panel's pivots (<= 512)
// and the interchange pairs of the last two panels.
constexpr int kMaxLuNb = 512;
constexpr int kPairsInts = 1 + 4 * kMaxLuNb;
constexpr size_t kLuWsBytes = cdf::kLeafWsBytes + (kMaxLuNb + 2 * kPairsInts) * sizeof(int) + 4096;

}  // namespace

namespace cdf {

// Recursive panel factorization of columns [c0, c0 + w) over rows [c0, m) of
// the m x ncols region A: factor the left half, form its U12 and update the
// right half, factor the right half.  Leaves (<= 32 columns) apply their
// interchanges to every other column of the region inside the leaf kernel,
// so the region stays consistently permuted.  Pivots are written relative to the region's row 0;
// info values are offset by info_off.
hipError_t lu_panel(cdf_handle_t h, const LeafArea &la, hipStream_t s, int m, int ncols, double *A, int lda,
                    int *ipiv, int *info, int c0, int w, int info_off, bool tourn) {
    if (w <= 32) {
        if (tourn)
            return tourn_leaf(h, la, s, m - c0, w, A + c0 + (size_t)c0 * lda, lda, ipiv + c0, c0, info,
                              info_off + c0, A, m, ncols);
        return lu_leaf(h, la, s, m - c0, w, A + c0 + (size_t)c0 * lda, lda, ipiv + c0, c0, info, info_off + c0,
                       h->params[CDF_PARAM_LU_LEAF_ROWS], A, m, ncols, c0);
    }
    const int n1 = ((w / 2 + 31) / 32) * 32;
    const int n2 = w - n1;
    CDF_HIP_RET(lu_panel(h, la, s, m, ncols, A, lda, ipiv, info, c0, n1, info_off, tourn));
    double *a11 = A + c0 + (size_t)c0 * lda;
    double *a12 = A + c0 + (size_t)(c0 + n1) * lda;
    double *a21 = A + (c0 + n1) + (size_t)c0 * lda;
    double *a22 = A + (c0 + n1) + (size_t)(c0 + n1) * lda;
    const GemmCtx gc = gemm_ctx(h);
    CDF_HIP_RET(trsm_blocked(s, TRSM_LLNU, n1, n2, a11, lda, a12, lda, 64, &gc));
    CDF_HIP_RET(dgemm(s, 0, 0, m - c0 - n1, n2, n1, -1.0, a21, lda, a12, lda, 1.0, a22, lda, false, nullptr, &gc));
    return lu_panel(h, la, s, m, ncols, A, lda, ipiv, info, c0 + n1, n2, info_off, tourn);
}

// Blocked right-looking lower Cholesky of the n x n matrix A: potrf of each
// diagonal block, trsm of the block column below it, triangular (lower
// tiles only) update of the trailing matrix.  Stops (all later launches are
// no-ops) once *info != 0; info values are offset by info_off.
hipError_t ensure_aux(cdf_handle_t h) {
    if (!h->aux) CDF_HIP_RET(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
    if (!h->aux2) CDF_HIP_RET(hipStreamCreateWithFlags(&h->aux2, hipStreamNonBlocking));
    for (auto &e : h->ev)
        if (!e) CDF_HIP_RET(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return hipSuccess;
}

// Block column of a lower Cholesky: the m x kb column [A11; A21] with its kb
// x kb diagonal block on top, factored right-looking over sub-blocks of at
// most 64 columns (the register-resident right-side solve's limit, so that
// the panel fits beside the update GEMM on another stream); each sub-block
// updates only the rest of this block column.  Launches go to stream s;
// info values are offset by info_off.  prio raises the issue priority of
// the diagonal blocks and solves (measured: a gain beside the low-precision
// SYRK, a loss beside the binary64 update, whose panel is not critical).
hipError_t potrf_panel(cdf_handle_t h, hipStream_t s, int m, int kb, double *A, int lda, int *info, int info_off,
                       bool prio) {
    const GemmCtx gc = gemm_ctx(h);
    constexpr int kSub = 64;
    for (int j = 0; j < kb; j += kSub) {
        const int jb = kSub < kb - j ? kSub : kb - j;
        double *a11 = A + j + (size_t)j * lda;
        CDF_HIP_RET(potrf_diag(s, jb, a11, lda, info, info_off + j, prio));
        const int below = m - j - jb;
        if (below > 0) CDF_HIP_RET(trsm_rltn_small(s, jb, below, a11, lda, a11 + jb, lda, info, prio));
        const int c = j + jb, w = kb - c;  // remaining columns of the block column
        if (w > 0) {
            double *l = A + c + (size_t)j * lda;  // rows [c, m) of the sub-block's L
            CDF_HIP_RET(dgemm(s, 0, 1, w, w, jb, -1.0, l, lda, l, lda, 1.0, A + c + (size_t)c * lda, lda, true, info,
                              &gc));
            if (m - c - w > 0)
                CDF_HIP_RET(dgemm(s, 0, 1, m - c - w, w, jb, -1.0, l + w, lda, l, lda, 1.0,
                                  A + (c + w) + (size_t)c * lda, lda, false, info, &gc));
        }
    }
    return hipSuccess;
}


}  // namespace cdf

namespace {

struct LuWs {
    cdf::LeafArea leaf;  // the leaf's exchange area
    int *ipt;    // region-relative pivots of the current panel
    int *pairs;  // its interchange pairs (one of the two buffers below)
    int *buf[2];
    // Optional (both null: U12 by blocked substitution in place):
    double *W;       // U12 of the current step, kb x (n - k - kb), leading dimension kb
    double *Li[2];   // L11^-1 of panels p (buffer p mod 2), kMaxLuNb x kMaxLuNb
    int *good[2];    // 1: Li holds L11^-1; 0: it was rejected (and is the identity)
};

hipError_t panel_inverse(cdf_handle_t h, hipStream_t s, int kb, const double *l11, int lda, double *Li, int *good) {
    const cdf::GemmCtx gu = cdf::gemm_ctx(h, cdf::PROF_U12);
    return cdf::unit_lower_inverse(s, kb, l11, lda, Li, kMaxLuNb, good, &gu);
}

// Columns [c, c + cols) of step k's block row: U12 = L11^-1 A12 into W
// (columns offset by c - k1), then A22 -= L21 U12, then U12 back into A.
// Where the guard rejected L11^-1 (too large an entry: the product would
// lose the accuracy of substitution), A12 is first solved in place by
// substitution and the GEMM with the identity copies it to W exactly.
// Without the workspace: blocked substitution in place, then the update.
hipError_t u12_and_update(cdf_handle_t h, hipStream_t s, int n, double *A, int lda, int k, int kb, int c, int cols,
                          const LuWs &ws, const double *Li, const int *good) {
    const int k1 = k + kb;
    double *a12 = A + k + (size_t)c * lda;
    const double *a21 = A + k1 + (size_t)k * lda;
    double *a22 = A + k1 + (size_t)c * lda;
    const cdf::GemmCtx gc = cdf::gemm_ctx(h), gu = cdf::gemm_ctx(h, cdf::PROF_U12);
    if (!ws.W) {
        CDF_HIP_RET(cdf::trsm_blocked(s, cdf::TRSM_LLNU, kb, cols, A + k + (size_t)k * lda, lda, a12, lda, 64, &gu));
        return cdf::dgemm(s, 0, 0, n - k1, cols, kb, -1.0, a21, lda, a12, lda, 1.0, a22, lda, false, nullptr, &gc);
    }
    double *w = ws.W + (size_t)(c - k1) * kb;
    CDF_HIP_RET(cdf::trsm_small(s, cdf::TRSM_LLNU, kb, cols, A + k + (size_t)k * lda, lda, a12, lda, good, 512));
    CDF_HIP_RET(cdf::dgemm(s, 0, 0, kb, cols, kb, 1.0, Li, kMaxLuNb, a12, lda, 0.0, w, kb, false, nullptr, &gu));
    CDF_HIP_RET(cdf::dgemm(s, 0, 0, n - k1, cols, kb, -1.0, a21, lda, w, kb, 1.0, a22, lda, false, nullptr, &gc));
    return hipMemcpy2DAsync(a12, (size_t)lda * sizeof(double), w, (size_t)kb * sizeof(double), (size_t)kb * sizeof(double),
                            cols, hipMemcpyDeviceToDevice, s);
}

// Panel [k, k+kb) over rows [k, n) as a region: pivots relative to row k in
// ws.ipt, absolute (1-based) in ipiv[k..k+kb), pairs built for the region.
hipError_t factor_panel(cdf_handle_t h, hipStream_t s, int n, double *A, int lda, int *ipiv, int *info, int k,
                        int kb, LuWs &ws, int nb) {
    double *R = A + k + (size_t)k * lda;
    CDF_HIP_RET(cdf::lu_panel(h, ws.leaf, s, n - k, kb, R, lda, ws.ipt, info, 0, kb, k,
                              h->params[CDF_PARAM_LU_PIVOT] == 1));
    CDF_HIP_RET(cdf::offset_pivots(s, ws.ipt, ipiv + k, kb, k));
    CDF_HIP_RET(cdf::build_pairs(s, ws.ipt, 0, kb, n - k, ws.pairs));
    // the inverse is needed only while columns remain right of the panel
    if (ws.W && k + kb < n) CDF_HIP_RET(panel_inverse(h, s, kb, R, lda, ws.Li[(k / nb) & 1], ws.good[(k / nb) & 1]));
    return hipSuccess;
}

// Blocked right-looking LU with look-ahead of depth one: while the trailing
// update of panel k runs on the handle's stream, panel k+1 (whose columns
// were updated first) is factored on a second stream; its interchanges are
// applied to the trailing columns once both are done.  Their application to
// the finished L columns to the left, which no later step reads, runs on a
// third stream beside the next steps (panel p's pairs live in buffer p mod 2,
// so panel p+2 waits for that stream's use of panel p's pairs).  On the
// trailing columns, only the next panel's are swapped on the handle's stream;
// the rest are swapped on the third stream while the next panel's columns are
// updated, and the handle's stream waits for them before updating the rest.
// With one_stream, the same schedule is issued in the same order on the
// handle's stream alone (no second or third stream, no events).
hipError_t getrf_impl(cdf_handle_t h, const cdf::LeafArea &la, bool one_stream, int n, double *A, int lda,
                      int *ipiv, int *info, int *ipt, int *pairs, double *W, double *Li) {
    hipStream_t s0 = h->stream, s1 = s0, s2 = s0;
    if (!one_stream) {
        CDF_HIP_RET(cdf::ensure_aux(h));
        s1 = h->aux;
        s2 = h->aux2;
    }
    // event record / wait between two of the streams (nothing on one stream,
    // where submission order already orders the work)
    auto rec = [&](hipEvent_t e, hipStream_t s) { return one_stream ? hipSuccess : hipEventRecord(e, s); };
    auto wait = [&](hipStream_t s, hipEvent_t e) { return one_stream ? hipSuccess : hipStreamWaitEvent(s, e, 0); };
    hipEvent_t *left_done = h->ev + 3;  // per pairs buffer
    hipEvent_t rest_swapped = h->ev[5];
    CDF_HIP_RET(cdf::fill_int(s0, info, 1, 0));
    CDF_HIP_RET(cdf::leaf_reset_error(la, s0));
    h->last_err = cdf::leaf_error_word(la);
    const int nb = lu_nb(h, n);
    LuWs ws;
    ws.leaf = la;
    ws.ipt = ipt;
    ws.buf[0] = pairs;
    ws.buf[1] = pairs + kPairsInts;
    ws.pairs = ws.buf[0];
    ws.W = W;
    ws.Li[0] = Li;
    ws.Li[1] = Li ? Li + (size_t)kMaxLuNb * kMaxLuNb : nullptr;
    ws.good[0] = Li ? reinterpret_cast<int *>(Li + 2 * (size_t)kMaxLuNb * kMaxLuNb) : nullptr;
    ws.good[1] = ws.good[0] ? ws.good[0] + 1 : nullptr;
    // the third stream starts after everything already queued on the handle's
    CDF_HIP_RET(rec(h->ev[2], s0));
    CDF_HIP_RET(wait(s2, h->ev[2]));
    const int kb0 = nb < n ? nb : n;
    CDF_HIP_RET(factor_panel(h, s0, n, A, lda, ipiv, info, 0, kb0, ws, nb));
    CDF_HIP_RET(cdf::apply_pairs(s0, kb0, n, A, lda, ws.pairs));
    for (int k = 0; k < n; k += nb) {
        const int kb = nb < n - k ? nb : n - k;
        const int k1 = k + kb;
        if (k1 >= n) break;
        const int kb1 = nb < n - k1 ? nb : n - k1;
        const int rest = n - k1;
        const int b = (k1 / nb) & 1;  // pairs buffer of panel k1
        ws.pairs = ws.buf[b];
        const double *li = ws.Li[(k / nb) & 1];
        const int *good = ws.good[(k / nb) & 1];
        // next panel's columns first
        CDF_HIP_RET(u12_and_update(h, s0, n, A, lda, k, kb, k1, kb1, ws, li, good));
        if (rest > kb1) {
            CDF_HIP_RET(rec(h->ev[0], s0));
            CDF_HIP_RET(wait(s1, h->ev[0]));
            CDF_HIP_RET(wait(s1, left_done[b]));
            CDF_HIP_RET(factor_panel(h, s1, n, A, lda, ipiv, info, k1, kb1, ws, nb));
            CDF_HIP_RET(rec(h->ev[1], s1));
            const int c2 = k1 + kb1;
            CDF_HIP_RET(wait(s0, rest_swapped));
            CDF_HIP_RET(u12_and_update(h, s0, n, A, lda, k, kb, c2, n - c2, ws, li, good));
            CDF_HIP_RET(wait(s0, h->ev[1]));
        } else {
            CDF_HIP_RET(wait(s0, left_done[b]));
            CDF_HIP_RET(factor_panel(h, s0, n, A, lda, ipiv, info, k1, kb1, ws, nb));
        }
        // panel k1's interchanges: columns [0, k1) (their last reader, this
        // step's update, is done) and those right of the panel after next on
        // the third stream; the next panel's columns here
        const int c2 = k1 + kb1, kb2 = nb < n - c2 ? nb : n - c2, c3 = c2 + (kb2 > 0 ? kb2 : 0);
        CDF_HIP_RET(rec(h->ev[2], s0));
        CDF_HIP_RET(wait(s2, h->ev[2]));
        if (c3 < n) {
            CDF_HIP_RET(cdf::apply_pairs(s2, c3, n, A + k1, lda, ws.pairs));
            CDF_HIP_RET(rec(rest_swapped, s2));
        }
        CDF_HIP_RET(cdf::apply_pairs(s2, 0, k1, A + k1, lda, ws.pairs));
        CDF_HIP_RET(rec(left_done[b], s2));
        CDF_HIP_RET(cdf::apply_pairs(s0, c2, c3 < n ? c3 : n, A + k1, lda, ws.pairs));
    }
    CDF_HIP_RET(rec(h->ev[2], s2));
    CDF_HIP_RET(wait(s0, h->ev[2]));
    return hipSuccess;
}

// Blocked right-looking lower Cholesky with look-ahead of depth one: the
// next block column is updated first, then its diagonal block (potrf) and
// L21 (trsm) run on the second stream while the rest of the trailing lower
// triangle is updated on the handle's stream.  Only the lower triangle is
// touched; every launch after a failed pivot is a no-op (stop = info).
hipError_t potrf_impl(cdf_handle_t h, int n, double *A, int lda, int *info) {
    hipStream_t s0 = h->stream;
    const cdf::GemmCtx gc = cdf::gemm_ctx(h);
    CDF_HIP_RET(cdf::ensure_aux(h));
    hipStream_t s1 = h->aux;
    CDF_HIP_RET(cdf::fill_int(s0, info, 1, 0));
    const int nb = chol_nb(h, n);
    // block column [k, k+kb) over rows [k, n)
    auto panel = [&](hipStream_t s, int k, int kb) -> hipError_t {
        return cdf::potrf_panel(h, s, n - k, kb, A + k + (size_t)k * lda, lda, info, k);
    };
    CDF_HIP_RET(panel(s0, 0, nb < n ? nb : n));
    for (int k = 0; k < n; k += nb) {
        const int kb = nb < n - k ? nb : n - k;
        const int k1 = k + kb;
        if (k1 >= n) break;
        const int kb1 = nb < n - k1 ? nb : n - k1;
        const int rest = n - k1;
        double *l21 = A + k1 + (size_t)k * lda;                 // rest x kb
        double *d1 = A + k1 + (size_t)k1 * lda;                 // next diagonal block
        // next block column: its diagonal block (lower only) and the rows below it
        CDF_HIP_RET(cdf::dgemm(s0, 0, 1, kb1, kb1, kb, -1.0, l21, lda, l21, lda, 1.0, d1, lda, true, info, &gc));
        if (rest > kb1)
            CDF_HIP_RET(cdf::dgemm(s0, 0, 1, rest - kb1, kb1, kb, -1.0, l21 + kb1, lda, l21, lda, 1.0, d1 + kb1, lda,
                                   false, info, &gc));
        if (rest > kb1) {
            CDF_HIP_RET(hipEventRecord(h->ev[0], s0));
            CDF_HIP_RET(hipStreamWaitEvent(s1, h->ev[0], 0));
            CDF_HIP_RET(panel(s1, k1, kb1));
            CDF_HIP_RET(hipEventRecord(h->ev[1], s1));
            const int c2 = k1 + kb1;
            CDF_HIP_RET(cdf::dgemm(s0, 0, 1, n - c2, n - c2, kb, -1.0, l21 + kb1, lda, l21 + kb1, lda, 1.0,
                                   A + c2 + (size_t)c2 * lda, lda, true, info, &gc));
            CDF_HIP_RET(hipStreamWaitEvent(s0, h->ev[1], 0));
        } else {
            CDF_HIP_RET(panel(s0, k1, kb1));
        }
    }
    return hipSuccess;
}

}  // namespace

namespace cdf {

size_t getrf_ws_ints() { return kMaxLuNb + 2 * kPairsInts; }

size_t getrf_w_doubles(int n) { return (size_t)kMaxLuNb * n + 2 * (size_t)kMaxLuNb * kMaxLuNb + 32; }

hipError_t getrf_fp64(cdf_handle_t h, int n, double *A, int lda, int *ipiv, int *info, int *ws_ints,
                      double *lu_w) {
    const bool inv = lu_w != nullptr && h->params[CDF_PARAM_LU_U12] == 0;
    return getrf_impl(h, cdf::handle_leaf_area(h), false, n, A, lda, ipiv, info, ws_ints, ws_ints + kMaxLuNb,
                      inv ? lu_w : nullptr, inv ? lu_w + (size_t)kMaxLuNb * n : nullptr);
}

hipError_t getrf_inplace_one_stream(cdf_handle_t h, const LeafArea &la, int n, double *A, int lda, int *ipiv,
                                    int *info, int *ws_ints) {
    return getrf_impl(h, la, true, n, A, lda, ipiv, info, ws_ints, ws_ints + kMaxLuNb, nullptr, nullptr);
}

hipError_t potrf_fp64(cdf_handle_t h, int n, double *A, int lda, int *info) {
    return potrf_impl(h, n, A, lda, info);
}

__global__ void offset_kernel(const int *__restrict__ a, int *__restrict__ b, int count, int off) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) b[i] = a[i] + off;
}

hipError_t offset_pivots(hipStream_t s, const int *ipiv_in, int *ipiv_out, int count, int off) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(offset_kernel, dim3((count + 255) / 256), dim3(256), 0, s, ipiv_in, ipiv_out, count, off);
    return hipGetLastError();
}

// L^-1 of the unit lower triangle L (kb x kb) into Li: identity, then
// blocked forward substitution (the same solve the in-place U12 path uses,
// with the identity as right-hand side).
hipError_t unit_lower_inverse(hipStream_t s, int kb, const double *L, int ldl, double *Li, int ldi, int *good,
                              const GemmCtx *ctx) {
    if (kb <= 0) return hipSuccess;
    hipLaunchKernelGGL(eye_kernel, dim3((kb + 255) / 256, kb), dim3(256), 0, s, kb, Li, ldi, good);
    CDF_HIP_RET(hipGetLastError());
    CDF_HIP_RET(trsm_blocked(s, TRSM_LLNU, kb, kb, L, ldl, Li, ldi, 64, ctx));
    // accepted while no entry exceeds kInverseBound: pivoting keeps
    // |L(i,j)| <= 1, and for the inverse's growth the products' rounding
    // error stays within a small multiple of substitution's
    hipLaunchKernelGGL(inverse_check_kernel, dim3((kb + 7) / 8), dim3(256), 0, s, kb, Li, ldi, kInverseBound, good);
    CDF_HIP_RET(hipGetLastError());
    hipLaunchKernelGGL(inverse_reset_kernel, dim3((kb + 255) / 256, kb), dim3(256), 0, s, kb, Li, ldi, good);
    return hipGetLastError();
}

hipError_t fill_int(hipStream_t s, int *p, int count, int v) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_int_kernel, dim3((count + 255) / 256), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

cdf_status_t ws_reserve(cdf_handle_t h, size_t bytes) {
    if (bytes <= h->ws_bytes) return CDF_OK;
    if (h->ws_limit && bytes > h->ws_limit) return CDF_ERR_ALLOC;
    const size_t want = align_up(bytes, (size_t)1 << 20);
    if (h->ws) {
        if (hipStreamSynchronize(h->stream) != hipSuccess) return CDF_ERR_HIP;
        (void)hipFree(h->ws);
        h->ws = nullptr;
        h->ws_bytes = 0;
        h->last_err = nullptr;
    }
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return CDF_ERR_ALLOC;
    }
    h->ws = p;
    h->ws_bytes = want;
    h->leaf_epoch = 0;  // fresh memory: the leaf re-zeroes its tag area before use
    return CDF_OK;
}

}  // namespace cdf

extern "C" {

cdf_status_t cdf_create(cdf_handle_t *h) {
    if (!h) return CDF_ERR_INVALID_ARG;
    *h = nullptr;
    cdf_handle_s *p = new (std::nothrow) cdf_handle_s();
    if (!p) return CDF_ERR_ALLOC;
    if (hipGetDevice(&p->device) != hipSuccess) { delete p; return CDF_ERR_HIP; }
    int cus = 0, khz = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cus > 0)
        p->num_cus = cus;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, p->device) == hipSuccess && khz > 0)
        p->wall_khz = khz;
    // the allocation-free LU's scratch address on this device (a failure
    // only disables that entry point, which then returns CDF_ERR_HIP)
    (void)cdf::noalloc_setup(p->device);
    *h = p;
    return CDF_OK;
}

cdf_status_t cdf_destroy(cdf_handle_t h) {
    if (!h) return CDF_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(h->stream);
    if (h->ws) (void)hipFree(h->ws);
    if (h->aux) { (void)hipStreamSynchronize(h->aux); (void)hipStreamDestroy(h->aux); }
    if (h->aux2) { (void)hipStreamSynchronize(h->aux2); (void)hipStreamDestroy(h->aux2); }
    for (auto &e : h->ev)
        if (e) (void)hipEventDestroy(e);
    cdf::prof_free(h->prof);
    delete h;
    return CDF_OK;
}

cdf_status_t cdf_device_status(cdf_handle_t h) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->bad_arg = 0;
    CDF_HIP_TRY(hipStreamSynchronize(h->stream));
    if (h->aux) CDF_HIP_TRY(hipStreamSynchronize(h->aux));
    if (h->aux2) CDF_HIP_TRY(hipStreamSynchronize(h->aux2));
    if (!h->last_err) return CDF_OK;
    int e = 0;
    CDF_HIP_TRY(hipMemcpy(&e, h->last_err, sizeof(int), hipMemcpyDeviceToHost));
    return e != 0 ? CDF_ERR_TIMEOUT : CDF_OK;
}

cdf_status_t cdf_profile_begin(cdf_handle_t h) {
    if (!h) return CDF_ERR_INVALID_ARG;
    CDF_HIP_TRY(cdf::prof_enable(&h->prof));
    return CDF_OK;
}

cdf_status_t cdf_profile_end(cdf_handle_t h, int kernel, long long *launches, double *total_ms, double *flops,
                             double *bytes) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->bad_arg = 0;
    if (kernel < 0 || kernel >= cdf::PROF_KINDS) { h->bad_arg = 2; return CDF_ERR_INVALID_ARG; }
    if (!launches) { h->bad_arg = 3; return CDF_ERR_INVALID_ARG; }
    if (!total_ms) { h->bad_arg = 4; return CDF_ERR_INVALID_ARG; }
    if (!flops) { h->bad_arg = 5; return CDF_ERR_INVALID_ARG; }
    if (!bytes) { h->bad_arg = 6; return CDF_ERR_INVALID_ARG; }
    CDF_HIP_TRY(cdf::prof_collect(h->prof, kernel, launches, total_ms, flops, bytes));
    return CDF_OK;
}

cdf_status_t cdf_set_stream(cdf_handle_t h, void *stream) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->stream = static_cast<hipStream_t>(stream);
    return CDF_OK;
}

cdf_status_t cdf_set_workspace_limit(cdf_handle_t h, size_t bytes) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->ws_limit = bytes;
    return CDF_OK;
}

size_t cdf_workspace_bytes(cdf_handle_t h) { return h ? h->ws_bytes : 0; }

int cdf_last_bad_arg(cdf_handle_t h) { return h ? h->bad_arg : 0; }

const char *cdf_status_string(cdf_status_t s) {
    switch (s) {
        case CDF_OK: return "CDF_OK";
        case CDF_ERR_INVALID_ARG: return "CDF_ERR_INVALID_ARG";
        case CDF_ERR_HIP: return "CDF_ERR_HIP";
        case CDF_ERR_ALLOC: return "CDF_ERR_ALLOC";
        case CDF_ERR_NOT_CONVERGED: return "CDF_ERR_NOT_CONVERGED";
        case CDF_ERR_UNSUPPORTED: return "CDF_ERR_UNSUPPORTED";
        case CDF_ERR_TIMEOUT: return "CDF_ERR_TIMEOUT";
    }
    return "CDF_ERR_UNKNOWN";
}

cdf_status_t cdf_set_param(cdf_handle_t h, cdf_param_t p, int value) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->bad_arg = 0;
    if ((int)p < 0 || (int)p >= CDF_PARAM_COUNT) return bad(h, 2);
    if (value < 0) return bad(h, 3);
    if ((p == CDF_PARAM_LU_NB || p == CDF_PARAM_CHOL_NB || p == CDF_PARAM_MIXED_NB) && value != 0 &&
        (value % 32 != 0 || value > kMaxLuNb))
        return bad(h, 3);
    if (p == CDF_PARAM_LU_LEAF_ROWS && !(value == 0 || value == 1 || value == 2)) return bad(h, 3);
    if (p == CDF_PARAM_VBATCH_NB && !(value == 0 || value == 16)) return bad(h, 3);
    if (p == CDF_PARAM_VBATCH_WG_PER_CU && value > 2) return bad(h, 3);
    if (p == CDF_PARAM_GEMM_WG_PER_CU && !(value == 0 || (value >= 3 && value <= 5))) return bad(h, 3);
    if (p == CDF_PARAM_LU_U12 && value > 1) return bad(h, 3);
    if (p == CDF_PARAM_TEST_EXCHANGE_FAIL && value > 1) return bad(h, 3);
    if (p == CDF_PARAM_SPD_REFINE && value > 2) return bad(h, 3);
    if (p == CDF_PARAM_GEMM_TILE && !(value == 0 || value == 64 || value == 128)) return bad(h, 3);
    if (p == CDF_PARAM_LU_PIVOT && value > 1) return bad(h, 3);
    if (p == CDF_PARAM_TOURN_BLOCK && value != 0 && (value < 32 || value > 256)) return bad(h, 3);
    if (p == CDF_PARAM_TOURN_FANIN && value != 0 && (value < 2 || value > 8)) return bad(h, 3);
    h->params[p] = value;
    return CDF_OK;
}

cdf_status_t cdf_mixed_report(cdf_handle_t h, int *method, double *shift, int *factorizations, int *corrections,
                              int *pcg_iterations) {
    if (!h) return CDF_ERR_INVALID_ARG;
    const cdf::MixedReport &r = h->mixed_report;
    if (method) *method = r.method;
    if (shift) *shift = r.shift;
    if (factorizations) *factorizations = r.factorizations;
    if (corrections) *corrections = r.corrections;
    if (pcg_iterations) *pcg_iterations = r.pcg_iterations;
    return CDF_OK;
}

int cdf_get_param(cdf_handle_t h, cdf_param_t p) {
    if (!h || (int)p < 0 || (int)p >= CDF_PARAM_COUNT) return -1;
    return h->params[p];
}

cdf_status_t cdf_dgetrf(cdf_handle_t h, int n, double *A, int lda, int *ipiv, int *info) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->bad_arg = 0;
    if (n < 0) return bad(h, 2);
    if (lda < (n > 1 ? n : 1)) return bad(h, 4);
    if (n > 0 && !A) return bad(h, 3);
    if (n > 0 && !ipiv) return bad(h, 5);
    if (!info) return bad(h, 6);
    if (n == 0) {
        CDF_HIP_TRY(cdf::fill_int(h->stream, info, 1, 0));
        return CDF_OK;
    }
    // U12 through L11^-1 needs kMaxLuNb x n doubles for U12 and two inverses;
    // if the workspace cap refuses them, U12 is solved in place instead.
    const size_t off = cdf::align_up(kLuWsBytes, 256);
    const size_t big = off + cdf::getrf_w_doubles(n) * sizeof(double);
    double *W = nullptr, *Li = nullptr;
    if (h->params[CDF_PARAM_LU_U12] == 0 && cdf::ws_reserve(h, big) == CDF_OK) {
        W = reinterpret_cast<double *>(static_cast<char *>(h->ws) + off);
        Li = W + (size_t)kMaxLuNb * n;
    } else {
        cdf_status_t st = cdf::ws_reserve(h, kLuWsBytes);
        if (st != CDF_OK) return st;
    }
    char *base = static_cast<char *>(h->ws) + cdf::kLeafWsBytes;
    CDF_HIP_TRY(getrf_impl(h, cdf::handle_leaf_area(h), false, n, A, lda, ipiv, info, reinterpret_cast<int *>(base),
                           reinterpret_cast<int *>(base + kMaxLuNb * sizeof(int)), W, Li));
    return CDF_OK;
}

// Flag area of the single-launch few-right-hand-side solves, after the leaf's
// exchange area (the LU's own work area there is idle once it has returned
// on this stream); null (one launch per block) if the workspace cannot grow.
static int *solve_sync(cdf_handle_t h, int n) {
    if (cdf::ws_reserve(h, cdf::kLeafWsBytes + cdf::trsv_sync_ints(n) * sizeof(int)) != CDF_OK) return nullptr;
    return reinterpret_cast<int *>(static_cast<char *>(h->ws) + cdf::kLeafWsBytes);
}

cdf_status_t cdf_dgetrs(cdf_handle_t h, char trans, int n, int nrhs, const double *A, int lda, const int *ipiv,
                        double *B, int ldb) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->bad_arg = 0;
    if (trans != 'N' && trans != 'n') {
        if (trans == 'T' || trans == 't' || trans == 'C' || trans == 'c') return CDF_ERR_UNSUPPORTED;
        return bad(h, 2);
    }
    if (n < 0) return bad(h, 3);
    if (nrhs < 0) return bad(h, 4);
    if (lda < (n > 1 ? n : 1)) return bad(h, 6);
    if (ldb < (n > 1 ? n : 1)) return bad(h, 9);
    if (n == 0 || nrhs == 0) return CDF_OK;
    if (!A) return bad(h, 5);
    if (!ipiv) return bad(h, 7);
    if (!B) return bad(h, 8);
    hipStream_t s = h->stream;
    CDF_HIP_TRY(cdf::laswp(s, 0, nrhs, B, ldb, ipiv, 0, n, n));
    if (nrhs <= 4) {
        int *sync = solve_sync(h, n);
        CDF_HIP_TRY(cdf::trsv_blocked(s, cdf::TRSM_LLNU, n, nrhs, A, lda, B, ldb, sync));
        CDF_HIP_TRY(cdf::trsv_blocked(s, cdf::TRSM_LUNN, n, nrhs, A, lda, B, ldb, sync));
        return CDF_OK;
    }
    CDF_HIP_TRY(cdf::trsm_blocked(s, cdf::TRSM_LLNU, n, nrhs, A, lda, B, ldb));
    CDF_HIP_TRY(cdf::trsm_blocked(s, cdf::TRSM_LUNN, n, nrhs, A, lda, B, ldb));
    return CDF_OK;
}

cdf_status_t cdf_dpotrf(cdf_handle_t h, char uplo, int n, double *A, int lda, int *info) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->bad_arg = 0;
    if (uplo != 'L' && uplo != 'l') {
        if (uplo == 'U' || uplo == 'u') return CDF_ERR_UNSUPPORTED;
        return bad(h, 2);
    }
    if (n < 0) return bad(h, 3);
    if (lda < (n > 1 ? n : 1)) return bad(h, 5);
    if (n > 0 && !A) return bad(h, 4);
    if (!info) return bad(h, 6);
    if (n == 0) {
        CDF_HIP_TRY(cdf::fill_int(h->stream, info, 1, 0));
        return CDF_OK;
    }
    CDF_HIP_TRY(potrf_impl(h, n, A, lda, info));
    return CDF_OK;
}

cdf_status_t cdf_dpotrs(cdf_handle_t h, char uplo, int n, int nrhs, const double *A, int lda, double *B,
                        int ldb) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->bad_arg = 0;
    if (uplo != 'L' && uplo != 'l') {
        if (uplo == 'U' || uplo == 'u') return CDF_ERR_UNSUPPORTED;
        return bad(h, 2);
    }
    if (n < 0) return bad(h, 3);
    if (nrhs < 0) return bad(h, 4);
    if (lda < (n > 1 ? n : 1)) return bad(h, 6);
    if (ldb < (n > 1 ? n : 1)) return bad(h, 8);
    if (n == 0 || nrhs == 0) return CDF_OK;
    if (!A) return bad(h, 5);
    if (!B) return bad(h, 7);
    hipStream_t s = h->stream;
    if (nrhs <= 4) {
        CDF_HIP_TRY(cdf::trsv_blocked(s, cdf::TRSM_LLNN, n, nrhs, A, lda, B, ldb, solve_sync(h, n)));
        CDF_HIP_TRY(cdf::trsv_blocked(s, cdf::TRSM_LLTN, n, nrhs, A, lda, B, ldb));
        return CDF_OK;
    }
    CDF_HIP_TRY(cdf::trsm_blocked(s, cdf::TRSM_LLNN, n, nrhs, A, lda, B, ldb));
    CDF_HIP_TRY(cdf::trsm_blocked(s, cdf::TRSM_LLTN, n, nrhs, A, lda, B, ldb));
    return CDF_OK;
}

cdf_status_t cdf_dgemm_update(cdf_handle_t h, int m, int n, int k, const double *A, int lda, const double *B,
                              int ldb, double *C, int ldc) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->bad_arg = 0;
    if (m < 0) return bad(h, 2);
    if (n < 0) return bad(h, 3);
    if (k < 0) return bad(h, 4);
    if (lda < (m > 1 ? m : 1)) return bad(h, 6);
    if (ldb < (k > 1 ? k : 1)) return bad(h, 8);
    if (ldc < (m > 1 ? m : 1)) return bad(h, 10);
    if (m == 0 || n == 0 || k == 0) return CDF_OK;
    if (!A) return bad(h, 5);
    if (!B) return bad(h, 7);
    if (!C) return bad(h, 9);
    const cdf::GemmCtx gc = cdf::gemm_ctx(h);
    CDF_HIP_TRY(cdf::dgemm(h->stream, 0, 0, m, n, k, -1.0, A, lda, B, ldb, 1.0, C, ldc, false, nullptr, &gc));
    return CDF_OK;
}

double cdf_io_lower_bound_elems(int kind, double n, double m_elems) {
    if (!(m_elems > 0.0) || n < 0.0) return -1.0;
    const double sm = std::sqrt(m_elems);
    if (kind == 0) return (2.0 * n * n * n - 6.0 * n * n + 4.0 * n) / (3.0 * sm) + n * (n - 1.0) / 2.0;
    if (kind == 1) return n * n * n / (3.0 * sm) + n * n / 2.0 + n;
    return -1.0;
}

}  // extern "C"
