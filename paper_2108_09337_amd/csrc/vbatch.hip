// Batched small factorizations of uneven sizes in one persistent launch.
//
// The plan sorts the problems by estimated cost, largest first (longest-
// processing-time order).  A run is two launches: a gather kernel writes one
// descriptor per problem in that order (pointer, order, leading dimension,
// pivots, info) from the caller's arrays and clears the work counter, then
// the persistent kernel's workgroups repeatedly take the next problem from
// the counter (claiming the following one while they factor) and factor it
// alone, blocked right-looking as in Sec. 7 with a panel of NB columns:
//   LU       : panel with partial pivoting (argmax by wave shuffles), row
//              interchanges on the other columns, U12 = L11^-1 A12 in
//              registers, trailing update A22 -= L21 U12 on the matrix cores
//              with both operands from LDS;
//   Cholesky : panel = potrf of the diagonal block and L21 in one pass
//              (Sec. 6.2 statements on the panel), trailing lower update.
// Every workgroup exits once the counter passes the batch size.
#include "internal.h"
#include "pairs.h"
#include "wave.h"

#include <algorithm>
#include <climits>
#include <new>
#include <numeric>
#include <type_traits>
#include <vector>

namespace {

constexpr int NT = 512;  // threads per workgroup: the panels keep one row per thread up to n = 512
constexpr int UC = 64;          // U12 columns staged in LDS per chunk
constexpr size_t LDS_BYTES = 144 * 1024;

// One problem as the persistent kernel sees it, in schedule order: built
// from the caller's pointer arrays by a gather kernel before each run, so a
// workgroup reaches its next problem with one uniform load.
struct __align__(16) VDesc {
    void *A;
    int *ipiv;  // null for Cholesky
    int *info;
    int n, kind, lda, pad;
};

template <typename T>
__device__ inline T tabs(T x) { return x < T(0) ? -x : x; }

// Global-memory view of the problems' pointers, which the kernel reads from
// memory (generic pointers otherwise): their loads and stores then count only
// against the vector-memory counter, and an LDS wait before a barrier does
// not also wait for them.
template <typename T>
using G = __attribute__((address_space(1))) T;

// Panel width for an n x n problem: 32 if the n x 32 panel fits in 128 KB
// (with a 32 x 64 U12 chunk beside it: the kernel's 144 KB), else 16.
template <typename T>
__host__ __device__ inline int panel_nb(int n, int nb_pref) {
    if (nb_pref == 16) return 16;
    return (size_t)n * 32 * sizeof(T) <= 128 * 1024 ? 32 : 16;
}

template <typename T>
__device__ __attribute__((always_inline)) void block_argmax(T v, int idx, T *rv, int *ri, int *out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off >= 1; off >>= 1) {
        const T ov = __shfl_xor(v, off);
        const int oi = __shfl_xor(idx, off);
        if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
    }
    if (lane == 0) { rv[wave] = v; ri[wave] = idx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        T bv = rv[0];
        int bi = ri[0];
        for (int w = 1; w < NT / 64; ++w)
            if (rv[w] > bv || (rv[w] == bv && ri[w] < bi)) { bv = rv[w]; bi = ri[w]; }
        *out = bi;
    }
    __syncthreads();
}

// Trailing update C (rows x cols at C, ldc) -= L (rows x kb, LDS, ld ldl) *
// U (kb x cols, LDS, U(k, c) at U[k * ldu + c]); lower: only entries with
// row + diag >= col.  On the matrix cores (FP64 16x16x4 / FP32 16x16x4
// MFMA): the product is formed transposed, D = -(U^T) (L^T), so that a
// lane's results lie down a column of C (16 consecutive rows: coalesced).
// Each wave takes 32 x 32 blocks of C in turn (2 x 2 MFMA blocks, four
// independent accumulators) and loads the next block's C while it works on
// the current one.
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ static v4 op(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    // result register v of lane (li + 16 lk) holds D row 4 v + lk
    __device__ static int drow(int v, int lk) { return 4 * v + lk; }
};
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ static v4 op(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    // result register v of lane (li + 16 lk) holds D row 4 lk + v
    __device__ static int drow(int v, int lk) { return 4 * lk + v; }
};

template <typename T, int NB>
__device__ __attribute__((always_inline)) void lds_update(G<T> *C, int ldc, int rows, int cols, int kb, const T *L,
                                                          int ldl, const T *U, int ldu, bool lower, int diag) {
    typedef typename Mfma<T>::v4 v4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nbr = (rows + 31) / 32, nbc = (cols + 31) / 32, nblk = nbr * nbc;
    // block b covers rows [32 (b % nbr), +32), columns [32 (b / nbr), +32);
    // those wholly above the diagonal are skipped
    auto skip = [&](int b) { return lower && 32 * (b % nbr) + 31 + diag < 32 * (b / nbr); };
    auto next_block = [&](int b) {
        do b += NT / 64; while (b < nblk && skip(b));
        return b;
    };
    // C entry of result register v, MFMA block (i, j), of block b: row
    // r0 + 16 i + li, column c0 + 16 j + D row
    // Every load is issued (out-of-range ones read C[0] and are discarded):
    // no load sits in a branch, so the wait counts stay exact and the next
    // block's loads are not waited for by this block's products.
    auto load = [&](int b, v4 (&acc)[2][2]) {
        const bool live = b < nblk;
        const int r0 = live ? 32 * (b % nbr) : 0, c0 = live ? 32 * (b / nbr) : 0;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = r0 + 16 * i + li, c = c0 + 16 * j + Mfma<T>::drow(v, lk);
                    const bool ok = live && r < rows && c < cols;
                    const T val = C[ok ? (size_t)r + (size_t)c * ldc : 0];
                    acc[i][j][v] = ok ? -val : T(0);
                }
    };
    int b = wave;
    if (b < nblk && skip(b)) b = next_block(b);
    v4 cur[2][2], nxt[2][2];
    load(b, cur);
    while (b < nblk) {
        const int bn = next_block(b);
        load(bn, nxt);
        const int r0 = 32 * (b % nbr), c0 = 32 * (b / nbr);
        // the accumulators hold -C: D = (U^T)(L^T) - C^T, stored negated.
        // All NB / 4 steps, unrolled; a block inside the matrix with a full
        // panel reads its operands without checks, an edge block reads them
        // clamped to element 0 and zeroes what lies outside.
        auto steps = [&](auto edge_tag) {
            constexpr bool EDGE = decltype(edge_tag)::value;
#pragma unroll 2
            for (int k0 = 0; k0 < NB; k0 += 4) {
                const int kk = k0 + lk;
                T a[2], bb[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) {  // A operand: (U^T)[c][k], c = column of C
                    const int c = c0 + 16 * j + li;
                    if (EDGE) {
                        const bool ok = kk < kb && c < cols;
                        const T u = U[ok ? kk * ldu + c : 0];
                        a[j] = ok ? u : T(0);
                    } else {
                        a[j] = U[kk * ldu + c];
                    }
                }
#pragma unroll
                for (int i = 0; i < 2; ++i) {  // B operand: (L^T)[k][r], r = row of C
                    const int r = r0 + 16 * i + li;
                    if (EDGE) {
                        const bool ok = kk < kb && r < rows;
                        const T l = L[ok ? kk * ldl + r : 0];
                        bb[i] = ok ? l : T(0);
                    } else {
                        bb[i] = L[kk * ldl + r];
                    }
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) cur[i][j] = Mfma<T>::op(a[j], bb[i], cur[i][j]);
            }
        };
        if (kb < NB || r0 + 32 > rows || c0 + 32 > cols) steps(std::true_type());
        else steps(std::false_type());
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = r0 + 16 * i + li, c = c0 + 16 * j + Mfma<T>::drow(v, lk);
                    if (r < rows && c < cols && (!lower || r + diag >= c)) C[(size_t)r + (size_t)c * ldc] = -cur[i][j][v];
                }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) cur[i][j] = nxt[i][j];
        b = bn;
    }
}

template <typename T>
__device__ inline void better(T &bv, int &bi, T ov, int oi) {
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
}

typedef unsigned long long u64;

// A wave's pivot candidate (key, row) as one 16-byte LDS slot.
struct __align__(16) Slot {
    u64 key;
    int idx, pad;
};

// LU of the panel [k0, k0 + kb) over rows [k0, n), m = n - k0 <= NT rows:
// thread t owns panel row t, its kb columns in registers (the column loop is
// unrolled at compile time).  One barrier per column: before it, every wave
// reduces its best candidate (largest |a|, lowest row on ties; NaN never
// wins; a DPP maximum of the keys and a ballot for the lowest lane holding
// it) and the candidate's owner writes the whole row to the wave's slot,
// and the owner of row j writes row j (slots by column parity); after it,
// every thread picks the winner among the slots and swaps, scales (division)
// and updates its own row.  pv[j] = 1 + pivot row relative to k0.
template <typename T, int NB>
__device__ __attribute__((always_inline)) int lu_panel_regs(int m, int kb, G<T> *A, int lda, int k0, int *pv, G<int> *ipiv, int first_zero, T *P) {
    constexpr int NW = NT / 64;
    __shared__ T cand[2][NW][NB];
    __shared__ T rowj[2][NB];
    __shared__ Slot ws[2][NW];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    // a wave past the panel's last row only keeps the barriers: its slots
    // say "no candidate" for the whole panel
    const bool wact = wave * 64 < m;
    if (!wact && lane == 0) ws[0][wave] = ws[1][wave] = Slot{0ull, INT_MAX, 0};
    T x[NB];
    cdf::static_for<0, NB>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        // every load issued (out-of-range ones read the panel's first entry
        // and are discarded): no load sits in a branch
        const bool ok = t < m && c < kb;
        const T v = A[ok ? (size_t)(k0 + t) + (size_t)(k0 + c) * lda : (size_t)k0 + (size_t)k0 * lda];
        x[c] = ok ? v : T(0);
    });
    cdf::static_for<0, NB>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (j >= kb) return;
        const int par = j & 1;
        if (wact) {
            // the wave's best row: largest key, then the lowest lane (= row)
            const u64 key = (t >= j && t < m) ? pivot_key(x[j]) : 0ull;
            const u64 wk = wave_max_key(key);
            const u64 hit = __ballot(key == wk && wk != 0ull);
            const int bi = hit ? (t & ~63) + __builtin_ctzll(hit) : INT_MAX;
            if (t == bi) cdf::static_for<0, NB>([&](auto cc) { cand[par][wave][decltype(cc)::value] = x[decltype(cc)::value]; });
            if (t == j) cdf::static_for<0, NB>([&](auto cc) { rowj[par][decltype(cc)::value] = x[decltype(cc)::value]; });
            if (lane == 0) ws[par][wave] = Slot{wk, bi, 0};
        }
        __syncthreads();
        if (!wact) return;
        // all slots read at once, then a branchless maximum; a later wave
        // holds higher rows, so strictly greater keeps the lowest row on ties
        Slot sl[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) sl[q] = ws[par][q];
        u64 v = sl[0].key;
        int p = sl[0].idx, w = 0;
#pragma unroll
        for (int q = 1; q < NW; ++q) {
            const bool gt = sl[q].key > v;
            v = gt ? sl[q].key : v;
            p = gt ? sl[q].idx : p;
            w = gt ? q : w;
        }
        const T *prow = p == INT_MAX ? rowj[par] : cand[par][w];
        if (p == INT_MAX) p = j;  // no ordered candidate (NaN column): no interchange
        const T piv = prow[j];
        if (t == 0) { pv[j] = p + 1; ipiv[k0 + j] = k0 + p + 1; }
        if (piv == T(0) && !first_zero) first_zero = k0 + j + 1;
        if (t == j) {
            cdf::static_for<0, NB>([&](auto cc) { x[decltype(cc)::value] = prow[decltype(cc)::value]; });
        } else if (t > j && t < m) {
            if (t == p) cdf::static_for<0, NB>([&](auto cc) { x[decltype(cc)::value] = rowj[par][decltype(cc)::value]; });
            if (piv != T(0)) {
                const T l = x[j] / piv;
                x[j] = l;
                cdf::static_for<j + 1, NB>([&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    x[c] = fma(-l, prow[c], x[c]);
                });
            }
        }
    });
    cdf::static_for<0, NB>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        if (t < m && c < kb) {
            A[(size_t)(k0 + t) + (size_t)(k0 + c) * lda] = x[c];
            P[(size_t)c * m + t] = x[c];
        }
    });
    return first_zero;
}

// The same panel for m > NT rows, in LDS (orders up to 1024).
template <typename T, int NB>
__device__ __attribute__((always_inline)) int lu_panel_lds(int m, int kb, G<T> *A, int lda, int k0, int *pv, G<int> *ipiv, int first_zero, T *P) {
    __shared__ T rv[NT / 64];
    __shared__ int ri[NT / 64];
    __shared__ int s_p;
    const int t = threadIdx.x;
    for (int e = t; e < m * kb; e += NT) P[e] = A[(size_t)(k0 + e % m) + (size_t)(k0 + e / m) * lda];
    __syncthreads();
    for (int j = 0; j < kb; ++j) {
        T bv = T(-1);
        int bi = INT_MAX;
        for (int r = j + t; r < m; r += NT) better(bv, bi, tabs(P[(size_t)j * m + r]), r);
        block_argmax<T>(bv, bi, rv, ri, &s_p);
        const int p = s_p == INT_MAX ? j : s_p;
        if (t == 0) { pv[j] = p + 1; ipiv[k0 + j] = k0 + p + 1; }
        if (p != j)
            for (int c = t; c < kb; c += NT) {
                const T tmp = P[(size_t)c * m + j];
                P[(size_t)c * m + j] = P[(size_t)c * m + p];
                P[(size_t)c * m + p] = tmp;
            }
        __syncthreads();
        const T piv = P[(size_t)j * m + j];
        if (piv == T(0)) {
            if (!first_zero) first_zero = k0 + j + 1;
            continue;
        }
        for (int r = j + 1 + t; r < m; r += NT) P[(size_t)j * m + r] /= piv;
        __syncthreads();
        for (int c = j + 1; c < kb; ++c)
            for (int r = j + 1 + t; r < m; r += NT)
                P[(size_t)c * m + r] = fma(-P[(size_t)j * m + r], P[(size_t)c * m + j], P[(size_t)c * m + r]);
        __syncthreads();
    }
    for (int e = t; e < m * kb; e += NT) A[(size_t)(k0 + e % m) + (size_t)(k0 + e / m) * lda] = P[e];
    return first_zero;
}

template <typename T, int NB>
__device__ __attribute__((always_inline)) void lu_one(int n, G<T> *A, int lda, G<int> *ipiv, G<int> *info, char *smem) {
    __shared__ int pv[NB];
    __shared__ int pdst[2 * NB], psrc[2 * NB];
    __shared__ int s_np;
    const int t = threadIdx.x;
    T *P = reinterpret_cast<T *>(smem);                      // panel, m x kb, ld m
    T *Uc = P + (size_t)n * NB;                              // U12 chunk, kb x UC, ld UC
    int first_zero = 0;
    for (int k0 = 0; k0 < n; k0 += NB) {
        const int kb = min(NB, n - k0), m = n - k0;
        first_zero = m <= NT ? lu_panel_regs<T, NB>(m, kb, A, lda, k0, pv, ipiv, first_zero, P)
                             : lu_panel_lds<T, NB>(m, kb, A, lda, k0, pv, ipiv, first_zero, P);
        __syncthreads();
        // the panel's interchanges on the other columns [0, k0) and [k0 + kb, n):
        // (dst, src) pairs by one wave, then every moved row read before any is written
        if (t < 64) {
            const int np = build_pairs_wave(pv, 0, kb, m, pdst, psrc, 0);
            if (t == 0) s_np = np;
        }
        __syncthreads();
        const int np = s_np, others = n - kb;
        for (int cb = 0; cb < others && np > 0; cb += 128) {
            const int cols = min(128, others - cb), total = np * cols;
            constexpr int PER = 2 * NB * 128 / NT + 1;
            T v[PER];
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                const int e = t + NT * r;
                if (e < total) {
                    const int q = cb + e / np, c = q < k0 ? q : q + kb;
                    v[r] = A[(size_t)(k0 + psrc[e % np]) + (size_t)c * lda];
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                const int e = t + NT * r;
                if (e < total) {
                    const int q = cb + e / np, c = q < k0 ? q : q + kb;
                    A[(size_t)(k0 + pdst[e % np]) + (size_t)c * lda] = v[r];
                }
            }
            __syncthreads();
        }
        const int rest = n - k0 - kb;
        if (rest <= 0) continue;  // the last panel (then kb may be < NB; otherwise kb == NB)
        // L11^-1 (unit lower) in LDS by rank-1 steps (no register arrays:
        // the kernel's registers are spoken for), in the U12 chunk's area:
        // Y = I, then for k = 0.., Y(i, j) -= L(i, k) Y(k, j) for i > k >= j
        // (row k of Y is final by step k).  Then written over L11 in the
        // panel's LDS copy (L21 below it is what the update reads):
        // Linv(i, j) = P[j * m + i].  Accepted if no entry exceeds 16 in
        // magnitude; otherwise U12 is solved by substitution with L11 from A.
        __shared__ int s_bad;
        T *Y = Uc;  // NB x NB, row-major
        for (int e = t; e < NB * NB; e += NT) Y[e] = (e / NB == e % NB) ? T(1) : T(0);
        if (t == 0) s_bad = 0;
        __syncthreads();
        for (int k = 0; k < NB - 1; ++k) {
            const int rows = NB - 1 - k, cols_k = k + 1;  // i in (k, NB), j in [0, k]
            for (int e = t; e < rows * cols_k; e += NT) {
                const int i = k + 1 + e / cols_k, j = e % cols_k;
                Y[i * NB + j] = fma(-P[(size_t)k * m + i], Y[k * NB + j], Y[i * NB + j]);
            }
            __syncthreads();
        }
        for (int e = t; e < NB * NB; e += NT) {
            const int i = e / NB, j = e % NB;
            const T v = Y[e];
            P[(size_t)j * m + i] = v;
            if (!(tabs(v) <= T(16))) s_bad = 1;
        }
        __syncthreads();
        const bool good = s_bad == 0;
        for (int cb = 0; cb < rest; cb += UC) {
            const int cols = min(UC, rest - cb);
            for (int e = t; e < NB * cols; e += NT) {
                const int i = e % NB, c = e / NB;
                Uc[(size_t)i * UC + c] = A[(size_t)(k0 + i) + (size_t)(k0 + kb + cb + c) * lda];
            }
            __syncthreads();
            // U12 chunk = L11^-1 A12 chunk in LDS: the product (every element
            // read before any is written), or substitution, one column per
            // thread
            if (good) {
                constexpr int PE = NB * UC / NT;
                T u[PE];
#pragma unroll
                for (int r = 0; r < PE; ++r) {
                    const int e = t + NT * r, c = e % UC, i = e / UC;
                    T acc = T(0);
                    if (c < cols)
                        for (int k = 0; k <= i; ++k) acc = fma(P[(size_t)k * m + i], Uc[(size_t)k * UC + c], acc);
                    u[r] = acc;
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < PE; ++r) {
                    const int e = t + NT * r, c = e % UC, i = e / UC;
                    if (c < cols) Uc[(size_t)i * UC + c] = u[r];
                }
            } else if (t < cols) {
                for (int i = 1; i < NB; ++i) {
                    T acc = Uc[(size_t)i * UC + t];
                    for (int k = 0; k < i; ++k)
                        acc = fma(-A[(size_t)(k0 + i) + (size_t)(k0 + k) * lda], Uc[(size_t)k * UC + t], acc);
                    Uc[(size_t)i * UC + t] = acc;
                }
            }
            __syncthreads();
            for (int e = t; e < NB * cols; e += NT) {
                const int i = e % NB, c = e / NB;
                A[(size_t)(k0 + i) + (size_t)(k0 + kb + cb + c) * lda] = Uc[(size_t)i * UC + c];
            }
            lds_update<T, NB>(A + (k0 + kb) + (size_t)(k0 + kb + cb) * lda, lda, rest, cols, kb, P + kb, m, Uc, UC, false,
                              0);
            __syncthreads();
        }
    }
    if (t == 0) *info = first_zero;
}

// Cholesky of the panel [k0, k0 + kb) over rows [k0, n), m <= NT: thread t
// owns panel row t (its columns c <= t in registers).  Two barriers per
// column: after the first every thread has the pivot a_jj (published by
// row j) and divides its own entry (the multiplier l_tj); the rows of the
// diagonal block publish theirs (by column parity), and after the second
// every row updates its entries with them.  Returns false at a pivot that
// is not > 0 (fail = its 1-based column).
template <typename T, int NB>
__device__ __attribute__((always_inline)) bool chol_panel_regs(int m, int kb, G<T> *A, int lda, int k0, int &fail, T *P) {
    __shared__ T djj[2];
    __shared__ T lcol[2][NB];
    const int t = threadIdx.x;
    T x[NB];
    cdf::static_for<0, NB>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        const bool ok = t < m && c < kb && c <= t;
        const T v = A[ok ? (size_t)(k0 + t) + (size_t)(k0 + c) * lda : (size_t)k0 + (size_t)k0 * lda];
        x[c] = ok ? v : T(0);
    });
    bool ok = true;
    // waves past the panel's last row only keep the barriers (rows j and
    // the diagonal block's rows lie in wave 0)
    const bool wact = (t >> 6) * 64 < m;
    cdf::static_for<0, NB>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (j >= kb || !ok) return;
        const int par = j & 1;
        if (t == j) djj[par] = x[j];
        __syncthreads();
        const T d = djj[par];
        if (!(d > T(0))) {  // uniform
            ok = false;
            fail = k0 + j + 1;
            return;
        }
        T l = T(0);
        if (wact) {
            const T ljj = sqrt(d);
            if (t == j) {
                x[j] = ljj;
            } else if (t > j && t < m) {
                l = x[j] / ljj;
                x[j] = l;
                if (t < kb) lcol[par][t] = l;  // the diagonal block's multipliers, for every row's update
            }
        }
        __syncthreads();
        if (wact && t > j && t < m)
            cdf::static_for<j + 1, NB>([&](auto cc) {
                constexpr int c = decltype(cc)::value;
                if (c < kb && c <= t) x[c] = fma(-l, lcol[par][c], x[c]);
            });
    });
    cdf::static_for<0, NB>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        if (t < m && c < kb && c <= t) {
            A[(size_t)(k0 + t) + (size_t)(k0 + c) * lda] = x[c];
            P[(size_t)c * m + t] = x[c];
        }
    });
    return ok;
}

// The same panel for m > NT rows, in LDS.
template <typename T, int NB>
__device__ __attribute__((always_inline)) bool chol_panel_lds(int m, int kb, G<T> *A, int lda, int k0, int &fail, T *P) {
    __shared__ int s_fail;
    const int t = threadIdx.x;
    if (t == 0) s_fail = 0;
    for (int e = t; e < m * kb; e += NT) {
        const int r = e % m, c = e / m;
        P[e] = r >= c ? A[(size_t)(k0 + r) + (size_t)(k0 + c) * lda] : T(0);
    }
    __syncthreads();
    for (int j = 0; j < kb; ++j) {
        if (t == 0) {
            const T d = P[(size_t)j * m + j];
            if (!(d > T(0))) s_fail = k0 + j + 1;
            else P[(size_t)j * m + j] = sqrt(d);
        }
        __syncthreads();
        if (s_fail) break;
        const T ljj = P[(size_t)j * m + j];
        for (int r = j + 1 + t; r < m; r += NT) P[(size_t)j * m + r] /= ljj;
        __syncthreads();
        for (int c = j + 1; c < kb; ++c)
            for (int r = c + t; r < m; r += NT)
                P[(size_t)c * m + r] = fma(-P[(size_t)j * m + r], P[(size_t)j * m + c], P[(size_t)c * m + r]);
        __syncthreads();
    }
    for (int e = t; e < m * kb; e += NT) {
        const int r = e % m, c = e / m;
        if (r >= c) A[(size_t)(k0 + r) + (size_t)(k0 + c) * lda] = P[e];
    }
    __syncthreads();
    if (s_fail) fail = s_fail;
    return s_fail == 0;
}

template <typename T, int NB>
__device__ __attribute__((always_inline)) void chol_one(int n, G<T> *A, int lda, G<int> *info, char *smem) {
    const int t = threadIdx.x;
    T *P = reinterpret_cast<T *>(smem);  // panel, m x kb, ld m (lower part used)
    int fail = 0;
    for (int k0 = 0; k0 < n; k0 += NB) {
        const int kb = min(NB, n - k0), m = n - k0;
        const bool ok = m <= NT ? chol_panel_regs<T, NB>(m, kb, A, lda, k0, fail, P)
                                : chol_panel_lds<T, NB>(m, kb, A, lda, k0, fail, P);
        __syncthreads();
        if (!ok) break;
        const int rest = n - k0 - kb;
        // lower(A22) -= L21 L21^T with L21 = rows [kb, m) of the panel
        if (rest > 0) lds_update<T, NB>(A + (k0 + kb) + (size_t)(k0 + kb) * lda, lda, rest, rest, kb, P + kb, m, P + kb, m,
                                    true, 0);
        __syncthreads();
    }
    if (t == 0) *info = fail;
}

template <typename T>
__global__ __launch_bounds__(NT) void vbatch_kernel(const VDesc *__restrict__ desc, int batch, int *counter,
                                                    int nb_pref) {
    extern __shared__ __align__(16) char smem[];
    __shared__ int s_idx;
    if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
    __syncthreads();
    int idx = s_idx;
    for (;;) {
        idx = __builtin_amdgcn_readfirstlane(idx);
        if (idx >= batch) break;
        // the next problem is claimed now: the atomic's round trip overlaps
        // with this one's factorization
        int next = 0;
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        const VDesc d = desc[idx];
        G<T> *A = (G<T> *)d.A;
        G<int> *info = (G<int> *)d.info;
        if (d.kind == 0) {
            G<int> *ipiv = (G<int> *)d.ipiv;
            if (panel_nb<T>(d.n, nb_pref) == 32) lu_one<T, 32>(d.n, A, d.lda, ipiv, info, smem);
            else lu_one<T, 16>(d.n, A, d.lda, ipiv, info, smem);
        } else {
            if (panel_nb<T>(d.n, nb_pref) == 32) chol_one<T, 32>(d.n, A, d.lda, info, smem);
            else chol_one<T, 16>(d.n, A, d.lda, info, smem);
        }
        __syncthreads();
        if (threadIdx.x == 0) s_idx = next;
        __syncthreads();
        idx = s_idx;
    }
}

// desc[i] = problem order[i] of the caller's arrays; thread 0 also clears
// the work counter.
__global__ void gather_desc_kernel(int batch, const int *__restrict__ order, const int *__restrict__ n,
                                   const int *__restrict__ kind, void *const *A, const int *lda, int *const *ipiv,
                                   int *info, VDesc *desc, int *counter) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *counter = 0;
    if (i >= batch) return;
    const int p = order[i];
    VDesc d;
    d.A = A[p];
    d.kind = kind[p];
    d.ipiv = d.kind == 0 ? ipiv[p] : nullptr;
    d.info = info + p;
    d.n = n[p];
    d.lda = lda[p];
    d.pad = 0;
    desc[i] = d;
}

}  // namespace

struct cdf_vbatch_plan_s {
    int device = 0;
    int batch = 0;
    cdf_dtype_t dt = CDF_F64;
    int grid = 0;
    int nb_pref = 0;
    size_t lds = 0;
    void *dev = nullptr;  // sizes, kinds, schedule, counter, descriptors
    int *n = nullptr, *kind = nullptr, *order = nullptr, *counter = nullptr;
    VDesc *desc = nullptr;
};

extern "C" {

cdf_status_t cdf_vbatch_plan_create(cdf_handle_t h, int batch, const int *n_host, const int *kind_host, cdf_dtype_t dt,
                                    cdf_vbatch_plan_t *plan) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->bad_arg = 0;
    auto bad = [&](int pos) { h->bad_arg = pos; return CDF_ERR_INVALID_ARG; };
    if (batch < 0) return bad(2);
    if (batch > 0 && !n_host) return bad(3);
    if (batch > 0 && !kind_host) return bad(4);
    if (dt != CDF_F64 && dt != CDF_F32) return bad(5);
    if (!plan) return bad(6);
    *plan = nullptr;
    for (int i = 0; i < batch; ++i) {
        if (n_host[i] < 1 || n_host[i] > 1024) return bad(3);
        if (kind_host[i] != 0 && kind_host[i] != 1) return bad(4);
    }
    cdf_vbatch_plan_s *p = new (std::nothrow) cdf_vbatch_plan_s();
    if (!p) return CDF_ERR_ALLOC;
    p->device = h->device;
    p->batch = batch;
    p->dt = dt;
    p->nb_pref = h->params[CDF_PARAM_VBATCH_NB];
    const int wpc = h->params[CDF_PARAM_VBATCH_WG_PER_CU] > 0 ? h->params[CDF_PARAM_VBATCH_WG_PER_CU] : 1;
    p->grid = std::max(1, std::min(batch, h->num_cus * wpc));
    // longest-processing-time order: estimated flops, largest first (stable)
    std::vector<int> order(batch);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const double ca = (double)n_host[a] * n_host[a] * n_host[a] * (kind_host[a] == 0 ? 2.0 : 1.0);
        const double cb = (double)n_host[b] * n_host[b] * n_host[b] * (kind_host[b] == 0 ? 2.0 : 1.0);
        return ca > cb;
    });
    const size_t nb4 = cdf::align_up((size_t)std::max(batch, 1) * sizeof(int), 256);
    const size_t bytes = 3 * nb4 + 256 + cdf::align_up((size_t)std::max(batch, 1) * sizeof(VDesc), 256);
    if (hipMalloc(&p->dev, bytes) != hipSuccess) { delete p; return CDF_ERR_ALLOC; }
    char *base = static_cast<char *>(p->dev);
    p->n = reinterpret_cast<int *>(base);
    p->kind = reinterpret_cast<int *>(base + nb4);
    p->order = reinterpret_cast<int *>(base + 2 * nb4);
    p->counter = reinterpret_cast<int *>(base + 3 * nb4);
    p->desc = reinterpret_cast<VDesc *>(base + 3 * nb4 + 256);
    bool ok = true;
    if (batch > 0) {
        ok = ok && hipMemcpy(p->n, n_host, batch * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(p->kind, kind_host, batch * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(p->order, order.data(), batch * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
    }
    const void *fn = dt == CDF_F64 ? reinterpret_cast<const void *>(&vbatch_kernel<double>)
                                   : reinterpret_cast<const void *>(&vbatch_kernel<float>);
    // LDS: the largest panel (n x nb) plus one U12 chunk (nb x UC)
    size_t lds = 1024;
    const size_t es = dt == CDF_F64 ? sizeof(double) : sizeof(float);
    for (int i = 0; i < batch; ++i) {
        const int nbp = dt == CDF_F64 ? panel_nb<double>(n_host[i], p->nb_pref) : panel_nb<float>(n_host[i], p->nb_pref);
        lds = std::max(lds, ((size_t)n_host[i] * nbp + (size_t)nbp * UC) * es);
    }
    p->lds = cdf::align_up(lds, 256);
    ok = ok && p->lds <= LDS_BYTES;
    ok = ok && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_BYTES) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        (void)hipFree(p->dev);
        delete p;
        return CDF_ERR_HIP;
    }
    *plan = p;
    return CDF_OK;
}

cdf_status_t cdf_vbatch_run(cdf_handle_t h, cdf_vbatch_plan_t plan, void *const *A_array, const int *lda_array,
                            int *const *ipiv_array, int *info_array) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->bad_arg = 0;
    auto bad = [&](int pos) { h->bad_arg = pos; return CDF_ERR_INVALID_ARG; };
    if (!plan) return bad(2);
    if (plan->batch == 0) return CDF_OK;
    if (!A_array) return bad(3);
    if (!lda_array) return bad(4);
    if (!ipiv_array) return bad(5);
    if (!info_array) return bad(6);
    if (plan->device != h->device) return bad(2);
    hipLaunchKernelGGL(gather_desc_kernel, dim3((plan->batch + 255) / 256), dim3(256), 0, h->stream, plan->batch,
                       plan->order, plan->n, plan->kind, A_array, lda_array, ipiv_array, info_array, plan->desc,
                       plan->counter);
    CDF_HIP_TRY(hipGetLastError());
    if (plan->dt == CDF_F64)
        hipLaunchKernelGGL((vbatch_kernel<double>), dim3(plan->grid), dim3(NT), plan->lds, h->stream, plan->desc,
                           plan->batch, plan->counter, plan->nb_pref);
    else
        hipLaunchKernelGGL((vbatch_kernel<float>), dim3(plan->grid), dim3(NT), plan->lds, h->stream, plan->desc,
                           plan->batch, plan->counter, plan->nb_pref);
    CDF_HIP_TRY(hipGetLastError());
    return CDF_OK;
}

cdf_status_t cdf_vbatch_plan_destroy(cdf_vbatch_plan_t plan) {
    if (!plan) return CDF_ERR_INVALID_ARG;
    (void)hipDeviceSynchronize();
    if (plan->dev) (void)hipFree(plan->dev);
    delete plan;
    return CDF_OK;
}

}  // extern "C"
