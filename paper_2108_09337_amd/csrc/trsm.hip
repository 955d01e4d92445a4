// Triangular solves (Sec. 7, routines A10 / A01: local trsm; Table 1) and
// the blocked solves used by the factor-solve calls.
//
// Small solves keep a strip of the right-hand block in LDS and walk the
// triangle one row/column at a time; the triangle's column (or row) for
// each step is read from L2 (the triangle is at most 256 x 256).
//   left kinds : B (nb x ncols), 16 columns per workgroup, 16 row groups
//   right kind : B (nrows x nb), 64 rows per workgroup, one per lane, the
//                later columns of each block split over 4 waves
#include "internal.h"

namespace {

constexpr int NT = 256;
constexpr int LNC = 16;          // columns per workgroup (left solves): 8.7 KB of LDS at
                                 // nb = 64, so a solve fits beside the update GEMMs
constexpr int LRG = NT / LNC;    // row groups
constexpr int LPAD = LNC + 1;
constexpr int RNR = 64;          // rows per workgroup (right solve)
constexpr int MAXNB = 256;       // right solves (LDS: row block + staged panel)
constexpr int MAXNB_LEFT = 512;  // left solves (LDS: nb x LPAD doubles)

template <int KIND, typename TB>
__global__ __launch_bounds__(NT) void trsm_left_kernel(int nb, int ncols, const double *__restrict__ T,
                                                       int ldt, TB *__restrict__ B, int ldb,
                                                       const int *stop) {
    if (stop != nullptr && *stop != 0) return;
    extern __shared__ double X[];  // X[r * LPAD + c]
    const int t = threadIdx.x;
    const int c = t % LNC, rg = t / LNC;
    // column blocks in a grid-stride loop (the grid may be capped)
    for (int c0 = blockIdx.x * LNC; c0 < ncols; c0 += gridDim.x * LNC) {
        if (c0 != blockIdx.x * LNC) __syncthreads();  // the previous block's results are stored
        for (int e = t; e < nb * LNC; e += NT) {
            const int r = e % nb, cc = e / nb;
            X[r * LPAD + cc] = (c0 + cc < ncols) ? (double)B[(size_t)r + (size_t)(c0 + cc) * ldb] : 0.0;
        }
        __syncthreads();
        constexpr bool forward = (KIND == cdf::TRSM_LLNU || KIND == cdf::TRSM_LLNN);
        constexpr bool unit = (KIND == cdf::TRSM_LLNU);
        if (forward && nb <= 4 * LRG) {
            // Forward solve with at most four rows per thread: the triangle's
            // entries of step j + 1 are loaded during step j, and the step
            // barrier waits for LDS only (not for those loads), so no step
            // waits on a global load.  Same updates in the same order as the
            // general loop below.
            double ta[4], tb[4], da = 0.0, db = 0.0;
            auto load = [&](int j, double (&t)[4], double &d) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = rg + LRG * q;
                    t[q] = i < nb ? T[(size_t)i + (size_t)j * ldt] : 0.0;
                }
                if (!unit) d = T[(size_t)j + (size_t)j * ldt];
            };
            auto lds_barrier = [] {
                asm volatile("" ::: "memory");
                __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vector loads may stay in flight
                __builtin_amdgcn_s_barrier();
                asm volatile("" ::: "memory");
            };
            auto step = [&](int j, const double (&t)[4], double d) {
                if (!unit) {
                    if (rg == j % LRG) X[j * LPAD + c] = X[j * LPAD + c] / d;
                    lds_barrier();
                }
                const double xj = X[j * LPAD + c];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = rg + LRG * q;
                    if (i > j && i < nb) X[i * LPAD + c] = fma(-t[q], xj, X[i * LPAD + c]);
                }
                lds_barrier();
            };
            load(0, ta, da);
            for (int j = 0; j < nb; j += 2) {
                if (j + 1 < nb) load(j + 1, tb, db);
                step(j, ta, da);
                if (j + 1 >= nb) break;
                if (j + 2 < nb) load(j + 2, ta, da);
                step(j + 1, tb, db);
            }
        } else
        for (int s = 0; s < nb; ++s) {
            const int j = forward ? s : nb - 1 - s;
            if (!unit) {
                if (rg == j % LRG) X[j * LPAD + c] = X[j * LPAD + c] / T[(size_t)j + (size_t)j * ldt];
                __syncthreads();
            }
            const double xj = X[j * LPAD + c];
            if (forward) {
                for (int i = j + 1 + ((rg - (j + 1)) & (LRG - 1)); i < nb; i += LRG)
                    X[i * LPAD + c] = fma(-T[(size_t)i + (size_t)j * ldt], xj, X[i * LPAD + c]);
            } else if (KIND == cdf::TRSM_LUNN) {
                for (int i = rg; i < j; i += LRG)
                    X[i * LPAD + c] = fma(-T[(size_t)i + (size_t)j * ldt], xj, X[i * LPAD + c]);
            } else {  // TRSM_LLTN: (L^T)(i, j) = L(j, i)
                for (int i = rg; i < j; i += LRG)
                    X[i * LPAD + c] = fma(-T[(size_t)j + (size_t)i * ldt], xj, X[i * LPAD + c]);
            }
            __syncthreads();
        }
        for (int e = t; e < nb * LNC; e += NT) {
            const int r = e % nb, cc = e / nb;
            if (c0 + cc < ncols) B[(size_t)r + (size_t)(c0 + cc) * ldb] = (TB)X[r * LPAD + cc];
        }
    }
}

// B (nrows x nb) <- B L^-T with L lower, non-unit.  Rows are independent
// (row r solves L x_r^T = b_r^T by forward substitution).  A workgroup takes
// 64 rows (lane l of every wave owns row l) and keeps them in LDS
// (X[c * RNR + l]).  For each block of 16 columns: the triangle's columns
// J..J+15 (rows J..nb) are staged in LDS; every wave solves the block for
// its lanes' rows in registers (x_j = x_j / L(j,j), x_i -= x_j L(i,j)), the
// same values in all waves; then wave w applies the block to the later
// columns c = w (mod 4), accumulating -x_j L(c,j) over the block's j in
// order -- the operations and order of column-by-column right-looking
// substitution.
template <typename TB>
__global__ __launch_bounds__(NT) void trsm_rltn_kernel(int nb, int nrows, const double *__restrict__ T,
                                                       int ldt, TB *__restrict__ B, int ldb,
                                                       const int *stop) {
    if (stop != nullptr && *stop != 0) return;
    constexpr int CB = 16;
    constexpr int NW = NT / 64;
    extern __shared__ double X[];         // X[c * RNR + lane]
    double *P = X + (size_t)nb * RNR;     // P[jj * nb + (c - J)] = T(c, J + jj)
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int r = blockIdx.x * RNR + lane;
    const bool live = r < nrows;
    for (int c0 = wave * 8; c0 < nb; c0 += 8 * NW) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (live && c0 + q < nb) ? (double)B[(size_t)r + (size_t)(c0 + q) * ldb] : 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (c0 + q < nb) X[(c0 + q) * RNR + lane] = v[q];
    }
    for (int J = 0; J < nb; J += CB) {
        const int jb = nb - J < CB ? nb - J : CB;
        for (int e = t; e < jb * (nb - J); e += NT) {
            const int jj = e / (nb - J), c = J + e % (nb - J);
            P[jj * nb + (c - J)] = T[(size_t)c + (size_t)(J + jj) * ldt];
        }
        __syncthreads();  // panel staged; X of this block final
        double x[CB];
#pragma unroll
        for (int jj = 0; jj < CB; ++jj) x[jj] = jj < jb ? X[(J + jj) * RNR + lane] : 0.0;
#pragma unroll
        for (int jj = 0; jj < CB; ++jj) {
            if (jj < jb) {
                x[jj] = x[jj] / P[jj * nb + jj];
#pragma unroll
                for (int ii = jj + 1; ii < CB; ++ii)
                    if (ii < jb) x[ii] = fma(-x[jj], P[jj * nb + ii], x[ii]);
            }
        }
        __syncthreads();  // every wave has read the block before it is overwritten
        if (wave == 0) {
#pragma unroll
            for (int jj = 0; jj < CB; ++jj)
                if (jj < jb) X[(J + jj) * RNR + lane] = x[jj];
        }
        for (int c = J + jb + wave; c < nb; c += NW) {
            double acc = X[c * RNR + lane];
#pragma unroll
            for (int jj = 0; jj < CB; ++jj)
                if (jj < jb) acc = fma(-x[jj], P[jj * nb + (c - J)], acc);
            X[c * RNR + lane] = acc;
        }
        __syncthreads();  // later columns updated; P may be restaged
    }
    if (live)
        for (int c = wave; c < nb; c += NW) B[(size_t)r + (size_t)c * ldb] = (TB)X[c * RNR + lane];
}

// The same solve for triangles of at most 64 columns with no LDS at all:
// lane = row, the row in registers (compile-time column loop), the
// triangle's entries as wave-uniform (scalar) loads.  Same operations in the
// same order as above.  Fits on a CU beside the update GEMM's workgroups,
// which take all of its LDS.
constexpr int RNC = 64;
// FULL: nb == 64, so no entry is guarded and the compiler batches (and
// merges) the triangle's scalar loads instead of waiting on each one.
// PRIO: raised issue priority (a separate instantiation, so the other one
// keeps its register allocation).
template <typename TB, bool FULL, bool PRIO = false>
__global__ __launch_bounds__(64) void trsm_rltn_reg_kernel(int nb_in, int nrows, const double *__restrict__ T, int ldt,
                                                           TB *__restrict__ B, int ldb, const int *stop) {
    if (stop != nullptr && *stop != 0) return;
    if (PRIO) __builtin_amdgcn_s_setprio(2);
    const int nb = FULL ? RNC : nb_in;
    const int r = blockIdx.x * 64 + threadIdx.x;
    const bool live = r < nrows;
    double x[RNC];
    cdf::static_for<0, RNC>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        x[c] = (live && c < nb) ? (double)B[(size_t)r + (size_t)c * ldb] : 0.0;
    });
    cdf::static_for<0, RNC>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (FULL || j < nb) {
            x[j] = x[j] / T[(size_t)j + (size_t)j * ldt];
            cdf::static_for<j + 1, RNC>([&](auto cc) {
                constexpr int c = decltype(cc)::value;
                if (FULL || c < nb) x[c] = fma(-x[j], T[(size_t)c + (size_t)j * ldt], x[c]);
            });
        }
    });
    if (live)
        cdf::static_for<0, RNC>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            if (c < nb) B[(size_t)r + (size_t)c * ldb] = (TB)x[c];
        });
}

template <int KIND, typename TB>
hipError_t launch_left(hipStream_t s, int nb, int ncols, const double *T, int ldt, TB *B, int ldb,
                       const int *stop, int max_wg) {
    static bool attr = false;
    const size_t lds = (size_t)nb * LPAD * sizeof(double);
    if (!attr) {
        CDF_HIP_RET(hipFuncSetAttribute(reinterpret_cast<const void *>(&trsm_left_kernel<KIND, TB>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        MAXNB_LEFT * LPAD * sizeof(double)));
        attr = true;
    }
    int grid = (ncols + LNC - 1) / LNC;
    if (max_wg > 0 && grid > max_wg) grid = max_wg;
    hipLaunchKernelGGL((trsm_left_kernel<KIND, TB>), dim3(grid), dim3(NT), lds, s, nb, ncols, T, ldt, B, ldb, stop);
    return hipGetLastError();
}

template <typename TB>
hipError_t launch_right(hipStream_t s, int nb, int nrows, const double *T, int ldt, TB *B, int ldb,
                        const int *stop, bool prio = false) {
    const dim3 grid((nrows + 63) / 64);
    if (nb == RNC) {
        if (prio)
            hipLaunchKernelGGL((trsm_rltn_reg_kernel<TB, true, true>), grid, dim3(64), 0, s, nb, nrows, T, ldt, B, ldb,
                               stop);
        else
            hipLaunchKernelGGL((trsm_rltn_reg_kernel<TB, true>), grid, dim3(64), 0, s, nb, nrows, T, ldt, B, ldb, stop);
        return hipGetLastError();
    }
    if (nb < RNC) {
        if (prio)
            hipLaunchKernelGGL((trsm_rltn_reg_kernel<TB, false, true>), grid, dim3(64), 0, s, nb, nrows, T, ldt, B,
                               ldb, stop);
        else
            hipLaunchKernelGGL((trsm_rltn_reg_kernel<TB, false>), grid, dim3(64), 0, s, nb, nrows, T, ldt, B, ldb,
                               stop);
        return hipGetLastError();
    }
    static bool attr = false;
    const size_t lds = (size_t)nb * (RNR + 16) * sizeof(double);  // row block + staged triangle panel
    if (!attr) {
        CDF_HIP_RET(hipFuncSetAttribute(reinterpret_cast<const void *>(&trsm_rltn_kernel<TB>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        MAXNB * (RNR + 16) * sizeof(double)));
        attr = true;
    }
    hipLaunchKernelGGL((trsm_rltn_kernel<TB>), dim3((nrows + RNR - 1) / RNR), dim3(NT), lds, s, nb, nrows, T, ldt,
                       B, ldb, stop);
    return hipGetLastError();
}

// Few right-hand sides: one wave per column; lane i holds row i of the
// 64-row diagonal block, the block of T sits in LDS; the solved value of row
// j is broadcast with a shuffle.
template <int KIND>
__global__ __launch_bounds__(256) void trsv_diag_kernel(int kb, int nrhs, const double *__restrict__ T, int ldt,
                                                        double *__restrict__ B, int ldb) {
    __shared__ double Ts[64 * 65];
    const int t = threadIdx.x, lane = t & 63, c = t >> 6;
    for (int e = t; e < kb * kb; e += 256) {
        const int i = e % kb, j = e / kb;
        Ts[i + j * 65] = T[(size_t)i + (size_t)j * ldt];
    }
    __syncthreads();
    if (c >= nrhs) return;
    double x = lane < kb ? B[(size_t)lane + (size_t)c * ldb] : 0.0;
    if (KIND == cdf::TRSM_LLNU || KIND == cdf::TRSM_LLNN) {
        for (int j = 0; j < kb; ++j) {
            if (KIND == cdf::TRSM_LLNN && lane == j) x = x / Ts[j + j * 65];
            const double xj = __shfl(x, j);
            if (lane > j && lane < kb) x = fma(-Ts[lane + j * 65], xj, x);
        }
    } else {
        for (int j = kb - 1; j >= 0; --j) {
            if (lane == j) x = x / Ts[j + j * 65];
            const double xj = __shfl(x, j);
            if (lane < j) x = fma(KIND == cdf::TRSM_LUNN ? -Ts[lane + j * 65] : -Ts[j + lane * 65], xj, x);
        }
    }
    if (lane < kb) B[(size_t)lane + (size_t)c * ldb] = x;
}

// One step of a blocked triangular solve with few right-hand sides (<= 4):
// the block x[k, k+kb) is final.  Every workgroup subtracts its
// contribution from 64 of the remaining rows [rbeg, rend) -- forward: chunk
// b is rows rbeg + 64b.., backward: rows rend - 64(b+1).. -- with the block's
// columns split over the 4 waves and the partial sums added in wave order;
// then workgroup 0, whose rows are exactly the next diagonal block
// [nk, nk + nkb), solves that block (one wave per right-hand side, lane =
// row), so a step costs one launch.
template <int KIND>
__global__ __launch_bounds__(256) void trsv_step_kernel(int nrhs, const double *__restrict__ T, int ldt,
                                                        double *__restrict__ B, int ldb, int k, int kb, int rbeg,
                                                        int rend, int nk, int nkb) {
    constexpr bool forward = (KIND == cdf::TRSM_LLNU || KIND == cdf::TRSM_LLNN);
    __shared__ double xs[4][64];
    __shared__ double red[4][4][64];
    __shared__ double ynew[4][64];
    __shared__ double Ts[64 * 65];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (t < kb * nrhs) xs[t / kb][t % kb] = B[(size_t)(k + t % kb) + (size_t)(t / kb) * ldb];
    const bool diag = blockIdx.x == 0 && nkb > 0;
    if (diag)
        for (int e = t; e < nkb * nkb; e += 256) {
            const int i = e % nkb, j = e / nkb;
            Ts[i + j * 65] = T[(size_t)(nk + i) + (size_t)(nk + j) * ldt];
        }
    __syncthreads();
    const int r0 = forward ? rbeg + 64 * (int)blockIdx.x : rend - 64 * ((int)blockIdx.x + 1);
    if (KIND != cdf::TRSM_LLTN) {
        // lanes = rows: T(r, k + jj) is contiguous over the lanes
        const int r = r0 + lane;
        const bool live = r >= rbeg && r < rend;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        const int j0 = 16 * wave, j1 = min(j0 + 16, kb);
        for (int jj = j0; jj < j1; ++jj) {
            const double tv = live ? T[(size_t)r + (size_t)(k + jj) * ldt] : 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < nrhs) acc[c] = fma(tv, xs[c][jj], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) red[wave][c][lane] = acc[c];
    } else {
        // (L^T)(r, k + j) = L(k + j, r): lanes = j (contiguous), wave w takes rows r0 + 16w .. + 16
        for (int rr = 0; rr < 16; ++rr) {
            const int r = r0 + 16 * wave + rr;
            const bool live = r >= rbeg && r < rend && lane < kb;
            const double lv = live ? T[(size_t)(k + lane) + (size_t)r * ldt] : 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double p = c < nrhs ? lv * xs[c][lane < kb ? lane : 0] : 0.0;
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) p += __shfl_xor(p, off);
                if (lane == 0) red[0][c][16 * wave + rr] = p;
            }
        }
    }
    __syncthreads();
    if (wave == 0) {
        const int r = r0 + lane;
        const bool live = r >= rbeg && r < rend;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (c >= nrhs) continue;
            const double sum = KIND == cdf::TRSM_LLTN
                                   ? red[0][c][lane]
                                   : ((red[0][c][lane] + red[1][c][lane]) + red[2][c][lane]) + red[3][c][lane];
            double y = live ? B[(size_t)r + (size_t)c * ldb] - sum : 0.0;
            ynew[c][lane] = y;
            if (live && !diag) B[(size_t)r + (size_t)c * ldb] = y;
        }
    }
    if (!diag) return;
    __syncthreads();
    // next diagonal block: rows [nk, nk + nkb) are this workgroup's rows
    if (wave >= nrhs) return;
    const int c = wave;
    const int off = nk - r0;  // 0 forward; 64 - nkb never occurs (backward blocks are full)
    double x = lane < nkb ? ynew[c][lane + off] : 0.0;
    if (forward) {
        for (int j = 0; j < nkb; ++j) {
            if (KIND == cdf::TRSM_LLNN && lane == j) x = x / Ts[j + j * 65];
            const double xj = __shfl(x, j);
            if (lane > j && lane < nkb) x = fma(-Ts[lane + j * 65], xj, x);
        }
    } else {
        for (int j = nkb - 1; j >= 0; --j) {
            if (lane == j) x = x / Ts[j + j * 65];
            const double xj = __shfl(x, j);
            if (lane < j) x = fma(KIND == cdf::TRSM_LUNN ? -Ts[lane + j * 65] : -Ts[j + lane * 65], xj, x);
        }
    }
    if (lane < nkb) B[(size_t)(nk + lane) + (size_t)c * ldb] = x;
}

// Single-launch solve for few right-hand sides (kinds with the triangle's
// rows contiguous over the lanes: LLNU, LLNN, LUNN).  A workgroup takes the
// next row block in start order (an atomic ticket, so every block it waits
// for belongs to a workgroup that started earlier), accumulates T(rb, jb) x_jb
// over the blocks solved before it as their flags appear (wave w takes every
// fourth block; lanes = rows), then solves its diagonal block (one wave per
// right-hand side) and publishes x_rb: device-coherent stores, completed,
// then the block's flag.  sync[0] is the ticket, sync[1 + b] block b's flag;
// all start at zero.
__device__ inline double ld_coh(const double *p) {
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_coh(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int KIND>
__global__ __launch_bounds__(256) void trsv_sf_kernel(int n, int nrhs, const double *__restrict__ T, int ldt,
                                                      double *B, int ldb, int *sync) {
    constexpr bool forward = (KIND == cdf::TRSM_LLNU || KIND == cdf::TRSM_LLNN);
    __shared__ int s_q;
    __shared__ double xs[4][4][64];
    __shared__ double red[4][4][64];
    __shared__ double Ts[64 * 65];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nblk = (n + 63) / 64;
    if (t == 0) s_q = atomicAdd(sync, 1);
    __syncthreads();
    const int q = s_q;
    const int rb = forward ? q : nblk - 1 - q;
    const int r0 = rb * 64, kb = min(64, n - r0);
    for (int e = t; e < kb * kb; e += 256) {
        const int i = e % kb, j = e / kb;
        Ts[i + j * 65] = T[(size_t)(r0 + i) + (size_t)(r0 + j) * ldt];
    }
    const int r = r0 + lane;
    const bool live = lane < kb;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int nj = forward ? rb : nblk - 1 - rb;  // blocks solved before this one
    for (int sj = wave; sj < nj; sj += 4) {
        const int jb = forward ? sj : nblk - 1 - sj;
        const int c0 = jb * 64, jn = min(64, n - c0);
        // the block of T does not depend on x: all 64 loads are issued
        // before waiting for x_jb, so one memory latency covers the block
        double tv[64];
#pragma unroll
        for (int u = 0; u < 64; ++u) tv[u] = (live && u < jn) ? T[(size_t)r + (size_t)(c0 + u) * ldt] : 0.0;
        if (lane == 0)
            while (__hip_atomic_load(sync + 1 + jb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
                __builtin_amdgcn_s_sleep(2);
        asm volatile("" ::: "memory");  // x_jb is read only after its flag was seen
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c < nrhs) xs[wave][c][lane] = lane < jn ? ld_coh(B + (size_t)(c0 + lane) + (size_t)c * ldb) : 0.0;
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_waitcnt(0xC07F);  // this wave's LDS writes done (lgkmcnt 0)
        asm volatile("" ::: "memory");
#pragma unroll
        for (int u = 0; u < 64; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < nrhs && u < jn) acc[c] = fma(tv[u], xs[wave][c][u], acc[c]);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_waitcnt(0xC07F);  // reads of xs done before the next block overwrites it
        asm volatile("" ::: "memory");
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) red[wave][c][lane] = acc[c];
    __syncthreads();
    if (wave < nrhs) {
        const int c = wave;
        const double sum = ((red[0][c][lane] + red[1][c][lane]) + red[2][c][lane]) + red[3][c][lane];
        double x = live ? B[(size_t)r + (size_t)c * ldb] - sum : 0.0;
        // x_j from lane j by readlane (a register read, where a shuffle is
        // an LDS round trip on each of the 64 dependent steps)
        auto from_lane = [](double v, int l) {
            const long long b = __double_as_longlong(v);
            const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, l);
            const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
            return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
        };
        if (forward) {
            for (int j = 0; j < kb; ++j) {
                if (KIND == cdf::TRSM_LLNN && lane == j) x = x / Ts[j + j * 65];
                const double xj = from_lane(x, j);
                if (lane > j && lane < kb) x = fma(-Ts[lane + j * 65], xj, x);
            }
        } else {
            for (int j = kb - 1; j >= 0; --j) {
                if (lane == j) x = x / Ts[j + j * 65];
                const double xj = from_lane(x, j);
                if (lane < j) x = fma(-Ts[lane + j * 65], xj, x);
            }
        }
        if (live) st_coh(B + (size_t)r + (size_t)c * ldb, x);
        __builtin_amdgcn_s_waitcnt(0);  // the stores have completed
    }
    __syncthreads();
    if (t == 0) __hip_atomic_store(sync + 1 + rb, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int KIND>
hipError_t launch_step(hipStream_t s, int nrhs, const double *T, int ldt, double *B, int ldb, int k, int kb, int rbeg,
                       int rend, int nk, int nkb) {
    const int rows = rend - rbeg;
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL((trsv_step_kernel<KIND>), dim3((rows + 63) / 64), dim3(256), 0, s, nrhs, T, ldt, B, ldb, k, kb,
                       rbeg, rend, nk, nkb);
    return hipGetLastError();
}

template <int KIND>
hipError_t launch_diag(hipStream_t s, int kb, int nrhs, const double *T, int ldt, double *B, int ldb) {
    hipLaunchKernelGGL((trsv_diag_kernel<KIND>), dim3(1), dim3(256), 0, s, kb, nrhs, T, ldt, B, ldb);
    return hipGetLastError();
}

}  // namespace

namespace cdf {

size_t trsv_sync_ints(int n) { return (size_t)(n + 63) / 64 + 1; }

hipError_t trsv_blocked(hipStream_t s, TrsmKind kind, int n, int ncols, const double *T, int ldt, double *B,
                        int ldb, int *sync) {
    constexpr int BS = 64;
    if (n <= 0 || ncols <= 0) return hipSuccess;
    if (ncols > 4) return hipErrorInvalidValue;
    if (sync != nullptr && kind != TRSM_LLTN) {
        const int nblk = (n + 63) / 64;
        CDF_HIP_RET(fill_int(s, sync, nblk + 1, 0));
        switch (kind) {
            case TRSM_LLNU:
                hipLaunchKernelGGL((trsv_sf_kernel<TRSM_LLNU>), dim3(nblk), dim3(256), 0, s, n, ncols, T, ldt, B, ldb,
                                   sync);
                break;
            case TRSM_LLNN:
                hipLaunchKernelGGL((trsv_sf_kernel<TRSM_LLNN>), dim3(nblk), dim3(256), 0, s, n, ncols, T, ldt, B, ldb,
                                   sync);
                break;
            default:
                hipLaunchKernelGGL((trsv_sf_kernel<TRSM_LUNN>), dim3(nblk), dim3(256), 0, s, n, ncols, T, ldt, B, ldb,
                                   sync);
                break;
        }
        return hipGetLastError();
    }
    auto diag = [&](int k, int kb) -> hipError_t {
        const double *Tk = T + k + (size_t)k * ldt;
        switch (kind) {
            case TRSM_LLNU: return launch_diag<TRSM_LLNU>(s, kb, ncols, Tk, ldt, B + k, ldb);
            case TRSM_LLNN: return launch_diag<TRSM_LLNN>(s, kb, ncols, Tk, ldt, B + k, ldb);
            case TRSM_LUNN: return launch_diag<TRSM_LUNN>(s, kb, ncols, Tk, ldt, B + k, ldb);
            case TRSM_LLTN: return launch_diag<TRSM_LLTN>(s, kb, ncols, Tk, ldt, B + k, ldb);
            default: return hipErrorInvalidValue;
        }
    };
    auto step = [&](int k, int kb, int rbeg, int rend, int nk, int nkb) -> hipError_t {
        switch (kind) {
            case TRSM_LLNU: return launch_step<TRSM_LLNU>(s, ncols, T, ldt, B, ldb, k, kb, rbeg, rend, nk, nkb);
            case TRSM_LLNN: return launch_step<TRSM_LLNN>(s, ncols, T, ldt, B, ldb, k, kb, rbeg, rend, nk, nkb);
            case TRSM_LUNN: return launch_step<TRSM_LUNN>(s, ncols, T, ldt, B, ldb, k, kb, rbeg, rend, nk, nkb);
            case TRSM_LLTN: return launch_step<TRSM_LLTN>(s, ncols, T, ldt, B, ldb, k, kb, rbeg, rend, nk, nkb);
            default: return hipErrorInvalidValue;
        }
    };
    if (kind == TRSM_LLNU || kind == TRSM_LLNN) {
        CDF_HIP_RET(diag(0, min(BS, n)));
        for (int k = 0; k < n; k += BS) {
            const int kb = min(BS, n - k), nk = k + kb;
            if (nk >= n) break;
            CDF_HIP_RET(step(k, kb, nk, n, nk, min(BS, n - nk)));
        }
        return hipSuccess;
    }
    const int last = ((n - 1) / BS) * BS;
    CDF_HIP_RET(diag(last, n - last));
    for (int k = last; k > 0; k -= BS) CDF_HIP_RET(step(k, min(BS, n - k), 0, k, k - BS, BS));
    return hipSuccess;
}

template <typename TB>
hipError_t trsm_small_impl(hipStream_t s, TrsmKind kind, int nb, int ncols, const double *T, int ldt, TB *B,
                           int ldb, const int *stop, int max_wg) {
    if (nb <= 0 || ncols <= 0) return hipSuccess;
    if (nb > (kind == TRSM_RLTN ? MAXNB : MAXNB_LEFT)) return hipErrorInvalidValue;
    switch (kind) {
        case TRSM_LLNU: return launch_left<TRSM_LLNU, TB>(s, nb, ncols, T, ldt, B, ldb, stop, max_wg);
        case TRSM_LLNN: return launch_left<TRSM_LLNN, TB>(s, nb, ncols, T, ldt, B, ldb, stop, max_wg);
        case TRSM_LLTN: return launch_left<TRSM_LLTN, TB>(s, nb, ncols, T, ldt, B, ldb, stop, max_wg);
        case TRSM_LUNN: return launch_left<TRSM_LUNN, TB>(s, nb, ncols, T, ldt, B, ldb, stop, max_wg);
        case TRSM_RLTN: return launch_right<TB>(s, nb, ncols, T, ldt, B, ldb, stop);
    }
    return hipErrorInvalidValue;
}

hipError_t trsm_small(hipStream_t s, TrsmKind kind, int nb, int ncols, const double *T, int ldt,
                      double *B, int ldb, const int *stop, int max_wg) {
    return trsm_small_impl<double>(s, kind, nb, ncols, T, ldt, B, ldb, stop, max_wg);
}

hipError_t trsm_small(hipStream_t s, TrsmKind kind, int nb, int ncols, const double *T, int ldt,
                      float *B, int ldb, const int *stop, int max_wg) {
    return trsm_small_impl<float>(s, kind, nb, ncols, T, ldt, B, ldb, stop, max_wg);
}

hipError_t trsm_rltn_small(hipStream_t s, int nb, int nrows, const double *T, int ldt, double *B, int ldb,
                           const int *stop, bool prio) {
    if (nb <= 0 || nrows <= 0) return hipSuccess;
    if (nb > RNC) return hipErrorInvalidValue;
    return launch_right<double>(s, nb, nrows, T, ldt, B, ldb, stop, prio);
}

// Blocked solve with an n x n triangle: 128-wide diagonal solves, the rest
// of the right-hand block updated with the FP64 GEMM.
hipError_t trsm_blocked(hipStream_t s, TrsmKind kind, int n, int ncols, const double *T, int ldt,
                        double *B, int ldb, int BS, const GemmCtx *ctx) {
    if (BS <= 0 || BS > MAXNB) return hipErrorInvalidValue;
    if (n <= 0 || ncols <= 0) return hipSuccess;
    if (kind == TRSM_LLNU || kind == TRSM_LLNN) {
        for (int k = 0; k < n; k += BS) {
            const int kb = min(BS, n - k);
            CDF_HIP_RET(trsm_small(s, kind, kb, ncols, T + k + (size_t)k * ldt, ldt, B + k, ldb));
            if (k + kb < n)
                CDF_HIP_RET(dgemm(s, 0, 0, n - k - kb, ncols, kb, -1.0, T + (k + kb) + (size_t)k * ldt, ldt,
                                  B + k, ldb, 1.0, B + k + kb, ldb, false, nullptr, ctx));
        }
        return hipSuccess;
    }
    if (kind == TRSM_LUNN || kind == TRSM_LLTN) {
        const int last = ((n - 1) / BS) * BS;
        for (int k = last; k >= 0; k -= BS) {
            const int kb = min(BS, n - k);
            CDF_HIP_RET(trsm_small(s, kind, kb, ncols, T + k + (size_t)k * ldt, ldt, B + k, ldb));
            if (k > 0) {
                if (kind == TRSM_LUNN)
                    CDF_HIP_RET(dgemm(s, 0, 0, k, ncols, kb, -1.0, T + (size_t)k * ldt, ldt, B + k, ldb, 1.0, B,
                                      ldb, false, nullptr, ctx));
                else  // rows [0,k) -= L(k:k+kb, 0:k)^T X(k:k+kb)
                    CDF_HIP_RET(dgemm(s, 1, 0, k, ncols, kb, -1.0, T + k, ldt, B + k, ldb, 1.0, B, ldb, false,
                                      nullptr, ctx));
            }
        }
        return hipSuccess;
    }
    return hipErrorInvalidValue;
}

}  // namespace cdf
