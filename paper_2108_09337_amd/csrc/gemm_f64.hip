// FP64 matrix-core GEMM for the Schur-complement update (Sec. 7, routine
// A11; Table 1: local gemm for LU, triangular gemm for Cholesky).
//
//   C = beta * C + alpha * op(A) * op(B)
//
// Output-stationary tiling: a square tile of C per workgroup (4 waves in a
// 2 x 2 arrangement, each wave W x W blocks of the 16x16x4 FP64 MFMA),
// streamed over k in steps of 16 through LDS with register prefetch of the
// next step.  This is the tile-streaming schedule the I/O bound of Sec. 6.1
// is attained by (each element of op(A) / op(B) brought into LDS feeds one
// multiply-add per tile column / row).  A single wave per SIMD does not keep
// the FP64 matrix pipe busy, so the LU's kernels use 64 x 64 tiles (about
// 100 registers, 17 KB of LDS: four or more workgroups per CU, some issuing
// MFMAs while others sit at a barrier or in their epilogue); the Cholesky's
// (B transposed, lower-triangle SYRK) run faster on 128 x 128 tiles.
//
// Workgroups are remapped so that each XCD (hardware assigns workgroup b to
// XCD b % 8) gets a contiguous run of tiles, and runs are walked in groups of
// 8 tile-rows so the A and B panels an XCD touches stay in its L2.
#include "internal.h"


namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int BK = 16;
constexpr int NT = 256;

// Tile shape per kernel: W x W blocks of 16x16 per wave, 2 x 2 waves, sized
// for OCC workgroups per CU.  The LU's updates (op(B) = B) run best on
// 64 x 64 tiles, the Cholesky's (op(B) = B^T, including the lower-triangle
// SYRK) on 128 x 128 tiles (measured).
template <int TB>
struct Shape {
    static constexpr int W = TB == 1 ? 4 : 2;
    static constexpr int B = 32 * W;
    static constexpr int OCC = TB == 1 ? 2 : 4;
};
constexpr int GROUP_M = 8;

// LDS tile of R (rows of the op-operand along M or N) x BK.
// RC (contiguous along R in global): stored [BK][R]; else [R][BK + 1].
template <int R, bool RC>
struct Tile {
    static constexpr int SIZE = RC ? BK * R : R * (BK + 1);
    static constexpr int PER_THREAD = R * BK / NT;
    __device__ static inline int idx(int r, int kk) { return RC ? kk * R + r : r * (BK + 1) + kk; }
    __device__ static inline void coords(int e, int &r, int &kk) {
        if (RC) { r = e % R; kk = e / R; } else { kk = e % BK; r = e / BK; }
    }
};

// Element (r, kk) of the operand is X[(r0+r) + (k0+kk)*ld] if RC, else
// X[(k0+kk) + (r0+r)*ld].  Out-of-range elements read as zero.
template <int R, bool RC>
__device__ inline void load_tile(const double *__restrict__ X, int ld, int r0, int rmax, int k0,
                                 int kmax, double (&reg)[Tile<R, RC>::PER_THREAD], int t) {
#pragma unroll
    for (int q = 0; q < Tile<R, RC>::PER_THREAD; ++q) {
        int r, kk;
        Tile<R, RC>::coords(t + NT * q, r, kk);
        const int gr = r0 + r, gk = k0 + kk;
        double v = 0.0;
        if (gr < rmax && gk < kmax)
            v = RC ? X[(size_t)gr + (size_t)gk * ld] : X[(size_t)gk + (size_t)gr * ld];
        reg[q] = v;
    }
}

template <int R, bool RC>
__device__ inline void store_tile(double *lds, const double (&reg)[Tile<R, RC>::PER_THREAD], int t) {
#pragma unroll
    for (int q = 0; q < Tile<R, RC>::PER_THREAD; ++q) {
        int r, kk;
        Tile<R, RC>::coords(t + NT * q, r, kk);
        lds[Tile<R, RC>::idx(r, kk)] = reg[q];
    }
}

__device__ inline int xcd_remap(int bid, int nwg) {
    const int full = nwg & ~7;
    if (bid >= full) return bid;
    const int per = full >> 3;
    return (bid & 7) * per + (bid >> 3);
}

__device__ inline void grouped_tile(int L, int tiles_m, int tiles_n, int &tm, int &tn) {
    const int group = GROUP_M * tiles_n;
    const int g = L / group;
    const int first_m = g * GROUP_M;
    const int gm = min(tiles_m - first_m, GROUP_M);
    const int in = L - g * group;
    tm = first_m + in % gm;
    tn = in / gm;
}

__device__ inline void lower_tile(int L, int tiles_m, int &tm, int &tn) {
    // Lower triangle in bands of GROUP_M tile rows, each band column by
    // column, so that consecutive workgroups (which share an XCD's L2) reuse
    // one B column strip across the band's rows, as grouped_tile does for
    // full matrices.  The band of L is that of its row in the row-wise
    // enumeration L = r(r+1)/2 + c, since bands are made of whole rows.
    int r = (int)((sqrt(8.0 * (double)L + 1.0) - 1.0) * 0.5);
    while ((r + 1) * (r + 2) / 2 <= L) ++r;
    while (r * (r + 1) / 2 > L) --r;
    const int r0 = r / GROUP_M * GROUP_M;
    const int gr = min(GROUP_M, tiles_m - r0);
    int in = L - r0 * (r0 + 1) / 2;
    if (in < r0 * gr) {  // full columns left of the band's diagonal block
        tn = in / gr;
        tm = r0 + in % gr;
        return;
    }
    in -= r0 * gr;  // the band's gr x gr diagonal block, column c has gr - c tiles
    int c = 0;
    while (in >= gr - c) {
        in -= gr - c;
        ++c;
    }
    tn = r0 + c;
    tm = r0 + c + in;
}

template <int TA, int TB, bool LOWER>
__global__ __launch_bounds__(NT, Shape<TB>::OCC) void dgemm_kernel(int m, int n, int k, double alpha,
                                                      const double *__restrict__ A, int lda,
                                                      const double *__restrict__ B, int ldb,
                                                      double beta, double *__restrict__ C, int ldc,
                                                      int tiles_m, int tiles_n, const int *stop) {
    constexpr int WI = Shape<TB>::W, WJ = Shape<TB>::W, BM = Shape<TB>::B, BN = Shape<TB>::B;
    if (stop != nullptr && *stop != 0) return;
    constexpr bool A_RC = (TA == 0);  // op(A)(i, kk): A[i + kk*lda] when not transposed
    constexpr bool B_RC = (TB == 1);  // op(B)(kk, j) viewed as (j, kk): B[j + kk*ldb] when transposed
    using TA_ = Tile<BM, A_RC>;
    using TB_ = Tile<BN, B_RC>;
    __shared__ double As[TA_::SIZE];
    __shared__ double Bs[TB_::SIZE];

    const int L = xcd_remap(blockIdx.x, gridDim.x);
    int tm, tn;
    if (LOWER) lower_tile(L, tiles_m, tm, tn);
    else grouped_tile(L, tiles_m, tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;

    v4d acc[WI][WJ];
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
        for (int j = 0; j < WJ; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    double ra[TA_::PER_THREAD];
    double rb[TB_::PER_THREAD];
    const int nk = (k + BK - 1) / BK;
    if (nk > 0) {
        load_tile<BM, A_RC>(A, lda, m0, m, 0, k, ra, t);
        load_tile<BN, B_RC>(B, ldb, n0, n, 0, k, rb, t);
        store_tile<BM, A_RC>(As, ra, t);
        store_tile<BN, B_RC>(Bs, rb, t);
    }
    __syncthreads();

    const int lrow = lane & 15;
    const int lk = lane >> 4;
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) {
            load_tile<BM, A_RC>(A, lda, m0, m, (kt + 1) * BK, k, ra, t);
            load_tile<BN, B_RC>(B, ldb, n0, n, (kt + 1) * BK, k, rb, t);
        }
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            const int kk = ks * 4 + lk;
            double af[WI], bf[WJ];
#pragma unroll
            for (int i = 0; i < WI; ++i) af[i] = As[TA_::idx(wm * (16 * WI) + i * 16 + lrow, kk)];
#pragma unroll
            for (int j = 0; j < WJ; ++j) bf[j] = Bs[TB_::idx(wn * (16 * WJ) + j * 16 + lrow, kk)];
#pragma unroll
            for (int i = 0; i < WI; ++i)
#pragma unroll
                for (int j = 0; j < WJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
        if (kt + 1 < nk) {
            store_tile<BM, A_RC>(As, ra, t);
            store_tile<BN, B_RC>(Bs, rb, t);
            __syncthreads();
        }
    }

    // 16x16 output block layout of the FP64 MFMA: register v of a lane holds
    // row 4*v + lane/16, column lane%16.
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
        for (int j = 0; j < WJ; ++j) {
            const int col = n0 + wn * (16 * WJ) + j * 16 + lrow;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * (16 * WI) + i * 16 + v * 4 + lk;
                if (row < m && col < n && (!LOWER || row >= col)) {
                    double *p = C + (size_t)row + (size_t)col * ldc;
                    const double c0 = beta == 0.0 ? 0.0 : beta * *p;
                    *p = fma(alpha, acc[i][j][v], c0);
                }
            }
        }
}

// C = beta C + alpha A op(B) (op(B) = B or B^T; LOWER: lower-triangle tiles
// only, as the SYRK of the Cholesky) with the operands brought into LDS
// by the direct global-to-LDS path (global_load_lds_dwordx4): no staging
// registers and no LDS store instructions, two LDS stages, one barrier per
// K step.  32 KB of LDS and about 70 registers give five workgroups per CU;
// a 64 x 64 tile per workgroup as above.  Lane l of an A load instruction
// writes bytes [16 l, 16 l + 16) of a 1 KB block: rows 2(l % 32) and
// 2(l % 32) + 1 of k-column l / 32.  A B instruction covers 8 columns x 16
// k; its lanes fetch k-pairs in XOR-swizzled order, so that the fragment
// reads of 16 consecutive columns spread over the LDS banks.  Requirements,
// checked by the launcher: k % 16 == 0, m (and n for B^T) and both leading
// dimensions even, A and B 16-byte aligned.  For op(B) = B^T the B tile is
// loaded like the A tile.  Rows and columns past the matrix are clamped to
// valid ones, and their results are discarded.
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glob_void;

// Workgroups resident per CU: the kernel's 32 KB of static LDS fits five in
// a CU's 160 KB; dynamic LDS that the kernel never touches pads each one so
// that fewer fit, leaving LDS (and registers) to kernels on other streams.
// The count comes with each call (the calling handle's setting).
inline size_t dl_pad_bytes(int wg_per_cu) {
    const int w = wg_per_cu >= 3 && wg_per_cu <= 5 ? wg_per_cu : 5;
    if (w >= 5) return 0;
    return (size_t)(160 * 1024 / w) / 512 * 512 - 32 * 1024;
}

// TAG only names the launch (0: the Schur-complement updates, 1: the
// products forming L11^-1 and U12 = L11^-1 A12), so that kernel traces and
// counter runs report the two apart; the code is the same.
template <int TB, bool LOWER, int TAG = 0>
__global__ __launch_bounds__(NT, 5) void dgemm_dl_kernel(int m, int n, int k, double alpha,
                                                         const double *__restrict__ A, int lda,
                                                         const double *__restrict__ B, int ldb, double beta,
                                                         double *__restrict__ C, int ldc, int tiles_m, int tiles_n,
                                                         const int *stop) {
    if (stop != nullptr && *stop != 0) return;
    constexpr int W = 2, BT = 64, STAGE = 2 * BT * BK;  // doubles per stage (A then B)
    __shared__ __attribute__((aligned(16))) double S[2 * STAGE];
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    int tm, tn;
    if (LOWER) lower_tile(L, tiles_m, tm, tn);
    else grouped_tile(L, tiles_m, tiles_n, tm, tn);
    const int m0 = tm * BT, n0 = tn * BT;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1, lrow = lane & 15, lk = lane >> 4;
    const int arow = min(m0 + 2 * (lane & 31), m - 2);
    const double *asrc = A + arow + (size_t)(lane >> 5) * lda;
    // op(B) = B: column-major k x n, 8 columns x 16 k per instruction, k-pairs swizzled;
    // op(B) = B^T: B is n x k, loaded like A (2 columns of op(B) per lane, 2 k per instruction)
    const int bq = (lane & 7) ^ (lane >> 3);
    const double *bsrc0, *bsrc1;
    if (TB == 0) {
        bsrc0 = B + 2 * bq + (size_t)min(n0 + 16 * wave + (lane >> 3), n - 1) * ldb;
        bsrc1 = B + 2 * bq + (size_t)min(n0 + 16 * wave + 8 + (lane >> 3), n - 1) * ldb;
    } else {
        bsrc0 = B + min(n0 + 2 * (lane & 31), n - 2) + (size_t)(lane >> 5) * ldb;
        bsrc1 = bsrc0;
    }
    auto issue = [&](int kt) {
        double *st = S + (kt & 1) * STAGE;
        const size_t k0 = (size_t)kt * BK;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = 2 * wave + u;  // k-columns 2i, 2i + 1
            __builtin_amdgcn_global_load_lds((glob_void *)(asrc + (k0 + 2 * i) * lda), (lds_void *)(st + i * 128), 16, 0,
                                             0);
        }
        if (TB == 0) {
            __builtin_amdgcn_global_load_lds((glob_void *)(bsrc0 + k0), (lds_void *)(st + BT * BK + (2 * wave) * 128),
                                             16, 0, 0);
            __builtin_amdgcn_global_load_lds((glob_void *)(bsrc1 + k0),
                                             (lds_void *)(st + BT * BK + (2 * wave + 1) * 128), 16, 0, 0);
        } else {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int i = 2 * wave + u;
                __builtin_amdgcn_global_load_lds((glob_void *)(bsrc0 + (k0 + 2 * i) * ldb),
                                                 (lds_void *)(st + BT * BK + i * 128), 16, 0, 0);
            }
        }
    };
    v4d acc[W][W];
#pragma unroll
    for (int i = 0; i < W; ++i)
#pragma unroll
        for (int j = 0; j < W; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    const int nk = k / BK;
    if (nk > 0) issue(0);
    for (int kt = 0; kt < nk; ++kt) {
        __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0): this stage's loads have landed in LDS
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();       // ... for every wave; the other stage is free
        asm volatile("" ::: "memory");
        if (kt + 1 < nk) issue(kt + 1);
        const double *As = S + (kt & 1) * STAGE;
        const double *Bs = As + BT * BK;
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            const int kk = ks * 4 + lk;
            double af[W], bf[W];
#pragma unroll
            for (int i = 0; i < W; ++i) af[i] = As[kk * BT + wm * 32 + i * 16 + lrow];
#pragma unroll
            for (int j = 0; j < W; ++j) {
                const int cc = wn * 32 + j * 16 + lrow;
                bf[j] = TB == 0 ? Bs[cc * BK + (((kk >> 1) ^ (cc & 7)) << 1) + (kk & 1)] : Bs[kk * BT + cc];
            }
#pragma unroll
            for (int i = 0; i < W; ++i)
#pragma unroll
                for (int j = 0; j < W; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < W; ++i)
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const int col = n0 + wn * 32 + j * 16 + lrow;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 32 + i * 16 + v * 4 + lk;
                if (row < m && col < n && (!LOWER || row >= col)) {
                    double *p = C + (size_t)row + (size_t)col * ldc;
                    const double c0 = beta == 0.0 ? 0.0 : beta * *p;
                    *p = fma(alpha, acc[i][j][v], c0);
                }
            }
        }
}

// C = beta C + alpha A B with 128 x 128 tiles (op(B) = B, the LU's update):
// the same direct-to-LDS operand path, each wave computing a 64 x 64 block
// (4 x 4 MFMA blocks, 16 independent accumulators).  Per K step a workgroup
// brings 32 KB into LDS for 0.5 MFLOP, half the bytes per flop of the 64 x 64
// tile, whose loads (16 KB per 0.13 MFLOP, four or five workgroups per CU)
// press on the CU's load path.  Two stages of 34 KB: two workgroups per CU.
// A instruction i of a wave brings k-column 4 wave + i (128 rows; lane l
// rows 2l, 2l + 1); the k-columns sit 144 doubles apart in LDS so that the
// two 16-lane groups of a half-wave reading neighbouring k fall in different
// banks.  B as in the 64 x 64 kernel: 8 columns x 16 k per instruction, k
// pairs XOR-swizzled; wave w brings columns 32 w .. 32 w + 31.
template <int TAG = 0>
__global__ __launch_bounds__(NT, 2) void dgemm_dl128_kernel(int m, int n, int k, double alpha,
                                                            const double *__restrict__ A, int lda,
                                                            const double *__restrict__ B, int ldb, double beta,
                                                            double *__restrict__ C, int ldc, int tiles_m,
                                                            int tiles_n, const int *stop) {
    if (stop != nullptr && *stop != 0) return;
    constexpr int W = 4, BT = 128, AKS = 144;            // A: k-column stride in LDS (doubles)
    constexpr int ASZ = BK * AKS, STAGE = ASZ + BT * BK;  // doubles per stage (A then B)
    __shared__ __attribute__((aligned(16))) double S[2 * STAGE];
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    int tm, tn;
    grouped_tile(L, tiles_m, tiles_n, tm, tn);
    const int m0 = tm * BT, n0 = tn * BT;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1, lrow = lane & 15, lk = lane >> 4;
    const double *asrc = A + min(m0 + 2 * lane, m - 2);
    const int bq = (lane & 7) ^ (lane >> 3);
    const double *bsrc = B + 2 * bq;
    int bcol[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) bcol[u] = min(n0 + 32 * wave + 8 * u + (lane >> 3), n - 1);
    auto issue = [&](int kt) {
        double *st = S + (kt & 1) * STAGE;
        const size_t k0 = (size_t)kt * BK;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = 4 * wave + u;
            __builtin_amdgcn_global_load_lds((glob_void *)(asrc + (k0 + kk) * lda), (lds_void *)(st + kk * AKS), 16, 0,
                                             0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            __builtin_amdgcn_global_load_lds((glob_void *)(bsrc + k0 + (size_t)bcol[u] * ldb),
                                             (lds_void *)(st + ASZ + (4 * wave + u) * 128), 16, 0, 0);
    };
    v4d acc[W][W];
#pragma unroll
    for (int i = 0; i < W; ++i)
#pragma unroll
        for (int j = 0; j < W; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    const int nk = k / BK;
    if (nk > 0) issue(0);
    for (int kt = 0; kt < nk; ++kt) {
        __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0): this stage's loads have landed in LDS
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();       // ... for every wave; the other stage is free
        asm volatile("" ::: "memory");
        if (kt + 1 < nk) issue(kt + 1);
        const double *As = S + (kt & 1) * STAGE;
        const double *Bs = As + ASZ;
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            const int kk = ks * 4 + lk;
            double af[W], bf[W];
#pragma unroll
            for (int i = 0; i < W; ++i) af[i] = As[kk * AKS + wm * 64 + i * 16 + lrow];
#pragma unroll
            for (int j = 0; j < W; ++j) {
                const int cc = wn * 64 + j * 16 + lrow;
                bf[j] = Bs[cc * BK + (((kk >> 1) ^ (cc & 7)) << 1) + (kk & 1)];
            }
#pragma unroll
            for (int i = 0; i < W; ++i)
#pragma unroll
                for (int j = 0; j < W; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < W; ++i)
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const int col = n0 + wn * 64 + j * 16 + lrow;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 64 + i * 16 + v * 4 + lk;
                if (row < m && col < n) {
                    double *p = C + (size_t)row + (size_t)col * ldc;
                    const double c0 = beta == 0.0 ? 0.0 : beta * *p;
                    *p = fma(alpha, acc[i][j][v], c0);
                }
            }
        }
}

// 128 x 128 tiles for the NN update only when the handle asks for them
// (CDF_PARAM_GEMM_TILE = 128).  Measured on one MI355X: alone, on a 32768 x
// 32768 x 512 product, 62.4 TF/s against 59.8 for 64 x 64 tiles, but 49 against
// 55 TF/s on the LU's 65024 x 512 x 512 next-panel product and 49.7 against
// 54 on K = 256; inside the N = 65536 LU the update launches averaged 51.5
// TF/s against 53.6 (two large workgroups per CU leave the panel kernels on
// the second stream less room).  So 64 x 64 stays the default.
inline bool use_tile128(const cdf::GemmCtx &ctx, int m, int n) {
    return ctx.tile == 128 && m >= 128 && n >= 128;
}

bool dl_ok(int tb, int m, int n, int k, const double *A, int lda, const double *B, int ldb) {
    return k % BK == 0 && m >= 2 && m % 2 == 0 && lda % 2 == 0 && ldb % 2 == 0 && (tb == 0 || (n >= 2 && n % 2 == 0)) &&
           (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0;
}

template <int TA, int TB, bool LOWER>
hipError_t launch(hipStream_t s, int m, int n, int k, double alpha, const double *A, int lda,
                  const double *B, int ldb, double beta, double *C, int ldc, const int *stop,
                  const cdf::GemmCtx &ctx) {
    constexpr int BM = Shape<TB>::B, BN = Shape<TB>::B;
    const int kind = ctx.tag >= 0 ? ctx.tag : (LOWER ? cdf::PROF_SYRK : TA * 2 + TB);
    const double flops = LOWER ? (double)m * (m + 1) * k : 2.0 * m * n * k;
    // algorithmic bytes: C read and written once, each operand read once
    const double bytes = 8.0 * (LOWER ? (double)m * (m + 1) + 2.0 * m * k : 2.0 * m * n + (double)m * k + (double)k * n);
    if (TA == 0 && TB == 0 && !LOWER && dl_ok(TB, m, n, k, A, lda, B, ldb) && use_tile128(ctx, m, n)) {
        // direct-to-LDS kernel, 128 x 128 tiles
        const int tm = (m + 127) / 128, tn = (n + 127) / 128;
        const long long nwg = (long long)tm * tn;
        if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
        const int slot = cdf::prof_begin(ctx.prof, s, kind, flops, bytes);
        if (ctx.tag == cdf::PROF_U12)
            hipLaunchKernelGGL((dgemm_dl128_kernel<1>), dim3((unsigned)nwg), dim3(NT), 0, s, m, n, k, alpha, A, lda, B,
                               ldb, beta, C, ldc, tm, tn, stop);
        else
            hipLaunchKernelGGL((dgemm_dl128_kernel<0>), dim3((unsigned)nwg), dim3(NT), 0, s, m, n, k, alpha, A, lda, B,
                               ldb, beta, C, ldc, tm, tn, stop);
        const hipError_t e = hipGetLastError();
        cdf::prof_end(ctx.prof, s, slot);
        return e;
    }
    if (TA == 0 && dl_ok(TB, m, n, k, A, lda, B, ldb)) {
        // direct-to-LDS kernel, 64 x 64 tiles
        const int tm64 = (m + 63) / 64, tn64 = (n + 63) / 64;
        const long long nwg = LOWER ? (long long)tm64 * (tm64 + 1) / 2 : (long long)tm64 * tn64;
        if (nwg <= 0) return hipSuccess;
        if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
        const int slot = cdf::prof_begin(ctx.prof, s, kind, flops, bytes);
        if (TB == 0 && !LOWER && ctx.tag == cdf::PROF_U12)
            hipLaunchKernelGGL((dgemm_dl_kernel<TB, LOWER, 1>), dim3((unsigned)nwg), dim3(NT),
                               dl_pad_bytes(ctx.wg_per_cu), s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, tm64,
                               tn64, stop);
        else
            hipLaunchKernelGGL((dgemm_dl_kernel<TB, LOWER>), dim3((unsigned)nwg), dim3(NT),
                               dl_pad_bytes(ctx.wg_per_cu), s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, tm64,
                               tn64, stop);
        const hipError_t e = hipGetLastError();
        cdf::prof_end(ctx.prof, s, slot);
        return e;
    }
    const int tiles_m = (m + BM - 1) / BM;
    const int tiles_n = (n + BN - 1) / BN;
    long long nwg = LOWER ? (long long)tiles_m * (tiles_m + 1) / 2 : (long long)tiles_m * tiles_n;
    if (nwg <= 0) return hipSuccess;
    if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
    const int slot = cdf::prof_begin(ctx.prof, s, kind, flops, bytes);
    hipLaunchKernelGGL((dgemm_kernel<TA, TB, LOWER>), dim3((unsigned)nwg), dim3(NT), 0, s, m, n, k,
                       alpha, A, lda, B, ldb, beta, C, ldc, tiles_m, tiles_n, stop);
    const hipError_t e = hipGetLastError();
    cdf::prof_end(ctx.prof, s, slot);
    return e;
}

}  // namespace

namespace cdf {

GemmCtx gemm_ctx(cdf_handle_t h, int tag) {
    GemmCtx c;
    c.wg_per_cu = h->params[CDF_PARAM_GEMM_WG_PER_CU];
    c.prof = h->prof;
    c.tag = tag;
    c.tile = h->params[CDF_PARAM_GEMM_TILE];
    return c;
}

hipError_t dgemm(hipStream_t s, int ta, int tb, int m, int n, int k, double alpha, const double *A,
                 int lda, const double *B, int ldb, double beta, double *C, int ldc, bool lower,
                 const int *stop, const GemmCtx *ctx) {
    if (m <= 0 || n <= 0) return hipSuccess;
    const GemmCtx c = ctx ? *ctx : GemmCtx();
    if (lower) {
        if (m != n) return hipErrorInvalidValue;
        if (ta == 0 && tb == 1) return launch<0, 1, true>(s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stop, c);
        return hipErrorInvalidValue;
    }
    if (ta == 0 && tb == 0) return launch<0, 0, false>(s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stop, c);
    if (ta == 0 && tb == 1) return launch<0, 1, false>(s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stop, c);
    if (ta == 1 && tb == 0) return launch<1, 0, false>(s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stop, c);
    return launch<1, 1, false>(s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stop, c);
}

}  // namespace cdf
