// Mixed-precision factorizations: the trailing Schur-complement update
// (Sec. 7, routine A11) runs on low-precision matrix cores (BF16, FP16 or
// OCP E4M3 operands, binary32 accumulation) while the panel, pivot search,
// triangular solves and diagonal-block Cholesky stay in binary64; binary64
// iterative refinement with the original matrix recovers full accuracy
// (low-precision LU with refinement is the related work of Sec. 11).
//
// Operand encoding: tiles of 128 rows of L21 (all nb columns) and of 128
// columns of U12 carry one power-of-two scale 2^e each, e = floor(log2(
// maxfinite / amax)); the product of two tiles is rescaled by 2^-(ea+eb)
// once, exactly, after the binary32 accumulation.  Quantized operands are
// stored K-contiguous (k + row * ld), K zero-padded to a multiple of 32.
#include "internal.h"

#include <cmath>
#include <vector>

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

enum { FMT_BF16 = 1, FMT_FP16 = 2, FMT_E4M3 = 3 };
constexpr int QT = 128;    // quantization tile = update tile
constexpr int KSTEP = 32;  // K of one MFMA; quantized K is padded to this
constexpr int NT = 256;

// ------------------------------------------------------------- encoders
// Round-to-nearest-even from a binary32 value, by integer arithmetic on
// its bits (normal range) or an exact rescale and rint (subnormal range).

__device__ inline unsigned short enc_bf16(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ inline unsigned short enc_f16(float y) {  // |y| <= 65504
    const unsigned u = __float_as_uint(y);
    const unsigned s = (u >> 16) & 0x8000u;
    const unsigned a = u & 0x7fffffffu;
    if ((int)(a >> 23) - 127 >= -14) {
        const unsigned r = (a + 0xfffu + ((a >> 13) & 1u)) >> 13;
        return (unsigned short)(s | (r - ((127u - 15u) << 10)));
    }
    return (unsigned short)(s | (unsigned)rintf(__uint_as_float(a) * 16777216.0f));
}

__device__ inline unsigned char enc_e4m3(float y) {  // saturating at 448
    const unsigned u = __float_as_uint(y);
    const unsigned s = (u >> 24) & 0x80u;
    const unsigned a = u & 0x7fffffffu;
    if (a >= 0x43e00000u) return (unsigned char)(s | 0x7eu);
    if ((int)(a >> 23) - 127 >= -6) {
        const unsigned r = (a + 0x7ffffu + ((a >> 20) & 1u)) >> 20;
        const unsigned c = r - ((127u - 7u) << 3);
        return (unsigned char)(s | (c > 0x7eu ? 0x7eu : c));
    }
    return (unsigned char)(s | (unsigned)rintf(__uint_as_float(a) * 512.0f));
}

// e = floor(log2(maxfinite / amax)) from the binary32 fields of amax, capped at 64.
__device__ inline int tile_exp(int fmt, float amax) {
    if (fmt == FMT_BF16 || !(amax > 0.0f)) return 0;
    const unsigned u = __float_as_uint(amax);
    const int ef = (int)(u >> 23);
    if (ef == 0) return 64;
    const int Ef = fmt == FMT_FP16 ? 15 : 8;
    const unsigned mf = fmt == FMT_FP16 ? 0x7fe000u : 0x600000u;  // fraction bits of 65504 / 448
    const int e = Ef - (ef - 127) - ((u & 0x7fffffu) > mf ? 1 : 0);
    return e > 64 ? 64 : e;
}

template <int FMT>
__device__ inline void put_code(void *Q, size_t off, float y) {
    if (FMT == FMT_E4M3) static_cast<unsigned char *>(Q)[off] = enc_e4m3(y);
    else if (FMT == FMT_FP16) static_cast<unsigned short *>(Q)[off] = enc_f16(y);
    else static_cast<unsigned short *>(Q)[off] = enc_bf16(y);
}

__device__ inline float block_max(float v, float *red) {
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    float r = red[0];
    for (int w = 1; w < NT / 64; ++w) r = fmaxf(r, red[w]);
    return r;
}

// One workgroup per tile (tm x tn of X).  kdim is the K extent (columns of X
// when trans, rows otherwise); codes for K in [kdim, kpad) are written as 0
// by the tiles on the K boundary.  trans: X rows are the output rows
// (Q[k + i*ldq] = code(X[i, k])), via an LDS transpose; else Q[i + j*ldq] = code(X[i, j]).
template <int FMT>
__global__ __launch_bounds__(NT) void quantize_kernel(int m, int n, const float *__restrict__ X, int ldx, int tm,
                                                      int tn, void *__restrict__ Q, int ldq, int *__restrict__ exps,
                                                      int kpad, int trans) {
    __shared__ float red[NT / 64];
    __shared__ float chunk[64][65];
    const int ti = blockIdx.x, tj = blockIdx.y;
    const int i0 = ti * tm, j0 = tj * tn;
    const int i1 = min(i0 + tm, m), j1 = min(j0 + tn, n);
    const int h = i1 - i0, w = j1 - j0;
    const int t = threadIdx.x;
    float amax = 0.0f;
    for (int e = t; e < h * w; e += NT) {
        const int i = i0 + e % h, j = j0 + e / h;
        amax = fmaxf(amax, fabsf(X[(size_t)i + (size_t)j * ldx]));
    }
    amax = block_max(amax, red);
    const int ex = tile_exp(FMT, amax);
    if (t == 0) exps[ti + tj * gridDim.x] = ex;
    if (!trans) {
        // rows are K; pad rows [m, kpad) with zeros on the last row tile
        const int iend = (i1 == m) ? max(kpad, m) : i1;
        const int hh = iend - i0;
        for (int e = t; e < hh * w; e += NT) {
            const int i = i0 + e % hh, j = j0 + e / hh;
            const float y = i < m ? ldexpf(X[(size_t)i + (size_t)j * ldx], ex) : 0.0f;
            put_code<FMT>(Q, (size_t)i + (size_t)j * ldq, y);
        }
        return;
    }
    // columns are K; pad columns [n, kpad) with zeros on the last column tile
    const int jend = (j1 == n) ? max(kpad, n) : j1;
    for (int ib = i0; ib < i1; ib += 64)
        for (int jb = j0; jb < jend; jb += 64) {
            __syncthreads();
            for (int e = t; e < 64 * 64; e += NT) {
                const int r = e % 64, c = e / 64;
                const int i = ib + r, j = jb + c;
                chunk[r][c] = (i < i1 && j < j1) ? X[(size_t)i + (size_t)j * ldx] : 0.0f;
            }
            __syncthreads();
            for (int e = t; e < 64 * 64; e += NT) {
                const int c = e % 64, r = e / 64;
                const int i = ib + r, j = jb + c;
                if (i < i1 && j < jend) put_code<FMT>(Q, (size_t)j + (size_t)i * ldq, ldexpf(chunk[r][c], ex));
            }
        }
}

// ------------------------------------------------------------- update GEMM

template <int FMT>
struct Frag;
template <>
struct Frag<FMT_BF16> {
    typedef v8bf T;
    static constexpr int ES = 2;
    __device__ static T lds(const unsigned char *p) { return *reinterpret_cast<const T *>(p); }
    __device__ static v4f mma(T a, T b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
template <>
struct Frag<FMT_FP16> {
    typedef v8h T;
    static constexpr int ES = 2;
    __device__ static T lds(const unsigned char *p) { return *reinterpret_cast<const T *>(p); }
    __device__ static v4f mma(T a, T b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};
template <>
struct Frag<FMT_E4M3> {
    typedef long T;
    static constexpr int ES = 1;
    __device__ static T lds(const unsigned char *p) { return *reinterpret_cast<const long *>(p); }
    __device__ static v4f mma(T a, T b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0); }
};

__device__ inline int xcd_remap(int bid, int nwg) {
    const int full = nwg & ~7;
    if (bid >= full) return bid;
    return (bid & 7) * (full >> 3) + (bid >> 3);
}

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glob_void;

// C (binary32) -= dq(QA) dq(QB): a 128 x 128 tile per workgroup, 64 x 64 per
// wave as 4 x 4 blocks of the 16x16x32 MFMA, two workgroups per CU.  The
// update streams C once (read + write, 8 bytes per element against 2k
// flops), so it is bound by HBM: C is read with 16-byte loads at the start
// into registers of its own and written once at the end as C - 2^-(ea+eb)
// acc.  The operands come in chunks of 64 bytes of K per row, loaded
// straight into LDS (no register staging) through a ring of four stages, so
// that three chunks are in flight while one is multiplied: the operand rows
// are shared by many tiles and mostly hit L2 or the last-level cache, whose
// latency one chunk of work does not cover.  In LDS a row's four 16-byte
// pieces are stored XOR-swizzled by bits 2..3 of the row, so the fragment
// reads of 16 consecutive rows fall in distinct banks without padding.
template <int FMT, bool LOWER>
__global__ __launch_bounds__(NT, 2) void lowp_gemm_kernel(int m, int n, int kpad, const void *__restrict__ QA, int lda,
                                                          const int *__restrict__ ea, const void *__restrict__ QB,
                                                          int ldb, const int *__restrict__ eb, float *__restrict__ C,
                                                          int ldc, int tiles_m, int tiles_n, const int *stop) {
    if (stop != nullptr && *stop != 0) return;
    using F = Frag<FMT>;
    constexpr int ES = F::ES;    // bytes per code
    constexpr int CB = 64;       // bytes of K per row and chunk
    constexpr int KC = CB / ES;  // K per chunk (one or two MFMA steps)
    constexpr int NS = 4;        // LDS stages
    constexpr int SB = 2 * QT * CB;  // bytes per stage: A rows, then B rows
    __shared__ __attribute__((aligned(16))) unsigned char S[NS * SB];
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    int tm, tn;
    if (LOWER) {
        int r = (int)((sqrt(8.0 * (double)L + 1.0) - 1.0) * 0.5);
        while ((r + 1) * (r + 2) / 2 <= L) ++r;
        while (r * (r + 1) / 2 > L) --r;
        tm = r;
        tn = L - r * (r + 1) / 2;
    } else {
        constexpr int GM = 8;
        const int group = GM * tiles_n, g = L / group, first = g * GM, gm = min(tiles_m - first, GM);
        const int in = L - g * group;
        tm = first + in % gm;
        tn = in / gm;
    }
    const int m0 = tm * QT, n0 = tn * QT;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int lrow = lane & 15, lk = lane >> 4;
    const int sc = ea[tm] + eb[tn];
    // interior tile (the whole tile inside C, and for the lower form strictly
    // below the diagonal) with 16-byte aligned columns: every lane takes the
    // vector path.  The test is uniform over the workgroup, so the vector
    // loads are issued back to back (a per-lane choice between vector and
    // element loads into the same registers makes each vector load wait for
    // all earlier ones).
    const bool full = ((reinterpret_cast<uintptr_t>(C) & 15) == 0) && (ldc & 3) == 0 && m0 + QT <= m &&
                      n0 + QT <= n && (!LOWER || tm > tn);

    // 16x16 f32 output block: register v of a lane holds row 4*(lane/16)+v, column lane%16.
    v4f acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    // C in whole column segments: wave w holds tile columns 32 w .. 32 w + 31,
    // register q of lane l the rows 4 (l % 32) .. 4 (l % 32) + 3 of column
    // 32 w + 2 q + l / 32, so each load and store instruction covers two
    // 512-byte column pieces.
    const int crow = 4 * (lane & 31);
    v4f cc[16];
    if (full) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int col = n0 + 32 * wave + 2 * q + (lane >> 5);
            cc[q] = *reinterpret_cast<const v4f *>(C + (size_t)(m0 + crow) + (size_t)col * ldc);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int col = n0 + 32 * wave + 2 * q + (lane >> 5);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + crow + v;
                cc[q][v] = (row < m && col < n && (!LOWER || row >= col)) ? C[(size_t)row + (size_t)col * ldc] : 0.f;
            }
        }
    }

    // Loads of a chunk: wave w brings row groups 2w, 2w + 1 (16 rows each) of
    // A and of B, one 1 KB instruction per group: lane l writes the group's
    // LDS bytes 16 l .. 16 l + 15, i.e. slot l % 4 of row l / 4, which holds
    // the row's piece (l % 4) ^ ((row / 4) % 4).  Rows past the matrix read
    // its last row and pieces past the padded K its last piece (the products
    // of such rows are not stored; such K steps are skipped).
    const unsigned char *qa = static_cast<const unsigned char *>(QA);
    const unsigned char *qb = static_cast<const unsigned char *>(QB);
    const int kbytes = kpad * ES;
    const int lr = lane >> 2, piece = (lane & 3) ^ ((lr >> 2) & 3);
    const unsigned char *asrc[2], *bsrc[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int g = 2 * wave + u;
        asrc[u] = qa + (size_t)min(m0 + 16 * g + lr, m - 1) * lda * ES;
        bsrc[u] = qb + (size_t)min(n0 + 16 * g + lr, n - 1) * ldb * ES;
    }
    auto issue = [&](int c) {
        unsigned char *st = S + (c % NS) * SB;
        const int off = min(c * CB + piece * 16, kbytes - 16);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int g = 2 * wave + u;
            __builtin_amdgcn_global_load_lds((glob_void *)(asrc[u] + off), (lds_void *)(st + g * 1024), 16, 0, 0);
            __builtin_amdgcn_global_load_lds((glob_void *)(bsrc[u] + off), (lds_void *)(st + QT * CB + g * 1024), 16,
                                             0, 0);
        }
    };
    // LDS byte of (row, byte b of the chunk) in a stage
    auto lds_at = [](int row, int b) { return row * CB + ((((b >> 4) ^ (row >> 2)) & 3) << 4) + (b & 15); };
    const int nc = (kbytes + CB - 1) / CB;
#pragma unroll
    for (int q = 0; q < NS - 1; ++q)
        if (q < nc) issue(q);
    for (int c = 0; c < nc; ++c) {
        // this wave's loads of chunk c have landed: the later chunks issued
        // so far (4 loads each) may still be in flight
        const int ahead = min(nc - 1 - c, NS - 2);
        if (ahead >= 2) __builtin_amdgcn_s_waitcnt(0xF78);       // vmcnt(8)
        else if (ahead == 1) __builtin_amdgcn_s_waitcnt(0xF74);  // vmcnt(4)
        else __builtin_amdgcn_s_waitcnt(0xF70);                  // vmcnt(0)
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();  // ... for every wave; the stage of chunk c - 1 is free
        asm volatile("" ::: "memory");
        if (c + NS - 1 < nc) issue(c + NS - 1);
        const unsigned char *As = S + (c % NS) * SB;
        const unsigned char *Bs = As + QT * CB;
#pragma unroll
        for (int ks = 0; ks < KC / KSTEP; ++ks) {
            if (c * KC + ks * KSTEP >= kpad) break;
            const int b = (ks * KSTEP + lk * 8) * ES;
            typename F::T af[4], bf[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                af[i] = F::lds(As + lds_at(wm * 64 + i * 16 + lrow, b));
                bf[i] = F::lds(Bs + lds_at(wn * 64 + i * 16 + lrow, b));
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = F::mma(af[i], bf[j], acc[i][j]);
        }
    }

    // 2^-(ea+eb) acc through LDS (the operand stages are free once every
    // wave is past its last chunk) into the column layout of C: tile column
    // c holds its 32 four-row pieces at slots XOR-ed with c % 32, so the
    // writes of 16 columns and the reads of one column are conflict-free.
    __syncthreads();
    float *X = reinterpret_cast<float *>(S);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = wn * 64 + j * 16 + lrow;
            const int piece = (wm * 64 + i * 16 + lk * 4) >> 2;
            v4f a;
#pragma unroll
            for (int v = 0; v < 4; ++v) a[v] = ldexpf(acc[i][j][v], -sc);
            *reinterpret_cast<v4f *>(X + col * QT + ((piece ^ (col & 31)) << 2)) = a;
        }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int tc = 32 * wave + 2 * q + (lane >> 5), col = n0 + tc;
        const v4f a = *reinterpret_cast<const v4f *>(X + tc * QT + ((((lane & 31) ^ (tc & 31))) << 2));
        v4f out;
#pragma unroll
        for (int v = 0; v < 4; ++v) out[v] = cc[q][v] - a[v];
        if (full) {
            *reinterpret_cast<v4f *>(C + (size_t)(m0 + crow) + (size_t)col * ldc) = out;
        } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + crow + v;
                if (row < m && col < n && (!LOWER || row >= col)) C[(size_t)row + (size_t)col * ldc] = out[v];
            }
        }
    }
}

// ------------------------------------------------------------- elementwise

template <typename S, typename D>
__global__ void convert_kernel(int m, int n, const S *__restrict__ a, int lda, D *__restrict__ b, int ldb, int lower) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= m || j >= n) return;
    if (lower && i < j) return;
    b[(size_t)i + (size_t)j * ldb] = (D)a[(size_t)i + (size_t)j * lda];
}

__global__ void add_offset_kernel(const int *__restrict__ src, int *__restrict__ dst, int count, int off) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = src[i] + off;
}

// Row sums of |A| (partial over a column slab), accumulated by atomics into rs.
__global__ void rowsum_abs_kernel(int n, const double *__restrict__ a, int lda, double *__restrict__ rs, int cols) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j0 = blockIdx.y * cols;
    if (i >= n) return;
    double s = 0.0;
    const int j1 = min(n, j0 + cols);
    for (int j = j0; j < j1; ++j) s += fabs(a[(size_t)i + (size_t)j * lda]);
    atomicAdd(rs + i, s);
}

__device__ inline void atomic_max_pos(double *p, double v) {
    // values are >= 0: their bit patterns order as unsigned 64-bit integers
    atomicMax(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}

__global__ void vec_absmax_kernel(int n, const double *__restrict__ x, double *__restrict__ out) {
    __shared__ double red[4];
    double v = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) v = fmax(v, fabs(x[i]));
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, red[w]);
        atomic_max_pos(out, r);
    }
}

// R = B - A X for nrhs <= 4 (binary64): 64 rows per workgroup, one row per
// lane, the 4 waves take interleaved column slabs; partial sums are combined
// in a fixed order (deterministic).
__global__ __launch_bounds__(256) void residual_gemv_kernel(int n, int nrhs, const double *__restrict__ A, int lda,
                                                            const double *__restrict__ X, int ldx,
                                                            const double *__restrict__ B, int ldb,
                                                            double *__restrict__ R, int ldr) {
    __shared__ double part[4][4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = blockIdx.x * 64 + lane;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (r < n) {
        for (int j0 = wave * 64; j0 < n; j0 += 256) {
            const int j1 = min(j0 + 64, n);
            for (int j = j0; j < j1; ++j) {
                const double a = A[(size_t)r + (size_t)j * lda];
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (c < nrhs) acc[c] = fma(a, X[(size_t)j + (size_t)c * ldx], acc[c]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) part[wave][c][lane] = acc[c];
    __syncthreads();
    if (wave == 0 && r < n)
        for (int c = 0; c < nrhs; ++c) {
            const double ax = ((part[0][c][lane] + part[1][c][lane]) + part[2][c][lane]) + part[3][c][lane];
            R[(size_t)r + (size_t)c * ldr] = B[(size_t)r + (size_t)c * ldb] - ax;
        }
}

// -------------------------------------------- preconditioned CG (SPD)
// The fallback of the SPD solver when classical refinement fails: block PCG,
// every right-hand side its own CG recurrence (Hestenes-Stiefel with the
// low-precision Cholesky factor as preconditioner), binary64.  The per-column
// scalars stay on the device; dot products are reduced in a fixed order.

// W(i, i) = binary32(A(i, i) * (1 + sigma)): the diagonal of the shifted
// matrix A + sigma diag(A) (sigma a power of two, so 1 + sigma is exact).
__global__ void shift_diag_kernel(int n, const double *__restrict__ a, int lda, float *__restrict__ w, int ldw,
                                  double sigma) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[(size_t)i + (size_t)i * ldw] = (float)(a[(size_t)i + (size_t)i * lda] * (1.0 + sigma));
}

constexpr int kDotBlocks = 64;  // partial sums per column
constexpr int kMaxShifts = 6;   // shifted factorizations tried after a breakdown

// part[c * kDotBlocks + b] = sum over the rows block b visits of x(i, c) y(i, c)
__global__ __launch_bounds__(256) void dot_partial_kernel(int n, const double *__restrict__ x, int ldx,
                                                          const double *__restrict__ y, int ldy,
                                                          double *__restrict__ part) {
    __shared__ double red[4];
    const int c = blockIdx.y, b = blockIdx.x;
    double v = 0.0;
    for (int i = b * 256 + threadIdx.x; i < n; i += kDotBlocks * 256)
        v = fma(x[(size_t)i + (size_t)c * ldx], y[(size_t)i + (size_t)c * ldy], v);
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) part[(size_t)c * kDotBlocks + b] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ void dot_finish_kernel(int nrhs, const double *__restrict__ part, double *__restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    double s = 0.0;
    for (int b = 0; b < kDotBlocks; ++b) s += part[(size_t)c * kDotBlocks + b];
    out[c] = s;
}

// alpha = rho / (p.q) (0 where p.q = 0); x += alpha p; r -= alpha q
__global__ void pcg_xr_kernel(int n, int nrhs, const double *__restrict__ rho, const double *__restrict__ pq,
                              const double *__restrict__ p, const double *__restrict__ q, double *__restrict__ x,
                              int ldx, double *__restrict__ r) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n || c >= nrhs) return;
    const double d = pq[c];
    const double alpha = d != 0.0 ? rho[c] / d : 0.0;
    const size_t o = (size_t)i + (size_t)c * n;
    x[(size_t)i + (size_t)c * ldx] += alpha * p[o];
    r[o] -= alpha * q[o];
}

// beta = rho_new / rho_old (0 where rho_old = 0); p = z + beta p
__global__ void pcg_p_kernel(int n, int nrhs, const double *__restrict__ rho_new, const double *__restrict__ rho_old,
                             const double *__restrict__ z, double *__restrict__ p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n || c >= nrhs) return;
    const double d = rho_old[c];
    const double beta = d != 0.0 ? rho_new[c] / d : 0.0;
    const size_t o = (size_t)i + (size_t)c * n;
    p[o] = z[o] + beta * p[o];
}

// out[3 c + slot] = max |x(i, c)| over i (out zeroed beforehand)
__global__ __launch_bounds__(256) void col_absmax_kernel(int n, const double *__restrict__ x, int ldx,
                                                         double *__restrict__ out, int slot) {
    __shared__ double red[4];
    const int c = blockIdx.y;
    double v = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
        v = fmax(v, fabs(x[(size_t)i + (size_t)c * ldx]));
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(reinterpret_cast<unsigned long long *>(out + 3 * c + slot),
                  (unsigned long long)__double_as_longlong(fmax(fmax(red[0], red[1]), fmax(red[2], red[3]))));
}

__global__ void zero_d_kernel(double *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0;
}

__global__ void axpy_kernel(int n, int nrhs, const double *__restrict__ d, int ldd, double *__restrict__ x, int ldx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i < n && c < nrhs) x[(size_t)i + (size_t)c * ldx] += d[(size_t)i + (size_t)c * ldd];
}

__global__ void copy_kernel(int n, int nrhs, const double *__restrict__ s, int lds, double *__restrict__ d, int ldd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i < n && c < nrhs) d[(size_t)i + (size_t)c * ldd] = s[(size_t)i + (size_t)c * lds];
}

template <int FMT>
hipError_t quantize_t(hipStream_t s, int m, int n, const float *X, int ldx, int tm, int tn, void *Q, int ldq, int *exps,
                      int kpad, bool trans) {
    const int mt = (m + tm - 1) / tm, nt = (n + tn - 1) / tn;
    hipLaunchKernelGGL((quantize_kernel<FMT>), dim3(mt, nt), dim3(NT), 0, s, m, n, X, ldx, tm, tn, Q, ldq, exps, kpad,
                       trans ? 1 : 0);
    return hipGetLastError();
}

template <int FMT, bool LOWER>
hipError_t lowp_t(hipStream_t s, int m, int n, int kpad, const void *QA, int lda, const int *ea, const void *QB, int ldb,
                  const int *eb, float *C, int ldc, const int *stop) {
    const int tm = (m + QT - 1) / QT, tn = (n + QT - 1) / QT;
    const long long nwg = LOWER ? (long long)tm * (tm + 1) / 2 : (long long)tm * tn;
    if (nwg <= 0) return hipSuccess;
    hipLaunchKernelGGL((lowp_gemm_kernel<FMT, LOWER>), dim3((unsigned)nwg), dim3(NT), 0, s, m, n, kpad, QA, lda, ea, QB,
                       ldb, eb, C, ldc, tm, tn, stop);
    return hipGetLastError();
}

inline int kpad_of(int k) { return (k + KSTEP - 1) / KSTEP * KSTEP; }
inline size_t esize(int fmt) { return fmt == FMT_E4M3 ? 1 : 2; }

}  // namespace

namespace cdf {

int lowp_tile(int) { return QT; }

hipError_t convert_d2s(hipStream_t s, int m, int n, const double *A, int lda, float *W, int ldw, bool lower_only) {
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL((convert_kernel<double, float>), dim3((m + 255) / 256, n), dim3(256), 0, s, m, n, A, lda, W,
                       ldw, lower_only ? 1 : 0);
    return hipGetLastError();
}

hipError_t convert_s2d(hipStream_t s, int m, int n, const float *W, int ldw, double *A, int lda, bool lower_only) {
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL((convert_kernel<float, double>), dim3((m + 255) / 256, n), dim3(256), 0, s, m, n, W, ldw, A,
                       lda, lower_only ? 1 : 0);
    return hipGetLastError();
}

hipError_t quantize(hipStream_t s, int fmt, int m, int n, const float *X, int ldx, int tm, int tn, void *Q, int ldq,
                    int *exps, bool transpose_out) {
    if (m <= 0 || n <= 0) return hipSuccess;
    const int kpad = min(transpose_out ? kpad_of(n) : kpad_of(m), ldq);
    if (fmt == FMT_BF16) return quantize_t<FMT_BF16>(s, m, n, X, ldx, tm, tn, Q, ldq, exps, kpad, transpose_out);
    if (fmt == FMT_FP16) return quantize_t<FMT_FP16>(s, m, n, X, ldx, tm, tn, Q, ldq, exps, kpad, transpose_out);
    if (fmt == FMT_E4M3) return quantize_t<FMT_E4M3>(s, m, n, X, ldx, tm, tn, Q, ldq, exps, kpad, transpose_out);
    return hipErrorInvalidValue;
}

hipError_t lowp_update(hipStream_t s, int fmt, int m, int n, int k, const void *QA, int lda, const int *ea,
                       const void *QB, int ldb, const int *eb, float *C, int ldc, bool lower, const int *stop) {
    if (m <= 0 || n <= 0 || k <= 0) return hipSuccess;
    const int kp = kpad_of(k);
#define CDF_LOWP(F)                                                                              \
    return lower ? lowp_t<F, true>(s, m, n, kp, QA, lda, ea, QB, ldb, eb, C, ldc, stop)          \
                 : lowp_t<F, false>(s, m, n, kp, QA, lda, ea, QB, ldb, eb, C, ldc, stop)
    if (fmt == FMT_BF16) { CDF_LOWP(FMT_BF16); }
    if (fmt == FMT_FP16) { CDF_LOWP(FMT_FP16); }
    if (fmt == FMT_E4M3) { CDF_LOWP(FMT_E4M3); }
#undef CDF_LOWP
    return hipErrorInvalidValue;
}

hipError_t axpy_cols(hipStream_t s, int n, int nrhs, const double *D, int ldd, double *X, int ldx) {
    hipLaunchKernelGGL(axpy_kernel, dim3((n + 255) / 256, nrhs), dim3(256), 0, s, n, nrhs, D, ldd, X, ldx);
    return hipGetLastError();
}

hipError_t copy_cols(hipStream_t s, int n, int nrhs, const double *S, int lds, double *D, int ldd) {
    hipLaunchKernelGGL(copy_kernel, dim3((n + 255) / 256, nrhs), dim3(256), 0, s, n, nrhs, S, lds, D, ldd);
    return hipGetLastError();
}

}  // namespace cdf

namespace {

struct MixedWs {
    float *W = nullptr;        // binary32 working copy, n x n
    double *Wd = nullptr;      // binary64 copy of the finished factor (for the solves)
    double *Afull = nullptr;   // symmetric extension of A (Cholesky residual)
    double *P[2] = {nullptr, nullptr};  // binary64 panels, n x nb each (double-buffered for look-ahead)
    double *U = nullptr;       // binary64 staging of U12, nb x n
    double *U2 = nullptr;      // LU: U12 = L11^-1 U, nb x n
    double *Li[2] = {nullptr, nullptr};  // LU: L11^-1 of panels (buffer p mod 2), nb x nb
    int *good = nullptr;       // LU: per buffer, 1 if Li was accepted (else it is the identity)
    void *QA = nullptr, *QB = nullptr;
    int *ea = nullptr, *eb = nullptr, *ipt = nullptr, *ipiv = nullptr;
    int *lu_ws = nullptr;      // work area of the binary64 LU (fp64 mode)
    double *lu_w = nullptr;    // its U12 / L11^-1 area (fp64 mode)
    int *tsync = nullptr;      // flags of the single-launch triangular solves
    double *R = nullptr, *red = nullptr;
    // SPD fallback (block PCG): z, p, q (n x nrhs each), the per-column
    // scalars (two rho buffers by parity, p.q) and the dot partial sums
    double *Z = nullptr, *Pv = nullptr, *Q = nullptr, *scal = nullptr, *part = nullptr;
    // SPD solves with more than four right-hand sides: inverted diagonal
    // blocks of the factor and an n x nrhs intermediate
    double *Tinv = nullptr, *Yv = nullptr;
};

constexpr int kInvBs = 512;  // diagonal block of the inverse-based triangular solves


cdf_status_t mixed_layout(cdf_handle_t h, int n, int nrhs, int nb, int fmt, bool chol, MixedWs &w,
                          bool factor_only = false, bool fp64_lu = false) {
    size_t off = cdf::kLeafWsBytes;  // LU leaf exchange at the workspace head
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = cdf::align_up(off + bytes, 256);
        return o;
    };
    const size_t nn = (size_t)n * n;
    const size_t kp = kpad_of(nb);
    const size_t oW = factor_only ? 0 : take(nn * sizeof(float));
    const size_t oWd = factor_only ? 0 : take(nn * sizeof(double));
    const size_t oAf = (chol && !factor_only) ? take(nn * sizeof(double)) : 0;
    const size_t oP = take((size_t)n * nb * sizeof(double)), oP1 = take((size_t)n * nb * sizeof(double));
    const size_t oU = take((size_t)n * nb * sizeof(double));
    const size_t oU2 = chol ? 0 : take((size_t)n * nb * sizeof(double));
    const size_t oLi = chol ? 0 : take(2 * (size_t)nb * nb * sizeof(double));
    const size_t ogood = chol ? 0 : take(2 * sizeof(int));
    const size_t oQA = take(kp * n * esize(fmt));
    const size_t oQB = take(kp * n * esize(fmt));
    const int nt = (n + QT - 1) / QT + 1;
    const size_t oea = take(nt * sizeof(int)), oeb = take(nt * sizeof(int));
    const size_t oipt = take((size_t)nb * sizeof(int)), oipiv = take((size_t)n * sizeof(int));
    const size_t olw = take(cdf::getrf_ws_ints() * sizeof(int));
    const size_t olww = fp64_lu ? take(cdf::getrf_w_doubles(n) * sizeof(double)) : 0;
    const size_t ots = take(cdf::trsv_sync_ints(n) * sizeof(int));
    const size_t oR = take((size_t)n * nrhs * sizeof(double));
    const size_t ored = take(((size_t)n + 4 * (size_t)nrhs + 8) * sizeof(double));
    const bool pcg = chol && !factor_only;
    const size_t oZ = pcg ? take(3 * (size_t)n * nrhs * sizeof(double)) : 0;
    const size_t oscal = pcg ? take(4 * (size_t)nrhs * sizeof(double)) : 0;
    const size_t opart = pcg ? take((size_t)kDotBlocks * nrhs * sizeof(double)) : 0;
    const bool inv = pcg && nrhs > 4;
    const size_t oTinv = inv ? take(cdf::inv_blocks_doubles(n, kInvBs) * sizeof(double)) : 0;
    const size_t oYv = inv ? take((size_t)n * nrhs * sizeof(double)) : 0;
    cdf_status_t st = cdf::ws_reserve(h, off);
    if (st != CDF_OK) return st;
    char *base = static_cast<char *>(h->ws);
    w.W = factor_only ? nullptr : reinterpret_cast<float *>(base + oW);
    w.Wd = factor_only ? nullptr : reinterpret_cast<double *>(base + oWd);
    w.Afull = (chol && !factor_only) ? reinterpret_cast<double *>(base + oAf) : nullptr;
    w.P[0] = reinterpret_cast<double *>(base + oP);
    w.P[1] = reinterpret_cast<double *>(base + oP1);
    w.U = reinterpret_cast<double *>(base + oU);
    w.U2 = chol ? nullptr : reinterpret_cast<double *>(base + oU2);
    w.Li[0] = chol ? nullptr : reinterpret_cast<double *>(base + oLi);
    w.Li[1] = chol ? nullptr : w.Li[0] + (size_t)nb * nb;
    w.good = chol ? nullptr : reinterpret_cast<int *>(base + ogood);
    w.QA = base + oQA;
    w.QB = base + oQB;
    w.ea = reinterpret_cast<int *>(base + oea);
    w.eb = reinterpret_cast<int *>(base + oeb);
    w.ipt = reinterpret_cast<int *>(base + oipt);
    w.ipiv = reinterpret_cast<int *>(base + oipiv);
    w.lu_ws = reinterpret_cast<int *>(base + olw);
    w.lu_w = fp64_lu ? reinterpret_cast<double *>(base + olww) : nullptr;
    w.tsync = reinterpret_cast<int *>(base + ots);
    w.R = reinterpret_cast<double *>(base + oR);
    w.red = reinterpret_cast<double *>(base + ored);
    if (pcg) {
        w.Z = reinterpret_cast<double *>(base + oZ);
        w.Pv = w.Z + (size_t)n * nrhs;
        w.Q = w.Pv + (size_t)n * nrhs;
        w.scal = reinterpret_cast<double *>(base + oscal);
        w.part = reinterpret_cast<double *>(base + opart);
    }
    if (inv) {
        w.Tinv = reinterpret_cast<double *>(base + oTinv);
        w.Yv = reinterpret_cast<double *>(base + oYv);
    }
    return CDF_OK;
}

inline int mixed_nb(cdf_handle_t h, int n) {
    const int v = h->params[CDF_PARAM_MIXED_NB];
    return v > 0 ? v : (n >= 16384 ? 512 : 256);
}

// Blocked right-looking LU of the binary32 copy W (see the file comment);
// absolute 1-based pivots go to ipiv.  Look-ahead of depth one, as in the
// binary64 path: the next panel's columns are updated first and that panel
// is factored on the second stream while the rest of the trailing matrix is
// updated (when the panel width is a multiple of the quantization tile, so
// both parts of the update keep the tile exponents of U12).
hipError_t mixed_getrf(cdf_handle_t h, int fmt, int n, float *W, int ldw, int *ipiv, MixedWs &w, int nb, int *info) {
    hipStream_t s0 = h->stream;
    const cdf::GemmCtx gu = cdf::gemm_ctx(h, cdf::PROF_U12);
    CDF_HIP_RET(cdf::ensure_aux(h));
    const cdf::LeafArea la = cdf::handle_leaf_area(h);
    CDF_HIP_RET(cdf::leaf_reset_error(la, s0));
    h->last_err = cdf::leaf_error_word(la);
    hipStream_t s1 = h->aux;
    const int kp = kpad_of(nb);
    const bool split = nb % QT == 0;
    // panel of width kb at column k: binary64 copy in P, factored there,
    // pivots to w.ipt (relative) and ipiv (absolute), copied back to W
    const bool inv = h->params[CDF_PARAM_LU_U12] == 0 && w.Li[0] != nullptr;
    const bool tourn = h->params[CDF_PARAM_LU_PIVOT] == 1;
    auto panel = [&](hipStream_t s, int k, int kb, double *P, int buf) -> hipError_t {
        const int m = n - k;
        CDF_HIP_RET(cdf::convert_s2d(s, m, kb, W + k + (size_t)k * ldw, ldw, P, m, false));
        CDF_HIP_RET(cdf::lu_panel(h, la, s, m, kb, P, m, w.ipt, info, 0, kb, k, tourn));
        if (inv && k + kb < n) CDF_HIP_RET(cdf::unit_lower_inverse(s, kb, P, m, w.Li[buf], nb, w.good + buf, &gu));
        hipLaunchKernelGGL(add_offset_kernel, dim3((kb + 255) / 256), dim3(256), 0, s, w.ipt, ipiv + k, kb, k);
        CDF_HIP_RET(hipGetLastError());
        return cdf::convert_d2s(s, m, kb, P, m, W + k + (size_t)k * ldw, ldw, false);
    };
    CDF_HIP_RET(panel(s0, 0, nb < n ? nb : n, w.P[0], 0));
    for (int k = 0, it = 0; k < n; k += nb, ++it) {
        const int kb = nb < n - k ? nb : n - k;
        const int m = n - k, rest = n - k - kb;
        CDF_HIP_RET(cdf::slaswp(s0, 0, k, W + k, ldw, w.ipt, 0, kb, m));
        CDF_HIP_RET(cdf::slaswp(s0, k + kb, n, W + k, ldw, w.ipt, 0, kb, m));
        if (rest <= 0) break;
        float *w12 = W + k + (size_t)(k + kb) * ldw;
        float *w21 = W + (k + kb) + (size_t)k * ldw;
        float *w22 = W + (k + kb) + (size_t)(k + kb) * ldw;
        // U12 = L11^-1 A12 in binary64: one matrix-core GEMM with the
        // panel's inverse (formed on the panel's stream), or blocked
        // substitution in place
        CDF_HIP_RET(cdf::convert_s2d(s0, kb, rest, w12, ldw, w.U, kb, false));
        if (inv) {
            // substitution in place only where the guard rejected L11^-1 (the
            // GEMM with the identity then copies exactly)
            CDF_HIP_RET(cdf::trsm_small(s0, cdf::TRSM_LLNU, kb, rest, w.P[it & 1], m, w.U, kb, w.good + (it & 1), 512));
            CDF_HIP_RET(cdf::dgemm(s0, 0, 0, kb, rest, kb, 1.0, w.Li[it & 1], nb, w.U, kb, 0.0, w.U2, kb, false,
                                   nullptr, &gu));
            CDF_HIP_RET(cdf::convert_d2s(s0, kb, rest, w.U2, kb, w12, ldw, false));
        } else {
            CDF_HIP_RET(cdf::trsm_blocked(s0, cdf::TRSM_LLNU, kb, rest, w.P[it & 1], m, w.U, kb, 64, &gu));
            CDF_HIP_RET(cdf::convert_d2s(s0, kb, rest, w.U, kb, w12, ldw, false));
        }
        CDF_HIP_RET(cdf::quantize(s0, fmt, rest, kb, w21, ldw, QT, kb, w.QA, kp, w.ea, true));
        CDF_HIP_RET(cdf::quantize(s0, fmt, kb, rest, w12, ldw, kb, QT, w.QB, kp, w.eb, false));
        const int k1 = k + kb;
        const int kb1 = nb < n - k1 ? nb : n - k1;
        if (split && rest > kb1) {
            // next panel's columns, then that panel beside the rest of the update
            CDF_HIP_RET(cdf::lowp_update(s0, fmt, rest, kb1, kb, w.QA, kp, w.ea, w.QB, kp, w.eb, w22, ldw, false,
                                         nullptr));
            CDF_HIP_RET(hipEventRecord(h->ev[0], s0));
            CDF_HIP_RET(hipStreamWaitEvent(s1, h->ev[0], 0));
            CDF_HIP_RET(panel(s1, k1, kb1, w.P[(it + 1) & 1], (it + 1) & 1));
            CDF_HIP_RET(hipEventRecord(h->ev[1], s1));
            const char *qb = static_cast<const char *>(w.QB) + (size_t)kb1 * kp * esize(fmt);
            CDF_HIP_RET(cdf::lowp_update(s0, fmt, rest, rest - kb1, kb, w.QA, kp, w.ea, qb, kp, w.eb + kb1 / QT,
                                         w22 + (size_t)kb1 * ldw, ldw, false, nullptr));
            CDF_HIP_RET(hipStreamWaitEvent(s0, h->ev[1], 0));
        } else {
            CDF_HIP_RET(cdf::lowp_update(s0, fmt, rest, rest, kb, w.QA, kp, w.ea, w.QB, kp, w.eb, w22, ldw, false,
                                         nullptr));
            CDF_HIP_RET(panel(s0, k1, kb1, w.P[(it + 1) & 1], (it + 1) & 1));
        }
    }
    return hipSuccess;
}

// Blocked right-looking lower Cholesky of the binary32 copy W.  Each block
// column is copied to binary64 (P), factored there (diagonal block and the
// rows below it, in sub-blocks of 64 columns: binary64 L11 and L21 = A21
// L11^-T), rounded back to W, and its L21 tile-quantized for the
// low-precision SYRK of the trailing lower triangle.  Look-ahead of depth
// one, as in the binary64 path: the next block column is updated first and
// factored on the second stream while the rest of the trailing triangle is
// updated (when the block width is a multiple of the quantization tile, so
// both parts keep the tile exponents of L21); the quantized L21 of
// consecutive block columns alternates between two buffers.
hipError_t mixed_potrf(cdf_handle_t h, int fmt, int n, float *W, int ldw, MixedWs &w, int nb, int *info) {
    hipStream_t s0 = h->stream;
    CDF_HIP_RET(cdf::ensure_aux(h));
    hipStream_t s1 = h->aux;
    const int kp = kpad_of(nb);
    const bool split = nb % QT == 0;
    void *Q[2] = {w.QA, w.QB};
    int *E[2] = {w.ea, w.eb};
    auto panel = [&](hipStream_t s, int k, int kb, int buf) -> hipError_t {
        const int m = n - k;
        float *wk = W + k + (size_t)k * ldw;
        CDF_HIP_RET(cdf::convert_s2d(s, m, kb, wk, ldw, w.P[buf], m, true));
        CDF_HIP_RET(cdf::potrf_panel(h, s, m, kb, w.P[buf], m, info, k, true));
        CDF_HIP_RET(cdf::convert_d2s(s, m, kb, w.P[buf], m, wk, ldw, true));
        if (m > kb) CDF_HIP_RET(cdf::quantize(s, fmt, m - kb, kb, wk + kb, ldw, QT, kb, Q[buf], kp, E[buf], true));
        return hipSuccess;
    };
    CDF_HIP_RET(panel(s0, 0, nb < n ? nb : n, 0));
    for (int k = 0, it = 0; k < n; k += nb, ++it) {
        const int kb = nb < n - k ? nb : n - k;
        const int k1 = k + kb;
        if (k1 >= n) break;
        const int kb1 = nb < n - k1 ? nb : n - k1;
        const int rest = n - k1;
        const int b = it & 1;
        const char *q = static_cast<const char *>(Q[b]);  // L21 of block column k, rows [k1, n)
        const int *e = E[b];
        float *d1 = W + k1 + (size_t)k1 * ldw;             // next diagonal block
        if (split && rest > kb1) {
            const char *q2 = q + (size_t)kb1 * kp * esize(fmt);  // its rows [k1 + kb1, n)
            const int *e2 = e + kb1 / QT;
            // next block column: its diagonal block (lower) and the rows below it
            CDF_HIP_RET(cdf::lowp_update(s0, fmt, kb1, kb1, kb, q, kp, e, q, kp, e, d1, ldw, true, info));
            CDF_HIP_RET(cdf::lowp_update(s0, fmt, rest - kb1, kb1, kb, q2, kp, e2, q, kp, e, d1 + kb1, ldw, false,
                                         info));
            CDF_HIP_RET(hipEventRecord(h->ev[0], s0));
            CDF_HIP_RET(hipStreamWaitEvent(s1, h->ev[0], 0));
            CDF_HIP_RET(panel(s1, k1, kb1, b ^ 1));
            CDF_HIP_RET(hipEventRecord(h->ev[1], s1));
            CDF_HIP_RET(cdf::lowp_update(s0, fmt, rest - kb1, rest - kb1, kb, q2, kp, e2, q2, kp, e2,
                                         d1 + kb1 + (size_t)kb1 * ldw, ldw, true, info));
            CDF_HIP_RET(hipStreamWaitEvent(s0, h->ev[1], 0));
        } else {
            CDF_HIP_RET(cdf::lowp_update(s0, fmt, rest, rest, kb, q, kp, e, q, kp, e, d1, ldw, true, info));
            CDF_HIP_RET(panel(s0, k1, kb1, b ^ 1));
        }
    }
    return hipSuccess;
}

double hpl_from_norms(const std::vector<double> &v, int nrhs, double anorm, int n) {
    const double eps = std::ldexp(1.0, -53);
    double worst = 0.0;
    for (int c = 0; c < nrhs; ++c) {
        const double r = v[3 * c], x = v[3 * c + 1], b = v[3 * c + 2];
        const double den = eps * (anorm * x + b) * n;
        const double q = den > 0 ? r / den : (r > 0 ? INFINITY : 0.0);
        worst = q > worst ? q : worst;
    }
    return worst;
}

// Unit roundoff of the update format (the first shift of the fallback).
double unit_roundoff(int fmt) {
    return fmt == FMT_E4M3 ? std::ldexp(1.0, -4) : (fmt == FMT_FP16 ? std::ldexp(1.0, -11) : std::ldexp(1.0, -8));
}

cdf_status_t mixed_solve(cdf_handle_t h, int fmt, bool chol, int n, int nrhs, const double *A, int lda,
                         const double *B, int ldb, double *X, int ldx, int max_iter, int *iters, double *resid,
                         int *info) {
    hipStream_t s = h->stream;
    const int nb = mixed_nb(h, n);
    MixedWs w;
    cdf_status_t st = mixed_layout(h, n, nrhs, nb, fmt == 0 ? FMT_BF16 : fmt, chol, w, false, fmt == 0 && !chol);
    if (st != CDF_OK) return st;
    cdf::MixedReport &rep = h->mixed_report;
    rep = cdf::MixedReport();
    // refinement mode of the SPD solver: 0 auto, 1 classical only, 2 PCG
    const int mode = (chol && fmt != 0) ? h->params[CDF_PARAM_SPD_REFINE] : 1;
    const int pcg_max = h->params[CDF_PARAM_PCG_MAX_ITER] > 0 ? h->params[CDF_PARAM_PCG_MAX_ITER] : 400;
    CDF_HIP_TRY(cdf::fill_int(s, info, 1, 0));
    // binary64 ||A||_inf and the matrix the residual is computed with
    const double *Ares = A;
    int ldres = lda;
    if (chol) {
        CDF_HIP_TRY(cdf::copy_cols(s, n, n, A, lda, w.Afull, n));
        CDF_HIP_TRY(cdf::symmetrize_lower(s, n, w.Afull, n));
        Ares = w.Afull;
        ldres = n;
    }
    double *rs = w.red + 4 * nrhs + 8;
    hipLaunchKernelGGL(zero_d_kernel, dim3((n + 4 * nrhs + 8 + 255) / 256), dim3(256), 0, s, w.red, n + 4 * nrhs + 8);
    const int slab = 256;
    hipLaunchKernelGGL(rowsum_abs_kernel, dim3((n + 255) / 256, (n + slab - 1) / slab), dim3(256), 0, s, n, Ares, ldres,
                       rs, slab);
    hipLaunchKernelGGL(vec_absmax_kernel, dim3(256), dim3(256), 0, s, n, rs, w.red);
    CDF_HIP_TRY(hipGetLastError());
    // factorization of the working copy, A + sigma diag(A) for sigma > 0
    auto factor = [&](double sigma, int *hinfo) -> cdf_status_t {
        if (fmt == 0) {
            CDF_HIP_TRY(cdf::copy_cols(s, n, n, A, lda, w.Wd, n));
            if (chol) CDF_HIP_TRY(cdf::potrf_fp64(h, n, w.Wd, n, info));
            else CDF_HIP_TRY(cdf::getrf_fp64(h, n, w.Wd, n, w.ipiv, info, w.lu_ws, w.lu_w));
        } else {
            CDF_HIP_TRY(cdf::fill_int(s, info, 1, 0));
            CDF_HIP_TRY(cdf::convert_d2s(s, n, n, A, lda, w.W, n, chol));
            if (sigma > 0.0) {
                hipLaunchKernelGGL(shift_diag_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, A, lda, w.W, n, sigma);
                CDF_HIP_TRY(hipGetLastError());
            }
            if (chol) CDF_HIP_TRY(mixed_potrf(h, fmt, n, w.W, n, w, nb, info));
            else CDF_HIP_TRY(mixed_getrf(h, fmt, n, w.W, n, w.ipiv, w, nb, info));
            CDF_HIP_TRY(cdf::convert_s2d(s, n, n, w.W, n, w.Wd, n, chol));
        }
        if (w.Tinv) {  // L^T beside L, and the inverted diagonal blocks, for the solves
            CDF_HIP_TRY(cdf::symmetrize_lower(s, n, w.Wd, n));
            CDF_HIP_TRY(cdf::inv_lower_blocks(s, n, w.Wd, n, kInvBs, w.Tinv));
        }
        ++rep.factorizations;
        rep.shift = sigma;
        CDF_HIP_TRY(hipMemcpyAsync(hinfo, info, sizeof(int), hipMemcpyDeviceToHost, s));
        CDF_HIP_TRY(hipStreamSynchronize(s));
        return CDF_OK;
    };
    int hinfo = 0;
    double anorm = 0.0;
    if ((st = factor(0.0, &hinfo)) != CDF_OK) return st;
    CDF_HIP_TRY(hipMemcpyAsync(&anorm, w.red, sizeof(double), hipMemcpyDeviceToHost, s));
    CDF_HIP_TRY(hipStreamSynchronize(s));
    *iters = 0;
    *resid = INFINITY;
    if (hinfo == CDF_INFO_TIMEOUT) return CDF_ERR_TIMEOUT;
    auto tri = [&](cdf::TrsmKind kind, double *Y, int ldy) -> hipError_t {
        return nrhs <= 4 ? cdf::trsv_blocked(s, kind, n, nrhs, w.Wd, n, Y, ldy, w.tsync)
                         : cdf::trsm_blocked(s, kind, n, nrhs, w.Wd, n, Y, ldy);
    };
    auto solve = [&](double *Y, int ldy) -> hipError_t {
        if (chol && w.Tinv) {  // Y <- L^-T L^-1 Y through the inverted diagonal blocks
            CDF_HIP_RET(cdf::trsm_inv_lower(s, false, n, nrhs, w.Wd, n, w.Tinv, kInvBs, Y, ldy, w.Yv, n));
            return cdf::trsm_inv_lower(s, true, n, nrhs, w.Wd, n, w.Tinv, kInvBs, w.Yv, n, Y, ldy);
        }
        if (chol) {
            CDF_HIP_RET(tri(cdf::TRSM_LLNN, Y, ldy));
            return tri(cdf::TRSM_LLTN, Y, ldy);
        }
        CDF_HIP_RET(cdf::laswp(s, 0, nrhs, Y, ldy, w.ipiv, 0, n, n));
        CDF_HIP_RET(tri(cdf::TRSM_LLNU, Y, ldy));
        return tri(cdf::TRSM_LUNN, Y, ldy);
    };
    std::vector<double> norms(3 * nrhs);
    double *nrm = w.red + 1;
    // per-column inf-norms of (R, X, B) into nrm and the HPL scaled residual
    auto scaled = [&](const double *Rm, double *res) -> cdf_status_t {
        hipLaunchKernelGGL(zero_d_kernel, dim3((3 * nrhs + 255) / 256), dim3(256), 0, s, nrm, 3 * nrhs);
        const int gb = (n + 255) / 256 < 64 ? (n + 255) / 256 : 64;
        hipLaunchKernelGGL(col_absmax_kernel, dim3(gb, nrhs), dim3(256), 0, s, n, Rm, n, nrm, 0);
        hipLaunchKernelGGL(col_absmax_kernel, dim3(gb, nrhs), dim3(256), 0, s, n, X, ldx, nrm, 1);
        hipLaunchKernelGGL(col_absmax_kernel, dim3(gb, nrhs), dim3(256), 0, s, n, B, ldb, nrm, 2);
        CDF_HIP_TRY(hipGetLastError());
        CDF_HIP_TRY(hipMemcpyAsync(norms.data(), nrm, 3 * nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
        CDF_HIP_TRY(hipStreamSynchronize(s));
        *res = hpl_from_norms(norms, nrhs, anorm, n);
        return CDF_OK;
    };
    // R = B - A X (binary64, original A)
    auto residual = [&](double *Rm) -> hipError_t {
        if (nrhs <= 4) {
            hipLaunchKernelGGL(residual_gemv_kernel, dim3((n + 63) / 64), dim3(256), 0, s, n, nrhs, Ares, ldres, X, ldx,
                               B, ldb, Rm, n);
            return hipGetLastError();
        }
        CDF_HIP_RET(cdf::copy_cols(s, n, nrhs, B, ldb, Rm, n));
        return cdf::dgemm(s, 0, 0, n, nrhs, n, -1.0, Ares, ldres, X, ldx, 1.0, Rm, n, false);
    };
    bool need_pcg = false;
    if (hinfo == 0 && mode != 2) {
        // classical refinement: x0 = solve(b); r = b - A x; x += solve(r)
        rep.method = CDF_REFINE_CLASSICAL;
        CDF_HIP_TRY(cdf::copy_cols(s, n, nrhs, B, ldb, X, ldx));
        CDF_HIP_TRY(solve(X, ldx));
        std::vector<double> hist;
        for (int it = 0;; ++it) {
            CDF_HIP_TRY(residual(w.R));
            double res = 0.0;
            if ((st = scaled(w.R, &res)) != CDF_OK) return st;
            hist.push_back(res);
            *iters = it;
            *resid = res;
            rep.corrections = it;
            if (res <= 16.0) return CDF_OK;
            const size_t q = hist.size();
            const bool stagnated = q > 3 && res > 0.5 * hist[q - 4];
            // auto: after three corrections without reaching the target, the
            // SPD solver continues with PCG on the same factor
            if (mode == 0 && it >= 3) { need_pcg = true; break; }
            if (it >= max_iter || stagnated) return CDF_ERR_NOT_CONVERGED;
            CDF_HIP_TRY(solve(w.R, n));
            CDF_HIP_TRY(cdf::axpy_cols(s, n, nrhs, w.R, n, X, ldx));
        }
    } else if (hinfo != 0 && mode == 1) {
        return CDF_ERR_NOT_CONVERGED;  // the factorization broke down (info > 0)
    }
    if (!chol || mode == 1) return CDF_ERR_NOT_CONVERGED;
    // ---- SPD fallback: shifted low-precision Cholesky as the preconditioner
    // of binary64 PCG.  On breakdown, A + sigma diag(A) is factored for
    // sigma = u, 4u, 16u, ... (u: the format's unit roundoff).
    bool fresh_x = !need_pcg;
    if (hinfo != 0) {
        double sigma = unit_roundoff(fmt);
        for (int a = 0; a < kMaxShifts && hinfo != 0; ++a, sigma *= 4.0)
            if ((st = factor(sigma, &hinfo)) != CDF_OK) return st;
        if (hinfo == CDF_INFO_TIMEOUT) return CDF_ERR_TIMEOUT;
        if (hinfo != 0) return CDF_ERR_NOT_CONVERGED;
        fresh_x = true;
    }
    rep.method = CDF_REFINE_PCG;
    if (fresh_x) {  // x0 = M^-1 b
        CDF_HIP_TRY(cdf::copy_cols(s, n, nrhs, B, ldb, X, ldx));
        CDF_HIP_TRY(solve(X, ldx));
    }
    double *rho[2] = {w.scal, w.scal + nrhs};
    double *pq = w.scal + 2 * nrhs;
    const dim3 eg((n + 255) / 256, nrhs);
    auto dot = [&](const double *x, const double *y, double *out) -> hipError_t {
        hipLaunchKernelGGL(dot_partial_kernel, dim3(kDotBlocks, nrhs), dim3(256), 0, s, n, x, n, y, n, w.part);
        hipLaunchKernelGGL(dot_finish_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, s, nrhs, w.part, out);
        return hipGetLastError();
    };
    // r = b - A x; stop if converged already; z = M^-1 r; p = z; rho = r.z
    CDF_HIP_TRY(residual(w.R));
    double res = 0.0;
    if ((st = scaled(w.R, &res)) != CDF_OK) return st;
    *resid = res;
    if (res <= 16.0) return CDF_OK;
    CDF_HIP_TRY(cdf::copy_cols(s, n, nrhs, w.R, n, w.Z, n));
    CDF_HIP_TRY(solve(w.Z, n));
    CDF_HIP_TRY(cdf::copy_cols(s, n, nrhs, w.Z, n, w.Pv, n));
    CDF_HIP_TRY(dot(w.R, w.Z, rho[0]));
    for (int it = 1; it <= pcg_max; ++it) {
        double *rho_old = rho[(it + 1) & 1], *rho_new = rho[it & 1];
        // q = A p; alpha = rho / p.q; x += alpha p; r -= alpha q
        CDF_HIP_TRY(cdf::dgemm(s, 0, 0, n, nrhs, n, 1.0, Ares, ldres, w.Pv, n, 0.0, w.Q, n, false));
        CDF_HIP_TRY(dot(w.Pv, w.Q, pq));
        hipLaunchKernelGGL(pcg_xr_kernel, eg, dim3(256), 0, s, n, nrhs, rho_old, pq, w.Pv, w.Q, X, ldx, w.R);
        CDF_HIP_TRY(hipGetLastError());
        rep.pcg_iterations = it;
        *iters = rep.corrections + it;
        // the recurrence's residual estimates the scaled residual; once it is
        // below the target, the true residual b - A x decides
        double est = 0.0;
        if ((st = scaled(w.R, &est)) != CDF_OK) return st;
        if (!(est == est)) return CDF_ERR_NOT_CONVERGED;  // NaN
        *resid = est;
        if (est <= 16.0) {
            CDF_HIP_TRY(residual(w.Q));  // Q is free until the next A p
            if ((st = scaled(w.Q, &res)) != CDF_OK) return st;
            *resid = res;
            if (res <= 16.0) return CDF_OK;
        }
        // z = M^-1 r; rho' = r.z; p = z + (rho' / rho) p
        CDF_HIP_TRY(cdf::copy_cols(s, n, nrhs, w.R, n, w.Z, n));
        CDF_HIP_TRY(solve(w.Z, n));
        CDF_HIP_TRY(dot(w.R, w.Z, rho_new));
        hipLaunchKernelGGL(pcg_p_kernel, eg, dim3(256), 0, s, n, nrhs, rho_new, rho_old, w.Z, w.Pv);
        CDF_HIP_TRY(hipGetLastError());
    }
    return CDF_ERR_NOT_CONVERGED;
}

cdf_status_t check_mixed_args(cdf_handle_t h, cdf_update_prec_t p, int n, int nrhs, const double *A, int lda,
                              const double *B, int ldb, double *X, int ldx, int max_iter, int *iters, double *resid,
                              int *info) {
    h->bad_arg = 0;
    auto bad = [&](int pos) { h->bad_arg = pos; return CDF_ERR_INVALID_ARG; };
    if ((int)p < 0 || (int)p > 3) return bad(2);
    if (n < 0) return bad(3);
    if (nrhs < 0) return bad(4);
    if (lda < (n > 1 ? n : 1)) return bad(6);
    if (ldb < (n > 1 ? n : 1)) return bad(8);
    if (ldx < (n > 1 ? n : 1)) return bad(10);
    if (max_iter < 0) return bad(11);
    if (!iters) return bad(12);
    if (!resid) return bad(13);
    if (!info) return bad(14);
    if (n > 0 && !A) return bad(5);
    if (n > 0 && nrhs > 0 && !B) return bad(7);
    if (n > 0 && nrhs > 0 && !X) return bad(9);
    return CDF_OK;
}

}  // namespace

extern "C" {

cdf_status_t cdf_dgesv_mixed(cdf_handle_t h, cdf_update_prec_t p, int n, int nrhs, const double *A, int lda,
                             const double *B, int ldb, double *X, int ldx, int max_iter, int *iters,
                             double *scaled_resid, int *info) {
    if (!h) return CDF_ERR_INVALID_ARG;
    cdf_status_t st = check_mixed_args(h, p, n, nrhs, A, lda, B, ldb, X, ldx, max_iter, iters, scaled_resid, info);
    if (st != CDF_OK) return st;
    if (n == 0 || nrhs == 0) {
        *iters = 0;
        *scaled_resid = 0.0;
        CDF_HIP_TRY(cdf::fill_int(h->stream, info, 1, 0));
        return CDF_OK;
    }
    return mixed_solve(h, (int)p, false, n, nrhs, A, lda, B, ldb, X, ldx, max_iter, iters, scaled_resid, info);
}

cdf_status_t cdf_dposv_mixed(cdf_handle_t h, cdf_update_prec_t p, int n, int nrhs, const double *A, int lda,
                             const double *B, int ldb, double *X, int ldx, int max_iter, int *iters,
                             double *scaled_resid, int *info) {
    if (!h) return CDF_ERR_INVALID_ARG;
    cdf_status_t st = check_mixed_args(h, p, n, nrhs, A, lda, B, ldb, X, ldx, max_iter, iters, scaled_resid, info);
    if (st != CDF_OK) return st;
    if (n == 0 || nrhs == 0) {
        *iters = 0;
        *scaled_resid = 0.0;
        CDF_HIP_TRY(cdf::fill_int(h->stream, info, 1, 0));
        return CDF_OK;
    }
    return mixed_solve(h, (int)p, true, n, nrhs, A, lda, B, ldb, X, ldx, max_iter, iters, scaled_resid, info);
}

cdf_status_t cdf_sgetrf_mixed(cdf_handle_t h, cdf_update_prec_t p, int n, const double *A, int lda, float *W, int ldw,
                              int *ipiv, int *info) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->bad_arg = 0;
    auto bad = [&](int pos) { h->bad_arg = pos; return CDF_ERR_INVALID_ARG; };
    if ((int)p < 1 || (int)p > 3) return bad(2);
    if (n < 0) return bad(3);
    if (lda < (n > 1 ? n : 1)) return bad(5);
    if (ldw < (n > 1 ? n : 1)) return bad(7);
    if (!info) return bad(9);
    if (n == 0) { CDF_HIP_TRY(cdf::fill_int(h->stream, info, 1, 0)); return CDF_OK; }
    if (!A) return bad(4);
    if (!W) return bad(6);
    if (!ipiv) return bad(8);
    MixedWs w;
    const int nb = mixed_nb(h, n);
    cdf_status_t st = mixed_layout(h, n, 1, nb, (int)p, false, w, true);
    if (st != CDF_OK) return st;
    CDF_HIP_TRY(cdf::fill_int(h->stream, info, 1, 0));
    CDF_HIP_TRY(cdf::convert_d2s(h->stream, n, n, A, lda, W, ldw, false));
    CDF_HIP_TRY(mixed_getrf(h, (int)p, n, W, ldw, ipiv, w, nb, info));
    return CDF_OK;
}

cdf_status_t cdf_spotrf_mixed(cdf_handle_t h, cdf_update_prec_t p, char uplo, int n, const double *A, int lda,
                              float *W, int ldw, int *info) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->bad_arg = 0;
    auto bad = [&](int pos) { h->bad_arg = pos; return CDF_ERR_INVALID_ARG; };
    if ((int)p < 1 || (int)p > 3) return bad(2);
    if (uplo != 'L' && uplo != 'l') {
        if (uplo == 'U' || uplo == 'u') return CDF_ERR_UNSUPPORTED;
        return bad(3);
    }
    if (n < 0) return bad(4);
    if (lda < (n > 1 ? n : 1)) return bad(6);
    if (ldw < (n > 1 ? n : 1)) return bad(8);
    if (!info) return bad(9);
    if (n == 0) { CDF_HIP_TRY(cdf::fill_int(h->stream, info, 1, 0)); return CDF_OK; }
    if (!A) return bad(5);
    if (!W) return bad(7);
    MixedWs w;
    const int nb = mixed_nb(h, n);
    cdf_status_t st = mixed_layout(h, n, 1, nb, (int)p, true, w, true);
    if (st != CDF_OK) return st;
    CDF_HIP_TRY(cdf::fill_int(h->stream, info, 1, 0));
    CDF_HIP_TRY(cdf::convert_d2s(h->stream, n, n, A, lda, W, ldw, true));
    CDF_HIP_TRY(mixed_potrf(h, (int)p, n, W, ldw, w, nb, info));
    return CDF_OK;
}

cdf_status_t cdf_quantize(cdf_handle_t h, cdf_update_prec_t p, int m, int n, const float *X, int ldx, int tm, int tn,
                          void *Q, int ldq, int *exps) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->bad_arg = 0;
    auto bad = [&](int pos) { h->bad_arg = pos; return CDF_ERR_INVALID_ARG; };
    if ((int)p < 1 || (int)p > 3) return bad(2);
    if (m < 0) return bad(3);
    if (n < 0) return bad(4);
    if (ldx < (m > 1 ? m : 1)) return bad(6);
    if (tm <= 0) return bad(7);
    if (tn <= 0) return bad(8);
    if (ldq < (m > 1 ? m : 1)) return bad(10);
    if (m == 0 || n == 0) return CDF_OK;
    if (!X) return bad(5);
    if (!Q) return bad(9);
    if (!exps) return bad(11);
    CDF_HIP_TRY(cdf::quantize(h->stream, (int)p, m, n, X, ldx, tm, tn, Q, ldq, exps, false));
    return CDF_OK;
}

cdf_status_t cdf_lowp_update(cdf_handle_t h, cdf_update_prec_t p, int m, int n, int k, const void *QA, int lda,
                             const int *ea, const void *QB, int ldb, const int *eb, float *C, int ldc) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->bad_arg = 0;
    auto bad = [&](int pos) { h->bad_arg = pos; return CDF_ERR_INVALID_ARG; };
    if ((int)p < 1 || (int)p > 3) return bad(2);
    if (m < 0) return bad(3);
    if (n < 0) return bad(4);
    if (k < 0) return bad(5);
    if (lda < kpad_of(k) || lda % KSTEP) return bad(7);
    if (ldb < kpad_of(k) || ldb % KSTEP) return bad(10);
    if (ldc < (m > 1 ? m : 1)) return bad(13);
    if (m == 0 || n == 0 || k == 0) return CDF_OK;
    if (!QA || (reinterpret_cast<uintptr_t>(QA) & 15)) return bad(6);
    if (!ea) return bad(8);
    if (!QB || (reinterpret_cast<uintptr_t>(QB) & 15)) return bad(9);
    if (!eb) return bad(11);
    if (!C) return bad(12);
    CDF_HIP_TRY(cdf::lowp_update(h->stream, (int)p, m, n, k, QA, lda, ea, QB, ldb, eb, C, ldc, false, nullptr));
    return CDF_OK;
}

int cdf_update_tile(cdf_update_prec_t) { return QT; }

}  // extern "C"
