// Triangular solves with many right-hand sides through inverted diagonal
// blocks (the solves of the SPD solver's refinement and of its
// preconditioned CG, where the same factor is applied many times).
//
// Substitution (trsm_blocked) spends its time in the diagonal blocks: one
// barrier per row for a handful of workgroups.  Here the diagonal blocks of
// the lower factor L are inverted once per factorization, all blocks in one
// launch, and every solve is a chain of matrix products on the FP64 matrix
// cores: for a lower block k, y_k = L_kk^-1 x_k, then x_{>k} -= L_{>k,k} y_k.
// The backward solve with L^T uses the transpose of L stored in the upper
// triangle of the same array (filled by symmetrize_lower), so its updates are
// plain (not transposed) products as well; its diagonal blocks are the
// transposes of the same inverses.
#include "internal.h"

namespace {

constexpr int NT = 256;
constexpr int IC = 16;         // columns of the inverse per workgroup
constexpr int IPAD = IC + 1;

// Tinv block q (bs x bs, leading dimension bs, at Tinv + q * bs * bs) =
// L_qq^-1 for the diagonal block q of the lower, non-unit triangle T
// (kb = min(bs, n - q bs) rows; the rest of the block is left as it is).
// Workgroup (x, q) solves L_qq X = I for columns [16x, 16x + 16) by forward
// substitution in LDS, starting at its first column (X is lower
// triangular, so rows above the column stay zero).
__global__ __launch_bounds__(NT) void inv_lower_blocks_kernel(int n, int bs, const double *__restrict__ T, int ldt,
                                                              double *__restrict__ Tinv) {
    extern __shared__ double X[];  // X[r * IPAD + c], r < kb
    const int q = blockIdx.y;
    const int r0 = q * bs;
    const int kb = min(bs, n - r0);
    const int c0 = blockIdx.x * IC;
    if (c0 >= kb) return;
    const double *L = T + (size_t)r0 + (size_t)r0 * ldt;
    double *Y = Tinv + (size_t)q * bs * bs;
    const int t = threadIdx.x;
    const int c = t % IC, rg = t / IC;
    constexpr int RG = NT / IC;
    for (int e = t; e < kb * IC; e += NT) {
        const int r = e / IC, cc = e % IC;
        X[r * IPAD + cc] = (r == c0 + cc) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = c0; j < kb; ++j) {
        if (rg == j % RG) X[j * IPAD + c] = X[j * IPAD + c] / L[(size_t)j + (size_t)j * ldt];
        __syncthreads();
        const double xj = X[j * IPAD + c];
        for (int i = j + 1 + ((rg - (j + 1)) % RG + RG) % RG; i < kb; i += RG)
            X[i * IPAD + c] = fma(-L[(size_t)i + (size_t)j * ldt], xj, X[i * IPAD + c]);
        __syncthreads();
    }
    for (int e = t; e < kb * IC; e += NT) {
        const int r = e % kb, cc = e / kb;
        if (c0 + cc < kb) Y[(size_t)r + (size_t)(c0 + cc) * bs] = X[r * IPAD + cc];
    }
}

// a(j, i) = a(i, j) for i > j: the strict upper triangle receives the
// transpose of the strict lower one, through 64 x 64 LDS tiles (coalesced
// reads and writes).  Workgroup (bi, bj) with bi >= bj moves tile (bi, bj).
__global__ __launch_bounds__(NT) void symmetrize_tiled_kernel(int n, double *__restrict__ a, int lda) {
    __shared__ double tile[64][65];
    const int bi = blockIdx.x, bj = blockIdx.y;
    if (bi < bj) return;
    const int i0 = bi * 64, j0 = bj * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int jj = ty; jj < 64; jj += 4) {
        const int i = i0 + tx, j = j0 + jj;
        if (i < n && j < n) tile[jj][tx] = a[(size_t)i + (size_t)j * lda];
    }
    __syncthreads();
    // element (i0 + x, j0 + y) goes to (j0 + y, i0 + x): column i0 + x, row j0 + y
    for (int xx = ty; xx < 64; xx += 4) {
        const int col = i0 + xx, row = j0 + tx;
        if (col < n && row < n && col > row) a[(size_t)row + (size_t)col * lda] = tile[tx][xx];
    }
}

}  // namespace

namespace cdf {

size_t inv_blocks_doubles(int n, int bs) { return (size_t)((n + bs - 1) / bs) * bs * bs; }

hipError_t symmetrize_lower(hipStream_t s, int n, double *A, int lda) {
    if (n <= 1) return hipSuccess;
    const int tiles = (n + 63) / 64;
    hipLaunchKernelGGL(symmetrize_tiled_kernel, dim3(tiles, tiles), dim3(NT), 0, s, n, A, lda);
    return hipGetLastError();
}

hipError_t inv_lower_blocks(hipStream_t s, int n, const double *T, int ldt, int bs, double *Tinv) {
    if (n <= 0) return hipSuccess;
    if (bs <= 0 || bs > 512) return hipErrorInvalidValue;
    const size_t lds = (size_t)bs * IPAD * sizeof(double);
    // dynamic LDS above 64 KB needs the kernel attribute (bs = 512: 68 KB);
    // set once (thread-safe static initialization)
    static const hipError_t attr =
        hipFuncSetAttribute(reinterpret_cast<const void *>(&inv_lower_blocks_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 512 * IPAD * (int)sizeof(double));
    CDF_HIP_RET(attr);
    const int nblk = (n + bs - 1) / bs;
    hipLaunchKernelGGL(inv_lower_blocks_kernel, dim3((bs + IC - 1) / IC, nblk), dim3(NT), lds, s, n, bs, T, ldt,
                       Tinv);
    return hipGetLastError();
}

hipError_t trsm_inv_lower(hipStream_t s, bool transposed, int n, int nrhs, const double *T, int ldt,
                          const double *Tinv, int bs, double *X, int ldx, double *Y, int ldy) {
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    const int nblk = (n + bs - 1) / bs;
    if (!transposed) {
        // L y = x: y_k = L_kk^-1 x_k, then x_{>k} -= L_{>k,k} y_k
        for (int q = 0; q < nblk; ++q) {
            const int k = q * bs, kb = min(bs, n - k);
            CDF_HIP_RET(dgemm(s, 0, 0, kb, nrhs, kb, 1.0, Tinv + (size_t)q * bs * bs, bs, X + k, ldx, 0.0, Y + k, ldy,
                              false));
            if (k + kb < n)
                CDF_HIP_RET(dgemm(s, 0, 0, n - k - kb, nrhs, kb, -1.0, T + (k + kb) + (size_t)k * ldt, ldt, Y + k, ldy,
                                  1.0, X + k + kb, ldx, false));
        }
        return hipSuccess;
    }
    // L^T y = x with U = L^T in the strict upper triangle of T (and L's
    // diagonal): y_k = (L_kk^-1)^T x_k, then x_{<k} -= U_{<k,k} y_k
    for (int q = nblk - 1; q >= 0; --q) {
        const int k = q * bs, kb = min(bs, n - k);
        CDF_HIP_RET(dgemm(s, 1, 0, kb, nrhs, kb, 1.0, Tinv + (size_t)q * bs * bs, bs, X + k, ldx, 0.0, Y + k, ldy,
                          false));
        if (k > 0)
            CDF_HIP_RET(dgemm(s, 0, 0, k, nrhs, kb, -1.0, T + (size_t)k * ldt, ldt, Y + k, ldy, 1.0, X, ldx, false));
    }
    return hipSuccess;
}

}  // namespace cdf
