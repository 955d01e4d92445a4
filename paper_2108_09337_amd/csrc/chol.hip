// Cholesky of one diagonal block (Sec. 7.5 / Table 1: potrf of A00), the
// three statements of the Cholesky listing (Sec. 6.2) applied to an n x n
// block (n <= 128) held in LDS by one workgroup:
//   S1: L(k,k) = sqrt(L(k,k));  S2: L(i,k) /= L(k,k);  S3: L(i,j) -= L(i,k) L(j,k)
// A pivot that is not strictly positive (or NaN) stops the block and records
// the LAPACK info.  Only the lower triangle is read or written.
#include "internal.h"

namespace {

constexpr int NT = 256;
constexpr int MAXN = 128;
constexpr int LD = MAXN + 1;

__global__ __launch_bounds__(NT) void potrf_diag_kernel(int n, double *__restrict__ A, int lda,
                                                        int *__restrict__ info, int info_base) {
    if (*info != 0) return;
    extern __shared__ double L[];  // L[i + j * LD]
    __shared__ int fail;
    const int t = threadIdx.x;
    for (int e = t; e < n * n; e += NT) {
        const int i = e % n, j = e / n;
        if (i >= j) L[i + j * LD] = A[(size_t)i + (size_t)j * lda];
    }
    if (t == 0) fail = 0;
    __syncthreads();
    int kdone = n;
    for (int k = 0; k < n; ++k) {
        if (t == 0) {
            const double d = L[k + k * LD];
            if (!(d > 0.0)) fail = k + 1;
            else L[k + k * LD] = sqrt(d);
        }
        __syncthreads();
        if (fail) { kdone = k; break; }
        const double lkk = L[k + k * LD];
        for (int i = k + 1 + t; i < n; i += NT) L[i + k * LD] = L[i + k * LD] / lkk;
        __syncthreads();
        // trailing lower triangle: rows i = k+1+ (t%64) + 64q, columns j = k+1 + t/64 + 4r
        const int r0 = k + 1 + (t & 63), cg = t >> 6;
        for (int j = k + 1 + cg; j < n; j += 4) {
            const double ljk = L[j + k * LD];
            for (int i = r0; i < n; i += 64)
                if (i >= j) L[i + j * LD] = fma(-L[i + k * LD], ljk, L[i + j * LD]);
        }
        __syncthreads();
    }
    (void)kdone;
    for (int e = t; e < n * n; e += NT) {
        const int i = e % n, j = e / n;
        if (i >= j) A[(size_t)i + (size_t)j * lda] = L[i + j * LD];
    }
    if (t == 0 && fail) *info = info_base + fail;
}

}  // namespace

namespace cdf {

hipError_t potrf_diag(hipStream_t s, int n, double *A, int lda, int *info, int info_base) {
    if (n <= 0) return hipSuccess;
    if (n > MAXN) return hipErrorInvalidValue;
    static bool attr = false;
    if (!attr) {
        CDF_HIP_RET(hipFuncSetAttribute(reinterpret_cast<const void *>(&potrf_diag_kernel),
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        MAXN * LD * sizeof(double)));
        attr = true;
    }
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(NT), (size_t)n * LD * sizeof(double), s, n, A, lda, info,
                       info_base);
    return hipGetLastError();
}

}  // namespace cdf
