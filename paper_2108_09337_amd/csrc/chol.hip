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

// One workgroup of 256 threads; the block's lower triangle lives in
// registers: thread (wave w, lane l) owns rows l and l + 64 of columns
// j = w + 4q (q < 32).  Column k (k = 4 kq + kw): its diagonal owner
// publishes d = L(k,k); every thread checks d > 0 (S1's domain); the owners
// of column k form sqrt(d) (S1) and the scaled column (S2, division) and
// publish it in LDS (double-buffered by parity); every thread then updates
// its elements right of column k (S3) from the published column.  Two
// barriers per column.
__global__ __launch_bounds__(NT) void potrf_diag_kernel(int n, double *__restrict__ A, int lda,
                                                        int *__restrict__ info, int info_base) {
    if (*info != 0) return;
    __shared__ double sc[2][MAXN];
    __shared__ double sd;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    double a[2][32];
    cdf::static_for<0, 2>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        cdf::static_for<0, 32>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const int i = lane + 64 * r, j = w + 4 * q;
            a[r][q] = (i < n && j < n && i >= j) ? A[(size_t)i + (size_t)j * lda] : 0.0;
        });
    });
    int fail = 0;  // uniform: every thread reads the same published diagonal
    cdf::static_for<0, 32>([&](auto kqc) {
        constexpr int kq = decltype(kqc)::value;
        for (int kw = 0; kw < 4; ++kw) {
            const int k = 4 * kq + kw;
            if (fail || k >= n) continue;
            const int par = k & 1;
            const bool own = (w == kw);
            if (own && lane == (k & 63)) sd = a[kq >> 4][kq];
            __syncthreads();
            const double d = sd;
            if (!(d > 0.0)) {
                fail = k + 1;
                continue;
            }
            if (own) {
                const double lkk = sqrt(d);
                cdf::static_for<0, 2>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    const int i = lane + 64 * r;
                    if (i >= k && i < n) {
                        const double v = i == k ? lkk : a[r][kq] / lkk;
                        a[r][kq] = v;
                        sc[par][i - k] = v;
                    }
                });
            }
            __syncthreads();
            // S3 on the elements right of column k: j = w + 4q > k
            const int i0 = lane, i1 = lane + 64;
            const double l0 = (i0 > k && i0 < n) ? sc[par][i0 - k] : 0.0;
            const double l1 = (i1 > k && i1 < n) ? sc[par][i1 - k] : 0.0;
            cdf::static_for<kq, 32>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                const int j = w + 4 * q;
                if (j > k && j < n) {
                    const double lj = sc[par][j - k];
                    if (i0 >= j) a[0][q] = fma(-l0, lj, a[0][q]);
                    if (i1 >= j && i1 < n) a[1][q] = fma(-l1, lj, a[1][q]);
                }
            });
        }
    });
    cdf::static_for<0, 2>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        cdf::static_for<0, 32>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const int i = lane + 64 * r, j = w + 4 * q;
            if (i < n && j < n && i >= j) A[(size_t)i + (size_t)j * lda] = a[r][q];
        });
    });
    if (t == 0 && fail) *info = info_base + fail;
}

// Blocks of at most 64 columns beside the low-precision SYRK (the mixed
// Cholesky's panel, on the critical path there): one wave at raised issue
// priority, lane i holding row i of the block in registers.  Column k: the diagonal and the
// later rows of column k are read from their lanes (readlane), so no LDS
// and no barrier; the same operations in the same order as above (S1, S2
// by division, S3 as fma(-L(i,k), L(j,k), a(i,j)) over j > k).  Elements
// above the diagonal are updated too (their lanes simply compute with
// them) but never read or stored.
__device__ __forceinline__ double lane_value(double v, int l) {
    const long long x = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)x, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(x >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// (Beside the binary64 update, where the panel is not critical, the
// four-wave kernel above measured faster: 183 against 238 us per block.)
__global__ __launch_bounds__(64) void potrf64_kernel(int n, double *__restrict__ A, int lda, int *__restrict__ info,
                                                     int info_base) {
    if (*info != 0) return;
    __builtin_amdgcn_s_setprio(2);
    const int i = threadIdx.x;
    double a[64];
    cdf::static_for<0, 64>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        a[j] = (i < n && j < n && i >= j) ? A[(size_t)i + (size_t)j * lda] : 0.0;
    });
    int fail = 0;  // uniform
    cdf::static_for<0, 64>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        if (k < n && !fail) {
            const double d = lane_value(a[k], k);
            if (!(d > 0.0)) {
                fail = k + 1;
            } else {
                const double lkk = sqrt(d);
                if (i == k) a[k] = lkk;
                else if (i > k) a[k] = a[k] / lkk;
                cdf::static_for<k + 1, 64>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    if (j < n) a[j] = fma(-a[k], lane_value(a[k], j), a[j]);
                    // keep the broadcasts next to their uses (hoisted, they
                    // would exhaust the scalar registers)
                    if constexpr ((j & 7) == 7) __builtin_amdgcn_sched_barrier(0);
                });
            }
        }
    });
    cdf::static_for<0, 64>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (i < n && j < n && i >= j) A[(size_t)i + (size_t)j * lda] = a[j];
    });
    if (i == 0 && fail) *info = info_base + fail;
}

}  // namespace

namespace cdf {

hipError_t potrf_diag(hipStream_t s, int n, double *A, int lda, int *info, int info_base, bool prio) {
    if (n <= 0) return hipSuccess;
    if (n > MAXN) return hipErrorInvalidValue;
    if (n <= 64 && prio)
        hipLaunchKernelGGL(potrf64_kernel, dim3(1), dim3(64), 0, s, n, A, lda, info, info_base);
    else
        hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(NT), 0, s, n, A, lda, info, info_base);
    return hipGetLastError();
}

}  // namespace cdf
