// LU panel factorization with partial pivoting (Sec. 7, routine A00 and the
// column-by-column pivot search that partial pivoting requires, Sec. 7.3)
// and row interchanges: the host side of the panel leaf (its kernel is in
// lu_leaf.h; this file instantiates it for one row per thread,
// lu_leaf_r2.hip for two), and the interchange kernels.
#include "lu_leaf.h"

namespace {

// ---------------------------------------------------------------- interchanges



// Applies interchanges ipiv[k1..k2) (k2 - k1 <= 64) to the ncols columns of
// A, 64 columns per workgroup: all rows moved are read before any is written.
template <typename T>
__global__ __launch_bounds__(256) void laswp_kernel(int ncols, T *__restrict__ A, int lda,
                                                    const int *__restrict__ ipiv, int k1, int k2, int nrows) {
    __shared__ int dst[MAXPAIRS], src[MAXPAIRS];
    __shared__ int s_np;
    if (threadIdx.x < 64) {
        const int np = build_pairs_wave(ipiv, k1, k2, nrows, dst, src);
        if (threadIdx.x == 0) s_np = np;
    }
    __syncthreads();
    const int np = s_np;
    if (np == 0) return;
    const int cbase = blockIdx.x * 64;
    const int total = np * 64;
    constexpr int PER = MAXPAIRS * 64 / 256;
    T v[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int e = threadIdx.x + 256 * r;
        if (e < total) {
            const int q = e % np, c = cbase + e / np;
            if (c < ncols) v[r] = A[(size_t)src[q] + (size_t)c * lda];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int e = threadIdx.x + 256 * r;
        if (e < total) {
            const int q = e % np, c = cbase + e / np;
            if (c < ncols) A[(size_t)dst[q] + (size_t)c * lda] = v[r];
        }
    }
}

template <typename T>
hipError_t laswp_impl(hipStream_t s, int c0, int c1, T *A, int lda, const int *ipiv, int k1, int k2,
                      int nrows) {
    // columns [c0, c1) ; interchanges in chunks of MAXSW
    const int ncols = c1 - c0;
    if (ncols <= 0 || k2 <= k1) return hipSuccess;
    for (int kk = k1; kk < k2; kk += MAXSW) {
        const int ke = min(k2, kk + MAXSW);
        hipLaunchKernelGGL((laswp_kernel<T>), dim3((ncols + 63) / 64), dim3(256), 0, s, ncols,
                           A + (size_t)c0 * lda, lda, ipiv, kk, ke, nrows);
        CDF_HIP_RET(hipGetLastError());
    }
    return hipSuccess;
}


// ------------------------------------------------- panel-wide interchanges

constexpr int PMAX = 512;            // interchanges per panel
constexpr int PPAIRS = 2 * PMAX;

// (dst, src) pairs of the interchanges ipiv[k1..k2) (k2 - k1 <= 512,
// relative to row 0 of the region, 1-based; entries outside [k+1, nrows]
// ignored), simulated by one thread on LDS: positions [k1, k2) in a direct
// array, the other rows touched in an open-addressing hash table.
// pairs[0] = count, pairs[1 + q] = dst row, pairs[1 + PPAIRS + q] = src row.
__global__ __launch_bounds__(256) void pairs_kernel(const int *__restrict__ ipiv, int k1, int k2, int nrows,
                                                    int *__restrict__ pairs) {
    constexpr int HS = 2048;  // at most PMAX rows outside [k1, k2) are touched: load <= 1/4
    __shared__ int blk[PMAX];
    __shared__ int piv[PMAX];
    __shared__ int hkey[HS], hval[HS];
    __shared__ int cnt;
    const int t = threadIdx.x;
    const int nk = k2 - k1;
    for (int i = t; i < HS; i += 256) hkey[i] = -1;
    for (int i = t; i < nk; i += 256) {
        blk[i] = k1 + i;
        const int p = ipiv[k1 + i] - 1;
        piv[i] = (p < k1 + i || p >= nrows) ? k1 + i : p;
    }
    if (t == 0) cnt = 0;
    __syncthreads();
    if (t == 0) {
        for (int j = 0; j < nk; ++j) {
            const int k = k1 + j, p = piv[j];
            if (p == k) continue;
            const int ck = blk[j];
            if (p < k2) {
                blk[j] = blk[p - k1];
                blk[p - k1] = ck;
            } else {
                unsigned hsh = ((unsigned)p * 2654435761u) >> 21;  // 11 bits
                while (hkey[hsh] != -1 && hkey[hsh] != p) hsh = (hsh + 1) & (HS - 1);
                if (hkey[hsh] == -1) { hkey[hsh] = p; hval[hsh] = p; }
                blk[j] = hval[hsh];
                hval[hsh] = ck;
            }
        }
    }
    __syncthreads();
    for (int i = t; i < nk; i += 256)
        if (blk[i] != k1 + i) {
            const int o = atomicAdd(&cnt, 1);
            pairs[1 + o] = k1 + i;
            pairs[1 + PPAIRS + o] = blk[i];
        }
    for (int i = t; i < HS; i += 256)
        if (hkey[i] != -1 && hval[i] != hkey[i]) {
            const int o = atomicAdd(&cnt, 1);
            pairs[1 + o] = hkey[i];
            pairs[1 + PPAIRS + o] = hval[i];
        }
    __syncthreads();
    if (t == 0) pairs[0] = cnt;
}

// Applies prebuilt pairs to columns [0, ncols) of A (rows offset by the
// region base already folded into A): 8 columns per workgroup, every moved
// row read before any is written.
template <typename T>
__global__ __launch_bounds__(256) void apply_pairs_kernel(int ncols, T *__restrict__ A, int lda,
                                                          const int *__restrict__ pairs) {
    constexpr int CW = 8, PER = PPAIRS * CW / 256;
    const int np = pairs[0];
    if (np == 0) return;
    const int cbase = blockIdx.x * CW;
    const int total = np * CW;
    T v[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int e = threadIdx.x + 256 * r;
        const int q = e % np, c = cbase + e / np;
        if (e < total && c < ncols) v[r] = A[(size_t)pairs[1 + PPAIRS + q] + (size_t)c * lda];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int e = threadIdx.x + 256 * r;
        const int q = e % np, c = cbase + e / np;
        if (e < total && c < ncols) A[(size_t)pairs[1 + q] + (size_t)c * lda] = v[r];
    }
}

}  // namespace

static_assert(kExchBytes <= cdf::kTournOffset, "tournament area overlaps the exchange");
static_assert(cdf::kTournOffset + 2 * cdf::kTournMaxSets * 33 * sizeof(int) + 32 * 32 * sizeof(double) <=
                  cdf::kLeafWsBytes - 256,
              "tournament area overlaps the error word");

namespace cdf {

LeafArea handle_leaf_area(cdf_handle_t h) { return LeafArea{h->ws, &h->leaf_epoch}; }

int *leaf_error_word(const LeafArea &la) {
    return reinterpret_cast<int *>(static_cast<char *>(la.base) + kLeafWsBytes - 256);
}

hipError_t leaf_reset_error(const LeafArea &la, hipStream_t stream) {
    return fill_int(stream, leaf_error_word(la), 1, 0);
}

hipError_t lu_leaf(cdf_handle_t h, const LeafArea &la, hipStream_t stream, int m, int n, double *A, int lda,
                   int *ipiv, int row0, int *info, int info_base, int rows_per_thread, double *region,
                   int region_rows, int region_cols, int c0) {
    if (m <= 0 || n <= 0) return hipSuccess;
    if (n > LW || n > m) return hipErrorInvalidValue;
    int R = rows_per_thread;
    // one row per thread whenever the grid fits the CUs: two rows per thread
    // need more registers, so beside the update GEMM the leaf waits longer
    // for all of its workgroups to become resident
    if (R != 1 && R != 2) R = (m + LT - 1) / LT > h->num_cus ? 2 : 1;
    int G = (m + LT * R - 1) / (LT * R);
    if (G > h->num_cus && R == 1) { R = 2; G = (m + LT * R - 1) / (LT * R); }
    if (G > h->num_cus || G > GMAX) return hipErrorInvalidValue;
    const void *fn = R == 1 ? reinterpret_cast<const void *>(&lu_leaf_kernel<1>) : leaf_kernel_r2();
    // The exchange needs all G workgroups resident at once: G must not
    // exceed what the device holds of this kernel alone (at most one per CU
    // is assumed of the CUs, whatever else runs beside it).
    int &occ = h->leaf_occ[R - 1];
    if (occ == 0) {
        int b = 0;
        CDF_HIP_RET(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, LT, 0));
        occ = b > 0 ? b : -1;
    }
    if (occ < 0 || G > h->num_cus * occ) return hipErrorInvalidValue;
    // bounded waits: the wall-clock budget and a poll-count cap
    const long long us = h->params[CDF_PARAM_LEAF_WAIT_US] > 0 ? h->params[CDF_PARAM_LEAF_WAIT_US] : kLeafWaitUsDefault;
    long long budget = us * (long long)h->wall_khz / 1000;
    if (budget < 1) budget = 1;
    const long long cap = us * 64 + 4096;
    unsigned max_polls = cap > 0x7fffffffLL ? 0x7fffffffu : (unsigned)cap;
    unsigned skew = h->params[CDF_PARAM_TEST_EXCHANGE_FAIL] ? 32u : 0u;
    int *err = leaf_error_word(la);
    // Epochs are unique per launch and column; the exchange area (tags and
    // row words) is zeroed on first use of a workspace and on wrap-around,
    // and epochs below 64 are never issued, so no stale word can carry a
    // current epoch.
    unsigned &epoch = *la.epoch;
    if (epoch < 64u || epoch > 0xffffff00u) {
        CDF_HIP_RET(fill_int(stream, static_cast<int *>(la.base), (int)(kExchBytes / sizeof(int)), 0));
        epoch = 64u;
    }
    unsigned e0 = epoch;
    epoch += 64u;
    u64 *tags = static_cast<u64 *>(la.base);
    u64 *rows = reinterpret_cast<u64 *>(static_cast<char *>(la.base) + kTagBytes);
    void *args[] = {&m, &n, &A, &lda, &ipiv, &row0, &info, &info_base, &tags, &rows, &e0, &region, &region_rows,
                    &region_cols, &c0, &err, &budget, &max_polls, &skew};
    const size_t lds = 0;  // the block lives in registers
    // A plain launch: G <= number of CUs and each CU fits a leaf workgroup, so
    // all G become resident at the latest when the (finite) kernels that may
    // run beside it on other streams have drained; the exchange then
    // completes.  (A cooperative launch would forbid that overlap.)  Should
    // residency fail all the same, the bounded waits end every workgroup.
    return hipLaunchKernel(fn, dim3(G), dim3(LT), args, lds, stream);
}

size_t pairs_ints() { return 1 + 2 * PPAIRS; }

hipError_t build_pairs(hipStream_t s, const int *ipiv, int k1, int k2, int nrows, int *pairs) {
    if (k2 - k1 > PMAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pairs_kernel, dim3(1), dim3(256), 0, s, ipiv, k1, k2, nrows, pairs);
    return hipGetLastError();
}

hipError_t apply_pairs(hipStream_t s, int c0, int c1, double *A, int lda, const int *pairs) {
    if (c1 <= c0) return hipSuccess;
    hipLaunchKernelGGL((apply_pairs_kernel<double>), dim3((c1 - c0 + 7) / 8), dim3(256), 0, s, c1 - c0,
                       A + (size_t)c0 * lda, lda, pairs);
    return hipGetLastError();
}

hipError_t apply_pairs(hipStream_t s, int c0, int c1, float *A, int lda, const int *pairs) {
    if (c1 <= c0) return hipSuccess;
    hipLaunchKernelGGL((apply_pairs_kernel<float>), dim3((c1 - c0 + 7) / 8), dim3(256), 0, s, c1 - c0,
                       A + (size_t)c0 * lda, lda, pairs);
    return hipGetLastError();
}

hipError_t laswp(hipStream_t s, int c0, int c1, double *A, int lda, const int *ipiv, int k1, int k2,
                 int nrows) {
    return laswp_impl<double>(s, c0, c1, A, lda, ipiv, k1, k2, nrows);
}

hipError_t slaswp(hipStream_t s, int c0, int c1, float *A, int lda, const int *ipiv, int k1, int k2,
                  int nrows) {
    return laswp_impl<float>(s, c0, c1, A, lda, ipiv, k1, k2, nrows);
}

}  // namespace cdf
