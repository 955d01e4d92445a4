// Tournament pivoting for an LU panel leaf (Sec. 7.3, "Tournament Pivoting"
// and "Pivoting in COnfLUX"; Table 1, row "pivoting"), the alternative to the
// leaf's column-by-column pivot search for the mixed-precision LU.
//
// A leaf of w <= 32 columns over M rows picks its w pivot rows in rounds
// instead of with one grid-wide exchange per column:
//   1. every block of `block` consecutive rows (one workgroup, one row per
//      thread) runs LU with partial pivoting on its rows' w columns and keeps
//      the rows it brings to the top (its candidates, in pivot order);
//   2. round by round, `fanin` candidate sets at a time are stacked in order
//      and a workgroup runs the same local LU on their original rows, keeping
//      w; the round with a single set left is the final one, and its local LU
//      is also the factorization L00 U00 of the chosen rows in pivot order;
//   3. one thread turns the pivot order into LAPACK interchanges, which are
//      applied to every column of the region (the leaf's own columns too);
//   4. the leaf's rows are then written without further interchanges: the
//      top w rows from L00 U00, every lower row as the solution l of
//      l U00 = a (its multipliers), one row per thread.
// Between the rounds the kernel boundaries order the candidate sets, so the
// leaf has no grid-wide wait.  Zero pivots: recorded in info, the column's
// multipliers left unscaled, as the partial-pivoting leaf does.
#include "internal.h"
#include "wave.h"

#include <climits>

namespace {

constexpr int TW = 32;   // leaf width
constexpr int TN = 256;  // threads per node workgroup (rows per node, at most)
constexpr int TNW = TN / 64;
constexpr int SET = 1 + TW;  // a candidate set: count, then row ids

struct __align__(16) TSlot {
    u64 key;
    int idx, pad;
};

// One node of the tournament: the rows of the node (level 0: rows
// [node * block, +block) of the leaf; later levels: the candidate sets
// [node * fanin, +fanin) of `in`, stacked in order) are loaded with their
// original values (thread t: stacked row t), factored with partial pivoting
// for min(w, rows) steps, and the ids then at the top are written to
// out[node] in pivot order.  The node of a one-node launch (the final round)
// also writes its factored top w x w block to F (row-major by pivot order:
// F[j * TW + c]).
__global__ __launch_bounds__(TN) void tourn_node_kernel(int M, int w, const double *__restrict__ A, int lda,
                                                        int level0, int block, const int *__restrict__ in,
                                                        int nin, int fanin, int *__restrict__ out,
                                                        double *__restrict__ F) {
    __shared__ double cand[2][TNW][TW];
    __shared__ double rowj[2][TW];
    __shared__ TSlot ws[2][TNW];
    __shared__ int ids[TN];
    __shared__ int s_rows;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int node = blockIdx.x;
    if (t == 0) {
        int r = 0;
        if (level0) {
            const int r0 = node * block;
            r = min(block, M - r0);
        } else {
            for (int s = node * fanin; s < min(nin, node * fanin + fanin); ++s) r += in[s * SET];
        }
        s_rows = r;
    }
    __syncthreads();
    const int rows = s_rows;
    // stacked row ids
    if (level0) {
        if (t < rows) ids[t] = node * block + t;
    } else if (t < 64) {
        int base = 0;
        for (int s = node * fanin; s < min(nin, node * fanin + fanin); ++s) {
            const int c = in[s * SET];
            if (lane < c) ids[base + lane] = in[s * SET + 1 + lane];
            base += c;
        }
    }
    __syncthreads();
    int rid = t < rows ? ids[t] : -1;
    double x[TW];
    cdf::static_for<0, TW>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        const bool ok = rid >= 0 && c < w;
        const double v = A[ok ? (size_t)rid + (size_t)c * lda : 0];
        x[c] = ok ? v : 0.0;
    });
    const int k = min(w, rows);
    const bool wact = wave * 64 < rows;
    if (!wact && lane == 0) ws[0][wave] = ws[1][wave] = TSlot{0ull, INT_MAX, 0};
    __shared__ int rid_slot[2][TNW];
    __shared__ int ridj[2];
    cdf::static_for<0, TW>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (j >= k) return;
        const int par = j & 1;
        if (wact) {
            const u64 key = (t >= j && t < rows) ? pivot_key(x[j]) : 0ull;
            const u64 wk = wave_max_key(key);
            const u64 hit = __ballot(key == wk && wk != 0ull);
            const int bi = hit ? (t & ~63) + __builtin_ctzll(hit) : INT_MAX;
            if (t == bi) {
                cdf::static_for<0, TW>([&](auto cc) { cand[par][wave][decltype(cc)::value] = x[decltype(cc)::value]; });
                rid_slot[par][wave] = rid;
            }
            if (t == j) {
                cdf::static_for<0, TW>([&](auto cc) { rowj[par][decltype(cc)::value] = x[decltype(cc)::value]; });
                ridj[par] = rid;
            }
            if (lane == 0) ws[par][wave] = TSlot{wk, bi, 0};
        }
        __syncthreads();
        if (!wact) return;
        TSlot sl[TNW];
#pragma unroll
        for (int q = 0; q < TNW; ++q) sl[q] = ws[par][q];
        u64 v = sl[0].key;
        int p = sl[0].idx, wsel = 0;
#pragma unroll
        for (int q = 1; q < TNW; ++q) {
            const bool gt = sl[q].key > v;
            v = gt ? sl[q].key : v;
            p = gt ? sl[q].idx : p;
            wsel = gt ? q : wsel;
        }
        const double *prow = p == INT_MAX ? rowj[par] : cand[par][wsel];
        const int prid = p == INT_MAX ? ridj[par] : rid_slot[par][wsel];
        if (p == INT_MAX) p = j;  // no ordered candidate: no interchange
        const double piv = prow[j];
        if (t == j) {
            cdf::static_for<0, TW>([&](auto cc) { x[decltype(cc)::value] = prow[decltype(cc)::value]; });
            rid = prid;
        } else if (t > j && t < rows) {
            if (t == p) {
                cdf::static_for<0, TW>([&](auto cc) { x[decltype(cc)::value] = rowj[par][decltype(cc)::value]; });
                rid = ridj[par];
            }
            if (piv != 0.0) {
                const double l = x[j] / piv;
                x[j] = l;
                cdf::static_for<j + 1, TW>([&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    x[c] = fma(-l, prow[c], x[c]);
                });
            }
        }
    });
    if (t < k) out[node * SET + 1 + t] = rid;
    if (t == 0) out[node * SET] = k;
    if (gridDim.x == 1 && t < k)
        cdf::static_for<0, TW>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            F[t * TW + c] = x[c];
        });
}

// The final pivot order (set `fin`, leaf-relative row ids) as LAPACK
// interchanges: for j = 0.., the row holding the j-th winner is swapped
// with row j.  ipiv gets region-relative 1-based rows (row0 + position + 1).
// Also the first zero pivot of U00 into *info (info_base + j + 1) if unset.
// One thread; the positions moved so far (at most 2 w) are kept in LDS.
__global__ void tourn_order_kernel(const int *__restrict__ fin, const double *__restrict__ F, int *__restrict__ ipiv,
                                   int row0, int *__restrict__ info, int info_base) {
    __shared__ int pos[2 * TW], who[2 * TW];  // position pos[i] holds original row who[i]
    if (threadIdx.x != 0) return;
    const int k = fin[0];
    int nm = 0;
    auto row_at = [&](int p) {
        for (int i = 0; i < nm; ++i)
            if (pos[i] == p) return who[i];
        return p;
    };
    auto set_at = [&](int p, int r) {
        for (int i = 0; i < nm; ++i)
            if (pos[i] == p) { who[i] = r; return; }
        pos[nm] = p;
        who[nm] = r;
        ++nm;
    };
    auto where = [&](int r) {
        for (int i = 0; i < nm; ++i)
            if (who[i] == r) return pos[i];
        return r;  // never moved
    };
    for (int j = 0; j < k; ++j) {
        const int r = fin[1 + j];
        const int q = where(r);
        ipiv[j] = row0 + q + 1;
        if (q != j) {
            const int rj = row_at(j);
            set_at(j, r);
            set_at(q, rj);
        }
    }
    if (*info == 0)
        for (int j = 0; j < k; ++j)
            if (F[j * TW + j] == 0.0) { *info = info_base + j + 1; break; }
}

// The leaf's rows after the interchanges: rows j < w from F (L00 \ U00),
// rows >= w as the solution l of l U00 = a (columns in order; a zero U_cc
// leaves l_c unscaled).  One row per thread.
__global__ __launch_bounds__(256) void tourn_lower_kernel(int M, int w, double *__restrict__ A, int lda,
                                                          const double *__restrict__ F) {
    __shared__ double U[TW * TW];
    for (int e = threadIdx.x; e < TW * TW; e += 256) U[e] = F[e];
    __syncthreads();
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= M) return;
    double x[TW];
    cdf::static_for<0, TW>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        if (c < w) x[c] = r < w ? U[r * TW + c] : A[(size_t)r + (size_t)c * lda];
    });
    if (r >= w)
        cdf::static_for<0, TW>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            if (c < w) {
                const double ucc = U[c * TW + c];
                if (ucc != 0.0) x[c] = x[c] / ucc;
                cdf::static_for<c + 1, TW>([&](auto dd) {
                    constexpr int d = decltype(dd)::value;
                    if (d < w) x[d] = fma(-x[c], U[c * TW + d], x[d]);
                });
            }
        });
    cdf::static_for<0, TW>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        if (c < w) A[(size_t)r + (size_t)c * lda] = x[c];
    });
}

}  // namespace

namespace cdf {

size_t tourn_ws_bytes() { return 2 * (size_t)kTournMaxSets * SET * sizeof(int) + TW * TW * sizeof(double) + 256; }

hipError_t tourn_leaf(cdf_handle_t h, const LeafArea &la, hipStream_t s, int m, int w, double *A, int lda,
                      int *ipiv, int row0, int *info, int info_base, double *region, int region_rows,
                      int region_cols) {
    if (m <= 0 || w <= 0) return hipSuccess;
    if (w > TW || w > m) return hipErrorInvalidValue;
    int block = h->params[CDF_PARAM_TOURN_BLOCK] > 0 ? h->params[CDF_PARAM_TOURN_BLOCK] : TN;
    int fanin = h->params[CDF_PARAM_TOURN_FANIN] > 0 ? h->params[CDF_PARAM_TOURN_FANIN] : TN / TW;
    if (block < TW || block > TN || fanin < 2 || fanin * TW > TN) return hipErrorInvalidValue;
    // at most kTournMaxSets first-round blocks: larger blocks where the leaf
    // has more rows than that many blocks of the requested size hold
    if ((m + block - 1) / block > kTournMaxSets) block = (((m + kTournMaxSets - 1) / kTournMaxSets + TW - 1) / TW) * TW;
    const int G0 = (m + block - 1) / block;
    if (block > TN || G0 > kTournMaxSets) return hipErrorInvalidValue;  // more than 131072 rows
    char *base = static_cast<char *>(la.base) + kTournOffset;
    int *sets[2] = {reinterpret_cast<int *>(base), reinterpret_cast<int *>(base) + kTournMaxSets * SET};
    double *F = reinterpret_cast<double *>(base + 2 * (size_t)kTournMaxSets * SET * sizeof(int));
    hipLaunchKernelGGL(tourn_node_kernel, dim3(G0), dim3(TN), 0, s, m, w, A, lda, 1, block, nullptr, 0, fanin,
                       sets[0], F);
    CDF_HIP_RET(hipGetLastError());
    int nsets = G0, cur = 0;
    while (nsets > 1) {
        const int nn = (nsets + fanin - 1) / fanin;
        hipLaunchKernelGGL(tourn_node_kernel, dim3(nn), dim3(TN), 0, s, m, w, A, lda, 0, block, sets[cur], nsets,
                           fanin, sets[cur ^ 1], F);
        CDF_HIP_RET(hipGetLastError());
        nsets = nn;
        cur ^= 1;
    }
    hipLaunchKernelGGL(tourn_order_kernel, dim3(1), dim3(64), 0, s, sets[cur], F, ipiv, row0, info, info_base);
    CDF_HIP_RET(hipGetLastError());
    // the interchanges on every column of the region, the leaf's included
    CDF_HIP_RET(laswp(s, 0, region_cols, region, lda, ipiv - row0, row0, row0 + w, region_rows));
    hipLaunchKernelGGL(tourn_lower_kernel, dim3((m + 255) / 256), dim3(256), 0, s, m, w, A, lda, F);
    return hipGetLastError();
}

}  // namespace cdf
