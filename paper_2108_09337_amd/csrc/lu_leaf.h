// The LU panel leaf (Sec. 7, routine A00, with the column-by-column pivot
// search that partial pivoting requires, Sec. 7.3), included by the two
// sources that instantiate it for one and two rows per thread.
//
// Leaf kernel: factors an m x n (n <= 32) column block.  The rows are spread
// over G workgroups (at most one per CU), 256*R rows each; every thread keeps
// its R rows of the block in registers (the column loop is unrolled at
// compile time), so the kernel needs almost no LDS and fits on a CU beside
// the update GEMM's workgroups.  Every column costs one grid-wide exchange,
// done without atomics or cache-wide fences:
//   1. each workgroup finds its best candidate (largest |a|, lowest row on
//      ties) with wave shuffles and LDS, then writes the candidate's whole
//      row (and, if it owns it, the current row j) to its slot and three tag
//      words: the candidate's |a| split in two 32-bit halves and its row
//      index.  Every 64-bit word written (row entries too, as two words per
//      double) pairs 32 data bits with a 32-bit epoch unique to this launch
//      and column, so nothing waits for the row stores to complete: a reader
//      re-reads a word until it carries the current epoch;
//   2. every workgroup polls the G tag triples with device-coherent loads
//      until all carry the current epoch (each 64-bit word is written
//      whole, so a word with the current epoch holds the current half), and
//      reduces them identically;
//   3. it reads the winning row (and row j), each entry once both of its
//      words carry the current epoch, then each thread swaps, scales
//      (division) and rank-1 updates its own rows.
// Slots are double-buffered by column parity: a workgroup can only overwrite
// the slots of column j once every workgroup has published column j + 1,
// which each does after it finished reading column j.  With G = 1 the
// exchange stays in LDS.
//
// Every wait of the exchange is bounded.  A workgroup that has waited longer
// than its budget (constant-rate wall clock, plus a poll-count cap) sets the
// device error word, marks the call's info with CDF_INFO_TIMEOUT and stops;
// any workgroup that finds the error word set while it waits stops too, and
// later leaf launches of the same factorization return at once.  So every
// workgroup ends normally even if the grid never becomes co-resident, and
// the host learns of it from info or cdf_device_status().  A stopped leaf
// leaves identity interchanges for its unfinished columns, so the kernels
// after it stay in bounds.
#pragma once

#include "internal.h"
#include "pairs.h"
#include "wave.h"

#include <climits>

namespace {

constexpr int LW = 32;   // leaf width (columns)
constexpr int LT = 256;  // threads per workgroup
constexpr int GMAX = 256;
constexpr int MAXSW = 64;          // interchanges per pair map
constexpr int MAXPAIRS = 2 * MAXSW;
typedef unsigned long long u64;

// Workspace layout of the exchange (at the head of the handle's workspace).
constexpr size_t kTagWords = 4;  // per slot: |a| high half, |a| low half, row index, padding
constexpr size_t kTagBytes = 2 * GMAX * kTagWords * sizeof(u64);
constexpr size_t kRowWords = 2 * GMAX * LW * 2;  // candidate rows: two tagged words per entry
constexpr size_t kRowjWords = 2 * LW * 2;        // row j
constexpr size_t kExchBytes = kTagBytes + (kRowWords + kRowjWords) * sizeof(u64);
static_assert(kExchBytes <= cdf::kLeafWsBytes, "leaf workspace");

__device__ inline void put_tag(u64 *p, u64 v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline u64 get_tag(const u64 *p) {
    return __hip_atomic_load(const_cast<u64 *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int get_err(const int *p) {
    return __hip_atomic_load(const_cast<int *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void set_err(int *p) { __hip_atomic_store(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Budget of one wait: give up once the wall clock has advanced `ticks` past
// the start, or after `max_polls` polls (a cap that holds even if the clock
// stalls), or as soon as another workgroup has given up.  The error word and
// the clock are read in the same round as the polled words, so that checking
// them adds no round trip to a poll.
struct WaitBudget {
    long long t0, ticks;
    unsigned polls, max_polls;
    __device__ WaitBudget(long long budget_ticks, unsigned maxp)
        : t0(wall_clock64()), ticks(budget_ticks), polls(0), max_polls(maxp) {}
    // true: stop waiting (timed out, or the error word `errv` read this round
    // is set); uniform over the active lanes
    __device__ bool spent(int errv, long long now, bool *timed_out) {
        if (__builtin_amdgcn_readfirstlane(errv) != 0) { *timed_out = false; return true; }
        if (now - t0 > ticks || ++polls > max_polls) { *timed_out = true; return true; }
        return false;
    }
};

// A double as two tagged words (high half, low half), each with epoch e.
__device__ inline void put_pair(u64 *p, double v, u64 e) {
    const u64 bits = (u64)__double_as_longlong(v);
    put_tag(p, e | (bits >> 32));
    put_tag(p + 1, e | (bits & 0xffffffffull));
}
// Reads the doubles at pa and (unless null) pb once all their words carry
// epoch e, polling both in the same rounds; false if the wait ran out of
// budget first.
__device__ inline bool get_two(const u64 *pa, const u64 *pb, u64 e, double *va, double *vb, WaitBudget &wb,
                               const int *err, bool *timed_out) {
    for (;;) {
        const int ev = get_err(err);
        const long long now = wall_clock64();
        const u64 a0 = get_tag(pa), a1 = get_tag(pa + 1);
        u64 b0 = e, b1 = e;
        if (pb) {
            b0 = get_tag(pb);
            b1 = get_tag(pb + 1);
        }
        if ((a0 & ~0xffffffffull) == e && (a1 & ~0xffffffffull) == e && (b0 & ~0xffffffffull) == e &&
            (b1 & ~0xffffffffull) == e) {
            *va = __longlong_as_double((long long)((a0 << 32) | (a1 & 0xffffffffull)));
            if (pb) *vb = __longlong_as_double((long long)((b0 << 32) | (b1 & 0xffffffffull)));
            return true;
        }
        if (wb.spent(ev, now, timed_out)) return false;
        __builtin_amdgcn_s_sleep(1);
    }
}

template <int R>
__global__ __launch_bounds__(LT) void lu_leaf_kernel(int m, int n, double *__restrict__ A, int lda,
                                                     int *__restrict__ ipiv, int row0,
                                                     int *__restrict__ info, int info_base,
                                                     u64 *__restrict__ tags, u64 *__restrict__ rows,
                                                     unsigned epoch0, double *__restrict__ Reg, int rm,
                                                     int rcols, int rc0, int *__restrict__ err,
                                                     long long budget_ticks, unsigned max_polls,
                                                     unsigned epoch_skew) {
    constexpr int RT = LT * R;  // rows per workgroup
    constexpr int NW = LT / 64;
    __shared__ double prow[LW], oldj[LW], candw[2][NW][LW], lrowj[2][LW];
    __shared__ u64 wk_s[2][NW];
    __shared__ unsigned wr_s[2][NW];
    __shared__ int xi[1];
    __shared__ int spiv[LW];  // region row (1-based) swapped with row rc0 + j
    __shared__ int pdst[MAXPAIRS], psrc[MAXPAIRS];
    __shared__ int s_np;
    __shared__ int s_stop;    // 1 once this workgroup has stopped waiting (monotone)

    const int G = gridDim.x;
    const int g = blockIdx.x;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int rbase = g * RT;
    u64 *rowj = rows + kRowWords;
    // the leaf is the critical path and shares its CUs with the update
    // GEMM's workgroups: its waves win the instruction arbitration
    __builtin_amdgcn_s_setprio(3);

    // an earlier leaf of this factorization gave up: return at once
    if (t == 0) s_stop = G > 1 ? get_err(err) : 0;
    __syncthreads();
    if (s_stop) {
        if (g == 0 && t < n) ipiv[t] = row0 + t + 1;
        return;
    }
    int stopped_at = -1;  // first column not factored (uniform), or -1

    // the thread's rows rbase + s*LT + t, all columns, in registers
    double x[R][LW];
    cdf::static_for<0, R>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        const int r = rbase + s * LT + t;
        cdf::static_for<0, LW>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            x[s][c] = (r < m && c < n) ? A[(size_t)r + (size_t)c * lda] : 0.0;
        });
    });

    cdf::static_for<0, LW>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (j >= n || stopped_at >= 0) return;
        const int par = j & 1;
        // 1. local candidate of column j among rows >= j: the largest key,
        //    then the smallest row (a thread's rows ascend with s), by wave
        //    DPP reductions; each wave's winner writes its row to the wave's
        //    slot and the owner of row j writes row j (slots by column
        //    parity), then one barrier and a branch-free choice among the
        //    waves' (key, row) pairs
        u64 tk = 0ull;
        unsigned tr = ~0u;
        cdf::static_for<0, R>([&](auto sc) {
            constexpr int s = decltype(sc)::value;
            const int r = rbase + s * LT + t;
            const u64 k = (r < m && r >= j) ? pivot_key(x[s][j]) : 0ull;
            if (k > tk) { tk = k; tr = (unsigned)r; }
        });
        unsigned wrow;
        const u64 wkey = wave_best(tk, tr, &wrow);
        cdf::static_for<0, R>([&](auto sc) {
            constexpr int s = decltype(sc)::value;
            const int r = rbase + s * LT + t;
            if (wkey != 0ull && (unsigned)r == wrow)
                cdf::static_for<0, LW>([&](auto cc) { candw[par][wave][decltype(cc)::value] = x[s][decltype(cc)::value]; });
            if (r == j)
                cdf::static_for<0, LW>([&](auto cc) { lrowj[par][decltype(cc)::value] = x[s][decltype(cc)::value]; });
        });
        if (lane == 0) { wk_s[par][wave] = wkey; wr_s[par][wave] = wrow; }
        __syncthreads();
        u64 v = wk_s[par][0];
        unsigned pr_u = wr_s[par][0];
        int wsel = 0;
#pragma unroll
        for (int q = 1; q < NW; ++q) {
            const u64 kq = wk_s[par][q];
            const unsigned rq = wr_s[par][q];
            const bool b = kq > v || (kq == v && rq < pr_u);
            v = b ? kq : v;
            pr_u = b ? rq : pr_u;
            wsel = b ? q : wsel;
        }
        int p = v != 0ull ? (int)pr_u : INT_MAX;
        const double *cand = candw[par][wsel];
        if (G > 1) {
            const u64 e = (u64)(epoch0 + (unsigned)j) << 32;
            // the epoch waited for: e, except under the test setting that
            // makes every wait run out of budget
            const u64 ew = (u64)(epoch0 + epoch_skew + (unsigned)j) << 32;
            if (wave == 0) {
                // publish rows and tags, all words tagged with the epoch
                if (p != INT_MAX && t < n) put_pair(rows + (((size_t)par * GMAX + g) * LW + t) * 2, cand[t], e);
                if (j >= rbase && j < rbase + RT && t < n)
                    put_pair(rowj + ((size_t)par * LW + t) * 2, lrowj[par][t], e);
                if (t < 3) {
                    // the candidate's key in two halves, then its row
                    const u64 half = t == 0 ? v >> 32 : (t == 1 ? v & 0xffffffffull : (u64)(unsigned)p);
                    put_tag(tags + ((size_t)par * GMAX + g) * kTagWords + t, e | half);
                }
            }
            // 2. wave 0 polls every workgroup's tags (up to GMAX / 64 per lane,
            //    pausing between rounds so that the polling leaves the memory
            //    path to kernels running beside the leaf); waves 1.. wait at
            //    the barrier.  The winner is the largest key, then the
            //    smallest row (DPP reductions): a total order, so the
            //    reduction order is free.
            if (wave == 0) {
                constexpr int QPL = GMAX / 64;
                u64 w[QPL][3];
                bool all, quit = false, timed_out = false;
                WaitBudget wb(budget_ticks, max_polls);
                do {
                    const int ev = get_err(err);
                    const long long now = wall_clock64();
                    bool ok = true;
#pragma unroll
                    for (int i = 0; i < QPL; ++i) {
                        const int q = lane + 64 * i;
                        if (q < G) {
                            const u64 *tq = tags + ((size_t)par * GMAX + q) * kTagWords;
                            w[i][0] = get_tag(tq);
                            w[i][1] = get_tag(tq + 1);
                            w[i][2] = get_tag(tq + 2);
                            ok = ok && (w[i][0] & ~0xffffffffull) == ew && (w[i][1] & ~0xffffffffull) == ew &&
                                 (w[i][2] & ~0xffffffffull) == ew;
                        }
                    }
                    all = __all(ok);
                    if (!all) {
                        if (wb.spent(ev, now, &timed_out)) { quit = true; break; }
                        __builtin_amdgcn_s_sleep(1);
                    }
                } while (!all);
                if (quit && lane == 0) {
                    s_stop = 1;
                    if (timed_out) {
                        set_err(err);
                        atomicExch(info, CDF_INFO_TIMEOUT);
                    }
                }
                u64 ck = 0ull;
                unsigned cr = ~0u;
#pragma unroll
                for (int i = 0; i < QPL; ++i) {
                    const int q = lane + 64 * i;
                    if (q < G) {
                        const u64 ok_ = ((w[i][0] & 0xffffffffull) << 32) | (w[i][1] & 0xffffffffull);
                        const unsigned orow = (unsigned)(w[i][2] & 0xffffffffull);
                        if (ok_ > ck || (ok_ == ck && orow < cr)) { ck = ok_; cr = orow; }
                    }
                }
                unsigned crow;
                const u64 ckey = wave_best(ck, cr, &crow);
                if (lane == 0) xi[0] = ckey != 0ull ? (int)crow : INT_MAX;
            }
            __syncthreads();
            p = xi[0];
            const int win = p == INT_MAX ? 0 : p / RT;  // the workgroup that owns row p
            // 3. winning row and current row j
            if (t < n && !s_stop) {
                // row j is always published (by its owner); a candidate row
                // only where that workgroup had one, which the winner did
                WaitBudget wb(budget_ticks, max_polls);
                bool timed_out = false;
                double oj = 0.0, pr = 0.0;
                // both rows in the same rounds (one round trip, not two)
                const bool ok = get_two(rowj + ((size_t)par * LW + t) * 2,
                                        p != INT_MAX ? rows + (((size_t)par * GMAX + win) * LW + t) * 2 : nullptr,
                                        ew, &oj, &pr, wb, err, &timed_out);
                if (p == INT_MAX) pr = oj;
                oldj[t] = oj;
                prow[t] = pr;
                if (!ok) {
                    s_stop = 1;
                    if (timed_out) {
                        set_err(err);
                        atomicExch(info, CDF_INFO_TIMEOUT);
                    }
                }
            }
        } else if (t < n) {
            oldj[t] = lrowj[par][t];
            prow[t] = p == INT_MAX ? lrowj[par][t] : cand[t];
        }
        if (p == INT_MAX) p = j;  // no ordered candidate (NaN column): no interchange
        __syncthreads();
        if (s_stop) {  // uniform: every thread reads it after the barrier
            stopped_at = j;
            return;
        }
        const double piv = prow[j];
        if (t == 0) spiv[j] = rc0 + p + 1;
        if (g == 0 && t == 0) {
            ipiv[j] = row0 + p + 1;
            if (piv == 0.0 && *info == 0) *info = info_base + j + 1;
        }
        // swap rows j and p, scale and update; every thread owns its rows
        cdf::static_for<0, R>([&](auto sc) {
            constexpr int s = decltype(sc)::value;
            const int r = rbase + s * LT + t;
            if (r == j) {
                cdf::static_for<0, LW>([&](auto cc) { x[s][decltype(cc)::value] = prow[decltype(cc)::value]; });
            } else if (r > j && r < m) {
                const bool moved = (r == p);
                if (moved)
                    cdf::static_for<0, j>([&](auto cc) { x[s][decltype(cc)::value] = oldj[decltype(cc)::value]; });
                const double aj = moved ? oldj[j] : x[s][j];
                if (piv != 0.0) {
                    const double l = aj / piv;
                    x[s][j] = l;
                    cdf::static_for<j + 1, LW>([&](auto cc) {
                        constexpr int c = decltype(cc)::value;
                        x[s][c] = fma(-l, prow[c], moved ? oldj[c] : x[s][c]);
                    });
                } else if (moved) {
                    cdf::static_for<j, LW>([&](auto cc) { x[s][decltype(cc)::value] = oldj[decltype(cc)::value]; });
                }
            }
        });
    });

    if (stopped_at >= 0) {
        // gave up: identity interchanges for the columns not factored, so
        // that the kernels after this one stay in bounds; A is left as it is
        if (g == 0 && t >= stopped_at && t < n) ipiv[t] = row0 + t + 1;
        return;
    }

    cdf::static_for<0, R>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        const int r = rbase + s * LT + t;
        cdf::static_for<0, LW>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            if (r < m && c < n) A[(size_t)r + (size_t)c * lda] = x[s][c];
        });
    });

    // the block's interchanges on the region's other columns [0, rc0) and
    // [rc0 + n, rcols): pairs from the pivots (same in every workgroup), then
    // each wave moves one column at a time (all rows read before any write)
    if (rcols <= n) return;
    __syncthreads();
    if (wave == 0) {
        const int np = build_pairs_wave(spiv, rc0, rc0 + n, rm, pdst, psrc, rc0);
        if (lane == 0) s_np = np;
    }
    __syncthreads();
    const int np = s_np;
    if (np == 0) return;
    const int others = rcols - n;
    for (int q = g * (LT / 64) + wave; q < others; q += G * (LT / 64)) {
        const int c = q < rc0 ? q : q + n;
        double v0 = 0.0, v1 = 0.0;
        if (lane < np) v0 = Reg[(size_t)psrc[lane] + (size_t)c * lda];
        if (lane + 64 < np) v1 = Reg[(size_t)psrc[lane + 64] + (size_t)c * lda];
        if (lane < np) Reg[(size_t)pdst[lane] + (size_t)c * lda] = v0;
        if (lane + 64 < np) Reg[(size_t)pdst[lane + 64] + (size_t)c * lda] = v1;
    }
}

}  // namespace
