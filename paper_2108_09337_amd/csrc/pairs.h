// Interchange pairs built by one wave (shared by the LU panel leaf, the
// laswp kernel and the batched factorizations).
#pragma once

#include "internal.h"

namespace {

// Builds the (dst, src) row pairs equivalent to applying the interchanges
// ipiv[k1 - off .. k2 - off) (rows k1..k2-1 swapped with absolute, 1-based
// rows, k2 - k1 <= 64) in order:
//   new row dst[q] = old row src[q].
// Executed by one full wave: the simulated positions (at most 128 distinct
// rows) live in registers, two per lane, and are searched with ballots.
// Returns the pair count (wave-uniform); dst/src are written to LDS.
__device__ int build_pairs_wave(const int *__restrict__ ipiv, int k1, int k2, int nrows, int *dst, int *src,
                                 int off = 0) {
    const int lane = threadIdx.x & 63;
    int myp = (k1 + lane < k2) ? ipiv[k1 + lane - off] - 1 : -1;
    if (myp < k1 + lane || myp >= nrows) myp = k1 + lane;  // out-of-range interchange: ignored
    int pos0 = -1, cont0 = -1, pos1 = -1, cont1 = -1;
    int np = 0;
    for (int k = k1; k < k2; ++k) {
        const int p = __shfl(myp, k - k1);
        if (p == k) continue;
        unsigned long long b0 = __ballot(pos0 == k), b1 = __ballot(pos1 == k);
        int ik = b0 ? __builtin_ctzll(b0) : (b1 ? 64 + __builtin_ctzll(b1) : -1);
        b0 = __ballot(pos0 == p);
        b1 = __ballot(pos1 == p);
        int ip = b0 ? __builtin_ctzll(b0) : (b1 ? 64 + __builtin_ctzll(b1) : -1);
        if (ik < 0) {
            if (lane == (np & 63)) { if (np < 64) { pos0 = k; cont0 = k; } else { pos1 = k; cont1 = k; } }
            ik = np++;
        }
        if (ip < 0) {
            if (lane == (np & 63)) { if (np < 64) { pos0 = p; cont0 = p; } else { pos1 = p; cont1 = p; } }
            ip = np++;
        }
        const int ck = ik < 64 ? __shfl(cont0, ik) : __shfl(cont1, ik - 64);
        const int cp = ip < 64 ? __shfl(cont0, ip) : __shfl(cont1, ip - 64);
        if (lane == (ik & 63)) { if (ik < 64) cont0 = cp; else cont1 = cp; }
        if (lane == (ip & 63)) { if (ip < 64) cont0 = ck; else cont1 = ck; }
    }
    // compaction of the moved positions
    const bool m0 = pos0 >= 0 && cont0 != pos0;
    const bool m1 = pos1 >= 0 && cont1 != pos1;
    const unsigned long long bm0 = __ballot(m0), bm1 = __ballot(m1);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int c0 = __popcll(bm0);
    if (m0) { const int q = __popcll(bm0 & below); dst[q] = pos0; src[q] = cont0; }
    if (m1) { const int q = c0 + __popcll(bm1 & below); dst[q] = pos1; src[q] = cont1; }
    return c0 + __popcll(bm1);
}

}  // namespace
