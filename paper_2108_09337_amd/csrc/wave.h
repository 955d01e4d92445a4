// Wave-wide reductions by DPP data movement (no LDS round trips), shared by
// the pivot searches: the LU panel leaf, the tournament nodes and the
// batched panels.
#pragma once

#include "internal.h"

namespace {

typedef unsigned long long u64;

// Pivot key of a candidate: 1 + the bit pattern of |a| (the patterns of
// non-negative floating-point values order like the values), 0 for a row
// that takes no part and for NaN (which never wins).
__device__ inline u64 pivot_key(double a) {
    return a == a ? (u64)__double_as_longlong(fabs(a)) + 1ull : 0ull;
}
__device__ inline u64 pivot_key(float a) { return a == a ? (u64)__float_as_uint(fabsf(a)) + 1ull : 0ull; }

// One step of a wave maximum / minimum of 32-bit values: v = max(v, v of
// the lane the DPP control selects) (min likewise); lanes without a source
// see the operation's identity.  The compiler folds each step into one
// v_max_u32 / v_min_u32 with a DPP source.
template <int CTRL, int ROW_MASK>
__device__ inline unsigned dpp_max_step(unsigned v) {
    const unsigned o = (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, false);
    return o > v ? o : v;
}
template <int CTRL, int ROW_MASK>
__device__ inline unsigned dpp_min_step(unsigned v) {
    const unsigned o = (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, CTRL, ROW_MASK, 0xf, false);
    return o < v ? o : v;
}

// Largest / smallest value over the wave, in every lane: row shifts by 1, 2,
// 4, 8 leave each row's result in its lane 15, two row broadcasts bring all
// four to lane 63, which is read back.
__device__ inline unsigned wave_max_u32(unsigned v) {
    v = dpp_max_step<0x111, 0xf>(v);  // row_shr:1
    v = dpp_max_step<0x112, 0xf>(v);  // row_shr:2
    v = dpp_max_step<0x114, 0xf>(v);  // row_shr:4
    v = dpp_max_step<0x118, 0xf>(v);  // row_shr:8
    v = dpp_max_step<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_max_step<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ inline unsigned wave_min_u32(unsigned v) {
    v = dpp_min_step<0x111, 0xf>(v);
    v = dpp_min_step<0x112, 0xf>(v);
    v = dpp_min_step<0x114, 0xf>(v);
    v = dpp_min_step<0x118, 0xf>(v);
    v = dpp_min_step<0x142, 0xa>(v);
    v = dpp_min_step<0x143, 0xc>(v);
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Largest 64-bit key over the wave, in every lane: the largest high half,
// then the largest low half among the lanes that hold it (two passes of
// single-instruction 32-bit steps).
__device__ inline u64 wave_max_key(u64 key) {
    const unsigned hi = (unsigned)(key >> 32), lo = (unsigned)key;
    const unsigned mh = wave_max_u32(hi);
    const unsigned ml = wave_max_u32(hi == mh ? lo : 0u);
    return ((u64)mh << 32) | ml;
}

// The wave's best (key, row): the largest key, then the smallest row among
// the lanes holding it (rows as unsigned; a lane with key 0 takes no part).
// Returns the key (0: no candidate) and the row in *row (~0u then).
__device__ inline u64 wave_best(u64 key, unsigned row, unsigned *best_row) {
    const u64 wk = wave_max_key(key);
    *best_row = wave_min_u32(key == wk && wk != 0ull ? row : ~0u);
    return wk;
}

}  // namespace
