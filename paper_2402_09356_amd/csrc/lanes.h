// Cross-lane moves inside a wave through DPP (data-parallel primitives):
// register-to-register within a row of 16 lanes, with no trip through the LDS
// crossbar that __shfl / ds_bpermute takes.  A double moves as two 32-bit
// halves.  All source lanes of the patterns used here lie inside the row, so
// no lane reads a disabled or out-of-row source.
#pragma once

#include <hip/hip_runtime.h>

namespace tlr {

// DPP control words (gfx9 encoding).
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]: lane l reads l ^ 1
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]: lane l reads l ^ 2
constexpr int kDppHalfMirror = 0x141;  // lane l reads 7 - l within its 8 lanes
constexpr int kDppMirror = 0x140;      // lane l reads 15 - l within its row
constexpr int kDppRowBcast0 = 0x150;   // + j: every lane of a row reads the row's lane j

// Every lane is written from a valid source, so the destination's old value
// is never kept: the plain move form needs no initialisation of it.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL>((int)b);
    const int hi = dpp_i<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lane j's value of each row of 16, in every lane of that row.
template <int J>
__device__ __forceinline__ double row_bcast(double v) {
    static_assert(J >= 0 && J < 16, "lane within a row");
    return dpp_d<kDppRowBcast0 + J>(v);
}

// row_bcast<j> for a j that is a constant once the caller's loop is unrolled.
__device__ __forceinline__ double row_bcast_at(double v, int j) {
    switch (j) {
        case 0: return row_bcast<0>(v);
        case 1: return row_bcast<1>(v);
        case 2: return row_bcast<2>(v);
        case 3: return row_bcast<3>(v);
        case 4: return row_bcast<4>(v);
        case 5: return row_bcast<5>(v);
        case 6: return row_bcast<6>(v);
        case 7: return row_bcast<7>(v);
        case 8: return row_bcast<8>(v);
        case 9: return row_bcast<9>(v);
        case 10: return row_bcast<10>(v);
        case 11: return row_bcast<11>(v);
        case 12: return row_bcast<12>(v);
        case 13: return row_bcast<13>(v);
        case 14: return row_bcast<14>(v);
        default: return row_bcast<15>(v);
    }
}

// Sum over each row of 16 lanes, the same in all 16 lanes.  The pairing is
// that of an xor butterfly over distances 1, 2, 4, 8 (once a quad, then a
// half row, holds one value, mirroring reaches a lane of the partner group),
// so every lane ends with the same bits.
__device__ __forceinline__ double red16(double v) {
    v += dpp_d<kDppXor1>(v);
    v += dpp_d<kDppXor2>(v);
    v += dpp_d<kDppHalfMirror>(v);
    v += dpp_d<kDppMirror>(v);
    return v;
}

// Orders LDS traffic between the lanes of one wave: writes before the call
// are visible to reads after it in any lane of the same wave.  (The hardware
// runs a wave's LDS operations in order; the fences stop the compiler from
// moving accesses across the point.)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Broadcast of lane l's double to the whole wave (two v_readlane; l uniform).
__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

}  // namespace tlr
