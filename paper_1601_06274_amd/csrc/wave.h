// wave.h - wavefront-level primitives for gfx950 (wave64, DPP, permlane swaps).
//
// A "group" is G consecutive lanes (G = 1, 2, 4, 8, 16, 32 or 64) that cooperate
// on one chain; a wave of 64 lanes holds 64/G groups.  All helpers are executed by
// every lane of the wave (no divergence inside the helpers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dm {

// Large finite value used for labels that do not exist (K not a multiple of the tile).
// Finite on purpose: it survives additions of costs without overflowing to Inf.
constexpr float kBig = 1.0e30f;

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
    // Full-mask DPP move; used only with patterns whose sources are always in range.
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
// DPP move whose out-of-range source lanes receive `fill`.
template <int CTRL>
__device__ __forceinline__ float dpp_fill(float x, float fill) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, fill),
                                                                 __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}

// DPP control codes (GFX9 encoding).
constexpr int kQuadXor1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;
constexpr int kWaveShr1 = 0x138;     // lane i <- lane i-1
constexpr int kWaveShl1 = 0x130;     // lane i <- lane i+1
constexpr int kRowShr1 = 0x111;      // lane i <- lane i-1 within a row of 16
constexpr int kRowShl1 = 0x101;      // lane i <- lane i+1 within a row of 16

// Orders this wave's LDS accesses: all lanes' earlier LDS writes are visible to later LDS
// reads of any lane.  For a workgroup of one wave no barrier is needed, and unlike
// __syncthreads (a workgroup fence) this does not wait for global loads in flight.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// An opaque copy: keeps the compiler from treating the two operands of a permlane swap
// as the same value (it would otherwise fold min(swap.first, swap.second)).
__device__ __forceinline__ uint32_t opaque_copy(uint32_t x) {
    uint32_t y;
    asm volatile("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
    return y;
}

// min over the 32-lane halves' rows: row r <-> row r^1 (rows of 16 lanes).
__device__ __forceinline__ float swap16_min(float x) {
    uint32_t a = __builtin_bit_cast(uint32_t, x);
    auto p = __builtin_amdgcn_permlane16_swap(a, opaque_copy(a), false, false);
    return fminf(__builtin_bit_cast(float, (uint32_t)p[0]), __builtin_bit_cast(float, (uint32_t)p[1]));
}
// min across the two 32-lane halves.
__device__ __forceinline__ float swap32_min(float x) {
    uint32_t a = __builtin_bit_cast(uint32_t, x);
    auto p = __builtin_amdgcn_permlane32_swap(a, opaque_copy(a), false, false);
    return fminf(__builtin_bit_cast(float, (uint32_t)p[0]), __builtin_bit_cast(float, (uint32_t)p[1]));
}
__device__ __forceinline__ int swap16_min_i(int x) {
    uint32_t a = (uint32_t)x;
    auto p = __builtin_amdgcn_permlane16_swap(a, opaque_copy(a), false, false);
    return min((int)p[0], (int)p[1]);
}
__device__ __forceinline__ int swap32_min_i(int x) {
    uint32_t a = (uint32_t)x;
    auto p = __builtin_amdgcn_permlane32_swap(a, opaque_copy(a), false, false);
    return min((int)p[0], (int)p[1]);
}

// All-reduce min over each group of G lanes; every lane of the group gets the result.
template <int G>
__device__ __forceinline__ float group_min(float x) {
    if constexpr (G >= 2) x = fminf(x, dpp<kQuadXor1>(x));
    if constexpr (G >= 4) x = fminf(x, dpp<kQuadXor2>(x));
    if constexpr (G >= 8) x = fminf(x, dpp<kRowHalfMirror>(x));
    if constexpr (G >= 16) x = fminf(x, dpp<kRowMirror>(x));
    if constexpr (G >= 32) x = swap16_min(x);
    if constexpr (G >= 64) x = swap32_min(x);
    return x;
}
// Two independent all-reduce minima over groups of G lanes (a and b each get their
// group's minimum in every lane).  For G = 32 and 64 the cross-row steps carry a and b
// in the two operands of one permlane swap, so the pair costs little more than one.
template <int G>
__device__ __forceinline__ void group_min2(float& a, float& b) {
    if constexpr (G == 64 || G == 32) {
        a = group_min<16>(a);
        b = group_min<16>(b);
        const uint32_t ua = __builtin_bit_cast(uint32_t, a), ub = __builtin_bit_cast(uint32_t, b);
        if constexpr (G == 64) {
            // rows 2,3 of a <-> rows 0,1 of b: c = a's minimum over rows {0,2}, {1,3} in
            // rows 0, 1 and b's in rows 2, 3
            auto p = __builtin_amdgcn_permlane32_swap(ua, ub, false, false);
            const float c = swap16_min(fminf(__builtin_bit_cast(float, (uint32_t)p[0]),
                                             __builtin_bit_cast(float, (uint32_t)p[1])));
            // c: a's minimum in lanes 0-31, b's in lanes 32-63; one more swap spreads both
            const uint32_t uc = __builtin_bit_cast(uint32_t, c);
            auto q = __builtin_amdgcn_permlane32_swap(uc, opaque_copy(uc), false, false);
            a = __builtin_bit_cast(float, (uint32_t)q[0]);
            b = __builtin_bit_cast(float, (uint32_t)q[1]);
        } else {
            // rows 1,3 of a <-> rows 0,2 of b: c = a's group minimum in rows 0, 2 and
            // b's in rows 1, 3
            auto p = __builtin_amdgcn_permlane16_swap(ua, ub, false, false);
            const uint32_t uc = __builtin_bit_cast(uint32_t, fminf(__builtin_bit_cast(float, (uint32_t)p[0]),
                                                                   __builtin_bit_cast(float, (uint32_t)p[1])));
            auto q = __builtin_amdgcn_permlane16_swap(uc, opaque_copy(uc), false, false);
            a = __builtin_bit_cast(float, (uint32_t)q[0]);
            b = __builtin_bit_cast(float, (uint32_t)q[1]);
        }
    } else {
        a = group_min<G>(a);
        b = group_min<G>(b);
    }
}

template <int G>
__device__ __forceinline__ int group_min_i(int x) {
    if constexpr (G >= 2) x = min(x, dpp_i<kQuadXor1>(x));
    if constexpr (G >= 4) x = min(x, dpp_i<kQuadXor2>(x));
    if constexpr (G >= 8) x = min(x, dpp_i<kRowHalfMirror>(x));
    if constexpr (G >= 16) x = min(x, dpp_i<kRowMirror>(x));
    if constexpr (G >= 32) x = swap16_min_i(x);
    if constexpr (G >= 64) x = swap32_min_i(x);
    return x;
}

}  // namespace dm
