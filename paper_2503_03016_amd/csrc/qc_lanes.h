// Cross-lane exchanges of a 64-lane wavefront through VALU data paths
// (DPP row shifts and mirrors, v_permlane16/32_swap of gfx950) instead of
// LDS permutes: no LDS traffic and no LDS round-trip latency.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qcx {
namespace lanes {

// DPP controls: row_shl:n = 0x100 + n, row_mirror, row_half_mirror, quad_perm
constexpr int kRowMirror = 0x140, kRowHalfMirror = 0x141;
constexpr int kQuadXor1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;   // quad_perm [2,3,0,1]

// value of x on lane (lane + 2^B), valid on the lanes whose bit B is clear
template <int B>
__device__ __forceinline__ uint32_t up(uint32_t x) {
    static_assert(B >= 0 && B < 6, "lane bit");
    if constexpr (B < 4)
        return uint32_t(__builtin_amdgcn_mov_dpp(int(x), 0x100 | (1 << B), 0xf, 0xf, false));
    else if constexpr (B == 4)   // rows 0, 2 receive rows 1, 3 in the second result
        return __builtin_amdgcn_permlane16_swap(x, x, false, false)[1];
    else                          // lanes 0..31 receive lanes 32..63 in the second result
        return __builtin_amdgcn_permlane32_swap(x, x, false, false)[1];
}
template <int B>
__device__ __forceinline__ float up(float x) {
    return __uint_as_float(up<B>(__float_as_uint(x)));
}
template <int B>
__device__ __forceinline__ double up(double x) {
    const uint64_t u = uint64_t(__double_as_longlong(x));
    const uint32_t lo = up<B>(uint32_t(u)), hi = up<B>(uint32_t(u >> 32));
    return __longlong_as_double(int64_t((uint64_t(hi) << 32) | lo));
}

template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
    const uint64_t u = uint64_t(__double_as_longlong(x));
    const uint32_t lo = uint32_t(__builtin_amdgcn_mov_dpp(int(uint32_t(u)), CTRL, 0xf, 0xf, false));
    const uint32_t hi = uint32_t(__builtin_amdgcn_mov_dpp(int(uint32_t(u >> 32)), CTRL, 0xf, 0xf, false));
    return __longlong_as_double(int64_t((uint64_t(hi) << 32) | lo));
}

// x(lane) + x(lane ^ 16) (W32 false) or x(lane) + x(lane ^ 32) (W32 true):
// the swap leaves one of the two values in each result register
template <bool W32>
__device__ __forceinline__ double swap_add(double x) {
    const uint64_t u = uint64_t(__double_as_longlong(x));
    const uint32_t lo = uint32_t(u), hi = uint32_t(u >> 32);
    const auto rl = W32 ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                        : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto rh = W32 ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                        : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const double a = __longlong_as_double(int64_t((uint64_t(rh[0]) << 32) | rl[0]));
    const double b = __longlong_as_double(int64_t((uint64_t(rh[1]) << 32) | rl[1]));
    return a + b;
}

// OR over the 64 lanes, on every lane (same exchange pattern as the sum)
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
    v |= uint32_t(__builtin_amdgcn_mov_dpp(int(v), kQuadXor1, 0xf, 0xf, false));
    v |= uint32_t(__builtin_amdgcn_mov_dpp(int(v), kQuadXor2, 0xf, 0xf, false));
    v |= uint32_t(__builtin_amdgcn_mov_dpp(int(v), kRowHalfMirror, 0xf, 0xf, false));
    v |= uint32_t(__builtin_amdgcn_mov_dpp(int(v), kRowMirror, 0xf, 0xf, false));
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = r[0] | r[1];
    const auto q = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return q[0] | q[1];
}

// sum over the 64 lanes, on every lane: pairs within quads, quads within
// eights (half mirror), eights within rows (mirror), rows by swaps; the two
// lanes of each exchange add the same two values, so every lane ends with
// the same sum
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp<kQuadXor1>(v);
    v += dpp<kQuadXor2>(v);
    v += dpp<kRowHalfMirror>(v);
    v += dpp<kRowMirror>(v);
    v = swap_add<false>(v);
    return swap_add<true>(v);
}

}  // namespace lanes
}  // namespace qcx
