// Cross-lane helpers shared by the on-chip kernels: DPP and gfx950 permlane
// reductions of doubles, and lane broadcasts.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace rg {
namespace {

// Cross-lane sums of doubles without LDS: DPP within a 16-lane row, gfx950
// permlane swaps between rows.  Each step adds two operands in an order that
// is the same on both lanes of a pair, so every lane ends with the same bits.
__device__ inline double from_halves(int lo, int hi) {
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ inline double dpp(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return from_halves(__builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false),
                       __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false));
}
// Sum over the 16 lanes of a DPP row: xor 1, xor 2 (quad_perm), then the
// half-row and row mirrors pair the quads and the half-rows.
__device__ inline double sum16(double v) {
    v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);  // row_half_mirror
    v += dpp<0x140>(v);  // row_mirror
    return v;
}
// Sum over the 4 DPP rows of a wave (same lane pj): permlane16_swap pairs
// rows (0,1) and (2,3), permlane32_swap pairs the two halves.
__device__ inline double sum_rows(double v) {
    {
        const int lo = __double2loint(v), hi = __double2hiint(v);
        const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        v = from_halves(a[0], b[0]) + from_halves(a[1], b[1]);
    }
    {
        const int lo = __double2loint(v), hi = __double2hiint(v);
        const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        v = from_halves(a[0], b[0]) + from_halves(a[1], b[1]);
    }
    return v;
}
__device__ inline double sum64(double v) { return sum_rows(sum16(v)); }

// Reduce-scatter of four values over the 4 DPP rows of a wave, pairing two
// different values per swap: permlane32_swap(a, b) gives rows (a0, a1, b0, b1)
// and (a2, a3, b2, b3); permlane16_swap(a, b) gives (a0, b0, a2, b2) and
// (a1, b1, a3, b3).  Returns, on row q of the wave, the total over the 4 rows
// of v[q].
__device__ inline double swap_add32(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
    return from_halves(lo[0], hi[0]) + from_halves(lo[1], hi[1]);
}
__device__ inline double swap_add16(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
    return from_halves(lo[0], hi[0]) + from_halves(lo[1], hi[1]);
}
__device__ inline double scatter4(double v0, double v1, double v2, double v3) {
    // rows 0,1 now hold partials of v0 / v1, rows 2,3 of v2 / v3
    const double u0 = swap_add32(v0, v2), u1 = swap_add32(v1, v3);
    return swap_add16(u0, u1);
}

// Value of v on lane K of this lane's DPP row of 16 (row_newbcast: one
// 64-bit move, the result in a vector register).
template <int K>
__device__ inline double bcast16(double v) {
    static_assert(K >= 0 && K < 16, "lane within a row of 16");
    return __builtin_amdgcn_mov_dpp(v, 0x150 + K, 0xF, 0xF, false);
}

// f(std::integral_constant<int, k>{}) for k = 0 .. N-1 in order, so that k can
// select an immediate such as a DPP control.
template <typename F, int... K>
__device__ inline void static_for_impl(F &&f, std::integer_sequence<int, K...>) {
    (f(std::integral_constant<int, K>{}), ...);
}
template <int N, typename F>
__device__ inline void static_for(F &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Value of v on lane `lane` (wave-uniform lane index), for doubles.
__device__ inline double read_lane(double v, int lane) {
    return from_halves(__builtin_amdgcn_readlane(__double2loint(v), lane),
                       __builtin_amdgcn_readlane(__double2hiint(v), lane));
}

}  // namespace
}  // namespace rg
