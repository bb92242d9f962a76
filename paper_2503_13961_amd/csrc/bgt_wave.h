// Cross-lane sums for wave64 on gfx950, built from DPP moves (within 16-lane
// rows) and the v_permlane16/32_swap exchanges between rows and wave halves.
#pragma once
#include <hip/hip_runtime.h>

namespace bgt {

template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f(float v) {
    // bound_ctrl: lanes whose source is outside the row/wave read 0
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}

// The value `send` of this lane's partner across lane-index bit BIT
// (hi = that bit of this lane).  Bits 0 and 1: quad_perm; bit 3: row_ror:8;
// bit 2: row_shr:4 or row_shl:4; bits 4 and 5: swapping `send` with itself
// across neighbouring rows (wave halves) leaves the lower row's value in the
// first result and the upper row's in the second.
template <int BIT>
__device__ __forceinline__ float partner_of(float send, bool hi) {
    if constexpr (BIT == 0) {
        return dpp_f<0xB1, 0xF>(send);  // quad_perm [1,0,3,2]
    } else if constexpr (BIT == 1) {
        return dpp_f<0x4E, 0xF>(send);  // quad_perm [2,3,0,1]
    } else if constexpr (BIT == 3) {
        return dpp_f<0x128, 0xF>(send);  // row_ror:8
    } else if constexpr (BIT == 2) {
        const float from_lo = dpp_f<0x114, 0xF>(send), from_hi = dpp_f<0x104, 0xF>(send);  // row_shr:4, row_shl:4
        return hi ? from_lo : from_hi;
    } else if constexpr (BIT == 4) {
        const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(send), __float_as_uint(send), false, false);
        return __uint_as_float(hi ? q[0] : q[1]);
    } else {
        const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(send), __float_as_uint(send), false, false);
        return __uint_as_float(hi ? p[0] : p[1]);
    }
}

// One butterfly: the lanes with bit BIT clear keep the even values of each
// pair, those with it set the odd ones, each adding its partner's copy.
// v[0..N) becomes v[0..(N+1)/2); an odd last value pairs with zero.
template <int N, int BIT>
__device__ __forceinline__ void rs_stage(float *v, int lane) {
    const bool hi = ((lane >> BIT) & 1) != 0;
#pragma unroll
    for (int k = 0; k < N / 2; ++k) {
        const float keep = hi ? v[2 * k + 1] : v[2 * k], send = hi ? v[2 * k] : v[2 * k + 1];
        v[k] = keep + partner_of<BIT>(send, hi);
    }
    if constexpr ((N & 1) != 0) {
        const float keep = hi ? 0.f : v[N - 1], send = hi ? v[N - 1] : 0.f;
        v[N / 2] = keep + partner_of<BIT>(send, hi);
    }
}

// Reduce-scatter of N <= 64 per-lane values over the wave: afterwards lane l
// holds in v[0] the wave total of value scatter_index(l) (0 when that index is
// >= N).  About 3.4 operations per value instead of 6 per value for plain
// tree sums, and the totals land on distinct lanes, ready for one
// multi-lane store or atomic.
template <int N>
__device__ __forceinline__ void wave_reduce_scatter(float *v, int lane) {
    static_assert(N >= 1 && N <= 64, "at most 64 values per call");
    rs_stage<N, 0>(v, lane);
    rs_stage<(N + 1) / 2, 1>(v, lane);
    rs_stage<(N + 3) / 4, 3>(v, lane);
    rs_stage<(N + 7) / 8, 2>(v, lane);
    rs_stage<(N + 15) / 16, 4>(v, lane);
    rs_stage<(N + 31) / 32, 5>(v, lane);
}

__device__ __forceinline__ int scatter_index(int lane) {
    return (lane & 3) | (((lane >> 3) & 1) << 2) | (((lane >> 2) & 1) << 3) | (lane & 48);
}

}  // namespace bgt
