// Deterministic FP64 block reductions (fixed combination order, 64-wide wavefronts).
#pragma once
#include <hip/hip_runtime.h>

namespace eit {

// One DPP data movement of a double (both 32-bit halves); lanes whose row is outside
// ROW_MASK, or whose source lane is outside the row, read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wavefront, returned in every lane; all 64 lanes must be active.
// Fixed order: quad sums (lane pairs, then pairs of pairs), 8- and 16-lane sums (half-row and
// row mirrors), then rows 0 + 1 and 2 + 3 (row broadcast 15) and their sum (row broadcast
// 31) in lane 63, which every lane reads. Cross-lane moves are DPP operand modifiers, not
// LDS permutes.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0xB1, 0xF>(v);     // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E, 0xF>(v);     // quad_perm [2,3,0,1]
    v += dpp_f64<0x141, 0xF>(v);    // row_half_mirror
    v += dpp_f64<0x140, 0xF>(v);    // row_mirror
    v += dpp_f64<0x142, 0xA>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xC>(v);    // row_bcast:31 into rows 2 and 3
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum of `v` over the block; result valid in every thread. `scratch` must hold
// blockDim.x/64 doubles. Contains two __syncthreads().
__device__ __forceinline__ double block_sum(double v, double* scratch) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += scratch[w];   // fixed order
    __syncthreads();
    return s;
}

}  // namespace eit
