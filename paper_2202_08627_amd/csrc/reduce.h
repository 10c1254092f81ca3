// Deterministic FP64 block reductions (fixed combination order, 64-wide wavefronts).
#pragma once
#include <hip/hip_runtime.h>

namespace eit {

__device__ __forceinline__ double wave_sum(double v) {
    // butterfly over the 64 lanes of a wavefront; every lane ends with the same sum
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
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
