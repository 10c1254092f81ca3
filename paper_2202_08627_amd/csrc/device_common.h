// Device helpers shared by the library's HIP translation units.
#pragma once
#include "eit_internal.h"
#include "reduce.h"

namespace eit {

__device__ __forceinline__ bool skipped(const SliceDesc& d) {
    return d.skip != nullptr && *d.skip != 0;
}
__device__ __forceinline__ bool skipped_adj(const SliceDesc& d) {
    return (d.skip != nullptr && *d.skip != 0) || (d.skip_adj != nullptr && *d.skip_adj != 0);
}

// Pointers read out of a descriptor are generic; these casts let the compiler use global
// (vector) loads and, for wavefront-uniform addresses of read-only tables, scalar loads.
typedef const __attribute__((address_space(1))) float gfloat;
__device__ __forceinline__ gfloat* as_global(const float* p) { return (gfloat*)p; }
template <class T>
__device__ __forceinline__ T cld(const T* p) {
    return *(const __attribute__((address_space(4))) T*)p;
}

// Raw buffer resource over `bytes` bytes from `p` (gfx9 descriptor word 3): loads at offsets
// >= bytes return 0 without touching memory. Every offset is carried in the VGPR operand.
constexpr int kBufOOB = 0x7ffffff0;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const float* p, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, int voff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
}


}  // namespace eit
