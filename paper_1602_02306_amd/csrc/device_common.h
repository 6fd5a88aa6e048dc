// Small device helpers shared by the kernel files of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ecnt {

// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X, each
// with its own L2.  Remap the hardware block id so that each XCD walks a
// contiguous range of logical tiles: neighbouring rows (stencil neighbours,
// rows sharing CSR columns) then meet in the same L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb)
{
    const int64_t per = nb >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
}

template <typename T>
__device__ __forceinline__ double ld(const T *p, size_t i)
{
    return static_cast<double>(p[i]);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

}  // namespace ecnt
