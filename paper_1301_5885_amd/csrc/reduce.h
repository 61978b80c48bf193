// Fixed-order workgroup reductions (wave64 shuffles, then LDS across the
// four waves of a 256-thread workgroup).  The tree shape depends only on the
// workgroup size, so results are bitwise reproducible.
#pragma once
#include <hip/hip_runtime.h>

namespace gabi {

// Sum of v over the workgroup; the result is valid in every thread.
// lds must hold blockDim.x / 64 doubles.  Contains __syncthreads().
__device__ __forceinline__ double block_sum(double v, double *lds) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = lds[0];
    const int nw = blockDim.x >> 6;
    for (int w = 1; w < nw; ++w) s += lds[w];
    return s;
}

}  // namespace gabi
