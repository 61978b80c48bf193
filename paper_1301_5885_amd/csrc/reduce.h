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

namespace gabi {

// Rotation of a value across the 64 lanes of a wave by one lane (DPP
// wave_ror:1): after 64 rotations every value is back in its lane.  All 64
// lanes must be active.
__device__ __forceinline__ float wave_rotate(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x13C, 0xf, 0xf, true));
}
__device__ __forceinline__ double wave_rotate(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, 0x13C, 0xf, 0xf, true);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), 0x13C, 0xf, 0xf, true);
    return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}

}  // namespace gabi
