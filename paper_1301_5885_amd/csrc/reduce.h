// Fixed-order workgroup reductions (DPP lane moves within a wave64, then LDS
// across the waves of the workgroup).  The tree shape depends only on the
// workgroup size, so results are bitwise reproducible.
#pragma once
#include <hip/hip_runtime.h>

namespace gabi {

// Fixed-order sum over the 64 lanes of a wave with DPP lane moves; the total
// lands in lane 63.  Within each row of 16 lanes, shifts by 1, 2, 4 and 8
// build the row prefix in lane 15 of the row; row_bcast:15 adds row 0 into
// row 1 and row 2 into row 3, row_bcast:31 adds rows 0-1 into rows 2-3.
// Lanes whose source is outside the pattern receive zero.  All 64 lanes must
// be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW_MASK, 0xf, false);
    const int hi =
        __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW_MASK, 0xf, false);
    return __builtin_bit_cast(double, (unsigned long long)(unsigned)lo |
                                          ((unsigned long long)(unsigned)hi << 32));
}

__device__ __forceinline__ double wave_total_lane63(double v) {
    v += dpp_move<0x111, 0xf>(v);  // row_shr:1
    v += dpp_move<0x112, 0xf>(v);  // row_shr:2
    v += dpp_move<0x114, 0xf>(v);  // row_shr:4
    v += dpp_move<0x118, 0xf>(v);  // row_shr:8
    v += dpp_move<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Sum of v over the workgroup; the result is valid in every thread.
// lds must hold blockDim.x / 64 doubles.  Contains __syncthreads().  Every
// thread of the workgroup must call it.
__device__ __forceinline__ double block_sum(double v, double *lds) {
    v = wave_total_lane63(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 63) lds[wave] = v;
    __syncthreads();
    double s = lds[0];
    const int nw = blockDim.x >> 6;
    for (int w = 1; w < nw; ++w) s += lds[w];
    return s;
}

}  // namespace gabi

namespace gabi {

// Rotation of a value across the 64 lanes of a wave by one lane: lane l
// receives lane (l - 1) mod 64's value, so after 64 rotations every value is
// back in its lane.  All 64 lanes must be active.
//
// The float rotation goes through the LDS crossbar (ds_bpermute; `from` is
// the byte address of the source lane, rotate_from()), which leaves the VALU
// to the pair arithmetic: measured 2-4% faster for the FP32 symmetric kernel
// at N >= 46,080.  The double rotation uses DPP wave_ror:1 on each half: two
// crossbar moves per double cost the FP64 kernel (four waves per SIMD) 3%,
// and adding the FP64 column sums in per-wave LDS arrays (ds_add_f64) instead
// of rotating them was 2% slower at N = 327,680 (measured on one box).
__device__ __forceinline__ int rotate_from() {
    return (int)(((threadIdx.x & 63u) + 63u) & 63u) << 2;
}
__device__ __forceinline__ float wave_rotate(float v, int from) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(from, __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double wave_rotate(double v, int) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, 0x13C, 0xf, 0xf, true);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), 0x13C, 0xf, 0xf, true);
    return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}

}  // namespace gabi
