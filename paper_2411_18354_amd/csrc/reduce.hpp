// Deterministic reductions: every workgroup reduces its lanes in a fixed
// order (wavefront butterfly, then the wavefronts in index order) and writes
// one partial per workgroup; a final kernel sums the partials in index order.
// No floating-point atomics, so results are reproducible run to run.
#pragma once

#include "gate_math.hpp"

namespace sv {

constexpr int kRedThreads = 256;
constexpr int kMaxPartials = 2048;  // workgroups of a reducing launch

// v from the lane DPP control CTRL names, within rows of 16 lanes.
template <int CTRL> __device__ __forceinline__ double dpp_double(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_value(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Sum of v over the 64 lanes of a wavefront, the same value in every lane.
// Inside each row of 16 lanes by data-parallel-primitive moves (partner lane
// xor 1, xor 2, then the mirrored lane within 8 and within 16: after each
// step both partners hold the same sum, a + b = b + a), then the four row
// sums read from lanes 0, 16, 32, 48 and added in a fixed order.  No LDS
// round trip (lane exchanges through ds_bpermute took six dependent ones).
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_double<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_double<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_double<0x141>(v);  // row_half_mirror
    v += dpp_double<0x140>(v);  // row_mirror
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Sum of v over the whole workgroup (blockDim.x lanes, a multiple of 64);
// valid in every lane.  scratch: blockDim.x / 64 doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double *scratch) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        scratch[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i)
        s += scratch[i];
    return s;
}

inline unsigned reduce_grid(uint64_t work_items) {
    const uint64_t b = (work_items + kRedThreads - 1) / kRedThreads;
    return (unsigned)(b < 1 ? 1 : (b > (uint64_t)kMaxPartials ? (uint64_t)kMaxPartials : b));
}

// Sum partials[0 .. count) in a fixed order with one workgroup.
__device__ __forceinline__ double block_sum_array(const double *partials, int count, double *scratch) {
    double v = 0.0;
    for (int i = threadIdx.x; i < count; i += blockDim.x)
        v += partials[i];
    return block_sum(v, scratch);
}

} // namespace sv
