// Deterministic reductions: every workgroup reduces its lanes in a fixed
// order (wavefront butterfly, then the wavefronts in index order) and writes
// one partial per workgroup; a final kernel sums the partials in index order.
// No floating-point atomics, so results are reproducible run to run.
#pragma once

#include "gate_math.hpp"

namespace sv {

constexpr int kRedThreads = 256;
constexpr int kMaxPartials = 2048;  // workgroups of a reducing launch

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        v += lane_xor(v, m);
    return v;
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
