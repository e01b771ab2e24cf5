// LDS-staged tile pass: a run of gates whose targets lie below the tile width
// applied to one 2^m-amplitude contiguous tile held in LDS, so the run costs
// one HBM read and one HBM write of each touched tile instead of one pass per
// gate (gate fusion, named as future work in Sec. V).
//
// Controls below m are part of the in-tile index expansion (the same
// control-aware scheduling as the single-gate kernels, at tile scope);
// controls at or above m are a predicate on the tile's base index, so a tile
// whose high control bits fail skips the gate, and a tile that no gate of the
// run touches is neither read nor written.
#pragma once

#include "gate_math.hpp"

namespace sv {

constexpr int kTileSeg = 16;   // m <= 14 gives at most 15 segments
constexpr int kTileMaxLog = 14;

struct TileGate {
    double m[8];          // matrix (a, b, c, d as re, im), double precision
    uint32_t target;      // < m
    uint32_t nseg;        // in-tile expansion of the reduced index
    uint32_t shift[kTileSeg];
    uint32_t mask[kTileSeg];
    uint32_t fixed;       // low control bits that must be 1
    uint32_t npairs;      // 2^(m - 1 - low controls)
    uint64_t hi_mask;     // controls >= m, as amplitude-index bits
    uint64_t hi_vals;
    int32_t src_gate;     // index of the gate in its circuit (host bookkeeping)
    int32_t pad2;
};

// Build the tile descriptor of one gate for tile width m (host).
TileGate make_tile_gate(int m, int target, uint64_t cmask, uint64_t cvals, const double *U);

template <int NG> struct InlineGates {
    TileGate g[NG];
    int count;
    __device__ __forceinline__ const TileGate &get(int i) const { return g[i]; }
    __device__ __forceinline__ int size() const { return count; }
};

struct DeviceGates {
    const TileGate *g;
    int count;
    __device__ __forceinline__ const TileGate &get(int i) const { return g[i]; }
    __device__ __forceinline__ int size() const { return count; }
};

template <typename R>
__device__ __forceinline__ Mat2<R> tile_mat(const TileGate &g) {
    return Mat2<R>{(R)g.m[0], (R)g.m[1], (R)g.m[2], (R)g.m[3],
                   (R)g.m[4], (R)g.m[5], (R)g.m[6], (R)g.m[7]};
}

__device__ __forceinline__ uint32_t tile_expand(const TileGate &g, uint32_t x) {
    uint32_t p = g.fixed;
    for (uint32_t s = 0; s < g.nseg; ++s)
        p |= (x << g.shift[s]) & g.mask[s];
    return p;
}

// One workgroup per tile.  Dynamic LDS holds the 2^m amplitudes.
template <typename R, int THREADS, typename Src>
__global__ __launch_bounds__(THREADS) void k_tile(cplx_t<R> *__restrict__ psi, int m, Src gates) {
    extern __shared__ unsigned char lds_raw[];
    cplx_t<R> *tile = reinterpret_cast<cplx_t<R> *>(lds_raw);
    const uint64_t base = (uint64_t)blockIdx.x << m;
    const uint32_t T = 1u << m;

    // a tile that no gate of the run touches is left alone
    bool any = false;
    for (int i = 0; i < gates.size(); ++i) {
        const TileGate &g = gates.get(i);
        any |= ((base & g.hi_mask) == g.hi_vals);
    }
    if (!any)
        return;

    for (uint32_t j = threadIdx.x; j < T; j += THREADS)
        tile[j] = ld_stream<R>(psi + base + j);
    __syncthreads();

    for (int i = 0; i < gates.size(); ++i) {
        const TileGate &g = gates.get(i);
        if ((base & g.hi_mask) != g.hi_vals)
            continue;  // uniform across the workgroup
        const Mat2<R> mm = tile_mat<R>(g);
        const uint32_t st = 1u << g.target;
        for (uint32_t r = threadIdx.x; r < g.npairs; r += THREADS) {
            const uint32_t p1 = tile_expand(g, r);
            cplx_t<R> x = tile[p1], y = tile[p1 | st];
            apply_pair<R>(mm, x, y);
            tile[p1] = x;
            tile[p1 | st] = y;
        }
        __syncthreads();
    }

    for (uint32_t j = threadIdx.x; j < T; j += THREADS)
        st_stream<R>(psi + base + j, tile[j]);
}

} // namespace sv
