// LDS-staged tile pass: a run of gates applied to one tile of 2^m amplitudes
// held in LDS, so the run costs one HBM read and one HBM write of each touched
// tile instead of one pass per gate (gate fusion, named as future work in
// Sec. V).
//
// A tile is the set of amplitudes that agree on every index bit outside a
// chosen qubit set S of m qubits: the `a` lowest qubits (so each tile is made
// of contiguous runs of 2^a amplitudes, which keeps loads coalesced) plus up
// to m - a further qubits chosen by the planner.  Tile-local index bit i
// stands for the i-th qubit of S in ascending order.
//
// Two kinds of operations run inside a tile:
//  - a pair gate whose target is in S: controls in S are part of the in-tile
//    index expansion (the control-aware scheduling of Sec. III-B at tile
//    scope); controls outside S are a predicate on the tile's base index, so
//    a tile whose outer control bits fail skips the gate;
//  - a diagonal gate (any target): it scales each amplitude whose controls
//    hold by a or d, picked by its target bit; consecutive diagonal gates are
//    applied together in one sweep over the tile.
// A tile that no operation of the run touches is neither read nor written.
#pragma once

#include "gate_math.hpp"

namespace sv {

constexpr int kTileSeg = 16;   // m <= 14 gives at most 15 segments
constexpr int kTileMaxLog = 14;
constexpr int kTileMaxHigh = 8;  // qubits of S above the contiguous low block

struct TileGate {
    double m[8];          // matrix (a, b, c, d as re, im), double precision
    uint32_t diag;        // 1: diagonal gate applied elementwise
    uint32_t target;      // pair gate: tile-local bit; diagonal: global qubit
    uint32_t nseg;        // pair gate: in-tile expansion of the reduced index
    uint32_t shift[kTileSeg];
    uint32_t mask[kTileSeg];
    uint32_t fixed;       // in-tile control bits that must be 1
    uint32_t npairs;      // 2^(m - 1 - in-tile controls)
    uint64_t hi_mask;     // controls outside S (global bits; diagonal: all controls)
    uint64_t hi_vals;
    int32_t src_gate;     // index of the gate in its circuit (host bookkeeping)
    int32_t pad2;
};

// Where a tile's amplitudes live: base = deposit(tile index) over the qubits
// outside S; local index j maps to base | (j & (2^a - 1)) | scatter(j >> a)
// over the high qubits of S.
// Control bits outside S that every operation of a run requires (with the
// same value) are inserted into the tile index too, so only tiles that can
// be touched are launched: the control-aware scheduling of Sec. III-B
// applied at tile granularity.
struct TileMap {
    uint32_t m;
    uint32_t a;        // S holds qubits 0 .. a-1 (contiguous runs of 2^a)
    uint32_t nh;       // and these further qubits, ascending
    uint32_t hpos[kTileMaxHigh];
    uint32_t nseg;     // local bits >= a scattered as (j & in_mask) << shift
    uint32_t seg_in[kTileMaxHigh];
    uint32_t seg_shift[kTileMaxHigh];
    Expand outer;
    uint64_t ntiles;  // launched tiles: 2^(n - m - fixed outer bits)
};

// Tile map for S = {0 .. a-1} u high (host).  high: ascending qubits >= a;
// fixed_mask/fixed_vals: outer index bits every launched tile has.
TileMap make_tile_map(int n, int m, int a, const std::vector<int> &high, uint64_t fixed_mask = 0,
                      uint64_t fixed_vals = 0);
// Descriptor of one gate for a tile map (host).  A pair gate's target must be
// in S.
TileGate make_tile_gate(const TileMap &tm, int target, uint64_t cmask, uint64_t cvals, const double *U,
                        bool diagonal);
// Contiguous tiles (S = {0 .. m-1}).
TileMap contiguous_tile_map(int n, int m);

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

__device__ __forceinline__ uint64_t tile_offset(const TileMap &tm, uint32_t j) {
    uint64_t o = j & ((1u << tm.a) - 1);
    for (uint32_t s = 0; s < tm.nseg; ++s)
        o |= (uint64_t)(j & tm.seg_in[s]) << tm.seg_shift[s];
    return o;
}

// One workgroup per tile.  Dynamic LDS holds the 2^m amplitudes.
template <typename R, int THREADS, typename Src>
__global__ __launch_bounds__(THREADS) void k_tile(cplx_t<R> *__restrict__ psi, TileMap tm, Src gates) {
    extern __shared__ unsigned char lds_raw[];
    cplx_t<R> *tile = reinterpret_cast<cplx_t<R> *>(lds_raw);
    const uint64_t base = expand_index<uint64_t>(tm.outer, (uint64_t)blockIdx.x);
    const uint32_t T = 1u << tm.m;

    // a tile that no operation of the run touches is left alone
    bool any = false;
    for (int i = 0; i < gates.size(); ++i) {
        const TileGate &g = gates.get(i);
        any |= g.diag ? true : ((base & g.hi_mask) == g.hi_vals);
    }
    if (!any)
        return;

    for (uint32_t j = threadIdx.x; j < T; j += THREADS)
        tile[j] = ld_stream<R>(psi + (base | tile_offset(tm, j)));
    __syncthreads();

    int i = 0;
    while (i < gates.size()) {
        const TileGate &g = gates.get(i);
        if (g.diag) {
            int e = i + 1;
            while (e < gates.size() && gates.get(e).diag)
                ++e;
            for (uint32_t j = threadIdx.x; j < T; j += THREADS) {
                const uint64_t k = base | tile_offset(tm, j);
                R fr = (R)1, fi = (R)0;
                for (int q = i; q < e; ++q) {
                    const TileGate &d = gates.get(q);
                    if ((k & d.hi_mask) != d.hi_vals)
                        continue;
                    const int o = ((k >> d.target) & 1ull) ? 6 : 0;
                    const R ur = (R)d.m[o], ui = (R)d.m[o + 1];
                    const R nr = fr * ur - fi * ui;
                    fi = fr * ui + fi * ur;
                    fr = nr;
                }
                const cplx_t<R> v = tile[j];
                cplx_t<R> w;
                w.x = v.x * fr - v.y * fi;
                w.y = v.x * fi + v.y * fr;
                tile[j] = w;
            }
            __syncthreads();
            i = e;
            continue;
        }
        if ((base & g.hi_mask) == g.hi_vals) {  // uniform across the workgroup
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
        ++i;
    }

    for (uint32_t j = threadIdx.x; j < T; j += THREADS)
        st_stream<R>(psi + (base | tile_offset(tm, j)), tile[j]);
}

} // namespace sv
