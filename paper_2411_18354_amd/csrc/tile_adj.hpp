// The reverse sweep on one tile of psi and one of lambda held together in
// LDS (tile layout and operation kinds as in the forward tile pass): shared
// by the single-circuit adjoint and the batched one.
//
// Operation i of a run un-applies its gate (the descriptor holds U^dag).
// When gslot[i] >= 0, its gradient term 2 Re <lambda|Pi_c A|psi> (A: the
// generator in gens[8 gslot[i] ..]) is taken first, over exactly the pairs
// the scheduling enumerates.  It is added to one accumulator per wavefront
// in LDS, for the k-th parameterised gate of the run accl[k * kAdjWaves + w],
// so a gate needs a wavefront reduction, not a workgroup barrier.
#pragma once

#include "reduce.hpp"
#include "tile.hpp"

namespace sv {

constexpr int kAdjTileThreads = 512;
constexpr int kAdjWaves = kAdjTileThreads / 64;

// Zero the accumulators of the run's parameterised gates (all threads;
// ends with a barrier).  Returns how many there are.
__device__ __forceinline__ int adj_acc_zero(const DeviceGates &gates, const int32_t *gslot, double *accl) {
    int npg = 0;
    for (int i = 0; i < gates.size(); ++i)
        npg += gslot[i] >= 0 ? 1 : 0;
    for (int k = threadIdx.x; k < npg * kAdjWaves; k += blockDim.x)
        accl[k] = 0.0;
    __syncthreads();
    return npg;
}

// Generator slot of the k-th parameterised gate of the run.
__device__ __forceinline__ int adj_acc_slot(const DeviceGates &gates, const int32_t *gslot, int k) {
    int c = 0;
    for (int i = 0; i < gates.size(); ++i)
        if (gslot[i] >= 0) {
            if (c == k)
                return gslot[i];
            ++c;
        }
    return -1;
}

// The k-th accumulator summed over the wavefronts in index order.
__device__ __forceinline__ double adj_acc_sum(const double *accl, int k) {
    double s = 0.0;
    for (int q = 0; q < kAdjWaves; ++q)
        s += accl[k * kAdjWaves + q];
    return s;
}

__device__ __forceinline__ bool adj_tile_touched(uint64_t base, const DeviceGates &gates) {
    for (int i = 0; i < gates.size(); ++i) {
        const TileGate &g = gates.get(i);
        if (g.diag ? ((base & g.o_mask) == g.o_vals) : ((base & g.hi_mask) == g.hi_vals))
            return true;  // uniform
    }
    return false;
}

// One pair gate un-applied on both tiles, with its gradient term (sl >= 0;
// generator a[8]) summed per lane in pair order.  The in-tile expansion is
// held in NS register segments, as in the forward pass's pair loop (NS = 0:
// read from the descriptor for every pair).
template <typename R, int THREADS, int NS>
__device__ __forceinline__ double adj_tile_pairs(cplx_t<R> *tp, cplx_t<R> *tl, const TileGate &g, int sl,
                                                 const double *a) {
    constexpr int N = NS > 0 ? NS : 1;
    uint32_t sh[N], mk[N];
#pragma unroll
    for (int s = 0; s < N; ++s) {
        sh[s] = s < (int)g.nseg ? g.shift[s] : 0u;
        mk[s] = s < (int)g.nseg ? g.mask[s] : 0u;
    }
    const uint32_t fixed = g.fixed;
    const Mat2<R> u = tile_mat<R>(g);
    const uint32_t st = 1u << g.target;
    double acc = 0.0;
    for (uint32_t r = threadIdx.x; r < g.npairs; r += THREADS) {
        uint32_t p1;
        if (NS > 0) {
            p1 = fixed;
#pragma unroll
            for (int s = 0; s < N; ++s)
                p1 |= (r << sh[s]) & mk[s];
        } else {
            p1 = tile_expand(g, r);
        }
        cplx_t<R> x = tp[p1], y = tp[p1 | st], lx = tl[p1], ly = tl[p1 | st];
        if (sl >= 0) {
            const double xr = x.x, xi = x.y, yr = y.x, yi = y.y;
            const double axr = a[0] * xr - a[1] * xi + a[2] * yr - a[3] * yi;
            const double axi = a[0] * xi + a[1] * xr + a[2] * yi + a[3] * yr;
            const double ayr = a[4] * xr - a[5] * xi + a[6] * yr - a[7] * yi;
            const double ayi = a[4] * xi + a[5] * xr + a[6] * yi + a[7] * yr;
            acc += 2.0 * ((double)lx.x * axr + (double)lx.y * axi + (double)ly.x * ayr + (double)ly.y * ayi);
        }
        apply_pair<R>(u, x, y);
        apply_pair<R>(u, lx, ly);
        tp[p1] = x;
        tp[p1 | st] = y;
        tl[p1] = lx;
        tl[p1 | st] = ly;
    }
    return acc;
}

template <typename R, int THREADS>
__device__ __forceinline__ void adj_tile_run(cplx_t<R> *tp, cplx_t<R> *tl, uint64_t base, uint32_t T,
                                             const DeviceGates &gates, const int32_t *__restrict__ gslot,
                                             const double *__restrict__ gens, double *accl) {
    const int w = threadIdx.x >> 6;
    int kacc = 0;  // parameterised gates seen so far in this run
    for (int i = 0; i < gates.size(); ++i) {
        const TileGate &g = gates.get(i);
        const int sl = gslot[i];
        double a[8];
        for (int q = 0; q < 8; ++q)
            a[q] = sl >= 0 ? gens[8 * sl + q] : 0.0;
        double acc = 0.0;
        bool did = false;
        if (g.diag) {
            if ((base & g.o_mask) == g.o_vals) {  // uniform
                did = true;
                const bool tin = g.l_target >= 0;
                const bool tone = (base >> g.target) & 1ull;
                // entries made wave-uniform before the per-lane select
                const R m0r = (R)uniform_f64(g.m[0]), m0i = (R)uniform_f64(g.m[1]);
                const R m1r = (R)uniform_f64(g.m[6]), m1i = (R)uniform_f64(g.m[7]);
                for (uint32_t j = threadIdx.x; j < T; j += THREADS) {
                    if ((j & g.l_mask) != g.l_vals)
                        continue;
                    const bool one = tin ? ((j >> g.l_target) & 1u) : tone;
                    const cplx_t<R> x = tp[j], lx = tl[j];
                    if (sl >= 0) {
                        const double gr = one ? a[6] : a[0], gi = one ? a[7] : a[1];
                        const double axr = gr * x.x - gi * x.y, axi = gr * x.y + gi * x.x;
                        acc += 2.0 * ((double)lx.x * axr + (double)lx.y * axi);
                    }
                    const R ur = one ? m1r : m0r, ui = one ? m1i : m0i;
                    cplx_t<R> nx, nl;
                    nx.x = x.x * ur - x.y * ui;
                    nx.y = x.x * ui + x.y * ur;
                    nl.x = lx.x * ur - lx.y * ui;
                    nl.y = lx.x * ui + lx.y * ur;
                    tp[j] = nx;
                    tl[j] = nl;
                }
            }
        } else if ((base & g.hi_mask) == g.hi_vals) {  // uniform
            did = true;
            // the loop's index arithmetic sized to the gate (uniform branches)
            if (g.nseg <= 2)
                acc = adj_tile_pairs<R, THREADS, 2>(tp, tl, g, sl, a);
            else if (g.nseg <= 3)
                acc = adj_tile_pairs<R, THREADS, 3>(tp, tl, g, sl, a);
            else if (g.nseg <= 4)
                acc = adj_tile_pairs<R, THREADS, 4>(tp, tl, g, sl, a);
            else if (g.nseg <= (uint32_t)kExpRegs)
                acc = adj_tile_pairs<R, THREADS, kExpRegs>(tp, tl, g, sl, a);
            else
                acc = adj_tile_pairs<R, THREADS, 0>(tp, tl, g, sl, a);
        }
        if (did) {  // uniform
            if (sl >= 0) {
                const double s = wave_sum(acc);
                if ((threadIdx.x & 63) == 0)
                    accl[kacc * kAdjWaves + w] += s;
            }
            __syncthreads();
        }
        kacc += sl >= 0 ? 1 : 0;
    }
}

} // namespace sv
