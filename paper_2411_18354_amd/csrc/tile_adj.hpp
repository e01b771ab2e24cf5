// The reverse sweep on one tile of psi and one of lambda held together in
// LDS (tile layout and operation kinds as in the forward tile pass): shared
// by the single-circuit adjoint and the batched one.
//
// Operation i of a run un-applies its gate (the descriptor holds U^dag).
// When gslot[i] >= 0, its gradient term 2 Re <lambda|Pi_c A|psi> (A: the
// generator in gens[8 gslot[i] ..]) is taken first, over exactly the pairs
// the scheduling enumerates.  It is added to one accumulator per wavefront
// in LDS, for the k-th parameterised gate of the run accl[k * nw + w] (nw:
// the workgroup's wavefronts),
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
    for (int k = threadIdx.x; k < npg * (int)(blockDim.x >> 6); k += blockDim.x)
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
    const int nw = (int)(blockDim.x >> 6);
    double s = 0.0;
    for (int q = 0; q < nw; ++q)
        s += accl[k * nw + q];
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

// Gradient term of one amplitude pair: 2 Re <lambda| A |psi> restricted to
// the pair, A = a[8] (the generator, 2x2 complex) acting on (x, y).
template <typename R>
__device__ __forceinline__ double adj_pair_term(const double *a, const cplx_t<R> &x, const cplx_t<R> &y,
                                                const cplx_t<R> &lx, const cplx_t<R> &ly) {
    const double xr = x.x, xi = x.y, yr = y.x, yi = y.y;
    const double axr = a[0] * xr - a[1] * xi + a[2] * yr - a[3] * yi;
    const double axi = a[0] * xi + a[1] * xr + a[2] * yi + a[3] * yr;
    const double ayr = a[4] * xr - a[5] * xi + a[6] * yr - a[7] * yi;
    const double ayi = a[4] * xi + a[5] * xr + a[6] * yi + a[7] * yr;
    return 2.0 * ((double)lx.x * axr + (double)lx.y * axi + (double)ly.x * ayr + (double)ly.y * ayi);
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
        if (sl >= 0)
            acc += adj_pair_term<R>(a, x, y, lx, ly);
        apply_pair<R>(u, x, y);
        apply_pair<R>(u, lx, ly);
        tp[p1] = x;
        tp[p1 | st] = y;
        tl[p1] = lx;
        tl[p1 | st] = ly;
    }
    return acc;
}

// A coset pair (marked on the host, as in the forward pass) un-applied on
// both tiles: g1 then g2 over every 4-amplitude coset, each gate's gradient
// term taken on the values it sees in the sequential order (acc1, acc2).
template <typename R, int THREADS>
__device__ __forceinline__ void adj_tile_pairs2(cplx_t<R> *tp, cplx_t<R> *tl, uint32_t T, const TileGate &g1,
                                                const TileGate &g2, int sl1, int sl2, const double *a1,
                                                const double *a2, double *acc1, double *acc2) {
    const uint32_t t1 = g1.target, t2 = g2.target;
    const uint32_t lo = min(t1, t2), hi = max(t1, t2);
    const uint32_t s1 = 1u << t1, s2 = 1u << t2;
    const bool c1 = (g1.l_mask >> t2) & 1u, c2 = (g2.l_mask >> t1) & 1u;
    const uint32_t v1 = (g1.l_vals >> t2) & 1u, v2 = (g2.l_vals >> t1) & 1u;
    const bool p0 = !c1 || v1 == 0, p1 = !c1 || v1 == 1, q0 = !c2 || v2 == 0, q1 = !c2 || v2 == 1;
    const Mat2<R> u1 = tile_mat<R>(g1), u2 = tile_mat<R>(g2);
    double s_1 = 0.0, s_2 = 0.0;
    for (uint32_t r = threadIdx.x; r < (T >> 2); r += THREADS) {
        uint32_t b = ((r >> lo) << (lo + 1)) | (r & ((1u << lo) - 1u));
        b = ((b >> hi) << (hi + 1)) | (b & ((1u << hi) - 1u));
        const uint32_t i01 = b | s1, i10 = b | s2, i11 = b | s1 | s2;
        cplx_t<R> x00 = tp[b], x01 = tp[i01], x10 = tp[i10], x11 = tp[i11];
        cplx_t<R> l00 = tl[b], l01 = tl[i01], l10 = tl[i10], l11 = tl[i11];
        if (p0) {
            if (sl1 >= 0)
                s_1 += adj_pair_term<R>(a1, x00, x01, l00, l01);
            apply_pair<R>(u1, x00, x01);
            apply_pair<R>(u1, l00, l01);
        }
        if (p1) {
            if (sl1 >= 0)
                s_1 += adj_pair_term<R>(a1, x10, x11, l10, l11);
            apply_pair<R>(u1, x10, x11);
            apply_pair<R>(u1, l10, l11);
        }
        if (q0) {
            if (sl2 >= 0)
                s_2 += adj_pair_term<R>(a2, x00, x10, l00, l10);
            apply_pair<R>(u2, x00, x10);
            apply_pair<R>(u2, l00, l10);
        }
        if (q1) {
            if (sl2 >= 0)
                s_2 += adj_pair_term<R>(a2, x01, x11, l01, l11);
            apply_pair<R>(u2, x01, x11);
            apply_pair<R>(u2, l01, l11);
        }
        tp[b] = x00;
        tp[i01] = x01;
        tp[i10] = x10;
        tp[i11] = x11;
        tl[b] = l00;
        tl[i01] = l01;
        tl[i10] = l10;
        tl[i11] = l11;
    }
    *acc1 = s_1;
    *acc2 = s_2;
}

// A block [i, e) of consecutive diagonal gates un-applied in one pass over
// both tiles.  Un-applying a unit-modulus diagonal gate multiplies psi_j and
// lambda_j by the same factor f_j, so w_j = conj(lambda_j) psi_j is the same
// before and after every gate of the block, and a gate's gradient term
// 2 Re <lambda| A |psi> = sum_j 2 Re(a_j w_j) (a_j: the generator's diagonal
// entry on amplitude j's target bit, over the amplitudes whose controls
// hold) needs only w_j.  So each lane forms w_j once, adds every
// parameterised gate's term (a wavefront sum into that gate's accumulator),
// multiplies the factors and writes psi_j f_j and lambda_j f_j once.  Every
// gate of an adjoint sweep is unitary (checked on the host).  Returns the
// accumulator index after the block.
template <typename R, int THREADS>
__device__ __forceinline__ int adj_diag_block(cplx_t<R> *tp, cplx_t<R> *tl, uint64_t base, uint32_t T,
                                              const DeviceGates &gates, int i, int e, const int32_t *gslot,
                                              const double *gens, double *accl, int kacc) {
    const int w = threadIdx.x >> 6;
    const uint32_t nch = (T + 4 * THREADS - 1) / (4 * THREADS);  // uniform
    int k = kacc;
    for (uint32_t ch = 0; ch < nch; ++ch) {
        uint32_t j[4];
        bool in[4];
        cplx_t<R> x[4], l[4];
        double wr[4], wi[4];
        R fr[4], fi[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            j[q] = ch * 4 * THREADS + q * THREADS + threadIdx.x;
            in[q] = j[q] < T;
            if (in[q]) {
                x[q] = tp[j[q]];
                l[q] = tl[j[q]];
            } else {
                x[q].x = x[q].y = l[q].x = l[q].y = (R)0;
            }
            wr[q] = (double)l[q].x * (double)x[q].x + (double)l[q].y * (double)x[q].y;
            wi[q] = (double)l[q].x * (double)x[q].y - (double)l[q].y * (double)x[q].x;
            fr[q] = (R)1;
            fi[q] = (R)0;
        }
        k = kacc;
        for (int q = i; q < e; ++q) {
            const TileGate &d = gates.get(q);
            const int sl = gslot[q];
            if ((base & d.o_mask) != d.o_vals) {  // uniform: the gate skips this tile
                k += sl >= 0 ? 1 : 0;
                continue;
            }
            const bool tin = d.l_target >= 0;
            const bool tone = (base >> d.target) & 1ull;
            if (sl >= 0) {  // uniform
                const double a0r = gens[8 * sl + 0], a0i = gens[8 * sl + 1];
                const double a1r = gens[8 * sl + 6], a1i = gens[8 * sl + 7];
                double part = 0.0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (!in[u] || (j[u] & d.l_mask) != d.l_vals)
                        continue;
                    const bool one = tin ? ((j[u] >> d.l_target) & 1u) : tone;
                    const double gr = one ? a1r : a0r, gi = one ? a1i : a0i;
                    part += 2.0 * (gr * wr[u] - gi * wi[u]);
                }
                const double sum = wave_sum(part);
                if ((threadIdx.x & 63) == 0)
                    accl[k * (THREADS / 64) + w] += sum;
                ++k;
            }
            const R m0r = (R)uniform_f64(d.m[0]), m0i = (R)uniform_f64(d.m[1]);
            const R m1r = (R)uniform_f64(d.m[6]), m1i = (R)uniform_f64(d.m[7]);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool on = (j[u] & d.l_mask) == d.l_vals;
                const bool one = tin ? ((j[u] >> d.l_target) & 1u) : tone;
                const R ur = on ? (one ? m1r : m0r) : (R)1, ui = on ? (one ? m1i : m0i) : (R)0;
                const R nr = fr[u] * ur - fi[u] * ui;
                fi[u] = fr[u] * ui + fi[u] * ur;
                fr[u] = nr;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!in[q])
                continue;
            cplx_t<R> nx, nl;
            nx.x = x[q].x * fr[q] - x[q].y * fi[q];
            nx.y = x[q].x * fi[q] + x[q].y * fr[q];
            nl.x = l[q].x * fr[q] - l[q].y * fi[q];
            nl.y = l[q].x * fi[q] + l[q].y * fr[q];
            tp[j[q]] = nx;
            tl[j[q]] = nl;
        }
    }
    return k;
}

// A permutation run (marked on the host, as in the forward pass) on both
// tiles: X gates carry no parameter, so the run only moves amplitudes, and
// psi and lambda move alike.  Requires 2 T <= perm_per_lane<R>() * THREADS.
template <typename R, int THREADS>
__device__ __forceinline__ void adj_tile_permute(cplx_t<R> *tp, cplx_t<R> *tl, uint32_t T, uint64_t base,
                                                 const DeviceGates &gates, int i, int L) {
    constexpr int NP = perm_per_lane<R>() / 2;
    uint32_t src[NP];
    perm_sources<NP, THREADS>(src, base, gates, i, L);
    R vx[NP], vy[NP], wx[NP], wy[NP];  // components apart (see tile_permute)
#pragma unroll
    for (int k = 0; k < NP; ++k)
        if (threadIdx.x + k * THREADS < T) {
            const cplx_t<R> a = tp[src[k]], b = tl[src[k]];
            vx[k] = a.x;
            vy[k] = a.y;
            wx[k] = b.x;
            wy[k] = b.y;
        }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const uint32_t j = threadIdx.x + k * THREADS;
        if (j < T) {
            cplx_t<R> a, b;
            a.x = vx[k];
            a.y = vy[k];
            b.x = wx[k];
            b.y = wy[k];
            tp[j] = a;
            tl[j] = b;
        }
    }
    __syncthreads();
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
        const uint32_t slen = sweep_word(g) & 0xffffu;
        if (g.diag && slen > 1) {  // a block of diagonal gates (uniform)
            const int e = min(gates.size(), i + (int)slen);
            kacc = adj_diag_block<R, THREADS>(tp, tl, base, T, gates, i, e, gslot, gens, accl, kacc);
            __syncthreads();
            i = e - 1;
            continue;
        }
        const uint32_t plen = __builtin_amdgcn_readfirstlane(g.perm_len);
        if (!g.diag && plen >= 2 && 2 * T <= (uint32_t)(perm_per_lane<R>() * THREADS)) {  // a permutation run
            const int L = min((int)plen, gates.size() - i);
            adj_tile_permute<R, THREADS>(tp, tl, T, base, gates, i, L);
            i += L - 1;
            continue;
        }
        if (!g.diag && slen == 2 && i + 1 < gates.size()) {  // a coset pair (uniform)
            const TileGate &g2 = gates.get(i + 1);
            if ((base & g.hi_mask) == g.hi_vals && (base & g2.hi_mask) == g2.hi_vals) {
                const int sl2 = gslot[i + 1];
                double a1[8], a2[8];
                for (int q = 0; q < 8; ++q) {
                    a1[q] = sl >= 0 ? gens[8 * sl + q] : 0.0;
                    a2[q] = sl2 >= 0 ? gens[8 * sl2 + q] : 0.0;
                }
                double acc1, acc2;
                adj_tile_pairs2<R, THREADS>(tp, tl, T, g, g2, sl, sl2, a1, a2, &acc1, &acc2);
                if (sl >= 0) {
                    const double s1 = wave_sum(acc1);
                    if ((threadIdx.x & 63) == 0)
                        accl[kacc * (THREADS / 64) + w] += s1;
                    ++kacc;
                }
                if (sl2 >= 0) {
                    const double s2 = wave_sum(acc2);
                    if ((threadIdx.x & 63) == 0)
                        accl[kacc * (THREADS / 64) + w] += s2;
                    ++kacc;
                }
                __syncthreads();
                ++i;
                continue;
            }
        }
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
                    accl[kacc * (THREADS / 64) + w] += s;
            }
            __syncthreads();
        }
        kacc += sl >= 0 ? 1 : 0;
    }
}

} // namespace sv
