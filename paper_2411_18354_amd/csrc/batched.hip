// Batched execution of many independent circuits of uneven width in one
// persistent launch, and their batched adjoint gradients.
//
// Every workgroup repeatedly takes the next circuit from a device work queue
// (an atomic counter; circuits ordered by decreasing cost so the longest ones
// start first) and runs it alone, so no barrier ever spans workgroups and
// every workgroup leaves the loop once the queue is empty.
//  - A state that fits the workgroup's LDS (2^n amplitudes <= kBatchLds
//    bytes) is read once, all gates are applied in LDS, and it is written
//    back once.
//  - A larger state is processed pass by pass from global memory with the
//    circuit's fused plan (the same planner and tile code as single
//    circuits): a fused run visits the state tile by tile, a tile being the
//    2^m amplitudes that share the index bits outside the run's qubit set S,
//    held in LDS while the run's operations act on it (pair gates, and
//    diagonal sweeps through the phase tables); other gates are pair loops
//    over the state.  A workgroup barrier separates passes.
// Each gate visits only the amplitude pairs whose controls hold: the pair
// index is built by inserting the target bit (0) and the control bits (their
// values) into the iteration counter, lowest position first (Sec. III-B).
#include <algorithm>
#include <atomic>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>

#include "circuit.hpp"
#include "gates.hpp"
#include "pauli.hpp"
#include "tile_adj.hpp"

namespace sv {

int validate_circuit_gate(int n, int nparams, const sv_gate_t &g, int index);
int validate_unitary_gate(const sv_gate_t &g, int index);

constexpr int kBatchThreads = 512;
constexpr int kBatchAdjMaxThreads = 1024;  // the batched adjoint's wider shape
// amplitudes per lane in flight when the batched adjoint writes a tile pair
// back (the batched kernels have fewer registers to spare than the
// single-circuit ones: they load tiles by direct HBM-to-LDS copies and the
// forward one writes one amplitude at a time)
constexpr int kBatchCopy = 2;
constexpr size_t kBatchLds = 65536;  // the tile (or a whole resident state)
// dynamic LDS: the work-item slot, the tile, then the diagonal-sweep tables
constexpr size_t kBatchSlot = 64;
constexpr size_t kBatchDynLds = kBatchSlot + kBatchLds + sizeof(double) * diag_table_doubles(13);  // tile widths up to 13

struct BGate {
    double m[8];      // matrix of a fixed gate
    int32_t kind;     // matrix recomputed from params[param] when param >= 0
    int32_t param;    // index into the concatenated parameter array, or -1
    int32_t target;
    int32_t pad;
    uint64_t cmask, cvals;
};

// One pass of a circuit's fused plan.
struct BPass {
    TileMap tm;       // fused: the tiles' qubit set (tm.tab set: tables reserved)
    int32_t fused;    // 1: tile descriptors [first, first + count); 0: gate `gate`
    int32_t gate;     // single: index among the circuit's gates
    int32_t first, count;
    // circuits split over several workgroups: the pass's chunks are tickets
    // [chunk0, chunk0 + nchunks) of the circuit, each chunk_len tiles (fused)
    // or pairs (single gate)
    int32_t chunk0, nchunks;
    uint64_t chunk_len;
};

// A parameterised gate inside a fused run: its descriptor's matrix (and
// phases) is recomputed from the angle before each batched run.
struct BTileJob {
    int32_t kind, param, tile, pad;
};

struct BCirc {
    void *psi;
    void *lam;           // adjoint only
    int32_t n;
    int32_t m;           // tile width of the fused plan
    int32_t first_pass, npasses;  // forward: the fused plan
    int32_t first_apass, napasses;  // adjoint: the fused plan of the reverse sweep
    int32_t first_gate;  // gates [first_gate, first_gate + ngates), in program order
    int32_t ngates;
    int32_t first_param, nparams;  // adjoint: gradient slots
    int32_t first_term, nterms;    // adjoint: Hamiltonian terms
    int32_t group;       // forward: >= 0 when split over workgroups (its ticket counters)
    int32_t nchunks;     // forward, split: tickets over all passes
};

// Insert the target bit (0) and the control bits (their values) into x,
// lowest position first.  I: uint32_t when every index fits 32 bits.
template <typename I> __device__ __forceinline__ I insert_bits(I x, I positions, I vals) {
    while (positions) {
        const int p = sizeof(I) == 8 ? __builtin_ctzll((uint64_t)positions) : __builtin_ctz((uint32_t)positions);
        positions &= positions - 1;
        const I lo = x & (((I)1 << p) - 1);
        x = ((x >> p) << (p + 1)) | (((vals >> p) & (I)1) << p) | lo;
    }
    return x;
}

// The gate's matrix (angle from params when parameterised), or its conjugate
// transpose for the reverse sweep.
template <typename R>
__device__ __forceinline__ Mat2<R> bgate_mat(const BGate &g, const double *params, bool adjoint) {
    double m[8];
    if (g.param >= 0)
        gate_matrix(g.kind, params[g.param], nullptr, m);
    else
        for (int k = 0; k < 8; ++k)
            m[k] = g.m[k];
    if (adjoint)
        return Mat2<R>{(R)m[0], (R)-m[1], (R)m[4], (R)-m[5], (R)m[2], (R)-m[3], (R)m[6], (R)-m[7]};
    return Mat2<R>{(R)m[0], (R)m[1], (R)m[2], (R)m[3], (R)m[4], (R)m[5], (R)m[6], (R)m[7]};
}

constexpr int kBatchPairUnroll = 4;  // pairs per lane per step of a pair loop

// Apply one gate (target, controls) to amplitudes held at base[0 .. 2^nbits)
// (LDS or global), controls below nbits enumerated, controls at or above
// nbits already known to hold: the iteration indices [lo, min(hi, pairs)).
template <typename R, typename I>
__device__ __forceinline__ void gate_on_block_i(cplx_t<R> *base, int nbits, int target, uint64_t cmask,
                                                uint64_t cvals, const Mat2<R> &mm, uint64_t lo, uint64_t hi) {
    const uint64_t lowm = (nbits >= 64) ? ~0ull : ((1ull << nbits) - 1);
    const I cm = (I)(cmask & lowm);
    const I pos = cm | ((I)1 << target);
    const uint64_t all = 1ull << (nbits - 1 - __popcll((uint64_t)cm));
    const I npairs = (I)(hi < all ? hi : all);
    const I st = (I)1 << target;
    const I cv = (I)(cvals & cm);
    constexpr int U = kBatchPairUnroll;  // 2U loads in flight
    for (I i0 = (I)lo + threadIdx.x; i0 < npairs; i0 += (I)U * kBatchThreads) {
        cplx_t<R> x[U], y[U];
        I p1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const I i = i0 + (I)u * kBatchThreads;
            p1[u] = insert_bits<I>(i, pos, cv);
            if (i < npairs) {
                x[u] = base[p1[u]];
                y[u] = base[p1[u] | st];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (i0 + (I)u * kBatchThreads < npairs) {
                apply_pair<R>(mm, x[u], y[u]);
                base[p1[u]] = x[u];
                base[p1[u] | st] = y[u];
            }
        }
    }
}

// 32-bit index arithmetic whenever the block's indices fit (always for LDS
// tiles; for global memory up to n = 32).
template <typename R>
__device__ __forceinline__ void gate_on_block(cplx_t<R> *base, int nbits, int target, uint64_t cmask, uint64_t cvals,
                                              const Mat2<R> &mm, uint64_t lo = 0, uint64_t hi = ~0ull) {
    if (nbits <= 32)
        gate_on_block_i<R, uint32_t>(base, nbits, target, cmask, cvals, mm, lo, hi);
    else
        gate_on_block_i<R, uint64_t>(base, nbits, target, cmask, cvals, mm, lo, hi);
}

// Tiles [lo, hi) of a fused pass over the state in global memory.
template <typename R>
__device__ __forceinline__ void fused_tiles(cplx_t<R> *psi, const BPass &p, const TileGate *__restrict__ tiles,
                                            const SweepPat *__restrict__ pats, const SweepMember *__restrict__ mems,
                                            cplx_t<R> *lds, uint64_t lo, uint64_t hi) {
    const DeviceGates dg{tiles + p.first, p.count, pats, mems};
    const uint32_t T = 1u << p.tm.m;
    for (uint64_t tt = lo; tt < hi; ++tt) {
        const uint64_t base = expand_index<uint64_t>(p.tm.outer, tt);
        if (!tile_touched(base, dg))
            continue;  // uniform
        tile_load_dma<R, kBatchThreads>(lds, psi, base, p.tm, T);
        __syncthreads();
        tile_run<R, kBatchThreads, false>(lds, base, p.tm, dg);  // at its register limit
        tile_store<R, kBatchThreads, false, 1>(psi, lds, base, p.tm, T);
        __syncthreads();
    }
}

template <typename R>
__device__ void run_circuit_block(const BCirc &c, const BGate *__restrict__ gates, const BPass *__restrict__ passes,
                                  const TileGate *__restrict__ tiles, const SweepPat *__restrict__ pats,
                                  const SweepMember *__restrict__ mems, const double *__restrict__ params,
                                  cplx_t<R> *lds) {
    cplx_t<R> *psi = reinterpret_cast<cplx_t<R> *>(c.psi);
    const uint64_t N = 1ull << c.n;
    if (N * sizeof(cplx_t<R>) <= kBatchLds) {
        for (uint64_t k = threadIdx.x; k < N; k += kBatchThreads)
            lds[k] = psi[k];
        __syncthreads();
        for (int i = 0; i < c.ngates; ++i) {
            const BGate &g = gates[c.first_gate + i];
            gate_on_block<R>(lds, c.n, g.target, g.cmask, g.cvals, bgate_mat<R>(g, params, false));
            __syncthreads();
        }
        for (uint64_t k = threadIdx.x; k < N; k += kBatchThreads)
            psi[k] = lds[k];
        return;
    }
    for (int pi = 0; pi < c.npasses; ++pi) {
        const BPass &p = passes[c.first_pass + pi];
        if (p.fused) {  // uniform
            fused_tiles<R>(psi, p, tiles, pats, mems, lds, 0, p.tm.ntiles);
        } else {
            const BGate &g = gates[c.first_gate + p.gate];
            gate_on_block<R>(psi, c.n, g.target, g.cmask, g.cvals, bgate_mat<R>(g, params, false));
            __syncthreads();
        }
    }
}

// Wait (lane 0 polling, the workgroup held at a barrier) until *ctr >= target,
// then make other workgroups' writes visible to this one.  The wait is
// bounded: after `limit` clock ticks it gives up and counts a timeout in
// *err (the results of that run are then undefined).
__device__ __forceinline__ void wait_count(unsigned int *ctr, unsigned int target, uint64_t limit,
                                           unsigned int *err) {
    if (threadIdx.x == 0) {
        if (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            const uint64_t t0 = wall_clock64();
            do {
                __builtin_amdgcn_s_sleep(2);
                if (wall_clock64() - t0 > limit) {
                    atomicAdd(err, 1u);
                    break;
                }
            } while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the CU's and the XCD's caches refetch
    }
    __syncthreads();
}

// A circuit split over several workgroups.  Every workgroup that joins it
// takes chunk tickets from the circuit's counter: the chunks of all passes
// are numbered in program order, and a chunk of pass p starts once the
// circuit's completion count has reached the first ticket of p.  Chunks of
// p and later cannot complete before that, so the count then says that every
// chunk of the earlier passes is written.  The holder of the lowest unfinished
// ticket never waits, so the circuit progresses whatever the number of
// workgroups that have joined (one is enough); a workgroup that finds the
// tickets used up goes back to the work queue.  Each tile or pair is
// computed exactly as by one workgroup, so results do not depend on the
// split.
template <typename R>
__device__ void run_circuit_split(const BCirc &c, const BGate *__restrict__ gates, const BPass *__restrict__ passes,
                                  const TileGate *__restrict__ tiles, const SweepPat *__restrict__ pats,
                                  const SweepMember *__restrict__ mems, const double *__restrict__ params,
                                  unsigned int *gstate, uint64_t limit, unsigned int *err, cplx_t<R> *lds,
                                  int *slot) {
    cplx_t<R> *psi = reinterpret_cast<cplx_t<R> *>(c.psi);
    unsigned int *next = gstate + 2 * c.group, *done = next + 1;
    int pi = 0, ready = -1;
    for (;;) {
        if (threadIdx.x == 0)
            *slot = (int)__hip_atomic_fetch_add(next, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int k = *slot;
        __syncthreads();
        if (k >= c.nchunks)
            break;
        while (k >= passes[c.first_pass + pi].chunk0 + passes[c.first_pass + pi].nchunks)
            ++pi;  // tickets only grow
        const BPass &p = passes[c.first_pass + pi];
        if (ready != pi) {
            wait_count(done, (unsigned int)p.chunk0, limit, err);
            ready = pi;
        }
        const uint64_t lo = (uint64_t)(k - p.chunk0) * p.chunk_len;
        if (p.fused) {  // uniform
            const uint64_t hi = lo + p.chunk_len < p.tm.ntiles ? lo + p.chunk_len : p.tm.ntiles;
            fused_tiles<R>(psi, p, tiles, pats, mems, lds, lo, hi);
        } else {
            const BGate &g = gates[c.first_gate + p.gate];
            gate_on_block<R>(psi, c.n, g.target, g.cmask, g.cvals, bgate_mat<R>(g, params, false), lo,
                             lo + p.chunk_len);
        }
        // Publish the chunk: every wavefront waits until its own stores have
        // reached the L2 (a workgroup barrier alone does not wait for them),
        // then lane 0's device-scope release writes the L2 back once and
        // counts the chunk.  (A release in every wavefront writes the L2 back
        // eight times: a 256-circuit batch of width 16 ran 2.95 ms against
        // 2.15 ms this way.)
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Angles of the parameterised gates inside fused runs, into their tile
// descriptors (matrix, and phases of diagonal ones).
__global__ void k_batch_tile_params(const BTileJob *__restrict__ jobs, int njobs, const double *__restrict__ params,
                                    TileGate *__restrict__ tiles, SweepMember *__restrict__ mems) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= njobs)
        return;
    const BTileJob j = jobs[i];
    double m[8];
    gate_matrix(j.kind, params[j.param], nullptr, m);
    TileGate &t = tiles[j.tile];
    for (int k = 0; k < 8; ++k)
        t.m[k] = m[k];
    if (t.diag) {
        diag_phases(m, t.ph, &t.unit);
        for (int s = 0; s < 2; ++s)  // the phase-sweep members holding ph (forward plans)
            if (mems && t.mem[s] >= 0)
                mems[t.mem[s]].theta = t.ph[s];
    }
}

// Work items: items[i] is a circuit; a circuit split over workgroups appears
// once per workgroup that may join it.
template <typename R>
__global__ __launch_bounds__(kBatchThreads, 4) void k_batched(const BCirc *__restrict__ circs,
                                                           const int32_t *__restrict__ items, int nitems,
                                                           const BGate *__restrict__ gates,
                                                           const BPass *__restrict__ passes,
                                                           const TileGate *__restrict__ tiles,
                                                           const SweepPat *__restrict__ pats,
                                                           const SweepMember *__restrict__ mems,
                                                           const double *__restrict__ params,
                                                           unsigned int *__restrict__ queue,
                                                           unsigned int *gstate, uint64_t limit,
                                                           unsigned int *err, uint64_t *__restrict__ stamps) {
    extern __shared__ unsigned char lds_raw[];
    int *item = reinterpret_cast<int *>(lds_raw);
    int *ticket = item + 1;
    cplx_t<R> *lds = reinterpret_cast<cplx_t<R> *>(lds_raw + kBatchSlot);
    for (;;) {
        if (threadIdx.x == 0)
            *item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int it = *item;
        __syncthreads();
        if (it >= nitems)
            break;
        const uint64_t t0 = stamps ? wall_clock64() : 0;
        const BCirc &c = circs[items[it]];
        if (c.group >= 0)  // uniform
            run_circuit_split<R>(c, gates, passes, tiles, pats, mems, params, gstate, limit, err, lds, ticket);
        else
            run_circuit_block<R>(c, gates, passes, tiles, pats, mems, params, lds);
        __syncthreads();
        if (stamps && threadIdx.x == 0) {
            stamps[2 * it] = t0;
            stamps[2 * it + 1] = wall_clock64();
        }
    }
}

__global__ void k_zero_u32(unsigned int *p) { *p = 0u; }

__global__ void k_zero_words(unsigned int *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        p[i] = 0u;
}

// ----------------------------------------------------------------- adjoint

// One gate of the reverse sweep over the whole state in global memory:
// gradient term (when parameterised) and un-apply on psi and lambda.
template <typename R, int THREADS>
__device__ void adj_gate_global(const BCirc &c, const BGate &g, int gs, const double *__restrict__ params,
                                const double *__restrict__ gens, cplx_t<R> *psi, cplx_t<R> *lam,
                                double *__restrict__ grad, double *scratch) {
    const Mat2<R> ud = bgate_mat<R>(g, params, true);
    double a[8];
    for (int k = 0; k < 8; ++k)
        a[k] = gs >= 0 ? gens[8 * gs + k] : 0.0;
    const uint64_t pos = g.cmask | (1ull << g.target);
    const uint64_t npairs = 1ull << (c.n - 1 - __popcll(g.cmask));
    const uint64_t st = 1ull << g.target;
    double acc = 0.0;
    for (uint64_t it = threadIdx.x; it < npairs; it += THREADS) {
        const uint64_t p1 = insert_bits<uint64_t>(it, pos, g.cvals);
        cplx_t<R> x = psi[p1], y = psi[p1 | st], lx = lam[p1], ly = lam[p1 | st];
        if (gs >= 0) {
            const double xr = x.x, xi = x.y, yr = y.x, yi = y.y;
            const double axr = a[0] * xr - a[1] * xi + a[2] * yr - a[3] * yi;
            const double axi = a[0] * xi + a[1] * xr + a[2] * yi + a[3] * yr;
            const double ayr = a[4] * xr - a[5] * xi + a[6] * yr - a[7] * yi;
            const double ayi = a[4] * xi + a[5] * xr + a[6] * yi + a[7] * yr;
            acc += 2.0 * ((double)lx.x * axr + (double)lx.y * axi + (double)ly.x * ayr + (double)ly.y * ayi);
        }
        apply_pair<R>(ud, x, y);
        apply_pair<R>(ud, lx, ly);
        psi[p1] = x;
        psi[p1 | st] = y;
        lam[p1] = lx;
        lam[p1 | st] = ly;
    }
    if (gs >= 0) {  // uniform
        const double s = block_sum(acc, scratch);
        if (threadIdx.x == 0)
            grad[g.param] += s;
    }
    __syncthreads();
}

// One circuit's adjoint inside one workgroup: lambda = H psi (and the loss),
// then the reverse sweep: the fused plan of the inverse circuit, tiles of psi
// and lambda together in LDS (adj_tile_run, shared with the single-circuit
// adjoint), and single gates over global memory.  Gradient sums are reduced
// in a fixed order (per wavefront, then wavefronts in index order, then
// passes in order), so results are reproducible.
template <typename R, int THREADS>
__device__ void adjoint_block(const BCirc &c, const BGate *__restrict__ gates, const BPass *__restrict__ apasses,
                              const TileGate *__restrict__ atiles, const int32_t *__restrict__ atslot,
                              const int32_t *__restrict__ slot_param, const double *__restrict__ params,
                              const DTerm *__restrict__ terms, const double *__restrict__ gens,
                              const int32_t *__restrict__ gen_of, double *__restrict__ grad,
                              double *__restrict__ loss, double *scratch, unsigned char *dyn) {
    cplx_t<R> *psi = reinterpret_cast<cplx_t<R> *>(c.psi);
    cplx_t<R> *lam = reinterpret_cast<cplx_t<R> *>(c.lam);
    const uint64_t N = 1ull << c.n;
    for (int j = threadIdx.x; j < c.nparams; j += THREADS)
        grad[c.first_param + j] = 0.0;
    // lambda = H psi; terms are sorted by x mask
    double lp = 0.0;
    for (uint64_t k = threadIdx.x; k < N; k += THREADS) {
        double ar = 0.0, ai = 0.0;
        for (int j = 0; j < c.nterms; ++j) {
            const DTerm T = terms[c.first_term + j];
            const uint64_t X = (uint64_t)T.idx;  // the term's x mask (stored in idx for the batch)
            const uint64_t kx = k ^ X;
            const cplx_t<R> v = psi[kx];
            const double s = odd_parity(T.z & kx) ? -T.coef : T.coef;
            const double cr = re_ipow(T.ny, s, 0.0), ci = im_ipow(T.ny, s, 0.0);
            ar += cr * (double)v.x - ci * (double)v.y;
            ai += cr * (double)v.y + ci * (double)v.x;
        }
        cplx_t<R> o;
        o.x = (R)ar;
        o.y = (R)ai;
        lam[k] = o;
        const cplx_t<R> p = psi[k];
        lp += (double)p.x * ar + (double)p.y * ai;
    }
    const double L = block_sum(lp, scratch);
    if (threadIdx.x == 0)
        loss[0] = L;
    __syncthreads();
    cplx_t<R> *tp = reinterpret_cast<cplx_t<R> *>(dyn);
    for (int pi = 0; pi < c.napasses; ++pi) {
        const BPass &p = apasses[c.first_apass + pi];
        if (p.fused) {  // uniform
            const DeviceGates dg{atiles + p.first, p.count};
            const int32_t *gs = atslot + p.first;
            const uint32_t T = 1u << p.tm.m;
            cplx_t<R> *tl = tp + T;
            double *accl = reinterpret_cast<double *>(tl + T);
            const int npg = adj_acc_zero(dg, gs, accl);
            for (uint64_t tt = 0; tt < p.tm.ntiles; ++tt) {
                const uint64_t base = expand_index<uint64_t>(p.tm.outer, tt);
                if (!adj_tile_touched(base, dg))
                    continue;  // uniform
                tile_load_dma<R, THREADS>(tp, psi, base, p.tm, T);
                tile_load_dma<R, THREADS>(tl, lam, base, p.tm, T);
                __syncthreads();
                adj_tile_run<R, THREADS>(tp, tl, base, T, dg, gs, gens, accl);
                tile_store2<R, THREADS, false, kBatchCopy>(psi, lam, tp, tl, base, p.tm, T);
                __syncthreads();
            }
            if (threadIdx.x == 0)  // in order: gates may share a parameter
                for (int k = 0; k < npg; ++k)
                    grad[slot_param[adj_acc_slot(dg, gs, k)]] += adj_acc_sum(accl, k);
            __syncthreads();
        } else {
            const int f = p.gate;  // forward index of the gate un-applied here
            adj_gate_global<R, THREADS>(c, gates[c.first_gate + f], gen_of[c.first_gate + f], params, gens, psi, lam, grad,
                               scratch);
        }
    }
}

// THREADS = 512 (two workgroups per CU) or 1024 (one per CU, for batches of
// at most one circuit per CU: twice the wavefronts on each circuit).
template <typename R, int THREADS>
__global__ __launch_bounds__(THREADS, 2048 / THREADS) void k_batched_adjoint(
    const BCirc *__restrict__ circs, const int32_t *__restrict__ order, int ncirc, const BGate *__restrict__ gates,
    const BPass *__restrict__ apasses, const TileGate *__restrict__ atiles, const int32_t *__restrict__ atslot,
    const int32_t *__restrict__ slot_param, const double *__restrict__ params, const DTerm *__restrict__ terms,
    const double *__restrict__ gens, const int32_t *__restrict__ gen_of, double *__restrict__ grad,
    double *__restrict__ loss, unsigned int *__restrict__ queue, uint64_t *__restrict__ stamps) {
    extern __shared__ unsigned char lds_raw[];  // psi and lambda tiles, then gradient accumulators
    __shared__ double scratch[THREADS / 64];
    __shared__ int item;
    for (;;) {
        if (threadIdx.x == 0)
            item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int it = item;
        __syncthreads();
        if (it >= ncirc)
            break;
        const int ci = order[it];
        const uint64_t t0 = stamps ? wall_clock64() : 0;
        adjoint_block<R, THREADS>(circs[ci], gates, apasses, atiles, atslot, slot_param, params, terms, gens, gen_of, grad,
                         loss + ci, scratch, lds_raw);
        __syncthreads();
        if (stamps && threadIdx.x == 0) {
            stamps[2 * ci] = t0;
            stamps[2 * ci + 1] = wall_clock64();
        }
    }
}

// ----------------------------------------------------------------- host

// One circuit's tables, built independently of the others (so circuits can
// be planned in parallel) and concatenated afterwards.
struct CircBuild {
    BCirc bc;
    std::vector<BGate> gates;
    std::vector<BPass> passes;     // forward plan (circuit-local indices)
    std::vector<TileGate> tiles;
    std::vector<SweepPat> pats;    // phase patterns of the table sweeps (circuit-local)
    std::vector<SweepMember> mems;
    std::vector<BTileJob> jobs;    // tile indices circuit-local
    // adjoint: the reverse sweep's fused plan, each descriptor's generator
    // slot (circuit-local, -1 none), each slot's parameter (batch-global)
    std::vector<BPass> apasses;
    std::vector<TileGate> atiles;
    std::vector<BTileJob> ajobs;
    std::vector<int32_t> atslot, slot_param;
    size_t adj_lds = 0;            // dynamic LDS its fused passes need
    std::vector<double> gens;      // generators of the parameterised gates
    std::vector<int32_t> gen_of;   // per gate: index into gens / 8, or -1
    std::vector<DTerm> terms;
    double cost = 0.0;
    int err = SV_OK;
    std::string msg;
};

struct BatchArgs {
    const sv_state_t *states, *lams;
    int ncirc;
    const sv_gate_t *gates;
    const int64_t *gate_off, *param_off;
    int64_t nparams_total;
    const sv_pauli_t *terms;
    const int64_t *term_off;
};

// Tables of circuit c: its gates in program order, and either the forward
// fused plan (passes, tile descriptors, parameter jobs; none when the state
// is LDS-resident) or, for the adjoint, generators and the Hamiltonian.
static int build_circuit(const BatchArgs &A, int c, int dtype, bool adjoint, CircBuild *out) {
    const sv_state_t &s = A.states[c];
    const int64_t g0 = A.gate_off[c], g1 = A.gate_off[c + 1];
    const int64_t p0 = A.param_off ? A.param_off[c] : 0, p1 = A.param_off ? A.param_off[c + 1] : 0;
    BCirc &bc = out->bc;
    memset(&bc, 0, sizeof(bc));
    bc.group = -1;
    bc.psi = s.data;
    bc.lam = adjoint ? A.lams[c].data : nullptr;
    bc.n = s.n;
    // the fused tiles must fit the workgroup's LDS buffer
    const int m_cap = dtype == SV_C128 ? 12 : 13;  // 2^m amplitudes <= kBatchLds bytes
    const int tl = tuning().tile_log2[dtype == SV_C128 ? 0 : 1];
    bc.m = std::min(std::min(tl, s.n), m_cap);
    bc.ngates = (int32_t)(g1 - g0);
    bc.first_param = (int32_t)p0;
    bc.nparams = (int32_t)(p1 - p0);
    if (bc.ngates > 0) {
        for (int64_t i = g0; i < g1; ++i) {
            SV_TRY(validate_circuit_gate(s.n, (int)(p1 - p0), A.gates[i], (int)(i - g0)));
            if (adjoint)
                SV_TRY(validate_unitary_gate(A.gates[i], (int)(i - g0)));
        }
        const bool resident = ((size_t)1 << s.n) * amp_bytes(dtype) <= kBatchLds;
        if (!adjoint && !resident) {
            std::vector<PlanPass> pp;
            int m_used = 0;
            SV_TRY(circuit_plan_tiles(s.n, dtype, A.gates + g0, bc.ngates, (int)(p1 - p0), m_cap, &pp, &out->tiles,
                                      &m_used, &out->pats, &out->mems));
            if (m_used != bc.m)
                return fail(SV_EINVAL, "planner tile width %d != %d", m_used, bc.m);
            for (const PlanPass &q : pp) {
                BPass b;
                memset(&b, 0, sizeof(b));
                b.fused = q.fused;
                b.gate = q.gate;
                b.first = q.first;
                b.count = q.count;
                if (q.fused) {
                    if (q.tm.m > (uint32_t)m_cap)
                        return fail(SV_EINVAL, "tile width %u beyond the batch limit", q.tm.m);
                    b.tm = q.tm;
                    b.tm.tab = 1;  // the launch reserves the tables
                }
                out->passes.push_back(b);
            }
            for (size_t t = 0; t < out->tiles.size(); ++t) {
                const sv_gate_t &g = A.gates[g0 + out->tiles[t].src_gate];
                if (g.param >= 0)
                    out->jobs.push_back(BTileJob{g.kind, (int32_t)(p0 + g.param), (int32_t)t, 0});
            }
        }
    }
    bc.npasses = (int32_t)out->passes.size();
    double work = 0.0;
    out->gates.reserve(bc.ngates);
    for (int k = 0; k < bc.ngates; ++k) {
        const sv_gate_t &g = A.gates[g0 + k];
        BGate b;
        memset(&b, 0, sizeof(b));
        if (g.param < 0)
            gate_matrix(g.kind, g.theta, g.U, b.m);
        else
            for (int q = 0; q < 8; ++q)
                b.m[q] = g.U[q];
        b.kind = g.kind;
        b.param = g.param >= 0 ? (int32_t)(p0 + g.param) : -1;
        b.target = g.target;
        b.cmask = g.ctrl_mask;
        b.cvals = g.ctrl_vals;
        int gs = -1;
        if (adjoint && g.param >= 0) {
            double a[8];
            gate_generator(g.kind, a);
            if (g.kind & SV_G_ADJOINT) {
                for (int q = 1; q < 8; q += 2)
                    a[q] = -a[q];
                std::swap(a[2], a[4]);
                std::swap(a[3], a[5]);
            }
            gs = (int)(out->gens.size() / 8);
            out->gens.insert(out->gens.end(), a, a + 8);
            out->slot_param.push_back((int32_t)(p0 + g.param));
        }
        out->gen_of.push_back(gs);
        out->gates.push_back(b);
        work += std::ldexp(1.0, s.n - popcount64(g.ctrl_mask));
    }
    if (adjoint && bc.ngates > 0) {
        // the reverse sweep: inverses in reverse order, planned like a forward
        // circuit with two tiles (psi and lambda) in the LDS of one
        const int m_cap_adj = m_cap - 1;
        std::vector<sv_gate_t> rev(bc.ngates);
        for (int r = 0; r < bc.ngates; ++r) {
            rev[r] = A.gates[g0 + bc.ngates - 1 - r];
            rev[r].kind ^= SV_G_ADJOINT;
        }
        std::vector<PlanPass> pp;
        int m_used = 0;
        SV_TRY(circuit_plan_tiles(s.n, dtype, rev.data(), bc.ngates, (int)(p1 - p0), m_cap_adj, &pp, &out->atiles,
                                  &m_used));
        for (const PlanPass &q : pp) {
            BPass b;
            memset(&b, 0, sizeof(b));
            b.fused = q.fused;
            b.first = q.first;
            b.count = q.count;
            if (q.fused) {
                if (q.tm.m > (uint32_t)m_cap_adj)
                    return fail(SV_EINVAL, "tile width %u beyond the batch limit", q.tm.m);
                b.tm = q.tm;
                size_t npg = 0;
                for (int j = 0; j < q.count; ++j)
                    npg += out->gen_of[bc.ngates - 1 - out->atiles[q.first + j].src_gate] >= 0 ? 1 : 0;
                out->adj_lds = std::max(out->adj_lds, ((size_t)2 << q.tm.m) * amp_bytes(dtype) +
                                                          npg * (kBatchAdjMaxThreads / 64) * sizeof(double));
            } else {
                b.gate = bc.ngates - 1 - q.gate;  // forward index
            }
            out->apasses.push_back(b);
        }
        for (size_t t = 0; t < out->atiles.size(); ++t) {
            const int f = bc.ngates - 1 - out->atiles[t].src_gate;
            out->atslot.push_back(out->gen_of[f]);
            const sv_gate_t &g = A.gates[g0 + f];
            if (g.param >= 0)
                out->ajobs.push_back(BTileJob{g.kind ^ SV_G_ADJOINT, (int32_t)(p0 + g.param), (int32_t)t, 0});
        }
        bc.napasses = (int32_t)out->apasses.size();
    }
    if (adjoint) {
        const int64_t t0 = A.term_off[c], t1 = A.term_off[c + 1];
        if (t0 < 0 || t1 <= t0)
            return fail(SV_EINVAL, "needs at least one term");
        const uint64_t full = (1ull << s.n) - 1;
        bc.nterms = (int32_t)(t1 - t0);
        for (int64_t j = t0; j < t1; ++j) {
            if ((A.terms[j].x_mask | A.terms[j].z_mask) & ~full)
                return fail(SV_EINVAL, "term %lld acts on qubits >= n", (long long)(j - t0));
            DTerm d;
            d.coef = A.terms[j].coef;
            d.z = A.terms[j].z_mask;
            d.ny = popcount64(A.terms[j].x_mask & A.terms[j].z_mask) & 3;
            d.idx = (int32_t)A.terms[j].x_mask;  // x mask (n <= 31 in batches)
            out->terms.push_back(d);
        }
        work *= 2.0;
    }
    out->cost = work;
    return SV_OK;
}

struct BatchHost {
    std::vector<BCirc> circs;
    std::vector<BGate> gates;
    std::vector<BPass> passes;
    std::vector<TileGate> tiles;
    std::vector<SweepPat> pats;
    std::vector<SweepMember> mems;
    std::vector<BTileJob> jobs;
    std::vector<BPass> apasses;
    std::vector<TileGate> atiles;
    std::vector<BTileJob> ajobs;
    std::vector<int32_t> atslot, slot_param;
    size_t adj_lds = 0;
    std::vector<int32_t> order;    // work items in queue order (each a circuit)
    int ngroups = 0;               // circuits split over workgroups
    std::vector<double> gens;
    std::vector<int32_t> gen_of;
    std::vector<DTerm> terms;
};

// A chunk wait gives up after this long.  A chunk takes far less (its tiles
// or pair steps are bounded), so only a workgroup stalled from outside (the
// device preempted, a fault elsewhere) can reach it.
constexpr uint64_t kWaitLimitSeconds = 10;

// A circuit that costs more than the batch's mean load per workgroup is
// split into that many workgroups' worth of work items (at most the
// "batch_split" knob): else the widest circuits, started first, still run
// long after the rest of the batch is done.  A split circuit's passes are cut
// into chunk tickets of whole tiles (fused passes) or whole pair-loop steps
// (single gates), kChunksPerWorker per joining workgroup.  Measured on the
// 4096-circuit batch (widths 10-20): splitting also the circuits above a
// quarter or a half of the mean load, or into items of half of it, was
// slower, and so were 8 or 16 chunks per workgroup.
constexpr int kChunksPerWorker = 4;

static void split_circuits(BatchHost *h, const std::vector<double> &cost, std::vector<int32_t> *workers) {
    const int gmax = tuning().batch_split;
    if (gmax <= 1)
        return;
    DeviceInfo di;
    const double P = device_info(&di) == SV_OK ? 2.0 * di.num_cus : 512.0;  // persistent workgroups
    double W = 0.0;
    for (double c : cost)
        W += c;
    const double load = W / P;
    const int kc = kChunksPerWorker;
    for (size_t c = 0; c < h->circs.size(); ++c) {
        BCirc &bc = h->circs[c];
        if (bc.npasses == 0 || !(cost[c] > load))
            continue;  // LDS-resident, empty, or short enough
        const int g = (int)std::min<double>(gmax, std::ceil(cost[c] / load));
        if (g < 2 || (int64_t)bc.npasses * g * kc > (1 << 30))
            continue;
        int64_t k = 0;
        for (int pi = 0; pi < bc.npasses; ++pi) {
            BPass &p = h->passes[bc.first_pass + pi];
            uint64_t total, unit;
            if (p.fused) {
                total = p.tm.ntiles;
                unit = 1;
            } else {
                const BGate &gt = h->gates[bc.first_gate + p.gate];
                total = 1ull << (bc.n - 1 - popcount64(gt.cmask));
                unit = (uint64_t)kBatchPairUnroll * kBatchThreads;
            }
            const uint64_t steps = (total + unit - 1) / unit;
            const uint64_t want = std::max<uint64_t>(1, std::min<uint64_t>(steps, (uint64_t)g * kc));
            const uint64_t len = (steps + want - 1) / want * unit;
            p.chunk0 = (int32_t)k;
            p.nchunks = (int32_t)((total + len - 1) / len);
            p.chunk_len = len;
            k += p.nchunks;
        }
        bc.group = h->ngroups++;
        bc.nchunks = (int32_t)k;  // at most npasses * 4 * 64
        (*workers)[c] = g;
    }
}

// Checks the batch description, plans every circuit (in parallel over host
// threads for large batches) and concatenates the tables; circuits are
// ordered by decreasing cost per workgroup for the work queue.
static int build_batch(const BatchArgs &A, bool adjoint, BatchHost *h, int *dtype) {
    if (A.ncirc < 1 || !A.states || !A.gate_off || (A.gate_off[A.ncirc] > 0 && !A.gates))
        return fail(SV_EINVAL, "bad batch description (ncirc %d)", A.ncirc);
    if (adjoint && (!A.term_off || !A.terms || !A.lams || !A.param_off))
        return fail(SV_EINVAL, "batched adjoint needs lambda states, param offsets, terms and term offsets");
    *dtype = A.states[0].dtype;
    int64_t total_gates = 0;
    for (int c = 0; c < A.ncirc; ++c) {
        const sv_state_t &s = A.states[c];
        int r = validate_state(&s);
        if (r != SV_OK)
            return fail(r, "circuit %d: %s", c, sv_last_error());
        if (s.dtype != *dtype)
            return fail(SV_EINVAL, "circuit %d: all states of a batch need one dtype", c);
        if (adjoint) {
            r = validate_state(&A.lams[c]);
            if (r != SV_OK)
                return fail(r, "circuit %d (lambda): %s", c, sv_last_error());
            if (A.lams[c].n != s.n || A.lams[c].dtype != s.dtype || A.lams[c].data == s.data)
                return fail(SV_EINVAL, "circuit %d: lambda must be a distinct state of the same shape", c);
            if (s.n > 31)
                return fail(SV_EINVAL, "circuit %d: batched adjoint supports n <= 31", c);
        }
        const int64_t g0 = A.gate_off[c], g1 = A.gate_off[c + 1];
        if (g0 < 0 || g1 < g0 || g1 - g0 > INT32_MAX)
            return fail(SV_EINVAL, "circuit %d: bad gate offsets", c);
        const int64_t p0 = A.param_off ? A.param_off[c] : 0, p1 = A.param_off ? A.param_off[c + 1] : 0;
        if (p0 < 0 || p1 < p0 || p1 > A.nparams_total)
            return fail(SV_EINVAL, "circuit %d: bad parameter offsets", c);
        total_gates += g1 - g0;
    }
    if (total_gates > INT32_MAX)
        return fail(SV_EINVAL, "batch holds %lld gates (at most 2^31 - 1)", (long long)total_gates);
    std::vector<CircBuild> cb(A.ncirc);
    auto work = [&](int lo, int hi) {
        for (int c = lo; c < hi; ++c) {
            CircBuild &b = cb[c];
            b.err = build_circuit(A, c, *dtype, adjoint, &b);
            if (b.err != SV_OK) {
                b.msg = sv_last_error();  // error text is per thread
                return;
            }
        }
    };
    unsigned nth = std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
    if (total_gates < 20000)
        nth = 1;
    nth = std::min<unsigned>(nth, (unsigned)A.ncirc);
    if (nth <= 1) {
        work(0, A.ncirc);
    } else {
        int dev = 0;
        const bool have_dev = hipGetDevice(&dev) == hipSuccess;
        std::vector<std::thread> pool;
        std::atomic<int> next{0};
        constexpr int kChunk = 16;
        for (unsigned t = 0; t < nth; ++t)
            pool.emplace_back([&, have_dev, dev] {
                if (have_dev)
                    (void)hipSetDevice(dev);  // planner queries use the caller's device
                for (;;) {
                    const int lo = next.fetch_add(kChunk);
                    if (lo >= A.ncirc)
                        break;
                    work(lo, std::min(A.ncirc, lo + kChunk));
                }
            });
        for (auto &t : pool)
            t.join();
    }
    std::vector<double> cost(A.ncirc);
    for (int c = 0; c < A.ncirc; ++c) {
        CircBuild &b = cb[c];
        if (b.err != SV_OK)
            return fail(b.err, "circuit %d: %s", c, b.msg.c_str());
        b.bc.first_gate = (int32_t)h->gates.size();
        b.bc.first_term = (int32_t)h->terms.size();
        b.bc.first_pass = (int32_t)h->passes.size();
        const int32_t tbase = (int32_t)h->tiles.size();
        for (BPass p : b.passes) {
            if (p.fused)
                p.first += tbase;
            h->passes.push_back(p);
        }
        for (BTileJob j : b.jobs) {
            j.tile += tbase;
            h->jobs.push_back(j);
        }
        // phase patterns: rebase the descriptors' and patterns' indices
        const uint32_t pbase = (uint32_t)h->pats.size(), mbase = (uint32_t)h->mems.size();
        for (TileGate t : b.tiles) {
            if (t.diag) {
                t.pat0 += pbase;
                for (int s = 0; s < 2; ++s)
                    if (t.mem[s] >= 0)
                        t.mem[s] += (int32_t)mbase;
            }
            h->tiles.push_back(t);
        }
        for (SweepPat p : b.pats) {
            p.first += mbase;
            h->pats.push_back(p);
        }
        h->mems.insert(h->mems.end(), b.mems.begin(), b.mems.end());
        const int32_t gbase = (int32_t)(h->gens.size() / 8);  // generator slots before this circuit's
        b.bc.first_apass = (int32_t)h->apasses.size();
        const int32_t abase = (int32_t)h->atiles.size();
        for (BPass p : b.apasses) {
            if (p.fused)
                p.first += abase;
            h->apasses.push_back(p);
        }
        for (BTileJob j : b.ajobs) {
            j.tile += abase;
            h->ajobs.push_back(j);
        }
        h->atiles.insert(h->atiles.end(), b.atiles.begin(), b.atiles.end());
        for (int32_t sl : b.atslot)
            h->atslot.push_back(sl >= 0 ? sl + gbase : -1);
        h->slot_param.insert(h->slot_param.end(), b.slot_param.begin(), b.slot_param.end());
        h->adj_lds = std::max(h->adj_lds, b.adj_lds);
        for (int32_t g : b.gen_of)
            h->gen_of.push_back(g >= 0 ? g + gbase : -1);
        h->gates.insert(h->gates.end(), b.gates.begin(), b.gates.end());
        h->gens.insert(h->gens.end(), b.gens.begin(), b.gens.end());
        h->terms.insert(h->terms.end(), b.terms.begin(), b.terms.end());
        h->circs.push_back(b.bc);
        cost[c] = b.cost;
    }
    std::vector<int32_t> workers(A.ncirc, 1);
    if (!adjoint)
        split_circuits(h, cost, &workers);
    std::vector<int32_t> circ(A.ncirc);
    std::iota(circ.begin(), circ.end(), 0);
    std::stable_sort(circ.begin(), circ.end(),
                     [&](int a, int b) { return cost[a] / workers[a] > cost[b] / workers[b]; });
    for (int c : circ)
        h->order.insert(h->order.end(), (size_t)workers[c], c);
    return SV_OK;
}

struct BatchDevice {
    BCirc *circs = nullptr;
    BGate *gates = nullptr;
    BPass *passes = nullptr;
    TileGate *tiles = nullptr;
    SweepPat *pats = nullptr;
    SweepMember *mems = nullptr;
    BTileJob *jobs = nullptr;
    int njobs = 0;
    BPass *apasses = nullptr;
    TileGate *atiles = nullptr;
    BTileJob *ajobs = nullptr;
    int najobs = 0;
    int32_t *atslot = nullptr, *slot_param = nullptr;
    size_t adj_lds = 0;
    int32_t *order = nullptr, *gen_of = nullptr;
    int nitems = 0;
    double *gens = nullptr;
    DTerm *terms = nullptr;
    unsigned int *queue = nullptr;
    // split circuits: two ticket counters each, then the count of waits
    // that timed out
    unsigned int *gstate = nullptr;
    int ngroups = 0;
    uint64_t wait_limit = 0;  // clock ticks
};

// Stream-ordered release when async (after the kernels enqueued on st),
// otherwise an immediate free.
static void batch_release(BatchDevice *d, bool async, hipStream_t st) {
    void *ps[] = {d->circs,  d->gates,  d->passes, d->tiles,  d->pats, d->mems, d->jobs,  d->apasses,
                  d->atiles, d->ajobs,  d->atslot, d->slot_param, d->order, d->gen_of, d->gens,    d->terms,
                  d->queue, d->gstate};
    for (void *p : ps)
        if (p)
            (void)(async ? hipFreeAsync(p, st) : hipFree(p));
    *d = BatchDevice();
}

template <typename T>
static int dev_copy(T **dst, const std::vector<T> &src, bool async, hipStream_t st, size_t min_count = 0) {
    const size_t cnt = std::max(src.size(), min_count);
    *dst = nullptr;
    if (cnt == 0)
        return SV_OK;
    hipError_t e = async ? hipMallocAsync((void **)dst, cnt * sizeof(T), st) : hipMalloc((void **)dst, cnt * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return fail(SV_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    if (!src.empty()) {
        if (async)
            SV_HIP_TRY(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st));
        else
            SV_HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    }
    return SV_OK;
}

static int upload_batch(const BatchHost &h, bool async, hipStream_t st, BatchDevice *d) {
    int r = dev_copy(&d->circs, h.circs, async, st);
    if (r == SV_OK)
        r = dev_copy(&d->gates, h.gates, async, st, 1);
    if (r == SV_OK)
        r = dev_copy(&d->passes, h.passes, async, st, 1);
    if (r == SV_OK)
        r = dev_copy(&d->tiles, h.tiles, async, st, 1);
    if (r == SV_OK)
        r = dev_copy(&d->pats, h.pats, async, st, 1);
    if (r == SV_OK)
        r = dev_copy(&d->mems, h.mems, async, st, 1);
    if (r == SV_OK)
        r = dev_copy(&d->jobs, h.jobs, async, st, 1);
    d->njobs = (int)h.jobs.size();
    if (r == SV_OK)
        r = dev_copy(&d->apasses, h.apasses, async, st, 1);
    if (r == SV_OK)
        r = dev_copy(&d->atiles, h.atiles, async, st, 1);
    if (r == SV_OK)
        r = dev_copy(&d->ajobs, h.ajobs, async, st, 1);
    d->najobs = (int)h.ajobs.size();
    if (r == SV_OK)
        r = dev_copy(&d->atslot, h.atslot, async, st, 1);
    if (r == SV_OK)
        r = dev_copy(&d->slot_param, h.slot_param, async, st, 1);
    d->adj_lds = h.adj_lds;
    if (r == SV_OK)
        r = dev_copy(&d->order, h.order, async, st);
    d->nitems = (int)h.order.size();
    if (r == SV_OK)
        r = dev_copy(&d->gen_of, h.gen_of, async, st, 1);
    if (r == SV_OK)
        r = dev_copy(&d->gens, h.gens, async, st, 8);
    if (r == SV_OK)
        r = dev_copy(&d->terms, h.terms, async, st, 1);
    if (r == SV_OK) {
        hipError_t e = async ? hipMallocAsync((void **)&d->queue, sizeof(unsigned int), st)
                             : hipMalloc((void **)&d->queue, sizeof(unsigned int));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            d->queue = nullptr;
            r = fail(SV_ENOMEM, "device allocation failed");
        }
    }
    d->ngroups = h.ngroups;
    if (r == SV_OK && h.ngroups > 0) {
        const int words = 2 * h.ngroups + 1;
        hipError_t e = async ? hipMallocAsync((void **)&d->gstate, words * sizeof(unsigned int), st)
                             : hipMalloc((void **)&d->gstate, words * sizeof(unsigned int));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            d->gstate = nullptr;
            r = fail(SV_ENOMEM, "device allocation failed");
        } else {
            hipLaunchKernelGGL(k_zero_words, dim3((words + 255) / 256), dim3(256), 0, st, d->gstate, words);
            if (!async)
                r = hipStreamSynchronize(st) == hipSuccess ? SV_OK : fail(SV_EHIP, "clearing the batch counters failed");
            int dev = 0, khz = 0;
            if (r == SV_OK && (hipGetDevice(&dev) != hipSuccess ||
                               hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
                               khz <= 0))
                r = fail(SV_EHIP, "device reports no constant-rate clock");
            d->wait_limit = (uint64_t)khz * 1000ull * kWaitLimitSeconds;
        }
    }
    if (r != SV_OK)
        batch_release(d, async, st);
    return r;
}

static unsigned persistent_grid(int ncirc) {
    DeviceInfo di;
    if (device_info(&di) != SV_OK)
        return 256;
    const unsigned g = (unsigned)di.num_cus * 2;  // two 512-lane workgroups per CU
    return std::min<unsigned>(g, (unsigned)ncirc);
}

static int launch_forward(int dtype, const BatchDevice &d, int ncirc, const double *params, hipStream_t s,
                          uint64_t *stamps = nullptr) {
    hipError_t a = dtype == SV_C128 ? hipFuncSetAttribute((const void *)k_batched<double>,
                                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                                          (int)kBatchDynLds)
                                    : hipFuncSetAttribute((const void *)k_batched<float>,
                                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                                          (int)kBatchDynLds);
    if (a != hipSuccess)
        return fail(SV_EHIP, "LDS limit: %s", hipGetErrorString(a));
    (void)ncirc;
    const unsigned grid = persistent_grid(d.nitems);
    if (d.njobs > 0)
        hipLaunchKernelGGL(k_batch_tile_params, dim3((d.njobs + 255) / 256), dim3(256), 0, s, d.jobs, d.njobs, params,
                           d.tiles, d.mems);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, d.queue);
    if (d.ngroups > 0)  // the ticket counters, not the timeout count after them
        hipLaunchKernelGGL(k_zero_words, dim3((2 * d.ngroups + 255) / 256), dim3(256), 0, s, d.gstate,
                           2 * d.ngroups);
    unsigned int *err = d.gstate ? d.gstate + 2 * d.ngroups : nullptr;
    if (dtype == SV_C128)
        hipLaunchKernelGGL(k_batched<double>, dim3(grid), dim3(kBatchThreads), kBatchDynLds, s, d.circs, d.order,
                           d.nitems, d.gates, d.passes, d.tiles, d.pats, d.mems, params, d.queue, d.gstate,
                           d.wait_limit, err, stamps);
    else
        hipLaunchKernelGGL(k_batched<float>, dim3(grid), dim3(kBatchThreads), kBatchDynLds, s, d.circs, d.order,
                           d.nitems, d.gates, d.passes, d.tiles, d.pats, d.mems, params, d.queue, d.gstate,
                           d.wait_limit, err, stamps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(SV_EHIP, "batched launch failed: %s", hipGetErrorString(e));
    return SV_OK;
}

template <typename R, int THREADS>
static int go_adjoint(const BatchDevice &d, int ncirc, unsigned grid, size_t lds, const double *params, double *grad,
                      double *loss, hipStream_t s, uint64_t *stamps) {
    hipError_t a = hipFuncSetAttribute((const void *)k_batched_adjoint<R, THREADS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (a != hipSuccess)
        return fail(SV_EHIP, "LDS limit: %s", hipGetErrorString(a));
    hipLaunchKernelGGL((k_batched_adjoint<R, THREADS>), dim3(grid), dim3(THREADS), lds, s, d.circs, d.order, ncirc,
                       d.gates, d.apasses, d.atiles, d.atslot, d.slot_param, params, d.terms, d.gens, d.gen_of, grad,
                       loss, d.queue, stamps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(SV_EHIP, "batched adjoint launch failed: %s", hipGetErrorString(e));
    return SV_OK;
}

// A batch of at most one circuit per CU runs one 1024-lane workgroup per
// circuit (two 512-lane ones per CU would leave half the workgroups idle);
// larger batches run two 512-lane workgroups per CU.
static int launch_adjoint(int dtype, const BatchDevice &d, int ncirc, const double *params, double *grad,
                          double *loss, hipStream_t s, uint64_t *stamps = nullptr) {
    constexpr size_t kLdsPerWorkgroup = 160 * 1024;  // gfx950, with the opt-in limit raised
    const size_t lds = std::max<size_t>(d.adj_lds, 8);
    if (lds + 1024 > kLdsPerWorkgroup)
        return fail(SV_ENOTSUP, "a fused reverse pass needs %zu bytes of LDS", lds);
    DeviceInfo di;
    const int cus = device_info(&di) == SV_OK ? di.num_cus : 256;
    const bool wide = ncirc <= cus;
    const unsigned grid = wide ? (unsigned)std::max(1, ncirc) : persistent_grid(ncirc);
    if (d.najobs > 0)
        hipLaunchKernelGGL(k_batch_tile_params, dim3((d.najobs + 255) / 256), dim3(256), 0, s, d.ajobs, d.najobs,
                           params, d.atiles, nullptr);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, d.queue);
    if (dtype == SV_C128)
        return wide ? go_adjoint<double, kBatchAdjMaxThreads>(d, ncirc, grid, lds, params, grad, loss, s, stamps)
                    : go_adjoint<double, kBatchThreads>(d, ncirc, grid, lds, params, grad, loss, s, stamps);
    return wide ? go_adjoint<float, kBatchAdjMaxThreads>(d, ncirc, grid, lds, params, grad, loss, s, stamps)
                : go_adjoint<float, kBatchThreads>(d, ncirc, grid, lds, params, grad, loss, s, stamps);
}

} // namespace sv

// A planned batch resident on one device (the C ABI's opaque sv_batch_t).
struct sv_batch {
    int dtype = 0, ncirc = 0, device = 0;
    int64_t nparams_total = 0;
    bool has_adjoint = false;
    sv::BatchDevice fwd, adj;
    std::vector<int32_t> items; // the forward run's work items (circuits), in queue order
    hipEvent_t done = nullptr;  // end of the last run
    uint64_t *stamps = nullptr; // per-circuit start/end clock of later runs (measurement), or none
};

using namespace sv;

extern "C" {

int sv_batch_create(const sv_state_t *states, const sv_state_t *lam_states, int ncirc, const sv_gate_t *gates,
                    const int64_t *gate_offsets, const int64_t *param_offsets, int64_t nparams_total,
                    const sv_pauli_t *terms, const int64_t *term_offsets, sv_batch_t **out) {
    clear_error();
    if (!out)
        return fail(SV_EINVAL, "out is NULL");
    *out = nullptr;
    const bool adj = lam_states != nullptr;
    BatchArgs A{states, lam_states, ncirc, gates, gate_offsets, param_offsets, nparams_total, terms, term_offsets};
    BatchHost hf, ha;
    int dtype = 0;
    SV_TRY(build_batch(A, false, &hf, &dtype));
    if (adj)
        SV_TRY(build_batch(A, true, &ha, &dtype));
    sv_batch *b = new sv_batch();
    b->dtype = dtype;
    b->ncirc = ncirc;
    b->nparams_total = nparams_total;
    b->has_adjoint = adj;
    int r = hipGetDevice(&b->device) == hipSuccess ? SV_OK : fail(SV_EHIP, "no current device");
    b->items = hf.order;
    if (r == SV_OK)
        r = upload_batch(hf, false, nullptr, &b->fwd);
    if (r == SV_OK && adj)
        r = upload_batch(ha, false, nullptr, &b->adj);
    if (r != SV_OK) {
        batch_release(&b->fwd, false, nullptr);
        batch_release(&b->adj, false, nullptr);
        delete b;
        return r;
    }
    *out = b;
    return SV_OK;
}

static int batch_check(sv_batch_t *b, const double *params_dev) {
    if (!b)
        return fail(SV_EINVAL, "batch is NULL");
    if (b->nparams_total > 0 && !params_dev)
        return fail(SV_EINVAL, "params_dev is NULL");
    int dev = 0;
    SV_HIP_TRY(hipGetDevice(&dev));
    if (dev != b->device)
        return fail(SV_EINVAL, "batch was created on device %d, current device is %d", b->device, dev);
    return SV_OK;
}

static int batch_done(sv_batch_t *b, hipStream_t st) {
    if (!b->done)
        SV_HIP_TRY(hipEventCreateWithFlags(&b->done, hipEventDisableTiming));
    SV_HIP_TRY(hipEventRecord(b->done, st));
    return SV_OK;
}

int sv_batch_run(sv_batch_t *b, const double *params_dev, sv_stream_t st) {
    clear_error();
    SV_TRY(batch_check(b, params_dev));
    SV_TRY(launch_forward(b->dtype, b->fwd, b->ncirc, params_dev, (hipStream_t)st, b->stamps));
    return batch_done(b, (hipStream_t)st);
}

int sv_batch_adjoint(sv_batch_t *b, const double *params_dev, double *grad_dev, double *loss_dev, sv_stream_t st) {
    clear_error();
    SV_TRY(batch_check(b, params_dev));
    if (!b->has_adjoint)
        return fail(SV_EINVAL, "batch was created without lambda states and terms");
    if (!grad_dev || !loss_dev)
        return fail(SV_EINVAL, "grad_dev and loss_dev are required");
    SV_TRY(launch_adjoint(b->dtype, b->adj, b->ncirc, params_dev, grad_dev, loss_dev, (hipStream_t)st, b->stamps));
    return batch_done(b, (hipStream_t)st);
}

int sv_batch_set_timing(sv_batch_t *b, uint64_t *stamps_dev, double *ns_per_tick) {
    clear_error();
    if (!b)
        return fail(SV_EINVAL, "batch is NULL");
    b->stamps = stamps_dev;
    if (ns_per_tick) {
        int khz = 0;
        SV_HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device));
        if (khz <= 0)
            return fail(SV_EHIP, "device reports no constant-rate clock");
        *ns_per_tick = 1e6 / (double)khz;
    }
    return SV_OK;
}

int sv_batch_info(sv_batch_t *b, int64_t *nitems, int32_t *item_circuit, int64_t cap, uint64_t *wait_timeouts) {
    clear_error();
    if (!b)
        return fail(SV_EINVAL, "batch is NULL");
    const int64_t n = (int64_t)b->items.size();
    if (nitems)
        *nitems = n;
    if (item_circuit) {
        if (cap < n)
            return fail(SV_EINVAL, "item_circuit holds %lld entries, the batch has %lld items", (long long)cap,
                        (long long)n);
        std::copy(b->items.begin(), b->items.end(), item_circuit);
    }
    if (wait_timeouts) {
        *wait_timeouts = 0;
        if (b->fwd.ngroups > 0) {
            if (b->done)
                SV_HIP_TRY(hipEventSynchronize(b->done));
            unsigned int v = 0;
            SV_HIP_TRY(hipMemcpy(&v, b->fwd.gstate + 2 * b->fwd.ngroups, sizeof(v), hipMemcpyDeviceToHost));
            *wait_timeouts = v;
        }
    }
    return SV_OK;
}

int sv_batch_destroy(sv_batch_t *b) {
    clear_error();
    if (!b)
        return SV_OK;
    if (b->done) {
        (void)hipEventSynchronize(b->done);
        (void)hipEventDestroy(b->done);
    }
    batch_release(&b->fwd, false, nullptr);
    batch_release(&b->adj, false, nullptr);
    delete b;
    return SV_OK;
}

int sv_apply_circuits_batched(const sv_state_t *states, int ncirc, const sv_gate_t *gates, const int64_t *gate_offsets,
                              const double *params_dev, const int64_t *param_offsets, int64_t nparams_total,
                              sv_stream_t st) {
    clear_error();
    BatchArgs A{states, nullptr, ncirc, gates, gate_offsets, param_offsets, nparams_total, nullptr, nullptr};
    BatchHost h;
    int dtype = 0;
    SV_TRY(build_batch(A, false, &h, &dtype));
    if (nparams_total > 0 && !params_dev)
        return fail(SV_EINVAL, "params_dev is NULL");
    BatchDevice d;
    hipStream_t s = (hipStream_t)st;
    SV_TRY(upload_batch(h, true, s, &d));
    const int r = launch_forward(dtype, d, ncirc, params_dev, s);
    batch_release(&d, true, s);
    return r;
}

int sv_adjoint_grad_batched(const sv_state_t *psi_states, const sv_state_t *lam_states, int ncirc,
                            const sv_gate_t *gates, const int64_t *gate_offsets, const double *params_dev,
                            const int64_t *param_offsets, int64_t nparams_total, const sv_pauli_t *terms,
                            const int64_t *term_offsets, double *grad_dev, double *loss_dev, sv_stream_t st) {
    clear_error();
    if (!lam_states || !grad_dev || !loss_dev || !param_offsets)
        return fail(SV_EINVAL, "batched adjoint needs lambda states, param offsets, grad_dev and loss_dev");
    BatchArgs A{psi_states, lam_states, ncirc, gates, gate_offsets, param_offsets, nparams_total, terms,
                term_offsets};
    BatchHost h;
    int dtype = 0;
    SV_TRY(build_batch(A, true, &h, &dtype));
    if (nparams_total > 0 && !params_dev)
        return fail(SV_EINVAL, "params_dev is NULL");
    BatchDevice d;
    hipStream_t s = (hipStream_t)st;
    SV_TRY(upload_batch(h, true, s, &d));
    const int r = launch_adjoint(dtype, d, ncirc, params_dev, grad_dev, loss_dev, s);
    batch_release(&d, true, s);
    return r;
}

} // extern "C"
