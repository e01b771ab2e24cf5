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
constexpr int kTileMaxHigh = 10;  // qubits of S above the contiguous low block
// Phase patterns of one diagonal sweep: at most this many (their per-tile
// phases sit in LDS after the tables); a longer sweep is split.
constexpr int kSweepMaxPats = 512;
// pattern classes of a sweep: A, B, one per tile-local bit q >= 6 (R[q], or
// D in class 2), then the per-amplitude rest; one slot more for the end
constexpr int kSweepClassSlots = 12;

// A condition (j & lmask) == lvals on the tile-local index j under which the
// phases of the members [first, first + count) are added.
struct SweepPat {
    uint32_t lmask, lvals;
    uint32_t first, count;
};

// One phase of a diagonal gate in a sweep: theta is added where the tile's
// outer index bits satisfy (base & om) == ov (the gate's controls outside S,
// and its target bit when the target is outside S) and the pattern holds.
struct SweepMember {
    uint64_t om, ov;
    double theta;
    uint64_t pad;
};

struct TileGate {
    // The first 64 bytes hold what the loops over a run read for every gate,
    // so a gate costs one scalar load there (the descriptors of a long run
    // must also fit the scalar cache).
    uint64_t hi_mask;     // controls outside S (global bits; diagonal: all controls)
    uint64_t hi_vals;
    // diagonal gate split over the tile's qubit set S: controls outside S
    // (global bits; a tile predicate), controls inside S (tile-local bits)
    // and the target's tile-local bit, or -1 when the target is outside S
    // (pair gates use l_mask/l_vals for their tile-local controls too)
    uint64_t o_mask, o_vals;
    uint32_t diag;        // 1: diagonal gate applied elementwise
    uint32_t target;      // pair gate: tile-local bit; diagonal: global qubit
    uint32_t npairs;      // pair gate: 2^(m - 1 - in-tile controls); first gate of a
                          // diagonal sweep: its table summary (kSweep* bits)
    uint32_t fixed;       // in-tile control bits that must be 1
    uint32_t l_mask, l_vals;
    int32_t l_target;
    // first gate of a block of consecutive diagonal gates: the block's
    // length, and whether it is long enough and of unit modulus throughout
    // to add phases (bit 0); set on the host.  A pair gate with sweep_len 2
    // is applied together with the next gate over 4-amplitude cosets (see
    // mark_coset_pairs).
    uint16_t sweep_len, sweep_phase;
    // diagonal gate: phases of its two entries, and whether both have unit
    // modulus (then a sweep may add phases instead of multiplying factors)
    double ph[2];
    uint32_t unit;
    uint32_t nseg;        // pair gate: in-tile expansion of the reduced index
    double m[8];          // matrix (a, b, c, d as re, im), double precision
    uint32_t shift[kTileSeg];
    uint32_t mask[kTileSeg];
    int32_t src_gate;     // index of the gate in its circuit (host bookkeeping)
    // first gate of a diagonal sweep that uses the phase tables: its first
    // phase pattern (an index into the run's pattern array) and the start of
    // each pattern class relative to it (see build_sweep_patterns)
    uint32_t pat0;
    uint32_t sweep_cls[kSweepClassSlots];
    // diagonal gate: the phase-pattern members that hold its phases ph[0]
    // and ph[1] (-1: none), refreshed with ph when the angle is a parameter
    int32_t mem[2];
    // first gate of a permutation run (see mark_permutation_runs): its length
    uint32_t perm_len;
    uint32_t pad3;
};

// Summary bits of a diagonal sweep's gates (host), kept in the first gate's
// npairs: bits 0-5 um and 8-13 uv (the common condition on u of R-type
// gates), and flags.
constexpr uint32_t kSweepHaveR = 1u << 16, kSweepRank1 = 1u << 17, kSweepAnyRest = 1u << 18,
                   kSweepInfoValid = 1u << 31;

// Mark the blocks of consecutive diagonal gates among tiles[0 .. count) (one
// fused run; host): length, phase-sum eligibility (unit modulus and at least
// phase_min gates reading tile-local bits) and table summary at each block's
// first gate.  param_gate[i] != 0: the entries of gate i come from parameters
// at run time (their kinds are unitary), so it counts as unit modulus.
void mark_diag_sweeps(TileGate *tiles, int count, const char *param_gate, int phase_min);

// Phase patterns of the table sweeps among tiles[0 .. count) (one fused run
// over tiles of width m >= 7, after mark_diag_sweeps; host).  Every phase
// of a sweep's gates becomes a member of the pattern given by its tile-local
// condition (controls in S, and the target bit when the target is in S),
// with a predicate on the outer bits; gates with the same tile-local
// condition share one pattern.  Patterns are appended to pats sorted by
// class (A, B, R[q] or D, rest) in order of first appearance, members in
// gate order; the sweep's first gate gets pat0, sweep_cls and the table
// summary, and each gate the indices of its members.  A sweep with more
// than kSweepMaxPats patterns is split into several sweeps.
void build_sweep_patterns(TileGate *tiles, int count, int m, const char *param_gate, std::vector<SweepPat> &pats,
                          std::vector<SweepMember> &mems);

// Permutation runs among tiles[0 .. count) (one fused run; host): maximal
// runs of at least two consecutive pair gates whose matrix is exactly X
// (any controls).  Such a run maps basis states to basis states, so inside
// a tile it is one gather: amplitude j of the result is amplitude
// g_1(g_2(... g_L(j))) of the tile, each g flipping its target bit where
// its controls hold (outer controls decide per tile).  One LDS read and
// write of the tile then replace one per gate.  A run is marked only when
// its gates together touch at least 1.5 tiles' worth of amplitudes (a gate
// with c tile-local controls touches 2^-c of the tile), where one gather
// moves less than the gates would.  The first gate gets perm_len.
void mark_permutation_runs(TileGate *tiles, int count);

// Mark coset pairs among tiles[0 .. count) (one fused run; host): two
// adjacent pair gates on different tile-local targets t1, t2 whose
// tile-local controls lie only on the other gate's target.  Every coset
// {b, b + 2^t1, b + 2^t2, b + 2^t1 + 2^t2} is then closed under both gates,
// so one LDS read and write of its four amplitudes applies both, with the
// same pair arithmetic in the same order as two separate loops.  The first
// gate of a pair gets sweep_len = 2; pairs do not overlap.
void mark_coset_pairs(TileGate *tiles, int count);

// Phases of the diagonal entries m[0..1] and m[6..7] (host and device).
__host__ __device__ inline void diag_phases(const double *m, double *ph, uint32_t *unit) {
    ph[0] = atan2(m[1], m[0]);
    ph[1] = atan2(m[7], m[6]);
    const double a = m[0] * m[0] + m[1] * m[1], b = m[6] * m[6] + m[7] * m[7];
    *unit = (fabs(a - 1.0) <= 1e-12 && fabs(b - 1.0) <= 1e-12) ? 1u : 0u;
}

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
    uint32_t tab;     // the launch reserves the diagonal-sweep tables after the tile
    uint32_t pad;
    uint64_t tile0;   // index of the launch's first tile (launches split at kMaxGridBlocks)
};

// Doubles of the diagonal-sweep tables for tile width m (0 below m = 7):
// A[64] over tile-local bits 0..5, B[2^(m-6)] over bits 6..m-1, for each
// bit q >= 6 and value b a row R[q][b][64] over bits 0..5, then the phases
// of up to kSweepMaxPats patterns for the current tile.
__host__ __device__ constexpr uint32_t diag_pattern_offset(uint32_t m) {
    return 64u + (1u << (m - 6)) + (m - 6) * 128u;
}
__host__ __device__ constexpr uint32_t diag_table_doubles(uint32_t m) {
    return m < 7 ? 0u : diag_pattern_offset(m) + (uint32_t)kSweepMaxPats;
}

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
    // no phase patterns: sweeps take the per-amplitude path
    __device__ __forceinline__ const SweepPat *pats() const { return nullptr; }
    __device__ __forceinline__ const SweepMember *mems() const { return nullptr; }
};

// A run's descriptors in device memory, with the phase patterns of its
// table sweeps (null: sweeps take the per-amplitude path).
struct DeviceGates {
    const TileGate *g;
    int count;
    const SweepPat *p = nullptr;
    const SweepMember *mm = nullptr;
    __device__ __forceinline__ const TileGate &get(int i) const { return g[i]; }
    __device__ __forceinline__ int size() const { return count; }
    __device__ __forceinline__ const SweepPat *pats() const { return p; }
    __device__ __forceinline__ const SweepMember *mems() const { return mm; }
};

// sweep_len (low half) and sweep_phase (high half) read as one 32-bit word,
// which keeps the read a scalar load
__device__ __forceinline__ uint32_t sweep_word(const TileGate &g) {
    uint32_t w;
    __builtin_memcpy(&w, &g.sweep_len, sizeof(w));
    return __builtin_amdgcn_readfirstlane(w);
}

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

// Most expansion segments a pair loop holds in registers (the target plus up
// to four tile-local controls); a gate with more reads its expansion from
// the descriptor for every pair.
constexpr int kExpRegs = 6;

__device__ __forceinline__ uint64_t tile_offset(const TileMap &tm, uint32_t j) {
    uint64_t o = j & ((1u << tm.a) - 1);
    for (uint32_t s = 0; s < tm.nseg; ++s)
        o |= (uint64_t)(j & tm.seg_in[s]) << tm.seg_shift[s];
    return o;
}

// Copies between a state in global memory and tiles in LDS.  Each lane
// forms the addresses of NB amplitudes (kTileBatch by default) and issues
// all their loads before its first LDS write, so NB loads per lane are in
// flight instead of one (a loop of load, wait, write keeps a single one in
// flight and leaves the load phase latency-bound).  NT: nontemporal accesses (a
// pass streams the state once); without it the accesses may stay in the
// caches (small batched states).  With two states, both tiles are copied
// together (psi's and lambda's loads in flight at once).
constexpr int kTileBatch = 8;

template <typename R, bool NT>
__device__ __forceinline__ cplx_t<R> tile_ld(const cplx_t<R> *p) {
    if constexpr (NT)
        return ld_stream<R>(p);
    else
        return *p;
}

template <typename R, bool NT>
__device__ __forceinline__ void tile_st(cplx_t<R> *p, const cplx_t<R> &v) {
    if constexpr (NT)
        st_stream<R>(p, v);
    else
        *p = v;
}

template <typename R, int THREADS, bool NT = true, int NB = kTileBatch>
__device__ __forceinline__ void tile_load(cplx_t<R> *tile, const cplx_t<R> *psi, uint64_t base, const TileMap &tm,
                                          uint32_t T) {
    for (uint32_t j0 = threadIdx.x; j0 < T; j0 += NB * THREADS) {
        cplx_t<R> v[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const uint32_t j = j0 + u * THREADS;
            if (j < T)
                v[u] = tile_ld<R, NT>(psi + (base | tile_offset(tm, j)));
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const uint32_t j = j0 + u * THREADS;
            if (j < T)
                tile[j] = v[u];
        }
    }
}

template <typename R, int THREADS, bool NT = true, int NB = kTileBatch>
__device__ __forceinline__ void tile_store(cplx_t<R> *psi, const cplx_t<R> *tile, uint64_t base, const TileMap &tm,
                                           uint32_t T) {
    for (uint32_t j0 = threadIdx.x; j0 < T; j0 += NB * THREADS) {
        cplx_t<R> v[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const uint32_t j = j0 + u * THREADS;
            if (j < T)
                v[u] = tile[j];
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const uint32_t j = j0 + u * THREADS;
            if (j < T)
                tile_st<R, NT>(psi + (base | tile_offset(tm, j)), v[u]);
        }
    }
}

template <typename R, int THREADS, bool NT = true, int NB = kTileBatch>
__device__ __forceinline__ void tile_load2(cplx_t<R> *tp, cplx_t<R> *tl, const cplx_t<R> *psi, const cplx_t<R> *lam,
                                           uint64_t base, const TileMap &tm, uint32_t T) {
    constexpr int B = NB / 2;
    for (uint32_t j0 = threadIdx.x; j0 < T; j0 += B * THREADS) {
        cplx_t<R> v[B], w[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const uint32_t j = j0 + u * THREADS;
            if (j < T) {
                const uint64_t o = base | tile_offset(tm, j);
                v[u] = tile_ld<R, NT>(psi + o);
                w[u] = tile_ld<R, NT>(lam + o);
            }
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const uint32_t j = j0 + u * THREADS;
            if (j < T) {
                tp[j] = v[u];
                tl[j] = w[u];
            }
        }
    }
}

template <typename R, int THREADS, bool NT = true, int NB = kTileBatch>
__device__ __forceinline__ void tile_store2(cplx_t<R> *psi, cplx_t<R> *lam, const cplx_t<R> *tp, const cplx_t<R> *tl,
                                            uint64_t base, const TileMap &tm, uint32_t T) {
    constexpr int B = NB / 2;
    for (uint32_t j0 = threadIdx.x; j0 < T; j0 += B * THREADS) {
        cplx_t<R> v[B], w[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const uint32_t j = j0 + u * THREADS;
            if (j < T) {
                v[u] = tp[j];
                w[u] = tl[j];
            }
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const uint32_t j = j0 + u * THREADS;
            if (j < T) {
                const uint64_t o = base | tile_offset(tm, j);
                tile_st<R, NT>(psi + o, v[u]);
                tile_st<R, NT>(lam + o, w[u]);
            }
        }
    }
}

// A tile copied from the state into LDS by direct HBM-to-LDS loads (for
// kernels without registers to spare): each wavefront fills 1 KiB of the
// tile per instruction, lane l writing its bytes 16 l .. 16 l + 15 (one
// complex128 amplitude, or two adjacent complex64 ones, which lie in the
// tile's contiguous low block), so no register holds the data and all of a
// lane's loads are in flight together.  The caller's barrier waits for them.
// Tiles smaller than one wavefront's 1 KiB (T a power of two below 64 * 16 /
// sizeof(amplitude)) are copied by the plain loop instead.
template <typename R, int THREADS>
__device__ __forceinline__ void tile_load_dma(cplx_t<R> *tile, const cplx_t<R> *psi, uint64_t base, const TileMap &tm,
                                              uint32_t T) {
    constexpr uint32_t A = 16 / sizeof(cplx_t<R>);  // amplitudes per lane and load
    constexpr uint32_t CH = 64 * A;                 // amplitudes per wavefront and load
    if (T < CH) {  // uniform
        for (uint32_t j = threadIdx.x; j < T; j += THREADS)
            tile[j] = psi[base | tile_offset(tm, j)];
        return;
    }
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    for (uint32_t c0 = wave * CH; c0 < T; c0 += (THREADS / 64) * CH) {  // uniform per wavefront
        const uint32_t j = c0 + lane * A;
        __builtin_amdgcn_global_load_lds((const void *)(psi + (base | tile_offset(tm, j))),
                                         (__attribute__((address_space(3))) void *)(tile + c0), 16, 0, 0);
    }
}



// A wave-uniform double held in scalar registers.
__device__ __forceinline__ double uniform_f64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// sin and cos of a phase: quadrant reduction by pi/2 held as two doubles
// (their sum is pi/2 to about 1e-33), then Taylor polynomials on
// |r| <= pi/4 (the first omitted terms are below 1e-19).  The phases here are
// sums of gate phases, |theta| well below 2^20.
__device__ __forceinline__ void phase_sincos(double th, double *sn, double *cs) {
    constexpr double kPio2Hi = 1.5707963267948966;     // nearest double to pi/2
    constexpr double kPio2Lo = 6.123233995736766e-17;  // pi/2 - kPio2Hi
    const double k = rint(th * 0.63661977236758134);  // th / (pi/2)
    double r = fma(-k, kPio2Hi, th);
    r = fma(-k, kPio2Lo, r);
    const double r2 = r * r;
    // sin r = r (1 - r^2/3! + r^4/5! - ...), cos r = 1 - r^2/2! + r^4/4! - ...
    double ps = 1.0 / 355687428096000.0;  // 1/17!
    ps = fma(ps, -r2, 1.0 / 1307674368000.0);
    ps = fma(ps, -r2, 1.0 / 6227020800.0);
    ps = fma(ps, -r2, 1.0 / 39916800.0);
    ps = fma(ps, -r2, 1.0 / 362880.0);
    ps = fma(ps, -r2, 1.0 / 5040.0);
    ps = fma(ps, -r2, 1.0 / 120.0);
    ps = fma(ps, -r2, 1.0 / 6.0);
    ps = fma(ps, -r2, 1.0);
    const double s = r * ps;  // signs alternate through the -r2 factors
    double pc = 1.0 / 20922789888000.0;  // 1/16!
    pc = fma(pc, -r2, 1.0 / 87178291200.0);
    pc = fma(pc, -r2, 1.0 / 479001600.0);
    pc = fma(pc, -r2, 1.0 / 3628800.0);
    pc = fma(pc, -r2, 1.0 / 40320.0);
    pc = fma(pc, -r2, 1.0 / 720.0);
    pc = fma(pc, -r2, 1.0 / 24.0);
    pc = fma(pc, -r2, 1.0 / 2.0);
    pc = fma(pc, -r2, 1.0);
    const double c = pc;
    const int q = (int)((int64_t)k & 3);
    // th = r + q pi/2: rotate (c, s) by q quarter turns
    *sn = q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
    *cs = q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}

// Single-precision factor for complex64 states: the quadrant reduction stays
// in double precision, the polynomials (to r^9 / r^8, truncation below 3e-8
// on |r| <= pi/4) run in single precision.
__device__ __forceinline__ void phase_sincos_f(double th, float *sn, float *cs) {
    constexpr double kPio2Hi = 1.5707963267948966;
    constexpr double kPio2Lo = 6.123233995736766e-17;
    const double k = rint(th * 0.63661977236758134);
    double rd = fma(-k, kPio2Hi, th);
    rd = fma(-k, kPio2Lo, rd);
    const float r = (float)rd, r2 = r * r;
    float ps = 1.0f / 362880.0f;
    ps = fmaf(ps, -r2, 1.0f / 5040.0f);
    ps = fmaf(ps, -r2, 1.0f / 120.0f);
    ps = fmaf(ps, -r2, 1.0f / 6.0f);
    ps = fmaf(ps, -r2, 1.0f);
    const float s = r * ps;
    float pc = 1.0f / 40320.0f;
    pc = fmaf(pc, -r2, 1.0f / 720.0f);
    pc = fmaf(pc, -r2, 1.0f / 24.0f);
    pc = fmaf(pc, -r2, 1.0f / 2.0f);
    pc = fmaf(pc, -r2, 1.0f);
    const float c = pc;
    const int q = (int)((int64_t)k & 3);
    *sn = q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
    *cs = q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}

// exp(i th) in the state's precision.
template <typename R> __device__ __forceinline__ void phase_factor(double th, R *fr, R *fi);
template <> __device__ __forceinline__ void phase_factor<double>(double th, double *fr, double *fi) {
    phase_sincos(th, fi, fr);
}
template <> __device__ __forceinline__ void phase_factor<float>(double th, float *fr, float *fi) {
    phase_sincos_f(th, fi, fr);
}

// A sweep of consecutive diagonal gates [i, e) whose entries all have unit
// modulus: each amplitude is multiplied by exp(i theta), theta being the sum
// of the phases its index selects (a tile-uniform part plus the gates that
// read tile-local bits), accumulated in double precision.
template <typename R, int THREADS, typename Src>
__device__ __forceinline__ void diag_sweep_phases(cplx_t<R> *tile, uint64_t base, uint32_t T, const Src &gates,
                                                  int i, int e) {
    double th0 = 0.0;
    bool any_local = false;
    for (int q = i; q < e; ++q) {
        const TileGate &d = gates.get(q);
        if ((base & d.o_mask) != d.o_vals)
            continue;
        if (d.l_target >= 0 || d.l_mask) {
            any_local = true;
            continue;
        }
        th0 += ((base >> d.target) & 1ull) ? d.ph[1] : d.ph[0];
    }
    // eight amplitudes per lane at a time (named scalars, not an array), so
    // each gate's uniform checks and loads are shared by eight updates
    for (uint32_t j0 = threadIdx.x; j0 < T; j0 += 8 * THREADS) {
        double t0 = th0, t1 = th0, t2 = th0, t3 = th0, t4 = th0, t5 = th0, t6 = th0, t7 = th0;
        if (any_local) {  // uniform
            for (int q = i; q < e; ++q) {
                const TileGate &d = gates.get(q);
                if ((base & d.o_mask) != d.o_vals || (d.l_target < 0 && !d.l_mask))
                    continue;  // uniform
                const double p0 = uniform_f64(d.ph[0]), p1 = uniform_f64(d.ph[1]);
                const bool tin = d.l_target >= 0;
                const double pt = ((base >> d.target) & 1ull) ? p1 : p0;
                auto add = [&](double &t, uint32_t j) {
                    const double p = tin ? (((j >> d.l_target) & 1u) ? p1 : p0) : pt;
                    t += ((j & d.l_mask) == d.l_vals) ? p : 0.0;
                };
                add(t0, j0);
                add(t1, j0 + THREADS);
                add(t2, j0 + 2 * THREADS);
                add(t3, j0 + 3 * THREADS);
                add(t4, j0 + 4 * THREADS);
                add(t5, j0 + 5 * THREADS);
                add(t6, j0 + 6 * THREADS);
                add(t7, j0 + 7 * THREADS);
            }
        }
        auto put = [&](double t, uint32_t j) {
            if (j < T) {
                R fr, fi;
                phase_factor<R>(t, &fr, &fi);
                const cplx_t<R> v = tile[j];
                cplx_t<R> w;
                w.x = v.x * fr - v.y * fi;
                w.y = v.x * fi + v.y * fr;
                tile[j] = w;
            }
        };
        put(t0, j0);
        put(t1, j0 + THREADS);
        put(t2, j0 + 2 * THREADS);
        put(t3, j0 + 3 * THREADS);
        put(t4, j0 + 4 * THREADS);
        put(t5, j0 + 5 * THREADS);
        put(t6, j0 + 6 * THREADS);
        put(t7, j0 + 7 * THREADS);
    }
    __syncthreads();
}

// Long unit-modulus sweep with tables.  The host turned the sweep's gates
// into phase patterns (build_sweep_patterns): a pattern adds its members'
// phases where a condition on the tile-local index j holds, each member
// only in tiles whose outer bits satisfy its predicate.  Per tile, the
// wavefronts first sum each pattern's members that hold for this tile.
// Then with u = bits 0..5 of j and v = bits 6..m-1,
//   theta(j) = A[u] + B[v] + sum over q of R[q][bit q of v][u] + rest,
// where A collects the patterns reading only bits of u (or none), B those
// reading only bits of v, R[q] those reading bits of u and the single bit
// 6+q, and rest (evaluated per amplitude) those reading bits of u and two or
// more bits of v.  When every R-type pattern depends on u through one
// condition (u & um) == uv, their terms sum to [(u & um) == uv] * D[v] with
// a single table D instead of the m-6 tables R[q].  Patterns come sorted by
// table, so a wavefront building a table walks only that table's patterns;
// every walk is wave-uniform (scalar loads of the host's records).
template <typename R, int THREADS, typename Src>
__device__ __forceinline__ void diag_sweep_tables(cplx_t<R> *tile, double *tab, uint64_t base, uint32_t m,
                                                  const Src &gates, int i) {
    const uint32_t T = 1u << m;
    const int Hb = (int)m - 6;
    double *A = tab, *B = tab + 64, *Rt = tab + 64 + (1 << Hb);
    double *thp = tab + diag_pattern_offset(m);  // this tile's pattern phases
    // the wavefront index is uniform: keep it (and the pattern loops) scalar
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    constexpr int kWaves = THREADS / 64;
    const TileGate &g = gates.get(i);
    const uint32_t info = __builtin_amdgcn_readfirstlane(g.npairs);
    const uint32_t um = info & 63u, uv = (info >> 8) & 63u;
    const bool have_r = (info & kSweepHaveR) != 0, rank1 = (info & kSweepRank1) != 0;
    const bool any_rest = (info & kSweepAnyRest) != 0;
    const SweepPat *P = gates.pats() + __builtin_amdgcn_readfirstlane(g.pat0);
    const SweepMember *M = gates.mems();
    const uint32_t np = __builtin_amdgcn_readfirstlane(g.sweep_cls[3 + Hb]);
    // 1. pattern phases of this tile: one wavefront per pattern
    for (uint32_t p = (uint32_t)w; p < np; p += kWaves) {
        const uint32_t f = __builtin_amdgcn_readfirstlane(P[p].first);
        const uint32_t e = f + __builtin_amdgcn_readfirstlane(P[p].count);
        double s = 0.0;
        for (uint32_t k = f; k < e; ++k) {
            const SweepMember &mm = M[k];
            if ((base & mm.om) == mm.ov)  // uniform
                s += uniform_f64(mm.theta);
        }
        if (lane == 0)
            thp[p] = s;
    }
    __syncthreads();
    const bool use_d = have_r && rank1;
    // table tb: 0 = A, 1 = B, then D (use_d) or 2 + q = R[q] (R patterns of
    // several conditions); entries per lane: A 1, B and D ceil(2^Hb / 64)
    // (lanes beyond 2^Hb idle when Hb < 6), R 2.  D uses the R area.
    const uint32_t nb = 1u << Hb;
    const int ntab = 2 + (!have_r ? 0 : (use_d ? 1 : Hb));
    for (int tb = w; tb < ntab; tb += kWaves) {  // uniform per wavefront
        const bool dtab = use_d && tb == 2;
        const int ne = tb == 0 ? 1 : ((tb == 1 || dtab) ? (int)((nb + 63) / 64) : 2);
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
        // the tile-local index an entry stands for
        auto at = [&](int k) -> uint32_t {
            return tb == 0   ? (uint32_t)lane
                   : tb == 1 ? (uint32_t)(lane + 64 * k) << 6
                   : dtab    ? ((uint32_t)(lane + 64 * k) << 6) | uv
                             : (uint32_t)lane | ((uint32_t)k << (4 + tb));
        };
        const uint32_t c0 = __builtin_amdgcn_readfirstlane(g.sweep_cls[tb]);
        const uint32_t c1 = __builtin_amdgcn_readfirstlane(g.sweep_cls[tb + 1]);
        for (uint32_t p = c0; p < c1; ++p) {
            const uint32_t lm = __builtin_amdgcn_readfirstlane(P[p].lmask);
            const uint32_t lv = __builtin_amdgcn_readfirstlane(P[p].lvals);
            const double th = thp[p];
            acc0 += (at(0) & lm) == lv ? th : 0.0;
            if (ne > 1)
                acc1 += (at(1) & lm) == lv ? th : 0.0;
            if (ne > 2) {
                acc2 += (at(2) & lm) == lv ? th : 0.0;
                acc3 += (at(3) & lm) == lv ? th : 0.0;
            }
        }
        double *dst = tb == 0 ? A : tb == 1 ? B : Rt + (tb - 2) * 128;
        if ((tb != 1 && !dtab) || (uint32_t)lane < nb)
            dst[lane] = acc0;
        if (ne > 1)
            dst[lane + 64] = acc1;
        if (ne > 2) {
            dst[lane + 128] = acc2;
            dst[lane + 192] = acc3;
        }
    }
    __syncthreads();
    // When every term sits in A, B and D (no R tables, no per-amplitude
    // terms), the three phase tables become unit factors once per tile, in
    // the free part of the R area after D's phases, and an amplitude costs
    // two or three complex products instead of a sine and cosine.
    constexpr int kSlots = (int)(sizeof(cplx_t<R>) / sizeof(double));  // table slots per factor
    const int fbase = use_d ? (int)nb : 0;  // D's phases occupy Rt[0 .. nb)
    const bool factors = !any_rest && (use_d || !have_r) && fbase + kSlots * (64 + 2 * (int)nb) <= Hb * 128;
    if (factors) {  // uniform
        cplx_t<R> *FA = reinterpret_cast<cplx_t<R> *>(Rt + fbase);
        cplx_t<R> *FB = FA + 64, *FD = FB + nb;
        const uint32_t nf = 64 + (use_d ? 2 : 1) * nb;
        for (uint32_t k = threadIdx.x; k < nf; k += THREADS) {
            const double ph = k < 64 ? A[k] : (k < 64 + nb ? B[k - 64] : Rt[k - 64 - nb]);
            R fr, fi;
            phase_factor<R>(ph, &fr, &fi);
            cplx_t<R> f;
            f.x = fr;
            f.y = fi;
            FA[k] = f;  // FA, FB and FD are consecutive
        }
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < T; j += THREADS) {
            const uint32_t u = j & 63u, v = j >> 6;
            const cplx_t<R> a = FA[u], b = FB[v];
            cplx_t<R> f;
            f.x = a.x * b.x - a.y * b.y;
            f.y = a.x * b.y + a.y * b.x;
            if (use_d && ((u & um) == uv)) {
                const cplx_t<R> d = FD[v];
                const R fx = f.x * d.x - f.y * d.y;
                f.y = f.x * d.y + f.y * d.x;
                f.x = fx;
            }
            const cplx_t<R> x = tile[j];
            cplx_t<R> y;
            y.x = x.x * f.x - x.y * f.y;
            y.y = x.x * f.y + x.y * f.x;
            tile[j] = y;
        }
        __syncthreads();
        return;
    }
    const uint32_t r0 = __builtin_amdgcn_readfirstlane(g.sweep_cls[2 + Hb]);
    for (uint32_t j = threadIdx.x; j < T; j += THREADS) {
        const uint32_t u = j & 63u, v = j >> 6;
        double t = A[u] + B[v];
        if (use_d) {  // uniform
            t += ((u & um) == uv) ? Rt[v] : 0.0;
        } else if (have_r) {
            for (int q = 0; q < Hb; ++q)
                t += Rt[q * 128 + ((v >> q) & 1u) * 64 + u];
        }
        if (any_rest) {  // uniform
            for (uint32_t p = r0; p < np; ++p) {
                const uint32_t lm = __builtin_amdgcn_readfirstlane(P[p].lmask);
                const uint32_t lv = __builtin_amdgcn_readfirstlane(P[p].lvals);
                t += (j & lm) == lv ? thp[p] : 0.0;
            }
        }
        R fr, fi;
        phase_factor<R>(t, &fr, &fi);
        const cplx_t<R> x = tile[j];
        cplx_t<R> y;
        y.x = x.x * fr - x.y * fi;
        y.y = x.x * fi + x.y * fr;
        tile[j] = y;
    }
    __syncthreads();
}

// The pair loop of one gate on the tile.  The in-tile expansion of the
// reduced index is held in NS register segments (the gate's own count or
// more; unused ones have an empty mask), so the index costs two
// instructions per segment: a gate with no tile-local control has at most
// two segments, each tile-local control adds one.  NS = 0: the expansion is
// read from the descriptor for every pair (long segment lists).
template <typename R, int THREADS, int NS>
__device__ __forceinline__ void tile_pairs(cplx_t<R> *tile, const Mat2<R> &mm, const TileGate &g, uint32_t st,
                                           uint32_t np) {
    constexpr int N = NS > 0 ? NS : 1;
    uint32_t sh[N], mk[N];
#pragma unroll
    for (int s = 0; s < N; ++s) {
        sh[s] = s < (int)g.nseg ? g.shift[s] : 0u;
        mk[s] = s < (int)g.nseg ? g.mask[s] : 0u;
    }
    const uint32_t fixed = g.fixed;
    for (uint32_t r = threadIdx.x; r < np; r += THREADS) {
        uint32_t p1;
        if (NS > 0) {
            p1 = fixed;
#pragma unroll
            for (int s = 0; s < N; ++s)
                p1 |= (r << sh[s]) & mk[s];
        } else {
            p1 = tile_expand(g, r);
        }
        cplx_t<R> x = tile[p1], y = tile[p1 | st];
        apply_pair<R>(mm, x, y);
        tile[p1] = x;
        tile[p1 | st] = y;
    }
}

// Two pair gates over 4-amplitude cosets (a coset pair marked on the host):
// g1 on target t1, then g2 on target t2, each possibly controlled by the
// other's target; the coset's other bits are free, so every coset is
// visited.
template <typename R, int THREADS>
__device__ __forceinline__ void tile_pairs2(cplx_t<R> *tile, uint32_t T, const TileGate &g1, const TileGate &g2) {
    const uint32_t t1 = g1.target, t2 = g2.target;
    const uint32_t lo = min(t1, t2), hi = max(t1, t2);
    const uint32_t s1 = 1u << t1, s2 = 1u << t2;
    // g1 controlled by t2 (value v1) acts on one of its two pairs; likewise g2
    const bool c1 = (g1.l_mask >> t2) & 1u, c2 = (g2.l_mask >> t1) & 1u;
    const uint32_t v1 = (g1.l_vals >> t2) & 1u, v2 = (g2.l_vals >> t1) & 1u;
    const bool a0 = !c1 || v1 == 0, a1 = !c1 || v1 == 1, b0 = !c2 || v2 == 0, b1 = !c2 || v2 == 1;
    const Mat2<R> m1 = tile_mat<R>(g1), m2 = tile_mat<R>(g2);
    for (uint32_t r = threadIdx.x; r < (T >> 2); r += THREADS) {
        uint32_t b = ((r >> lo) << (lo + 1)) | (r & ((1u << lo) - 1u));
        b = ((b >> hi) << (hi + 1)) | (b & ((1u << hi) - 1u));
        // x_{bit t2, bit t1}
        cplx_t<R> x00 = tile[b], x01 = tile[b | s1], x10 = tile[b | s2], x11 = tile[b | s1 | s2];
        if (a0)
            apply_pair<R>(m1, x00, x01);
        if (a1)
            apply_pair<R>(m1, x10, x11);
        if (b0)
            apply_pair<R>(m2, x00, x10);
        if (b1)
            apply_pair<R>(m2, x01, x11);
        tile[b] = x00;
        tile[b | s1] = x01;
        tile[b | s2] = x10;
        tile[b | s1 | s2] = x11;
    }
}

// Amplitudes per lane a permutation run gathers at most (its lane's part of
// the tile, or of both tiles in the reverse sweep, held in registers between
// the gather and the write-back): 128 bytes per lane.
template <typename R> constexpr int perm_per_lane() { return 128 / (int)sizeof(cplx_t<R>); }

// Source indices of the lane's tile-local indices threadIdx.x + k THREADS
// (k < NP) under the permutation run [i, i + L): the run's gates applied to
// each index last to first (each X gate is its own inverse), those whose
// outer controls fail skipped for the whole tile.  The gate loop is outside
// so that every register index stays a constant.
template <int NP, int THREADS, typename Src>
__device__ __forceinline__ void perm_sources(uint32_t *src, uint64_t base, const Src &gates, int i, int L) {
#pragma unroll
    for (int k = 0; k < NP; ++k)
        src[k] = threadIdx.x + k * THREADS;
    for (int q = i + L - 1; q >= i; --q) {
        const TileGate &d = gates.get(q);
        if ((base & d.hi_mask) != d.hi_vals)
            continue;  // uniform
        const uint32_t lm = d.l_mask, lv = d.l_vals, flip = 1u << d.target;
#pragma unroll
        for (int k = 0; k < NP; ++k)
            src[k] ^= ((src[k] & lm) == lv) ? flip : 0u;
    }
}

// A permutation run on one tile: every lane gathers its amplitudes from
// their source indices, then (after a barrier) writes them back in place.
// Requires T <= perm_per_lane<R>() * THREADS (checked by the caller).
template <typename R, int THREADS, typename Src>
__device__ __forceinline__ void tile_permute(cplx_t<R> *tile, uint32_t T, uint64_t base, const Src &gates, int i,
                                             int L) {
    constexpr int NP = perm_per_lane<R>();
    uint32_t src[NP];
    perm_sources<NP, THREADS>(src, base, gates, i, L);
    R vx[NP], vy[NP];  // components apart: an array of vector-typed values filled from LDS stays in scratch
#pragma unroll
    for (int k = 0; k < NP; ++k)
        if (threadIdx.x + k * THREADS < T) {
            const cplx_t<R> a = tile[src[k]];
            vx[k] = a.x;
            vy[k] = a.y;
        }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const uint32_t j = threadIdx.x + k * THREADS;
        if (j < T) {
            cplx_t<R> a;
            a.x = vx[k];
            a.y = vy[k];
            tile[j] = a;
        }
    }
    __syncthreads();
}

// Whether any operation of the run acts on the tile at base.
template <typename Src> __device__ __forceinline__ bool tile_touched(uint64_t base, const Src &gates) {
    bool any = false;
    for (int i = 0; i < gates.size(); ++i) {
        const TileGate &g = gates.get(i);
        any |= g.diag ? ((base & g.o_mask) == g.o_vals) : ((base & g.hi_mask) == g.hi_vals);
        if (any)
            break;  // uniform
    }
    return any;
}

// The run's operations applied to the tile held in LDS (all threads of the
// workgroup; the tile is complete in LDS on entry and on exit).
// PERM: permutation runs are applied as gathers (false: as their gates, for
// kernels without the registers to spare).
template <typename R, int THREADS, bool PERM = true, typename Src>
__device__ __forceinline__ void tile_run(cplx_t<R> *tile, uint64_t base, const TileMap &tm, const Src &gates) {
    const uint32_t T = 1u << tm.m;
    int i = 0;
    while (i < gates.size()) {
        const TileGate &g = gates.get(i);
        if (g.diag) {
            // the block marked on the host, kept inside the run
            const uint32_t sw = sweep_word(g);
            const int e = min(gates.size(), i + max(1, (int)(sw & 0xffffu)));
            // Diagonal gates commute, so the sweep multiplies each amplitude
            // by the product of its factors.  Gates whose target and controls
            // all lie outside S give the whole tile one factor (computed
            // once); the others are evaluated per amplitude on tile-local bits.
            // When every factor has unit modulus, phases are added instead and
            // turned into one factor per amplitude at the end.
            // Long sweeps whose factors all have unit modulus add phases
            // (one sine and cosine per amplitude); short ones multiply.
            if (sw >> 16) {  // uniform: a phase sweep
                if (tm.tab && tm.m >= 7 && gates.pats() != nullptr)
                    diag_sweep_tables<R, THREADS>(tile, reinterpret_cast<double *>(tile + T), base, tm.m, gates, i);
                else
                    diag_sweep_phases<R, THREADS>(tile, base, T, gates, i, e);
                i = e;
                continue;
            }
            // multiply the factors: gates that read no tile-local bit give one
            // factor for the whole tile, the others are applied per amplitude
            R ur0 = (R)1, ui0 = (R)0;
            for (int q = i; q < e; ++q) {
                const TileGate &d = gates.get(q);
                if ((base & d.o_mask) != d.o_vals || d.l_target >= 0 || d.l_mask)
                    continue;
                const bool one = (base >> d.target) & 1ull;
                const R ur = (R)(one ? d.m[6] : d.m[0]), ui = (R)(one ? d.m[7] : d.m[1]);
                const R nr = ur0 * ur - ui0 * ui;
                ui0 = ur0 * ui + ui0 * ur;
                ur0 = nr;
            }
            // four amplitudes per lane at a time (named scalars, not an array:
            // the descriptor loads are shared and everything stays in registers)
            for (uint32_t j0 = threadIdx.x; j0 < T; j0 += 4 * THREADS) {
                const uint32_t j1 = j0 + THREADS, j2 = j0 + 2 * THREADS, j3 = j0 + 3 * THREADS;
                R f0r = ur0, f0i = ui0, f1r = ur0, f1i = ui0, f2r = ur0, f2i = ui0, f3r = ur0, f3i = ui0;
                for (int q = i; q < e; ++q) {
                    const TileGate &d = gates.get(q);
                    if ((base & d.o_mask) != d.o_vals || (d.l_target < 0 && !d.l_mask))
                        continue;  // uniform
                    const bool tin = d.l_target >= 0;
                    const bool tone = (base >> d.target) & 1ull;
                    const R m0r = (R)uniform_f64(d.m[0]), m0i = (R)uniform_f64(d.m[1]);
                    const R m1r = (R)uniform_f64(d.m[6]), m1i = (R)uniform_f64(d.m[7]);
                    auto mul = [&](R &fr, R &fi, uint32_t j) {
                        const bool on = (j & d.l_mask) == d.l_vals;
                        const bool one = tin ? ((j >> d.l_target) & 1u) : tone;
                        const R ur = on ? (one ? m1r : m0r) : (R)1, ui = on ? (one ? m1i : m0i) : (R)0;
                        const R nr = fr * ur - fi * ui;
                        fi = fr * ui + fi * ur;
                        fr = nr;
                    };
                    mul(f0r, f0i, j0);
                    mul(f1r, f1i, j1);
                    mul(f2r, f2i, j2);
                    mul(f3r, f3i, j3);
                }
                auto put = [&](R fr, R fi, uint32_t j) {
                    if (j < T) {
                        const cplx_t<R> v = tile[j];
                        cplx_t<R> w;
                        w.x = v.x * fr - v.y * fi;
                        w.y = v.x * fi + v.y * fr;
                        tile[j] = w;
                    }
                };
                put(f0r, f0i, j0);
                put(f1r, f1i, j1);
                put(f2r, f2i, j2);
                put(f3r, f3i, j3);
            }
            __syncthreads();
            i = e;
            continue;
        }
        const uint32_t plen = __builtin_amdgcn_readfirstlane(g.perm_len);
        if (PERM && plen >= 2 && T <= (uint32_t)(perm_per_lane<R>() * THREADS)) {  // a permutation run (uniform)
            const int L = min((int)plen, gates.size() - i);
            tile_permute<R, THREADS>(tile, T, base, gates, i, L);
            i += L;
            continue;
        }
        if ((sweep_word(g) & 0xffffu) == 2 && i + 1 < gates.size()) {  // a coset pair (uniform)
            const TileGate &g2 = gates.get(i + 1);
            const bool p1 = (base & g.hi_mask) == g.hi_vals, p2 = (base & g2.hi_mask) == g2.hi_vals;
            if (p1 && p2) {  // uniform across the workgroup
                tile_pairs2<R, THREADS>(tile, T, g, g2);
                __syncthreads();
                i += 2;
                continue;
            }
        }
        if ((base & g.hi_mask) == g.hi_vals) {  // uniform across the workgroup
            const Mat2<R> mm = tile_mat<R>(g);
            const uint32_t st = 1u << g.target;
            const uint32_t np = g.npairs;
            // the loop's index arithmetic sized to the gate (uniform branches)
            if (g.nseg <= 2)
                tile_pairs<R, THREADS, 2>(tile, mm, g, st, np);
            else if (g.nseg <= 3)
                tile_pairs<R, THREADS, 3>(tile, mm, g, st, np);
            else if (g.nseg <= 4)
                tile_pairs<R, THREADS, 4>(tile, mm, g, st, np);
            else if (g.nseg <= (uint32_t)kExpRegs)
                tile_pairs<R, THREADS, kExpRegs>(tile, mm, g, st, np);
            else
                tile_pairs<R, THREADS, 0>(tile, mm, g, st, np);
            __syncthreads();
        }
        ++i;
    }
}

// One workgroup per tile.  Dynamic LDS holds the 2^m amplitudes.  Two
// 64 KiB tiles share a CU, so registers are capped for 4 waves per SIMD.
template <typename R, int THREADS, typename Src>
__global__ __launch_bounds__(THREADS, 4) void k_tile(cplx_t<R> *__restrict__ psi, TileMap tm, Src gates) {
    extern __shared__ unsigned char lds_raw[];
    cplx_t<R> *tile = reinterpret_cast<cplx_t<R> *>(lds_raw);
    const uint64_t base = expand_index<uint64_t>(tm.outer, tm.tile0 + blockIdx.x);
    const uint32_t T = 1u << tm.m;
    // a tile that no operation of the run touches is left alone
    if (!tile_touched(base, gates))
        return;
    tile_load<R, THREADS>(tile, psi, base, tm, T);
    __syncthreads();
    tile_run<R, THREADS>(tile, base, tm, gates);
    tile_store<R, THREADS>(psi, tile, base, tm, T);
}

} // namespace sv
