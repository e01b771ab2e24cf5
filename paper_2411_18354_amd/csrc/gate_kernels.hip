// Single-gate kernels: the control-scheduled pair kernel, the masked
// baseline, the low-target wavefront kernel and the single-gate LDS tile
// pass, plus sv_apply_gate.
//
// All kernels are in-place read-modify-write streams over the touched
// amplitudes and are HBM-bound (0.44 flop/B in complex128), so the design
// goal is full 16-byte (complex128) coalesced accesses and enough loads in
// flight per lane; the index arithmetic is a handful of integer ops per pair.
#include <algorithm>
#include <cstring>

#include "tile.hpp"

namespace sv {

// One wavefront per workgroup for the wavefront kernel and 64 pairs per
// workgroup for the pair kernel (one wavefront holding one pair per lane, or
// two wavefronts holding one element each, k_pair_xw): measured on MI355X,
// these stream an in-place 4 GiB gate at 6.4-6.8 TB/s, against 5.7-5.8 TB/s
// for 256-lane workgroups with four pairs per lane.  The masked baseline's
// workgroup size is a knob ("masked_block": 64 or 256).
constexpr int kThreads = 64;

// What a pair or lane does when its lane-tested controls fail.
constexpr int kSkip = 0;     // no load, no store (the baseline kernel figure)
constexpr int kRewrite = 1;  // load and store the unchanged values, so that
                             // writes cover whole cache lines

// ---------------------------------------------------------------------------
// Pair kernel.  Iteration i of the launch is one amplitude pair; its first
// element is p1 = expand(i), the second p1 | 2^t.
//   Scheduled (Sec. III-B): i runs over the reduced iteration set and the
//     expansion inserts the target bit (0) and every scheduled control bit
//     (its required value), so every iteration updates memory.  Controls
//     below the granule bit (tmask) are tested per pair instead, because a
//     pair skipped there shares its cache lines with pairs that are updated.
//   Masked baseline (Sec. III-A, baseline kernel figure): i runs over all
//     2^(n-1) pairs, the expansion inserts only the target bit, and the pair
//     is skipped unless all its control bits (tmask) match.
// A workgroup has T lanes; each lane handles K iterations spaced T apart so
// a wavefront's loads are contiguous and 2K loads per lane are in flight.
// ---------------------------------------------------------------------------
template <typename R, typename I, int K, int POLICY, int T, typename MS>
__global__ __launch_bounds__(T) void k_pair(cplx_t<R> *__restrict__ psi, uint64_t niter, Expand e,
                                            uint64_t tmask, uint64_t tvals, uint32_t t, MS ms, uint64_t block0) {
    const Mat2<R> m = ms.get();
    const uint64_t base = (block0 + blockIdx.x) * (T * K) + threadIdx.x;
    const I st = (I)1 << t;
    cplx_t<R> x[K], y[K];
    I p1[K];
    bool in[K], pass[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint64_t i = base + (uint64_t)j * T;
        p1[j] = expand_index<I>(e, (I)i);
        in[j] = i < niter;
        pass[j] = in[j] && (((uint64_t)p1[j] & tmask) == tvals);
        if (POLICY == kRewrite ? in[j] : pass[j]) {
            x[j] = ld_stream<R>(psi + p1[j]);
            y[j] = ld_stream<R>(psi + (p1[j] | st));
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (pass[j])
            apply_pair<R>(m, x[j], y[j]);
        if (POLICY == kRewrite ? in[j] : pass[j]) {
            st_stream<R>(psi + p1[j], x[j]);
            st_stream<R>(psi + (p1[j] | st), y[j]);
        }
    }
}

// ---------------------------------------------------------------------------
// Pair kernel, one amplitude per lane (the form scheduled complex128
// launches take).  A 128-lane workgroup holds 64 pairs: wavefront 0 loads
// their first elements p1 = expand(i), wavefront 1 their second elements
// p1 | 2^t, each lane one 16-byte load; the partners meet in LDS and
// each lane stores its own row of the 2x2 update.  So every wavefront
// streams one contiguous run, as the wavefront kernel does, instead of two
// runs 2^t apart.  Measured on the n=28 complex128 sweep (sum of the 27
// gates' times): 8.58 -> 8.34 ms; the uncontrolled gates at t=13 and 27 take
// about 1290 us instead of 1350 (the HBM probe streams the same state in
// 1280).  Scheduling, the tested controls and the two policies are those of
// k_pair.
template <typename R, typename I, int POLICY, typename MS>
__global__ __launch_bounds__(2 * kThreads) void k_pair_xw(cplx_t<R> *__restrict__ psi, uint64_t niter, Expand e,
                                                          uint64_t tmask, uint64_t tvals, uint32_t t, MS ms,
                                                          uint64_t block0) {
    __shared__ cplx_t<R> xs[2 * kThreads];
    const Mat2<R> m = ms.get();
    const bool second = threadIdx.x >= kThreads;  // wavefront 1: the pairs' second elements
    const uint64_t i = (block0 + blockIdx.x) * kThreads + (threadIdx.x & (kThreads - 1));
    const I p1 = expand_index<I>(e, (I)i);
    const bool in = i < niter;
    const bool pass = in && (((uint64_t)p1 & tmask) == tvals);
    const bool touch = POLICY == kRewrite ? in : pass;  // the same for both elements of a pair
    const I k = second ? (p1 | ((I)1 << t)) : p1;
    cplx_t<R> v;
    v.x = (R)0;
    v.y = (R)0;
    if (touch)
        v = ld_stream<R>(psi + k);
    xs[threadIdx.x] = v;
    __syncthreads();
    if (touch) {
        cplx_t<R> out = v;
        if (pass) {
            const cplx_t<R> u = xs[threadIdx.x ^ kThreads];
            cplx_t<R> x = second ? u : v, y = second ? v : u;
            apply_pair<R>(m, x, y);
            out = second ? y : x;
        }
        st_stream<R>(psi + k, out);
    }
}

// ---------------------------------------------------------------------------
// Wavefront kernel for targets whose partner lies in the same wavefront.
// Iteration a of the launch is one amplitude, at index expand(a): the
// expansion inserts the scheduled control bits only, so the target bit stays
// a free bit of a.  A wavefront covers 64 consecutive iterations with one
// contiguous load per lane (lane l holds iteration 64w + l); when the target
// is free bit tl < 6 of a, the partner amplitude sits in lane l ^ 2^tl and is
// exchanged across lanes.  Controls below the granule bit are tested per
// lane.  This schedules at amplitude granularity: only amplitudes whose
// scheduled controls hold are visited, every lane of a visited wavefront is
// busy, and the loads stay fully contiguous.
// ---------------------------------------------------------------------------
template <typename R, int K, int POLICY, typename MS>
__global__ __launch_bounds__(kThreads) void k_wave(cplx_t<R> *__restrict__ psi, uint64_t nwaves, Expand ae,
                                                   uint32_t tmask, uint32_t tvals, uint32_t tl, MS ms,
                                                   uint64_t block0) {
    const Mat2<R> m = ms.get();
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = threadIdx.x >> 6;
    constexpr int W = kThreads / 64;
    const bool upper = (lane >> tl) & 1;
    const int xm = 1 << tl;
    cplx_t<R> v[K];
    uint64_t addr[K];
    bool in[K], pass[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint64_t w = ((block0 + blockIdx.x) * K + j) * W + wave;
        in[j] = w < nwaves;
        addr[j] = expand_index<uint64_t>(ae, (w << 6) | lane);
        pass[j] = in[j] && (((uint32_t)addr[j] & tmask) == tvals);
        if (POLICY == kRewrite ? in[j] : pass[j])
            v[j] = ld_stream<R>(psi + addr[j]);
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (!in[j])
            continue;  // uniform across the wavefront
        const cplx_t<R> p = lane_xor<R>(v[j], xm);
        // component-wise selects keep everything in registers
        cplx_t<R> lo, hi, o;
        lo.x = upper ? p.x : v[j].x;
        lo.y = upper ? p.y : v[j].y;
        hi.x = upper ? v[j].x : p.x;
        hi.y = upper ? v[j].y : p.y;
        apply_pair<R>(m, lo, hi);
        o.x = pass[j] ? (upper ? hi.x : lo.x) : v[j].x;
        o.y = pass[j] ? (upper ? hi.y : lo.y) : v[j].y;
        if (POLICY == kRewrite || pass[j])
            st_stream<R>(psi + addr[j], o);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

int tile_log2(int dtype) { return tuning().tile_log2[dtype == SV_C128 ? 0 : 1]; }

template <typename R> static int set_lds_limit(const void *fn, size_t bytes) {
    static bool done[2] = {false, false};
    (void)done;
    if (bytes > 65536)
        SV_HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return SV_OK;
}

// Pairs (or wavefronts) per lane: the "pair_unroll" / "masked_unroll" knob
// (1 or 4) once the launch has enough work to fill the chip several times
// over, 1 below that so small launches still spread over every CU.
constexpr uint64_t kBigLaunch = (uint64_t)256 * 4 * 2048;

int make_gate_plan(const GateSpec &g, int dtype, int mode, GatePlan *p) {
    const Tuning &tn = tuning();
    const int gb = std::min(tn.granule_bits[dtype == SV_C128 ? 0 : 1], 6);
    const uint64_t low = (1ull << gb) - 1;
    const uint64_t sched = g.cmask & ~low;  // controls scheduled by index expansion
    p->tmask = g.cmask & low;               // controls tested per pair or lane
    p->tvals = g.cvals & low;
    p->policy = tn.low_policy;
    p->target = g.target;
    const int below_t = popcount64(sched & ((1ull << g.target) - 1));
    const int tl = g.target - below_t;  // target's bit in the wave iteration index
    const bool wave_ok = tl < 6 && g.n - popcount64(sched) >= 6;
    int k = mode;
    if (mode == SV_MODE_AUTO)
        k = (wave_ok && tn.wave_auto) ? SV_MODE_WAVE : SV_MODE_PAIR;
    std::vector<int> pos, bits;
    switch (k) {
    case SV_MODE_MASKED:
        p->kind = GateKernel::Masked;
        pos.push_back(g.target);
        bits.push_back(0);
        p->e = make_expand(g.n, pos, bits);
        p->tmask = g.cmask;
        p->tvals = g.cvals;
        p->policy = kSkip;
        p->niter = 1ull << (g.n - 1);
        break;
    case SV_MODE_PAIR: {
        p->kind = GateKernel::Pair;
        GateSpec gs{g.n, g.target, sched, g.cvals & sched};
        gate_positions(gs, pos, bits);
        p->e = make_expand(g.n, pos, bits);
        p->niter = 1ull << (g.n - 1 - popcount64(sched));
        break;
    }
    case SV_MODE_WAVE:
        if (!wave_ok)
            return fail(SV_EINVAL, "SV_MODE_WAVE needs the target among the 6 lowest free index bits and "
                                   "n - scheduled controls >= 6 (target %d, n %d)", g.target, g.n);
        p->kind = GateKernel::Wave;
        for (int q = 0; q < g.n; ++q)
            if (sched & (1ull << q)) {
                pos.push_back(q);
                bits.push_back((int)((g.cvals >> q) & 1));
            }
        p->e = make_expand(g.n, pos, bits);
        p->target = tl;
        p->niter = 1ull << (g.n - popcount64(sched) - 6);  // wavefronts of 64 amplitudes
        break;
    case SV_MODE_TILE: {
        const int m = std::min(tile_log2(dtype), g.n);
        if (g.target >= m)
            return fail(SV_EINVAL, "SV_MODE_TILE needs target < %d (target %d)", m, g.target);
        p->kind = GateKernel::Tile;
        p->niter = 1ull << (g.n - m);
        break;
    }
    default:
        return fail(SV_EINVAL, "unknown mode %d", mode);
    }
    const uint64_t work = p->kind == GateKernel::Wave ? p->niter * 64 : p->niter;
    const int knob = p->kind == GateKernel::Masked ? tn.masked_unroll : tn.pair_unroll;
    p->unroll = (work >= kBigLaunch && knob >= 4) ? 4 : 1;
    p->block = p->kind == GateKernel::Masked ? tn.masked_block : kThreads;
    if (p->kind == GateKernel::Masked || p->kind == GateKernel::Pair)
        p->index64 = g.n > 32;
    else
        p->index64 = true;
    return SV_OK;
}

// Scheduled complex128 pair launches with one pair per lane run the
// cross-wavefront form.  complex64 keeps both elements in one lane: with one
// 8-byte element per lane a wavefront has half the bytes in flight, and the
// n=28 complex64 sweep ran 4491 gates/s that way against 5020.
static bool pair_xw(const GatePlan &p, bool dbl) {
    return dbl && p.kind == GateKernel::Pair && p.unroll == 1 && p.block == kThreads;
}

std::string gate_plan_name(const GatePlan &p, int dtype, const char *matsrc) {
    const char *R = dtype == SV_C128 ? "double" : "float";
    char buf[256];
    switch (p.kind) {
    case GateKernel::Masked:
    case GateKernel::Pair:
        if (pair_xw(p, dtype == SV_C128))
            snprintf(buf, sizeof(buf), "sv::k_pair_xw<%s, %s, %d, sv::%s<%s> >", R,
                     p.index64 ? "unsigned long" : "unsigned int", p.policy, matsrc, R);
        else
            snprintf(buf, sizeof(buf), "sv::k_pair<%s, %s, %d, %d, %d, sv::%s<%s> >", R,
                     p.index64 ? "unsigned long" : "unsigned int", p.unroll, p.policy, p.block, matsrc, R);
        break;
    case GateKernel::Wave:
        snprintf(buf, sizeof(buf), "sv::k_wave<%s, %d, %d, sv::%s<%s> >", R, p.unroll, p.policy, matsrc, R);
        break;
    default:
        snprintf(buf, sizeof(buf), "sv::k_tile<%s, 512, sv::InlineGates<1> >", R);
        break;
    }
    return buf;
}

template <typename R, typename I, int K, int T, typename MS>
static void go_pair(cplx_t<R> *psi, const GatePlan &p, const MS &ms, hipStream_t st) {
    const uint64_t blocks = (p.niter + T * K - 1) / (T * K);
    const bool xw = K == 1 && T == kThreads && pair_xw(p, sizeof(R) == 8);  // 64 pairs per 128-lane workgroup
    for (uint64_t b0 = 0; b0 < blocks; b0 += kMaxGridBlocks) {
        const dim3 grid((unsigned)std::min(kMaxGridBlocks, blocks - b0));
        if (xw && p.policy == kRewrite)
            hipLaunchKernelGGL((k_pair_xw<R, I, kRewrite, MS>), grid, dim3(2 * kThreads), 0, st, psi, p.niter, p.e,
                               p.tmask, p.tvals, (uint32_t)p.target, ms, b0);
        else if (xw)
            hipLaunchKernelGGL((k_pair_xw<R, I, kSkip, MS>), grid, dim3(2 * kThreads), 0, st, psi, p.niter, p.e,
                               p.tmask, p.tvals, (uint32_t)p.target, ms, b0);
        else if (p.policy == kRewrite)
            hipLaunchKernelGGL((k_pair<R, I, K, kRewrite, T, MS>), grid, dim3(T), 0, st, psi, p.niter, p.e, p.tmask,
                               p.tvals, (uint32_t)p.target, ms, b0);
        else
            hipLaunchKernelGGL((k_pair<R, I, K, kSkip, T, MS>), grid, dim3(T), 0, st, psi, p.niter, p.e, p.tmask,
                               p.tvals, (uint32_t)p.target, ms, b0);
    }
}

template <typename R, typename I, typename MS>
static void go_pair_shape(cplx_t<R> *psi, const GatePlan &p, const MS &ms, hipStream_t st) {
    if (p.block == 256) {
        if (p.unroll == 4)
            go_pair<R, I, 4, 256>(psi, p, ms, st);
        else
            go_pair<R, I, 1, 256>(psi, p, ms, st);
    } else {
        if (p.unroll == 4)
            go_pair<R, I, 4, kThreads>(psi, p, ms, st);
        else
            go_pair<R, I, 1, kThreads>(psi, p, ms, st);
    }
}

template <typename R, int K, typename MS>
static void go_wave(cplx_t<R> *psi, const GatePlan &p, const MS &ms, hipStream_t st) {
    constexpr uint64_t W = kThreads / 64;
    const uint64_t blocks = (p.niter + W * K - 1) / (W * K);
    for (uint64_t b0 = 0; b0 < blocks; b0 += kMaxGridBlocks) {
        const dim3 grid((unsigned)std::min(kMaxGridBlocks, blocks - b0));
        if (p.policy == kRewrite)
            hipLaunchKernelGGL((k_wave<R, K, kRewrite, MS>), grid, dim3(kThreads), 0, st, psi, p.niter, p.e,
                               (uint32_t)p.tmask, (uint32_t)p.tvals, (uint32_t)p.target, ms, b0);
        else
            hipLaunchKernelGGL((k_wave<R, K, kSkip, MS>), grid, dim3(kThreads), 0, st, psi, p.niter, p.e,
                               (uint32_t)p.tmask, (uint32_t)p.tvals, (uint32_t)p.target, ms, b0);
    }
}

template <typename R, typename MS>
int launch_plan(cplx_t<R> *psi, const GatePlan &p, const MS &ms, hipStream_t st) {
    switch (p.kind) {
    case GateKernel::Masked:
    case GateKernel::Pair:
        if (p.index64)
            go_pair_shape<R, uint64_t>(psi, p, ms, st);
        else
            go_pair_shape<R, uint32_t>(psi, p, ms, st);
        break;
    case GateKernel::Wave:
        if (p.unroll == 4)
            go_wave<R, 4>(psi, p, ms, st);
        else
            go_wave<R, 1>(psi, p, ms, st);
        break;
    default:
        return fail(SV_EINVAL, "launch_plan: tile plans go through the tile launcher");
    }
    SV_LAUNCH_CHECK();
    return SV_OK;
}

template int launch_plan<double, MatVal<double>>(double2 *, const GatePlan &, const MatVal<double> &, hipStream_t);
template int launch_plan<float, MatVal<float>>(float2 *, const GatePlan &, const MatVal<float> &, hipStream_t);
template int launch_plan<double, MatPtr<double>>(double2 *, const GatePlan &, const MatPtr<double> &, hipStream_t);
template int launch_plan<float, MatPtr<float>>(float2 *, const GatePlan &, const MatPtr<float> &, hipStream_t);

template <typename R>
static int launch_tile1(const sv_state_t *s, const GateSpec &g, const double *U, hipStream_t st) {
    const int m = std::min(tile_log2(s->dtype), g.n);
    TileMap tm = contiguous_tile_map(g.n, m);
    InlineGates<1> gs;
    gs.g[0] = make_tile_gate(tm, g.target, g.cmask, g.cvals, U, false);
    gs.count = 1;
    const size_t lds = ((size_t)1 << m) * sizeof(cplx_t<R>);
    auto fn = k_tile<R, 512, InlineGates<1>>;
    SV_TRY(set_lds_limit<R>((const void *)fn, lds));
    const uint64_t ntiles = tm.ntiles;
    for (uint64_t t0 = 0; t0 < ntiles; t0 += kMaxGridBlocks) {
        tm.tile0 = t0;
        hipLaunchKernelGGL(fn, dim3((unsigned)std::min(kMaxGridBlocks, ntiles - t0)), dim3(512), lds, st,
                           reinterpret_cast<cplx_t<R> *>(s->data), tm, gs);
        SV_LAUNCH_CHECK();
    }
    return SV_OK;
}

// ---------------------------------------------------------------------------
// HBM probe (measurement helper, not part of the method): the same streaming
// access as the scheduled kernels (64-lane workgroups, one 16- or 8-byte
// amplitude per lane, nontemporal) over the amplitudes whose index bits
// match a fixed pattern, with no arithmetic beyond a multiply by 1.  It gives
// the bandwidth a gate's own address set can reach, and a kernel of known
// traffic for calibrating the byte counters of the profiler.
//   OP 0: read and write back every selected amplitude (unchanged values)
//   OP 1: read only;  OP 2: write zeros
// ---------------------------------------------------------------------------
template <typename R, int OP>
__global__ __launch_bounds__(kThreads) void k_hbm_probe(cplx_t<R> *__restrict__ psi, uint64_t count, Expand e,
                                                        R scale, R *__restrict__ sink, uint64_t block0) {
    const uint64_t i = (block0 + blockIdx.x) * kThreads + threadIdx.x;
    if (i >= count)
        return;
    const uint64_t k = expand_index<uint64_t>(e, i);
    if (OP == 2) {
        cplx_t<R> z;
        z.x = (R)0;
        z.y = (R)0;
        st_stream<R>(psi + k, z);
        return;
    }
    cplx_t<R> v = ld_stream<R>(psi + k);
    if (OP == 0) {
        v.x *= scale;  // scale is 1: the values stay as they were
        v.y *= scale;
        st_stream<R>(psi + k, v);
    } else if (v.x == scale) {  // scale is NaN for reads: never true, keeps the load
        sink[0] = v.y;
    }
}

template <typename R, int OP>
static int go_probe(void *psi, uint64_t count, const Expand &e, hipStream_t st) {
    const uint64_t blocks = (count + kThreads - 1) / kThreads;
    const R scale = OP == 1 ? (R)__builtin_nan("") : (R)1;
    for (uint64_t b0 = 0; b0 < blocks; b0 += kMaxGridBlocks) {
        const dim3 grid((unsigned)std::min(kMaxGridBlocks, blocks - b0));
        hipLaunchKernelGGL((k_hbm_probe<R, OP>), grid, dim3(kThreads), 0, st, reinterpret_cast<cplx_t<R> *>(psi),
                           count, e, scale, reinterpret_cast<R *>(psi), b0);
    }
    SV_LAUNCH_CHECK();
    return SV_OK;
}

int launch_gate(const sv_state_t *s, const GateSpec &g, const double *U, int mode, hipStream_t st) {
    if (is_fixed(s->dtype)) {
        if (mode < SV_MODE_AUTO || mode > SV_MODE_TILE)
            return fail(SV_EINVAL, "unknown mode %d", mode);
        FixedPlan q;
        SV_TRY(make_fixed_plan(g, s->dtype, mode == SV_MODE_MASKED, &q));
        return launch_fixed_gate(s->data, q, U, nullptr, st);
    }
    GatePlan p;
    SV_TRY(make_gate_plan(g, s->dtype, mode, &p));
    if (p.kind == GateKernel::Tile)
        return s->dtype == SV_C128 ? launch_tile1<double>(s, g, U, st) : launch_tile1<float>(s, g, U, st);
    if (s->dtype == SV_C128)
        return launch_plan<double>(reinterpret_cast<double2 *>(s->data), p, MatVal<double>{to_mat<double>(U)}, st);
    return launch_plan<float>(reinterpret_cast<float2 *>(s->data), p, MatVal<float>{to_mat<float>(U)}, st);
}

} // namespace sv

using namespace sv;

extern "C" {

int sv_apply_gate_masks(const sv_state_t *s, int target, uint64_t ctrl_mask, uint64_t ctrl_vals, const double *U,
                        int mode, sv_stream_t st) {
    clear_error();
    SV_TRY(validate_state(s, true));
    if (!U)
        return fail(SV_EINVAL, "U is NULL");
    GateSpec g{s->n, target, ctrl_mask, ctrl_vals};
    SV_TRY(validate_gate(g));
    return launch_gate(s, g, U, mode, (hipStream_t)st);
}

int sv_apply_gate(const sv_state_t *s, int target, const int32_t *controls, int ncontrols, uint64_t ctrl_vals,
                  const double *U, int mode, sv_stream_t st) {
    clear_error();
    SV_TRY(validate_state(s, true));
    if (!U)
        return fail(SV_EINVAL, "U is NULL");
    if (target < 0 || target >= s->n)
        return fail(SV_EINVAL, "target %d outside [0, %d)", target, s->n);
    uint64_t mask = 0;
    SV_TRY(controls_to_mask(s->n, target, controls, ncontrols, &mask));
    GateSpec g{s->n, target, mask, ctrl_vals};
    SV_TRY(validate_gate(g));
    return launch_gate(s, g, U, mode, (hipStream_t)st);
}

int sv_hbm_probe(const sv_state_t *s, uint64_t fixed_mask, uint64_t fixed_vals, int op, sv_stream_t st) {
    clear_error();
    SV_TRY(validate_state(s));
    const uint64_t full = (s->n >= 64) ? ~0ull : ((1ull << s->n) - 1);
    if (fixed_mask & ~full)
        return fail(SV_EINVAL, "fixed_mask 0x%llx has bits >= n=%d", (unsigned long long)fixed_mask, s->n);
    if (fixed_vals & ~fixed_mask)
        return fail(SV_EINVAL, "fixed_vals 0x%llx has bits outside fixed_mask 0x%llx",
                    (unsigned long long)fixed_vals, (unsigned long long)fixed_mask);
    if (op < 0 || op > 2)
        return fail(SV_EINVAL, "unknown probe operation %d", op);
    std::vector<int> pos, bits;
    for (int q = 0; q < s->n; ++q)
        if (fixed_mask & (1ull << q)) {
            pos.push_back(q);
            bits.push_back((int)((fixed_vals >> q) & 1));
        }
    const Expand e = make_expand(s->n, pos, bits);
    const uint64_t count = 1ull << (s->n - popcount64(fixed_mask));
    const hipStream_t hs = (hipStream_t)st;
    if (s->dtype == SV_C128)
        return op == 0 ? go_probe<double, 0>(s->data, count, e, hs)
               : op == 1 ? go_probe<double, 1>(s->data, count, e, hs)
                         : go_probe<double, 2>(s->data, count, e, hs);
    return op == 0 ? go_probe<float, 0>(s->data, count, e, hs)
           : op == 1 ? go_probe<float, 1>(s->data, count, e, hs)
                     : go_probe<float, 2>(s->data, count, e, hs);
}

int sv_gate_plan(int n, int dtype, int target, uint64_t ctrl_mask, uint64_t ctrl_vals, int mode, char *kernel,
                 int kernel_len, uint64_t *iterations) {
    clear_error();
    if (!known_dtype(dtype))
        return fail(SV_EINVAL, "unknown dtype %d", dtype);
    if (n < 1 || n > max_qubits(dtype))
        return fail(SV_EINVAL, "n=%d outside [1, %d]", n, max_qubits(dtype));
    GateSpec g{n, target, ctrl_mask, ctrl_vals};
    SV_TRY(validate_gate(g));
    std::string name;
    if (is_fixed(dtype)) {
        if (mode < SV_MODE_AUTO || mode > SV_MODE_TILE)
            return fail(SV_EINVAL, "unknown mode %d", mode);
        FixedPlan q;
        SV_TRY(make_fixed_plan(g, dtype, mode == SV_MODE_MASKED, &q));
        name = fixed_plan_name(q, "MatVal");
        if (iterations)
            *iterations = q.units;
    } else {
        GatePlan p;
        SV_TRY(make_gate_plan(g, dtype, mode, &p));
        name = gate_plan_name(p, dtype, "MatVal");
        if (iterations)
            *iterations = p.niter;
    }
    if (kernel && kernel_len > 0) {
        strncpy(kernel, name.c_str(), (size_t)kernel_len - 1);
        kernel[kernel_len - 1] = '\0';
    }
    return SV_OK;
}

} // extern "C"
