// Internal declarations shared by the translation units of libsv.so.
//
// Holds the complex storage types, the index-expansion plan that turns a
// reduced iteration index into an amplitude index (control-aware scheduling,
// arXiv:2411.18354 Sec. III-B), status/error plumbing and host-side argument
// validation.  Nothing here is visible through the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/sv.h"

namespace sv {

// ---------------------------------------------------------------- errors

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define SV_HIP_TRY(expr)                                                       \
    do {                                                                       \
        hipError_t _e = (expr);                                                \
        if (_e != hipSuccess)                                                  \
            return ::sv::fail(SV_EHIP, "%s failed: %s (%s:%d)", #expr,         \
                              hipGetErrorString(_e), __FILE__, __LINE__);      \
    } while (0)

#define SV_LAUNCH_CHECK()                                                      \
    do {                                                                       \
        hipError_t _e = hipGetLastError();                                     \
        if (_e != hipSuccess)                                                  \
            return ::sv::fail(SV_EHIP, "kernel launch failed: %s (%s:%d)",     \
                              hipGetErrorString(_e), __FILE__, __LINE__);      \
    } while (0)

#define SV_TRY(expr)                                                           \
    do {                                                                       \
        int _r = (expr);                                                       \
        if (_r != SV_OK)                                                       \
            return _r;                                                         \
    } while (0)

// ---------------------------------------------------------------- storage

template <typename R> struct cplx;
template <> struct cplx<double> { using type = double2; };
template <> struct cplx<float> { using type = float2; };
template <typename R> using cplx_t = typename cplx<R>::type;

inline bool known_dtype(int dtype) { return dtype >= SV_C128 && dtype <= SV_CQ32; }
inline bool is_fixed(int dtype) { return dtype == SV_CQ16 || dtype == SV_CQ32; }
inline size_t amp_bytes(int dtype) { return dtype == SV_C128 ? 16 : dtype == SV_CQ16 ? 4 : 8; }
inline int max_qubits(int dtype) {
    return dtype == SV_C128   ? SV_MAX_QUBITS_C128
           : dtype == SV_C64  ? SV_MAX_QUBITS_C64
           : dtype == SV_CQ16 ? SV_MAX_QUBITS_CQ16
                              : SV_MAX_QUBITS_CQ32;
}
// Fixed-point states: 64 amplitudes share one int8 scale, stored after the
// 2^n code pairs.
constexpr int kQBlockBits = 6;
inline uint64_t q16_blocks(int n) { return n >= kQBlockBits ? (1ull << (n - kQBlockBits)) : 1ull; }
inline size_t state_bytes(int n, int dtype) {
    return ((size_t)1 << n) * amp_bytes(dtype) + (is_fixed(dtype) ? (size_t)q16_blocks(n) : 0);
}

// 2x2 gate matrix in the compute precision: a, b, c, d as (re, im).
template <typename R> struct Mat2 {
    R ar, ai, br, bi, cr, ci, dr, di;
};

template <typename R> inline Mat2<R> to_mat(const double *U) {
    return Mat2<R>{(R)U[0], (R)U[1], (R)U[2], (R)U[3], (R)U[4], (R)U[5], (R)U[6], (R)U[7]};
}

// ---------------------------------------------------------------- expansion
//
// A gate with target t and controls C (values V) touches exactly the
// amplitude indices whose bits at positions {t} u C are fixed (0 at t, v_j at
// c_j).  The paper maps a reduced iteration index to a global iteration index
// one control at a time (adjusted control, skip interval 2^{c_adj}, ascending
// controls), then inserts a 0 at t.  Inserting a bit b at position p of x is
// ((x >> p) << (p+1)) | (b << p) | (x & (2^p - 1)); for b = 1 this is exactly
// the skip-interval step x + (floor(x / 2^p) + 1) 2^p.  Doing every insertion
// in ascending position order equals one bit deposit: the free bits of x are
// spread over the non-fixed positions in order.  The plan stores that deposit
// as a few (shift, mask) segments so a lane computes
//     p1 = fixed | OR_j ((x << shift_j) & mask_j)
// with no data-dependent control flow.

constexpr int kMaxSeg = SV_MAX_QUBITS_C64 + 2;

// A dispatch covers fewer than 2^32 work-items per grid dimension, which
// the largest registers exceed (2^34 pairs); launches whose grid grows with
// 2^n are split into pieces of at most this many workgroups, each told the
// index of its first workgroup.
constexpr uint64_t kMaxGridBlocks = 1ull << 22;

struct Expand {
    uint32_t nseg;
    uint32_t shift[kMaxSeg];
    uint64_t mask[kMaxSeg];
    uint64_t fixed;
};

// positions: ascending insertion positions; bits: value at each position.
Expand make_expand(int n, const std::vector<int> &positions, const std::vector<int> &bits);

template <typename I>
__device__ __forceinline__ I expand_index(const Expand &e, I x) {
    I p = (I)e.fixed;
    for (uint32_t s = 0; s < e.nseg; ++s)
        p |= (I)((x << e.shift[s]) & (I)e.mask[s]);
    return p;
}

// ---------------------------------------------------------------- validation

struct GateSpec {
    int n;
    int target;
    uint64_t cmask;
    uint64_t cvals;
};

// allow_fixed: the caller handles fixed-point states (SV_ENOTSUP otherwise).
int validate_state(const sv_state_t *s, bool allow_fixed = false);
int validate_gate(const GateSpec &g);
int controls_to_mask(int n, int target, const int32_t *controls, int nc, uint64_t *mask);
// Sorted insertion positions of a gate: target (bit 0) and controls (their values).
void gate_positions(const GateSpec &g, std::vector<int> &pos, std::vector<int> &bits);
inline int popcount64(uint64_t v) { return __builtin_popcountll(v); }

// ---------------------------------------------------------------- devices

struct DeviceInfo {
    int device;
    int num_cus;
    int max_lds;
    std::string arch;
};
int device_info(DeviceInfo *out);

// ---------------------------------------------------------------- tuning

// Library-wide launch choices; defaults are set from measurements on
// MI355X and can be changed through sv_tune_set (the autotuner does).
struct Tuning {
    int granule_bits[2];  // [c128, c64]: controls on lower index bits are
                          // tested per pair/lane instead of scheduled
    int low_policy;       // 0: failing pairs skipped, 1: rewritten unchanged
    int wave_auto;        // SV_MODE_AUTO may pick the wavefront kernel
    int tile_log2[2];     // fused-pass tile width (amplitudes = 2^m)
    int tile_low_bits[2]; // lowest qubits always inside a fused tile (contiguous runs)
    int fuse_min_gates;   // shortest run worth an LDS pass
    int dense_qubits;     // k of dense k-qubit blocks (SV_DENSE)
    int dense_min_gates;  // shortest stretch on qubits < k made a dense block
    int pair_unroll;      // pairs (wavefronts) per lane of large scheduled launches: 1 or 4
    int masked_unroll;    // the same for the masked baseline kernel
    int masked_block;     // lanes per workgroup of the masked baseline kernel: 64 or 256
    int fuse_group;       // fused runs: gather diagonal gates into blocks (commutation moves)
    int fuse_pairs;       // fused runs: apply adjacent coset-closed pair gates together
    int plan_lookahead;   // fused runs: lookahead depth choosing a run's high qubits (0-2)
    int fuse_perm;        // fused runs: apply runs of X gates as one gather
    int batch_split;      // batches: most workgroups one circuit may be split over
    int phase_sweep_min[2]; // [c128, c64] fused runs: a diagonal block with this many tile-local gates is one sweep
};
Tuning &tuning();

// ---------------------------------------------------------------- gate plans

enum class GateKernel { Masked, Pair, Wave, Tile };

struct GatePlan {
    GateKernel kind;
    Expand e;          // pair kernels: pair index; wave kernel: amplitude index
    uint64_t tmask, tvals;  // controls tested per pair or lane
    uint64_t niter;    // pairs, wavefronts (64 amplitudes) or tiles
    int target;        // pair kernels: t; wave kernel: t's bit in the iteration index
    int unroll;
    int block;         // lanes per workgroup (pair kernels)
    int policy;
    bool index64;
};

int make_gate_plan(const GateSpec &g, int dtype, int mode, GatePlan *p);
std::string gate_plan_name(const GatePlan &p, int dtype, const char *matsrc);
template <typename R, typename MS>
int launch_plan(cplx_t<R> *psi, const GatePlan &p, const MS &ms, hipStream_t st);

// Fixed-point gates (fixed.hip).  Work unit: one 64-amplitude block (target
// below bit 6) or the pair of blocks a target >= 6 couples.
struct FixedPlan {
    Expand e;                // scheduled: block index of a unit
    uint64_t units;          // work units
    uint64_t hmask, hvals;   // masked: control bits of the block index
    uint32_t lmask, lvals;   // controls on the 6 in-block bits, tested per amplitude
    int n, target;           // target: qubit (n < 6 or target < 6), else its block-index bit
    int dtype;               // SV_CQ16 or SV_CQ32
    bool masked, high, small;
};
int make_fixed_plan(const GateSpec &g, int dtype, bool masked, FixedPlan *p);
std::string fixed_plan_name(const FixedPlan &p, const char *matsrc);
// U: 8 doubles on the host (by value) or, when Ud is set, on the device.
int launch_fixed_gate(void *state, const FixedPlan &p, const double *U, const double *Ud, hipStream_t st);
int launch_fixed_basis(void *state, int n, int dtype, uint64_t basis, unsigned grid, hipStream_t st);

// Launch helpers implemented in gate_kernels.hip, shared with the circuit
// executor.
int launch_gate(const sv_state_t *s, const GateSpec &g, const double *U, int mode,
                hipStream_t st);
int tile_log2(int dtype);

} // namespace sv
