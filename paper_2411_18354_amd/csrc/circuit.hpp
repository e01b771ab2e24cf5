// Internal circuit plan shared by the circuit driver and the adjoint sweep.
#pragma once

#include "tile.hpp"

namespace sv {

struct ParamJob {
    int32_t kind;
    int32_t param;
    int32_t mat_slot;   // gate index: matrix at mats + 8 * mat_slot
    int32_t tile_slot;  // fused-run descriptor index or -1
};

// The complex type a fused tile holds: fixed-point states decode 16-bit
// codes to float and 32-bit codes to double.
inline int tile_dtype(int dtype) { return dtype == SV_CQ32 ? SV_C128 : dtype == SV_CQ16 ? SV_C64 : dtype; }

// Fused pass over a block-scaled fixed-point state (the tile's qubit set
// holds qubits 0..5): decode each tile into LDS, run, re-encode its blocks.
int launch_fixed_tile_pass(void *state, int n, int dtype, const TileMap &tm, const DeviceGates &dg, size_t lds,
                           hipStream_t st);
int fixed_tile_lds_limit(int dtype, size_t lds);

struct Pass {
    bool fused;
    bool dense = false;  // dense k-qubit block: gates [first, first+count) of the dense list
    int gate;        // single: gate index
    int first, count;  // fused: descriptors [first, first + count)
    GatePlan plan;   // single
    FixedPlan fx;    // single, fixed-point state
    TileMap tm;      // fused: which qubits a tile spans
};

} // namespace sv

struct sv_circuit {
    // (the C ABI's opaque sv_circuit_t)
    int n = 0, dtype = 0, flags = 0, nparams = 0, device = 0, m = 0;
    int m_cap = 64;  // upper bound on the tile width (callers with a fixed LDS budget)
    int max_lookahead = 2;  // cap on the planner's lookahead depth (one-shot plans and batches: 1)
    std::vector<sv_gate_t> gates;   // after the SV_REMAP relabelling, if any
    std::vector<int32_t> remap;      // SV_REMAP: qubit swaps a0 b0 a1 b1 ... (empty: none)
    std::vector<sv::Pass> passes;
    std::vector<int32_t> tile_src;  // gate index of every fused-run descriptor
    int dense_k = 0;                // qubits of dense blocks
    void *d_dense = nullptr;        // DenseGate list of all dense passes
    void *d_rmat = nullptr;         // one real embedding per dense pass
    int njobs = 0;
    int64_t fused_gates = 0, fused_runs = 0;
    double *d_mats = nullptr;
    sv::TileGate *d_tiles = nullptr;
    sv::ParamJob *d_jobs = nullptr;
    sv::SweepPat *d_pats = nullptr;      // phase patterns of the table sweeps
    sv::SweepMember *d_mems = nullptr;   // and their members
    bool async_buffers = false;  // allocated stream-ordered (one-shot use)
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *g_data = nullptr;
    const double *g_params = nullptr;
    hipEvent_t done = nullptr;
};


namespace sv {

// Validate, plan and upload a circuit (the body of sv_circuit_create).
// async: device buffers are allocated and released stream-ordered on st.
// m_cap bounds the tile width (callers with a fixed LDS budget).
// The fused plan of a circuit as data for other executors (the batched
// kernel): each pass is either one gate (fused == 0, gate = its index in the
// circuit) or the run of tile descriptors tiles[first .. first + count) over
// the tile map tm.  Tiles over any qubit set, diagonal gates fused whatever
// their target, tile width at most m_cap.
struct PlanPass {
    TileMap tm;
    int32_t fused, gate, first, count;
};
// pats/mems (optional): the phase patterns of the table sweeps, indexed
// from 0 (pat0 and mem[] of the descriptors refer to them).
int circuit_plan_tiles(int n, int dtype, const sv_gate_t *gates, int ngates, int nparams, int m_cap,
                       std::vector<PlanPass> *passes, std::vector<TileGate> *tiles, int *m_used,
                       std::vector<SweepPat> *pats = nullptr, std::vector<SweepMember> *mems = nullptr);

int circuit_create(int n, int dtype, const sv_gate_t *gates, int ngates, int nparams, int flags, bool async,
                   hipStream_t st, int m_cap, sv_circuit **out);
// Release device buffers (stream-ordered on st for async plans) and the plan.
void circuit_free(sv_circuit *c, hipStream_t st);
// Compute the matrices of parameterised gates from params (device) into the
// plan's tables.
int circuit_param_mats(sv_circuit *c, const double *params, hipStream_t st);

// Dense k-qubit blocks (dense.hip).
struct DenseGate {
    int32_t target, mat;  // mat: gate index into the circuit's matrix table
    uint64_t cmask, cvals;
};
// Disjoint qubit exchanges (permute.hip): pairs = a0 b0 a1 b1 ...
constexpr int kMaxSwapPairs = 32;
int check_swap_pairs(int n, const int32_t *pairs, int npairs);
int launch_swap_qubits(int dtype, void *psi, int n, const int32_t *pairs, int npairs, hipStream_t st);

bool dense_supported(int dtype, int kq, int n);
int launch_dense(int dtype, void *psi, int n, int kq, const void *rmat, hipStream_t st);
int launch_dense_compose(int dtype, const void *gates, int count, const double *mats, int kq, void *rmat,
                         hipStream_t st);

} // namespace sv
