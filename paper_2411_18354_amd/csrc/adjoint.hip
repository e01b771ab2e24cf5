// Adjoint (reverse-mode) gradient of L(theta) = <psi(theta)|H|psi(theta)>,
// psi(theta) = U_G ... U_1 |psi_0>, without a tape.
//
// Starting from the final state psi and the co-state lambda = H psi, the
// gates are visited in reverse.  At gate k, with psi = psi_k (before
// un-applying it) and lambda = U_{k+1}^dag ... U_G^dag H psi_G,
//     dL/dtheta += 2 Re <lambda| dU_k/dtheta |psi_{k-1}>
//                = 2 Re <lambda| Pi_c (A_k (x) ...) |psi_k>,
// where dU/dtheta = A U for the parameterised single-qubit gate (A = -i/2 P
// for the Pauli rotations, diag(0, i) for the phase gate) and Pi_c projects
// onto the amplitudes whose control bits hold.  So the gradient of a
// controlled gate is a sum over exactly the amplitude pairs that the
// control-aware scheduling enumerates (Sec. III-B), and the same kernel pass
// then un-applies the gate (U^dag) on both psi and lambda.  Memory: the two
// state vectors only.  (Jones & Gacon, arXiv:2009.02823, describe the
// method for uncontrolled gates.)
#include <algorithm>
#include <cstring>

#include "circuit.hpp"
#include "gates.hpp"
#include "pauli.hpp"
#include "tile_adj.hpp"

namespace sv {

int validate_circuit_gate(int n, int nparams, const sv_gate_t &g, int index);
int validate_unitary_gate(const sv_gate_t &g, int index);

// One gate of the reverse sweep on the pairs of a scheduled plan (pair index
// p1 = expand(i), partner p1 | 2^t; tmask/tvals as in the pair kernel).
template <typename R, typename I, int POLICY, bool GRAD>
__global__ __launch_bounds__(kRedThreads) void k_adj(cplx_t<R> *__restrict__ psi, cplx_t<R> *__restrict__ lam,
                                                     uint64_t niter, Expand e, uint64_t tmask, uint64_t tvals,
                                                     uint32_t t, const double *__restrict__ udag,
                                                     const double *__restrict__ gen, double *__restrict__ partial) {
    __shared__ double scratch[kRedThreads / 64];
    const Mat2<R> u = MatPtr<R>{udag}.get();
    double a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        a[k] = GRAD ? gen[k] : 0.0;
    const I st = (I)1 << t;
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kRedThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kRedThreads + threadIdx.x; i < niter; i += stride) {
        const I p1 = expand_index<I>(e, (I)i);
        const I p2 = p1 | st;
        const bool pass = ((uint64_t)p1 & tmask) == tvals;
        if (!(POLICY == 1 || pass))
            continue;
        cplx_t<R> x = ld_stream<R>(psi + p1), y = ld_stream<R>(psi + p2);
        cplx_t<R> lx = ld_stream<R>(lam + p1), ly = ld_stream<R>(lam + p2);
        if (pass) {
            if (GRAD) {
                const double xr = x.x, xi = x.y, yr = y.x, yi = y.y;
                const double axr = a[0] * xr - a[1] * xi + a[2] * yr - a[3] * yi;
                const double axi = a[0] * xi + a[1] * xr + a[2] * yi + a[3] * yr;
                const double ayr = a[4] * xr - a[5] * xi + a[6] * yr - a[7] * yi;
                const double ayi = a[4] * xi + a[5] * xr + a[6] * yi + a[7] * yr;
                acc += 2.0 * ((double)lx.x * axr + (double)lx.y * axi + (double)ly.x * ayr + (double)ly.y * ayi);
            }
            apply_pair<R>(u, x, y);
            apply_pair<R>(u, lx, ly);
        }
        st_stream<R>(psi + p1, x);
        st_stream<R>(psi + p2, y);
        st_stream<R>(lam + p1, lx);
        st_stream<R>(lam + p2, ly);
    }
    if (GRAD) {
        const double s = block_sum(acc, scratch);
        if (threadIdx.x == 0)
            partial[blockIdx.x] = s;
    }
}

// A fused run of the reverse sweep, one workgroup per group of tiles: psi
// and lambda tiles together in LDS, the run's operations un-applied by
// adj_tile_run (tile_adj.hpp), each workgroup's gradient partials written
// once at the end.
// Two workgroups share a CU (two 64 KiB tile pairs), so registers are capped
// for 4 waves per SIMD.
template <typename R>
__global__ __launch_bounds__(kAdjTileThreads, 4) void k_adj_tile(cplx_t<R> *__restrict__ psi, cplx_t<R> *__restrict__ lam,
                                                              TileMap tm, DeviceGates gates,
                                                              const int32_t *__restrict__ gslot,
                                                              const double *__restrict__ gens,
                                                              double *__restrict__ partials) {
    extern __shared__ unsigned char lds_raw[];
    const uint32_t T = 1u << tm.m;
    cplx_t<R> *tp = reinterpret_cast<cplx_t<R> *>(lds_raw);
    cplx_t<R> *tl = tp + T;
    double *accl = reinterpret_cast<double *>(tl + T);
    const int npg = adj_acc_zero(gates, gslot, accl);
    for (uint64_t t = blockIdx.x; t < tm.ntiles; t += gridDim.x) {
        const uint64_t base = expand_index<uint64_t>(tm.outer, t);
        if (!adj_tile_touched(base, gates))
            continue;  // uniform
        tile_load2<R, kAdjTileThreads>(tp, tl, psi, lam, base, tm, T);
        __syncthreads();
        adj_tile_run<R, kAdjTileThreads>(tp, tl, base, T, gates, gslot, gens, accl);
        tile_store2<R, kAdjTileThreads>(psi, lam, tp, tl, base, tm, T);
        __syncthreads();
    }
    // this workgroup's partial of every parameterised gate: its wavefronts'
    // accumulators summed in index order
    __syncthreads();
    for (int k = threadIdx.x; k < npg; k += kAdjTileThreads) {
        const int sl = adj_acc_slot(gates, gslot, k);
        partials[(size_t)sl * kMaxPartials + blockIdx.x] = adj_acc_sum(accl, k);
    }
}

// grad[j] = scale * sum over the slots of parameter j (slot_first[j] ..
// slot_first[j+1]) of that slot's partials, in a fixed order; the extra
// workgroup (blockIdx.x == nparams) reduces the loss partials.
__global__ __launch_bounds__(kRedThreads) void k_grad_final(int nparams, const int32_t *__restrict__ slot_first,
                                                            const int32_t *__restrict__ slots,
                                                            const int32_t *__restrict__ slot_blocks,
                                                            const double *__restrict__ partials,
                                                            const double *__restrict__ loss_partials,
                                                            int loss_blocks, const double *__restrict__ scale,
                                                            double *__restrict__ grad, double *__restrict__ loss) {
    __shared__ double scratch[kRedThreads / 64];
    const int j = blockIdx.x;
    if (j == nparams) {
        const double s = block_sum_array(loss_partials, loss_blocks, scratch);
        if (threadIdx.x == 0 && loss)
            loss[0] = s;
        return;
    }
    double g = 0.0;
    for (int k = slot_first[j]; k < slot_first[j + 1]; ++k) {
        const int s = slots[k];
        g += block_sum_array(partials + (size_t)s * kMaxPartials, slot_blocks[s], scratch);
    }
    if (threadIdx.x == 0)
        grad[j] = scale ? g * scale[0] : g;
}

template <typename R, typename I, int POLICY>
static void go_adj(cplx_t<R> *psi, cplx_t<R> *lam, const GatePlan &p, const double *udag, const double *gen,
                   double *partial, unsigned grid, hipStream_t st) {
    if (gen)
        hipLaunchKernelGGL((k_adj<R, I, POLICY, true>), dim3(grid), dim3(kRedThreads), 0, st, psi, lam, p.niter, p.e,
                           p.tmask, p.tvals, (uint32_t)p.target, udag, gen, partial);
    else
        hipLaunchKernelGGL((k_adj<R, I, POLICY, false>), dim3(grid), dim3(kRedThreads), 0, st, psi, lam, p.niter,
                           p.e, p.tmask, p.tvals, (uint32_t)p.target, udag, gen, partial);
}

template <typename R>
static void launch_adj(void *psi, void *lam, const GatePlan &p, const double *udag, const double *gen, double *partial,
                       unsigned grid, hipStream_t st) {
    auto *a = reinterpret_cast<cplx_t<R> *>(psi);
    auto *b = reinterpret_cast<cplx_t<R> *>(lam);
    if (p.index64) {
        if (p.policy == 1)
            go_adj<R, uint64_t, 1>(a, b, p, udag, gen, partial, grid, st);
        else
            go_adj<R, uint64_t, 0>(a, b, p, udag, gen, partial, grid, st);
    } else {
        if (p.policy == 1)
            go_adj<R, uint32_t, 1>(a, b, p, udag, gen, partial, grid, st);
        else
            go_adj<R, uint32_t, 0>(a, b, p, udag, gen, partial, grid, st);
    }
}

// The reverse sweep of one circuit and Hamiltonian, planned once: the
// reverse circuit's fused plan, the generator table, the reduction layout
// and the Pauli terms, on one device.
struct AdjointPlan {
    int n = 0, dtype = 0, ngates = 0, nparams = 0, nslots = 0, device = 0;
    bool async = false;
    sv_circuit *rc = nullptr;
    std::vector<int> gen_slot;
    std::vector<GatePlan> single_plan;
    std::vector<size_t> pass_lds;
    size_t off_slots = 0, off_blocks = 0;
    double *d_gen = nullptr, *d_partials = nullptr;
    int32_t *d_ints = nullptr, *d_dslot = nullptr;
    PauliDevice pd;
};

static void adjoint_free(AdjointPlan *a, hipStream_t st) {
    a->pd.partials = nullptr;  // borrowed from d_partials
    pauli_release(&a->pd, st);
    void *bufs[] = {a->d_gen, a->d_partials, a->d_ints, a->d_dslot};
    for (void *b : bufs)
        if (b)
            (void)(a->async ? hipFreeAsync(b, st) : hipFree(b));
    a->d_gen = a->d_partials = nullptr;
    a->d_ints = a->d_dslot = nullptr;
    if (a->rc)
        circuit_free(a->rc, st);
    a->rc = nullptr;
}

// Validate and plan; device tables allocated stream-ordered on st when async
// (a one-shot gradient), otherwise allocated and filled before returning.
static int adjoint_plan(int n, int dtype, const sv_gate_t *gates, int ngates, int nparams, const sv_pauli_t *terms,
                        int nterms, bool async, hipStream_t st, AdjointPlan *a) {
    if (dtype != SV_C128 && dtype != SV_C64)
        return fail(SV_EINVAL, "the adjoint takes complex128 and complex64 states (dtype %d)", dtype);
    if (n < 1 || n > max_qubits(dtype))
        return fail(SV_EINVAL, "n=%d outside [1, %d]", n, max_qubits(dtype));
    if (ngates < 0 || (ngates > 0 && !gates))
        return fail(SV_EINVAL, "bad gate list");
    if (nparams < 0)
        return fail(SV_EINVAL, "nparams %d", nparams);
    for (int i = 0; i < ngates; ++i) {
        SV_TRY(validate_circuit_gate(n, nparams, gates[i], i));
        SV_TRY(validate_unitary_gate(gates[i], i));
    }
    PauliPlan pplan;
    SV_TRY(make_pauli_plan(n, terms, nterms, &pplan));
    a->n = n;
    a->dtype = dtype;
    a->ngates = ngates;
    a->nparams = nparams;
    a->async = async;
    SV_HIP_TRY(hipGetDevice(&a->device));

    // The reverse sweep is the circuit of inverses in reverse order, planned
    // like a forward circuit (fused runs of two LDS tiles, so one size down).
    std::vector<sv_gate_t> rev(ngates);
    for (int r = 0; r < ngates; ++r) {
        rev[r] = gates[ngates - 1 - r];
        rev[r].kind ^= SV_G_ADJOINT;
    }
    // generator of every differentiated gate (A with dU/dtheta = A U; A^dag
    // for a gate given with the adjoint flag, as A commutes with U)
    a->gen_slot.assign(ngates, -1);
    std::vector<double> gen;
    std::vector<std::vector<int>> param_slots(nparams);
    for (int r = 0; r < ngates; ++r) {
        const sv_gate_t &g = gates[ngates - 1 - r];
        if (g.param < 0)
            continue;
        double A[8];
        gate_generator(g.kind, A);
        if (g.kind & SV_G_ADJOINT) {
            for (int k = 1; k < 8; k += 2)
                A[k] = -A[k];
            std::swap(A[2], A[4]);
            std::swap(A[3], A[5]);
        }
        a->gen_slot[r] = (int)(gen.size() / 8);
        gen.insert(gen.end(), A, A + 8);
        param_slots[g.param].push_back(a->gen_slot[r]);
    }
    const int nslots = (int)(gen.size() / 8);
    a->nslots = nslots;
    const int m_cap = std::max(1, tuning().tile_log2[dtype == SV_C128 ? 0 : 1] - 1);
    SV_TRY(circuit_create(n, dtype, rev.data(), ngates, nparams, SV_FUSE, async, st, m_cap, &a->rc));
    sv_circuit *rc = a->rc;

    // per pass: single passes need pair plans, fused ones per-descriptor slots
    a->single_plan.assign(rc->passes.size(), GatePlan());
    std::vector<int32_t> dslot(rc->tile_src.size(), -1);
    std::vector<int32_t> slot_blocks(std::max(1, nslots), 1);
    for (size_t pi = 0; pi < rc->passes.size(); ++pi) {
        const Pass &p = rc->passes[pi];
        if (p.fused) {
            const unsigned grid = (unsigned)std::min<uint64_t>(p.tm.ntiles, kMaxPartials);
            for (int j = 0; j < p.count; ++j) {
                const int gi = rc->tile_src[p.first + j];
                dslot[p.first + j] = a->gen_slot[gi];
                if (a->gen_slot[gi] >= 0)
                    slot_blocks[a->gen_slot[gi]] = (int32_t)grid;
            }
        } else {
            const sv_gate_t &g = rev[p.gate];
            GateSpec gs{n, g.target, g.ctrl_mask, g.ctrl_vals};
            SV_TRY(make_gate_plan(gs, dtype, SV_MODE_PAIR, &a->single_plan[pi]));
            if (a->gen_slot[p.gate] >= 0)
                slot_blocks[a->gen_slot[p.gate]] = (int32_t)reduce_grid(a->single_plan[pi].niter);
        }
    }
    std::vector<int32_t> ints;  // CSR of slots per parameter, then blocks per slot
    {
        int32_t acc = 0;
        for (int j = 0; j < nparams; ++j) {
            ints.push_back(acc);
            acc += (int32_t)param_slots[j].size();
        }
        ints.push_back(acc);
        for (int j = 0; j < nparams; ++j)
            for (int sidx : param_slots[j])
                ints.push_back(sidx);
        ints.insert(ints.end(), slot_blocks.begin(), slot_blocks.begin() + nslots);
    }
    a->off_slots = (size_t)nparams + 1;
    a->off_blocks = a->off_slots + (size_t)nslots;

    auto alloc = [&](void **ptr, size_t bytes) -> int {
        if (bytes == 0)
            return SV_OK;
        hipError_t e = async ? hipMallocAsync(ptr, bytes, st) : hipMalloc(ptr, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *ptr = nullptr;
            return fail(SV_ENOMEM, "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        }
        return SV_OK;
    };
    auto put = [&](void *dst, const void *src, size_t bytes) -> int {
        if (bytes == 0)
            return SV_OK;
        hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
        return e == hipSuccess ? SV_OK : fail(SV_EHIP, "copy failed: %s", hipGetErrorString(e));
    };
    SV_TRY(alloc((void **)&a->d_gen, gen.size() * sizeof(double)));
    SV_TRY(alloc((void **)&a->d_partials, ((size_t)nslots + 1) * kMaxPartials * sizeof(double)));
    SV_TRY(alloc((void **)&a->d_ints, ints.size() * sizeof(int32_t)));
    SV_TRY(alloc((void **)&a->d_dslot, dslot.size() * sizeof(int32_t)));
    SV_TRY(put(a->d_gen, gen.data(), gen.size() * sizeof(double)));
    SV_TRY(put(a->d_ints, ints.data(), ints.size() * sizeof(int32_t)));
    SV_TRY(put(a->d_dslot, dslot.data(), dslot.size() * sizeof(int32_t)));
    SV_TRY(pauli_upload(pplan, 0, st, &a->pd));
    // dynamic LDS: the two tiles, then 8 accumulators per parameterised gate
    // of the pass (sized for the largest pass)
    a->pass_lds.assign(rc->passes.size(), 0);
    size_t lds = 0;
    for (size_t pi = 0; pi < rc->passes.size(); ++pi) {
        const Pass &p = rc->passes[pi];
        if (!p.fused)
            continue;
        size_t npg = 0;
        for (int j = 0; j < p.count; ++j)
            npg += dslot[p.first + j] >= 0 ? 1 : 0;
        a->pass_lds[pi] = ((size_t)2 << rc->m) * amp_bytes(dtype) + npg * (kAdjTileThreads / 64) * sizeof(double);
        lds = std::max(lds, a->pass_lds[pi]);
    }
    constexpr size_t kLdsPerWorkgroup = 160 * 1024;  // gfx950, with the opt-in limit raised
    if (lds > kLdsPerWorkgroup)
        return fail(SV_ENOTSUP, "adjoint pass needs %zu bytes of LDS", lds);
    if (lds > 65536) {
        const hipError_t e = dtype == SV_C128 ? hipFuncSetAttribute((const void *)k_adj_tile<double>,
                                                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                                                    (int)lds)
                                              : hipFuncSetAttribute((const void *)k_adj_tile<float>,
                                                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                                                    (int)lds);
        if (e != hipSuccess)
            return fail(SV_EHIP, "LDS limit for %zu bytes: %s", lds, hipGetErrorString(e));
    }
    if (!async)
        SV_HIP_TRY(hipStreamSynchronize(st));  // the tables are in place before the plan is handed out
    return SV_OK;
}

// Enqueue one reverse sweep: lambda = H psi (and the loss partials), the
// passes of the reverse plan, the fixed-order final sums.
static int adjoint_enqueue(AdjointPlan *a, const sv_state_t *psi, const sv_state_t *lam, const double *params,
                           double *grad, double *loss, const double *scale, hipStream_t st) {
    sv_circuit *rc = a->rc;
    const int n = a->n, dtype = a->dtype, nparams = a->nparams;
    double *loss_partials = a->d_partials + (size_t)a->nslots * kMaxPartials;
    a->pd.partials = loss_partials;  // borrowed
    unsigned loss_blocks = 1;
    SV_TRY(circuit_param_mats(rc, params, st));
    SV_TRY(launch_apply_paulis(dtype, psi->data, lam->data, n, a->pd, st, &loss_blocks));
    for (size_t pi = 0; pi < rc->passes.size(); ++pi) {
        const Pass &p = rc->passes[pi];
        if (p.fused) {
            const unsigned grid = (unsigned)std::min<uint64_t>(p.tm.ntiles, kMaxPartials);
            const DeviceGates dg{rc->d_tiles + p.first, p.count};
            if (dtype == SV_C128)
                hipLaunchKernelGGL(k_adj_tile<double>, dim3(grid), dim3(kAdjTileThreads), a->pass_lds[pi], st,
                                   (double2 *)psi->data, (double2 *)lam->data, p.tm, dg, a->d_dslot + p.first,
                                   a->d_gen, a->d_partials);
            else
                hipLaunchKernelGGL(k_adj_tile<float>, dim3(grid), dim3(kAdjTileThreads), a->pass_lds[pi], st,
                                   (float2 *)psi->data, (float2 *)lam->data, p.tm, dg, a->d_dslot + p.first,
                                   a->d_gen, a->d_partials);
        } else {
            const GatePlan &gp = a->single_plan[pi];
            const int gi = p.gate;
            const unsigned grid = reduce_grid(gp.niter);
            const double *gptr = a->gen_slot[gi] >= 0 ? a->d_gen + (size_t)8 * a->gen_slot[gi] : nullptr;
            double *part = a->gen_slot[gi] >= 0 ? a->d_partials + (size_t)a->gen_slot[gi] * kMaxPartials : nullptr;
            if (dtype == SV_C128)
                launch_adj<double>(psi->data, lam->data, gp, rc->d_mats + (size_t)8 * gi, gptr, part, grid, st);
            else
                launch_adj<float>(psi->data, lam->data, gp, rc->d_mats + (size_t)8 * gi, gptr, part, grid, st);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return fail(SV_EHIP, "adjoint launch failed: %s", hipGetErrorString(e));
    }
    if (nparams > 0 || loss) {
        hipLaunchKernelGGL(k_grad_final, dim3((unsigned)nparams + 1), dim3(kRedThreads), 0, st, nparams, a->d_ints,
                           a->d_ints + a->off_slots, a->d_ints + a->off_blocks, a->d_partials, loss_partials,
                           (int)loss_blocks, scale, grad, loss);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return fail(SV_EHIP, "launch failed: %s", hipGetErrorString(e));
    }
    return SV_OK;
}

static int check_adjoint_states(const sv_state_t *psi, const sv_state_t *lam, int n, int dtype) {
    SV_TRY(validate_state(psi));
    SV_TRY(validate_state(lam));
    if (psi->n != lam->n || psi->dtype != lam->dtype)
        return fail(SV_EINVAL, "psi and lambda differ in size or dtype");
    if (psi->data == lam->data)
        return fail(SV_EINVAL, "psi and lambda must be different buffers");
    if (psi->n != n || psi->dtype != dtype)
        return fail(SV_EINVAL, "states (n=%d, dtype %d) do not match the plan (n=%d, dtype %d)", psi->n, psi->dtype, n,
                    dtype);
    return SV_OK;
}

int adjoint_impl(const sv_state_t *psi, const sv_state_t *lam, const sv_gate_t *gates, int ngates,
                 const double *params, int nparams, const sv_pauli_t *terms, int nterms, double *grad, double *loss,
                 const double *scale, hipStream_t st) {
    SV_TRY(validate_state(psi));
    if (nparams < 0 || (nparams > 0 && (!params || !grad)))
        return fail(SV_EINVAL, "nparams %d needs params_dev and grad_dev", nparams);
    SV_TRY(check_adjoint_states(psi, lam, psi->n, psi->dtype));
    AdjointPlan a;
    int r = adjoint_plan(psi->n, psi->dtype, gates, ngates, nparams, terms, nterms, true, st, &a);
    if (r == SV_OK)
        r = adjoint_enqueue(&a, psi, lam, params, grad, loss, scale, st);
    adjoint_free(&a, st);
    return r;
}

} // namespace sv

using namespace sv;

extern "C" {

int sv_adjoint_grad(const sv_state_t *psi, const sv_state_t *lam, const sv_gate_t *gates, int ngates,
                    const double *params_dev, int nparams, const sv_pauli_t *terms, int nterms, double *grad_dev,
                    double *loss_dev, const double *scale_dev, sv_stream_t st) {
    clear_error();
    return adjoint_impl(psi, lam, gates, ngates, params_dev, nparams, terms, nterms, grad_dev, loss_dev, scale_dev,
                        (hipStream_t)st);
}

int sv_adjoint_create(int n, int dtype, const sv_gate_t *gates, int ngates, int nparams, const sv_pauli_t *terms,
                      int nterms, sv_adjoint_t **out) {
    clear_error();
    if (!out)
        return fail(SV_EINVAL, "out is NULL");
    *out = nullptr;
    auto *a = new AdjointPlan();
    const int r = adjoint_plan(n, dtype, gates, ngates, nparams, terms, nterms, false, nullptr, a);
    if (r != SV_OK) {
        adjoint_free(a, nullptr);
        delete a;
        return r;
    }
    *out = reinterpret_cast<sv_adjoint_t *>(a);
    return SV_OK;
}

int sv_adjoint_run(sv_adjoint_t *plan, const sv_state_t *psi, const sv_state_t *lam, const double *params_dev,
                   double *grad_dev, double *loss_dev, const double *scale_dev, sv_stream_t st) {
    clear_error();
    if (!plan)
        return fail(SV_EINVAL, "plan is NULL");
    auto *a = reinterpret_cast<AdjointPlan *>(plan);
    SV_TRY(check_adjoint_states(psi, lam, a->n, a->dtype));
    if (a->nparams > 0 && (!params_dev || !grad_dev))
        return fail(SV_EINVAL, "nparams %d needs params_dev and grad_dev", a->nparams);
    int dev = 0;
    SV_HIP_TRY(hipGetDevice(&dev));
    if (dev != a->device)
        return fail(SV_EINVAL, "plan was made on device %d, current device is %d", a->device, dev);
    return adjoint_enqueue(a, psi, lam, params_dev, grad_dev, loss_dev, scale_dev, (hipStream_t)st);
}

int sv_adjoint_destroy(sv_adjoint_t *plan) {
    clear_error();
    if (!plan)
        return SV_OK;
    auto *a = reinterpret_cast<AdjointPlan *>(plan);
    (void)hipDeviceSynchronize();  // runs enqueued earlier may still read the tables
    adjoint_free(a, nullptr);
    delete a;
    return SV_OK;
}

} // extern "C"
