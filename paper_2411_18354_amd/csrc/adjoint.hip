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

#include "gates.hpp"
#include "pauli.hpp"

namespace sv {

int validate_circuit_gate(int n, int nparams, const sv_gate_t &g, int index);

struct AdjJob {
    int32_t kind;   // kind of the inverse gate
    int32_t param;
    int32_t gate;
};

__global__ void k_adj_mats(const AdjJob *__restrict__ jobs, int njobs, const double *__restrict__ params,
                           double *__restrict__ udag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= njobs)
        return;
    const AdjJob j = jobs[i];
    gate_matrix(j.kind, params[j.param], nullptr, udag + (size_t)8 * j.gate);
}

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

struct AdjBuffers {
    double *udag = nullptr, *gen = nullptr, *partials = nullptr;
    AdjJob *jobs = nullptr;
    int32_t *ints = nullptr;
};

static void adj_release(AdjBuffers *b, hipStream_t st) {
    void *ps[] = {b->udag, b->gen, b->partials, b->jobs, b->ints};
    for (void *p : ps)
        if (p)
            (void)hipFreeAsync(p, st);
    *b = AdjBuffers();
}

int adjoint_impl(const sv_state_t *psi, const sv_state_t *lam, const sv_gate_t *gates, int ngates,
                 const double *params, int nparams, const sv_pauli_t *terms, int nterms, double *grad, double *loss,
                 const double *scale, hipStream_t st) {
    SV_TRY(validate_state(psi));
    SV_TRY(validate_state(lam));
    if (psi->n != lam->n || psi->dtype != lam->dtype)
        return fail(SV_EINVAL, "psi and lambda differ in size or dtype");
    if (psi->data == lam->data)
        return fail(SV_EINVAL, "psi and lambda must be different buffers");
    if (ngates < 0 || (ngates > 0 && !gates))
        return fail(SV_EINVAL, "bad gate list");
    if (nparams < 0 || (nparams > 0 && (!params || !grad)))
        return fail(SV_EINVAL, "nparams %d needs params_dev and grad_dev", nparams);
    const int n = psi->n;
    for (int i = 0; i < ngates; ++i)
        SV_TRY(validate_circuit_gate(n, nparams, gates[i], i));
    PauliPlan pplan;
    SV_TRY(make_pauli_plan(n, terms, nterms, &pplan));

    // host tables
    std::vector<GatePlan> plans(ngates);
    std::vector<double> udag((size_t)8 * std::max(1, ngates), 0.0);
    std::vector<double> gen;
    std::vector<int> gen_slot(ngates, -1);
    std::vector<AdjJob> jobs;
    std::vector<std::vector<int>> param_slots(nparams);
    for (int i = 0; i < ngates; ++i) {
        const sv_gate_t &g = gates[i];
        GateSpec gs{n, g.target, g.ctrl_mask, g.ctrl_vals};
        SV_TRY(make_gate_plan(gs, psi->dtype, SV_MODE_PAIR, &plans[i]));
        const int inv = g.kind ^ SV_G_ADJOINT;
        if (g.param < 0) {
            gate_matrix(inv, g.theta, g.U, &udag[(size_t)8 * i]);
        } else {
            jobs.push_back(AdjJob{inv, g.param, i});
            double a[8];
            gate_generator(g.kind, a);
            if (g.kind & SV_G_ADJOINT) {
                // d/dtheta U^dag = (A U)^dag = U^dag A^dag = A^dag U^dag, as A
                // commutes with U for every parameterised kind: use A^dag
                for (int k = 1; k < 8; k += 2)
                    a[k] = -a[k];
                std::swap(a[2], a[4]);
                std::swap(a[3], a[5]);
            }
            gen_slot[i] = (int)(gen.size() / 8);
            gen.insert(gen.end(), a, a + 8);
            param_slots[g.param].push_back(gen_slot[i]);
        }
    }
    const int nslots = (int)(gen.size() / 8);
    // CSR of slots per parameter + blocks per slot
    std::vector<int32_t> ints;
    ints.reserve((size_t)nparams + 1 + 2 * (size_t)nslots);
    {
        int32_t acc = 0;
        for (int j = 0; j < nparams; ++j) {
            ints.push_back(acc);
            acc += (int32_t)param_slots[j].size();
        }
        ints.push_back(acc);
        for (int j = 0; j < nparams; ++j)
            for (int s : param_slots[j])
                ints.push_back(s);
        std::vector<int32_t> blocks(nslots, 1);
        for (int i = 0; i < ngates; ++i)
            if (gen_slot[i] >= 0)
                blocks[gen_slot[i]] = (int32_t)reduce_grid(plans[i].niter);
        ints.insert(ints.end(), blocks.begin(), blocks.end());
    }
    const size_t off_slots = (size_t)nparams + 1, off_blocks = off_slots + (size_t)nslots;

    // device buffers (stream-ordered)
    AdjBuffers B;
    PauliDevice pd;
    auto alloc = [&](void **p, size_t bytes) -> int {
        if (bytes == 0)
            return SV_OK;
        hipError_t e = hipMallocAsync(p, bytes, st);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
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
    int r = alloc((void **)&B.udag, udag.size() * sizeof(double));
    if (r == SV_OK)
        r = alloc((void **)&B.gen, gen.size() * sizeof(double));
    if (r == SV_OK)
        r = alloc((void **)&B.partials, ((size_t)nslots + 1) * kMaxPartials * sizeof(double));
    if (r == SV_OK)
        r = alloc((void **)&B.jobs, jobs.size() * sizeof(AdjJob));
    if (r == SV_OK)
        r = alloc((void **)&B.ints, ints.size() * sizeof(int32_t));
    if (r == SV_OK)
        r = put(B.udag, udag.data(), udag.size() * sizeof(double));
    if (r == SV_OK)
        r = put(B.gen, gen.data(), gen.size() * sizeof(double));
    if (r == SV_OK)
        r = put(B.jobs, jobs.data(), jobs.size() * sizeof(AdjJob));
    if (r == SV_OK)
        r = put(B.ints, ints.data(), ints.size() * sizeof(int32_t));
    if (r == SV_OK)
        r = pauli_upload(pplan, 0, st, &pd);
    if (r != SV_OK) {
        adj_release(&B, st);
        return r;
    }
    double *loss_partials = B.partials + (size_t)nslots * kMaxPartials;
    pd.partials = loss_partials;  // borrowed; released with B
    unsigned loss_blocks = 1;
    if (!jobs.empty()) {
        hipLaunchKernelGGL(k_adj_mats, dim3((unsigned)((jobs.size() + 127) / 128)), dim3(128), 0, st, B.jobs,
                           (int)jobs.size(), params, B.udag);
        r = hipGetLastError() == hipSuccess ? SV_OK : fail(SV_EHIP, "launch failed");
    }
    if (r == SV_OK)
        r = launch_apply_paulis(psi->dtype, psi->data, lam->data, n, pd, st, &loss_blocks);
    for (int i = ngates - 1; i >= 0 && r == SV_OK; --i) {
        const GatePlan &p = plans[i];
        const unsigned grid = reduce_grid(p.niter);
        const double *gptr = gen_slot[i] >= 0 ? B.gen + (size_t)8 * gen_slot[i] : nullptr;
        double *part = gen_slot[i] >= 0 ? B.partials + (size_t)gen_slot[i] * kMaxPartials : nullptr;
        if (psi->dtype == SV_C128)
            launch_adj<double>(psi->data, lam->data, p, B.udag + (size_t)8 * i, gptr, part, grid, st);
        else
            launch_adj<float>(psi->data, lam->data, p, B.udag + (size_t)8 * i, gptr, part, grid, st);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            r = fail(SV_EHIP, "adjoint launch failed: %s", hipGetErrorString(e));
    }
    if (r == SV_OK && (nparams > 0 || loss)) {
        hipLaunchKernelGGL(k_grad_final, dim3((unsigned)nparams + 1), dim3(kRedThreads), 0, st, nparams, B.ints,
                           B.ints + off_slots, B.ints + off_blocks, B.partials, loss_partials, (int)loss_blocks, scale,
                           grad, loss);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            r = fail(SV_EHIP, "launch failed: %s", hipGetErrorString(e));
    }
    pd.partials = nullptr;
    pauli_release(&pd, st);
    adj_release(&B, st);
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

} // extern "C"
