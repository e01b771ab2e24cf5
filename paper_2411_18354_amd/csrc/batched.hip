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
//    circuit's fused plan: fused runs tile by tile through LDS, other gates as
//    pair loops over the state; a workgroup barrier separates passes.
// Each gate visits only the amplitude pairs whose controls hold: the pair
// index is built by inserting the target bit (0) and the control bits (their
// values) into the iteration counter, lowest position first (Sec. III-B).
#include <algorithm>
#include <cstring>
#include <numeric>

#include "gates.hpp"
#include "pauli.hpp"

namespace sv {

int validate_circuit_gate(int n, int nparams, const sv_gate_t &g, int index);
int circuit_plan_capped(int n, int dtype, const sv_gate_t *gates, int ngates, int nparams, int flags, int m_cap,
                        int32_t *order, int32_t *pass_of, int64_t *npasses, int *m_used, bool general);

constexpr int kBatchThreads = 512;
constexpr size_t kBatchLds = 65536;

struct BGate {
    double m[8];      // matrix of a fixed gate
    int32_t kind;     // matrix recomputed from params[param] when param >= 0
    int32_t param;    // index into the concatenated parameter array, or -1
    int32_t target;
    int32_t pass;     // pass number within its circuit (fused runs share one)
    uint64_t cmask, cvals;
};

struct BCirc {
    void *psi;
    void *lam;           // adjoint only
    int32_t n;
    int32_t m;           // tile width of the fused plan
    int32_t first_gate;  // gates [first_gate, first_gate + ngates), in execution order
    int32_t ngates;
    int32_t first_param, nparams;  // adjoint: gradient slots
    int32_t first_term, nterms;    // adjoint: Hamiltonian terms
};

// Insert the target bit (0) and the control bits (their values) into x,
// lowest position first.
__device__ __forceinline__ uint64_t insert_bits(uint64_t x, uint64_t positions, uint64_t vals) {
    while (positions) {
        const int p = __builtin_ctzll(positions);
        positions &= positions - 1;
        const uint64_t lo = x & ((1ull << p) - 1);
        x = ((x >> p) << (p + 1)) | (((vals >> p) & 1ull) << p) | lo;
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

// Apply one gate to amplitudes held at base[0 .. 2^nbits) (LDS or global),
// controls below nbits enumerated, controls at or above nbits already known
// to hold.
template <typename R>
__device__ __forceinline__ void gate_on_block(cplx_t<R> *base, int nbits, const BGate &g, const Mat2<R> &mm) {
    const uint64_t lowm = (1ull << nbits) - 1;
    const uint64_t cm = g.cmask & lowm;
    const uint64_t pos = cm | (1ull << g.target);
    const uint64_t npairs = 1ull << (nbits - 1 - __popcll(cm));
    const uint64_t st = 1ull << g.target;
    const uint64_t cv = g.cvals & cm;
    constexpr int U = 4;  // pairs per lane per step: 2U loads in flight
    for (uint64_t i0 = threadIdx.x; i0 < npairs; i0 += (uint64_t)U * kBatchThreads) {
        cplx_t<R> x[U], y[U];
        uint64_t p1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = i0 + (uint64_t)u * kBatchThreads;
            p1[u] = insert_bits(i, pos, cv);
            if (i < npairs) {
                x[u] = base[p1[u]];
                y[u] = base[p1[u] | st];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (i0 + (uint64_t)u * kBatchThreads < npairs) {
                apply_pair<R>(mm, x[u], y[u]);
                base[p1[u]] = x[u];
                base[p1[u] | st] = y[u];
            }
        }
    }
}

template <typename R>
__device__ void run_circuit_block(const BCirc &c, const BGate *__restrict__ gates, const double *__restrict__ params,
                                  cplx_t<R> *lds) {
    cplx_t<R> *psi = reinterpret_cast<cplx_t<R> *>(c.psi);
    const uint64_t N = 1ull << c.n;
    if (N * sizeof(cplx_t<R>) <= kBatchLds) {
        for (uint64_t k = threadIdx.x; k < N; k += kBatchThreads)
            lds[k] = psi[k];
        __syncthreads();
        for (int i = 0; i < c.ngates; ++i) {
            const BGate &g = gates[c.first_gate + i];
            gate_on_block<R>(lds, c.n, g, bgate_mat<R>(g, params, false));
            __syncthreads();
        }
        for (uint64_t k = threadIdx.x; k < N; k += kBatchThreads)
            psi[k] = lds[k];
        return;
    }
    const uint64_t T = 1ull << c.m;
    int i = 0;
    while (i < c.ngates) {
        const int pass = gates[c.first_gate + i].pass;
        int j = i;
        while (j < c.ngates && gates[c.first_gate + j].pass == pass)
            ++j;
        if (j - i > 1) {  // fused run: every target < m
            for (uint64_t base = 0; base < N; base += T) {
                bool any = false;
                for (int k = i; k < j; ++k) {
                    const BGate &g = gates[c.first_gate + k];
                    const uint64_t hm = g.cmask & ~(T - 1);
                    any |= (base & hm) == (g.cvals & hm);
                }
                if (!any)
                    continue;
                for (uint64_t k = threadIdx.x; k < T; k += kBatchThreads)
                    lds[k] = psi[base + k];
                __syncthreads();
                for (int k = i; k < j; ++k) {
                    const BGate &g = gates[c.first_gate + k];
                    const uint64_t hm = g.cmask & ~(T - 1);
                    if ((base & hm) != (g.cvals & hm))
                        continue;
                    gate_on_block<R>(lds, c.m, g, bgate_mat<R>(g, params, false));
                    __syncthreads();
                }
                for (uint64_t k = threadIdx.x; k < T; k += kBatchThreads)
                    psi[base + k] = lds[k];
                __syncthreads();
            }
        } else {
            const BGate &g = gates[c.first_gate + i];
            gate_on_block<R>(psi, c.n, g, bgate_mat<R>(g, params, false));
            __syncthreads();
        }
        i = j;
    }
}

template <typename R>
__global__ __launch_bounds__(kBatchThreads) void k_batched(const BCirc *__restrict__ circs,
                                                           const int32_t *__restrict__ order, int ncirc,
                                                           const BGate *__restrict__ gates,
                                                           const double *__restrict__ params,
                                                           unsigned int *__restrict__ queue) {
    extern __shared__ unsigned char lds_raw[];
    cplx_t<R> *lds = reinterpret_cast<cplx_t<R> *>(lds_raw);
    int *item = reinterpret_cast<int *>(lds_raw + kBatchLds);
    for (;;) {
        if (threadIdx.x == 0)
            *item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int it = *item;
        __syncthreads();
        if (it >= ncirc)
            break;
        run_circuit_block<R>(circs[order[it]], gates, params, lds);
        __syncthreads();
    }
}

__global__ void k_zero_u32(unsigned int *p) { *p = 0u; }

// ----------------------------------------------------------------- adjoint

// One circuit's adjoint inside one workgroup: lambda = H psi (and the loss),
// then the reverse sweep with per-gate gradient sums reduced in the
// workgroup (a fixed order, so results are reproducible).
template <typename R>
__device__ void adjoint_block(const BCirc &c, const BGate *__restrict__ gates, const double *__restrict__ params,
                              const DTerm *__restrict__ terms, const double *__restrict__ gens,
                              const int32_t *__restrict__ gen_of, double *__restrict__ grad,
                              double *__restrict__ loss, double *scratch) {
    cplx_t<R> *psi = reinterpret_cast<cplx_t<R> *>(c.psi);
    cplx_t<R> *lam = reinterpret_cast<cplx_t<R> *>(c.lam);
    const uint64_t N = 1ull << c.n;
    for (int j = threadIdx.x; j < c.nparams; j += kBatchThreads)
        grad[c.first_param + j] = 0.0;
    // lambda = H psi; terms are sorted by x mask
    double lp = 0.0;
    for (uint64_t k = threadIdx.x; k < N; k += kBatchThreads) {
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
    for (int i = c.ngates - 1; i >= 0; --i) {
        const BGate &g = gates[c.first_gate + i];
        const Mat2<R> ud = bgate_mat<R>(g, params, true);
        const int gs = gen_of[c.first_gate + i];
        double a[8];
        for (int k = 0; k < 8; ++k)
            a[k] = gs >= 0 ? gens[8 * gs + k] : 0.0;
        const uint64_t pos = g.cmask | (1ull << g.target);
        const uint64_t npairs = 1ull << (c.n - 1 - __popcll(g.cmask));
        const uint64_t st = 1ull << g.target;
        double acc = 0.0;
        for (uint64_t it = threadIdx.x; it < npairs; it += kBatchThreads) {
            const uint64_t p1 = insert_bits(it, pos, g.cvals);
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
}

template <typename R>
__global__ __launch_bounds__(kBatchThreads) void k_batched_adjoint(
    const BCirc *__restrict__ circs, const int32_t *__restrict__ order, int ncirc, const BGate *__restrict__ gates,
    const double *__restrict__ params, const DTerm *__restrict__ terms, const double *__restrict__ gens,
    const int32_t *__restrict__ gen_of, double *__restrict__ grad, double *__restrict__ loss,
    unsigned int *__restrict__ queue) {
    __shared__ double scratch[kBatchThreads / 64];
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
        adjoint_block<R>(circs[ci], gates, params, terms, gens, gen_of, grad, loss + ci, scratch);
        __syncthreads();
    }
}

// ----------------------------------------------------------------- host

struct BatchHost {
    std::vector<BCirc> circs;
    std::vector<BGate> gates;
    std::vector<int32_t> order;
    std::vector<double> gens;
    std::vector<int32_t> gen_of;
    std::vector<DTerm> terms;
};

static int build_batch(const sv_state_t *states, const sv_state_t *lams, int ncirc, const sv_gate_t *gates,
                       const int64_t *gate_off, const int64_t *param_off, int64_t nparams_total,
                       const sv_pauli_t *terms, const int64_t *term_off, bool adjoint, BatchHost *h, int *dtype) {
    if (ncirc < 1 || !states || !gate_off || (gate_off[ncirc] > 0 && !gates))
        return fail(SV_EINVAL, "bad batch description (ncirc %d)", ncirc);
    *dtype = states[0].dtype;
    std::vector<double> cost(ncirc);
    const int tl = tuning().tile_log2[*dtype == SV_C128 ? 0 : 1];
    for (int c = 0; c < ncirc; ++c) {
        const sv_state_t &s = states[c];
        int r = validate_state(&s);
        if (r != SV_OK)
            return fail(r, "circuit %d: %s", c, sv_last_error());
        if (s.dtype != *dtype)
            return fail(SV_EINVAL, "circuit %d: all states of a batch need one dtype", c);
        if (adjoint) {
            r = validate_state(&lams[c]);
            if (r != SV_OK)
                return fail(r, "circuit %d (lambda): %s", c, sv_last_error());
            if (lams[c].n != s.n || lams[c].dtype != s.dtype || lams[c].data == s.data)
                return fail(SV_EINVAL, "circuit %d: lambda must be a distinct state of the same shape", c);
        }
        const int64_t g0 = gate_off[c], g1 = gate_off[c + 1];
        if (g0 < 0 || g1 < g0)
            return fail(SV_EINVAL, "circuit %d: bad gate offsets", c);
        const int64_t p0 = param_off ? param_off[c] : 0, p1 = param_off ? param_off[c + 1] : 0;
        if (p0 < 0 || p1 < p0 || p1 > nparams_total)
            return fail(SV_EINVAL, "circuit %d: bad parameter offsets", c);
        BCirc bc;
        memset(&bc, 0, sizeof(bc));
        bc.psi = s.data;
        bc.lam = adjoint ? lams[c].data : nullptr;
        bc.n = s.n;
        // the fused tiles must fit the workgroup's LDS buffer
        const int m_cap = *dtype == SV_C128 ? 12 : 13;  // 2^m amplitudes <= kBatchLds bytes
        bc.m = std::min(std::min(tl, s.n), m_cap);
        bc.first_gate = (int32_t)h->gates.size();
        bc.ngates = (int32_t)(g1 - g0);
        bc.first_param = (int32_t)p0;
        bc.nparams = (int32_t)(p1 - p0);
        // fused plan of this circuit (host planner, shared with sv_circuit_plan)
        std::vector<int32_t> ord(bc.ngates), pas(bc.ngates);
        if (bc.ngates > 0) {
            for (int64_t i = g0; i < g1; ++i) {
                r = validate_circuit_gate(s.n, (int)(p1 - p0), gates[i], (int)(i - g0));
                if (r != SV_OK)
                    return fail(r, "circuit %d: %s", c, sv_last_error());
            }
            if (adjoint) {
                std::iota(ord.begin(), ord.end(), 0);
                std::iota(pas.begin(), pas.end(), 0);
            } else {
                int64_t np = 0;
                int m_used = 0;
                r = circuit_plan_capped(s.n, *dtype, gates + g0, bc.ngates, (int)(p1 - p0), SV_FUSE, m_cap,
                                        ord.data(), pas.data(), &np, &m_used, false);
                if (r != SV_OK)
                    return fail(r, "circuit %d: %s", c, sv_last_error());
                if (m_used != bc.m)
                    return fail(SV_EINVAL, "circuit %d: planner tile width %d != %d", c, m_used, bc.m);
            }
        }
        double work = 0.0;
        for (int k = 0; k < bc.ngates; ++k) {
            const sv_gate_t &g = gates[g0 + ord[k]];
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
            b.pass = pas[k];
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
                gs = (int)(h->gens.size() / 8);
                h->gens.insert(h->gens.end(), a, a + 8);
            }
            h->gen_of.push_back(gs);
            h->gates.push_back(b);
            work += std::ldexp(1.0, s.n - popcount64(g.ctrl_mask));
        }
        if (adjoint) {
            if (!term_off || !terms)
                return fail(SV_EINVAL, "batched adjoint needs terms and term offsets");
            const int64_t t0 = term_off[c], t1 = term_off[c + 1];
            if (t0 < 0 || t1 <= t0)
                return fail(SV_EINVAL, "circuit %d: needs at least one term", c);
            const uint64_t full = (1ull << s.n) - 1;
            bc.first_term = (int32_t)h->terms.size();
            bc.nterms = (int32_t)(t1 - t0);
            for (int64_t j = t0; j < t1; ++j) {
                if ((terms[j].x_mask | terms[j].z_mask) & ~full)
                    return fail(SV_EINVAL, "circuit %d: term %lld acts on qubits >= n", c, (long long)(j - t0));
                DTerm d;
                d.coef = terms[j].coef;
                d.z = terms[j].z_mask;
                d.ny = popcount64(terms[j].x_mask & terms[j].z_mask) & 3;
                d.idx = (int32_t)terms[j].x_mask;  // x mask (n <= 31 in batches)
                h->terms.push_back(d);
            }
            work *= 2.0;
            if (s.n > 31)
                return fail(SV_EINVAL, "circuit %d: batched adjoint supports n <= 31", c);
        }
        cost[c] = work;
        h->circs.push_back(bc);
    }
    h->order.resize(ncirc);
    std::iota(h->order.begin(), h->order.end(), 0);
    std::stable_sort(h->order.begin(), h->order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    return SV_OK;
}

struct BatchDevice {
    BCirc *circs = nullptr;
    BGate *gates = nullptr;
    int32_t *order = nullptr, *gen_of = nullptr;
    double *gens = nullptr;
    DTerm *terms = nullptr;
    unsigned int *queue = nullptr;
};

static void batch_release(BatchDevice *d, hipStream_t st) {
    void *ps[] = {d->circs, d->gates, d->order, d->gen_of, d->gens, d->terms, d->queue};
    for (void *p : ps)
        if (p)
            (void)hipFreeAsync(p, st);
    *d = BatchDevice();
}

template <typename T> static int dev_copy(T **dst, const std::vector<T> &src, hipStream_t st, size_t min_count = 0) {
    const size_t cnt = std::max(src.size(), min_count);
    *dst = nullptr;
    if (cnt == 0)
        return SV_OK;
    hipError_t e = hipMallocAsync((void **)dst, cnt * sizeof(T), st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return fail(SV_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    if (!src.empty())
        SV_HIP_TRY(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return SV_OK;
}

static int upload_batch(const BatchHost &h, hipStream_t st, BatchDevice *d) {
    int r = dev_copy(&d->circs, h.circs, st);
    if (r == SV_OK)
        r = dev_copy(&d->gates, h.gates, st, 1);
    if (r == SV_OK)
        r = dev_copy(&d->order, h.order, st);
    if (r == SV_OK)
        r = dev_copy(&d->gen_of, h.gen_of, st, 1);
    if (r == SV_OK)
        r = dev_copy(&d->gens, h.gens, st, 8);
    if (r == SV_OK)
        r = dev_copy(&d->terms, h.terms, st, 1);
    if (r == SV_OK) {
        hipError_t e = hipMallocAsync((void **)&d->queue, sizeof(unsigned int), st);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            r = fail(SV_ENOMEM, "device allocation failed");
        }
    }
    if (r != SV_OK)
        batch_release(d, st);
    return r;
}

static unsigned persistent_grid(int ncirc) {
    DeviceInfo di;
    if (device_info(&di) != SV_OK)
        return 256;
    const unsigned g = (unsigned)di.num_cus * 2;  // two 512-lane workgroups per CU
    return std::min<unsigned>(g, (unsigned)ncirc);
}

} // namespace sv

using namespace sv;

extern "C" {

int sv_apply_circuits_batched(const sv_state_t *states, int ncirc, const sv_gate_t *gates, const int64_t *gate_offsets,
                              const double *params_dev, const int64_t *param_offsets, int64_t nparams_total,
                              sv_stream_t st) {
    clear_error();
    BatchHost h;
    int dtype = 0;
    SV_TRY(build_batch(states, nullptr, ncirc, gates, gate_offsets, param_offsets, nparams_total, nullptr, nullptr,
                       false, &h, &dtype));
    if (nparams_total > 0 && !params_dev)
        return fail(SV_EINVAL, "params_dev is NULL");
    BatchDevice d;
    hipStream_t s = (hipStream_t)st;
    SV_TRY(upload_batch(h, s, &d));
    const unsigned grid = persistent_grid(ncirc);
    constexpr size_t lds = kBatchLds + 64;  // the tile, then the work-item slot
    hipError_t a = dtype == SV_C128 ? hipFuncSetAttribute((const void *)k_batched<double>,
                                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                                    : hipFuncSetAttribute((const void *)k_batched<float>,
                                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (a != hipSuccess) {
        batch_release(&d, s);
        return fail(SV_EHIP, "LDS limit: %s", hipGetErrorString(a));
    }
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, d.queue);
    if (dtype == SV_C128)
        hipLaunchKernelGGL(k_batched<double>, dim3(grid), dim3(kBatchThreads), lds, s, d.circs, d.order, ncirc,
                           d.gates, params_dev, d.queue);
    else
        hipLaunchKernelGGL(k_batched<float>, dim3(grid), dim3(kBatchThreads), lds, s, d.circs, d.order, ncirc,
                           d.gates, params_dev, d.queue);
    hipError_t e = hipGetLastError();
    batch_release(&d, s);
    if (e != hipSuccess)
        return fail(SV_EHIP, "batched launch failed: %s", hipGetErrorString(e));
    return SV_OK;
}

int sv_adjoint_grad_batched(const sv_state_t *psi_states, const sv_state_t *lam_states, int ncirc,
                            const sv_gate_t *gates, const int64_t *gate_offsets, const double *params_dev,
                            const int64_t *param_offsets, int64_t nparams_total, const sv_pauli_t *terms,
                            const int64_t *term_offsets, double *grad_dev, double *loss_dev, sv_stream_t st) {
    clear_error();
    if (!lam_states || !grad_dev || !loss_dev || !param_offsets)
        return fail(SV_EINVAL, "batched adjoint needs lambda states, param offsets, grad_dev and loss_dev");
    BatchHost h;
    int dtype = 0;
    SV_TRY(build_batch(psi_states, lam_states, ncirc, gates, gate_offsets, param_offsets, nparams_total, terms,
                       term_offsets, true, &h, &dtype));
    if (nparams_total > 0 && !params_dev)
        return fail(SV_EINVAL, "params_dev is NULL");
    BatchDevice d;
    hipStream_t s = (hipStream_t)st;
    SV_TRY(upload_batch(h, s, &d));
    const unsigned grid = persistent_grid(ncirc);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, d.queue);
    if (dtype == SV_C128)
        hipLaunchKernelGGL(k_batched_adjoint<double>, dim3(grid), dim3(kBatchThreads), 0, s, d.circs, d.order, ncirc,
                           d.gates, params_dev, d.terms, d.gens, d.gen_of, grad_dev, loss_dev, d.queue);
    else
        hipLaunchKernelGGL(k_batched_adjoint<float>, dim3(grid), dim3(kBatchThreads), 0, s, d.circs, d.order, ncirc,
                           d.gates, params_dev, d.terms, d.gens, d.gen_of, grad_dev, loss_dev, d.queue);
    hipError_t e = hipGetLastError();
    batch_release(&d, s);
    if (e != hipSuccess)
        return fail(SV_EHIP, "batched adjoint launch failed: %s", hipGetErrorString(e));
    return SV_OK;
}

} // extern "C"
