// Pauli-sum expectation values <psi|H|psi> and the product H psi.
//
// For one x mask X != 0 the amplitudes pair up as (k, k ^ X); with b the
// lowest set bit of X and k running over indices with bit b clear, the two
// contributions of a pair to <psi|P|psi> are complex conjugates (P is
// Hermitian), so the term is 2 Re( conj(psi_k) i^{ny} (-1)^{z.(k^X)}
// psi_{k^X} ) summed over half the indices: one read of every amplitude per
// x-mask group, enumerated with the same index expansion as the gate
// kernels.  Diagonal terms (X = 0) sum |psi_k|^2 (-1)^{z.k}.  Terms of a
// group are evaluated together in one pass.  Reductions are deterministic
// (reduce.hpp).  Fixed-point states (SV_CQ16, SV_CQ32) are read through
// their codes: each amplitude is code * 2^scale of its 64-amplitude block,
// which double holds exactly, so an expectation of a fixed-point state is
// that of the decoded state with the same double arithmetic.
#include <algorithm>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <numeric>

#include "pauli.hpp"

namespace sv {

constexpr int kMaxT = 16;        // terms evaluated per pass
constexpr int kExpectLoads = 4;  // visits per lane loaded together

int make_pauli_plan(int n, const sv_pauli_t *terms, int nterms, PauliPlan *p) {
    if (nterms < 1 || !terms)
        return fail(SV_EINVAL, "need at least one term (nterms %d, terms %p)", nterms, (const void *)terms);
    const uint64_t full = (n >= 64) ? ~0ull : ((1ull << n) - 1);
    std::vector<int> idx(nterms);
    std::iota(idx.begin(), idx.end(), 0);
    for (int j = 0; j < nterms; ++j)
        if ((terms[j].x_mask | terms[j].z_mask) & ~full)
            return fail(SV_EINVAL, "term %d acts on qubits >= n=%d", j, n);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return terms[a].x_mask < terms[b].x_mask; });
    p->groups.clear();
    p->terms.clear();
    for (int k = 0; k < nterms; ++k) {
        const sv_pauli_t &t = terms[idx[k]];
        const bool start = p->groups.empty() || p->groups.back().x != t.x_mask || p->groups.back().count == kMaxT;
        if (start)
            p->groups.push_back(DGroup{t.x_mask, (int32_t)p->terms.size(), 0});
        DTerm d;
        d.coef = t.coef;
        d.z = t.z_mask;
        d.ny = popcount64(t.x_mask & t.z_mask) & 3;
        d.idx = idx[k];
        p->terms.push_back(d);
        p->groups.back().count++;
    }
    return SV_OK;
}

int pauli_upload(const PauliPlan &p, size_t partial_doubles, hipStream_t st, PauliDevice *d) {
    *d = PauliDevice();
    d->nterms = (int)p.terms.size();
    d->ngroups = (int)p.groups.size();
    auto alloc = [&](void **ptr, size_t bytes) -> int {
        hipError_t e = hipMallocAsync(ptr, bytes, st);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *ptr = nullptr;
            return fail(SV_ENOMEM, "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        }
        return SV_OK;
    };
    int r = alloc((void **)&d->terms, p.terms.size() * sizeof(DTerm));
    if (r == SV_OK)
        r = alloc((void **)&d->groups, p.groups.size() * sizeof(DGroup));
    if (r == SV_OK && partial_doubles)
        r = alloc((void **)&d->partials, partial_doubles * sizeof(double));
    if (r != SV_OK) {
        pauli_release(d, st);
        return r;
    }
    SV_HIP_TRY(hipMemcpyAsync(d->terms, p.terms.data(), p.terms.size() * sizeof(DTerm), hipMemcpyHostToDevice, st));
    SV_HIP_TRY(
        hipMemcpyAsync(d->groups, p.groups.data(), p.groups.size() * sizeof(DGroup), hipMemcpyHostToDevice, st));
    return SV_OK;
}

void pauli_release(PauliDevice *d, hipStream_t st) {
    if (d->terms)
        (void)hipFreeAsync(d->terms, st);
    if (d->groups)
        (void)hipFreeAsync(d->groups, st);
    if (d->partials)
        (void)hipFreeAsync(d->partials, st);
    *d = PauliDevice();
}

// Amplitude sources for the expectation passes: amplitude k as two doubles.
template <typename R> struct CplxAmps {
    const cplx_t<R> *__restrict__ psi;
    __device__ void get(uint64_t k, double &re, double &im) const {
        const cplx_t<R> v = psi[k];
        re = (double)v.x;
        im = (double)v.y;
    }
};

// SV_CQ16: one 32-bit word per amplitude, re in the low half.
struct Q16Amps {
    const uint32_t *__restrict__ codes;
    const int8_t *__restrict__ scales;
    __device__ void get(uint64_t k, double &re, double &im) const {
        const uint32_t w = codes[k];
        const int s = scales[k >> 6];
        re = ldexp((double)(int16_t)(w & 0xffffu), s);
        im = ldexp((double)(int16_t)(w >> 16), s);
    }
};

// SV_CQ32: two 32-bit words per amplitude (re, im).
struct Q32Amps {
    const uint2 *__restrict__ codes;
    const int8_t *__restrict__ scales;
    __device__ void get(uint64_t k, double &re, double &im) const {
        const uint2 w = codes[k];
        const int s = scales[k >> 6];
        re = ldexp((double)(int32_t)w.x, s);
        im = ldexp((double)(int32_t)w.y, s);
    }
};

// One pass for one group (<= kMaxT terms sharing the x mask X).
// partials[(first + j) * kMaxPartials + block] receives the workgroup's sum
// of <P_j> contributions.
template <typename A>
__global__ __launch_bounds__(kRedThreads) void k_expect_group(const A amps, uint64_t count, uint64_t X, uint32_t b,
                                                              const DTerm *__restrict__ terms, int first, int nt,
                                                              double *__restrict__ partials) {
    __shared__ double red[kRedThreads / 64];
    uint64_t z[kMaxT];
    int ny[kMaxT];
    double acc[kMaxT];
#pragma unroll
    for (int j = 0; j < kMaxT; ++j) {
        acc[j] = 0.0;
        z[j] = j < nt ? terms[first + j].z : 0;
        ny[j] = j < nt ? terms[first + j].ny : 0;
    }
    // Each lane visits i0, i0 + stride, i0 + 2 stride, ...; kExpectLoads of
    // those visits load before any of them is summed, so enough bytes are in
    // flight for the narrow formats too.  The lane's summation order is that
    // of the visits.
    const uint64_t stride = (uint64_t)gridDim.x * kRedThreads;
    const uint64_t lowb = (1ull << b) - 1;
    const uint64_t i0 = (uint64_t)blockIdx.x * kRedThreads + threadIdx.x;
    if (X == 0) {
        for (uint64_t i = i0; i < count; i += kExpectLoads * stride) {
            double vr[kExpectLoads], vi[kExpectLoads];
#pragma unroll
            for (int u = 0; u < kExpectLoads; ++u)  // visits past the end load the last amplitude, unused
                amps.get(min(i + u * stride, count - 1), vr[u], vi[u]);
#pragma unroll
            for (int u = 0; u < kExpectLoads; ++u) {
                const uint64_t iu = i + u * stride;
                if (iu < count) {
                    const double pr = vr[u] * vr[u] + vi[u] * vi[u];
#pragma unroll
                    for (int j = 0; j < kMaxT; ++j)
                        if (j < nt)
                            acc[j] += odd_parity(z[j] & iu) ? -pr : pr;
                }
            }
        }
    } else {
        for (uint64_t i = i0; i < count; i += kExpectLoads * stride) {
            double ur[kExpectLoads], ui[kExpectLoads], vr[kExpectLoads], vi[kExpectLoads];
#pragma unroll
            for (int u = 0; u < kExpectLoads; ++u) {  // visits past the end load the last pair, unused
                const uint64_t iu = min(i + u * stride, count - 1);
                const uint64_t k = ((iu >> b) << (b + 1)) | (iu & lowb);  // bit b cleared
                amps.get(k, ur[u], ui[u]);
                amps.get(k ^ X, vr[u], vi[u]);
            }
#pragma unroll
            for (int u = 0; u < kExpectLoads; ++u) {
                const uint64_t iu = i + u * stride;
                if (iu < count) {
                    const uint64_t k2 = (((iu >> b) << (b + 1)) | (iu & lowb)) ^ X;
                    // w = conj(u) * v
                    const double wr = ur[u] * vr[u] + ui[u] * vi[u];
                    const double wi = ur[u] * vi[u] - ui[u] * vr[u];
#pragma unroll
                    for (int j = 0; j < kMaxT; ++j)
                        if (j < nt) {
                            const double r = re_ipow(ny[j], wr, wi);
                            acc[j] += odd_parity(z[j] & k2) ? -r : r;
                        }
                }
            }
        }
    }
    const double scale = X == 0 ? 1.0 : 2.0;
#pragma unroll
    for (int j = 0; j < kMaxT; ++j) {
        if (j < nt) {  // uniform
            const double s = block_sum(acc[j], red);
            if (threadIdx.x == 0)
                partials[(size_t)(first + j) * kMaxPartials + blockIdx.x] = scale * s;
        }
    }
}

// Every term's sum of its partials, one workgroup per term (plan order,
// each in the fixed order of block_sum_array).
__global__ __launch_bounds__(kRedThreads) void k_expect_sums(const int32_t *__restrict__ nblk,
                                                             const double *__restrict__ partials,
                                                             double *__restrict__ sums) {
    __shared__ double red[kRedThreads / 64];
    const int j = blockIdx.x;
    const double s = block_sum_array(partials + (size_t)j * kMaxPartials, nblk[j], red);
    if (threadIdx.x == 0)
        sums[j] = s;
}

// Per-term values in the caller's order, and the coefficient-weighted total
// summed in plan order by one lane.
__global__ __launch_bounds__(64) void k_expect_final(const DTerm *__restrict__ terms, int nterms,
                                                     const double *__restrict__ sums, double *__restrict__ out_total,
                                                     double *__restrict__ out_terms) {
    if (out_terms)
        for (int j = threadIdx.x; j < nterms; j += blockDim.x)
            out_terms[terms[j].idx] = sums[j];
    if (threadIdx.x == 0 && out_total) {
        double total = 0.0;
        for (int j = 0; j < nterms; ++j)
            total += terms[j].coef * sums[j];
        out_total[0] = total;
    }
}

// out_k = sum_groups sum_terms coef i^ny (-1)^{z.(k^X)} psi_{k^X}; partials
// of Re conj(psi_k) out_k per workgroup.
template <typename R>
__global__ __launch_bounds__(kRedThreads) void k_apply_paulis(const cplx_t<R> *__restrict__ psi,
                                                              cplx_t<R> *__restrict__ out, uint64_t N,
                                                              const DGroup *__restrict__ groups, int ngroups,
                                                              const DTerm *__restrict__ terms,
                                                              double *__restrict__ partials) {
    __shared__ double red[kRedThreads / 64];
    double lp = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kRedThreads;
    for (uint64_t k = (uint64_t)blockIdx.x * kRedThreads + threadIdx.x; k < N; k += stride) {
        double ar = 0.0, ai = 0.0;
        for (int g = 0; g < ngroups; ++g) {
            const DGroup G = groups[g];
            const uint64_t kx = k ^ G.x;
            const cplx_t<R> v = psi[kx];
            double cr = 0.0, ci = 0.0;  // sum over the group's terms of coef i^ny (-1)^{z.kx}
            for (int j = G.first; j < G.first + G.count; ++j) {
                const DTerm T = terms[j];
                const double s = odd_parity(T.z & kx) ? -T.coef : T.coef;
                cr += re_ipow(T.ny, s, 0.0);
                ci += im_ipow(T.ny, s, 0.0);
            }
            ar += cr * (double)v.x - ci * (double)v.y;
            ai += cr * (double)v.y + ci * (double)v.x;
        }
        cplx_t<R> o;
        o.x = (R)ar;
        o.y = (R)ai;
        out[k] = o;
        const cplx_t<R> p = psi[k];
        lp += (double)p.x * ar + (double)p.y * ai;
    }
    const double s = block_sum(lp, red);
    if (threadIdx.x == 0 && partials)
        partials[blockIdx.x] = s;
}

int launch_apply_paulis(int dtype, const void *psi, void *out, int n, const PauliDevice &d, hipStream_t st,
                        unsigned *grid) {
    const uint64_t N = 1ull << n;
    const unsigned g = reduce_grid(N);
    if (dtype == SV_C128)
        hipLaunchKernelGGL(k_apply_paulis<double>, dim3(g), dim3(kRedThreads), 0, st, (const double2 *)psi,
                           (double2 *)out, N, d.groups, d.ngroups, d.terms, d.partials);
    else
        hipLaunchKernelGGL(k_apply_paulis<float>, dim3(g), dim3(kRedThreads), 0, st, (const float2 *)psi,
                           (float2 *)out, N, d.groups, d.ngroups, d.terms, d.partials);
    SV_LAUNCH_CHECK();
    if (grid)
        *grid = g;
    return SV_OK;
}


// Partial count of every term (the grid of its group's pass), in the plan's
// term order.
static void expect_partial_counts(int n, const PauliPlan &plan, std::vector<int32_t> &nblk) {
    nblk.assign(plan.terms.size(), 0);
    for (const DGroup &g : plan.groups) {
        const uint64_t count = g.x == 0 ? (1ull << n) : (1ull << (n - 1));
        for (int j = g.first; j < g.first + g.count; ++j)
            nblk[j] = (int32_t)reduce_grid(count);
    }
}

// The group passes and the final sums.  terms (the plan's terms), nblk (their
// partial counts), partials (terms * kMaxPartials doubles) and sums (terms
// doubles) are device arrays, the first two already filled or enqueued on st.
static int expect_launch(const sv_state_t *s, const PauliPlan &plan, const DTerm *terms, const int32_t *nblk,
                         double *partials, double *sums, double *out_total, double *out_terms, hipStream_t st) {
    const int n = s->n;
    for (const DGroup &g : plan.groups) {
        const uint64_t count = g.x == 0 ? (1ull << n) : (1ull << (n - 1));
        const unsigned grid = reduce_grid(count);
        const uint32_t b = g.x ? (uint32_t)__builtin_ctzll(g.x) : 0;
        const char *base = static_cast<const char *>(s->data);
        const int8_t *scales = reinterpret_cast<const int8_t *>(base + (((size_t)1 << n) * amp_bytes(s->dtype)));
        switch (s->dtype) {
        case SV_C128:
            hipLaunchKernelGGL(k_expect_group<CplxAmps<double>>, dim3(grid), dim3(kRedThreads), 0, st,
                               CplxAmps<double>{(const double2 *)base}, count, g.x, b, terms, g.first, g.count,
                               partials);
            break;
        case SV_C64:
            hipLaunchKernelGGL(k_expect_group<CplxAmps<float>>, dim3(grid), dim3(kRedThreads), 0, st,
                               CplxAmps<float>{(const float2 *)base}, count, g.x, b, terms, g.first, g.count,
                               partials);
            break;
        case SV_CQ16:
            hipLaunchKernelGGL(k_expect_group<Q16Amps>, dim3(grid), dim3(kRedThreads), 0, st,
                               Q16Amps{(const uint32_t *)base, scales}, count, g.x, b, terms, g.first, g.count,
                               partials);
            break;
        default:
            hipLaunchKernelGGL(k_expect_group<Q32Amps>, dim3(grid), dim3(kRedThreads), 0, st,
                               Q32Amps{(const uint2 *)base, scales}, count, g.x, b, terms, g.first, g.count,
                               partials);
            break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return fail(SV_EHIP, "expectation launch failed: %s", hipGetErrorString(e));
    }
    const int nt = (int)plan.terms.size();
    hipLaunchKernelGGL(k_expect_sums, dim3(nt), dim3(kRedThreads), 0, st, nblk, partials, sums);
    hipLaunchKernelGGL(k_expect_final, dim3(1), dim3(64), 0, st, terms, nt, sums, out_total, out_terms);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(SV_EHIP, "expectation launch failed: %s", hipGetErrorString(e));
    return SV_OK;
}

static int expect_impl(const sv_state_t *s, const sv_pauli_t *terms, int nterms, double *out_total,
                       double *out_terms, hipStream_t st) {
    SV_TRY(validate_state(s, true));
    PauliPlan plan;
    SV_TRY(make_pauli_plan(s->n, terms, nterms, &plan));
    std::vector<int32_t> nblk;
    expect_partial_counts(s->n, plan, nblk);
    PauliDevice d;
    SV_TRY(pauli_upload(plan, (size_t)plan.terms.size() * (kMaxPartials + 1), st, &d));
    int32_t *d_nblk = nullptr;
    int r = SV_OK;
    hipError_t e = hipMallocAsync((void **)&d_nblk, nblk.size() * sizeof(int32_t), st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        d_nblk = nullptr;
        r = fail(SV_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    } else {
        e = hipMemcpyAsync(d_nblk, nblk.data(), nblk.size() * sizeof(int32_t), hipMemcpyHostToDevice, st);
        if (e != hipSuccess)
            r = fail(SV_EHIP, "copy failed: %s", hipGetErrorString(e));
    }
    if (r == SV_OK)
        r = expect_launch(s, plan, d.terms, d_nblk, d.partials, d.partials + plan.terms.size() * kMaxPartials,
                          out_total, out_terms, st);
    if (d_nblk)
        (void)hipFreeAsync(d_nblk, st);
    pauli_release(&d, st);
    return r;
}

// ---------------------------------------------------------------------------
// Allocation-free expectation.  The term table, the partial counts and the
// partial sums live in one file-scope device array.  Host code never passes
// the array's name to a kernel: its device address is looked up once per
// device with hipGetSymbolAddress and kept.  The tables travel to the device
// as a kernel argument (no host-to-device copy), and every partial a call
// reads is written by that call first, so nothing needs clearing.  Every
// call on one device shares the array: calls that overlap on one device
// race.
// ---------------------------------------------------------------------------
constexpr int kNoAllocTerms = SV_EXPECT_NOALLOC_MAX_TERMS;

struct ExpectScratch {
    DTerm terms[kNoAllocTerms];
    int32_t nblk[kNoAllocTerms];
    double partials[(size_t)kNoAllocTerms * kMaxPartials];
    double sums[kNoAllocTerms];
};

struct ExpectTables {
    int32_t nterms, pad;
    DTerm terms[kNoAllocTerms];
    int32_t nblk[kNoAllocTerms];
};

static __device__ __align__(256) unsigned char scratch[sizeof(ExpectScratch)];

__global__ __launch_bounds__(64) void k_expect_tables(ExpectTables t, ExpectScratch *w) {
    for (int i = threadIdx.x; i < t.nterms; i += blockDim.x) {
        w->terms[i] = t.terms[i];
        w->nblk[i] = t.nblk[i];
    }
}

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of the scratch array on the current device (looked up on
// the first call per device).
static int scratch_address(ExpectScratch **out) {
    int dev = 0;
    SV_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(SV_ENOTSUP, "device %d beyond the %d devices the scratch table holds", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SV_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<ExpectScratch *>(g_scratch_ptr[dev]);
    return SV_OK;
}

static int expect_noalloc_impl(const sv_state_t *s, const sv_pauli_t *terms, int nterms, double *out_total,
                               hipStream_t st) {
    SV_TRY(validate_state(s, true));
    if (nterms > kNoAllocTerms)
        return fail(SV_EINVAL, "nterms %d exceeds the allocation-free limit of %d terms", nterms, kNoAllocTerms);
    PauliPlan plan;
    SV_TRY(make_pauli_plan(s->n, terms, nterms, &plan));
    std::vector<int32_t> nblk;
    expect_partial_counts(s->n, plan, nblk);
    ExpectTables t;
    memset(&t, 0, sizeof(t));
    t.nterms = (int32_t)plan.terms.size();
    for (size_t j = 0; j < plan.terms.size(); ++j) {
        t.terms[j] = plan.terms[j];
        t.nblk[j] = nblk[j];
    }
    ExpectScratch *w = nullptr;
    SV_TRY(scratch_address(&w));
    hipLaunchKernelGGL(k_expect_tables, dim3(1), dim3(64), 0, st, t, w);
    SV_LAUNCH_CHECK();
    // member addresses inside the device array (w is never dereferenced on the host)
    char *base = reinterpret_cast<char *>(w);
    return expect_launch(s, plan, reinterpret_cast<const DTerm *>(base + offsetof(ExpectScratch, terms)),
                         reinterpret_cast<const int32_t *>(base + offsetof(ExpectScratch, nblk)),
                         reinterpret_cast<double *>(base + offsetof(ExpectScratch, partials)),
                         reinterpret_cast<double *>(base + offsetof(ExpectScratch, sums)), out_total, nullptr, st);
}

} // namespace sv

using namespace sv;

extern "C" {

int sv_expect(const sv_state_t *s, const sv_pauli_t *terms, int nterms, double *out_dev, sv_stream_t st) {
    clear_error();
    if (!out_dev)
        return fail(SV_EINVAL, "out_dev is NULL");
    return expect_impl(s, terms, nterms, out_dev, nullptr, (hipStream_t)st);
}

int sv_expect_noalloc(const sv_state_t *s, const sv_pauli_t *terms, int nterms, double *out_dev, sv_stream_t st) {
    clear_error();
    if (!out_dev)
        return fail(SV_EINVAL, "out_dev is NULL");
    return expect_noalloc_impl(s, terms, nterms, out_dev, (hipStream_t)st);
}

int sv_expect_terms(const sv_state_t *s, const sv_pauli_t *terms, int nterms, double *out_dev, sv_stream_t st) {
    clear_error();
    if (!out_dev)
        return fail(SV_EINVAL, "out_dev is NULL");
    return expect_impl(s, terms, nterms, nullptr, out_dev, (hipStream_t)st);
}

int sv_apply_pauli_sum(const sv_state_t *in, const sv_state_t *out, const sv_pauli_t *terms, int nterms,
                       sv_stream_t st) {
    clear_error();
    SV_TRY(validate_state(in));
    SV_TRY(validate_state(out));
    if (in->n != out->n || in->dtype != out->dtype)
        return fail(SV_EINVAL, "states differ in size or dtype");
    if (in->data == out->data)
        return fail(SV_EINVAL, "in and out must not alias");
    PauliPlan plan;
    SV_TRY(make_pauli_plan(in->n, terms, nterms, &plan));
    PauliDevice d;
    SV_TRY(pauli_upload(plan, 0, (hipStream_t)st, &d));
    const int r = launch_apply_paulis(in->dtype, in->data, out->data, in->n, d, (hipStream_t)st, nullptr);
    pauli_release(&d, (hipStream_t)st);
    return r;
}

} // extern "C"
