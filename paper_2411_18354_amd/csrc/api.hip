// State management, validation, error reporting and the index debug entry
// point of libsv.so.
#include <algorithm>
#include <cstdarg>
#include <cstring>
#include <mutex>

#include "sv_internal.hpp"

namespace sv {

static thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = '\0'; }

Expand make_expand(int n, const std::vector<int> &positions, const std::vector<int> &bits) {
    Expand e;
    memset(&e, 0, sizeof(e));
    uint64_t fixed = 0;
    int prev = -1;
    const int np = (int)positions.size();
    for (int j = 0; j <= np; ++j) {
        const int hi = (j < np) ? positions[j] : n; // exclusive upper output bit
        const int lo = prev + 1;                    // first output bit of segment j
        if (hi > lo) {
            uint64_t m = (hi >= 64 ? ~0ull : ((1ull << hi) - 1)) & ~((1ull << lo) - 1);
            e.shift[e.nseg] = (uint32_t)j;
            e.mask[e.nseg] = m;
            e.nseg++;
        }
        if (j < np) {
            if (bits[j])
                fixed |= 1ull << positions[j];
            prev = positions[j];
        }
    }
    e.fixed = fixed;
    return e;
}

int validate_state(const sv_state_t *s, bool allow_fixed) {
    if (!s)
        return fail(SV_EINVAL, "state is NULL");
    if (!known_dtype(s->dtype))
        return fail(SV_EINVAL, "unknown dtype %d", s->dtype);
    if (is_fixed(s->dtype) && !allow_fixed)
        return fail(SV_ENOTSUP, "this call does not take fixed-point (SV_CQ16, SV_CQ32) states");
    if (s->n < 1 || s->n > max_qubits(s->dtype))
        return fail(SV_EINVAL, "n=%d outside [1, %d]", s->n, max_qubits(s->dtype));
    if (!s->data)
        return fail(SV_EINVAL, "state data is NULL");
    const size_t align = is_fixed(s->dtype) ? 16 : amp_bytes(s->dtype);
    if (((uintptr_t)s->data) % align)
        return fail(SV_EINVAL, "state data %p not aligned to %zu bytes", s->data, align);
    return SV_OK;
}

int validate_gate(const GateSpec &g) {
    if (g.target < 0 || g.target >= g.n)
        return fail(SV_EINVAL, "target %d outside [0, %d)", g.target, g.n);
    const uint64_t full = (g.n >= 64) ? ~0ull : ((1ull << g.n) - 1);
    if (g.cmask & ~full)
        return fail(SV_EINVAL, "control mask 0x%llx has qubits >= n=%d", (unsigned long long)g.cmask, g.n);
    if (g.cmask & (1ull << g.target))
        return fail(SV_EINVAL, "qubit %d is both target and control", g.target);
    if (g.cvals & ~g.cmask)
        return fail(SV_EINVAL, "ctrl_vals 0x%llx has bits outside the control mask 0x%llx",
                    (unsigned long long)g.cvals, (unsigned long long)g.cmask);
    return SV_OK;
}

int controls_to_mask(int n, int target, const int32_t *controls, int nc, uint64_t *mask) {
    if (nc < 0)
        return fail(SV_EINVAL, "ncontrols %d < 0", nc);
    if (nc > 0 && !controls)
        return fail(SV_EINVAL, "controls is NULL with ncontrols=%d", nc);
    uint64_t m = 0;
    for (int i = 0; i < nc; ++i) {
        const int q = controls[i];
        if (q < 0 || q >= n)
            return fail(SV_EINVAL, "control %d outside [0, %d)", q, n);
        if (q == target)
            return fail(SV_EINVAL, "control %d equals the target", q);
        if (m & (1ull << q))
            return fail(SV_EINVAL, "duplicate control %d", q);
        m |= 1ull << q;
    }
    *mask = m;
    return SV_OK;
}

void gate_positions(const GateSpec &g, std::vector<int> &pos, std::vector<int> &bits) {
    pos.clear();
    bits.clear();
    const uint64_t all = g.cmask | (1ull << g.target);
    for (int q = 0; q < g.n; ++q) {
        if (all & (1ull << q)) {
            pos.push_back(q);
            bits.push_back(q == g.target ? 0 : (int)((g.cvals >> q) & 1));
        }
    }
}

int device_info(DeviceInfo *out) {
    static std::mutex mu;
    static std::vector<DeviceInfo> cache;
    int dev = 0;
    SV_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    for (auto &d : cache)
        if (d.device == dev) {
            *out = d;
            return SV_OK;
        }
    hipDeviceProp_t p;
    SV_HIP_TRY(hipGetDeviceProperties(&p, dev));
    DeviceInfo d;
    d.device = dev;
    d.num_cus = p.multiProcessorCount;
    d.max_lds = (int)p.sharedMemPerBlock;
    d.arch = p.gcnArchName;
    cache.push_back(d);
    *out = d;
    return SV_OK;
}

// ---------------------------------------------------------------- kernels

template <typename R>
__global__ __launch_bounds__(256) void k_basis(cplx_t<R> *__restrict__ psi, uint64_t N, uint64_t b) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += stride) {
        cplx_t<R> v;
        v.x = (k == b) ? (R)1 : (R)0;
        v.y = (R)0;
        psi[k] = v;
    }
}

// Plain copy, 16 bytes per lane per iteration (grid-stride).
__global__ __launch_bounds__(256) void k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, uint64_t n16) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

template <typename I>
__global__ __launch_bounds__(256) void k_debug_indices(uint64_t *__restrict__ out, uint64_t count, Expand e) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        out[i] = (uint64_t)expand_index<I>(e, (I)i);
}

} // namespace sv

using namespace sv;

extern "C" {

const char *sv_last_error(void) { return g_err; }

int sv_version(void) { return 10000; }

int sv_alloc(sv_state_t *s, int n, int dtype) {
    clear_error();
    if (!s)
        return fail(SV_EINVAL, "state is NULL");
    if (!known_dtype(dtype))
        return fail(SV_EINVAL, "unknown dtype %d", dtype);
    if (n < 1 || n > max_qubits(dtype))
        return fail(SV_EINVAL, "n=%d outside [1, %d]", n, max_qubits(dtype));
    void *p = nullptr;
    const size_t bytes = state_bytes(n, dtype);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SV_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    s->data = p;
    s->n = n;
    s->dtype = dtype;
    return SV_OK;
}

int sv_free(sv_state_t *s) {
    clear_error();
    if (!s)
        return fail(SV_EINVAL, "state is NULL");
    if (s->data)
        SV_HIP_TRY(hipFree(s->data));
    s->data = nullptr;
    return SV_OK;
}

int sv_init(const sv_state_t *s, uint64_t basis_index, sv_stream_t st) {
    clear_error();
    SV_TRY(validate_state(s, true));
    const uint64_t N = 1ull << s->n;
    if (basis_index >= N)
        return fail(SV_EINVAL, "basis index %llu >= 2^%d", (unsigned long long)basis_index, s->n);
    DeviceInfo di;
    SV_TRY(device_info(&di));
    const uint64_t want = (N + 255) / 256;
    const unsigned grid = (unsigned)std::min<uint64_t>(want, (uint64_t)di.num_cus * 16);
    if (is_fixed(s->dtype))
        return launch_fixed_basis(s->data, s->n, s->dtype, basis_index, grid, (hipStream_t)st);
    if (s->dtype == SV_C128)
        hipLaunchKernelGGL(k_basis<double>, dim3(grid), dim3(256), 0, (hipStream_t)st,
                           (double2 *)s->data, N, basis_index);
    else
        hipLaunchKernelGGL(k_basis<float>, dim3(grid), dim3(256), 0, (hipStream_t)st,
                           (float2 *)s->data, N, basis_index);
    SV_LAUNCH_CHECK();
    return SV_OK;
}

int sv_copy_state(const sv_state_t *dst, const sv_state_t *src, sv_stream_t st) {
    clear_error();
    SV_TRY(validate_state(dst, true));
    SV_TRY(validate_state(src, true));
    if (dst->n != src->n || dst->dtype != src->dtype)
        return fail(SV_EINVAL, "copy between states of different size or dtype");
    if (dst->data == src->data)
        return SV_OK;
    const size_t bytes = state_bytes(src->n, src->dtype);
    const char *a = (const char *)src->data, *b = (const char *)dst->data;
    if (a < b + bytes && b < a + bytes)
        return fail(SV_EINVAL, "source and destination overlap");
    DeviceInfo di;
    SV_TRY(device_info(&di));
    const uint64_t n16 = bytes / 16;
    if (n16 > 0 && bytes % 16 == 0) {
        const unsigned grid = (unsigned)std::min<uint64_t>((n16 + 255) / 256, (uint64_t)di.num_cus * 8);
        hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, (hipStream_t)st, (const uint4 *)src->data,
                           (uint4 *)dst->data, n16);
        SV_LAUNCH_CHECK();
    } else {  // sizes that are not whole 16-byte chunks (small or fixed-point states)
        SV_HIP_TRY(hipMemcpyAsync(dst->data, src->data, bytes, hipMemcpyDeviceToDevice, (hipStream_t)st));
    }
    return SV_OK;
}

int sv_debug_pair_indices(int n, int target, const int32_t *controls, int ncontrols,
                          uint64_t ctrl_vals, uint64_t *out_dev, int64_t out_len, sv_stream_t st) {
    clear_error();
    if (n < 1 || n > SV_MAX_QUBITS_C128)
        return fail(SV_EINVAL, "n=%d outside [1, %d]", n, SV_MAX_QUBITS_C128);
    GateSpec g{n, target, 0, ctrl_vals};
    if (target < 0 || target >= n)
        return fail(SV_EINVAL, "target %d outside [0, %d)", target, n);
    SV_TRY(controls_to_mask(n, target, controls, ncontrols, &g.cmask));
    SV_TRY(validate_gate(g));
    if (!out_dev)
        return fail(SV_EINVAL, "out_dev is NULL");
    const uint64_t count = 1ull << (n - 1 - popcount64(g.cmask));
    if (out_len < 0 || (uint64_t)out_len < count)
        return fail(SV_EINVAL, "out_len %lld < %llu", (long long)out_len, (unsigned long long)count);
    std::vector<int> pos, bits;
    gate_positions(g, pos, bits);
    const Expand e = make_expand(n, pos, bits);
    const uint64_t blocks = std::min<uint64_t>((count + 255) / 256, kMaxGridBlocks);
    if (n <= 32)
        hipLaunchKernelGGL(k_debug_indices<uint32_t>, dim3((unsigned)blocks), dim3(256), 0,
                           (hipStream_t)st, out_dev, count, e);
    else
        hipLaunchKernelGGL(k_debug_indices<uint64_t>, dim3((unsigned)blocks), dim3(256), 0,
                           (hipStream_t)st, out_dev, count, e);
    SV_LAUNCH_CHECK();
    return SV_OK;
}

} // extern "C"
