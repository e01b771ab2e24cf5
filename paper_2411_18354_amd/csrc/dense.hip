// Dense k-qubit block on the lowest k qubits, applied with matrix cores.
//
// A run of gates that act only on qubits 0 .. k-1 is one 2^k x 2^k unitary M
// (composed on the device, so angles may come from device memory).  Viewing
// the state as rows of 2^k consecutive amplitudes, the run is row <- M row
// for every row: a dense contraction.  With interleaved (re, im) storage a
// row is D = 2^(k+1) reals and M acts through its real embedding
//     Re: R[2a][2b] = Re M[a][b],  R[2a][2b+1] = -Im M[a][b]
//     Im: R[2a+1][2b] = Im M[a][b], R[2a+1][2b+1] = Re M[a][b],
// so OUT = X R^T with X the (rows x D) real matrix: a GEMM on
// v_mfma_f64_16x16x4f64 (complex128) or v_mfma_f32_16x16x4f32 (complex64).
//
// Each wavefront takes 16 rows at a time.  R^T, the B operand, stays in
// registers for the whole launch.  The 16 rows move between HBM and the
// wavefront's LDS slice with 16-byte nontemporal accesses (consecutive lanes
// on consecutive 16 bytes); the next 16 rows are already being loaded while
// the current ones are multiplied.  The contraction index is permuted so
// that lane (row r, quarter q) supplies X[r][q D/4 + s] at MFMA step s: each
// lane then reads D/4 consecutive reals of its row from LDS with 16-byte
// reads, and the B registers use the same permutation.
//
// Roofline: 2^(k+3) flop per amplitude against 2 S bytes moved, i.e.
// 4 flop/B at k=4 in complex128 (FP64 ridge about 78.6 TFLOP/s / 8 TB/s =
// 10 flop/B) and 16 flop/B at k=5 in complex64 (FP32 MFMA ridge about
// 157 TFLOP/s / 8 TB/s = 20 flop/B): both HBM-bound on MI355X.
#include <algorithm>
#include <cstring>

#include "circuit.hpp"
#include "gates.hpp"

namespace sv {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ d4v mfma16x16x4(double a, double b, d4v c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4v mfma16x16x4(float a, float b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename R> struct Acc;
template <> struct Acc<double> { using type = d4v; };
template <> struct Acc<float> { using type = f4v; };
// 16 bytes of reals
template <typename R> struct Vec16;
template <> struct Vec16<double> { using type = d2v; };
template <> struct Vec16<float> { using type = f4v; };

// Result element (lane l, register r) of a 16x16 MFMA tile, as measured on
// gfx950: f64 -> row 4r + l/16; f32 -> row 4(l/16) + r; column l % 16.
template <typename R> __device__ __forceinline__ int acc_row(int l, int r);
template <> __device__ __forceinline__ int acc_row<double>(int l, int r) { return 4 * r + (l >> 4); }
template <> __device__ __forceinline__ int acc_row<float>(int l, int r) { return 4 * (l >> 4) + r; }

// LDS accesses of one wavefront to its own slice: the wavefront's lanes run
// in lockstep and its LDS operations complete in order, so ordering needs only
// the compiler not to move memory operations across this point.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kDenseThreads = 256;

// x: the state as reals; nwg: groups of 16 rows (one per wavefront pass);
// rmat: the D x D real embedding, row-major.
template <typename R, int KQ>
__global__ __launch_bounds__(kDenseThreads) void k_dense(R *__restrict__ x, uint64_t nwg,
                                                         const R *__restrict__ rmat) {
    using V = typename Vec16<R>::type;
    constexpr int D = 2 << KQ;               // reals per row
    constexpr int NS = D / 4;                // MFMA k-steps
    constexpr int NT = D / 16;               // 16-wide output tiles
    constexpr int VR = 16 / sizeof(R);       // reals per 16-byte vector
    constexpr int P = D + VR;                // padded LDS row, 16-byte aligned
    constexpr int NV = 16 * D / VR / 64;     // 16-byte vectors per lane per group
    constexpr int NA = NS / VR;              // 16-byte A reads per lane per group
    static_assert(NS % VR == 0 && NV >= 1, "tile shape");
    __shared__ __align__(16) R xs[(kDenseThreads / 64) * 16 * P];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int r16 = l & 15, q = l >> 4;
    R *xw = xs + w * 16 * P;
    // B operand at step s, tile jt: R^T[kk][j] = R[j][kk], kk = q NS + s, j = 16 jt + r16
    R b[NT][NS];
#pragma unroll
    for (int jt = 0; jt < NT; ++jt)
#pragma unroll
        for (int s = 0; s < NS; ++s)
            b[jt][s] = rmat[(jt * 16 + r16) * D + q * NS + s];
    const uint64_t stride = (uint64_t)gridDim.x * (kDenseThreads / 64);
    uint64_t g = (uint64_t)blockIdx.x * (kDenseThreads / 64) + w;
    V t[NV];
    if (g < nwg) {
        const V *src = reinterpret_cast<const V *>(x + g * 16 * D);
#pragma unroll
        for (int v = 0; v < NV; ++v)
            t[v] = __builtin_nontemporal_load(src + l + 64 * v);
    }
    while (g < nwg) {  // uniform per wavefront
        // vector e = l + 64 v holds reals [VR e, VR e + VR): row VR e / D, column VR e % D
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int e = l + 64 * v;
            *reinterpret_cast<V *>(xw + (e * VR / D) * P + (e * VR) % D) = t[v];
        }
        const uint64_t gn = g + stride;
        if (gn < nwg) {  // the next group's loads are in flight during the products
            const V *src = reinterpret_cast<const V *>(x + gn * 16 * D);
#pragma unroll
            for (int v = 0; v < NV; ++v)
                t[v] = __builtin_nontemporal_load(src + l + 64 * v);
        }
        wave_lds_sync();
        R a[NS];
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const V u = *reinterpret_cast<const V *>(xw + r16 * P + q * NS + i * VR);
#pragma unroll
            for (int c = 0; c < VR; ++c)
                a[i * VR + c] = u[c];
        }
        typename Acc<R>::type acc[NT];
#pragma unroll
        for (int jt = 0; jt < NT; ++jt)
            acc[jt] = typename Acc<R>::type{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int jt = 0; jt < NT; ++jt)
                acc[jt] = mfma16x16x4(a[s], b[jt][s], acc[jt]);
        wave_lds_sync();
#pragma unroll
        for (int jt = 0; jt < NT; ++jt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                xw[acc_row<R>(l, r) * P + jt * 16 + r16] = acc[jt][r];
        wave_lds_sync();
        V *dst = reinterpret_cast<V *>(x + g * 16 * D);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int e = l + 64 * v;
            __builtin_nontemporal_store(*reinterpret_cast<const V *>(xw + (e * VR / D) * P + (e * VR) % D),
                                        dst + l + 64 * v);
        }
        wave_lds_sync();
        g = gn;
    }
}

// One dense run's composition: column c of M is the run applied to |c>.

// Compose M (k qubits) from gates[0 .. count) using matrices mats + 8 * mat,
// then write the real embedding (D x D, in precision R) to rmat.
template <typename R>
__global__ void k_dense_compose(const DenseGate *__restrict__ gates, int count, const double *__restrict__ mats,
                                int kq, R *__restrict__ rmat) {
    __shared__ double mr[32 * 32], mi[32 * 32];  // column-major: M[a][c] at a + c*dim
    const int dim = 1 << kq;
    for (int e = threadIdx.x; e < dim * dim; e += blockDim.x) {
        mr[e] = (e % dim) == (e / dim) ? 1.0 : 0.0;
        mi[e] = 0.0;
    }
    __syncthreads();
    const int c = threadIdx.x;  // one column per lane
    if (c < dim) {
        for (int i = 0; i < count; ++i) {
            const DenseGate g = gates[i];
            const double *u = mats + 8 * g.mat;
            const int st = 1 << g.target;
            for (int a = 0; a < dim; ++a) {
                if ((a & st) || ((uint64_t)a & g.cmask) != g.cvals)
                    continue;
                const int b = a | st;
                const double xr = mr[a + c * dim], xi = mi[a + c * dim];
                const double yr = mr[b + c * dim], yi = mi[b + c * dim];
                mr[a + c * dim] = u[0] * xr - u[1] * xi + u[2] * yr - u[3] * yi;
                mi[a + c * dim] = u[0] * xi + u[1] * xr + u[2] * yi + u[3] * yr;
                mr[b + c * dim] = u[4] * xr - u[5] * xi + u[6] * yr - u[7] * yi;
                mi[b + c * dim] = u[4] * xi + u[5] * xr + u[6] * yi + u[7] * yr;
            }
        }
    }
    __syncthreads();
    const int D = 2 * dim;
    for (int e = threadIdx.x; e < dim * dim; e += blockDim.x) {
        const int a = e % dim, b = e / dim;  // M[a][b]
        const double re = mr[a + b * dim], im = mi[a + b * dim];
        rmat[(2 * a) * D + 2 * b] = (R)re;
        rmat[(2 * a) * D + 2 * b + 1] = (R)-im;
        rmat[(2 * a + 1) * D + 2 * b] = (R)im;
        rmat[(2 * a + 1) * D + 2 * b + 1] = (R)re;
    }
}

bool dense_supported(int dtype, int kq, int n) {
    if (n < kq + 6)
        return false;  // whole groups of 64 rows
    return dtype == SV_C128 ? kq == 4 : (kq == 4 || kq == 5);
}

// Workgroups of the persistent dense launch: as many as are resident at
// once (the kernel's occupancy times the CUs), never more than the 16-row
// groups need (4 per workgroup).  Every workgroup strides over the same
// share, so workgroups beyond the resident ones would run as a second round
// and stretch the launch (k = 4 complex128 holds 5 workgroups per CU: 8 per
// CU took 1.84 ms at n = 28 instead of 1.65).  The row groups all cost the
// same, so a static share loses nothing to imbalance.
static unsigned dense_grid(const void *kernel, uint64_t nwg) {
    DeviceInfo di;
    const uint64_t cus = device_info(&di) == SV_OK ? (uint64_t)di.num_cus : 256;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kDenseThreads, 0) != hipSuccess ||
        per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 4;
    }
    const uint64_t need = (nwg + kDenseThreads / 64 - 1) / (kDenseThreads / 64);
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(need, cus * (uint64_t)per_cu));
}

int launch_dense(int dtype, void *psi, int n, int kq, const void *rmat, hipStream_t st) {
    if (!dense_supported(dtype, kq, n))
        return fail(SV_ENOTSUP, "dense block of %d qubits unsupported for dtype %d, n=%d", kq, dtype, n);
    const uint64_t ngroups = 1ull << (n - kq - 4);  // groups of 16 rows of 2^kq amplitudes
    if (dtype == SV_C128)
        hipLaunchKernelGGL((k_dense<double, 4>), dim3(dense_grid((const void *)k_dense<double, 4>, ngroups)),
                           dim3(kDenseThreads), 0, st, (double *)psi, ngroups, (const double *)rmat);
    else if (kq == 4)
        hipLaunchKernelGGL((k_dense<float, 4>), dim3(dense_grid((const void *)k_dense<float, 4>, ngroups)),
                           dim3(kDenseThreads), 0, st, (float *)psi, ngroups, (const float *)rmat);
    else
        hipLaunchKernelGGL((k_dense<float, 5>), dim3(dense_grid((const void *)k_dense<float, 5>, ngroups)),
                           dim3(kDenseThreads), 0, st, (float *)psi, ngroups, (const float *)rmat);
    SV_LAUNCH_CHECK();
    return SV_OK;
}

int launch_dense_compose(int dtype, const void *gates, int count, const double *mats, int kq, void *rmat,
                         hipStream_t st) {
    if (dtype == SV_C128)
        hipLaunchKernelGGL(k_dense_compose<double>, dim3(1), dim3(64), 0, st, (const DenseGate *)gates, count, mats,
                           kq, (double *)rmat);
    else
        hipLaunchKernelGGL(k_dense_compose<float>, dim3(1), dim3(64), 0, st, (const DenseGate *)gates, count, mats,
                           kq, (float *)rmat);
    SV_LAUNCH_CHECK();
    return SV_OK;
}

} // namespace sv

using namespace sv;

extern "C" {

int sv_apply_dense_low(const sv_state_t *s, int k, const double *M, sv_stream_t st) {
    clear_error();
    SV_TRY(validate_state(s));
    if (!M)
        return fail(SV_EINVAL, "M is NULL");
    if (!dense_supported(s->dtype, k, s->n))
        return fail(SV_ENOTSUP, "dense block of %d qubits unsupported for dtype %d, n=%d (complex128: k=4; "
                                "complex64: k=4 or 5; n >= k+6)",
                    k, s->dtype, s->n);
    const int dim = 1 << k, D = 2 * dim;
    const size_t rb = (size_t)D * D * (s->dtype == SV_C128 ? 8 : 4);
    std::vector<unsigned char> host(rb);
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) {
            const double re = M[2 * (a * dim + b)], im = M[2 * (a * dim + b) + 1];
            const double v[4] = {re, -im, im, re};
            const int idx[4] = {(2 * a) * D + 2 * b, (2 * a) * D + 2 * b + 1, (2 * a + 1) * D + 2 * b,
                                (2 * a + 1) * D + 2 * b + 1};
            for (int q = 0; q < 4; ++q) {
                if (s->dtype == SV_C128)
                    reinterpret_cast<double *>(host.data())[idx[q]] = v[q];
                else
                    reinterpret_cast<float *>(host.data())[idx[q]] = (float)v[q];
            }
        }
    void *d = nullptr;
    hipError_t e = hipMallocAsync(&d, rb, (hipStream_t)st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SV_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    int r = SV_OK;
    e = hipMemcpyAsync(d, host.data(), rb, hipMemcpyHostToDevice, (hipStream_t)st);
    if (e != hipSuccess)
        r = fail(SV_EHIP, "copy failed: %s", hipGetErrorString(e));
    if (r == SV_OK)
        r = launch_dense(s->dtype, s->data, s->n, k, d, (hipStream_t)st);
    (void)hipFreeAsync(d, (hipStream_t)st);
    return r;
}

} // extern "C"
