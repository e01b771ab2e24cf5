// Block-scaled 16-bit fixed-point states (SV_CQ16): gate, basis-state and
// conversion kernels.
//
// The paper lists fixed-point state precision as future work (Sec. V); the
// format is defined in sv.h: 2^n amplitudes as two int16 codes (re, im),
// then one int8 scale per 64-amplitude block, value = code * 2^scale.  At 4
// bytes per amplitude a pass moves half the bytes of complex64.
//
// A gate works on whole blocks.  A block is decoded to float (exact), the
// pair update of Sec. III runs in float with the fused multiply-add order
// every other kernel uses (cmac2), and the block is re-encoded under the
// scale of its new largest component.  So the block is what the schedule
// enumerates: controls on qubits >= 6 are inserted into the block index
// (the skip-interval map of Sec. III-B, one level up), controls on the 6
// in-block qubits are tested per amplitude.
//
// Mapping: a 16-lane group holds one block, 4 amplitudes (16 bytes) per
// lane, so each group load is 256 contiguous bytes.  A target >= 6 couples
// block b with block b + 2^(t-6), which the group holds in a second set of
// registers; a target below 6 couples amplitudes inside a lane (t < 2) or
// lane j with lane j ^ 2^(t-2) of the group.  The block maximum is a
// reduction over the group's 16 lanes.  States with n < 6 are one block of
// 2^n amplitudes, handled by one wavefront with one amplitude per lane.
#include <algorithm>
#include <cstring>

#include "gate_math.hpp"

namespace sv {

constexpr int kQScaleMin = -126, kQScaleMax = 112;
constexpr int kQThreads = 256;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u32x4 ld_nt4(const u32x4 *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_nt4(u32x4 *p, u32x4 v) { __builtin_nontemporal_store(v, p); }

__device__ __forceinline__ float q_dec(int code, int s) { return ldexpf((float)code, s); }

// Scale of a block whose largest |component| is m >= 0.  With m = f 2^e,
// f in [0.5, 1), the scale is e - 15; e = biased exponent - 126, so the
// scale is the biased exponent - 141 (zero and subnormal m clamp to -126).
__device__ __forceinline__ int q_scale(float m) {
    const int e = (int)(__float_as_uint(m) >> 23) - 141;
    return min(max(e, kQScaleMin), kQScaleMax);
}

// Code of v under scale s: round to nearest even, saturate to +-32767.
__device__ __forceinline__ uint32_t q_code(float v, int s) {
    const float r = fminf(fmaxf(rintf(ldexpf(v, -s)), -32767.0f), 32767.0f);
    return (uint32_t)(uint16_t)(int16_t)(int)r;
}

__device__ __forceinline__ uint32_t q_word(float re, float im, int s) { return q_code(re, s) | (q_code(im, s) << 16); }

__device__ __forceinline__ void q_unword(uint32_t w, int s, float &re, float &im) {
    re = q_dec((int)(int16_t)(w & 0xffffu), s);
    im = q_dec((int)(int16_t)(w >> 16), s);
}

__device__ __forceinline__ void q4_decode(u32x4 w, int s, float (&re)[4], float (&im)[4]) {
    q_unword(w.x, s, re[0], im[0]);
    q_unword(w.y, s, re[1], im[1]);
    q_unword(w.z, s, re[2], im[2]);
    q_unword(w.w, s, re[3], im[3]);
}

__device__ __forceinline__ u32x4 q4_encode(const float (&re)[4], const float (&im)[4], int s) {
    u32x4 w;
    w.x = q_word(re[0], im[0], s);
    w.y = q_word(re[1], im[1], s);
    w.z = q_word(re[2], im[2], s);
    w.w = q_word(re[3], im[3], s);
    return w;
}

__device__ __forceinline__ float q4_absmax(const float (&re)[4], const float (&im)[4]) {
    float m = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        m = fmaxf(m, fmaxf(fabsf(re[i]), fabsf(im[i])));
    return m;
}

// Maximum over the 16 lanes of a group (lanes 16g .. 16g+15 of the wave).
__device__ __forceinline__ float group16_max(float v) {
    v = fmaxf(v, lane_xor(v, 1));
    v = fmaxf(v, lane_xor(v, 2));
    v = fmaxf(v, lane_xor(v, 4));
    v = fmaxf(v, lane_xor(v, 8));
    return v;
}

// Pair update of (x, y) = (C_k, C_{k+2^t}) in float.
__device__ __forceinline__ void q_pair(const Mat2<float> &M, float &xr, float &xi, float &yr, float &yi) {
    float2 x = make_float2(xr, xi), y = make_float2(yr, yi);
    apply_pair<float>(M, x, y);
    xr = x.x;
    xi = x.y;
    yr = y.x;
    yi = y.y;
}

// One row of the pair update for a lane that holds one element of the pair
// and receives the other (pr, pi) from its partner: the lane with the target
// bit clear computes a C_k + b C_{k+2^t}, the other c C_k + d C_{k+2^t}.
__device__ __forceinline__ void q_row(const Mat2<float> &M, bool hi, float &xr, float &xi, float pr, float pi) {
    const float ur = hi ? M.cr : M.ar, ui = hi ? M.ci : M.ai;
    const float vr = hi ? M.dr : M.br, vi = hi ? M.di : M.bi;
    const float2 p1 = hi ? make_float2(pr, pi) : make_float2(xr, xi);
    const float2 p2 = hi ? make_float2(xr, xi) : make_float2(pr, pi);
    const float2 o = cmac2<float>(ur, ui, p1, vr, vi, p2);
    xr = o.x;
    xi = o.y;
}

template <bool Masked, bool High, typename MS>
__global__ __launch_bounds__(kQThreads) void k_q16_gate(u32x4 *__restrict__ codes, int8_t *__restrict__ scales,
                                                        Q16Plan p, MS ms) {
    const int j = threadIdx.x & 15;
    const uint64_t gstride = ((uint64_t)gridDim.x * kQThreads) >> 4;
    const Mat2<float> M = ms.get();
    for (uint64_t u = ((uint64_t)blockIdx.x * kQThreads + threadIdx.x) >> 4; u < p.units; u += gstride) {
        uint64_t b;
        if (Masked) {
            b = High ? (((u >> p.target) << (p.target + 1)) | (u & ((1ull << p.target) - 1))) : u;
            if ((b & p.hmask) != p.hvals)
                continue;  // the whole group skips: lanes of a group share u
        } else {
            b = expand_index<uint64_t>(p.e, u);
        }
        u32x4 *ca = codes + b * 16 + j;
        if (High) {
            const uint64_t b2 = b | (1ull << p.target);
            u32x4 *cb = codes + b2 * 16 + j;
            const u32x4 wa = ld_nt4(ca), wb = ld_nt4(cb);
            const int sa = scales[b], sb = scales[b2];
            float xr[4], xi[4], yr[4], yi[4];
            q4_decode(wa, sa, xr, xi);
            q4_decode(wb, sb, yr, yi);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if ((((uint32_t)(4 * j + i)) & p.lmask) == p.lvals)
                    q_pair(M, xr[i], xi[i], yr[i], yi[i]);
            const int na = q_scale(group16_max(q4_absmax(xr, xi)));
            const int nb = q_scale(group16_max(q4_absmax(yr, yi)));
            st_nt4(ca, q4_encode(xr, xi, na));
            st_nt4(cb, q4_encode(yr, yi, nb));
            if (j == 0) {
                scales[b] = (int8_t)na;
                scales[b2] = (int8_t)nb;
            }
        } else {
            const u32x4 w = ld_nt4(ca);
            const int s = scales[b];
            float xr[4], xi[4];
            q4_decode(w, s, xr, xi);
            const int t = p.target;
            const uint32_t a0 = 4u * (uint32_t)j;
            if (t == 0) {
                if (((a0 + 0) & p.lmask) == p.lvals)
                    q_pair(M, xr[0], xi[0], xr[1], xi[1]);
                if (((a0 + 2) & p.lmask) == p.lvals)
                    q_pair(M, xr[2], xi[2], xr[3], xi[3]);
            } else if (t == 1) {
                if (((a0 + 0) & p.lmask) == p.lvals)
                    q_pair(M, xr[0], xi[0], xr[2], xi[2]);
                if (((a0 + 1) & p.lmask) == p.lvals)
                    q_pair(M, xr[1], xi[1], xr[3], xi[3]);
            } else {
                const int lm = 1 << (t - 2);
                const bool hi = (j & lm) != 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float pr = lane_xor(xr[i], lm), pi = lane_xor(xi[i], lm);
                    if (((a0 + i) & p.lmask) == p.lvals)
                        q_row(M, hi, xr[i], xi[i], pr, pi);
                }
            }
            const int ns = q_scale(group16_max(q4_absmax(xr, xi)));
            st_nt4(ca, q4_encode(xr, xi, ns));
            if (j == 0)
                scales[b] = (int8_t)ns;
        }
    }
}

// n < 6: the state is one block of 2^n amplitudes; lane l holds amplitude l.
template <typename MS>
__global__ __launch_bounds__(64) void k_q16_gate_small(uint32_t *__restrict__ codes, int8_t *__restrict__ scales,
                                                       Q16Plan p, MS ms) {
    const int l = threadIdx.x;
    const bool valid = l < (1 << p.n);
    const Mat2<float> M = ms.get();
    const int s = scales[0];
    float xr = 0.0f, xi = 0.0f;
    if (valid)
        q_unword(codes[l], s, xr, xi);
    const int tm = 1 << p.target;
    const float pr = lane_xor(xr, tm), pi = lane_xor(xi, tm);
    if (valid && (((uint32_t)l & p.lmask) == p.lvals))
        q_row(M, (l & tm) != 0, xr, xi, pr, pi);
    float m = fmaxf(fabsf(xr), fabsf(xi));  // 0 on lanes past the state
    for (int k = 1; k < 64; k <<= 1)
        m = fmaxf(m, lane_xor(m, k));
    const int ns = q_scale(m);
    if (valid)
        codes[l] = q_word(xr, xi, ns);
    if (l == 0)
        scales[0] = (int8_t)ns;
}

// ---------------------------------------------------------------- conversions

template <typename R>
__global__ __launch_bounds__(kQThreads) void k_q16_encode(const cplx_t<R> *__restrict__ src, u32x4 *__restrict__ codes,
                                                          int8_t *__restrict__ scales, uint64_t nblocks) {
    const int j = threadIdx.x & 15;
    const uint64_t gstride = ((uint64_t)gridDim.x * kQThreads) >> 4;
    for (uint64_t b = ((uint64_t)blockIdx.x * kQThreads + threadIdx.x) >> 4; b < nblocks; b += gstride) {
        const cplx_t<R> *v = src + b * 64 + 4 * j;
        float re[4], im[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const cplx_t<R> a = v[i];
            re[i] = (float)a.x;  // round to nearest
            im[i] = (float)a.y;
        }
        const int ns = q_scale(group16_max(q4_absmax(re, im)));
        codes[b * 16 + j] = q4_encode(re, im, ns);
        if (j == 0)
            scales[b] = (int8_t)ns;
    }
}

template <typename R>
__global__ __launch_bounds__(64) void k_q16_encode_small(const cplx_t<R> *__restrict__ src, uint32_t *__restrict__ codes,
                                                         int8_t *__restrict__ scales, int n) {
    const int l = threadIdx.x;
    const bool valid = l < (1 << n);
    float re = 0.0f, im = 0.0f;
    if (valid) {
        const cplx_t<R> a = src[l];
        re = (float)a.x;
        im = (float)a.y;
    }
    float m = fmaxf(fabsf(re), fabsf(im));
    for (int k = 1; k < 64; k <<= 1)
        m = fmaxf(m, lane_xor(m, k));
    const int ns = q_scale(m);
    if (valid)
        codes[l] = q_word(re, im, ns);
    if (l == 0)
        scales[0] = (int8_t)ns;
}

template <typename R>
__global__ __launch_bounds__(256) void k_q16_decode(const uint32_t *__restrict__ codes, const int8_t *__restrict__ scales,
                                                    cplx_t<R> *__restrict__ dst, uint64_t N) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += stride) {
        float re, im;
        q_unword(codes[k], scales[k >> kQBlockBits], re, im);
        cplx_t<R> o;
        o.x = (R)re;
        o.y = (R)im;
        dst[k] = o;
    }
}

template <typename RS, typename RD>
__global__ __launch_bounds__(256) void k_convert(const cplx_t<RS> *__restrict__ src, cplx_t<RD> *__restrict__ dst,
                                                 uint64_t N) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += stride) {
        const cplx_t<RS> a = src[k];
        cplx_t<RD> o;
        o.x = (RD)a.x;
        o.y = (RD)a.y;
        dst[k] = o;
    }
}

// |b>: code (16384, 0) under scale -14 (1.0 exactly) at amplitude b, every
// other amplitude 0 and every other block at the zero-block scale.
__global__ __launch_bounds__(256) void k_q16_basis(uint32_t *__restrict__ codes, int8_t *__restrict__ scales,
                                                   uint64_t N, uint64_t nblocks, uint64_t b) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t k = i0; k < N; k += stride)
        codes[k] = (k == b) ? 16384u : 0u;
    for (uint64_t k = i0; k < nblocks; k += stride)
        scales[k] = (int8_t)((k == (b >> kQBlockBits)) ? -14 : kQScaleMin);
}

// ---------------------------------------------------------------- host side

static int8_t *q16_scales(void *state, int n) { return (int8_t *)((char *)state + ((size_t)4 << n)); }

int make_q16_plan(const GateSpec &g, bool masked, Q16Plan *out) {
    Q16Plan q;
    memset(&q, 0, sizeof(q));
    q.n = g.n;
    q.masked = masked;
    if (g.n < kQBlockBits) {
        q.small = true;
        q.target = g.target;
        q.lmask = (uint32_t)g.cmask;
        q.lvals = (uint32_t)g.cvals;
        q.units = 1;
        *out = q;
        return SV_OK;
    }
    const int nb = g.n - kQBlockBits;
    const uint64_t low = (1ull << kQBlockBits) - 1;
    q.lmask = (uint32_t)(g.cmask & low);
    q.lvals = (uint32_t)(g.cvals & low);
    q.hmask = g.cmask >> kQBlockBits;
    q.hvals = g.cvals >> kQBlockBits;
    q.high = g.target >= kQBlockBits;
    q.target = q.high ? g.target - kQBlockBits : g.target;
    const int free_bits = nb - (q.high ? 1 : 0);
    if (masked) {
        q.units = 1ull << free_bits;
    } else {
        std::vector<int> pos, bits;
        for (int b = 0; b < nb; ++b) {
            if (q.high && b == q.target) {
                pos.push_back(b);
                bits.push_back(0);
            } else if ((q.hmask >> b) & 1ull) {
                pos.push_back(b);
                bits.push_back((int)((q.hvals >> b) & 1ull));
            }
        }
        q.e = make_expand(nb, pos, bits);
        q.units = 1ull << (free_bits - popcount64(q.hmask));
    }
    *out = q;
    return SV_OK;
}

std::string q16_plan_name(const Q16Plan &p, const char *matsrc) {
    char buf[256];
    if (p.small)
        snprintf(buf, sizeof(buf), "sv::k_q16_gate_small<sv::%s<float> >", matsrc);
    else
        snprintf(buf, sizeof(buf), "sv::k_q16_gate<%s, %s, sv::%s<float> >", p.masked ? "true" : "false",
                 p.high ? "true" : "false", matsrc);
    return buf;
}

static unsigned q16_grid(uint64_t groups) {
    DeviceInfo di;
    if (device_info(&di) != SV_OK)
        di.num_cus = 256;
    const uint64_t want = (groups + (kQThreads / 16) - 1) / (kQThreads / 16);
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)di.num_cus * 32));
}

template <typename MS> static int launch_q16(void *state, const Q16Plan &p, const MS &ms, hipStream_t st) {
    int8_t *sc = q16_scales(state, p.n);
    if (p.small) {
        hipLaunchKernelGGL((k_q16_gate_small<MS>), dim3(1), dim3(64), 0, st, (uint32_t *)state, sc, p, ms);
        SV_LAUNCH_CHECK();
        return SV_OK;
    }
    u32x4 *codes = (u32x4 *)state;
    const dim3 grid(q16_grid(p.units)), block(kQThreads);
    if (p.masked && p.high)
        hipLaunchKernelGGL((k_q16_gate<true, true, MS>), grid, block, 0, st, codes, sc, p, ms);
    else if (p.masked)
        hipLaunchKernelGGL((k_q16_gate<true, false, MS>), grid, block, 0, st, codes, sc, p, ms);
    else if (p.high)
        hipLaunchKernelGGL((k_q16_gate<false, true, MS>), grid, block, 0, st, codes, sc, p, ms);
    else
        hipLaunchKernelGGL((k_q16_gate<false, false, MS>), grid, block, 0, st, codes, sc, p, ms);
    SV_LAUNCH_CHECK();
    return SV_OK;
}

int launch_q16_gate(void *state, const Q16Plan &p, const double *U, const double *Ud, hipStream_t st) {
    if (Ud)
        return launch_q16(state, p, MatPtr<float>{Ud}, st);
    return launch_q16(state, p, MatVal<float>{to_mat<float>(U)}, st);
}

int launch_q16_basis(void *state, int n, uint64_t basis, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL(k_q16_basis, dim3(grid), dim3(256), 0, st, (uint32_t *)state, q16_scales(state, n),
                       1ull << n, q16_blocks(n), basis);
    SV_LAUNCH_CHECK();
    return SV_OK;
}

template <typename R> static int encode_from(const sv_state_t *dst, const sv_state_t *src, hipStream_t st) {
    const int n = src->n;
    int8_t *sc = q16_scales(dst->data, n);
    if (n < kQBlockBits)
        hipLaunchKernelGGL(k_q16_encode_small<R>, dim3(1), dim3(64), 0, st, (const cplx_t<R> *)src->data,
                           (uint32_t *)dst->data, sc, n);
    else
        hipLaunchKernelGGL(k_q16_encode<R>, dim3(q16_grid(q16_blocks(n))), dim3(kQThreads), 0, st,
                           (const cplx_t<R> *)src->data, (u32x4 *)dst->data, sc, q16_blocks(n));
    SV_LAUNCH_CHECK();
    return SV_OK;
}

static unsigned flat_grid(uint64_t N) {
    DeviceInfo di;
    if (device_info(&di) != SV_OK)
        di.num_cus = 256;
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((N + 255) / 256, (uint64_t)di.num_cus * 16));
}

template <typename R> static int decode_to(const sv_state_t *dst, const sv_state_t *src, hipStream_t st) {
    const uint64_t N = 1ull << src->n;
    hipLaunchKernelGGL(k_q16_decode<R>, dim3(flat_grid(N)), dim3(256), 0, st, (const uint32_t *)src->data,
                       (const int8_t *)q16_scales(src->data, src->n), (cplx_t<R> *)dst->data, N);
    SV_LAUNCH_CHECK();
    return SV_OK;
}

} // namespace sv

using namespace sv;

extern "C" {

int sv_state_bytes(int n, int dtype, uint64_t *bytes) {
    clear_error();
    if (!bytes)
        return fail(SV_EINVAL, "bytes is NULL");
    if (dtype != SV_C128 && dtype != SV_C64 && dtype != SV_CQ16)
        return fail(SV_EINVAL, "unknown dtype %d", dtype);
    if (n < 1 || n > max_qubits(dtype))
        return fail(SV_EINVAL, "n=%d outside [1, %d]", n, max_qubits(dtype));
    *bytes = (uint64_t)state_bytes(n, dtype);
    return SV_OK;
}

int sv_convert(const sv_state_t *dst, const sv_state_t *src, sv_stream_t st) {
    clear_error();
    SV_TRY(validate_state(dst, true));
    SV_TRY(validate_state(src, true));
    if (dst->n != src->n)
        return fail(SV_EINVAL, "convert between states of %d and %d qubits", src->n, dst->n);
    if (dst->dtype == src->dtype)
        return sv_copy_state(dst, src, st);
    const char *a = (const char *)src->data, *b = (const char *)dst->data;
    if (a < b + state_bytes(dst->n, dst->dtype) && b < a + state_bytes(src->n, src->dtype))
        return fail(SV_EINVAL, "source and destination overlap");
    const hipStream_t s = (hipStream_t)st;
    const uint64_t N = 1ull << src->n;
    if (dst->dtype == SV_CQ16)
        return src->dtype == SV_C128 ? encode_from<double>(dst, src, s) : encode_from<float>(dst, src, s);
    if (src->dtype == SV_CQ16)
        return dst->dtype == SV_C128 ? decode_to<double>(dst, src, s) : decode_to<float>(dst, src, s);
    if (src->dtype == SV_C128)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(flat_grid(N)), dim3(256), 0, s,
                           (const double2 *)src->data, (float2 *)dst->data, N);
    else
        hipLaunchKernelGGL((k_convert<float, double>), dim3(flat_grid(N)), dim3(256), 0, s,
                           (const float2 *)src->data, (double2 *)dst->data, N);
    SV_LAUNCH_CHECK();
    return SV_OK;
}

} // extern "C"
