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

// Code of v under scale s, given inv = 2^-s: v * 2^-s rounded to nearest,
// ties to even, saturated to +-32767.  |v * 2^-s| < 2^15, so adding
// C = 1.5 * 2^23 in one fused multiply-add (the product is exact) lands in
// [2^23, 2^24), where floats are the integers: that single rounding is the
// round-to-nearest-even of v * 2^-s (C is even, so ties keep their parity).
// Clamped to C +- 32767, the float's bits are 0x4B400000 + code, whose low
// 16 bits are the code in two's complement.
__device__ __forceinline__ uint32_t q_biased(float v, float inv) {
    const float y = __builtin_fmaf(v, inv, 12582912.0f);
    return __float_as_uint(__builtin_amdgcn_fmed3f(y, 12582912.0f - 32767.0f, 12582912.0f + 32767.0f));
}

__device__ __forceinline__ float q_inv(int s) { return ldexpf(1.0f, -s); }

__device__ __forceinline__ uint32_t q_word(float re, float im, float inv) {
    // low half: the re code, high half: the im code
    return __builtin_amdgcn_perm(q_biased(im, inv), q_biased(re, inv), 0x05040100u);
}

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
    const float inv = q_inv(s);
    u32x4 w;
    w.x = q_word(re[0], im[0], inv);
    w.y = q_word(re[1], im[1], inv);
    w.z = q_word(re[2], im[2], inv);
    w.w = q_word(re[3], im[3], inv);
    return w;
}

__device__ __forceinline__ float q4_absmax(const float (&re)[4], const float (&im)[4]) {
    const float a = fmaxf(fmaxf(fabsf(re[0]), fabsf(im[0])), fabsf(re[1]));
    const float b = fmaxf(fmaxf(fabsf(im[1]), fabsf(re[2])), fabsf(im[2]));
    return fmaxf(fmaxf(a, b), fmaxf(fabsf(re[3]), fabsf(im[3])));
}

template <int Ctrl> __device__ __forceinline__ float dpp_max(float v) {
    return fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), Ctrl, 0xf, 0xf, false)));
}

// Maximum over the 16 lanes of a group, which is one DPP row (lanes
// 16g .. 16g+15): swap neighbours and pairs inside each quad, then mirror
// each half row and the whole row.  All 16 lanes of a row are active
// together (a group shares its work unit).
__device__ __forceinline__ float group16_max(float v) {
    v = dpp_max<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v = dpp_max<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v = dpp_max<0x141>(v);  // row_half_mirror
    v = dpp_max<0x140>(v);  // row_mirror
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

// Block index of unit u, or -1 when a masked launch skips it.  Block
// indices have at most 30 bits.
template <bool Masked, bool High> __device__ __forceinline__ int q_unit_block(const Q16Plan &p, uint64_t u) {
    if (u >= p.units)
        return -1;
    const uint32_t v = (uint32_t)u;
    if (!Masked)
        return (int)expand_index<uint32_t>(p.e, v);
    const uint32_t b = High ? (((v >> p.target) << (p.target + 1)) | (v & ((1u << p.target) - 1))) : v;
    return ((b & (uint32_t)p.hmask) == (uint32_t)p.hvals) ? (int)b : -1;
}

// Units per loop iteration of a group: every load of an iteration is issued
// before any arithmetic.  Unit k of an iteration is u0 + k * (groups in the
// grid), so each wave-wide load covers 4 adjacent blocks.
template <bool High> struct QUnroll { static constexpr int K = High ? 2 : 4; };

// LowCtl: some control is one of the 6 in-block qubits (tested per
// amplitude); without, every amplitude of a visited block is updated.
template <bool Masked, bool High, bool LowCtl, typename MS>
__global__ __launch_bounds__(kQThreads) void k_q16_gate(u32x4 *__restrict__ codes, int8_t *__restrict__ scales,
                                                        Q16Plan p, MS ms) {
    constexpr int K = QUnroll<High>::K;
    const int j = threadIdx.x & 15;
    const uint32_t a0 = 4u * (uint32_t)j;  // first in-block amplitude of the lane
    const uint64_t groups = ((uint64_t)gridDim.x * kQThreads) >> 4;
    const Mat2<float> M = ms.get();
    const int t = p.target;
    // low targets 2..5: the partner is lane j ^ lm; this lane's row of G
    const int lm = (!High && t >= 2) ? (1 << (t - 2)) : 0;
    const bool hi = (j & lm) != 0;
    const float ur = hi ? M.cr : M.ar, ui = hi ? M.ci : M.ai;
    const float vr = hi ? M.dr : M.br, vi = hi ? M.di : M.bi;
    auto ok = [&](uint32_t a) { return !LowCtl || ((a & p.lmask) == p.lvals); };
    for (uint64_t u0 = ((uint64_t)blockIdx.x * kQThreads + threadIdx.x) >> 4; u0 < p.units; u0 += K * groups) {
        int b[K];
        u32x4 wa[K], wb[K];
        int sa[K], sb[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            b[k] = q_unit_block<Masked, High>(p, u0 + k * groups);  // the same for a group's 16 lanes
            if (b[k] >= 0) {
                wa[k] = ld_nt4(codes + (size_t)b[k] * 16 + j);
                sa[k] = scales[b[k]];
                if (High) {
                    const uint32_t b2 = (uint32_t)b[k] | (1u << t);
                    wb[k] = ld_nt4(codes + (size_t)b2 * 16 + j);
                    sb[k] = scales[b2];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (b[k] < 0)
                continue;
            u32x4 *ca = codes + (size_t)b[k] * 16 + j;
            float xr[4], xi[4];
            q4_decode(wa[k], sa[k], xr, xi);
            if (High) {
                const uint32_t b2 = (uint32_t)b[k] | (1u << t);
                float yr[4], yi[4];
                q4_decode(wb[k], sb[k], yr, yi);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float nxr = xr[i], nxi = xi[i], nyr = yr[i], nyi = yi[i];
                    q_pair(M, nxr, nxi, nyr, nyi);
                    const bool w = ok(a0 + i);
                    xr[i] = w ? nxr : xr[i];
                    xi[i] = w ? nxi : xi[i];
                    yr[i] = w ? nyr : yr[i];
                    yi[i] = w ? nyi : yi[i];
                }
                const int na = q_scale(group16_max(q4_absmax(xr, xi)));
                const int nb = q_scale(group16_max(q4_absmax(yr, yi)));
                st_nt4(ca, q4_encode(xr, xi, na));
                st_nt4(codes + (size_t)b2 * 16 + j, q4_encode(yr, yi, nb));
                if (j == 0) {
                    scales[b[k]] = (int8_t)na;
                    scales[b2] = (int8_t)nb;
                }
            } else {
                // pairs inside the lane (constant register indices)
                auto upd = [&](int i1, int i2) {
                    float nxr = xr[i1], nxi = xi[i1], nyr = xr[i2], nyi = xi[i2];
                    q_pair(M, nxr, nxi, nyr, nyi);
                    const bool w = ok(a0 + i1);
                    xr[i1] = w ? nxr : xr[i1];
                    xi[i1] = w ? nxi : xi[i1];
                    xr[i2] = w ? nyr : xr[i2];
                    xi[i2] = w ? nyi : xi[i2];
                };
                if (t == 0) {
                    upd(0, 1);
                    upd(2, 3);
                } else if (t == 1) {
                    upd(0, 2);
                    upd(1, 3);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float pr = lane_xor(xr[i], lm), pi = lane_xor(xi[i], lm);
                        const float2 p1 = hi ? make_float2(pr, pi) : make_float2(xr[i], xi[i]);
                        const float2 p2 = hi ? make_float2(xr[i], xi[i]) : make_float2(pr, pi);
                        const float2 o = cmac2<float>(ur, ui, p1, vr, vi, p2);
                        const bool w = ok(a0 + i);
                        xr[i] = w ? o.x : xr[i];
                        xi[i] = w ? o.y : xi[i];
                    }
                }
                const int ns = q_scale(group16_max(q4_absmax(xr, xi)));
                st_nt4(ca, q4_encode(xr, xi, ns));
                if (j == 0)
                    scales[b[k]] = (int8_t)ns;
            }
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
        codes[l] = q_word(xr, xi, q_inv(ns));
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
        codes[l] = q_word(re, im, q_inv(ns));
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
        snprintf(buf, sizeof(buf), "sv::k_q16_gate<%s, %s, %s, sv::%s<float> >", p.masked ? "true" : "false",
                 p.high ? "true" : "false", p.lmask ? "true" : "false", matsrc);
    return buf;
}

static unsigned q16_grid(uint64_t groups) {
    DeviceInfo di;
    if (device_info(&di) != SV_OK)
        di.num_cus = 256;
    const uint64_t want = (groups + (kQThreads / 16) - 1) / (kQThreads / 16);
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)di.num_cus * 32));
}

template <bool Masked, bool High, typename MS>
static void go_q16(bool low, dim3 grid, u32x4 *codes, int8_t *sc, const Q16Plan &p, const MS &ms, hipStream_t st) {
    if (low)
        hipLaunchKernelGGL((k_q16_gate<Masked, High, true, MS>), grid, dim3(kQThreads), 0, st, codes, sc, p, ms);
    else
        hipLaunchKernelGGL((k_q16_gate<Masked, High, false, MS>), grid, dim3(kQThreads), 0, st, codes, sc, p, ms);
}

template <typename MS> static int launch_q16(void *state, const Q16Plan &p, const MS &ms, hipStream_t st) {
    int8_t *sc = q16_scales(state, p.n);
    if (p.small) {
        hipLaunchKernelGGL((k_q16_gate_small<MS>), dim3(1), dim3(64), 0, st, (uint32_t *)state, sc, p, ms);
        SV_LAUNCH_CHECK();
        return SV_OK;
    }
    u32x4 *codes = (u32x4 *)state;
    const uint64_t per_group = p.high ? QUnroll<true>::K : QUnroll<false>::K;
    const dim3 grid(q16_grid((p.units + per_group - 1) / per_group));
    const bool low = p.lmask != 0;
    if (p.masked)
        p.high ? go_q16<true, true>(low, grid, codes, sc, p, ms, st) : go_q16<true, false>(low, grid, codes, sc, p, ms, st);
    else
        p.high ? go_q16<false, true>(low, grid, codes, sc, p, ms, st)
               : go_q16<false, false>(low, grid, codes, sc, p, ms, st);
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
