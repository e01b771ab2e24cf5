// Block-scaled fixed-point states (SV_CQ16, SV_CQ32): gate, basis-state and
// conversion kernels.
//
// The paper lists fixed-point state precision as future work (Sec. V); the
// formats are defined in sv.h.  A state holds 2^n amplitudes as two signed
// codes (re, im) each, 16-bit (SV_CQ16, 4 bytes per amplitude: half the
// bytes of complex64) or 32-bit (SV_CQ32, 8 bytes: the bytes of complex64
// with 31 significant bits per block instead of a 24-bit mantissa), then one
// int8 scale per 64-amplitude block; value = code * 2^scale.
//
// A gate works on whole blocks.  A block is decoded (exactly) to float
// (16-bit codes) or double (32-bit codes), the pair update of Sec. III runs
// with the fused multiply-add order every other kernel uses (cmac2), and the
// block is re-encoded under the scale of its new largest component.  So the
// block is what the schedule enumerates: controls on qubits >= 6 are
// inserted into the block index (the skip-interval map of Sec. III-B, one
// level up), controls on the 6 in-block qubits are tested per amplitude.
//
// Mapping: a 16-lane group holds one block, 4 amplitudes per lane (16 bytes
// of 16-bit codes, 32 of 32-bit codes), so each group load is contiguous.  A
// target >= 6 couples block b with block b + 2^(t-6), which the group holds
// in a second set of registers; a target below 6 couples amplitudes inside
// a lane (t < 2) or lane j with lane j ^ 2^(t-2) of the group.  The block
// maximum is a reduction over the group's 16 lanes.  States with n < 6 are
// one block of 2^n amplitudes, handled by one wavefront with one amplitude
// per lane.
#include <algorithm>
#include <cstring>

#include "circuit.hpp"

namespace sv {

constexpr int kQThreads = 256;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u32x4 ld_nt4(const u32x4 *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_nt4(u32x4 *p, u32x4 v) { __builtin_nontemporal_store(v, p); }

template <int Ctrl> __device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, Ctrl, 0xf, 0xf, false);
}

template <int Ctrl> __device__ __forceinline__ float dpp_max(float v) {
    return fmaxf(v, __uint_as_float(dpp_u32<Ctrl>(__float_as_uint(v))));
}

template <int Ctrl> __device__ __forceinline__ double dpp_max(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t o = ((uint64_t)dpp_u32<Ctrl>((uint32_t)(b >> 32)) << 32) | dpp_u32<Ctrl>((uint32_t)b);
    return fmax(v, __builtin_bit_cast(double, o));
}

// Maximum over the 16 lanes of a group, which is one DPP row (lanes
// 16g .. 16g+15): swap neighbours and pairs inside each quad, then mirror
// each half row and the whole row.  All 16 lanes of a row are active
// together (a group shares its work unit).  Values are >= 0.
template <typename R> __device__ __forceinline__ R group16_max(R v) {
    v = dpp_max<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v = dpp_max<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v = dpp_max<0x141>(v);  // row_half_mirror
    v = dpp_max<0x140>(v);  // row_mirror
    return v;
}

template <typename R> __device__ __forceinline__ R wave_max(R m) {
    for (int k = 1; k < 64; k <<= 1)
        m = fmax(m, lane_xor(m, k));
    return m;
}

template <typename R> __device__ __forceinline__ R absmax4(const R (&re)[4], const R (&im)[4]) {
    const R a = fmax(fmax(fabs(re[0]), fabs(im[0])), fabs(re[1]));
    const R b = fmax(fmax(fabs(im[1]), fabs(re[2])), fabs(im[2]));
    return fmax(fmax(a, b), fmax(fabs(re[3]), fabs(im[3])));
}

// ---------------------------------------------------------------- codecs
//
// Encoding a value v under scale s (inv = 2^-s): |v * 2^-s| < 2^B for B-bit
// codes (B = 15 or 31), so adding C = 1.5 * 2^P (P = 23 in float, 52 in
// double) in one fused multiply-add (the product is exact) lands in
// [2^P, 2^(P+1)), where the floats are the integers: that single rounding is
// the round-to-nearest-even of v * 2^-s (C is even, so ties keep their
// parity).  Clamped to C +- (2^B - 1), the value's bits are bits(C) + code,
// and bits(C) has zero low halves, so the low 16 or 32 bits are the code in
// two's complement.  The scale is the exponent e of the largest component
// m = f 2^e (f in [0.5, 1)) minus B, read off m's biased exponent field.

// 16-bit codes: one 32-bit word per amplitude (re in the low half), float.
struct Q16 {
    using R = float;
    static constexpr int kScaleMin = -126, kScaleMax = 112;  // zero blocks take kScaleMin
    static constexpr int kOneScale = -14;                    // 1.0 = 2^14 * 2^-14
    static constexpr size_t kAmpBytes = 4;
    struct Lane {
        u32x4 w;  // amplitudes 4j .. 4j+3 of the block
    };
    __device__ static Lane ld(const char *block, int j) { return {ld_nt4((const u32x4 *)block + j)}; }
    __device__ static void st(char *block, int j, const Lane &l) { st_nt4((u32x4 *)block + j, l.w); }
    __device__ static float dec(int code, int s) { return ldexpf((float)code, s); }
    __device__ static void unword(uint32_t w, int s, float &re, float &im) {
        re = dec((int)(int16_t)(w & 0xffffu), s);
        im = dec((int)(int16_t)(w >> 16), s);
    }
    __device__ static uint32_t biased(float v, float inv) {
        const float y = __builtin_fmaf(v, inv, 12582912.0f);
        return __float_as_uint(__builtin_amdgcn_fmed3f(y, 12582912.0f - 32767.0f, 12582912.0f + 32767.0f));
    }
    __device__ static uint32_t word(float re, float im, float inv) {
        return __builtin_amdgcn_perm(biased(im, inv), biased(re, inv), 0x05040100u);
    }
    __device__ static float inv(int s) { return ldexpf(1.0f, -s); }
    __device__ static int scale(float m) {
        const int e = (int)(__float_as_uint(m) >> 23) - 141;  // biased exponent - 126 - 15
        return min(max(e, kScaleMin), kScaleMax);
    }
    __device__ static void decode(const Lane &l, int s, float (&re)[4], float (&im)[4]) {
        unword(l.w.x, s, re[0], im[0]);
        unword(l.w.y, s, re[1], im[1]);
        unword(l.w.z, s, re[2], im[2]);
        unword(l.w.w, s, re[3], im[3]);
    }
    __device__ static Lane encode(const float (&re)[4], const float (&im)[4], int s) {
        const float iv = inv(s);
        Lane l;
        l.w.x = word(re[0], im[0], iv);
        l.w.y = word(re[1], im[1], iv);
        l.w.z = word(re[2], im[2], iv);
        l.w.w = word(re[3], im[3], iv);
        return l;
    }
    // one amplitude (states below one block)
    __device__ static void ld1(const char *codes, uint64_t k, int s, float &re, float &im) {
        unword(((const uint32_t *)codes)[k], s, re, im);
    }
    __device__ static void st1(char *codes, uint64_t k, float re, float im, int s) {
        ((uint32_t *)codes)[k] = word(re, im, inv(s));
    }
    __device__ static void st1_one(char *codes, uint64_t k, bool one) {  // basis state: 1.0 or 0
        ((uint32_t *)codes)[k] = one ? 16384u : 0u;
    }
};

// 32-bit codes: two 32-bit words per amplitude (re, im), double.
struct Q32 {
    using R = double;
    static constexpr int kScaleMin = -128, kScaleMax = 96;
    static constexpr int kOneScale = -30;  // 1.0 = 2^30 * 2^-30
    static constexpr size_t kAmpBytes = 8;
    struct Lane {
        u32x4 a, b;  // amplitudes 4j, 4j+1 and 4j+2, 4j+3: (re, im, re, im)
    };
    __device__ static Lane ld(const char *block, int j) {
        const u32x4 *p = (const u32x4 *)block + 2 * j;
        return {ld_nt4(p), ld_nt4(p + 1)};
    }
    __device__ static void st(char *block, int j, const Lane &l) {
        u32x4 *p = (u32x4 *)block + 2 * j;
        st_nt4(p, l.a);
        st_nt4(p + 1, l.b);
    }
    __device__ static double dec(uint32_t code, int s) { return ldexp((double)(int32_t)code, s); }
    __device__ static uint32_t code(double v, double iv) {
        const double y = __builtin_fma(v, iv, 6755399441055744.0);
        const double c = fmin(fmax(y, 6755399441055744.0 - 2147483647.0), 6755399441055744.0 + 2147483647.0);
        return (uint32_t)__builtin_bit_cast(uint64_t, c);
    }
    __device__ static double inv(int s) { return ldexp(1.0, -s); }
    __device__ static int scale(double m) {
        const int e = (int)(__builtin_bit_cast(uint64_t, m) >> 52) - 1053;  // biased exponent - 1022 - 31
        return min(max(e, kScaleMin), kScaleMax);
    }
    __device__ static void decode(const Lane &l, int s, double (&re)[4], double (&im)[4]) {
        re[0] = dec(l.a.x, s);
        im[0] = dec(l.a.y, s);
        re[1] = dec(l.a.z, s);
        im[1] = dec(l.a.w, s);
        re[2] = dec(l.b.x, s);
        im[2] = dec(l.b.y, s);
        re[3] = dec(l.b.z, s);
        im[3] = dec(l.b.w, s);
    }
    __device__ static Lane encode(const double (&re)[4], const double (&im)[4], int s) {
        const double iv = inv(s);
        Lane l;
        l.a.x = code(re[0], iv);
        l.a.y = code(im[0], iv);
        l.a.z = code(re[1], iv);
        l.a.w = code(im[1], iv);
        l.b.x = code(re[2], iv);
        l.b.y = code(im[2], iv);
        l.b.z = code(re[3], iv);
        l.b.w = code(im[3], iv);
        return l;
    }
    __device__ static void ld1(const char *codes, uint64_t k, int s, double &re, double &im) {
        const uint2 w = ((const uint2 *)codes)[k];
        re = dec(w.x, s);
        im = dec(w.y, s);
    }
    __device__ static void st1(char *codes, uint64_t k, double re, double im, int s) {
        const double iv = inv(s);
        ((uint2 *)codes)[k] = make_uint2(code(re, iv), code(im, iv));
    }
    __device__ static void st1_one(char *codes, uint64_t k, bool one) {
        ((uint2 *)codes)[k] = make_uint2(one ? (1u << 30) : 0u, 0u);
    }
};

// Pair update of (x, y) = (C_k, C_{k+2^t}).
template <typename R> __device__ __forceinline__ void q_pair(const Mat2<R> &M, R &xr, R &xi, R &yr, R &yi) {
    cplx_t<R> x, y;
    x.x = xr;
    x.y = xi;
    y.x = yr;
    y.y = yi;
    apply_pair<R>(M, x, y);
    xr = x.x;
    xi = x.y;
    yr = y.x;
    yi = y.y;
}

// One row of the pair update for a lane that holds one element of the pair
// and receives the other (pr, pi) from its partner: the lane with the target
// bit clear computes a C_k + b C_{k+2^t}, the other c C_k + d C_{k+2^t}.
template <typename R>
__device__ __forceinline__ void q_row(R ur, R ui, R vr, R vi, bool hi, R &xr, R &xi, R pr, R pi) {
    cplx_t<R> p1, p2;
    p1.x = hi ? pr : xr;
    p1.y = hi ? pi : xi;
    p2.x = hi ? xr : pr;
    p2.y = hi ? xi : pi;
    const cplx_t<R> o = cmac2<R>(ur, ui, p1, vr, vi, p2);
    xr = o.x;
    xi = o.y;
}

// Block index of unit u, or -1 when a masked launch skips it.  Block
// indices have at most 30 bits.
template <bool Masked, bool High> __device__ __forceinline__ int q_unit_block(const FixedPlan &p, uint64_t u) {
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
template <typename Q, bool Masked, bool High, bool LowCtl, typename MS>
__global__ __launch_bounds__(kQThreads) void k_fix_gate(char *__restrict__ codes, int8_t *__restrict__ scales,
                                                        FixedPlan p, MS ms) {
    using R = typename Q::R;
    constexpr size_t kBlockBytes = 64 * Q::kAmpBytes;
    constexpr int K = QUnroll<High>::K;
    const int j = threadIdx.x & 15;
    const uint32_t a0 = 4u * (uint32_t)j;  // first in-block amplitude of the lane
    const uint64_t groups = ((uint64_t)gridDim.x * kQThreads) >> 4;
    const Mat2<R> M = ms.get();
    const int t = p.target;
    // low targets 2..5: the partner is lane j ^ lm; this lane's row of G
    const int lm = (!High && t >= 2) ? (1 << (t - 2)) : 0;
    const bool hi = (j & lm) != 0;
    const R ur = hi ? M.cr : M.ar, ui = hi ? M.ci : M.ai;
    const R vr = hi ? M.dr : M.br, vi = hi ? M.di : M.bi;
    auto ok = [&](uint32_t a) { return !LowCtl || ((a & p.lmask) == p.lvals); };
    for (uint64_t u0 = ((uint64_t)blockIdx.x * kQThreads + threadIdx.x) >> 4; u0 < p.units; u0 += K * groups) {
        int b[K];
        typename Q::Lane wa[K], wb[K];
        int sa[K], sb[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            b[k] = q_unit_block<Masked, High>(p, u0 + k * groups);  // the same for a group's 16 lanes
            if (b[k] >= 0) {
                wa[k] = Q::ld(codes + (size_t)b[k] * kBlockBytes, j);
                sa[k] = scales[b[k]];
                if (High) {
                    const uint32_t b2 = (uint32_t)b[k] | (1u << t);
                    wb[k] = Q::ld(codes + (size_t)b2 * kBlockBytes, j);
                    sb[k] = scales[b2];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (b[k] < 0)
                continue;
            char *ca = codes + (size_t)b[k] * kBlockBytes;
            R xr[4], xi[4];
            Q::decode(wa[k], sa[k], xr, xi);
            if (High) {
                const uint32_t b2 = (uint32_t)b[k] | (1u << t);
                R yr[4], yi[4];
                Q::decode(wb[k], sb[k], yr, yi);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    R nxr = xr[i], nxi = xi[i], nyr = yr[i], nyi = yi[i];
                    q_pair<R>(M, nxr, nxi, nyr, nyi);
                    const bool w = ok(a0 + i);
                    xr[i] = w ? nxr : xr[i];
                    xi[i] = w ? nxi : xi[i];
                    yr[i] = w ? nyr : yr[i];
                    yi[i] = w ? nyi : yi[i];
                }
                const int na = Q::scale(group16_max<R>(absmax4<R>(xr, xi)));
                const int nb = Q::scale(group16_max<R>(absmax4<R>(yr, yi)));
                Q::st(ca, j, Q::encode(xr, xi, na));
                Q::st(codes + (size_t)b2 * kBlockBytes, j, Q::encode(yr, yi, nb));
                if (j == 0) {
                    scales[b[k]] = (int8_t)na;
                    scales[b2] = (int8_t)nb;
                }
            } else {
                // pairs inside the lane (constant register indices)
                auto upd = [&](int i1, int i2) {
                    R nxr = xr[i1], nxi = xi[i1], nyr = xr[i2], nyi = xi[i2];
                    q_pair<R>(M, nxr, nxi, nyr, nyi);
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
                        const R pr = lane_xor(xr[i], lm), pi = lane_xor(xi[i], lm);
                        R nr = xr[i], ni = xi[i];
                        q_row<R>(ur, ui, vr, vi, hi, nr, ni, pr, pi);
                        const bool w = ok(a0 + i);
                        xr[i] = w ? nr : xr[i];
                        xi[i] = w ? ni : xi[i];
                    }
                }
                const int ns = Q::scale(group16_max<R>(absmax4<R>(xr, xi)));
                Q::st(ca, j, Q::encode(xr, xi, ns));
                if (j == 0)
                    scales[b[k]] = (int8_t)ns;
            }
        }
    }
}

// n < 6: the state is one block of 2^n amplitudes; lane l holds amplitude l.
template <typename Q, typename MS>
__global__ __launch_bounds__(64) void k_fix_gate_small(char *__restrict__ codes, int8_t *__restrict__ scales,
                                                       FixedPlan p, MS ms) {
    using R = typename Q::R;
    const int l = threadIdx.x;
    const bool valid = l < (1 << p.n);
    const Mat2<R> M = ms.get();
    const int s = scales[0];
    R xr = 0, xi = 0;
    if (valid)
        Q::ld1(codes, (uint64_t)l, s, xr, xi);
    const int tm = 1 << p.target;
    const R pr = lane_xor(xr, tm), pi = lane_xor(xi, tm);
    const bool hi = (l & tm) != 0;
    if (valid && (((uint32_t)l & p.lmask) == p.lvals))
        q_row<R>(hi ? M.cr : M.ar, hi ? M.ci : M.ai, hi ? M.dr : M.br, hi ? M.di : M.bi, hi, xr, xi, pr, pi);
    const int ns = Q::scale(wave_max<R>(fmax(fabs(xr), fabs(xi))));  // 0 on lanes past the state
    if (valid)
        Q::st1(codes, (uint64_t)l, xr, xi, ns);
    if (l == 0)
        scales[0] = (int8_t)ns;
}

// ---------------------------------------------------------------- conversions

template <typename Q, typename RS>
__global__ __launch_bounds__(kQThreads) void k_fix_encode(const cplx_t<RS> *__restrict__ src, char *__restrict__ codes,
                                                          int8_t *__restrict__ scales, uint64_t nblocks) {
    using R = typename Q::R;
    const int j = threadIdx.x & 15;
    const uint64_t gstride = ((uint64_t)gridDim.x * kQThreads) >> 4;
    for (uint64_t b = ((uint64_t)blockIdx.x * kQThreads + threadIdx.x) >> 4; b < nblocks; b += gstride) {
        const cplx_t<RS> *v = src + b * 64 + 4 * j;
        R re[4], im[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const cplx_t<RS> a = v[i];
            re[i] = (R)a.x;  // to nearest (complex128 to float), or exact
            im[i] = (R)a.y;
        }
        const int ns = Q::scale(group16_max<R>(absmax4<R>(re, im)));
        Q::st(codes + b * 64 * Q::kAmpBytes, j, Q::encode(re, im, ns));
        if (j == 0)
            scales[b] = (int8_t)ns;
    }
}

template <typename Q, typename RS>
__global__ __launch_bounds__(64) void k_fix_encode_small(const cplx_t<RS> *__restrict__ src, char *__restrict__ codes,
                                                         int8_t *__restrict__ scales, int n) {
    using R = typename Q::R;
    const int l = threadIdx.x;
    const bool valid = l < (1 << n);
    R re = 0, im = 0;
    if (valid) {
        const cplx_t<RS> a = src[l];
        re = (R)a.x;
        im = (R)a.y;
    }
    const int ns = Q::scale(wave_max<R>(fmax(fabs(re), fabs(im))));
    if (valid)
        Q::st1(codes, (uint64_t)l, re, im, ns);
    if (l == 0)
        scales[0] = (int8_t)ns;
}

template <typename Q, typename RD>
__global__ __launch_bounds__(256) void k_fix_decode(const char *__restrict__ codes, const int8_t *__restrict__ scales,
                                                    cplx_t<RD> *__restrict__ dst, uint64_t N) {
    using R = typename Q::R;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += stride) {
        R re, im;
        Q::ld1(codes, k, scales[k >> kQBlockBits], re, im);
        cplx_t<RD> o;
        o.x = (RD)re;
        o.y = (RD)im;
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

// |b>: 1.0 exactly (code 2^14 under scale -14, or 2^30 under -30) at
// amplitude b, every other amplitude 0 and every other block at the
// zero-block scale.
template <typename Q>
__global__ __launch_bounds__(256) void k_fix_basis(char *__restrict__ codes, int8_t *__restrict__ scales, uint64_t N,
                                                   uint64_t nblocks, uint64_t b) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t k = i0; k < N; k += stride)
        Q::st1_one(codes, k, k == b);
    for (uint64_t k = i0; k < nblocks; k += stride)
        scales[k] = (int8_t)((k == (b >> kQBlockBits)) ? Q::kOneScale : Q::kScaleMin);
}

// ---------------------------------------------------------------- fused pass
//
// A fused run over a fixed-point state: each workgroup decodes one tile (the
// 2^m amplitudes sharing the index bits outside the run's qubit set, which
// holds qubits 0..5, so a tile is whole blocks) into LDS in the format's
// arithmetic type, applies the run's operations there with the same tile code
// as complex states (float tiles for 16-bit codes, double for 32-bit), and
// re-encodes every block of the tile once.  So a block is rounded once per
// pass instead of once per gate.  A 16-lane group holds one block, 4
// amplitudes per lane, as in the gate kernel.
template <typename Q>
__global__ __launch_bounds__(512, 4) void k_fix_tile(char *__restrict__ codes, int8_t *__restrict__ scales,
                                                     TileMap tm, DeviceGates gates) {
    using R = typename Q::R;
    constexpr size_t kBlockBytes = 64 * Q::kAmpBytes;
    extern __shared__ unsigned char lds_raw[];
    cplx_t<R> *tile = reinterpret_cast<cplx_t<R> *>(lds_raw);
    const uint64_t base = expand_index<uint64_t>(tm.outer, tm.tile0 + blockIdx.x);
    if (!tile_touched(base, gates))
        return;  // no operation of the run touches it: its blocks stay as they are
    const uint32_t nblk = 1u << (tm.m - kQBlockBits);
    const int j = threadIdx.x & 15;
    for (uint32_t bl = threadIdx.x >> 4; bl < nblk; bl += 512 / 16) {
        const uint32_t t0 = bl << kQBlockBits;  // tile index of the block's first amplitude
        const uint64_t b = (base | tile_offset(tm, t0)) >> kQBlockBits;
        const typename Q::Lane w = Q::ld(codes + b * kBlockBytes, j);
        R re[4], im[4];
        Q::decode(w, scales[b], re, im);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            cplx_t<R> v;
            v.x = re[i];
            v.y = im[i];
            tile[t0 + 4 * j + i] = v;
        }
    }
    __syncthreads();
    tile_run<R, 512>(tile, base, tm, gates);
    __syncthreads();
    for (uint32_t bl = threadIdx.x >> 4; bl < nblk; bl += 512 / 16) {
        const uint32_t t0 = bl << kQBlockBits;
        const uint64_t b = (base | tile_offset(tm, t0)) >> kQBlockBits;
        R re[4], im[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const cplx_t<R> v = tile[t0 + 4 * j + i];
            re[i] = v.x;
            im[i] = v.y;
        }
        const int s = Q::scale(group16_max<R>(absmax4<R>(re, im)));
        Q::st(codes + b * kBlockBytes, j, Q::encode(re, im, s));
        if (j == 0)
            scales[b] = (int8_t)s;
    }
}

// ---------------------------------------------------------------- host side

static int8_t *fixed_scales(void *state, int n, int dtype) {
    return (int8_t *)((char *)state + ((size_t)1 << n) * amp_bytes(dtype));
}

int make_fixed_plan(const GateSpec &g, int dtype, bool masked, FixedPlan *out) {
    FixedPlan q;
    memset(&q, 0, sizeof(q));
    q.n = g.n;
    q.dtype = dtype;
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

std::string fixed_plan_name(const FixedPlan &p, const char *matsrc) {
    const bool wide = p.dtype == SV_CQ32;
    const char *Q = wide ? "sv::Q32" : "sv::Q16";
    const char *R = wide ? "double" : "float";
    char buf[256];
    if (p.small)
        snprintf(buf, sizeof(buf), "sv::k_fix_gate_small<%s, sv::%s<%s> >", Q, matsrc, R);
    else
        snprintf(buf, sizeof(buf), "sv::k_fix_gate<%s, %s, %s, %s, sv::%s<%s> >", Q, p.masked ? "true" : "false",
                 p.high ? "true" : "false", p.lmask ? "true" : "false", matsrc, R);
    return buf;
}

static unsigned fix_grid(uint64_t groups) {
    DeviceInfo di;
    if (device_info(&di) != SV_OK)
        di.num_cus = 256;
    const uint64_t want = (groups + (kQThreads / 16) - 1) / (kQThreads / 16);
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)di.num_cus * 32));
}

template <typename Q, bool Masked, bool High, typename MS>
static void go_fix(bool low, dim3 grid, char *codes, int8_t *sc, const FixedPlan &p, const MS &ms, hipStream_t st) {
    if (low)
        hipLaunchKernelGGL((k_fix_gate<Q, Masked, High, true, MS>), grid, dim3(kQThreads), 0, st, codes, sc, p, ms);
    else
        hipLaunchKernelGGL((k_fix_gate<Q, Masked, High, false, MS>), grid, dim3(kQThreads), 0, st, codes, sc, p, ms);
}

template <typename Q, typename MS>
static int launch_fix(void *state, const FixedPlan &p, const MS &ms, hipStream_t st) {
    char *codes = (char *)state;
    int8_t *sc = fixed_scales(state, p.n, p.dtype);
    if (p.small) {
        hipLaunchKernelGGL((k_fix_gate_small<Q, MS>), dim3(1), dim3(64), 0, st, codes, sc, p, ms);
        SV_LAUNCH_CHECK();
        return SV_OK;
    }
    const uint64_t per_group = p.high ? QUnroll<true>::K : QUnroll<false>::K;
    const dim3 grid(fix_grid((p.units + per_group - 1) / per_group));
    const bool low = p.lmask != 0;
    if (p.masked)
        p.high ? go_fix<Q, true, true>(low, grid, codes, sc, p, ms, st)
               : go_fix<Q, true, false>(low, grid, codes, sc, p, ms, st);
    else
        p.high ? go_fix<Q, false, true>(low, grid, codes, sc, p, ms, st)
               : go_fix<Q, false, false>(low, grid, codes, sc, p, ms, st);
    SV_LAUNCH_CHECK();
    return SV_OK;
}

int launch_fixed_gate(void *state, const FixedPlan &p, const double *U, const double *Ud, hipStream_t st) {
    if (p.dtype == SV_CQ32) {
        if (Ud)
            return launch_fix<Q32>(state, p, MatPtr<double>{Ud}, st);
        return launch_fix<Q32>(state, p, MatVal<double>{to_mat<double>(U)}, st);
    }
    if (Ud)
        return launch_fix<Q16>(state, p, MatPtr<float>{Ud}, st);
    return launch_fix<Q16>(state, p, MatVal<float>{to_mat<float>(U)}, st);
}

int launch_fixed_basis(void *state, int n, int dtype, uint64_t basis, unsigned grid, hipStream_t st) {
    char *codes = (char *)state;
    int8_t *sc = fixed_scales(state, n, dtype);
    if (dtype == SV_CQ32)
        hipLaunchKernelGGL(k_fix_basis<Q32>, dim3(grid), dim3(256), 0, st, codes, sc, 1ull << n, q16_blocks(n), basis);
    else
        hipLaunchKernelGGL(k_fix_basis<Q16>, dim3(grid), dim3(256), 0, st, codes, sc, 1ull << n, q16_blocks(n), basis);
    SV_LAUNCH_CHECK();
    return SV_OK;
}

template <typename Q, typename RS> static int encode_from(const sv_state_t *dst, const sv_state_t *src, hipStream_t st) {
    const int n = src->n;
    char *codes = (char *)dst->data;
    int8_t *sc = fixed_scales(dst->data, n, dst->dtype);
    if (n < kQBlockBits)
        hipLaunchKernelGGL((k_fix_encode_small<Q, RS>), dim3(1), dim3(64), 0, st, (const cplx_t<RS> *)src->data, codes,
                           sc, n);
    else
        hipLaunchKernelGGL((k_fix_encode<Q, RS>), dim3(fix_grid(q16_blocks(n))), dim3(kQThreads), 0, st,
                           (const cplx_t<RS> *)src->data, codes, sc, q16_blocks(n));
    SV_LAUNCH_CHECK();
    return SV_OK;
}

static unsigned flat_grid(uint64_t N) {
    DeviceInfo di;
    if (device_info(&di) != SV_OK)
        di.num_cus = 256;
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((N + 255) / 256, (uint64_t)di.num_cus * 16));
}

int fixed_tile_lds_limit(int dtype, size_t lds) {
    const void *fn = dtype == SV_CQ16 ? (const void *)k_fix_tile<Q16> : (const void *)k_fix_tile<Q32>;
    SV_HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return SV_OK;
}

int launch_fixed_tile_pass(void *state, int n, int dtype, const TileMap &tm_in, const DeviceGates &dg, size_t lds,
                           hipStream_t st) {
    if (tm_in.m < (uint32_t)kQBlockBits || tm_in.a < (uint32_t)kQBlockBits)
        return fail(SV_EINVAL, "fixed-point tile (m=%u, contiguous %u) must hold whole blocks", tm_in.m, tm_in.a);
    char *codes = (char *)state;
    int8_t *sc = fixed_scales(state, n, dtype);
    TileMap tm = tm_in;
    tm.tab = 1;  // lds includes the tables
    for (uint64_t t0 = 0; t0 < tm.ntiles; t0 += kMaxGridBlocks) {
        tm.tile0 = t0;
        const dim3 grid((unsigned)std::min(kMaxGridBlocks, tm_in.ntiles - t0));
        if (dtype == SV_CQ16)
            hipLaunchKernelGGL(k_fix_tile<Q16>, grid, dim3(512), lds, st, codes, sc, tm, dg);
        else
            hipLaunchKernelGGL(k_fix_tile<Q32>, grid, dim3(512), lds, st, codes, sc, tm, dg);
        SV_LAUNCH_CHECK();
    }
    return SV_OK;
}

template <typename Q, typename RD> static int decode_to(const sv_state_t *dst, const sv_state_t *src, hipStream_t st) {
    const uint64_t N = 1ull << src->n;
    hipLaunchKernelGGL((k_fix_decode<Q, RD>), dim3(flat_grid(N)), dim3(256), 0, st, (const char *)src->data,
                       (const int8_t *)fixed_scales(src->data, src->n, src->dtype), (cplx_t<RD> *)dst->data, N);
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
    if (!known_dtype(dtype))
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
    if (is_fixed(dst->dtype) && is_fixed(src->dtype))
        return fail(SV_ENOTSUP, "conversion between the two fixed-point formats: convert through complex128");
    const char *a = (const char *)src->data, *b = (const char *)dst->data;
    if (a < b + state_bytes(dst->n, dst->dtype) && b < a + state_bytes(src->n, src->dtype))
        return fail(SV_EINVAL, "source and destination overlap");
    const hipStream_t s = (hipStream_t)st;
    const uint64_t N = 1ull << src->n;
    const bool from128 = src->dtype == SV_C128, to128 = dst->dtype == SV_C128;
    if (dst->dtype == SV_CQ16)
        return from128 ? encode_from<Q16, double>(dst, src, s) : encode_from<Q16, float>(dst, src, s);
    if (dst->dtype == SV_CQ32)
        return from128 ? encode_from<Q32, double>(dst, src, s) : encode_from<Q32, float>(dst, src, s);
    if (src->dtype == SV_CQ16)
        return to128 ? decode_to<Q16, double>(dst, src, s) : decode_to<Q16, float>(dst, src, s);
    if (src->dtype == SV_CQ32)
        return to128 ? decode_to<Q32, double>(dst, src, s) : decode_to<Q32, float>(dst, src, s);
    if (from128)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(flat_grid(N)), dim3(256), 0, s,
                           (const double2 *)src->data, (float2 *)dst->data, N);
    else
        hipLaunchKernelGGL((k_convert<float, double>), dim3(flat_grid(N)), dim3(256), 0, s,
                           (const float2 *)src->data, (double2 *)dst->data, N);
    SV_LAUNCH_CHECK();
    return SV_OK;
}

} // extern "C"
