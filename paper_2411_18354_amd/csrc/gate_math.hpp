// Device arithmetic shared by every kernel that applies a 2x2 gate, so that
// all kernels produce bit-identical amplitudes for the same pair.
#pragma once

#include "sv_internal.hpp"

namespace sv {

// out = u * x + v * y for complex u, v, x, y, with a fixed fused
// multiply-add order (one rounding chain per component).  Pair-update
// equation of Sec. III: new C_k = a C_k + b C_{k+2^t},
// new C_{k+2^t} = c C_k + d C_{k+2^t}.
template <typename R>
__device__ __forceinline__ cplx_t<R> cmac2(R ur, R ui, cplx_t<R> x, R vr, R vi, cplx_t<R> y) {
    cplx_t<R> o;
    o.x = __builtin_fma(ur, x.x, __builtin_fma(-ui, x.y, __builtin_fma(vr, y.x, -(vi * y.y))));
    o.y = __builtin_fma(ur, x.y, __builtin_fma(ui, x.x, __builtin_fma(vr, y.y, vi * y.x)));
    return o;
}

template <>
__device__ __forceinline__ cplx_t<float> cmac2<float>(float ur, float ui, cplx_t<float> x, float vr, float vi,
                                                      cplx_t<float> y) {
    cplx_t<float> o;
    o.x = __builtin_fmaf(ur, x.x, __builtin_fmaf(-ui, x.y, __builtin_fmaf(vr, y.x, -(vi * y.y))));
    o.y = __builtin_fmaf(ur, x.y, __builtin_fmaf(ui, x.x, __builtin_fmaf(vr, y.y, vi * y.x)));
    return o;
}

template <typename R>
__device__ __forceinline__ void apply_pair(const Mat2<R> &m, cplx_t<R> &x, cplx_t<R> &y) {
    const cplx_t<R> nx = cmac2<R>(m.ar, m.ai, x, m.br, m.bi, y);
    const cplx_t<R> ny = cmac2<R>(m.cr, m.ci, x, m.dr, m.di, y);
    x = nx;
    y = ny;
}

// Where a kernel takes its 2x2 matrix from: by value in the kernel arguments
// (single gates from the host), or from device memory written by an earlier
// kernel (circuits whose angles live on the device).
template <typename R> struct MatVal {
    Mat2<R> m;
    __device__ __forceinline__ Mat2<R> get() const { return m; }
};

template <typename R> struct MatPtr {
    const double *p;  // 8 doubles
    __device__ __forceinline__ Mat2<R> get() const {
        return Mat2<R>{(R)p[0], (R)p[1], (R)p[2], (R)p[3], (R)p[4], (R)p[5], (R)p[6], (R)p[7]};
    }
};

// Streaming global accesses.  Every amplitude of a pass is read once and
// written once, so the loads and stores carry the nontemporal hint (measured
// on MI355X: in-place read-modify-write of 4 GiB reaches about 5.9 TB/s with
// the hint against about 5.4 TB/s without).
template <typename R> __device__ __forceinline__ cplx_t<R> ld_stream(const cplx_t<R> *p) {
    cplx_t<R> v;
    v.x = __builtin_nontemporal_load(&p->x);
    v.y = __builtin_nontemporal_load(&p->y);
    return v;
}

template <typename R> __device__ __forceinline__ void st_stream(cplx_t<R> *p, cplx_t<R> v) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}

// Cross-lane exchange inside a 64-lane wavefront: value held by lane
// (lane ^ mask).
__device__ __forceinline__ int lane_xor_i(int v, int mask) {
    const int addr = (((int)__lane_id()) ^ mask) << 2;
    return __builtin_amdgcn_ds_bpermute(addr, v);
}

__device__ __forceinline__ double lane_xor(double v, int mask) {
    const int lo = lane_xor_i(__double2loint(v), mask);
    const int hi = lane_xor_i(__double2hiint(v), mask);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float lane_xor(float v, int mask) {
    return __int_as_float(lane_xor_i(__float_as_int(v), mask));
}

template <typename R>
__device__ __forceinline__ cplx_t<R> lane_xor(cplx_t<R> v, int mask) {
    cplx_t<R> o;
    o.x = lane_xor(v.x, mask);
    o.y = lane_xor(v.y, mask);
    return o;
}

} // namespace sv
