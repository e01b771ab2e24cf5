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
//
// Tile passes.  A tile is the 2^m amplitudes (m = min(n, 12)) whose indices
// agree outside a qubit set T made of qubits 0..5 and m - 6 others.  A term
// whose x mask lies inside T pairs amplitudes of one tile only, so one read
// of the state into LDS serves every such term: the terms are split into
// tile sets (the first is qubits 0..m-1; the others take the remaining x
// masks' qubits above 5, first fit, then are filled up to m with the lowest
// unused qubits), and one pass per set (<= 64 terms) evaluates them all.
// Diagonal terms join the first set.  Groups whose x mask has more than
// m - 6 qubits above 5 keep the one-pass-per-group kernel.
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

constexpr int kTileBits = 12;                                 // tile: 2^12 amplitudes, 64 KiB of double2
constexpr int kTileLow = 6;                                   // qubits 0..5 are in every tile
constexpr int kTileTerms = 64;                                // terms per tile pass: one lane each
constexpr int kTileThreads = 256;
constexpr int kTilePerLane = (1 << kTileBits) / kTileThreads;  // amplitudes per lane and tile

// A term of a tile pass, its masks split at the tile's qubit set T.
struct TTerm {
    uint64_t zh;      // z outside T: the sign set by the tile's fixed bits
    uint32_t xl, zl;  // x (inside T, nonzero unless diagonal) and z on T, as tile-local bits
    int32_t ny;       // |x & z| mod 4: the power of i
    int32_t slot;     // the term's position in the plan: its row of partials
};

// One tile pass.  Tile-local bit r < L (L = min(m, 6)) is qubit r; bit L + q
// is the q-th lowest qubit of himask; the tile number's bit r is the r-th
// lowest qubit of frmask.
struct TilePass {
    uint64_t himask, frmask;
    int32_t m, nfree;
    int32_t nt, nd, ne, pad;  // terms: nd diagonal, then ne with even ny, then odd ny
    TTerm t[kTileTerms];
};

// The bits of v, lowest first, placed at the set bits of mask, lowest first.
__device__ __forceinline__ uint64_t deposit_bits(uint64_t v, uint64_t mask) {
    uint64_t out = 0;
    while (mask) {
        if (v & 1ull)
            out |= mask & (~mask + 1ull);
        v >>= 1;
        mask &= mask - 1ull;
    }
    return out;
}

// Four terms of a tile pass at a time (independent chains for the
// scheduler to interleave): slots past the end repeat the last term and are
// dropped.  s(k) = (-1)^{zl.k}.  Lane tid's r-th amplitude of a tile is
// l = tid | (r << 8), and its r-th pair index tid | (r << 8); inserting a
// cleared bit b is linear over xor, so each sign splits into a lane part
// and a part per r (uniform), and every update is one fused multiply-add by
// +-1.  Off-diagonal terms take Re(i^ny w) from Re w (IM false, ny even) or
// Im w (IM true, ny odd) and add twice the sum over the lane's pairs
// (l, l ^ xl) of s(l ^ xl) Re(i^ny conj(t_l) t_{l^xl}).
struct TileTerms {
    uint32_t txl, tzl, tzh_lo, tzh_hi;
    int tny;
};

__device__ __forceinline__ void tile_accumulate(const TileTerms &T, int j, int end, const double (&ts)[4],
                                                uint64_t base, uint32_t lane, double &acc) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int jq = j + q;
        if (jq < end) {
            const uint64_t zh = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)T.tzh_hi, jq) << 32) |
                                (uint32_t)__builtin_amdgcn_readlane((int)T.tzh_lo, jq);
            if (lane == (uint32_t)jq)
                acc += odd_parity(zh & base) ? -ts[q] : ts[q];
        }
    }
}

// Walsh transform over the register bits: v[s] <- sum_r (-1)^{popc(s & r)} v[r].
__device__ __forceinline__ void walsh16(double (&v)[kTilePerLane]) {
#pragma unroll
    for (int h = 1; h < kTilePerLane; h <<= 1)
#pragma unroll
        for (int r = 0; r < kTilePerLane; ++r)
            if (!(r & h)) {
                const double a = v[r], b = v[r | h];
                v[r] = a + b;
                v[r | h] = a - b;
            }
}

// v[s] for a uniform s < 16 (static register indices).
__device__ __forceinline__ double pick16(const double (&v)[kTilePerLane], uint32_t s) {
    switch (s) {
    case 0: return v[0];
    case 1: return v[1];
    case 2: return v[2];
    case 3: return v[3];
    case 4: return v[4];
    case 5: return v[5];
    case 6: return v[6];
    case 7: return v[7];
    case 8: return v[8];
    case 9: return v[9];
    case 10: return v[10];
    case 11: return v[11];
    case 12: return v[12];
    case 13: return v[13];
    case 14: return v[14];
    default: return v[15];
    }
}

// Diagonal terms: the lane's sum of s(l) |t_l|^2 over l = tid | (r << 8) is
// (-1)^{zl.tid} times the Walsh coefficient of its |t|^2 at zl >> 8.
__device__ __forceinline__ void tile_diag(const TileTerms &T, int j0, int j1, const double (&wc)[kTilePerLane],
                                          uint32_t tid, uint64_t base, uint32_t lane, double &acc) {
    for (int j = j0; j < j1; j += 4) {
        double ts[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t zl = (uint32_t)__builtin_amdgcn_readlane((int)T.tzl, min(j + q, j1 - 1));
            ts[q] = pick16(wc, zl >> 8);
            if (__popc(zl & tid) & 1)
                ts[q] = -ts[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            ts[q] = wave_sum(ts[q]);
        tile_accumulate(T, j, j1, ts, base, lane, acc);
    }
}

template <bool IM>
__device__ __forceinline__ void tile_offdiag(const TileTerms &T, int j0, int j1, const double2 *tile, uint32_t tid,
                                             uint32_t M, uint64_t base, uint32_t lane, double &acc) {
    for (int j = j0; j < j1; j += 4) {
        uint32_t xl[4], zl[4], b[4], lt[4];
        double ts[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int jq = min(j + q, j1 - 1);
            xl[q] = (uint32_t)__builtin_amdgcn_readlane((int)T.txl, jq);
            zl[q] = (uint32_t)__builtin_amdgcn_readlane((int)T.tzl, jq);
            b[q] = (uint32_t)__builtin_ctz(xl[q]);
            lt[q] = ((tid >> b[q]) << (b[q] + 1)) | (tid & ((1u << b[q]) - 1));
            ts[q] = 0.0;
        }
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)kTilePerLane / 2; ++r) {
            if ((tid | (r << 8)) < M / 2) {
                const uint32_t ir = r << 8;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t lr = ((ir >> b[q]) << (b[q] + 1)) | (ir & ((1u << b[q]) - 1));
                    const uint32_t l = lt[q] ^ lr;
                    const double2 u = tile[l], v = tile[l ^ xl[q]];
                    const double w = IM ? u.x * v.y - u.y * v.x : u.x * v.x + u.y * v.y;
                    ts[q] = __builtin_fma((__popc(zl[q] & lr) & 1) ? -1.0 : 1.0, w, ts[q]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            // Re(i^ny w): ny = 0, 1, 2, 3 give Re w, -Im w, -Re w, Im w
            const int ny = __builtin_amdgcn_readlane(T.tny, min(j + q, j1 - 1));
            const bool neg = (ny == 1 || ny == 2) != (bool)(__popc(zl[q] & (lt[q] ^ xl[q])) & 1);
            ts[q] = wave_sum(neg ? -2.0 * ts[q] : 2.0 * ts[q]);
        }
        tile_accumulate(T, j, j1, ts, base, lane, acc);
    }
}

// Every tile of the pass into LDS once, then, once the next tile's loads
// are issued, every term of the pass over it: diagonal terms from a Walsh
// transform of the lane's |t|^2, then the pairs read from LDS.  Lane j of each
// wavefront holds term j's masks (read by every lane with readlane, so the
// term loops load nothing from memory) and accumulates term j over the
// wavefront's tiles, in tile order; the four wavefronts' sums are added in
// order at the end.
template <typename A>
__global__ __launch_bounds__(kTileThreads) void k_expect_tile(const A amps, const TilePass P,
                                                              double *__restrict__ partials) {
    __shared__ double2 tile[1 << kTileBits];
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    const uint32_t M = 1u << P.m;
    const int L = P.m < kTileLow ? P.m : kTileLow;
    const uint32_t lowmask = (1u << L) - 1;
    const uint64_t ntiles = 1ull << P.nfree, himask = P.himask, frmask = P.frmask;
    const int nt = P.nt, nd = P.nd, ne = P.ne;
    // this lane's amplitudes of a tile, l = tid | (r << 8): index bits on the
    // tile's qubits (lanes past a small tile's end take its last amplitude,
    // unused)
    uint64_t off[kTilePerLane];
#pragma unroll
    for (int r = 0; r < kTilePerLane; ++r) {
        const uint32_t l = min(tid | ((uint32_t)r << 8), M - 1);
        off[r] = (l & lowmask) | deposit_bits(l >> L, himask);
    }
    TileTerms T{0, 0, 0, 0, 0};
    if ((int)lane < nt) {
        T.txl = P.t[lane].xl;
        T.tzl = P.t[lane].zl;
        T.tny = P.t[lane].ny;
        T.tzh_lo = (uint32_t)P.t[lane].zh;
        T.tzh_hi = (uint32_t)(P.t[lane].zh >> 32);
    }
    double acc = 0.0;
    double vr[kTilePerLane], vi[kTilePerLane];
    uint64_t tl = blockIdx.x;
    if (tl < ntiles) {
        const uint64_t base = deposit_bits(tl, frmask);
#pragma unroll
        for (int r = 0; r < kTilePerLane; ++r)
            amps.get(base | off[r], vr[r], vi[r]);
    }
    for (; tl < ntiles; tl += gridDim.x) {
        const uint64_t base = deposit_bits(tl, frmask);
        __syncthreads();  // every read of the previous tile is done
        double wc[kTilePerLane];
#pragma unroll
        for (int r = 0; r < kTilePerLane; ++r) {
            const uint32_t l = tid | ((uint32_t)r << 8);
            if (l < M)
                tile[l] = make_double2(vr[r], vi[r]);
            wc[r] = l < M ? vr[r] * vr[r] + vi[r] * vi[r] : 0.0;
        }
        __syncthreads();
        if (tl + gridDim.x < ntiles) {
            const uint64_t nb = deposit_bits(tl + gridDim.x, frmask);
#pragma unroll
            for (int r = 0; r < kTilePerLane; ++r)
                amps.get(nb | off[r], vr[r], vi[r]);
        }
        if (nd) {
            walsh16(wc);
            tile_diag(T, 0, nd, wc, tid, base, lane, acc);
        }
        tile_offdiag<false>(T, nd, nd + ne, tile, tid, M, base, lane, acc);
        tile_offdiag<true>(T, nd + ne, nt, tile, tid, M, base, lane, acc);
    }
    __syncthreads();  // the tile's LDS now holds the wavefronts' sums
    double *wsum = reinterpret_cast<double *>(tile);
    wsum[tid] = acc;
    __syncthreads();
    if ((int)tid < nt) {
        double s = 0.0;
        for (int q = 0; q < kTileThreads / 64; ++q)
            s += wsum[q * 64 + tid];
        partials[(size_t)P.t[tid].slot * kMaxPartials + blockIdx.x] = s;
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


// The passes of one expectation call: tile passes for the terms whose x
// mask fits a tile set, one pass per group for the rest, and every plan
// term's partial count (the grid of the pass that evaluates it).
struct ExpectPlan {
    PauliPlan pp;
    std::vector<TilePass> tiles;
    std::vector<DGroup> rest;
    std::vector<int32_t> nblk;
    unsigned tile_grid = 0;
};

// mask's bits on the tile's qubits (0..L-1 and himask) as tile-local bits,
// and its other bits.
static void tile_split(uint64_t mask, int L, uint64_t himask, uint32_t *local, uint64_t *outside) {
    const uint64_t lowm = (1ull << L) - 1;
    uint32_t l = (uint32_t)(mask & lowm);
    int q = 0;
    for (uint64_t h = himask; h; h &= h - 1, ++q)
        if (mask & h & (~h + 1ull))
            l |= 1u << (L + q);
    *local = l;
    *outside = mask & ~lowm & ~himask;
}

static int make_expect_plan(int n, const sv_pauli_t *terms, int nterms, ExpectPlan *e) {
    SV_TRY(make_pauli_plan(n, terms, nterms, &e->pp));
    const PauliPlan &pp = e->pp;
    e->tiles.clear();
    e->rest.clear();
    e->nblk.assign(pp.terms.size(), 0);
    const int m = std::min(n, kTileBits), L = std::min(m, kTileLow), nh = m - L;
    const uint64_t lowm = (1ull << L) - 1;
    DeviceInfo di;
    const uint64_t cus = device_info(&di) == SV_OK ? (uint64_t)di.num_cus : 256;
    e->tile_grid = (unsigned)std::min<uint64_t>({1ull << (n - m), 2 * cus, (uint64_t)kMaxPartials});
    // tile sets (qubits above L), first fit; the first is qubits L..m-1
    std::vector<uint64_t> sets{((1ull << m) - 1) & ~lowm};
    std::vector<std::vector<int>> members(1);
    for (int gi = 0; gi < (int)pp.groups.size(); ++gi) {
        const DGroup &g = pp.groups[gi];
        const uint64_t h = g.x & ~lowm;
        int at = -1;
        for (size_t k = 0; k < sets.size() && at < 0; ++k)
            if (popcount64(sets[k] | h) <= nh)
                at = (int)k;
        if (at < 0 && popcount64(h) <= nh) {
            sets.push_back(0);
            members.emplace_back();
            at = (int)sets.size() - 1;
        }
        if (at < 0) {  // too many qubits above L for one tile
            e->rest.push_back(g);
            for (int j = g.first; j < g.first + g.count; ++j)
                e->nblk[j] = (int32_t)reduce_grid(g.x == 0 ? (1ull << n) : (1ull << (n - 1)));
            continue;
        }
        sets[at] |= h;
        members[at].push_back(gi);
    }
    for (size_t k = 0; k < sets.size(); ++k) {
        if (members[k].empty())
            continue;
        uint64_t set = sets[k];
        for (int q = L; q < n && popcount64(set) < nh; ++q)  // fill up with the lowest unused qubits
            set |= 1ull << q;
        TilePass P;
        memset(&P, 0, sizeof(P));
        P.m = m;
        P.nfree = n - m;
        P.himask = set;
        P.frmask = ((n >= 64) ? ~0ull : ((1ull << n) - 1)) & ~lowm & ~set;
        for (int gi : members[k]) {
            const DGroup &g = pp.groups[gi];
            for (int j = g.first; j < g.first + g.count; ++j) {
                if (P.nt == kTileTerms) {
                    e->tiles.push_back(P);
                    P.nt = 0;
                }
                TTerm &T = P.t[P.nt++];
                uint64_t xo = 0, zh = 0;
                tile_split(g.x, L, P.himask, &T.xl, &xo);
                tile_split(pp.terms[j].z, L, P.himask, &T.zl, &zh);
                if (xo)
                    return fail(SV_EINVAL, "internal: x mask 0x%llx outside its tile set", (unsigned long long)g.x);
                T.zh = zh;
                T.ny = pp.terms[j].ny;
                T.slot = j;
                e->nblk[j] = (int32_t)e->tile_grid;
            }
        }
        if (P.nt)
            e->tiles.push_back(P);
    }
    for (TilePass &P : e->tiles) {  // diagonal terms first, then even ny, then odd ny
        auto kind = [](const TTerm &t) { return t.xl == 0 ? 0 : 1 + (t.ny & 1); };
        std::stable_sort(P.t, P.t + P.nt, [&](const TTerm &a, const TTerm &b) { return kind(a) < kind(b); });
        P.nd = (int32_t)std::count_if(P.t, P.t + P.nt, [&](const TTerm &t) { return kind(t) == 0; });
        P.ne = (int32_t)std::count_if(P.t, P.t + P.nt, [&](const TTerm &t) { return kind(t) == 1; });
    }
    return SV_OK;
}

// f(amps) with the state's amplitude source.
template <typename F> static void with_amps(const sv_state_t *s, F &&f) {
    const char *base = static_cast<const char *>(s->data);
    const int8_t *scales = reinterpret_cast<const int8_t *>(base + (((size_t)1 << s->n) * amp_bytes(s->dtype)));
    switch (s->dtype) {
    case SV_C128:
        f(CplxAmps<double>{(const double2 *)base});
        break;
    case SV_C64:
        f(CplxAmps<float>{(const float2 *)base});
        break;
    case SV_CQ16:
        f(Q16Amps{(const uint32_t *)base, scales});
        break;
    default:
        f(Q32Amps{(const uint2 *)base, scales});
        break;
    }
}

// The passes and the final sums.  terms (the plan's terms), nblk (their
// partial counts), partials (terms * kMaxPartials doubles) and sums (terms
// doubles) are device arrays, the first two already filled or enqueued on st.
static int expect_launch(const sv_state_t *s, const ExpectPlan &plan, const DTerm *terms, const int32_t *nblk,
                         double *partials, double *sums, double *out_total, double *out_terms, hipStream_t st) {
    const int n = s->n;
    for (const TilePass &P : plan.tiles) {
        with_amps(s, [&](auto amps) {
            using A = decltype(amps);
            hipLaunchKernelGGL((k_expect_tile<A>), dim3(plan.tile_grid), dim3(kTileThreads), 0, st, amps, P,
                               partials);
        });
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return fail(SV_EHIP, "expectation launch failed: %s", hipGetErrorString(e));
    }
    for (const DGroup &g : plan.rest) {
        const uint64_t count = g.x == 0 ? (1ull << n) : (1ull << (n - 1));
        const unsigned grid = reduce_grid(count);
        const uint32_t b = g.x ? (uint32_t)__builtin_ctzll(g.x) : 0;
        with_amps(s, [&](auto amps) {
            using A = decltype(amps);
            hipLaunchKernelGGL((k_expect_group<A>), dim3(grid), dim3(kRedThreads), 0, st, amps, count, g.x, b, terms,
                               g.first, g.count, partials);
        });
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return fail(SV_EHIP, "expectation launch failed: %s", hipGetErrorString(e));
    }
    const int nt = (int)plan.pp.terms.size();
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
    ExpectPlan plan;
    SV_TRY(make_expect_plan(s->n, terms, nterms, &plan));
    const std::vector<int32_t> &nblk = plan.nblk;
    PauliDevice d;
    SV_TRY(pauli_upload(plan.pp, (size_t)plan.pp.terms.size() * (kMaxPartials + 1), st, &d));
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
        r = expect_launch(s, plan, d.terms, d_nblk, d.partials, d.partials + plan.pp.terms.size() * kMaxPartials,
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
    ExpectPlan plan;
    SV_TRY(make_expect_plan(s->n, terms, nterms, &plan));
    ExpectTables t;
    memset(&t, 0, sizeof(t));
    t.nterms = (int32_t)plan.pp.terms.size();
    for (size_t j = 0; j < plan.pp.terms.size(); ++j) {
        t.terms[j] = plan.pp.terms[j];
        t.nblk[j] = plan.nblk[j];
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
